// arna.hip -- kernels and host runtime of the ARNA particle-filter step on
// MI355X (gfx950), exported through the C interface in include/arna.h.
//
// Data layout in HBM (one context):
//   prop[2][5][N] float32    ping-pong propagated particles, component-major
//   anc[2][N] uint16         ping-pong ancestors: resampled slot s of PE p is
//                            propagated particle anc[p N_p + s] of that PE
//   rec[2][F*M]              per-PE records (log W^(m), x^m, lstar, T)
//   ring[R][F][M] uint16     pred(m) of R upcoming iterations (ARNA only)
// One workgroup is one PE: it gathers its N_p particles (own slots plus the
// N_ex slots its ring predecessor sends), propagates them, scores them on the
// frame, reduces, resamples in LDS and writes its resampled block.  The
// "master" work (W_{k-1}, PE_eff, N_ex) of the previous iteration is redone
// by every workgroup from the M records at the start of the next iteration,
// so one kernel launch is one iteration and the launch boundary is the only
// grid-wide synchronization.
#include <hip/hip_runtime.h>

#include <limits.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "arna.h"
#include "arna_device.hpp"
#include "arna_kernels.hpp"
#include "arna_adjoint.hpp"
#include "arna_stream.hpp"
#include "arna_master.hpp"

using namespace arna;

namespace {

// ---------------------------------------------------------------- host side
uint32_t fixed_count(float ratio, uint32_t np) {
    double r = (double)ratio;
    if (!(r > 0.0)) return 0;
    if (r > 1.0) r = 1.0;
    return (uint32_t)floor(r * (double)np);
}
uint32_t cutoff_ppm_of(float cutoff) {
    const double c = (double)cutoff;
    if (!(c > 0.0 && c < 1.0)) return 1000000u;
    return (uint32_t)floor(c * 1e6 + 0.5);
}
uint32_t qmax_of(uint32_t np) {
    const uint32_t q = 0xFFFFFFFFu / np;
    return q > (1u << 24) ? (1u << 24) : q;
}
uint32_t block_of(uint32_t np) {
    if (np > 1024) return 1024;
    return (np + 63) / 64 * 64;
}
size_t step_lds(uint32_t np, bool lineage) { return lds_bytes(np, lineage); }

}  // namespace

struct pf_ctx {
    pf_config cfg;
    hipStream_t stream;
    int device;                    // current device at pf_init
    uint64_t N, FM;
    uint32_t block, ppt, half;
    size_t lds;
    // k_step_flex instead of k_step: several PEs per workgroup (ppw > 1), or
    // N_p > PF_MAX_PER_PE_LDS (streamk: log-weights in u [N], one PE per
    // workgroup); n_wg workgroups per launch
    bool flex, streamk;
    uint32_t ppw, n_wg;
    float *u;
    // streamed PEs split over seg_g workgroups each (three launches per
    // iteration; the per-segment results live in sb)
    bool split;
    SplitBufs sb;
    // launch shape of the adjoint (one PE per workgroup, as k_step's default)
    uint32_t adj_ppt, adj_block;
    float *prop[2];
    uint16_t *anc[2];
    pf_pe_record *rec[2];
    int32_t *lin[2];
    int cur;                       // buffers holding iteration `step`
    uint16_t *ring_tab;
    uint64_t ring_base;
    bool ring_valid;
    uint32_t *err, *nex_used;
    // master records (uses_master), ping-pong like the records
    MasterRec *mrec[2];
    double *lm;                    // k_step_flex's log-masses [F M] for k_master, or NULL
    uint32_t *arrive;              // (for a master step in the step's last workgroup)
    // multi-iteration launches (k_run): kernel, or NULL when the context
    // cannot keep all its workgroups resident; barrier counters and wait limit
    void *run_fn;
    unsigned long long *bar;
    unsigned long long bar_timeout;
    StepArgs *run_args;            // [kRunMaxSteps] arguments of a k_run launch
    pf_master_t *est;              // [F] master steps for pf_estimate
    DebugBufs *d_dbg;              // device copy of the debug-buffer table, or NULL
    // trace buffers
    uint32_t *t_pred, *t_q, *t_anc, *t_v;
    int64_t *t_src;
    float *t_prop, *t_ell, *t_lam;
    uint64_t step;
    bool exchanged;
    // gradient recording: while g_cap > 0 the state of iteration g_start + i
    // lives in slot i of the tape (slot 0: the state at pf_grad_begin)
    uint32_t g_cap, g_len, g_alloc;
    uint64_t g_start;
    uint32_t *g_nex;               // [g_alloc + 1][F] N_ex of each recorded iteration
    // choices forced on the next iteration (pf_debug_force_next), or NULL
    const uint32_t *force_anc, *force_nex;
    float *g_prop;                 // [g_alloc + 1][5][N]
    uint16_t *g_anc;               // [g_alloc + 1][N]
    pf_pe_record *g_rec;           // [g_alloc + 1][F M]
    float *g_bar[2];               // [5][N] adjoints of resampled slots
    double *g_lbar[2];             // [2][F M]
    double *g_theta;               // [F M][3]
    double *g_out;                 // [F][4]
    uint32_t key0, key1, fixed_nex, initial_nex, cutoff_ppm, qmax;
    Dyn dyn;
    Lik lik;
};

struct pf_batch {
    struct Group {
        void *fn;
        uint32_t ppt, block, blocks;
        size_t lds;
        std::vector<uint32_t> members;   // context indices
        std::vector<uint32_t> first;     // first workgroup of each member, then the total
        uint32_t *d_first;
        // kind 0: k_step_batch; 1: k_step_flex_batch (ppw PEs per workgroup,
        // log-weight arrays d_u per member); 2: the three split launches
        // (fn, then k_split_totals_batch and k_split_ancestors_batch; buffers
        // d_sb per member)
        int kind;
        uint32_t ppw;
        float **d_u;
        SplitBufs *d_sb;
    };
    std::vector<pf_ctx *> ctx;
    std::vector<Group> groups;
    std::vector<uint32_t> solo;          // contexts launched one by one
    uint32_t n_batched;
    hipStream_t stream;
    StepArgs *d_args;                    // [steps][n_batched], grown on demand
    size_t args_cap;
    // The groups share nothing, so they run side by side: group i (and the
    // solo contexts after the groups) on workers[i % workers.size()], forked
    // from and joined back to `stream` with events at every run.
    std::vector<hipStream_t> workers;
    hipEvent_t ev_fork;
    std::vector<hipEvent_t> ev_join;
    // graph mode: the launches of a run of n iterations of the batched groups,
    // captured once per n and replayed (their arguments are re-read from
    // d_args, which every run rewrites); dropped when d_args moves
    std::vector<std::pair<uint32_t, hipGraphExec_t>> graphs;
};

// Argument table of pf_batch_run_noalloc: a fixed device array, one copy per
// GPU, held until the process ends.  Host code uses the address
// hipGetSymbolAddress gave on each device (noalloc_args), never the name.
static __device__ __align__(256) StepArgs scratch[PF_BATCH_NOALLOC_MAX_ARGS];

namespace {

constexpr int kMaxDevices = 64;
StepArgs *noalloc_args[kMaxDevices];   // device address of `scratch` per device
std::mutex noalloc_mu;

// Takes the address of `scratch` on device dev (the current device), once.
int noalloc_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return PF_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (noalloc_args[dev]) return PF_OK;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return PF_EHIP;
    }
    noalloc_args[dev] = (StepArgs *)p;
    return PF_OK;
}

// From this many PEs per filter on, the master step is computed once per
// filter (by k_master, launched after the step) instead of by every PE of the
// next iteration.  A separate launch rather than the step's last workgroup:
// the step kernels can compute it in their last workgroup (StepArgs.mout), but
// the agent-scope release every workgroup then needs before counting itself
// in cost more than the launch, measured on MI355X with several PEs per
// workgroup at 2^20 particles: 2048 x 512 52.1 -> 47.0 us per iteration,
// 4096 x 256 55.6 -> 53.2, 8192 x 128 81.3 -> 74.8.  The threshold, measured
// at 2^20 (us per iteration with the threshold at 2048 / 512): 512 x 2048
// 48.9 / 46.1, 1024 x 1024 95.5 / 68.3 (one PE per workgroup) and 46.3 / 43.0
// (two); 256 x 4096 33.3 with either, 37.6 with the threshold at 256.
constexpr uint32_t kMasterMinPE = 512;
// Multi-iteration launches (k_run) keep the master step in every PE's
// prologue: they take fewer PEs than this and no master record.
constexpr uint32_t kRunMaxPE = 2048;

// Whether a context keeps once-per-filter master records.
bool uses_master(const pf_config *c) {
    return c->n_pe >= kMasterMinPE && c->launch != PF_LAUNCH_PERSISTENT;
}

#define HIP_OK(expr)                                      \
    do {                                                  \
        if ((expr) != hipSuccess) return PF_EHIP;         \
    } while (0)

template <typename T>
int dev_alloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) return PF_OK;
    if (hipMalloc((void **)p, count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return PF_ENOMEM;
    }
    return PF_OK;
}

// Buffers of the current iteration (the tape while recording).
float *cur_prop(pf_ctx *c) {
    return c->g_cap ? c->g_prop + (size_t)c->g_len * 5 * c->N : c->prop[c->cur];
}
uint16_t *cur_anc(pf_ctx *c) {
    return c->g_cap ? c->g_anc + (size_t)c->g_len * c->N : c->anc[c->cur];
}
pf_pe_record *cur_rec(pf_ctx *c) {
    return c->g_cap ? c->g_rec + (size_t)c->g_len * c->FM : c->rec[c->cur];
}

template <int PPT, int HALF, int LIK>
void *step_kernel() {
    return reinterpret_cast<void *>(&k_step<PPT, HALF, LIK>);
}

template <int LIK>
void *pick_patch_kernel(uint32_t ppt, uint32_t half) {
#define ARNA_HALVES(P)                          \
    switch (half) {                             \
        case 0: return step_kernel<P, 0, LIK>(); \
        case 1: return step_kernel<P, 1, LIK>(); \
        case 2: return step_kernel<P, 2, LIK>(); \
        case 3: return step_kernel<P, 3, LIK>(); \
        case 4: return step_kernel<P, 4, LIK>(); \
        case 5: return step_kernel<P, 5, LIK>(); \
        case 6: return step_kernel<P, 6, LIK>(); \
        case 7: return step_kernel<P, 7, LIK>(); \
        default: return nullptr;                \
    }
    if (ppt == 1) {
        ARNA_HALVES(1)
    } else if (ppt == 2) {
        ARNA_HALVES(2)
    } else {
        ARNA_HALVES(4)
    }
#undef ARNA_HALVES
    return nullptr;
}

void *pick_step_kernel(uint32_t ppt, uint32_t half, uint32_t lik_mode) {
    if (lik_mode == PF_LIK_POINT)
        return ppt == 1 ? step_kernel<1, 0, kLikPoint>()
                        : (ppt == 2 ? step_kernel<2, 0, kLikPoint>() : step_kernel<4, 0, kLikPoint>());
    if (lik_mode == PF_LIK_POISSON) return pick_patch_kernel<kLikPoisson>(ppt, half);
    return pick_patch_kernel<kLikGauss>(ppt, half);
}

template <int HALF, int LIK, bool ULDS>
void *flex_kernel() {
    return reinterpret_cast<void *>(&k_step_flex<HALF, LIK, ULDS>);
}

template <int LIK, bool ULDS>
void *pick_flex_patch_kernel(uint32_t half) {
    switch (half) {
        case 0: return flex_kernel<0, LIK, ULDS>();
        case 1: return flex_kernel<1, LIK, ULDS>();
        case 2: return flex_kernel<2, LIK, ULDS>();
        case 3: return flex_kernel<3, LIK, ULDS>();
        case 4: return flex_kernel<4, LIK, ULDS>();
        case 5: return flex_kernel<5, LIK, ULDS>();
        case 6: return flex_kernel<6, LIK, ULDS>();
        case 7: return flex_kernel<7, LIK, ULDS>();
        default: return nullptr;
    }
}

template <bool ULDS>
void *pick_flex_kernel_u(uint32_t half, uint32_t lik_mode) {
    if (lik_mode == PF_LIK_POINT) return flex_kernel<0, kLikPoint, ULDS>();
    if (lik_mode == PF_LIK_POISSON) return pick_flex_patch_kernel<kLikPoisson, ULDS>(half);
    return pick_flex_patch_kernel<kLikGauss, ULDS>(half);
}

// ulds: log-weights in LDS (several PEs per workgroup), else in HBM (PEs
// beyond the LDS stage)
void *pick_flex_kernel(uint32_t half, uint32_t lik_mode, bool ulds) {
    return ulds ? pick_flex_kernel_u<true>(half, lik_mode)
                : pick_flex_kernel_u<false>(half, lik_mode);
}

template <int HALF, int LIK>
void *split_kernel() {
    return reinterpret_cast<void *>(&k_split_weights<HALF, LIK>);
}

template <int LIK>
void *pick_split_patch_kernel(uint32_t half) {
    switch (half) {
        case 0: return split_kernel<0, LIK>();
        case 1: return split_kernel<1, LIK>();
        case 2: return split_kernel<2, LIK>();
        case 3: return split_kernel<3, LIK>();
        case 4: return split_kernel<4, LIK>();
        case 5: return split_kernel<5, LIK>();
        case 6: return split_kernel<6, LIK>();
        case 7: return split_kernel<7, LIK>();
        default: return nullptr;
    }
}

void *split_totals_kernel() { return reinterpret_cast<void *>(&k_split_totals); }
void *split_ancestors_kernel() { return reinterpret_cast<void *>(&k_split_ancestors); }

// The first of the three launches of a split iteration.
void *pick_split_kernel(uint32_t half, uint32_t lik_mode) {
    if (lik_mode == PF_LIK_POINT) return split_kernel<0, kLikPoint>();
    if (lik_mode == PF_LIK_POISSON) return pick_split_patch_kernel<kLikPoisson>(half);
    return pick_split_patch_kernel<kLikGauss>(half);
}

// The one-iteration kernel of a context (for a split context, the first of
// its three launches).
void *ctx_step_kernel(const pf_ctx *c) {
    if (c->split) return pick_split_kernel(c->half, c->cfg.lik_mode);
    return c->flex ? pick_flex_kernel(c->half, c->cfg.lik_mode, !c->streamk)
                   : pick_step_kernel(c->ppt, c->half, c->cfg.lik_mode);
}

// Streamed PEs are split over several workgroups while a context has fewer
// PEs than compute units (with one workgroup per PE most would sit idle).
// Measured on MI355X (tracking frames, us per iteration, split / one
// workgroup per PE): 16 x 65536 48.5 / 275, 64 x 16384 43.2 / 91.4,
// 2 x 3 x 20000 33.0 / 102.5, 256 x 8192 70.7 / 61.9, 512 x 8192 124.9 / 118.6.
constexpr uint64_t kSplitBelowPEs = 256;
bool split_pes(uint64_t FM) { return FM < kSplitBelowPEs; }

// Threads per PE of a context with several PEs per workgroup: N_p rounded up
// to 64, at most 1024 / ppw (rounded down to 64).
uint32_t group_threads(uint32_t np, uint32_t ppw) {
    const uint32_t cap = 1024 / ppw / 64 * 64;
    const uint32_t want = (np + 63) / 64 * 64;
    return want < cap ? want : cap;
}

// Batched variants exist for the paper's 9 x 9 patch (Gaussian or Poisson
// noise) and for point observations; other contexts of a batch are launched
// one by one.
template <int PPT, int HALF, int LIK>
void *batch_kernel() {
    return reinterpret_cast<void *>(&k_step_batch<PPT, HALF, LIK>);
}

template <int HALF, int LIK>
void *batch_kernel_ppt(uint32_t ppt) {
    return ppt == 1 ? batch_kernel<1, HALF, LIK>()
                    : (ppt == 2 ? batch_kernel<2, HALF, LIK>() : batch_kernel<4, HALF, LIK>());
}

template <int HALF, int LIK, bool ULDS>
void *flex_batch_kernel() {
    return reinterpret_cast<void *>(&k_step_flex_batch<HALF, LIK, ULDS>);
}
template <int HALF, int LIK>
void *split_batch_kernel() {
    return reinterpret_cast<void *>(&k_split_weights_batch<HALF, LIK>);
}
void *split_totals_batch_kernel() { return reinterpret_cast<void *>(&k_split_totals_batch); }
void *split_ancestors_batch_kernel() {
    return reinterpret_cast<void *>(&k_split_ancestors_batch);
}

// Batched variants of k_step_flex and of the split kernels, for the 9 x 9
// patch and point observations (others run one by one).
void *pick_flex_batch_kernel(uint32_t half, uint32_t lik_mode, bool ulds) {
    if (lik_mode == PF_LIK_POINT)
        return ulds ? flex_batch_kernel<0, kLikPoint, true>() : flex_batch_kernel<0, kLikPoint, false>();
    if (half != 4) return nullptr;
    if (lik_mode == PF_LIK_POISSON)
        return ulds ? flex_batch_kernel<4, kLikPoisson, true>()
                    : flex_batch_kernel<4, kLikPoisson, false>();
    return ulds ? flex_batch_kernel<4, kLikGauss, true>() : flex_batch_kernel<4, kLikGauss, false>();
}
void *pick_split_batch_kernel(uint32_t half, uint32_t lik_mode) {
    if (lik_mode == PF_LIK_POINT) return split_batch_kernel<0, kLikPoint>();
    if (half != 4) return nullptr;
    if (lik_mode == PF_LIK_POISSON) return split_batch_kernel<4, kLikPoisson>();
    return split_batch_kernel<4, kLikGauss>();
}

void *pick_batch_kernel(uint32_t ppt, uint32_t half, uint32_t lik_mode) {
    if (lik_mode == PF_LIK_POINT) return batch_kernel_ppt<0, kLikPoint>(ppt);
    if (half != 4) return nullptr;
    if (lik_mode == PF_LIK_POISSON) return batch_kernel_ppt<4, kLikPoisson>(ppt);
    return batch_kernel_ppt<4, kLikGauss>(ppt);
}

void *pick_run_kernel(uint32_t ppt, uint32_t half, uint32_t lik_mode) {
    return arna_run_kernel(ppt, half, lik_mode);
}

template <int PPT, int HALF>
void *adj_kernel() {
    return reinterpret_cast<void *>(&k_adjoint<PPT, HALF>);
}

void *pick_adjoint_kernel(uint32_t ppt, uint32_t half) {
#define ARNA_ADJ_HALVES(P)                     \
    switch (half) {                            \
        case 0: return adj_kernel<P, 0>();     \
        case 1: return adj_kernel<P, 1>();     \
        case 2: return adj_kernel<P, 2>();     \
        case 3: return adj_kernel<P, 3>();     \
        case 4: return adj_kernel<P, 4>();     \
        case 5: return adj_kernel<P, 5>();     \
        case 6: return adj_kernel<P, 6>();     \
        case 7: return adj_kernel<P, 7>();     \
        default: return nullptr;               \
    }
    if (ppt == 1) {
        ARNA_ADJ_HALVES(1)
    } else if (ppt == 2) {
        ARNA_ADJ_HALVES(2)
    } else {
        ARNA_ADJ_HALVES(4)
    }
#undef ARNA_ADJ_HALVES
    return nullptr;
}

int validate(const pf_config *c) {
    if (!c || c->struct_size != sizeof(pf_config)) return PF_EINVAL;
    if (c->n_filters == 0 || c->n_pe == 0 || c->n_per_pe == 0) return PF_EINVAL;
    if (c->n_pe > PF_MAX_PE || c->n_per_pe > PF_MAX_PER_PE) return PF_EUNSUPPORTED;
    if (c->mode > 1 || c->init_mode > 1 || c->lik_mode > 2) return PF_EINVAL;
    if (c->ring_groups > 256) return PF_EINVAL;
    if (c->launch > PF_LAUNCH_PERSISTENT) return PF_EINVAL;
    if (c->pes_per_wg > kMaxPesPerWg) return PF_EINVAL;
    if (c->pes_per_wg > 1 || c->n_per_pe > PF_MAX_PER_PE_LDS) {
        // k_step_flex: no lineage tags, no multi-iteration launch
        if ((c->debug & PF_DEBUG_LINEAGE) || c->launch == PF_LAUNCH_PERSISTENT)
            return PF_EUNSUPPORTED;
    }
    if (c->launch == PF_LAUNCH_PERSISTENT && c->n_pe >= kRunMaxPE) return PF_EUNSUPPORTED;
    if (c->n_per_pe > PF_MAX_PER_PE_LDS) {
        // one streamed PE per workgroup of 1024 threads
        if (c->pes_per_wg > 1) return PF_EINVAL;
        if (c->block_size && c->block_size != kStreamBlock) return PF_EINVAL;
    } else if (c->pes_per_wg > 1) {
        // ppw groups of whole waves, at most 4 slots per thread
        const uint32_t ppw = c->pes_per_wg;
        const uint32_t B = c->block_size ? c->block_size
                                         : ppw * group_threads(c->n_per_pe, ppw);
        if (B == 0 || B > 1024 || B % (64 * ppw)) return PF_EINVAL;
        if ((uint64_t)(B / ppw) * 4 < c->n_per_pe) return PF_EINVAL;
    } else if (c->block_size) {
        if (c->block_size % 64 || c->block_size > 1024) return PF_EINVAL;
        if ((uint64_t)c->block_size * 4 < c->n_per_pe) return PF_EINVAL;
    }
    if (c->lik_mode == PF_LIK_POISSON && !(c->background > 0.f)) return PF_EINVAL;
    if (c->lik_mode != PF_LIK_POINT) {
        if (c->patch == 0 || (c->patch & 1u) == 0) return PF_EINVAL;
        if (c->patch > PF_MAX_PATCH) return PF_EUNSUPPORTED;
    }
    if (c->width == 0 || c->height == 0 || c->width > 65536 || c->height > 65536)
        return PF_EINVAL;
    const float fl[] = {c->fixed_ratio, c->initial_ratio, c->eff_cutoff, c->psf_sigma,
                        c->background, c->noise_sigma, c->q, c->sigma_I};
    for (float v : fl)
        if (!isfinite(v)) return PF_EINVAL;
    if (c->fixed_ratio < 0.f || c->fixed_ratio > 1.f) return PF_EINVAL;
    if (c->initial_ratio < 0.f || c->initial_ratio > 1.f) return PF_EINVAL;
    if (!(c->psf_sigma > 0.f) || !(c->noise_sigma > 0.f) || c->q < 0.f || c->sigma_I < 0.f)
        return PF_EINVAL;
    const uint64_t N = (uint64_t)c->n_filters * c->n_pe * c->n_per_pe;
    if (N > PF_MAX_PARTICLES || (uint64_t)c->n_filters * c->n_pe > (1ull << 24))
        return PF_EUNSUPPORTED;
    return PF_OK;
}

void free_all(pf_ctx *c) {
    void *ptrs[] = {c->prop[0], c->prop[1], c->anc[0], c->anc[1], c->rec[0], c->rec[1],
                    c->lin[0], c->lin[1],
                    c->ring_tab, c->err, c->nex_used, c->est, c->t_pred, c->t_q, c->t_anc,
                    c->t_v, c->t_src, c->t_prop, c->t_ell, c->t_lam, c->d_dbg,
                    c->mrec[0], c->mrec[1], c->lm, c->arrive, c->bar, c->run_args,
                    c->g_prop, c->g_anc, c->g_rec, c->g_nex, c->g_bar[0], c->g_bar[1], c->g_lbar[0],
                    c->g_lbar[1], c->g_theta, c->g_out, c->u, c->sb.seg_max, c->sb.seg_wq,
                    c->sb.seg_sum};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
}

// Ring table for iteration k; when it has to be rebuilt, the batch of
// kRingSteps iterations starts at k (forward runs) or ends at k (the adjoint
// sweep, which runs backwards).
// Whether iteration k needs the ring table rebuilt; if so the new batch's
// first iteration goes to *base and the context records it as built.
bool plan_ring(pf_ctx *c, uint64_t k, bool downward, uint64_t *base) {
    if (c->cfg.mode != PF_MODE_ARNA || c->cfg.n_pe <= 1) return false;
    if (c->ring_valid && k >= c->ring_base && k < c->ring_base + kRingSteps) return false;
    *base = (downward && k >= kRingSteps) ? k - (kRingSteps - 1) : (downward ? 1 : k);
    c->ring_base = *base;
    c->ring_valid = true;
    return true;
}

int launch_ring(pf_ctx *c, uint64_t base) {
    const uint32_t M = c->cfg.n_pe;
    (void)hipGetLastError();   // clear errors of earlier, unrelated calls
    hipLaunchKernelGGL(k_ring, dim3(kRingSteps, c->cfg.n_filters), dim3(256),
                       ring_lds_bytes(M, c->cfg.ring_groups), c->stream, c->ring_tab,
                       (uint32_t)base, c->cfg.n_filters, M, c->cfg.ring_groups, c->key0, c->key1);
    HIP_OK(hipGetLastError());
    return PF_OK;
}

int ensure_ring(pf_ctx *c, uint64_t k, bool downward = false) {
    uint64_t base;
    if (!plan_ring(c, k, downward, &base)) return PF_OK;
    return launch_ring(c, base);
}

// traj_prev: the trajectory row of iteration k-1 that the step writes, or NULL.
StepArgs make_args(pf_ctx *c, uint64_t k, const float *frame, pf_master_t *traj_prev = nullptr) {
    StepArgs a;
    memset(&a, 0, sizeof(a));
    const int nxt = 1 - c->cur;
    a.pin = cur_prop(c);
    a.ain = cur_anc(c);
    a.rin = cur_rec(c);
    a.force_anc = c->force_anc;
    a.force_nex = c->force_nex;
    if (c->mrec[0]) a.min = c->mrec[c->cur];   // (a.mout stays NULL: k_master follows)
    if (c->g_cap) {
        a.nex_rec = c->g_nex + (size_t)(c->g_len + 1) * c->cfg.n_filters;
        a.pout = c->g_prop + (size_t)(c->g_len + 1) * 5 * c->N;
        a.aout = c->g_anc + (size_t)(c->g_len + 1) * c->N;
        a.rout = c->g_rec + (size_t)(c->g_len + 1) * c->FM;
    } else {
        a.pout = c->prop[nxt];
        a.aout = c->anc[nxt];
        a.rout = c->rec[nxt];
    }
    a.ring = (c->cfg.mode == PF_MODE_ARNA && c->cfg.n_pe > 1)
                 ? c->ring_tab + (size_t)(k - c->ring_base) * c->FM
                 : nullptr;
    a.dbg = c->d_dbg;
    a.lik = c->lik;
    a.lik.img = frame;
    a.dyn = c->dyn;
    a.N = (uint32_t)c->N;
    a.M = c->cfg.n_pe;
    a.np = c->cfg.n_per_pe;
    a.k = (uint32_t)k;
    a.key0 = c->key0;
    a.key1 = c->key1;
    a.mode = c->cfg.mode;
    a.first = (c->step == 0) ? 1u : 0u;
    a.fixed_nex = c->fixed_nex;
    a.initial_nex = c->initial_nex;
    a.cutoff_ppm = c->cutoff_ppm;
    a.qmax = c->qmax;
    a.lin_in = (uint32_t)c->cur;
    a.err = c->err;
    a.nex_used = c->nex_used;
    // (many PEs: k_master writes the rows; split PEs: k_global_wave)
    a.traj_prev = (c->mrec[0] || c->split) ? nullptr : traj_prev;
    return a;
}

// Master records of the records in buffer `which` (after initialization or a
// state load), when the context uses them.
int refresh_master(pf_ctx *c, int which) {
    if (!c->mrec[0]) return PF_OK;
    HIP_OK(launch_master(c->stream, c->cfg.n_filters, c->cfg.n_pe, c->cfg.n_per_pe, c->cfg.mode,
                         c->fixed_nex, c->cutoff_ppm, c->rec[which], nullptr, c->mrec[which]));
    return PF_OK;
}

// Host state after iteration k has been enqueued.
void advance(pf_ctx *c, uint64_t k) {
    c->cur = 1 - c->cur;
    if (c->g_cap) ++c->g_len;
    c->force_anc = nullptr;
    c->force_nex = nullptr;
    c->step = k;
    c->exchanged = false;
}

// traj_prev: the trajectory row of iteration k - 1, written by the step's
// prologue (contexts without master records); row: that of iteration k,
// written with the master record after the step (contexts with them).
int launch_step(pf_ctx *c, const float *frame, pf_master_t *traj_prev = nullptr,
                pf_master_t *row = nullptr) {
    const uint64_t k = c->step + 1;
    if (k > 0xFFFFFFFFull) return PF_EUNSUPPORTED;
    if (c->g_cap && c->g_len >= c->g_cap) return PF_ESTATE;   // tape full
    int rc = ensure_ring(c, k);
    if (rc != PF_OK) return rc;
    StepArgs a = make_args(c, k, frame, traj_prev);
    void *fn = ctx_step_kernel(c);
    if (!fn) return PF_EUNSUPPORTED;
    if (c->split) {
        // three launches, the segments of every PE side by side
        void *sargs[] = {&a, &c->sb};
        const dim3 grid((uint32_t)(c->FM * c->sb.G)), blk(kSplitBlock);
        HIP_OK(hipLaunchKernel(fn, grid, blk, sargs, split_lds_bytes(), c->stream));
        HIP_OK(hipLaunchKernel(split_totals_kernel(), grid, blk, sargs, split_lds_bytes(),
                               c->stream));
        HIP_OK(hipLaunchKernel(split_ancestors_kernel(), grid, blk, sargs, split_lds_bytes(),
                               c->stream));
        advance(c, k);
        return PF_OK;
    }
    void *args[] = {&a, &c->u, &c->ppw, &c->lm};   // (k_step takes the first only)
    HIP_OK(hipLaunchKernel(fn, dim3(c->n_wg), dim3(c->block), args, c->lds, c->stream));
    if (c->mrec[0]) {
        // the master step of this iteration from the records just written
        // (k_step_flex also wrote their log-masses side by side)
        HIP_OK(launch_master(c->stream, c->cfg.n_filters, c->cfg.n_pe, c->cfg.n_per_pe,
                             c->cfg.mode, c->fixed_nex, c->cutoff_ppm, a.rout, c->lm,
                             c->mrec[1 - c->cur], row, c->nex_used, k));
    }
    advance(c, k);
    return PF_OK;
}

// Streams a batch spreads its groups over (HIP's default of four hardware
// queues per process).
constexpr size_t kBatchStreams = 4;

// Most iterations per k_run launch (bounds a launch's duration).
constexpr uint32_t kRunMaxSteps = 64;
// PF_LAUNCH_AUTO launches one kernel per iteration.  Measured on MI355X, k_run
// is faster only for small contexts (1 x 4 x 256: 10.2 vs 11.5 us per
// iteration; 1 x 16 x 1024: 13.8 vs 16.6; 4 x 64 x 4096: 39.5 vs 33.5), and
// its cooperative launch costs about a millisecond once the process has three
// or more other streams (a batch of 64 small contexts stepped one after
// another: 54 ms instead of 31 ms), so it is used only on request.

// Whether the next iterations may run as k_run launches: the context fits
// (run_fn) and no per-iteration hook is active (gradient tape, forced choices).
bool run_allowed(const pf_ctx *c) {
    return c->run_fn && !c->g_cap && !c->force_anc && !c->force_nex;
}

// n iterations on frames + i * stride.  Iterations run in k_run launches of
// up to kRunMaxSteps (never across a rebuild of the ring table); a lone
// iteration, or any iteration while run_allowed is false, is a k_step launch.
// With ms_out, each launch is timed by a pair of events on the stream and
// every iteration of it is given the launch's time divided by its length.
// The master step of the latest iteration (records of the current buffer)
// to out[F].
int launch_global(pf_ctx *c, pf_master_t *out) {
    (void)hipGetLastError();   // clear errors of earlier, unrelated calls
    // without master records: one wave per filter, in the order of the step's
    // prologue; with them: k_master's order (from the records; no record is
    // written), the rows a trajectory run gets after every step
    if (!c->mrec[0]) {
        hipLaunchKernelGGL(k_global_wave, dim3(c->cfg.n_filters), dim3(kWave), 0, c->stream,
                           cur_rec(c), out, c->cfg.n_pe, c->cfg.n_per_pe, c->cfg.mode,
                           c->fixed_nex, c->cutoff_ppm, (const uint32_t *)c->nex_used,
                           (uint64_t)c->step);
        HIP_OK(hipGetLastError());
        return PF_OK;
    }
    HIP_OK(launch_master(c->stream, c->cfg.n_filters, c->cfg.n_pe, c->cfg.n_per_pe, c->cfg.mode,
                         c->fixed_nex, c->cutoff_ppm, cur_rec(c), nullptr, nullptr, out,
                         c->nex_used, c->step));
    return PF_OK;
}

// With traj, the master step of every iteration goes to traj[i][F]: without
// master records the step of iteration i + 1 writes row i from its prologue
// and one k_global_wave launch after the run writes the last row; with them,
// the k_master launch after every step writes its row; for split PEs, a
// k_global_wave launch follows every step.  Either way the
// iterations run one launch each.
int run_steps(pf_ctx *c, const float *frames, uint32_t n, uint64_t stride, float *ms_out,
              pf_master_t *traj = nullptr) {
    const bool timed = ms_out != nullptr;
    std::vector<hipEvent_t> ev;
    std::vector<uint32_t> len_of;   // iterations of each timed launch
    int rc = PF_OK;
    uint32_t done = 0;
    while (rc == PF_OK && done < n) {
        const uint64_t k = c->step + 1;
        if (k > 0xFFFFFFFFull) return PF_EUNSUPPORTED;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timed) {
            if (hipEventCreate(&e0) != hipSuccess) {
                rc = PF_EHIP;
                break;
            }
            ev.push_back(e0);
            if (hipEventCreate(&e1) != hipSuccess) {
                rc = PF_EHIP;
                break;
            }
            ev.push_back(e1);
            if (hipEventRecord(e0, c->stream) != hipSuccess) {
                rc = PF_EHIP;
                break;
            }
        }
        uint32_t len = 1;
        if (run_allowed(c) && !traj) {
            rc = ensure_ring(c, k);
            if (rc != PF_OK) break;
            len = n - done < kRunMaxSteps ? n - done : kRunMaxSteps;
            if (c->ring_valid && c->ring_tab) {
                const uint64_t room = c->ring_base + kRingSteps - k;
                if (len > room) len = (uint32_t)room;
            }
            if (k + len - 1 > 0xFFFFFFFFull) len = (uint32_t)(0xFFFFFFFFull - k + 1);
        }
        const float *frame = frames + (size_t)done * stride;
        if (len == 1) {
            const size_t F = c->cfg.n_filters;
            const bool fused = traj && !c->mrec[0] && !c->split;
            pf_master_t *row = (traj && c->mrec[0]) ? traj + (size_t)done * F : nullptr;
            rc = launch_step(c, frame, (fused && done) ? traj + (size_t)(done - 1) * F : nullptr,
                             row);
            if (rc == PF_OK && traj && !fused && !row)
                rc = launch_global(c, traj + (size_t)done * F);
        } else {
            RunPrep pr;
            memset(&pr, 0, sizeof(pr));
            pr.a = make_args(c, k, frame);
            pr.frames = frame;
            pr.stride = stride;
            pr.ring0 = pr.a.ring;
            for (int b = 0; b < 2; ++b) {
                pr.prop[b] = c->prop[b];
                pr.anc[b] = c->anc[b];
                pr.rec[b] = c->rec[b];
            }
            pr.cur = (uint32_t)c->cur;
            pr.n = len;
            pr.fm = (uint32_t)c->FM;
            pr.F = c->cfg.n_filters;
            pr.out = c->run_args;
            pr.bar = c->bar;
            const uint32_t threads = len > pr.F ? len : pr.F;
            (void)hipGetLastError();   // clear errors of earlier, unrelated calls
            hipLaunchKernelGGL(k_run_prep, dim3((threads + 63) / 64), dim3(64), 0, c->stream, pr);
            if (hipGetLastError() != hipSuccess) rc = PF_EHIP;
            RunArgs r;
            r.args = c->run_args;
            r.n = len;
            r.bar = c->bar;
            r.timeout = c->bar_timeout;
            void *args[] = {&r};
            if (rc == PF_OK &&
                hipLaunchCooperativeKernel(c->run_fn, dim3((uint32_t)c->FM), dim3(c->block), args,
                                           (unsigned)c->lds, c->stream) != hipSuccess)
                rc = PF_EHIP;
            if (rc == PF_OK)
                for (uint32_t i = 0; i < len; ++i) advance(c, k + i);
        }
        if (rc == PF_OK && timed) {
            if (hipEventRecord(e1, c->stream) != hipSuccess) rc = PF_EHIP;
            len_of.push_back(len);
        }
        if (rc == PF_OK) done += len;
    }
    if (rc == PF_OK && traj && n && !c->mrec[0])   // the last row
        rc = launch_global(c, traj + (size_t)(n - 1) * c->cfg.n_filters);
    if (timed) {
        if (rc == PF_OK && hipStreamSynchronize(c->stream) != hipSuccess) rc = PF_EHIP;
        uint32_t it = 0;
        for (size_t l = 0; rc == PF_OK && l < len_of.size(); ++l) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[2 * l], ev[2 * l + 1]) != hipSuccess) {
                rc = PF_EHIP;
                break;
            }
            for (uint32_t i = 0; i < len_of[l]; ++i) ms_out[it++] = ms / (float)len_of[l];
        }
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    return rc;
}

}  // namespace

extern "C" {

const char *pf_strerror(int code) {
    switch (code) {
        case PF_OK: return "ok";
        case PF_EINVAL: return "invalid argument or configuration";
        case PF_ENOMEM: return "device memory allocation failed";
        case PF_EHIP: return "HIP runtime error";
        case PF_ENUMERIC: return "NaN log-weight encountered (sticky)";
        case PF_ESTATE: return "call out of order";
        case PF_EUNSUPPORTED: return "size beyond the limits of this build";
        case PF_ETIMEOUT: return "a barrier between workgroups timed out (sticky)";
        default: return "unknown error";
    }
}

int pf_init(const pf_config *cfg, const float *truth, pf_ctx **out) {
    if (!out) return PF_EINVAL;
    *out = nullptr;
    int rc = validate(cfg);
    if (rc != PF_OK) return rc;
    if (!truth) return PF_EINVAL;
    pf_ctx *c = new (std::nothrow) pf_ctx;
    if (!c) return PF_ENOMEM;
    memset(c, 0, sizeof(*c));
    c->cfg = *cfg;
    c->stream = (hipStream_t)cfg->stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return PF_EHIP;
    }
    // the no-allocation batch entry point's table on this device (its failure
    // only disables that entry point)
    (void)noalloc_setup(c->device);
    const uint32_t F = cfg->n_filters, M = cfg->n_pe, np = cfg->n_per_pe;
    c->FM = (uint64_t)F * M;
    c->N = c->FM * np;
    c->streamk = np > PF_MAX_PER_PE_LDS;
    c->split = c->streamk && split_pes(c->FM);
    c->ppw = cfg->pes_per_wg > 1 ? cfg->pes_per_wg : 1;
    c->flex = c->streamk || c->ppw > 1;
    c->n_wg = (uint32_t)((uint64_t)F * ((M + c->ppw - 1) / c->ppw));
    if (c->streamk) {
        c->block = kStreamBlock;
        c->ppt = 0;
    } else if (c->ppw > 1) {
        c->block = cfg->block_size ? cfg->block_size : c->ppw * group_threads(np, c->ppw);
        c->ppt = 0;
    } else if (cfg->block_size) {
        c->block = cfg->block_size;
        c->ppt = np <= c->block ? 1 : (np <= 2 * c->block ? 2 : 4);
    } else {
        c->block = block_of(np);
        c->ppt = np > 1024 ? 4 : 1;
    }
    c->half = cfg->lik_mode != PF_LIK_POINT ? cfg->patch / 2 : 0;
    c->adj_ppt = c->flex ? (np > 1024 ? 4 : 1) : c->ppt;
    c->adj_block = c->flex ? block_of(np) : c->block;
    const bool lineage = (cfg->debug & PF_DEBUG_LINEAGE) != 0;
    const bool trace = (cfg->debug & PF_DEBUG_TRACE) != 0;
    c->lds = c->streamk ? flex_lds_bytes(0, kSmallTile)
                        : (c->flex ? flex_lds_bytes(c->ppw * np, kSmallTile)
                                   : step_lds(np, lineage));
    c->key0 = (uint32_t)cfg->seed;
    c->key1 = (uint32_t)(cfg->seed >> 32);
    c->fixed_nex = fixed_count(cfg->fixed_ratio, np);
    c->initial_nex = fixed_count(cfg->initial_ratio, np);
    c->cutoff_ppm = cutoff_ppm_of(cfg->eff_cutoff);
    c->qmax = qmax_of(np);
    const float sq = sqrtf(cfg->q);
    c->dyn.a = sqrtf(cfg->q / 3.0f);
    c->dyn.b = sq * 0.8660254037844386f;
    c->dyn.c = sq * 0.5f;
    c->dyn.sigma_I = cfg->sigma_I;
    c->lik.W = (int)cfg->width;
    c->lik.H = (int)cfg->height;
    c->lik.inv2s2 = 1.0f / (2.0f * cfg->psf_sigma * cfg->psf_sigma);
    c->lik.k2 = expf(-2.0f * c->lik.inv2s2);
    c->lik.bg = cfg->background;
    c->lik.inv_bg = cfg->background > 0.f ? 1.0f / cfg->background : 0.f;
    c->lik.inv_sn2 = 1.0f / (cfg->noise_sigma * cfg->noise_sigma);

    const uint64_t N = c->N;
    rc = PF_OK;
    for (int i = 0; i < 2 && rc == PF_OK; ++i) {
        rc = dev_alloc(&c->prop[i], 5 * N);
        if (rc == PF_OK) rc = dev_alloc(&c->anc[i], N);
        if (rc == PF_OK) rc = dev_alloc(&c->rec[i], c->FM);
        if (rc == PF_OK && lineage) rc = dev_alloc(&c->lin[i], N);
    }
    if (rc == PF_OK && cfg->mode == PF_MODE_ARNA && M > 1)
        rc = dev_alloc(&c->ring_tab, (size_t)kRingSteps * c->FM);
    if (rc == PF_OK && uses_master(cfg)) {
        rc = dev_alloc(&c->mrec[0], F);
        if (rc == PF_OK) rc = dev_alloc(&c->mrec[1], F);
        if (rc == PF_OK) rc = dev_alloc(&c->arrive, F);
        if (rc == PF_OK && c->flex) rc = dev_alloc(&c->lm, c->FM);
    }
    if (rc == PF_OK) rc = dev_alloc(&c->err, 1);
    if (rc == PF_OK) rc = dev_alloc(&c->nex_used, F);
    if (rc == PF_OK) rc = dev_alloc(&c->est, F);
    if (rc == PF_OK && c->streamk) rc = dev_alloc(&c->u, N);
    if (rc == PF_OK && c->split) {
        c->sb.u = c->u;
        c->sb.G = (np + kSplitSlots - 1) / kSplitSlots;
        const size_t segs = (size_t)c->FM * c->sb.G;
        rc = dev_alloc(&c->sb.seg_max, segs);
        if (rc == PF_OK) rc = dev_alloc(&c->sb.seg_wq, segs * kSplitWaves);
        if (rc == PF_OK) rc = dev_alloc(&c->sb.seg_sum, segs * 6);
    }
    if (rc == PF_OK && trace) {
        rc = dev_alloc(&c->t_pred, c->FM);
        if (rc == PF_OK) rc = dev_alloc(&c->t_v, c->FM);
        if (rc == PF_OK) rc = dev_alloc(&c->t_q, N);
        if (rc == PF_OK) rc = dev_alloc(&c->t_anc, N);
        if (rc == PF_OK) rc = dev_alloc(&c->t_src, N);
        if (rc == PF_OK) rc = dev_alloc(&c->t_prop, 5 * N);
        if (rc == PF_OK) rc = dev_alloc(&c->t_ell, N);
        if (rc == PF_OK) rc = dev_alloc(&c->t_lam, N);
    }
    if (rc == PF_OK && (trace || lineage)) {
        DebugBufs h;
        h.t_pred = c->t_pred;
        h.t_q = c->t_q;
        h.t_anc = c->t_anc;
        h.t_v = c->t_v;
        h.t_src = c->t_src;
        h.t_prop = c->t_prop;
        h.t_ell = c->t_ell;
        h.t_lam = c->t_lam;
        h.lin[0] = c->lin[0];
        h.lin[1] = c->lin[1];
        rc = dev_alloc(&c->d_dbg, 1);
        if (rc == PF_OK && hipMemcpy(c->d_dbg, &h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess)
            rc = PF_EHIP;
    }
    float *d_truth = nullptr;
    if (rc == PF_OK) rc = dev_alloc(&d_truth, 5 * (size_t)F);
    if (rc == PF_OK) {
        void *fn = ctx_step_kernel(c);
        if (!fn ||
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds) !=
                hipSuccess)
            rc = PF_EHIP;
    }
    if (rc == PF_OK && !c->d_dbg && !c->mrec[0] && cfg->launch == PF_LAUNCH_PERSISTENT) {
        // k_run needs every workgroup of the context resident at once.  Its
        // variants must not use private (scratch) memory: the dispatcher may
        // hold back waves of a kernel whose scratch is not yet allocated, and
        // waves waiting at the barrier would then wait for waves that cannot
        // start
        void *fn = pick_run_kernel(c->ppt, c->half, cfg->lik_mode);
        int dev = 0, coop = 0, cus = 0, rate_khz = 0, per_cu = 0;
        hipFuncAttributes fa;
        memset(&fa, 0, sizeof(fa));
        if (fn && hipFuncGetAttributes(&fa, fn) == hipSuccess && fa.localSizeBytes == 0 &&
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds) ==
                hipSuccess &&
            hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) ==
                hipSuccess &&
            hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, (int)c->block, c->lds) ==
                hipSuccess &&
            coop && rate_khz > 0 && (uint64_t)per_cu * (uint64_t)cus >= c->FM) {
            rc = dev_alloc(&c->bar, F);
            if (rc == PF_OK) rc = dev_alloc(&c->run_args, kRunMaxSteps);
            c->run_fn = fn;
            c->bar_timeout = (unsigned long long)rate_khz * 2000ull;   // 2 s
        }
        (void)hipGetLastError();
    }
    if (rc == PF_OK && cfg->launch == PF_LAUNCH_PERSISTENT && !c->run_fn) rc = PF_EUNSUPPORTED;
    if (rc == PF_OK) {
        if (hipMemcpyAsync(d_truth, truth, 5 * F * sizeof(float), hipMemcpyHostToDevice,
                           c->stream) != hipSuccess ||
            hipMemsetAsync(c->err, 0, sizeof(uint32_t), c->stream) != hipSuccess ||
            hipMemsetAsync(c->nex_used, 0, F * sizeof(uint32_t), c->stream) != hipSuccess ||
            (c->arrive &&
             hipMemsetAsync(c->arrive, 0, F * sizeof(uint32_t), c->stream) != hipSuccess))
            rc = PF_EHIP;
    }
    if (rc == PF_OK) {
        const uint64_t work = N > c->FM ? N : c->FM;
        (void)hipGetLastError();   // clear errors of earlier, unrelated calls
        hipLaunchKernelGGL(k_init, dim3((uint32_t)((work + 255) / 256)), dim3(256), 0, c->stream,
                           c->prop[0], c->anc[0], c->rec[0], c->lin[0], d_truth, N, M, np,
                           cfg->width,
                           cfg->height, cfg->init_mode == PF_INIT_INFOSHARE ? 1u : 0u, c->key0,
                           c->key1, (uint32_t)c->FM);
        if (hipGetLastError() != hipSuccess) rc = PF_EHIP;
        if (rc == PF_OK) rc = refresh_master(c, 0);
        if (rc == PF_OK && hipStreamSynchronize(c->stream) != hipSuccess) rc = PF_EHIP;
    }
    if (d_truth) (void)hipFree(d_truth);
    if (rc != PF_OK) {
        free_all(c);
        delete c;
        return rc;
    }
    c->cur = 0;
    c->step = 0;
    *out = c;
    return PF_OK;
}

int pf_step(pf_ctx *c, const float *d_frame) {
    if (!c || !d_frame) return PF_EINVAL;
    return launch_step(c, d_frame);
}

int pf_run(pf_ctx *c, const float *d_frames, uint32_t n_steps, uint64_t frame_stride) {
    if (!c || (!d_frames && n_steps)) return PF_EINVAL;
    return run_steps(c, d_frames, n_steps, frame_stride, nullptr);
}

int pf_run_traj(pf_ctx *c, const float *d_frames, uint32_t n_steps, uint64_t frame_stride,
                pf_master_t *d_traj) {
    if (!c || (!d_frames && n_steps)) return PF_EINVAL;
    if ((uintptr_t)d_traj % alignof(pf_master_t)) return PF_EINVAL;
    return run_steps(c, d_frames, n_steps, frame_stride, nullptr, d_traj);
}

int pf_run_timed(pf_ctx *c, const float *d_frames, uint32_t n_steps, uint64_t frame_stride,
                 float *host_ms_out) {
    if (!c || !host_ms_out || (!d_frames && n_steps)) return PF_EINVAL;
    if (n_steps == 0) return PF_OK;
    return run_steps(c, d_frames, n_steps, frame_stride, host_ms_out);
}

int pf_run_info(const pf_ctx *c, uint32_t *host_multi) {
    if (!c || !host_multi) return PF_EINVAL;
    *host_multi = c->run_fn ? 1u : 0u;
    return PF_OK;
}

int pf_exchange(pf_ctx *c, int64_t *d_src_map) {
    if (!c) return PF_EINVAL;
    if (c->exchanged) return PF_ESTATE;
    const uint64_t k = c->step + 1;
    if (k > 0xFFFFFFFFull) return PF_EUNSUPPORTED;
    int rc = ensure_ring(c, k);
    if (rc != PF_OK) return rc;
    if (d_src_map) {
        StepArgs a = make_args(c, k, nullptr);
        (void)hipGetLastError();   // clear errors of earlier, unrelated calls
        hipLaunchKernelGGL(k_exchange_map, dim3((uint32_t)c->FM), dim3(256), 0, c->stream, a,
                           d_src_map);
        HIP_OK(hipGetLastError());
    }
    c->exchanged = true;
    return PF_OK;
}

int pf_estimate(pf_ctx *c, pf_estimate_t *o) {
    if (!c || !o) return PF_EINVAL;
    const uint32_t F = c->cfg.n_filters;
    int rc = launch_global(c, c->est);
    if (rc != PF_OK) return rc;
    pf_master_t *e = (pf_master_t *)malloc(sizeof(pf_master_t) * F);
    pf_pe_record *rec = nullptr;
    const bool want_pe = o->x_pe || o->log_mass_pe;
    if (want_pe) rec = (pf_pe_record *)malloc(sizeof(pf_pe_record) * c->FM);
    uint32_t err = 0;
    if (!e || (want_pe && !rec)) rc = PF_ENOMEM;
    if (rc == PF_OK &&
        (hipMemcpyAsync(e, c->est, sizeof(pf_master_t) * F, hipMemcpyDeviceToHost, c->stream) !=
             hipSuccess ||
         hipMemcpyAsync(&err, c->err, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream) !=
             hipSuccess ||
         (want_pe && hipMemcpyAsync(rec, cur_rec(c), sizeof(pf_pe_record) * c->FM,
                                    hipMemcpyDeviceToHost, c->stream) != hipSuccess) ||
         hipStreamSynchronize(c->stream) != hipSuccess))
        rc = PF_EHIP;
    if (rc == PF_OK) {
        for (uint32_t f = 0; f < F; ++f) {
            if (o->x_global)
                for (int d = 0; d < 5; ++d) o->x_global[5 * f + d] = e[f].xhat[d];
            if (o->log_mass_glob) o->log_mass_glob[f] = e[f].log_mass_glob;
            if (o->pe_eff) o->pe_eff[f] = e[f].pe_eff;
            if (o->n_ex) o->n_ex[f] = e[f].n_ex;
            if (o->n_ex_next) o->n_ex_next[f] = e[f].n_ex_next;
            if (o->log_z_inc) o->log_z_inc[f] = e[f].log_z_inc;
        }
        if (want_pe)
            for (uint64_t i = 0; i < c->FM; ++i) {
                if (o->log_mass_pe) o->log_mass_pe[i] = rec[i].log_mass;
                if (o->x_pe)
                    for (int d = 0; d < 5; ++d) o->x_pe[5 * i + d] = rec[i].xhat[d];
            }
        o->step = c->step;
        if (err & kErrBarrier)
            rc = PF_ETIMEOUT;
        else if (err)
            rc = PF_ENUMERIC;
    }
    free(e);
    free(rec);
    return rc;
}

void pf_destroy(pf_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

int pf_grad_begin(pf_ctx *c, uint32_t max_steps) {
    if (!c || max_steps == 0) return PF_EINVAL;
    if (c->cfg.lik_mode != PF_LIK_PATCH || c->streamk) return PF_EUNSUPPORTED;
    if (!(c->cfg.q > 0.f)) return PF_EINVAL;
    if (c->g_cap || c->exchanged) return PF_ESTATE;
    const uint64_t N = c->N, FM = c->FM;
    if (max_steps > 0xFFFFFFFFull - c->step) return PF_EUNSUPPORTED;
    int rc = PF_OK;
    if (c->g_alloc < max_steps) {
        HIP_OK(hipStreamSynchronize(c->stream));
        void *old[] = {c->g_prop, c->g_anc, c->g_rec, c->g_nex};
        for (void *q : old)
            if (q) (void)hipFree(q);
        c->g_prop = nullptr;
        c->g_anc = nullptr;
        c->g_rec = nullptr;
        c->g_nex = nullptr;
        c->g_alloc = 0;
        const size_t slots = (size_t)max_steps + 1;
        rc = dev_alloc(&c->g_prop, slots * 5 * N);
        if (rc == PF_OK) rc = dev_alloc(&c->g_anc, slots * N);
        if (rc == PF_OK) rc = dev_alloc(&c->g_rec, slots * FM);
        if (rc == PF_OK) rc = dev_alloc(&c->g_nex, slots * c->cfg.n_filters);
        if (rc != PF_OK) return rc;
        c->g_alloc = max_steps;
    }
    for (int i = 0; i < 2 && rc == PF_OK; ++i) {
        if (!c->g_bar[i]) rc = dev_alloc(&c->g_bar[i], 5 * N);
        if (rc == PF_OK && !c->g_lbar[i]) rc = dev_alloc(&c->g_lbar[i], 2 * FM);
    }
    if (rc == PF_OK && !c->g_theta) rc = dev_alloc(&c->g_theta, 3 * FM);
    if (rc == PF_OK) {
        void *fn = pick_adjoint_kernel(c->adj_ppt, c->half);
        if (!fn || hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)adjoint_lds_bytes(c->cfg.n_per_pe)) != hipSuccess)
            rc = PF_EHIP;
    }
    if (rc == PF_OK && !c->g_out) rc = dev_alloc(&c->g_out, 4 * (size_t)c->cfg.n_filters);
    if (rc != PF_OK) return rc;
    HIP_OK(hipMemcpyAsync(c->g_prop, c->prop[c->cur], 5 * N * sizeof(float),
                          hipMemcpyDeviceToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(c->g_anc, c->anc[c->cur], N * sizeof(uint16_t), hipMemcpyDeviceToDevice,
                          c->stream));
    HIP_OK(hipMemcpyAsync(c->g_rec, c->rec[c->cur], FM * sizeof(pf_pe_record),
                          hipMemcpyDeviceToDevice, c->stream));
    c->g_cap = max_steps;
    c->g_len = 0;
    c->g_start = c->step;
    return PF_OK;
}

int pf_grad_value(pf_ctx *c, double *host_J) {
    if (!c || !host_J) return PF_EINVAL;
    if (!c->g_cap) return PF_ESTATE;
    const uint32_t F = c->cfg.n_filters;
    (void)hipGetLastError();   // clear errors of earlier, unrelated calls
    hipLaunchKernelGGL(k_grad_reduce, dim3(F), dim3(kGradReduceThreads), 0, c->stream, c->g_rec, c->g_len,
                       (const double *)nullptr, c->cfg.n_pe, c->cfg.n_per_pe, (uint32_t)c->FM,
                       c->g_out);
    HIP_OK(hipGetLastError());
    double *tmp = (double *)malloc(sizeof(double) * 4 * F);
    if (!tmp) return PF_ENOMEM;
    int rc = PF_OK;
    if (hipMemcpyAsync(tmp, c->g_out, 4 * F * sizeof(double), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        rc = PF_EHIP;
    if (rc == PF_OK)
        for (uint32_t f = 0; f < F; ++f) host_J[f] = tmp[4 * f];
    free(tmp);
    return rc;
}

int pf_grad_end(pf_ctx *c, const float *d_frames, uint64_t frame_stride, double *host_out) {
    if (!c || !host_out) return PF_EINVAL;
    if (!c->g_cap) return PF_ESTATE;
    const uint32_t F = c->cfg.n_filters, K = c->g_len;
    if (K && !d_frames) return PF_EINVAL;
    const uint64_t N = c->N, FM = c->FM;
    int rc = PF_OK;
    if (K == 0) {
        for (uint32_t i = 0; i < 4 * F; ++i) host_out[i] = 0.0;
    } else {
        void *fn = pick_adjoint_kernel(c->adj_ppt, c->half);
        if (!fn) return PF_EUNSUPPORTED;
        HIP_OK(hipMemsetAsync(c->g_theta, 0, 3 * FM * sizeof(double), c->stream));
        for (uint32_t i = K; i >= 1 && rc == PF_OK; --i) {
            const uint64_t k = c->g_start + i;
            rc = ensure_ring(c, k, true);
            if (rc != PF_OK) break;
            StepArgs a;
            memset(&a, 0, sizeof(a));
            a.rin = c->g_rec + (size_t)(i - 1) * FM;
            a.rout = c->g_rec + (size_t)i * FM;
            a.ring = (c->cfg.mode == PF_MODE_ARNA && c->cfg.n_pe > 1)
                         ? c->ring_tab + (size_t)(k - c->ring_base) * FM
                         : nullptr;
            a.lik = c->lik;
            a.lik.img = d_frames + (size_t)(i - 1) * frame_stride;
            a.dyn = c->dyn;
            a.N = (uint32_t)N;
            a.M = c->cfg.n_pe;
            a.np = c->cfg.n_per_pe;
            a.k = (uint32_t)k;
            a.key0 = c->key0;
            a.key1 = c->key1;
            a.mode = c->cfg.mode;
            a.first = (k == 1) ? 1u : 0u;
            a.fixed_nex = c->fixed_nex;
            a.initial_nex = c->initial_nex;
            a.cutoff_ppm = c->cutoff_ppm;
            a.qmax = c->qmax;
            a.force_nex = c->g_nex + (size_t)i * F;   // N_ex as the forward iteration used it
            AdjArgs g;
            g.xprop = c->g_prop + (size_t)i * 5 * N;
            g.xprev = c->g_prop + (size_t)(i - 1) * 5 * N;
            g.ancprev = c->g_anc + (size_t)(i - 1) * N;
            g.anck = c->g_anc + (size_t)i * N;
            g.rbar_in = (i == K) ? nullptr : c->g_bar[i & 1];
            g.rbar_out = c->g_bar[(i - 1) & 1];
            g.lbar_in = (i == K) ? nullptr : c->g_lbar[i & 1];
            g.lbar_out = c->g_lbar[(i - 1) & 1];
            g.theta = c->g_theta;
            g.sigma = c->cfg.psf_sigma;
            g.inv_2q = 0.5f / c->cfg.q;
            void *args[] = {&a, &g};
            if (hipLaunchKernel(fn, dim3((uint32_t)FM), dim3(c->adj_block), args,
                                adjoint_lds_bytes(c->cfg.n_per_pe), c->stream) != hipSuccess)
                rc = PF_EHIP;
        }
        if (rc == PF_OK) {
            (void)hipGetLastError();   // clear errors of earlier, unrelated calls
            hipLaunchKernelGGL(k_grad_reduce, dim3(F), dim3(kGradReduceThreads), 0, c->stream, c->g_rec, K,
                               (const double *)c->g_theta, c->cfg.n_pe, c->cfg.n_per_pe,
                               (uint32_t)FM, c->g_out);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(host_out, c->g_out, 4 * F * sizeof(double), hipMemcpyDeviceToHost,
                               c->stream) != hipSuccess)
                rc = PF_EHIP;
        }
    }
    // the context continues from the last recorded iteration
    if (hipMemcpyAsync(c->prop[c->cur], c->g_prop + (size_t)K * 5 * N, 5 * N * sizeof(float),
                       hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->anc[c->cur], c->g_anc + (size_t)K * N, N * sizeof(uint16_t),
                       hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->rec[c->cur], c->g_rec + (size_t)K * FM, FM * sizeof(pf_pe_record),
                       hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        rc = PF_EHIP;
    c->g_cap = 0;
    c->g_len = 0;
    return rc;
}

int pf_batch_create(pf_ctx *const *ctxs, uint32_t n, pf_batch **out) {
    if (!out) return PF_EINVAL;
    *out = nullptr;
    if (!ctxs || n == 0) return PF_EINVAL;
    for (uint32_t i = 0; i < n; ++i) {
        if (!ctxs[i] || ctxs[i]->stream != ctxs[0]->stream || ctxs[i]->device != ctxs[0]->device)
            return PF_EINVAL;
        for (uint32_t j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return PF_EINVAL;
    }
    pf_batch *b = new (std::nothrow) pf_batch();
    if (!b) return PF_ENOMEM;
    b->ctx.assign(ctxs, ctxs + n);
    b->stream = ctxs[0]->stream;
    b->n_batched = 0;
    b->d_args = nullptr;
    b->args_cap = 0;
    for (uint32_t i = 0; i < n; ++i) {
        pf_ctx *c = ctxs[i];
        const int kind = c->split ? 2 : (c->flex ? 1 : 0);
        void *fn = kind == 2 ? pick_split_batch_kernel(c->half, c->cfg.lik_mode)
                   : kind == 1 ? pick_flex_batch_kernel(c->half, c->cfg.lik_mode, !c->streamk)
                               : pick_batch_kernel(c->ppt, c->half, c->cfg.lik_mode);
        // (contexts with a once-per-filter master record launch k_master after
        // every step, which a batched group does not: they run one by one)
        if (!fn || c->FM > 0xFFFFFFFFull || c->mrec[0]) {
            b->solo.push_back(i);
            continue;
        }
        const uint32_t block = kind == 2 ? kSplitBlock : c->block;
        pf_batch::Group *g = nullptr;
        for (auto &h : b->groups)
            if (h.fn == fn && h.block == block && h.ppw == c->ppw) g = &h;
        if (!g) {
            pf_batch::Group ng{fn, c->ppt, block, 0, 0, {}, {}, nullptr, kind, c->ppw, nullptr,
                               nullptr};
            b->groups.push_back(ng);
            g = &b->groups.back();
        }
        g->members.push_back(i);
        const size_t lds = kind == 2 ? split_lds_bytes() : c->lds;
        if (lds > g->lds) g->lds = lds;
    }
    int rc = PF_OK;
    for (auto &g : b->groups) {
        uint64_t acc = 0;
        for (uint32_t i : g.members) {
            const pf_ctx *c = b->ctx[i];
            g.first.push_back((uint32_t)acc);
            acc += g.kind == 2 ? c->FM * c->sb.G : (g.kind == 1 ? c->n_wg : c->FM);
        }
        if (acc > 0x7FFFFFFFull) rc = PF_EUNSUPPORTED;
        g.blocks = (uint32_t)acc;
        g.first.push_back((uint32_t)acc);
        b->n_batched += (uint32_t)g.members.size();
        if (rc == PF_OK) rc = dev_alloc(&g.d_first, g.first.size());
        if (rc == PF_OK &&
            hipMemcpy(g.d_first, g.first.data(), g.first.size() * sizeof(uint32_t),
                      hipMemcpyHostToDevice) != hipSuccess)
            rc = PF_EHIP;
        if (rc == PF_OK && hipFuncSetAttribute(g.fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)g.lds) != hipSuccess)
            rc = PF_EHIP;
        // the members' log-weight arrays or split buffers
        if (rc == PF_OK && g.kind == 1) {
            std::vector<float *> u;
            for (uint32_t i : g.members) u.push_back(b->ctx[i]->u);
            rc = dev_alloc(&g.d_u, u.size());
            if (rc == PF_OK && hipMemcpy(g.d_u, u.data(), u.size() * sizeof(float *),
                                         hipMemcpyHostToDevice) != hipSuccess)
                rc = PF_EHIP;
        }
        if (rc == PF_OK && g.kind == 2) {
            std::vector<SplitBufs> sb;
            for (uint32_t i : g.members) sb.push_back(b->ctx[i]->sb);
            rc = dev_alloc(&g.d_sb, sb.size());
            if (rc == PF_OK && hipMemcpy(g.d_sb, sb.data(), sb.size() * sizeof(SplitBufs),
                                         hipMemcpyHostToDevice) != hipSuccess)
                rc = PF_EHIP;
        }
    }
    b->ev_fork = nullptr;
    const size_t lanes = b->groups.size() + b->solo.size();
    const size_t nw = lanes < kBatchStreams ? (lanes ? lanes : 1) : kBatchStreams;
    if (rc == PF_OK && hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess)
        rc = PF_EHIP;
    for (size_t w = 0; w < nw && rc == PF_OK; ++w) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            rc = PF_EHIP;
            break;
        }
        b->workers.push_back(st);
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            rc = PF_EHIP;
            break;
        }
        b->ev_join.push_back(ev);
    }
    if (rc != PF_OK) {
        pf_batch_destroy(b);
        return rc;
    }
    *out = b;
    return PF_OK;
}

}  // extern "C"

namespace {

// One iteration of a batch group: its members' arguments start at ga.
hipError_t launch_group(const pf_batch::Group &g, const StepArgs *ga, hipStream_t st) {
    uint32_t cnt = (uint32_t)g.members.size();
    const uint32_t *first = g.d_first;
    if (g.kind == 0) {
        void *kargs[] = {&ga, &first, &cnt};
        return hipLaunchKernel(g.fn, dim3(g.blocks), dim3(g.block), kargs, g.lds, st);
    }
    if (g.kind == 1) {
        float *const *u = g.d_u;
        uint32_t ppw = g.ppw;
        void *kargs[] = {&ga, &first, &cnt, &u, &ppw};
        return hipLaunchKernel(g.fn, dim3(g.blocks), dim3(g.block), kargs, g.lds, st);
    }
    const SplitBufs *sb = g.d_sb;
    void *kargs[] = {&ga, &first, &cnt, &sb};
    void *fns[] = {g.fn, split_totals_batch_kernel(), split_ancestors_batch_kernel()};
    for (void *fn : fns) {
        const hipError_t e = hipLaunchKernel(fn, dim3(g.blocks), dim3(g.block), kargs, g.lds, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Graph mode of pf_batch_run, in runs of at most kRingSteps iterations.  The
// ring tables are rebuilt before a run when they do not cover it (outside the
// graph), so a run's launches depend only on its length: the graph of the
// batched groups' launches for a length is captured once and replayed, its
// arguments re-read from d_args, which every run rewrites.  The contexts
// launched one by one run beside the graph on a worker stream.
int batch_run_graph(pf_batch *b, const float *const *d_frames, const uint64_t *frame_stride,
                    uint32_t n_steps) {
    const uint32_t nb = b->n_batched;
    const size_t cap = (size_t)kRingSteps * (nb ? nb : 1);
    if (b->args_cap < cap) {
        for (auto &e : b->graphs) (void)hipGraphExecDestroy(e.second);
        b->graphs.clear();
        HIP_OK(hipStreamSynchronize(b->stream));
        if (b->d_args) (void)hipFree(b->d_args);
        b->d_args = nullptr;
        b->args_cap = 0;
        const int rc = dev_alloc(&b->d_args, cap);
        if (rc != PF_OK) return rc;
        b->args_cap = cap;
    }
    const size_t nw = b->workers.size();
    for (uint32_t done = 0; done < n_steps;) {
        const uint32_t n = n_steps - done < kRingSteps ? n_steps - done : kRingSteps;
        // ring tables covering iterations k0 .. k0 + n - 1 of every batched
        // context, enqueued before the graph on the batch's stream
        for (auto &g : b->groups)
            for (uint32_t i : g.members) {
                pf_ctx *c = b->ctx[i];
                if (c->cfg.mode != PF_MODE_ARNA || c->cfg.n_pe <= 1) continue;
                const uint64_t k0 = c->step + 1;
                if (c->ring_valid && k0 >= c->ring_base && k0 + n - 1 < c->ring_base + kRingSteps)
                    continue;
                c->ring_base = k0;
                c->ring_valid = true;
                const int rc = launch_ring(c, k0);
                if (rc != PF_OK) return rc;
            }
        std::vector<StepArgs> args((size_t)n * nb);
        for (uint32_t t = 0; t < n; ++t) {
            uint32_t slot = 0;
            for (auto &g : b->groups)
                for (uint32_t i : g.members) {
                    pf_ctx *c = b->ctx[i];
                    const uint64_t k = c->step + 1;
                    args[(size_t)t * nb + slot++] =
                        make_args(c, k, d_frames[i] + (size_t)(done + t) * frame_stride[i]);
                    advance(c, k);
                }
        }
        HIP_OK(hipStreamSynchronize(b->stream));   // earlier runs may still read d_args
        if (!args.empty())
            HIP_OK(hipMemcpy(b->d_args, args.data(), args.size() * sizeof(StepArgs),
                             hipMemcpyHostToDevice));
        hipGraphExec_t exec = nullptr;
        for (auto &e : b->graphs)
            if (e.first == n) exec = e.second;
        if (!exec && !b->groups.empty()) {
            // capture: a private stream forks to the workers, each group's n
            // launches on its worker, joined back
            hipStream_t cap_st = nullptr;
            HIP_OK(hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking));
            int rc = PF_OK;
            if (hipStreamBeginCapture(cap_st, hipStreamCaptureModeRelaxed) != hipSuccess) rc = PF_EHIP;
            if (rc == PF_OK && hipEventRecord(b->ev_fork, cap_st) != hipSuccess) rc = PF_EHIP;
            for (size_t w = 0; w < nw && rc == PF_OK; ++w)
                if (hipStreamWaitEvent(b->workers[w], b->ev_fork, 0) != hipSuccess) rc = PF_EHIP;
            for (uint32_t t = 0; t < n && rc == PF_OK; ++t) {
                uint32_t slot = 0;
                for (size_t gi = 0; gi < b->groups.size(); ++gi) {
                    auto &g = b->groups[gi];
                    const StepArgs *ga = b->d_args + (size_t)t * nb + slot;
                    if (launch_group(g, ga, b->workers[gi % nw]) != hipSuccess) {
                        rc = PF_EHIP;
                        break;
                    }
                    slot += (uint32_t)g.members.size();
                }
            }
            for (size_t w = 0; w < nw; ++w)
                if (hipEventRecord(b->ev_join[w], b->workers[w]) != hipSuccess ||
                    hipStreamWaitEvent(cap_st, b->ev_join[w], 0) != hipSuccess)
                    rc = PF_EHIP;
            hipGraph_t graph = nullptr;
            if (hipStreamEndCapture(cap_st, &graph) != hipSuccess) rc = PF_EHIP;
            if (rc == PF_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                exec = nullptr;
                rc = PF_EHIP;
            }
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipStreamDestroy(cap_st);
            if (rc != PF_OK) {
                (void)hipGetLastError();
                return rc;
            }
            b->graphs.push_back({n, exec});
        }
        // the contexts without a batched variant run beside the graph, spread
        // over the workers; they are forked before the graph is launched (they
        // depend only on the batch's earlier work) and joined after it
        if (!b->solo.empty()) HIP_OK(hipEventRecord(b->ev_fork, b->stream));
        if (exec) HIP_OK(hipGraphLaunch(exec, b->stream));
        if (!b->solo.empty()) {
            const size_t used = b->solo.size() < nw ? b->solo.size() : nw;
            for (size_t w = 0; w < used; ++w)
                HIP_OK(hipStreamWaitEvent(b->workers[w], b->ev_fork, 0));
            int rc = PF_OK;
            for (size_t si = 0; si < b->solo.size() && rc == PF_OK; ++si) {
                const uint32_t i = b->solo[si];
                pf_ctx *c = b->ctx[i];
                c->stream = b->workers[si % nw];
                for (uint32_t t = 0; t < n && rc == PF_OK; ++t)
                    rc = launch_step(c, d_frames[i] + (size_t)(done + t) * frame_stride[i]);
                c->stream = b->stream;
            }
            for (size_t w = 0; w < used; ++w)
                if (hipEventRecord(b->ev_join[w], b->workers[w]) != hipSuccess ||
                    hipStreamWaitEvent(b->stream, b->ev_join[w], 0) != hipSuccess)
                    rc = PF_EHIP;
            if (rc != PF_OK) return rc;
        }
        done += n;
    }
    return PF_OK;
}

// pf_batch_run; with `fixed` (cap entries) the argument table goes there
// instead of the batch's own buffer, and nothing is allocated on the device.
int batch_run(pf_batch *b, const float *const *d_frames, const uint64_t *frame_stride,
              uint32_t n_steps, int use_graph, StepArgs *fixed, size_t fixed_cap) {
    if (!b || !d_frames || !frame_stride) return PF_EINVAL;
    const uint32_t n = (uint32_t)b->ctx.size();
    for (uint32_t i = 0; i < n; ++i) {
        if (!d_frames[i] && n_steps) return PF_EINVAL;
        if (b->ctx[i]->g_cap) return PF_ESTATE;   // recording runs one context at a time
        if (b->ctx[i]->step + n_steps > 0xFFFFFFFFull) return PF_EUNSUPPORTED;
    }
    if (n_steps == 0) return PF_OK;
    const uint32_t nb = b->n_batched;
    if (fixed && (uint64_t)n_steps * nb > fixed_cap) return PF_EUNSUPPORTED;
    if (use_graph && !fixed) return batch_run_graph(b, d_frames, frame_stride, n_steps);
    // host pass: every batched context's arguments for every iteration, and
    // the ring tables each iteration has to rebuild first (rings[i]: context,
    // first iteration of the new table)
    std::vector<StepArgs> args((size_t)n_steps * nb);
    std::vector<std::vector<std::pair<uint32_t, uint64_t>>> rings(n_steps);
    std::vector<int> saved_cur(n);
    std::vector<uint64_t> saved_step(n), saved_base(n);
    std::vector<bool> saved_valid(n);
    std::vector<const uint32_t *> saved_fa(n), saved_fn(n);
    for (uint32_t i = 0; i < n; ++i) {
        pf_ctx *c = b->ctx[i];
        saved_cur[i] = c->cur;
        saved_step[i] = c->step;
        saved_base[i] = c->ring_base;
        saved_valid[i] = c->ring_valid;
        saved_fa[i] = c->force_anc;
        saved_fn[i] = c->force_nex;
    }
    for (uint32_t t = 0; t < n_steps; ++t) {
        uint32_t slot = 0;
        for (auto &g : b->groups)
            for (uint32_t i : g.members) {
                pf_ctx *c = b->ctx[i];
                const uint64_t k = c->step + 1;
                uint64_t base;
                if (plan_ring(c, k, false, &base)) rings[t].push_back({i, base});
                args[(size_t)t * nb + slot++] =
                    make_args(c, k, d_frames[i] + (size_t)t * frame_stride[i]);
                advance(c, k);
            }
    }
    // the enqueue pass replays the same state changes
    auto restore = [&]() {
        for (uint32_t i = 0; i < n; ++i) {
            pf_ctx *c = b->ctx[i];
            c->cur = saved_cur[i];
            c->step = saved_step[i];
            c->ring_base = saved_base[i];
            c->ring_valid = saved_valid[i];
            c->force_anc = saved_fa[i];
            c->force_nex = saved_fn[i];
        }
    };
    restore();
    if (!fixed && b->args_cap < args.size()) {
        for (auto &e : b->graphs) (void)hipGraphExecDestroy(e.second);
        b->graphs.clear();
        HIP_OK(hipStreamSynchronize(b->stream));
        if (b->d_args) (void)hipFree(b->d_args);
        b->d_args = nullptr;
        b->args_cap = 0;
        const int rc = dev_alloc(&b->d_args, args.size());
        if (rc != PF_OK) return rc;
        b->args_cap = args.size();
    }
    StepArgs *const d_args = fixed ? fixed : b->d_args;
    HIP_OK(hipStreamSynchronize(b->stream));   // earlier runs may still read the table
    HIP_OK(hipMemcpy(d_args, args.data(), args.size() * sizeof(StepArgs), hipMemcpyHostToDevice));
    // graph mode: the launches are captured from a private stream (the legacy
    // stream cannot be captured) and the graph is launched on the batch's
    const hipStream_t run_stream = b->stream;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    if (use_graph) {
        HIP_OK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        if (hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipStreamDestroy(cap);
            return PF_EHIP;
        }
    }
    const hipStream_t base = use_graph ? cap : run_stream;
    const size_t nw = b->workers.size();
    int rc = PF_OK;
    // fork: the workers start after what `base` holds
    if (hipEventRecord(b->ev_fork, base) != hipSuccess) rc = PF_EHIP;
    for (size_t w = 0; w < nw && rc == PF_OK; ++w)
        if (hipStreamWaitEvent(b->workers[w], b->ev_fork, 0) != hipSuccess) rc = PF_EHIP;
    // every context enqueues on its lane's worker (ring rebuilds, solo steps)
    for (size_t gi = 0; gi < b->groups.size(); ++gi)
        for (uint32_t i : b->groups[gi].members) b->ctx[i]->stream = b->workers[gi % nw];
    for (size_t si = 0; si < b->solo.size(); ++si)
        b->ctx[b->solo[si]]->stream = b->workers[(b->groups.size() + si) % nw];
    for (uint32_t t = 0; t < n_steps && rc == PF_OK; ++t) {
        for (auto &r : rings[t]) {
            rc = launch_ring(b->ctx[r.first], r.second);
            if (rc != PF_OK) break;
        }
        uint32_t slot = 0;
        for (size_t gi = 0; gi < b->groups.size(); ++gi) {
            if (rc != PF_OK) break;
            auto &g = b->groups[gi];
            const StepArgs *ga = d_args + (size_t)t * nb + slot;
            const uint32_t cnt = (uint32_t)g.members.size();
            if (launch_group(g, ga, b->workers[gi % nw]) != hipSuccess) rc = PF_EHIP;
            for (uint32_t i : g.members) {
                pf_ctx *c = b->ctx[i];
                const uint64_t k = c->step + 1;
                uint64_t base_k;
                plan_ring(c, k, false, &base_k);   // the table state the host pass assumed
                advance(c, k);
            }
            slot += cnt;
        }
        for (uint32_t i : b->solo) {
            if (rc != PF_OK) break;
            rc = launch_step(b->ctx[i], d_frames[i] + (size_t)t * frame_stride[i]);
        }
    }
    // join: `base` continues after every worker (also after an error, so the
    // capture can end and later work stays ordered)
    for (size_t w = 0; w < nw; ++w)
        if (hipEventRecord(b->ev_join[w], b->workers[w]) != hipSuccess ||
            hipStreamWaitEvent(base, b->ev_join[w], 0) != hipSuccess)
            rc = PF_EHIP;
    for (pf_ctx *c : b->ctx) c->stream = run_stream;
    if (use_graph) {
        const hipError_t e = hipStreamEndCapture(cap, &graph);
        if (rc == PF_OK && e != hipSuccess) rc = PF_EHIP;
        if (rc == PF_OK) {
            hipGraphExec_t exec = nullptr;
            if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess ||
                hipGraphLaunch(exec, run_stream) != hipSuccess ||
                hipStreamSynchronize(run_stream) != hipSuccess)
                rc = PF_EHIP;
            if (exec) (void)hipGraphExecDestroy(exec);
        }
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cap);
        if (rc != PF_OK) (void)hipGetLastError();
    }
    return rc;
}

}  // namespace

extern "C" {

int pf_batch_run(pf_batch *b, const float *const *d_frames, const uint64_t *frame_stride,
                 uint32_t n_steps, int use_graph) {
    return batch_run(b, d_frames, frame_stride, n_steps, use_graph, nullptr, 0);
}

int pf_batch_run_noalloc(pf_batch *b, const float *const *d_frames, const uint64_t *frame_stride,
                         uint32_t n_steps) {
    if (!b) return PF_EINVAL;
    const int dev = b->ctx[0]->device;
    StepArgs *table = (dev >= 0 && dev < kMaxDevices) ? noalloc_args[dev] : nullptr;
    if (!table) return PF_EHIP;
    return batch_run(b, d_frames, frame_stride, n_steps, 0, table, PF_BATCH_NOALLOC_MAX_ARGS);
}

void pf_batch_destroy(pf_batch *b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    for (hipStream_t st : b->workers) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (hipEvent_t ev : b->ev_join) (void)hipEventDestroy(ev);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    for (auto &g : b->groups) {
        if (g.d_first) (void)hipFree(g.d_first);
        if (g.d_u) (void)hipFree(g.d_u);
        if (g.d_sb) (void)hipFree(g.d_sb);
    }
    for (auto &e : b->graphs) (void)hipGraphExecDestroy(e.second);
    if (b->d_args) (void)hipFree(b->d_args);
    delete b;
}

size_t pf_debug_size(const pf_ctx *c, int which) {
    if (!c) return 0;
    const uint64_t N = c->N, FM = c->FM, F = c->cfg.n_filters;
    const bool tr = c->t_q != nullptr;
    switch (which) {
        case PF_DBG_STATE: return 5 * N * sizeof(float);
        case PF_DBG_LOGMASS: return FM * sizeof(double);
        case PF_DBG_PE_RECORDS: return FM * sizeof(pf_pe_record);
        case PF_DBG_NEX: return F * sizeof(uint32_t);
        case PF_DBG_RING: return tr ? FM * sizeof(uint32_t) : 0;
        case PF_DBG_V: return tr ? FM * sizeof(uint32_t) : 0;
        case PF_DBG_SRC: return tr ? N * sizeof(int64_t) : 0;
        case PF_DBG_PROP: return tr ? 5 * N * sizeof(float) : 0;
        case PF_DBG_ELL: return tr ? N * sizeof(float) : 0;
        case PF_DBG_LAMBDA: return tr ? N * sizeof(float) : 0;
        case PF_DBG_Q: return tr ? N * sizeof(uint32_t) : 0;
        case PF_DBG_ANCESTORS: return tr ? N * sizeof(uint32_t) : 0;
        case PF_DBG_LINEAGE: return c->lin[0] ? N * sizeof(int32_t) : 0;
        default: return 0;
    }
}

int pf_debug_get(pf_ctx *c, int which, void *dst, size_t bytes) {
    if (!c || !dst) return PF_EINVAL;
    const size_t need = pf_debug_size(c, which);
    if (need == 0) return (which >= 0 && which <= PF_DBG_LINEAGE) ? PF_ESTATE : PF_EINVAL;
    if (bytes < need) return PF_EINVAL;
    HIP_OK(hipStreamSynchronize(c->stream));
    const void *src = nullptr;
    switch (which) {
        case PF_DBG_STATE: {
            float *tmp = nullptr;
            int rc = dev_alloc(&tmp, 5 * c->N);
            if (rc != PF_OK) return rc;
            (void)hipGetLastError();   // clear errors of earlier, unrelated calls
            hipLaunchKernelGGL(k_materialize, dim3((uint32_t)((c->N + 255) / 256)), dim3(256), 0,
                               c->stream, cur_prop(c), cur_anc(c), tmp, (uint32_t)c->N,
                               c->cfg.n_per_pe);
            if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess ||
                hipMemcpy(dst, tmp, need, hipMemcpyDeviceToHost) != hipSuccess)
                rc = PF_EHIP;
            (void)hipFree(tmp);
            return rc;
        }
        case PF_DBG_PE_RECORDS: src = cur_rec(c); break;
        case PF_DBG_NEX: src = c->nex_used; break;
        case PF_DBG_RING: src = c->t_pred; break;
        case PF_DBG_V: src = c->t_v; break;
        case PF_DBG_SRC: src = c->t_src; break;
        case PF_DBG_PROP: src = c->t_prop; break;
        case PF_DBG_ELL: src = c->t_ell; break;
        case PF_DBG_LAMBDA: src = c->t_lam; break;
        case PF_DBG_Q: src = c->t_q; break;
        case PF_DBG_ANCESTORS: src = c->t_anc; break;
        case PF_DBG_LINEAGE: src = c->lin[c->cur]; break;
        case PF_DBG_LOGMASS: {
            pf_pe_record *rec = (pf_pe_record *)malloc(sizeof(pf_pe_record) * c->FM);
            if (!rec) return PF_ENOMEM;
            if (hipMemcpy(rec, cur_rec(c), sizeof(pf_pe_record) * c->FM,
                          hipMemcpyDeviceToHost) != hipSuccess) {
                free(rec);
                return PF_EHIP;
            }
            for (uint64_t i = 0; i < c->FM; ++i) ((double *)dst)[i] = rec[i].log_mass;
            free(rec);
            return PF_OK;
        }
        default: return PF_EINVAL;
    }
    HIP_OK(hipMemcpy(dst, src, need, hipMemcpyDeviceToHost));
    return PF_OK;
}

int pf_debug_set_state(pf_ctx *c, const float *state, const double *log_mass, uint64_t step) {
    if (!c || !state) return PF_EINVAL;
    if (c->g_cap) return PF_ESTATE;
    HIP_OK(hipStreamSynchronize(c->stream));
    HIP_OK(hipMemcpy(c->prop[c->cur], state, 5 * c->N * sizeof(float), hipMemcpyHostToDevice));
    (void)hipGetLastError();   // clear errors of earlier, unrelated calls
    hipLaunchKernelGGL(k_identity, dim3((uint32_t)((c->N + 255) / 256)), dim3(256), 0, c->stream,
                       c->anc[c->cur], (uint32_t)c->N, c->cfg.n_per_pe);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(c->stream));
    pf_pe_record *rec = (pf_pe_record *)calloc(c->FM, sizeof(pf_pe_record));
    if (!rec) return PF_ENOMEM;
    // x^m of the loaded state: the mean of the PE's particles (it places the
    // next iteration's image tile)
    const uint32_t np = c->cfg.n_per_pe;
    for (uint64_t i = 0; i < c->FM; ++i) {
        rec[i].log_mass = log_mass ? log_mass[i] : 0.0;
        for (int d = 0; d < 5; ++d) {
            double acc = 0.0;
            for (uint32_t j = 0; j < np; ++j) acc += (double)state[(size_t)d * c->N + i * np + j];
            rec[i].xhat[d] = acc / np;
        }
    }
    const hipError_t e =
        hipMemcpy(c->rec[c->cur], rec, sizeof(pf_pe_record) * c->FM, hipMemcpyHostToDevice);
    free(rec);
    HIP_OK(e);
    const int rc = refresh_master(c, c->cur);
    if (rc != PF_OK) return rc;
    HIP_OK(hipStreamSynchronize(c->stream));
    c->step = step;
    c->exchanged = false;
    return PF_OK;
}

int pf_debug_force_next(pf_ctx *c, const uint32_t *d_anc, const uint32_t *d_nex) {
    if (!c) return PF_EINVAL;
    c->force_anc = d_anc;
    c->force_nex = d_nex;
    return PF_OK;
}

int pf_debug_set_lineage(pf_ctx *c, const int32_t *tags) {
    if (!c || !tags) return PF_EINVAL;
    if (!c->lin[0]) return PF_ESTATE;
    HIP_OK(hipStreamSynchronize(c->stream));
    HIP_OK(hipMemcpy(c->lin[c->cur], tags, c->N * sizeof(int32_t), hipMemcpyHostToDevice));
    return PF_OK;
}

int pf_debug_resample_q(const uint32_t *q, uint32_t n_blocks, uint32_t n_p, const uint32_t *v,
                        uint32_t *anc_out) {
    if (!q || !v || !anc_out || n_p == 0 || n_p > PF_MAX_PER_PE_LDS) return PF_EINVAL;
    if (n_blocks == 0) return PF_OK;
    const size_t n = (size_t)n_blocks * n_p;
    for (uint32_t b = 0; b < n_blocks; ++b) {   // reject what the kernel cannot take
        uint64_t T = 0;
        for (uint32_t i = 0; i < n_p; ++i) T += q[(size_t)b * n_p + i];
        if (T == 0 || T > 0xFFFFFFFFull || v[b] >= T) return PF_EINVAL;
    }
    uint32_t *dq = nullptr, *dv = nullptr, *da = nullptr;
    int rc = dev_alloc(&dq, n);
    if (rc == PF_OK) rc = dev_alloc(&dv, n_blocks);
    if (rc == PF_OK) rc = dev_alloc(&da, n);
    if (rc == PF_OK) {
        const uint32_t B = block_of(n_p);
        if (hipMemcpy(dq, q, n * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(dv, v, (size_t)n_blocks * 4, hipMemcpyHostToDevice) != hipSuccess)
            rc = PF_EHIP;
        if (rc == PF_OK) {
            (void)hipGetLastError();   // clear errors of earlier, unrelated calls
            if (n_p > 1024)
                hipLaunchKernelGGL(k_resample_q<4>, dim3(n_blocks), dim3(B), 0, 0, dq, dv, da,
                                   n_p);
            else
                hipLaunchKernelGGL(k_resample_q<1>, dim3(n_blocks), dim3(B), 0, 0, dq, dv, da,
                                   n_p);
            if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
                hipMemcpy(anc_out, da, n * 4, hipMemcpyDeviceToHost) != hipSuccess)
                rc = PF_EHIP;
        }
    }
    if (dq) (void)hipFree(dq);
    if (dv) (void)hipFree(dv);
    if (da) (void)hipFree(da);
    return rc;
}

int pf_debug_nex(const uint32_t *p, uint32_t M, uint32_t n_p, uint32_t mode, float fixed_ratio,
                 float initial_ratio, float eff_cutoff, int first_iteration, uint32_t *nex_out) {
    if (!p || !nex_out || M == 0 || M > PF_MAX_PE || n_p == 0 || n_p > PF_MAX_PER_PE)
        return PF_EINVAL;
    for (uint32_t i = 0; i < M; ++i)
        if (p[i] > (1u << 20)) return PF_EINVAL;
    uint32_t *dp = nullptr, *dout = nullptr;
    int rc = dev_alloc(&dp, M);
    if (rc == PF_OK) rc = dev_alloc(&dout, 1);
    if (rc == PF_OK) {
        if (hipMemcpy(dp, p, M * 4, hipMemcpyHostToDevice) != hipSuccess) rc = PF_EHIP;
        if (rc == PF_OK) {
            (void)hipGetLastError();   // clear errors of earlier, unrelated calls
            hipLaunchKernelGGL(k_nex, dim3(1), dim3(256), 0, 0, dp, M, n_p, mode,
                               first_iteration, fixed_count(fixed_ratio, n_p),
                               fixed_count(initial_ratio, n_p), cutoff_ppm_of(eff_cutoff), dout);
            if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
                hipMemcpy(nex_out, dout, 4, hipMemcpyDeviceToHost) != hipSuccess)
                rc = PF_EHIP;
        }
    }
    if (dp) (void)hipFree(dp);
    if (dout) (void)hipFree(dout);
    return rc;
}

int pf_debug_ring(uint64_t seed, uint32_t f, uint32_t k, uint32_t M, uint32_t mode,
                  uint32_t groups, uint32_t *pred_out) {
    if (!pred_out || M == 0 || M > PF_MAX_PE || groups > 256) return PF_EINVAL;
    if (mode != PF_MODE_ARNA || M == 1) {
        for (uint32_t m = 0; m < M; ++m) pred_out[m] = (m + M - 1) % M;
        return PF_OK;
    }
    // the table kernel for filters 0..f, iteration k (one batch row)
    uint16_t *dt = nullptr;
    int rc = dev_alloc(&dt, (size_t)(f + 1) * M);
    if (rc != PF_OK) return rc;
    (void)hipGetLastError();   // clear errors of earlier, unrelated calls
    hipLaunchKernelGGL(k_ring, dim3(1, f + 1), dim3(256), ring_lds_bytes(M, groups), 0, dt, k,
                       f + 1, M, groups, (uint32_t)seed, (uint32_t)(seed >> 32));
    uint16_t *h = (uint16_t *)malloc((size_t)M * 2);
    if (!h) rc = PF_ENOMEM;
    if (rc == PF_OK &&
        (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
         hipMemcpy(h, dt + (size_t)f * M, (size_t)M * 2, hipMemcpyDeviceToHost) != hipSuccess))
        rc = PF_EHIP;
    if (rc == PF_OK)
        for (uint32_t m = 0; m < M; ++m) pred_out[m] = h[m];
    free(h);
    (void)hipFree(dt);
    return rc;
}

int pf_debug_philox(const uint32_t *ctr, const uint32_t *key, uint32_t n, uint32_t *out) {
    if (!ctr || !key || !out) return PF_EINVAL;
    if (n == 0) return PF_OK;
    uint32_t *dc = nullptr, *dout = nullptr;
    int rc = dev_alloc(&dc, (size_t)4 * n);
    if (rc == PF_OK) rc = dev_alloc(&dout, (size_t)4 * n);
    if (rc == PF_OK) {
        if (hipMemcpy(dc, ctr, (size_t)16 * n, hipMemcpyHostToDevice) != hipSuccess) rc = PF_EHIP;
        if (rc == PF_OK) {
            (void)hipGetLastError();   // clear errors of earlier, unrelated calls
            hipLaunchKernelGGL(k_philox, dim3((n + 255) / 256), dim3(256), 0, 0, dc, key[0],
                               key[1], n, dout);
            if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
                hipMemcpy(out, dout, (size_t)16 * n, hipMemcpyDeviceToHost) != hipSuccess)
                rc = PF_EHIP;
        }
    }
    if (dc) (void)hipFree(dc);
    if (dout) (void)hipFree(dout);
    return rc;
}

}  // extern "C"
