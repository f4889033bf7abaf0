// arna.hip -- kernels and host runtime of the ARNA particle-filter step on
// MI355X (gfx950), exported through the C interface in include/arna.h.
//
// Data layout in HBM (one context):
//   state[2][5][N] float32   ping-pong particle buffers, component-major
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

#include <new>

#include "arna.h"
#include "arna_device.hpp"

using namespace arna;

namespace {

constexpr uint32_t kRingSteps = 64;     // iterations per ring-table batch
constexpr int kRedDoubles = 128;        // LDS reduction scratch (>= 16 waves x 8)

struct EstDev {                         // written by k_global, one per filter
    double xhat[5];
    double log_mass_glob;
    double pe_eff;
    double log_z;
    uint32_t n_ex_next;
    uint32_t pad;
};

// Buffers kept only in debug modes (one device copy per context).
struct DebugBufs {
    // trace of the last iteration (PF_DEBUG_TRACE), else NULL
    uint32_t *t_pred, *t_q, *t_anc, *t_v;
    int64_t *t_src;
    float *t_prop, *t_ell, *t_lam;
    // lineage tags, ping-pong like the state (PF_DEBUG_LINEAGE), else NULL
    int32_t *lin[2];
};

struct StepArgs {
    const float *sin;                   // [5][N] resampled particles of k-1
    float *sout;                        // [5][N] resampled particles of k
    const pf_pe_record *rin;            // [F*M] records of k-1
    pf_pe_record *rout;                 // [F*M] records of k
    const uint16_t *ring;               // [F*M] pred(m) for this k, or NULL (fixed ring)
    const DebugBufs *dbg;               // NULL unless a debug mode is on
    Lik lik;
    Dyn dyn;
    uint32_t N;                         // F M N_p (< 2^31)
    uint32_t M, np, np_top;             // np_top: largest power of two <= N_p
    uint32_t k, key0, key1;
    uint32_t mode, first, fixed_nex, initial_nex, cutoff_ppm, qmax;
    uint32_t lin_in;                    // which lineage buffer holds iteration k-1
    double inv_np;                      // 1 / N_p
    uint32_t *err;                      // sticky numeric-error flag
    uint32_t *nex_used;                 // [F]
};

// What a PE knows after steps 1-2 (and the inputs of steps 3-4).
struct Prologue {
    uint32_t pred, nex, c_own, c_pred;
    float lam_own, lam_pred;
};

// Steps 1-2 and the renormalization constant of step 4, computed by one wave
// of every workgroup from the M records of the previous iteration:
//   L_glob = log sum_m W^(m)_{k-1},  P_m = floor(exp(L_m - max L) 2^20),
//   S = sum P, D = sum P^2  ->  N_ex (Eq. 3 with PE_eff = S^2 / D).
// Lane 0 writes the result to `out`.
__device__ void prologue_wave(const StepArgs &a, uint32_t f, uint32_t m, Prologue *out) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t M = a.M;
    const pf_pe_record *R = a.rin + (size_t)f * M;
    double lmax = -INFINITY;
    for (uint32_t i = lane; i < M; i += kWave) lmax = fmax(lmax, R[i].log_mass);
    lmax = wave_max_d(lmax);
    double acc = 0.0;
    uint64_t S = 0, D = 0;
    if (lmax != -INFINITY) {
        for (uint32_t i = lane; i < M; i += kWave) {
            const double e = exp(R[i].log_mass - lmax);
            acc += e;
            const uint64_t P = (uint64_t)floor(e * 1048576.0);
            S += P;
            D += P * P;
        }
    }
    acc = wave_sum(acc);
    S = wave_sum_u64(S);
    D = wave_sum_u64(D);
    if (lane == 0) {
        Prologue p;
        p.pred = (M == 1) ? m : (a.ring ? (uint32_t)a.ring[(size_t)f * M + m] : (m + M - 1) % M);
        p.nex = exchange_count(S, D, M, a.np, a.mode, (int)a.first, a.fixed_nex, a.initial_nex,
                               a.cutoff_ppm);
        if (p.nex > a.np) p.nex = a.np;
        const double lglob = (lmax == -INFINITY) ? -INFINITY : lmax + log(acc);
        if (lglob == -INFINITY) {
            p.lam_own = 0.f;
            p.lam_pred = 0.f;
        } else {
            p.lam_own = (float)(R[m].log_mass - lglob);
            p.lam_pred = (float)(R[p.pred].log_mass - lglob);
        }
        p.c_own = mulshift(philox(m, a.k, f, kTagExch << 24, a.key0, a.key1).x, a.np);
        p.c_pred = mulshift(philox(p.pred, a.k, f, kTagExch << 24, a.key0, a.key1).x, a.np);
        *out = p;
    }
}

// Step 3: PE m sends its slots s_t(m) = floor((t N_p + c_m) / N_ex), t < N_ex,
// and refills them with the slots s_t(pred(m)) that pred(m) sends.  The map
// recv[s_t(m)] = s_t(pred(m)) is built in LDS (0xFFFF = slot keeps its own
// particle); `recv` must hold 0xFFFF for every slot on entry.
__device__ __forceinline__ void build_receive_map(uint16_t *recv, const Prologue &p, uint32_t np) {
    for (uint32_t t = threadIdx.x; t < p.nex; t += blockDim.x) {
        const uint32_t dst = (t * np + p.c_own) / p.nex;
        const uint32_t src = (t * np + p.c_pred) / p.nex;
        recv[dst] = (uint16_t)src;
    }
}

// LDS image tile: 64 columns, up to 64 rows; holds z - B, zero outside the
// image.  The row pitch is 11 mod 32 (and mod 64), so the patch origins of a
// cluster of particles, which differ by a few rows and columns, fall on
// different LDS banks.
constexpr int kTileCols = 64, kTilePitch = 75, kTileRows = 64;
constexpr int kMaxWaves = 16;

// Dynamic LDS layout of k_step.
struct Lds {
    Prologue *pro;     // 1
    int *box;          // 4 (+4 pad)
    float *wmax;       // [16] wave maxima
    uint32_t *wq;      // [16][4] wave totals of Q, per slot level
    double *wsum;      // [16][6] wave sums (W, W x)
    float *st;         // [5][np] propagated particles
    uint32_t *cq;      // [np] inclusive sums C of the fixed-point weights
    float *tile;       // [kTileRows][kTilePitch]
    int32_t *lin;      // [np] (lineage only)
};
__device__ __forceinline__ Lds carve(unsigned char *base, uint32_t np) {
    Lds l;
    size_t o = 0;
    l.wsum = (double *)(base + o);
    o += kMaxWaves * 6 * sizeof(double);
    l.pro = (Prologue *)(base + o);
    o += 32;
    l.box = (int *)(base + o);
    o += 32;
    l.wmax = (float *)(base + o);
    o += kMaxWaves * sizeof(float);
    l.wq = (uint32_t *)(base + o);
    o += kMaxWaves * 4 * sizeof(uint32_t);
    l.st = (float *)(base + o);
    o += 5 * (size_t)np * sizeof(float);
    l.cq = (uint32_t *)(base + o);
    o += (size_t)np * sizeof(uint32_t);
    l.tile = (float *)(base + o);
    o += (size_t)kTileRows * kTilePitch * sizeof(float);
    l.lin = (int32_t *)(base + o);
    return l;
}
__host__ __device__ constexpr size_t lds_fixed_bytes() {
    return kMaxWaves * 6 * sizeof(double) + 32 + 32 + kMaxWaves * sizeof(float) +
           kMaxWaves * 4 * sizeof(uint32_t) + (size_t)kTileRows * kTilePitch * sizeof(float);
}

// Step 7 building blocks, shared by k_step and the debug entry point.
// Thread t holds the fixed-point weights of slots t + q B (q < PPT).
// Part 1: inclusive scans within each wave, per level q; the last lane of each
// wave leaves the wave totals in wq[wave][q].
template <int PPT>
__device__ __forceinline__ void scan_levels(const uint32_t (&Q)[PPT], uint32_t (&cinc)[PPT],
                                            uint32_t *wq) {
    const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < PPT; ++q) cinc[q] = wave_incl_scan_u32(Q[q]);
    if (lane == kWave - 1)
#pragma unroll
        for (int q = 0; q < PPT; ++q) wq[wave * 4 + q] = cinc[q];
}
// Part 2 (after a barrier): inclusive sums C in slot order written to C[],
// returns the total T.
template <int PPT>
__device__ __forceinline__ uint32_t scan_finish(const uint32_t (&cinc)[PPT], const uint32_t *wq,
                                                uint32_t *C, uint32_t np) {
    const uint32_t wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
    uint32_t T = 0;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        uint32_t level = 0, prior = 0;
        for (uint32_t w = 0; w < nwaves; ++w) {
            const uint32_t t = wq[w * 4 + q];
            level += t;
            if (w < wave) prior += t;
        }
        const uint32_t s = threadIdx.x + q * blockDim.x;
        if (s < np) C[s] = T + prior + cinc[q];
        T += level;
    }
    return T;
}
// Part 3 (after a barrier): ancestors of the outputs j = t + q B.
template <int PPT>
__device__ __forceinline__ void ancestors(const uint32_t *C, uint32_t np, uint32_t T, uint32_t V,
                                          uint32_t np_top, double inv_np, uint32_t (&anc)[PPT]) {
#pragma unroll
    for (int q = 0; q < PPT; ++q) {   // independent searches, interleaved
        const uint32_t j = threadIdx.x + q * blockDim.x;
        const uint32_t tau = div_floor((uint64_t)j * T + V, np, inv_np);
        anc[q] = (j < np) ? systematic_ancestor(C, np, tau, np_top) : 0u;
    }
}

// One ARNA / RNA iteration; one workgroup = one PE (f, m).  Thread t owns the
// slots s = t + q B, q < PPT (B = blockDim.x), so every global access of a
// slot level is coalesced.
template <int PPT, int HALF, bool POINT>
__global__ __launch_bounds__(1024) void k_step(StepArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int P = 2 * HALF + 1;
    const uint32_t M = a.M, np = a.np, N = a.N;
    const uint32_t f = blockIdx.x / M, m = blockIdx.x % M;
    const uint32_t tid = threadIdx.x, B = blockDim.x;
    const uint32_t lane = tid & (kWave - 1), wave = tid / kWave, nwaves = B / kWave;
    Lds L = carve(smem, np);
    uint16_t *recv = (uint16_t *)L.tile;   // receive map; the tile is loaded later
    const uint32_t pe_base = blockIdx.x * np;   // (f M + m) N_p
    const DebugBufs *D = a.dbg;
    const int32_t *lin_in = D ? D->lin[a.lin_in] : nullptr;
    int32_t *lin_out = D ? D->lin[1 - a.lin_in] : nullptr;
    const bool trace = D && D->t_q;

    // ---- phase 0: wave 0 redoes the master step of iteration k-1 (steps
    // 1-2); every thread issues the loads of its own slots (most slots keep
    // their particle) and draws the step-5 normals while they are in flight.
    if (tid < kWave) prologue_wave(a, f, m, L.pro);
    if (tid == 0) {
        L.box[0] = INT_MAX;
        L.box[1] = INT_MIN;
        L.box[2] = INT_MAX;
        L.box[3] = INT_MIN;
    }
    float x[PPT][5];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const uint32_t s = tid + q * B;
        if (s < np) {
            recv[s] = 0xFFFF;
#pragma unroll
            for (int c = 0; c < 5; ++c) x[q][c] = a.sin[c * N + pe_base + s];
        }
    }
    float e[PPT][5];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const uint32_t s = tid + q * B;
        if (s < np)
            five_normals(philox(m * np + s, a.k, f, kTagProp << 24, a.key0, a.key1), e[q]);
    }
    __syncthreads();   // barrier 1: prologue visible, receive map cleared
    const Prologue p = *L.pro;
    if (p.nex) {
        build_receive_map(recv, p, np);
        __syncthreads();   // barrier 1b: receive map
    }

    // ---- phase 1 (steps 3-5 P): received slots are refetched from pred(m);
    // propagate; stage in LDS; bounding box of the patch origins.
    int bx0 = INT_MAX, bx1 = INT_MIN, by0 = INT_MAX, by1 = INT_MIN;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const uint32_t s = tid + q * B;
        if (s >= np) continue;
        uint32_t gsrc = pe_base + s;
        float lam = p.lam_own;
        const uint32_t r = p.nex ? recv[s] : 0xFFFFu;
        if (r != 0xFFFFu) {
            gsrc = (f * M + p.pred) * np + r;
            lam = p.lam_pred;
#pragma unroll
            for (int c = 0; c < 5; ++c) x[q][c] = a.sin[c * N + gsrc];
        }
        if (lin_in) L.lin[s] = lin_in[gsrc];
        if (trace) {
            D->t_src[pe_base + s] = (int64_t)gsrc;
            D->t_lam[pe_base + s] = lam;
        }
        propagate(x[q], e[q], a.dyn);
#pragma unroll
        for (int c = 0; c < 5; ++c) L.st[c * np + s] = x[q][c];
        L.cq[s] = __float_as_uint(lam);   // parked until the likelihood is known
        if (!POINT) {
            int u0, v0;
            if (patch_origin<HALF>(x[q][0], x[q][1], a.lik.W, a.lik.H, u0, v0)) {
                bx0 = min(bx0, u0);
                bx1 = max(bx1, u0);
                by0 = min(by0, v0);
                by1 = max(by1, v0);
            }
        }
    }
    bool use_tile = false, tile_inside = false;
    int tx0 = 0, ty0 = 0;
    if (!POINT) {
        bx0 = wave_min_i32(bx0);
        bx1 = wave_max_i32(bx1);
        by0 = wave_min_i32(by0);
        by1 = wave_max_i32(by1);
        if (lane == 0 && bx0 <= bx1) {
            atomicMin(&L.box[0], bx0);
            atomicMax(&L.box[1], bx1);
            atomicMin(&L.box[2], by0);
            atomicMax(&L.box[3], by1);
        }
        __syncthreads();   // barrier 2: bounding box (receive map no longer read)
        tx0 = L.box[0];
        ty0 = L.box[2];
        int th = 0;
        if (tx0 <= L.box[1]) {   // at least one patch touches the image
            const int tw = L.box[1] - tx0 + P;
            th = L.box[3] - ty0 + P;
            use_tile = tw <= kTileCols && th <= kTileRows;
            tile_inside = tx0 >= 0 && ty0 >= 0 && tx0 + tw <= a.lik.W && ty0 + th <= a.lik.H;
        }
        if (use_tile) {
            // tile pixel (r, c) is image pixel (tx0 + c, ty0 + r)
            for (int idx = (int)tid; idx < th * kTileCols; idx += (int)B) {
                const int r = idx / kTileCols, c = idx % kTileCols;
                const int u = tx0 + c, v = ty0 + r;
                const bool in = (unsigned)u < (unsigned)a.lik.W && (unsigned)v < (unsigned)a.lik.H;
                L.tile[r * kTilePitch + c] =
                    in ? a.lik.img[(size_t)v * a.lik.W + u] - a.lik.bg : 0.f;
            }
            __syncthreads();   // barrier 3: tile
        }
    } else {
        __syncthreads();   // barrier 2: LDS staging complete
    }

    // ---- phase 2 (step 5 U): log-likelihood of every slot; u = lambda + l,
    // one slot at a time (the particle comes back from LDS), u parked in LDS.
    float umax = -INFINITY;
    bool bad = false;
#pragma unroll 1
    for (int q = 0; q < PPT; ++q) {
        const uint32_t s = tid + q * B;
        if (s >= np) break;
        float xs[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) xs[c] = L.st[c * np + s];
        float ell;
        if (POINT) {
            ell = loglik_point(xs, a.lik, f);
        } else if (use_tile) {
            int u0, v0;
            ell = 0.f;
            if (patch_origin<HALF>(xs[0], xs[1], a.lik.W, a.lik.H, u0, v0)) {
                const float *pix = L.tile + (v0 - ty0) * kTilePitch + (u0 - tx0);
                ell = tile_inside
                          ? patch_loglik<HALF, kFromTileInside>(xs, u0, v0, pix, kTilePitch, a.lik)
                          : patch_loglik<HALF, kFromTile>(xs, u0, v0, pix, kTilePitch, a.lik);
            }
        } else {
            ell = loglik_patch<HALF>(xs, a.lik);
        }
        bad |= (ell != ell);
        const float uu = __uint_as_float(L.cq[s]) + ell;
        umax = fmaxf(umax, uu);
        L.cq[s] = __float_as_uint(uu);
        if (trace) {
            D->t_ell[pe_base + s] = ell;
#pragma unroll
            for (int c = 0; c < 5; ++c) D->t_prop[c * N + pe_base + s] = xs[c];
        }
    }
    if (__any(bad) && lane == 0) atomicOr(a.err, 1u);
    umax = wave_max_f32(umax);
    if (lane == 0) L.wmax[wave] = umax;
    __syncthreads();   // barrier 4: wave maxima
    float lstar = L.wmax[0];
    for (uint32_t w = 1; w < nwaves; ++w) lstar = fmaxf(lstar, L.wmax[w]);

    // ---- phase 3 (steps 6-7): weights relative to lstar, fixed-point
    // Q = floor(w Q_max), per-PE sums in FP64, inclusive prefix sums of Q in
    // slot order (level q of thread t is slot t + q B).
    const float qmaxf = (float)a.qmax;
    double sums[6] = {0, 0, 0, 0, 0, 0};
    uint32_t Qv[PPT], cinc[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const uint32_t s = tid + q * B;
        Qv[q] = 0;
        if (s < np) {
            const float w =
                (lstar == -INFINITY) ? 1.0f : __expf(__uint_as_float(L.cq[s]) - lstar);
            float qf = floorf(w * qmaxf);
            qf = (qf >= 0.f) ? fminf(qf, qmaxf) : 0.f;
            Qv[q] = (uint32_t)qf;
            const double wd = (double)w;
            sums[0] += wd;
#pragma unroll
            for (int c = 0; c < 5; ++c) sums[1 + c] += wd * (double)L.st[c * np + s];
            if (trace) D->t_q[pe_base + s] = Qv[q];
        }
    }
    scan_levels<PPT>(Qv, cinc, L.wq);
#pragma unroll
    for (int c = 0; c < 6; ++c) sums[c] = wave_total_f64(sums[c]);
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < 6; ++c) L.wsum[wave * 6 + c] = sums[c];
    }
    __syncthreads();   // barrier 5: wave totals
    const uint32_t T = scan_finish<PPT>(cinc, L.wq, L.cq, np);
    const uint32_t V = mulshift(philox(m, a.k, f, kTagResample << 24, a.key0, a.key1).x, T);
    __syncthreads();   // barrier 6: C complete

    // ---- phase 4 (step 7): ancestors by search over C, gather from LDS.
    uint32_t anc[PPT];
    ancestors<PPT>(L.cq, np, T, V, a.np_top, a.inv_np, anc);
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const uint32_t j = tid + q * B;
        if (j >= np) continue;
#pragma unroll
        for (int c = 0; c < 5; ++c) a.sout[c * N + pe_base + j] = L.st[c * np + anc[q]];
        if (lin_out) lin_out[pe_base + j] = L.lin[anc[q]];
        if (trace) D->t_anc[pe_base + j] = anc[q];
    }

    // ---- steps 8-9: every particle now carries W^(m)_k; publish the record
    if (tid == 0) {
        double tot[6] = {0, 0, 0, 0, 0, 0};
        for (uint32_t w = 0; w < nwaves; ++w)
            for (int c = 0; c < 6; ++c) tot[c] += L.wsum[w * 6 + c];
        pf_pe_record r;
        r.log_mass = (lstar == -INFINITY) ? -INFINITY : (double)lstar + log(tot[0]);
        for (int c = 0; c < 5; ++c) r.xhat[c] = tot[1 + c] / tot[0];
        r.lstar = lstar;
        r.total_q = T;
        a.rout[blockIdx.x] = r;
        if (m == 0) a.nex_used[f] = p.nex;
        if (trace) {
            D->t_pred[blockIdx.x] = p.pred;
            D->t_v[blockIdx.x] = V;
        }
    }
}

// Step 1 for kRingSteps iterations at once: Fisher-Yates (Durstenfeld,
// i = M-1 .. 1, j = floor(r_i (i + 1) / 2^32)) over the M labels; the ring
// visits perm[0], perm[1], ... and closes.  Grid (steps, F).
__global__ __launch_bounds__(256) void k_ring(uint16_t *tab, uint32_t base, uint32_t F,
                                              uint32_t M, uint32_t key0, uint32_t key1) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t *perm = (uint16_t *)smem;
    uint16_t *jd = perm + M;
    const uint32_t k = base + blockIdx.x, f = blockIdx.y;
    for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) {
        perm[i] = (uint16_t)i;
        jd[i] = (i == 0) ? 0 : (uint16_t)mulshift(philox(i, k, f, kTagRing << 24, key0, key1).x,
                                                  i + 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t i = M - 1; i >= 1; --i) {
            const uint32_t j = jd[i];
            const uint16_t t = perm[i];
            perm[i] = perm[j];
            perm[j] = t;
        }
    }
    __syncthreads();
    uint16_t *out = tab + ((size_t)blockIdx.x * F + f) * M;
    for (uint32_t t = threadIdx.x; t < M; t += blockDim.x)
        out[perm[t]] = perm[(t + M - 1) % M];
}

// Initialization (Sec. V).  Tracking: every particle at the truth.
// Information sharing: PE 0 uniform in the radius-2 disk around the true
// position with the true velocity and intensity; other PEs uniform over the
// image, velocity in [-2, 2]^2, intensity in [0, 2 I].
__global__ void k_init(float *st, pf_pe_record *rec, int32_t *lin, const float *truth,
                       uint64_t N, uint32_t M, uint32_t np, uint32_t W, uint32_t H,
                       uint32_t infoshare, uint32_t key0, uint32_t key1, uint32_t FM) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < FM) {
        pf_pe_record r = {};
        r.log_mass = 0.0;
        rec[g] = r;
    }
    if (g >= N) return;
    const uint32_t pe = (uint32_t)(g / np), s = (uint32_t)(g % np);
    const uint32_t f = pe / M, m = pe % M;
    const float *t = truth + 5 * f;
    float v[5] = {t[0], t[1], t[2], t[3], t[4]};
    if (infoshare) {
        const uint32_t j = m * np + s;
        const u4 r0 = philox(j, 0, f, (kTagInit << 24) | 0u, key0, key1);
        const u4 r1 = philox(j, 0, f, (kTagInit << 24) | 1u, key0, key1);
        if (m == 0) {
            const float rad = 2.0f * __builtin_sqrtf(unif24(r0.x));
            const float ang = unif24(r0.y);
            v[0] = t[0] + rad * cos_rev(ang);
            v[1] = t[1] + rad * sin_rev(ang);
        } else {
            v[0] = -0.5f + (float)W * unif24(r0.x);
            v[1] = -0.5f + (float)H * unif24(r0.y);
            v[2] = -2.0f + 4.0f * unif24(r0.z);
            v[3] = -2.0f + 4.0f * unif24(r0.w);
            v[4] = 2.0f * t[4] * unif24(r1.x);
        }
    }
    for (int c = 0; c < 5; ++c) st[c * N + g] = v[c];
    if (lin) lin[g] = (int32_t)m;
}

// Master step of iteration k (Alg. 3, steps 9-10) for reporting: W_k, the
// global estimate x_k = sum_m W^(m) x^m / W_k, PE_eff and the next N_ex.
__global__ __launch_bounds__(256) void k_global(const pf_pe_record *rec, EstDev *est,
                                                uint32_t M, uint32_t np, uint32_t mode,
                                                uint32_t fixed_nex, uint32_t cutoff_ppm) {
    __shared__ double red[kRedDoubles];
    const uint32_t f = blockIdx.x;
    const pf_pe_record *R = rec + (size_t)f * M;
    double lmax = -INFINITY;
    for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) lmax = fmax(lmax, R[i].log_mass);
    lmax = block_max_d(lmax, red);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    uint64_t sd[2] = {0, 0};
    if (lmax != -INFINITY) {
        for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) {
            const double e = exp(R[i].log_mass - lmax);
            const uint64_t P = (uint64_t)floor(e * 1048576.0);
            sd[0] += P;
            sd[1] += P * P;
            acc[0] += e;
            if (e > 0.0)
                for (int c = 0; c < 5; ++c) acc[1 + c] += e * R[i].xhat[c];
        }
    }
    block_sum<6>(acc, red);
    block_sum_u64(sd, (uint64_t *)red);
    if (threadIdx.x == 0) {
        EstDev o;
        o.log_mass_glob = (lmax == -INFINITY) ? -INFINITY : lmax + log(acc[0]);
        for (int c = 0; c < 5; ++c) o.xhat[c] = acc[1 + c] / acc[0];
        o.pe_eff = sd[1] ? (double)sd[0] * (double)sd[0] / (double)sd[1] : 0.0;
        o.log_z = o.log_mass_glob - log((double)np);
        o.n_ex_next = exchange_count(sd[0], sd[1], M, np, mode, 0, fixed_nex, 0, cutoff_ppm);
        o.pad = 0;
        est[f] = o;
    }
}

// pf_exchange: steps 1-3 of the next iteration, exported as a source map.
__global__ __launch_bounds__(256) void k_exchange_map(StepArgs a, int64_t *src) {
    __shared__ Prologue pro;
    __shared__ uint16_t recv[PF_MAX_PER_PE];
    const uint32_t f = blockIdx.x / a.M, m = blockIdx.x % a.M;
    if (threadIdx.x < kWave) prologue_wave(a, f, m, &pro);
    for (uint32_t s = threadIdx.x; s < a.np; s += blockDim.x) recv[s] = 0xFFFF;
    __syncthreads();
    const Prologue p = pro;
    build_receive_map(recv, p, a.np);
    __syncthreads();
    for (uint32_t s = threadIdx.x; s < a.np; s += blockDim.x) {
        const uint32_t r = recv[s];
        const uint64_t g = (r == 0xFFFFu) ? (uint64_t)blockIdx.x * a.np + s
                                          : ((uint64_t)f * a.M + p.pred) * a.np + r;
        src[(uint64_t)blockIdx.x * a.np + s] = (int64_t)g;
    }
}

// Debug entry points: the integer stages alone, same device code as k_step.
template <int PPT>
__global__ __launch_bounds__(1024) void k_resample_q(const uint32_t *q, const uint32_t *v,
                                                     uint32_t *anc_out, uint32_t np,
                                                     uint32_t np_top, double inv_np) {
    __shared__ uint32_t wq[kMaxWaves * 4];
    __shared__ uint32_t C[PF_MAX_PER_PE];
    const uint32_t base = blockIdx.x * np;
    uint32_t Qv[PPT], cinc[PPT], anc[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint32_t s = threadIdx.x + k * blockDim.x;
        Qv[k] = (s < np) ? q[base + s] : 0u;
    }
    scan_levels<PPT>(Qv, cinc, wq);
    __syncthreads();
    const uint32_t T = scan_finish<PPT>(cinc, wq, C, np);
    __syncthreads();
    const uint32_t V = v[blockIdx.x];
    ancestors<PPT>(C, np, T, V, np_top, inv_np, anc);
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint32_t j = threadIdx.x + k * blockDim.x;
        if (j < np) anc_out[base + j] = anc[k];
    }
}

__global__ __launch_bounds__(256) void k_nex(const uint32_t *P, uint32_t M, uint32_t np,
                                             uint32_t mode, int first, uint32_t fixed_nex,
                                             uint32_t initial_nex, uint32_t cutoff_ppm,
                                             uint32_t *out) {
    __shared__ uint64_t red[64];
    uint64_t sd[2] = {0, 0};
    for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) {
        sd[0] += P[i];
        sd[1] += (uint64_t)P[i] * P[i];
    }
    block_sum_u64(sd, red);
    if (threadIdx.x == 0)
        *out = exchange_count(sd[0], sd[1], M, np, mode, first, fixed_nex, initial_nex,
                              cutoff_ppm);
}

__global__ void k_philox(const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t n,
                         uint32_t *out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u4 r = philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
    out[4 * i] = r.x;
    out[4 * i + 1] = r.y;
    out[4 * i + 2] = r.z;
    out[4 * i + 3] = r.w;
}

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
size_t step_lds(uint32_t np, bool lineage) {
    return lds_fixed_bytes() + 5 * (size_t)np * 4 + (size_t)np * 4 +
           (lineage ? (size_t)np * 4 : 0);
}

}  // namespace

struct pf_ctx {
    pf_config cfg;
    hipStream_t stream;
    uint64_t N, FM;
    uint32_t block, ppt, half;
    size_t lds;
    float *state[2];
    pf_pe_record *rec[2];
    int32_t *lin[2];
    int cur;                       // buffers holding iteration `step`
    uint16_t *ring_tab;
    uint64_t ring_base;
    bool ring_valid;
    uint32_t *err, *nex_used;
    EstDev *est;
    DebugBufs *d_dbg;              // device copy of the debug-buffer table, or NULL
    // trace buffers
    uint32_t *t_pred, *t_q, *t_anc, *t_v;
    int64_t *t_src;
    float *t_prop, *t_ell, *t_lam;
    uint64_t step;
    bool exchanged;
    uint32_t key0, key1, fixed_nex, initial_nex, cutoff_ppm, qmax;
    Dyn dyn;
    Lik lik;
};

namespace {

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

template <int PPT, int HALF, bool POINT>
void *step_kernel() {
    return reinterpret_cast<void *>(&k_step<PPT, HALF, POINT>);
}

void *pick_step_kernel(uint32_t ppt, uint32_t half, bool point) {
#define ARNA_HALVES(P)                            \
    switch (half) {                               \
        case 0: return step_kernel<P, 0, false>(); \
        case 1: return step_kernel<P, 1, false>(); \
        case 2: return step_kernel<P, 2, false>(); \
        case 3: return step_kernel<P, 3, false>(); \
        case 4: return step_kernel<P, 4, false>(); \
        case 5: return step_kernel<P, 5, false>(); \
        case 6: return step_kernel<P, 6, false>(); \
        case 7: return step_kernel<P, 7, false>(); \
        default: return nullptr;                  \
    }
    if (point) return ppt == 1 ? step_kernel<1, 0, true>() : step_kernel<4, 0, true>();
    if (ppt == 1) {
        ARNA_HALVES(1)
    } else {
        ARNA_HALVES(4)
    }
#undef ARNA_HALVES
    return nullptr;
}

int validate(const pf_config *c) {
    if (!c || c->struct_size != sizeof(pf_config)) return PF_EINVAL;
    if (c->n_filters == 0 || c->n_pe == 0 || c->n_per_pe == 0) return PF_EINVAL;
    if (c->n_pe > PF_MAX_PE || c->n_per_pe > PF_MAX_PER_PE) return PF_EUNSUPPORTED;
    if (c->mode > 1 || c->init_mode > 1 || c->lik_mode > 1) return PF_EINVAL;
    if (c->lik_mode == PF_LIK_PATCH) {
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
    if (N > (1ull << 31) || (uint64_t)c->n_filters * c->n_pe > (1ull << 24))
        return PF_EUNSUPPORTED;
    return PF_OK;
}

void free_all(pf_ctx *c) {
    void *ptrs[] = {c->state[0], c->state[1], c->rec[0], c->rec[1], c->lin[0], c->lin[1],
                    c->ring_tab, c->err, c->nex_used, c->est, c->t_pred, c->t_q, c->t_anc,
                    c->t_v, c->t_src, c->t_prop, c->t_ell, c->t_lam, c->d_dbg};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
}

int ensure_ring(pf_ctx *c, uint64_t k) {
    if (c->cfg.mode != PF_MODE_ARNA || c->cfg.n_pe <= 1) return PF_OK;
    if (c->ring_valid && k >= c->ring_base && k < c->ring_base + kRingSteps) return PF_OK;
    const uint32_t M = c->cfg.n_pe;
    hipLaunchKernelGGL(k_ring, dim3(kRingSteps, c->cfg.n_filters), dim3(256),
                       2 * M * sizeof(uint16_t), c->stream, c->ring_tab, (uint32_t)k,
                       c->cfg.n_filters, M, c->key0, c->key1);
    HIP_OK(hipGetLastError());
    c->ring_base = k;
    c->ring_valid = true;
    return PF_OK;
}

StepArgs make_args(pf_ctx *c, uint64_t k, const float *frame) {
    StepArgs a;
    memset(&a, 0, sizeof(a));
    const int nxt = 1 - c->cur;
    a.sin = c->state[c->cur];
    a.sout = c->state[nxt];
    a.rin = c->rec[c->cur];
    a.rout = c->rec[nxt];
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
    a.np_top = 1u << (31 - __builtin_clz(c->cfg.n_per_pe));
    a.inv_np = 1.0 / (double)c->cfg.n_per_pe;
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
    return a;
}

int launch_step(pf_ctx *c, const float *frame) {
    const uint64_t k = c->step + 1;
    if (k > 0xFFFFFFFFull) return PF_EUNSUPPORTED;
    int rc = ensure_ring(c, k);
    if (rc != PF_OK) return rc;
    StepArgs a = make_args(c, k, frame);
    void *fn = pick_step_kernel(c->ppt, c->half, c->cfg.lik_mode == PF_LIK_POINT);
    if (!fn) return PF_EUNSUPPORTED;
    void *args[] = {&a};
    HIP_OK(hipLaunchKernel(fn, dim3((uint32_t)c->FM), dim3(c->block), args, c->lds, c->stream));
    c->cur = 1 - c->cur;
    c->step = k;
    c->exchanged = false;
    return PF_OK;
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
    const uint32_t F = cfg->n_filters, M = cfg->n_pe, np = cfg->n_per_pe;
    c->FM = (uint64_t)F * M;
    c->N = c->FM * np;
    c->block = block_of(np);
    c->ppt = np > 1024 ? 4 : 1;
    c->half = cfg->lik_mode == PF_LIK_PATCH ? cfg->patch / 2 : 0;
    const bool lineage = (cfg->debug & PF_DEBUG_LINEAGE) != 0;
    const bool trace = (cfg->debug & PF_DEBUG_TRACE) != 0;
    c->lds = step_lds(np, lineage);
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
    c->lik.inv_sn2 = 1.0f / (cfg->noise_sigma * cfg->noise_sigma);

    const uint64_t N = c->N;
    rc = PF_OK;
    for (int i = 0; i < 2 && rc == PF_OK; ++i) {
        rc = dev_alloc(&c->state[i], 5 * N);
        if (rc == PF_OK) rc = dev_alloc(&c->rec[i], c->FM);
        if (rc == PF_OK && lineage) rc = dev_alloc(&c->lin[i], N);
    }
    if (rc == PF_OK && cfg->mode == PF_MODE_ARNA && M > 1)
        rc = dev_alloc(&c->ring_tab, (size_t)kRingSteps * c->FM);
    if (rc == PF_OK) rc = dev_alloc(&c->err, 1);
    if (rc == PF_OK) rc = dev_alloc(&c->nex_used, F);
    if (rc == PF_OK) rc = dev_alloc(&c->est, F);
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
        void *fn = pick_step_kernel(c->ppt, c->half, cfg->lik_mode == PF_LIK_POINT);
        if (!fn ||
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds) !=
                hipSuccess)
            rc = PF_EHIP;
    }
    if (rc == PF_OK) {
        if (hipMemcpyAsync(d_truth, truth, 5 * F * sizeof(float), hipMemcpyHostToDevice,
                           c->stream) != hipSuccess ||
            hipMemsetAsync(c->err, 0, sizeof(uint32_t), c->stream) != hipSuccess ||
            hipMemsetAsync(c->nex_used, 0, F * sizeof(uint32_t), c->stream) != hipSuccess)
            rc = PF_EHIP;
    }
    if (rc == PF_OK) {
        const uint64_t work = N > c->FM ? N : c->FM;
        hipLaunchKernelGGL(k_init, dim3((uint32_t)((work + 255) / 256)), dim3(256), 0, c->stream,
                           c->state[0], c->rec[0], c->lin[0], d_truth, N, M, np, cfg->width,
                           cfg->height, cfg->init_mode == PF_INIT_INFOSHARE ? 1u : 0u, c->key0,
                           c->key1, (uint32_t)c->FM);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
            rc = PF_EHIP;
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
    for (uint32_t i = 0; i < n_steps; ++i) {
        const int rc = launch_step(c, d_frames + (size_t)i * frame_stride);
        if (rc != PF_OK) return rc;
    }
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
        hipLaunchKernelGGL(k_exchange_map, dim3((uint32_t)c->FM), dim3(256), 0, c->stream, a,
                           d_src_map);
        HIP_OK(hipGetLastError());
    }
    c->exchanged = true;
    return PF_OK;
}

int pf_estimate(pf_ctx *c, pf_estimate_t *o) {
    if (!c || !o) return PF_EINVAL;
    const uint32_t F = c->cfg.n_filters, M = c->cfg.n_pe;
    hipLaunchKernelGGL(k_global, dim3(F), dim3(256), 0, c->stream, c->rec[c->cur], c->est, M,
                       c->cfg.n_per_pe, c->cfg.mode, c->fixed_nex, c->cutoff_ppm);
    HIP_OK(hipGetLastError());
    EstDev *e = (EstDev *)malloc(sizeof(EstDev) * F);
    uint32_t *nex = (uint32_t *)malloc(sizeof(uint32_t) * F);
    pf_pe_record *rec = nullptr;
    const bool want_pe = o->x_pe || o->log_mass_pe;
    if (want_pe) rec = (pf_pe_record *)malloc(sizeof(pf_pe_record) * c->FM);
    uint32_t err = 0;
    int rc = PF_OK;
    if (!e || !nex || (want_pe && !rec)) rc = PF_ENOMEM;
    if (rc == PF_OK &&
        (hipMemcpyAsync(e, c->est, sizeof(EstDev) * F, hipMemcpyDeviceToHost, c->stream) !=
             hipSuccess ||
         hipMemcpyAsync(nex, c->nex_used, sizeof(uint32_t) * F, hipMemcpyDeviceToHost,
                        c->stream) != hipSuccess ||
         hipMemcpyAsync(&err, c->err, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream) !=
             hipSuccess ||
         (want_pe && hipMemcpyAsync(rec, c->rec[c->cur], sizeof(pf_pe_record) * c->FM,
                                    hipMemcpyDeviceToHost, c->stream) != hipSuccess) ||
         hipStreamSynchronize(c->stream) != hipSuccess))
        rc = PF_EHIP;
    if (rc == PF_OK) {
        for (uint32_t f = 0; f < F; ++f) {
            if (o->x_global)
                for (int d = 0; d < 5; ++d) o->x_global[5 * f + d] = e[f].xhat[d];
            if (o->log_mass_glob) o->log_mass_glob[f] = e[f].log_mass_glob;
            if (o->pe_eff) o->pe_eff[f] = e[f].pe_eff;
            if (o->n_ex) o->n_ex[f] = nex[f];
            if (o->n_ex_next) o->n_ex_next[f] = e[f].n_ex_next;
            if (o->log_z_inc) o->log_z_inc[f] = e[f].log_z;
        }
        if (want_pe)
            for (uint64_t i = 0; i < c->FM; ++i) {
                if (o->log_mass_pe) o->log_mass_pe[i] = rec[i].log_mass;
                if (o->x_pe)
                    for (int d = 0; d < 5; ++d) o->x_pe[5 * i + d] = rec[i].xhat[d];
            }
        o->step = c->step;
        if (err) rc = PF_ENUMERIC;
    }
    free(e);
    free(nex);
    free(rec);
    return rc;
}

void pf_destroy(pf_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
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
        case PF_DBG_STATE: src = c->state[c->cur]; break;
        case PF_DBG_PE_RECORDS: src = c->rec[c->cur]; break;
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
            if (hipMemcpy(rec, c->rec[c->cur], sizeof(pf_pe_record) * c->FM,
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
    HIP_OK(hipStreamSynchronize(c->stream));
    HIP_OK(hipMemcpy(c->state[c->cur], state, 5 * c->N * sizeof(float), hipMemcpyHostToDevice));
    pf_pe_record *rec = (pf_pe_record *)calloc(c->FM, sizeof(pf_pe_record));
    if (!rec) return PF_ENOMEM;
    for (uint64_t i = 0; i < c->FM; ++i) rec[i].log_mass = log_mass ? log_mass[i] : 0.0;
    const hipError_t e =
        hipMemcpy(c->rec[c->cur], rec, sizeof(pf_pe_record) * c->FM, hipMemcpyHostToDevice);
    free(rec);
    HIP_OK(e);
    c->step = step;
    c->exchanged = false;
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
    if (!q || !v || !anc_out || n_p == 0 || n_p > PF_MAX_PER_PE) return PF_EINVAL;
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
            const uint32_t top = 1u << (31 - __builtin_clz(n_p));
            const double inv = 1.0 / (double)n_p;
            if (n_p > 1024)
                hipLaunchKernelGGL(k_resample_q<4>, dim3(n_blocks), dim3(B), 0, 0, dq, dv, da,
                                   n_p, top, inv);
            else
                hipLaunchKernelGGL(k_resample_q<1>, dim3(n_blocks), dim3(B), 0, 0, dq, dv, da,
                                   n_p, top, inv);
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
                  uint32_t *pred_out) {
    if (!pred_out || M == 0 || M > PF_MAX_PE) return PF_EINVAL;
    if (mode != PF_MODE_ARNA || M == 1) {
        for (uint32_t m = 0; m < M; ++m) pred_out[m] = (m + M - 1) % M;
        return PF_OK;
    }
    // the table kernel for filters 0..f, iteration k (one batch row)
    uint16_t *dt = nullptr;
    int rc = dev_alloc(&dt, (size_t)(f + 1) * M);
    if (rc != PF_OK) return rc;
    hipLaunchKernelGGL(k_ring, dim3(1, f + 1), dim3(256), 2 * M * sizeof(uint16_t), 0, dt, k,
                       f + 1, M, (uint32_t)seed, (uint32_t)(seed >> 32));
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
