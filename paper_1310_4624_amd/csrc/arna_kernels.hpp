// arna_kernels.hpp -- the kernels of the ARNA particle-filter step for gfx950
// and the device-side argument structures they share with the host runtime
// (arna.hip).  Included by arna.hip and arna_run.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <limits.h>
#include <math.h>
#include <stdint.h>

#include "arna.h"
#include "arna_device.hpp"

using namespace arna;

namespace {

constexpr uint32_t kRingSteps = 64;     // iterations per ring-table batch
constexpr int kRedDoubles = 128;        // LDS reduction scratch (>= 16 waves x 8)

// The master step of an iteration (Alg. 3 steps 9-10 and the input of step 2
// of the next), per filter: log W = log sum_m W^(m) and the next N_ex.  For
// many PEs it is computed once, by the last workgroup of the filter to
// finish, instead of by every PE of the next iteration.
struct MasterRec {
    double lglob;
    uint32_t nex_next;
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
    // Particles are kept lazily: the propagated particles of an iteration and,
    // per slot, the ancestor the resampling picked; resampled slot s of PE p
    // is propagated particle anc[p N_p + s] of that PE.
    const float *pin;                   // [5][N] propagated particles of k-1
    const uint16_t *ain;                // [N] ancestors of k-1 (slot within the PE)
    float *pout;                        // [5][N] propagated particles of k
    uint16_t *aout;                     // [N] ancestors of k
    const pf_pe_record *rin;            // [F*M] records of k-1
    pf_pe_record *rout;                 // [F*M] records of k
    const uint16_t *ring;               // [F*M] pred(m) for this k, or NULL (fixed ring)
    const DebugBufs *dbg;               // NULL unless a debug mode is on
    Lik lik;
    Dyn dyn;
    uint32_t N;                         // F M N_p (<= 2^29, so 5 N fits 32 bits)
    uint32_t M, np;
    uint32_t k, key0, key1;
    uint32_t mode, first, fixed_nex, initial_nex, cutoff_ppm, qmax;
    uint32_t lin_in;                    // which lineage buffer holds iteration k-1
    uint32_t *err;                      // sticky numeric-error flag
    uint32_t *nex_used;                 // [F]
    uint32_t *nex_rec;                  // [F] N_ex of this iteration, kept for the adjoint; or NULL
    const uint32_t *force_nex;          // [F] N_ex to use instead of step 2's, or NULL
    const uint32_t *force_anc;          // [N] ancestors to use instead of step 7's, or NULL
    // master steps (many PEs): of k-1, read by the prologue (NULL: every PE
    // recomputes it from the M records), and of k, written by the last
    // workgroup of each filter to finish (NULL: not written; the library
    // leaves it NULL and launches k_master after the step, which measured
    // faster than every workgroup's release before counting itself in)
    const MasterRec *min;
    MasterRec *mout;
    uint32_t *arrive;                   // [F] workgroups of the filter done with k
    // [F] row of iteration k-1 of a caller's trajectory: wave 0 of PE (f, 0)
    // writes the master step of k-1 there (the prologue reduces the same
    // records); NULL: no row (first iteration of a run, or many PEs)
    pf_master_t *traj_prev;
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
// Lane 0 writes the result to `out`.  With a.traj_prev, PE 0 of the filter
// also sums x_{k-1} = sum_m W^(m) x^m / W_{k-1} in the same loops and lane 0
// writes the whole master step of k-1 (Alg. 3 steps 9-10) to the row; the
// sums run in the order of k_global_wave, which gives the same bits.
__device__ Prologue prologue_wave(const StepArgs &a, uint32_t f, uint32_t m, Prologue *out,
                                  const uint32_t tid) {
    // Latency first: the ring predecessor is loaded with the records, this
    // PE's exchange offset is drawn while they are in flight, and the log
    // masses of this PE and of pred are taken from the lanes that loaded them
    // (a bit copy: the same values a second read would give).
    constexpr int kCached = 4;   // record chunks kept in registers (M <= 256)
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t M = a.M;
    const pf_pe_record *R = a.rin + (size_t)f * M;
    const uint32_t pred =
        (M == 1) ? m : (a.ring ? (uint32_t)a.ring[(size_t)f * M + m] : (m + M - 1) % M);
    const bool want_x = m == 0 && a.traj_prev != nullptr;   // the same in every lane
    double xs[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double lv[kCached];
    double lmax = -INFINITY, l_own = 0.0, l_pred = 0.0;
#pragma unroll
    for (int c = 0; c < kCached; ++c) {
        const uint32_t j0 = (uint32_t)c * kWave;
        lv[c] = -INFINITY;
        if (j0 < M) {
            if (j0 + lane < M) lv[c] = R[j0 + lane].log_mass;
            lmax = fmax(lmax, lv[c]);
            if ((m & ~(kWave - 1)) == j0) l_own = __shfl(lv[c], (int)(m & (kWave - 1)), kWave);
            if ((pred & ~(kWave - 1)) == j0) l_pred = __shfl(lv[c], (int)(pred & (kWave - 1)), kWave);
        }
    }
    for (uint32_t j0 = kCached * kWave; j0 < M; j0 += kWave) {
        const double l = (j0 + lane < M) ? R[j0 + lane].log_mass : -INFINITY;
        lmax = fmax(lmax, l);
        if ((m & ~(kWave - 1)) == j0) l_own = __shfl(l, (int)(m & (kWave - 1)), kWave);
        if ((pred & ~(kWave - 1)) == j0) l_pred = __shfl(l, (int)(pred & (kWave - 1)), kWave);
    }
    lmax = wave_max_d(lmax);
    double acc = 0.0;
    uint64_t S = 0, D = 0;
    if (lmax != -INFINITY) {
        // P_m = floor(exp(L_m - max L) 2^20); slots past M hold -inf: e = 0
#pragma unroll
        for (int c = 0; c < kCached; ++c) {
            if ((uint32_t)c * kWave < M) {
                const double e = exp(lv[c] - lmax);
                acc += e;
                const uint64_t P = (uint64_t)floor(e * 1048576.0);
                S += P;
                D += P * P;
                if (want_x && e > 0.0)   // (e = 0 past M)
#pragma unroll
                    for (int d = 0; d < 5; ++d) xs[d] += e * R[(uint32_t)c * kWave + lane].xhat[d];
            }
        }
        for (uint32_t i = kCached * kWave + lane; i < M; i += kWave) {
            const double e = exp(R[i].log_mass - lmax);
            acc += e;
            const uint64_t P = (uint64_t)floor(e * 1048576.0);
            S += P;
            D += P * P;
            if (want_x && e > 0.0)
#pragma unroll
                for (int d = 0; d < 5; ++d) xs[d] += e * R[i].xhat[d];
        }
    }
    acc = wave_sum(acc);
    S = wave_sum_u64(S);
    D = wave_sum_u64(D);
    if (want_x) {
#pragma unroll
        for (int d = 0; d < 5; ++d) xs[d] = wave_sum(xs[d]);
        if (lane == 0) {
            pf_master_t r;
            r.log_mass_glob = (lmax == -INFINITY) ? -INFINITY : lmax + log(acc);
#pragma unroll
            for (int d = 0; d < 5; ++d) r.xhat[d] = xs[d] / acc;
            r.pe_eff = D ? (double)S * (double)S / (double)D : 0.0;
            r.log_z_inc = r.log_mass_glob - log((double)a.np);
            r.n_ex = a.nex_used[f];   // (written at the end of k-1 by this PE)
            r.n_ex_next = exchange_count(S, D, M, a.np, a.mode, 0, a.fixed_nex, 0, a.cutoff_ppm);
            r.step = a.k - 1;
            a.traj_prev[f] = r;
        }
    }
    // Every lane finishes the prologue (the wave executes it once either
    // way) and returns it: its integer fields (pred, N_ex, offsets) are the
    // same in every lane -- S and D are exact sums -- while the FP64 sum acc,
    // reduced in a different order in each lane, can differ in the last bit,
    // so the record other waves read is lane 0's.
    Prologue p;
    p.pred = pred;
    p.nex = exchange_count(S, D, M, a.np, a.mode, (int)a.first, a.fixed_nex, a.initial_nex,
                           a.cutoff_ppm);
    if (a.force_nex) p.nex = a.force_nex[f];
    if (p.nex > a.np) p.nex = a.np;
    const double lglob = (lmax == -INFINITY) ? -INFINITY : lmax + log(acc);
    if (lglob == -INFINITY) {
        p.lam_own = 0.f;
        p.lam_pred = 0.f;
    } else {
        p.lam_own = (float)(l_own - lglob);
        p.lam_pred = (float)(l_pred - lglob);
    }
    p.c_own = mulshift(philox(m, a.k, f, kTagExch << 24, a.key0, a.key1).x, a.np);
    p.c_pred = mulshift(philox(pred, a.k, f, kTagExch << 24, a.key0, a.key1).x, a.np);
    if (lane == 0) *out = p;
    return p;
}

// The prologue from a precomputed master record, computed by every lane of one
// wave (uniform inputs: every lane gets the same values); lane 0 writes it.
__device__ Prologue prologue_master(const StepArgs &a, uint32_t f, uint32_t m, Prologue *out,
                                    const uint32_t tid) {
    const uint32_t M = a.M;
    const pf_pe_record *R = a.rin + (size_t)f * M;
    const MasterRec mr = a.min[f];
    Prologue p;
    p.pred = (M == 1) ? m : (a.ring ? (uint32_t)a.ring[(size_t)f * M + m] : (m + M - 1) % M);
    if (M <= 1)
        p.nex = 0;
    else if (a.mode == 0)
        p.nex = a.fixed_nex;
    else if (a.first)
        p.nex = a.initial_nex;
    else
        p.nex = mr.nex_next;
    if (a.force_nex) p.nex = a.force_nex[f];
    if (p.nex > a.np) p.nex = a.np;
    if (mr.lglob == -INFINITY) {
        p.lam_own = 0.f;
        p.lam_pred = 0.f;
    } else {
        p.lam_own = (float)(R[m].log_mass - mr.lglob);
        p.lam_pred = (float)(R[p.pred].log_mass - mr.lglob);
    }
    p.c_own = mulshift(philox(m, a.k, f, kTagExch << 24, a.key0, a.key1).x, a.np);
    p.c_pred = mulshift(philox(p.pred, a.k, f, kTagExch << 24, a.key0, a.key1).x, a.np);
    if ((tid & (kWave - 1)) == 0) *out = p;
    return p;
}

// Master record of filter f from its M PE records, by the whole workgroup
// (`red` >= 3 doubles per wave); thread 0 writes it.
__device__ void master_block(const pf_pe_record *R, uint32_t M, uint32_t np, uint32_t mode,
                             uint32_t fixed_nex, uint32_t cutoff_ppm, double *red,
                             MasterRec *out) {
    double lmax = -INFINITY;
    for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) lmax = fmax(lmax, R[i].log_mass);
    lmax = block_max_d(lmax, red);
    double acc[1] = {0.0};
    uint64_t sd[2] = {0, 0};
    if (lmax != -INFINITY)
        for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) {
            const double e = exp(R[i].log_mass - lmax);
            const uint64_t P = (uint64_t)floor(e * 1048576.0);
            acc[0] += e;
            sd[0] += P;
            sd[1] += P * P;
        }
    block_sum<1>(acc, red);
    block_sum_u64(sd, (uint64_t *)red);
    if (threadIdx.x == 0) {
        MasterRec r;
        r.lglob = (lmax == -INFINITY) ? -INFINITY : lmax + log(acc[0]);
        r.nex_next = exchange_count(sd[0], sd[1], M, np, mode, 0, fixed_nex, 0, cutoff_ppm);
        r.pad = 0;
        *out = r;
    }
}

// Step 3: PE m sends its slots s_t(m) = floor((t N_p + c_m) / N_ex), t < N_ex,
// and refills them with the slots s_t(pred(m)) that pred(m) sends.  The map
// recv[s_t(m)] = s_t(pred(m)) is built in LDS (0xFFFF = slot keeps its own
// particle); `recv` must hold 0xFFFF for every slot on entry.
__device__ __forceinline__ void build_receive_map(uint16_t *recv, const Prologue &p, uint32_t np,
                                                  const uint32_t tid) {
    for (uint32_t t = tid; t < p.nex; t += blockDim.x) {
        const uint32_t dst = (t * np + p.c_own) / p.nex;
        const uint32_t src = (t * np + p.c_pred) / p.nex;
        recv[dst] = (uint16_t)src;
    }
}

// Receive maps of up to kMapWave entries are built by wave 0 before barrier 1
// with kMapBatch loads in flight per lane, when the prologue leaves it the
// time (M <= 64: one record per lane); otherwise by the workgroup after it.
// Measured on MI355X at 2^20 particles: 4 x 64 x 4096 31.0 -> 30.1 us per
// step; 1 x 256 x 4096 32.3 -> 33.3 with wave 0's map, hence the M limit.
constexpr int kMapBatch = 8;
constexpr uint32_t kMapWave = kMapBatch * kWave;
__device__ __forceinline__ bool map_by_wave0(uint32_t nex, uint32_t M) {
    return nex <= kMapWave && M <= kWave;
}

// Step 3 for one slot: if slot s of PE m is refilled (s = s_t(m) for some
// t < N_ex), the slot s_t(pred(m)) of pred's resampled block it receives;
// else kNoSlot.  The t with floor((t N_p + c_own) / N_ex) = s is the least
// t >= (s N_ex - c_own) / N_p (at most one: N_ex <= N_p).
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
__device__ __forceinline__ uint32_t received_from(uint32_t s, const Prologue &p, uint32_t np) {
    if (p.nex == 0) return kNoSlot;
    const int64_t num = (int64_t)s * p.nex - (int64_t)p.c_own;
    const uint64_t t = num <= 0 ? 0u : (uint64_t)((num + np - 1) / np);
    if (t >= p.nex || (t * np + p.c_own) / p.nex != s) return kNoSlot;
    return (uint32_t)((t * np + p.c_pred) / p.nex);
}

// LDS image tile: 64 x 64 pixels of z - B, zero outside the image.  The row
// pitch decides how often the patch reads of a wave's particles, whose patch
// origins differ by a few rows and columns, meet in the same LDS bank; chosen
// by measurement on MI355X (one step at 2^20 particles, 4 x 64 x 4096):
// pitch 65: 37.9 us, 67: 32.9, 69-73: 30.8-30.9, 75: 33.2, 77: 31.0, 79: 33.5.
constexpr int kTileCols = 64, kTilePitch = 70, kTileRows = 64;
constexpr int kMaxWaves = 16;

// Dynamic LDS layout of k_step (the tile comes first: its reads use small
// immediate offsets from one base register per patch row).
struct Lds {
    float *tile;       // [kTileRows][kTilePitch]; later the offspring marks
    double *wsum;      // [16][6] wave sums (W, W x)
    Prologue *pro;     // 1
    float *wmax;       // [16] wave maxima
    uint32_t *wq;      // [16][4] wave totals of Q, per slot level
    float *st;         // [5][np] propagated particles
    uint32_t *cq;      // [np] carried weight, then u, then nothing
    uint16_t *recv;    // [np] per slot: pred's propagated particle it receives, or 0xFFFF
    int32_t *lin;      // [np] (lineage only)
};
__host__ __device__ constexpr size_t lds_fixed_bytes() {
    return (size_t)kTileRows * kTilePitch * sizeof(float) + kMaxWaves * 6 * sizeof(double) + 32 +
           kMaxWaves * sizeof(float) + kMaxWaves * 4 * sizeof(uint32_t);
}
__host__ __device__ constexpr size_t lds_bytes(uint32_t np, bool lineage) {
    return lds_fixed_bytes() + 5 * (size_t)np * 4 + (size_t)np * 4 + ((size_t)np * 2 + 15) / 16 * 16 +
           (lineage ? (size_t)np * 4 : 0);
}
__device__ __forceinline__ Lds carve(unsigned char *base, uint32_t np) {
    Lds l;
    size_t o = 0;
    l.tile = (float *)(base + o);
    o += (size_t)kTileRows * kTilePitch * sizeof(float);
    l.wsum = (double *)(base + o);
    o += kMaxWaves * 6 * sizeof(double);
    l.pro = (Prologue *)(base + o);
    o += 32;
    l.wmax = (float *)(base + o);
    o += kMaxWaves * sizeof(float);
    l.wq = (uint32_t *)(base + o);
    o += kMaxWaves * 4 * sizeof(uint32_t);
    l.st = (float *)(base + o);
    o += 5 * (size_t)np * sizeof(float);
    l.cq = (uint32_t *)(base + o);
    o += (size_t)np * sizeof(uint32_t);
    l.recv = (uint16_t *)(base + o);
    o += ((size_t)np * 2 + 15) / 16 * 16;
    l.lin = (int32_t *)(base + o);
    return l;
}

// Step 7 building blocks, shared by k_step and the debug entry point.
// Thread t holds the fixed-point weights of slots t + q B (q < PPT).
// Part 1: inclusive scans within each wave, per level q; the last lane of each
// wave leaves the wave totals in wq[wave][q].
template <int PPT>
__device__ __forceinline__ void scan_levels(const uint32_t (&Q)[PPT], uint32_t (&cinc)[PPT],
                                            uint32_t *wq, const uint32_t tid) {
    const uint32_t lane = tid & (kWave - 1), wave = tid / kWave;
#pragma unroll
    for (int q = 0; q < PPT; ++q) cinc[q] = wave_incl_scan_u32(Q[q]);
    if (lane == kWave - 1)
#pragma unroll
        for (int q = 0; q < PPT; ++q) wq[wave * 4 + q] = cinc[q];
}
// Part 2 (after a barrier): inclusive sums C of this thread's slots, in slot
// order, and the total T.  The (level, wave) totals, 64 values in slot order,
// are scanned across the lanes of every wave at once (lane q 16 + w holds level
// q of wave w), so no further barrier is needed.
template <int PPT>
__device__ __forceinline__ uint32_t scan_finish(uint32_t (&cinc)[PPT], const uint32_t *wq,
                                                const uint32_t tid) {
    const uint32_t lane = tid & (kWave - 1), wave = tid / kWave;
    const uint32_t nwaves = blockDim.x / kWave;
    const uint32_t lq = lane / 16, lw = lane % 16;
    const uint32_t mine = (lq < (uint32_t)PPT && lw < nwaves) ? wq[lw * 4 + lq] : 0u;
    const uint32_t incl = wave_incl_scan_u32(mine);
    const uint32_t T = lane63(incl);
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const uint32_t src = (uint32_t)q * 16 + wave;
        cinc[q] += (uint32_t)__builtin_amdgcn_readlane((int)(incl - mine), (int)src);
    }
    return T;
}

// Part 3: every particle with offspring marks its first output rank,
// mark[first_offspring(i)] = max(i); `mark` (>= n entries) must be zero.
template <int PPT>
__device__ __forceinline__ void mark_offspring(const uint32_t (&Q)[PPT], const uint32_t (&C)[PPT],
                                               uint32_t n, uint32_t T, uint32_t V, uint32_t *mark,
                                               const uint32_t tid) {
    const double inv_T = 1.0 / (double)T;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const uint32_t s = tid + q * blockDim.x;
        if (s < n && Q[q] > 0) {
            const uint32_t j = first_offspring(C[q] - Q[q], n, T, V, inv_T);
            if (j < n) atomicMax(&mark[j], s);
        }
    }
}

// Part 4 (after a barrier): the ancestor of output rank j is the largest
// particle that marked a rank <= j, i.e. min { i : n C_i > j T + V }.
// Thread t resolves the consecutive ranks t PPT + q; `wtmp` holds one value per
// wave.  Contains one barrier.
template <int PPT>
__device__ __forceinline__ void ancestors_from_marks(const uint32_t *mark, uint32_t n,
                                                     uint32_t *wtmp, uint32_t (&anc)[PPT],
                                                     const uint32_t tid) {
    const uint32_t lane = tid & (kWave - 1), wave = tid / kWave;
    const uint32_t j0 = tid * PPT;
    uint32_t run = 0;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const uint32_t m = (j0 + q < n) ? mark[j0 + q] : 0u;
        run = m > run ? m : run;
        anc[q] = run;
    }
    const uint32_t incl = wave_incl_max_u32(run);
    const uint32_t excl = wave_shr1(incl);
    if (lane == kWave - 1) wtmp[wave] = incl;
    __syncthreads();
    uint32_t before = excl;
    for (uint32_t w = 0; w < wave; ++w) before = wtmp[w] > before ? wtmp[w] : before;
#pragma unroll
    for (int q = 0; q < PPT; ++q) anc[q] = anc[q] > before ? anc[q] : before;
}

// Likelihood variants of k_step.
enum LikKind { kLikGauss = 0, kLikPoint = 1, kLikPoisson = 2 };

// One ARNA / RNA iteration; one workgroup = one PE (f, m).  Thread t owns the
// slots s = t + q B, q < PPT (B = blockDim.x), so every global access of a
// slot level is coalesced.
// RES (the multi-iteration kernel): xr holds the thread's resampled particles
// of the previous iteration (slots t + q B), so when from_regs is set the own
// slots are not read back from HBM; at the end xr receives the particles the
// resampling picked for those slots.  The values are those k_step would read
// back, so both kernels compute the same bits.
template <int PPT, int HALF, int LIK, bool RES = false>
__device__ __forceinline__ void step_body(const StepArgs &a, const uint32_t bid,
                                          float (&xr)[PPT][5], const bool from_regs,
                                          const uint32_t tid) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int P = 2 * HALF + 1;
    const uint32_t M = a.M, np = a.np, N = a.N;
    const uint32_t f = bid / M, m = bid % M;
    const uint32_t B = blockDim.x;
    const uint32_t lane = tid & (kWave - 1), wave = tid / kWave, nwaves = B / kWave;
    Lds L = carve(smem, np);
    uint16_t *recv = L.recv;
    const uint32_t pe_base = bid * np;   // (f M + m) N_p
    const DebugBufs *D = a.dbg;
    const int32_t *lin_in = D ? D->lin[a.lin_in] : nullptr;
    int32_t *lin_out = D ? D->lin[1 - a.lin_in] : nullptr;
    const bool trace = D && D->t_q;

    // ---- phase 0: wave 0 redoes the master step of iteration k-1 (steps
    // 1-2); every thread issues the loads of its own slots (most slots keep
    // their particle) and of its part of the image tile, and the other waves
    // draw the step-5 normals, those of wave 0's slots included (parked in
    // the LDS particle stage, which is free until phase 1).  The
    // tile is centred where this PE's estimate of k-1 moves in one step
    // (x + v); a particle whose patch does not fit in it reads the frame,
    // with the same arithmetic.
    if (wave == 0) {
        const Prologue p =
            a.min ? prologue_master(a, f, m, L.pro, tid) : prologue_wave(a, f, m, L.pro, tid);
        // Step 3's receive map, before this wave's own loads (the other waves
        // are drawing normals; wave 0 has slack until they reach barrier 1):
        // slot s_t(m) gets pred's propagated particle ain[s_t(pred)], the
        // ancestor lookup done here so that phase 1 needs a single load per
        // received component.  Lanes clear slots that other lanes then fill:
        // wavefront-scope release / acquire around a wave barrier order them.
        if (M <= kWave) {   // else each thread clears its own slots
            for (uint32_t s = lane; s < np; s += kWave) recv[s] = 0xFFFF;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // up to kMapBatch ancestor loads in flight per lane before any is used
        if (map_by_wave0(p.nex, M)) {
            const uint32_t pred_base = (f * M + p.pred) * np;
            uint16_t got[kMapBatch];
#pragma unroll
            for (int j = 0; j < kMapBatch; ++j) {
                const uint32_t t = lane + (uint32_t)j * kWave;
                if (t < p.nex) got[j] = a.ain[pred_base + (t * np + p.c_pred) / p.nex];
            }
#pragma unroll
            for (int j = 0; j < kMapBatch; ++j) {
                const uint32_t t = lane + (uint32_t)j * kWave;
                if (t < p.nex) recv[(t * np + p.c_own) / p.nex] = got[j];
            }
        }
    }
    const bool load_own = !(RES && from_regs);
    uint32_t own[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const uint32_t s = tid + q * B;
        own[q] = 0;
        if (s < np && load_own) own[q] = a.ain[pe_base + s];
        if (s < np && M > kWave) recv[s] = 0xFFFF;   // else wave 0 clears the map
    }
    int tx0 = 0, ty0 = 0;
    bool tile_on = false, tile_inside = false;
    constexpr bool POINT = LIK == kLikPoint;
    if (!POINT) {
        const double *xh = a.rin[bid].xhat;
        const double cx = xh[0] + xh[2], cy = xh[1] + xh[3];
        // the tile pays for its 4096 loads only with a full workgroup of particles
        if (B >= 1024 && fabs(cx) < 1e6 && fabs(cy) < 1e6) {   // false for NaN (a PE without mass)
            tx0 = (int)floor(cx + 0.5) - kTileCols / 2;
            ty0 = (int)floor(cy + 0.5) - kTileRows / 2;
            tile_on = tx0 < (int)a.lik.W && tx0 + kTileCols > 0 && ty0 < (int)a.lik.H &&
                      ty0 + kTileRows > 0;
            tile_inside = tx0 >= 0 && ty0 >= 0 && tx0 + kTileCols <= (int)a.lik.W &&
                          ty0 + kTileRows <= (int)a.lik.H;
        }
    }
    float x[PPT][5];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const uint32_t s = tid + q * B;
        if (s < np)
#pragma unroll
            for (int c = 0; c < 5; ++c)
                x[q][c] = load_own ? a.pin[c * N + pe_base + own[q]] : xr[q][c];
    }
    // Tile pixel i = r kTileCols + c is image pixel (tx0 + c, ty0 + r).  Its
    // first kTileRegs B pixels are loaded into registers now and written to
    // LDS at the end of the phase, so the loads overlap the other work.
    constexpr int kTileRegs = (kTileRows * kTileCols) / 1024;
    float tv[kTileRegs];
#pragma unroll
    for (int i = 0; i < kTileRegs; ++i) {
        const uint32_t idx = tid + (uint32_t)i * B;
        const int u = tx0 + (int)(idx % kTileCols), v = ty0 + (int)(idx / kTileCols);
        const bool in = tile_on && (unsigned)u < (unsigned)a.lik.W && (unsigned)v < (unsigned)a.lik.H;
        tv[i] = in ? a.lik.img[(size_t)v * a.lik.W + u] - a.lik.bg : 0.f;
    }
    float e[PPT][5];
    // waves 1..PPT draw wave 0's normals (one of its slot levels each)
    const bool helpers = nwaves > (uint32_t)PPT;
    if (helpers && tid >= kWave && tid < kWave * (PPT + 1)) {
        // wave 0's slot of lane j % 64 at level j / 64
        const uint32_t j = tid - kWave;
        const uint32_t s = j % kWave + (j / kWave) * B;
        if (s < np) {
            float t[5];
            five_normals(philox(m * np + s, a.k, f, kTagProp << 24, a.key0, a.key1), t);
#pragma unroll
            for (int c = 0; c < 5; ++c) L.st[c * np + s] = t[c];
        }
    }
    if (wave != 0 || !helpers) {
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const uint32_t s = tid + q * B;
            if (s < np)
                five_normals(philox(m * np + s, a.k, f, kTagProp << 24, a.key0, a.key1), e[q]);
        }
    }
    if (tile_on) {
#pragma unroll
        for (int i = 0; i < kTileRegs; ++i) {
            const uint32_t idx = tid + (uint32_t)i * B;
            L.tile[(idx / kTileCols) * kTilePitch + idx % kTileCols] = tv[i];
        }
        // the rest of the tile, only when B < 1024
        for (uint32_t idx = tid + kTileRegs * B; idx < (uint32_t)(kTileRows * kTileCols); idx += B) {
            const int u = tx0 + (int)(idx % kTileCols), v = ty0 + (int)(idx / kTileCols);
            const bool in = (unsigned)u < (unsigned)a.lik.W && (unsigned)v < (unsigned)a.lik.H;
            L.tile[(idx / kTileCols) * kTilePitch + idx % kTileCols] =
                in ? a.lik.img[(size_t)v * a.lik.W + u] - a.lik.bg : 0.f;
        }
    }
    __syncthreads();   // barrier 1: prologue, receive map, tile and wave 0's
                       // normals visible
    if (helpers && wave == 0) {
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const uint32_t s = tid + q * B;
            if (s < np)
#pragma unroll
                for (int c = 0; c < 5; ++c) e[q][c] = L.st[c * np + s];
        }
    }
    const Prologue p = *L.pro;
    if (p.nex && !map_by_wave0(p.nex, M)) {
        // the whole workgroup fills the receive map
        const uint32_t pb = (f * M + p.pred) * np;
        for (uint32_t t = tid; t < p.nex; t += B)
            recv[(t * np + p.c_own) / p.nex] = a.ain[pb + (t * np + p.c_pred) / p.nex];
        __syncthreads();   // barrier 1b: receive map (when not wave 0's)
    }

    // ---- phase 1 (steps 3-5 P): received slots are refetched from pred(m)
    // (all of a thread's loads issued before the first is used); propagate;
    // stage in LDS.  A thread reads back only its own slots, so the
    // likelihood follows without a barrier.
    const uint32_t pred_base = (f * M + p.pred) * np;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const uint32_t s = tid + q * B;
        if (s >= np) continue;
        uint32_t gsrc = pe_base + s;
        float lam = p.lam_own;
        const uint32_t pq = p.nex ? recv[s] : 0xFFFFu;
        if (pq != 0xFFFFu) {
            for (int c = 0; c < 5; ++c) x[q][c] = a.pin[c * N + pred_base + pq];
            lam = p.lam_pred;
            if (lin_in || trace) gsrc = pred_base + received_from(s, p, np);
        }
        if (lin_in) L.lin[s] = lin_in[gsrc];
        if (trace) {
            D->t_src[pe_base + s] = (int64_t)gsrc;
            D->t_lam[pe_base + s] = lam;
        }
        propagate(x[q], e[q], a.dyn);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            L.st[c * np + s] = x[q][c];
            a.pout[c * N + pe_base + s] = x[q][c];
        }
        L.cq[s] = __float_as_uint(lam);   // parked until the likelihood is known
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
        float ell = 0.f;
        int u0, v0;
        if (POINT) {
            ell = loglik_point(xs, a.lik, f);
        } else if (patch_origin<HALF>(xs[0], xs[1], a.lik.W, a.lik.H, u0, v0)) {
            const int du = u0 - tx0, dv = v0 - ty0;
            if (tile_on && (unsigned)du <= (unsigned)(kTileCols - P) &&
                (unsigned)dv <= (unsigned)(kTileRows - P)) {
                const float *pix = L.tile + dv * kTilePitch + du;
                if (LIK == kLikPoisson)
                    ell = patch_loglik_poisson<HALF, kFromTile>(xs, u0, v0, pix, kTilePitch, a.lik);
                else
                    ell = tile_inside
                              ? patch_loglik<HALF, kFromTileInside>(xs, u0, v0, pix, kTilePitch, a.lik)
                              : patch_loglik<HALF, kFromTile>(xs, u0, v0, pix, kTilePitch, a.lik);
            } else if (u0 >= 0 && v0 >= 0 && u0 + P <= (int)a.lik.W && v0 + P <= (int)a.lik.H) {
                const float *pix = a.lik.img + (size_t)v0 * a.lik.W + u0;
                ell = (LIK == kLikPoisson)
                          ? patch_loglik_poisson<HALF, kFromImage>(xs, u0, v0, pix, 0, a.lik)
                          : patch_loglik<HALF, kFromImage>(xs, u0, v0, pix, 0, a.lik);
            } else {
                ell = (LIK == kLikPoisson)
                          ? patch_loglik_poisson<HALF, kFromImageBorder>(xs, u0, v0, a.lik.img, 0,
                                                                          a.lik)
                          : patch_loglik<HALF, kFromImageBorder>(xs, u0, v0, a.lik.img, 0, a.lik);
            }
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
    __syncthreads();   // barrier 2: wave maxima (tile reads done)
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
    scan_levels<PPT>(Qv, cinc, L.wq, tid);
    uint32_t *mark = (uint32_t *)L.tile;   // the tile is no longer read
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const uint32_t s = tid + q * B;
        if (s < np) mark[s] = 0;
    }
    {
        const double t = wave_total6_f64(sums, lane);
        if ((lane & 7u) == 0 && lane < 48) L.wsum[wave * 6 + (lane >> 3)] = t;
    }
    __syncthreads();   // barrier 3: wave totals, marks cleared
    const uint32_t T = scan_finish<PPT>(cinc, L.wq, tid);
    const uint32_t V = mulshift(philox(m, a.k, f, kTagResample << 24, a.key0, a.key1).x, T);
    mark_offspring<PPT>(Qv, cinc, np, T, V, mark, tid);
    __syncthreads();   // barrier 4: marks complete

    // ---- phase 4 (step 7): ancestors as prefix maxima of the marks; only the
    // indices are stored (the propagated particles went out in phase 1).
    uint32_t anc[PPT];
    ancestors_from_marks<PPT>(mark, np, L.wq, anc, tid);
    if (a.force_anc) {   // replay of another run's choices (test support)
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const uint32_t j = tid * PPT + q;
            if (j < np) anc[q] = a.force_anc[pe_base + j];
        }
    }
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const uint32_t j = tid * PPT + q;
        if (j >= np) continue;
        a.aout[pe_base + j] = (uint16_t)anc[q];
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
        a.rout[bid] = r;
        // (the prologue record is read again from LDS, where it stays for
        // the whole iteration: nothing keeps it in registers until here)
        const Prologue *pr = L.pro;
        if (m == 0) {
            a.nex_used[f] = pr->nex;
            if (a.nex_rec) a.nex_rec[f] = pr->nex;
        }
        if (trace) {
            D->t_pred[bid] = pr->pred;
            D->t_v[bid] = V;
        }
    }
    if (RES) {
        // the particles of this thread's slots for the next iteration: the
        // ancestors go through LDS from the thread that found them (slots
        // t PPT + q) to the slot owners (slots t + q B)
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const uint32_t j = tid * PPT + q;
            if (j < np) recv[j] = (uint16_t)anc[q];
        }
        __syncthreads();
        // (every lane assigns all of xr, so its old values die here; lanes
        // past N_p read slot 0)
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const uint32_t s = tid + q * B;
            const uint32_t src = recv[s < np ? s : 0u];
#pragma unroll
            for (int c = 0; c < 5; ++c) xr[q][c] = L.st[c * np + src];
        }
    }
    if (a.mout) {
        // the last workgroup of the filter to publish its record computes the
        // master step of this iteration (records made visible by the fence
        // before the arrival count; the counter is reset for the next one)
        uint32_t *last = (uint32_t *)L.wmax;
        if (tid == 0) {
            __threadfence();
            *last = (atomicAdd(&a.arrive[f], 1u) == M - 1) ? 1u : 0u;
        }
        __syncthreads();
        if (*last) {
            __threadfence();
            master_block(a.rout + (size_t)f * M, M, np, a.mode, a.fixed_nex, a.cutoff_ppm,
                         L.wsum, a.mout + f);
            if (tid == 0) atomicExch(&a.arrive[f], 0u);
        }
    }
}

template <int PPT, int HALF, int LIK>
__global__ __launch_bounds__(1024) void k_step(StepArgs a) {
    float unused[PPT][5];
    step_body<PPT, HALF, LIK>(a, blockIdx.x, unused, false, threadIdx.x);
}

// Several independent filter contexts in one launch: context i owns the
// workgroups [first[i], first[i + 1]), one per PE, and its arguments are
// args[i] (all contexts of a launch share PPT, the block size, the patch size
// and the likelihood).  The work of a workgroup is exactly that of k_step.
template <int PPT, int HALF, int LIK>
__global__ __launch_bounds__(1024) void k_step_batch(const StepArgs *args, const uint32_t *first,
                                                     uint32_t n) {
    uint32_t lo = 0, hi = n;   // the context whose range holds this workgroup
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (first[mid] <= blockIdx.x)
            lo = mid;
        else
            hi = mid;
    }
    const StepArgs a = args[lo];
    float unused[PPT][5];
    step_body<PPT, HALF, LIK>(a, blockIdx.x - first[lo], unused, false, threadIdx.x);
}

// Several iterations of one context in one launch, each workgroup staying on
// its PE: the resampled particles of a PE's own slots stay in the registers of
// their threads from one iteration to the next, so only the N_ex received
// slots are read back from HBM; the propagated particles, ancestors and
// records still go out every iteration (the receivers and the next launch read
// them).  Between iterations the M workgroups of a filter meet at a barrier
// (all workgroups of the launch must be resident at once: cooperative launch).
struct RunArgs {
    const StepArgs *args;         // [n] arguments of iterations k0, k0 + 1, ...
    uint32_t n;                   // iterations in this launch
    unsigned long long *bar;      // [F] arrivals at the filter barrier, zero at launch
    unsigned long long timeout;   // longest wait at a barrier, wall-clock ticks
};

// What k_run_prep turns into the per-iteration arguments of a k_run launch.
struct RunPrep {
    StepArgs a;                   // iteration k0 = a.k (buffers, ring and frame set per iteration)
    const float *frames;          // frame of iteration k0 + i at frames + i * stride
    uint64_t stride;
    const uint16_t *ring0;        // pred(m) rows of iterations k0, k0 + 1, ... (F M each), or NULL
    float *prop[2];
    uint16_t *anc[2];
    pf_pe_record *rec[2];
    uint32_t cur;                 // buffer index holding iteration k0 - 1
    uint32_t n, fm, F;
    StepArgs *out;                // [n]
    unsigned long long *bar;      // [F], zeroed
};

__global__ void k_run_prep(RunPrep p) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p.n) {
        StepArgs a = p.a;
        const uint32_t in = (p.cur + i) & 1u, out = in ^ 1u;
        a.pin = p.prop[in];
        a.ain = p.anc[in];
        a.rin = p.rec[in];
        a.pout = p.prop[out];
        a.aout = p.anc[out];
        a.rout = p.rec[out];
        a.ring = p.ring0 ? p.ring0 + (size_t)i * p.fm : nullptr;
        a.lik.img = p.frames + (size_t)i * p.stride;
        a.k += i;
        if (i) a.first = 0u;
        p.out[i] = a;
    }
    if (i < p.F) p.bar[i] = 0ull;
}

// Error bit set when a barrier wait of k_run exceeds its limit (the launch
// then ends).
constexpr uint32_t kErrBarrier = 2u;

// Step 1 for kRingSteps iterations at once: Fisher-Yates (Durstenfeld,
// i = M-1 .. 1, j = floor(r_i (i + 1) / 2^32)) over the M labels; the ring
// visits perm[0], perm[1], ... and closes.  Grid (steps, F).
// With G > 1 groups (the hardware-aware ring of Sec. VI) PE m belongs to group
// (f M + m) mod G -- with G = 8 the accelerator die its workgroup runs on,
// since workgroups are dealt to the dies round-robin -- and the ring visits
// the groups in a shuffled order (draws Philox(i, k, f, RING | 1)), the
// members of each group, taken in increasing m, in a shuffled order (draws
// Philox(i, k, f, RING | 2 + g)); only G of its M edges join different groups.
// Dynamic LDS: ring_lds_bytes(M, G).
__host__ __device__ constexpr size_t ring_lds_bytes(uint32_t M, uint32_t G) {
    return 4 * (size_t)M + (G > 1 ? 12 * (size_t)G : 0) + 16;
}
__global__ __launch_bounds__(256) void k_ring(uint16_t *tab, uint32_t base, uint32_t F,
                                              uint32_t M, uint32_t G, uint32_t key0,
                                              uint32_t key1) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t *perm = (uint16_t *)smem;
    uint16_t *jd = perm + M;
    const uint32_t k = base + blockIdx.x, f = blockIdx.y;
    if (G <= 1) {
        for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) {
            perm[i] = (uint16_t)i;
            jd[i] = (i == 0) ? 0
                             : (uint16_t)mulshift(philox(i, k, f, kTagRing << 24, key0, key1).x,
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
    } else {
        uint32_t *gbase = (uint32_t *)(jd + M);   // start of group g, natural order
        uint32_t *pbase = gbase + G;               // start of group g along the ring
        uint16_t *order = (uint16_t *)(pbase + G);
        // PE m is in group (r0 + m mod G) mod G and is member number m / G of
        // it; group (r0 + d) mod G has q + (d < rem) members
        const uint32_t r0 = (uint32_t)(((uint64_t)f * M) % G);
        const uint32_t q = M / G, rem = M % G;
        if (threadIdx.x == 0) {
            uint32_t acc = 0;
            for (uint32_t g = 0; g < G; ++g) {
                gbase[g] = acc;
                acc += q + (((g + G - r0) % G) < rem ? 1u : 0u);
            }
        }
        for (uint32_t g = threadIdx.x; g < G; g += blockDim.x) order[g] = (uint16_t)g;
        __syncthreads();
        for (uint32_t m = threadIdx.x; m < M; m += blockDim.x) {
            const uint32_t g = (r0 + m % G) % G, idx = m / G;
            perm[gbase[g] + idx] = (uint16_t)m;
            jd[gbase[g] + idx] =
                (idx == 0) ? 0
                           : (uint16_t)mulshift(
                                 philox(idx, k, f, (kTagRing << 24) | (2u + g), key0, key1).x,
                                 idx + 1);
        }
        __syncthreads();
        // shuffle every group's members (one thread per group), then the
        // order of the groups
        for (uint32_t g = threadIdx.x; g < G; g += blockDim.x) {
            const uint32_t cnt = q + (((g + G - r0) % G) < rem ? 1u : 0u);
            uint16_t *seg = perm + gbase[g];
            const uint16_t *js = jd + gbase[g];
            for (uint32_t i = cnt - 1; i >= 1 && cnt > 1; --i) {
                const uint32_t j = js[i];
                const uint16_t t = seg[i];
                seg[i] = seg[j];
                seg[j] = t;
            }
        }
        if (threadIdx.x == 0) {
            for (uint32_t i = G - 1; i >= 1; --i) {
                const uint32_t j = mulshift(philox(i, k, f, (kTagRing << 24) | 1u, key0, key1).x,
                                            i + 1);
                const uint16_t t = order[i];
                order[i] = order[j];
                order[j] = t;
            }
            uint32_t acc = 0;
            for (uint32_t a = 0; a < G; ++a) {
                const uint32_t g = order[a];
                pbase[g] = acc;
                acc += q + (((g + G - r0) % G) < rem ? 1u : 0u);
            }
        }
        __syncthreads();
        // the groups in ring order (jd is free now), then back into perm
        for (uint32_t m = threadIdx.x; m < M; m += blockDim.x) {
            const uint32_t g = (r0 + m % G) % G, idx = m / G;
            jd[pbase[g] + idx] = perm[gbase[g] + idx];
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) perm[i] = jd[i];
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
__global__ void k_init(float *st, uint16_t *anc, pf_pe_record *rec, int32_t *lin, const float *truth,
                       uint64_t N, uint32_t M, uint32_t np, uint32_t W, uint32_t H,
                       uint32_t infoshare, uint32_t key0, uint32_t key1, uint32_t FM) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < FM) {
        // PE records of step 0: equal masses; x^m is the mean of the initial
        // cloud (the truth, or the centre of the uniform prior), which also
        // places the first step's image tile.
        const uint32_t pf = (uint32_t)g / M, pm = (uint32_t)g % M;
        const float *t = truth + 5 * pf;
        pf_pe_record r = {};
        r.log_mass = 0.0;
        const bool prior = infoshare && pm != 0;
        r.xhat[0] = prior ? 0.5 * ((double)W - 1.0) : (double)t[0];
        r.xhat[1] = prior ? 0.5 * ((double)H - 1.0) : (double)t[1];
        r.xhat[2] = prior ? 0.0 : (double)t[2];
        r.xhat[3] = prior ? 0.0 : (double)t[3];
        r.xhat[4] = (double)t[4];
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
    anc[g] = (uint16_t)s;
    if (lin) lin[g] = (int32_t)m;
}

// Resampled particles of the last iteration, out[c][g] = prop[c][anc of g]
// (checkpoints and pf_debug_get).
__global__ void k_materialize(const float *prop, const uint16_t *anc, float *out, uint32_t N,
                              uint32_t np) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    const uint32_t src = (g / np) * np + anc[g];
    for (int c = 0; c < 5; ++c) out[(size_t)c * N + g] = prop[(size_t)c * N + src];
}

// Identity ancestors (after a state is set from the host).
__global__ void k_identity(uint16_t *anc, uint32_t N, uint32_t np) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < N) anc[g] = (uint16_t)(g % np);
}

// Master step of iteration k (Alg. 3, steps 9-10) for reporting, for
// contexts without master records (with them k_master computes it), one wave
// per filter: W_k, the global estimate x_k = sum_m W^(m) x^m / W_k, PE_eff,
// the next N_ex and the likelihood increment, n_ex the N_ex iteration k used
// (nex_used[f]).  The sums run in the order of prologue_wave's (records in
// chunks of 64 lanes, the first kCached chunks, then the rest; wave
// butterflies), so that a trajectory row written by the prologue and this
// kernel's record agree bit for bit.
__global__ __launch_bounds__(64) void k_global_wave(const pf_pe_record *rec, pf_master_t *est,
                                                    uint32_t M, uint32_t np, uint32_t mode,
                                                    uint32_t fixed_nex, uint32_t cutoff_ppm,
                                                    const uint32_t *nex_used, uint64_t step) {
    constexpr int kCached = 4;
    const uint32_t f = blockIdx.x, lane = threadIdx.x;
    const pf_pe_record *R = rec + (size_t)f * M;
    double lv[kCached];
    double lmax = -INFINITY;
#pragma unroll
    for (int c = 0; c < kCached; ++c) {
        const uint32_t j0 = (uint32_t)c * kWave;
        lv[c] = -INFINITY;
        if (j0 < M) {
            if (j0 + lane < M) lv[c] = R[j0 + lane].log_mass;
            lmax = fmax(lmax, lv[c]);
        }
    }
    for (uint32_t j0 = kCached * kWave; j0 < M; j0 += kWave) {
        const double l = (j0 + lane < M) ? R[j0 + lane].log_mass : -INFINITY;
        lmax = fmax(lmax, l);
    }
    lmax = wave_max_d(lmax);
    double acc = 0.0, xs[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    uint64_t S = 0, D = 0;
    if (lmax != -INFINITY) {
#pragma unroll
        for (int c = 0; c < kCached; ++c) {
            if ((uint32_t)c * kWave < M) {
                const double e = exp(lv[c] - lmax);
                acc += e;
                const uint64_t P = (uint64_t)floor(e * 1048576.0);
                S += P;
                D += P * P;
                if (e > 0.0)
#pragma unroll
                    for (int d = 0; d < 5; ++d) xs[d] += e * R[(uint32_t)c * kWave + lane].xhat[d];
            }
        }
        for (uint32_t i = kCached * kWave + lane; i < M; i += kWave) {
            const double e = exp(R[i].log_mass - lmax);
            acc += e;
            const uint64_t P = (uint64_t)floor(e * 1048576.0);
            S += P;
            D += P * P;
            if (e > 0.0)
#pragma unroll
                for (int d = 0; d < 5; ++d) xs[d] += e * R[i].xhat[d];
        }
    }
    acc = wave_sum(acc);
    S = wave_sum_u64(S);
    D = wave_sum_u64(D);
#pragma unroll
    for (int d = 0; d < 5; ++d) xs[d] = wave_sum(xs[d]);
    if (lane == 0) {
        pf_master_t r;
        r.log_mass_glob = (lmax == -INFINITY) ? -INFINITY : lmax + log(acc);
#pragma unroll
        for (int d = 0; d < 5; ++d) r.xhat[d] = xs[d] / acc;
        r.pe_eff = D ? (double)S * (double)S / (double)D : 0.0;
        r.log_z_inc = r.log_mass_glob - log((double)np);
        r.n_ex = nex_used ? nex_used[f] : 0u;
        r.n_ex_next = exchange_count(S, D, M, np, mode, 0, fixed_nex, 0, cutoff_ppm);
        r.step = step;
        est[f] = r;
    }
}

// pf_exchange: steps 1-3 of the next iteration, exported as a source map
// (the receive map in LDS up to PF_MAX_PER_PE_LDS slots, else slot by slot).
__global__ __launch_bounds__(256) void k_exchange_map(StepArgs a, int64_t *src) {
    __shared__ Prologue pro;
    __shared__ uint16_t recv[PF_MAX_PER_PE_LDS];
    const uint32_t f = blockIdx.x / a.M, m = blockIdx.x % a.M;
    const bool lds_map = a.np <= PF_MAX_PER_PE_LDS;
    if (threadIdx.x < kWave) prologue_wave(a, f, m, &pro, threadIdx.x);
    if (lds_map)
        for (uint32_t s = threadIdx.x; s < a.np; s += blockDim.x) recv[s] = 0xFFFF;
    __syncthreads();
    const Prologue p = pro;
    if (lds_map) build_receive_map(recv, p, a.np, threadIdx.x);
    __syncthreads();
    for (uint32_t s = threadIdx.x; s < a.np; s += blockDim.x) {
        const uint32_t r = lds_map ? (recv[s] == 0xFFFFu ? kNoSlot : recv[s])
                                   : received_from(s, p, a.np);
        const uint64_t g = (r == kNoSlot) ? (uint64_t)blockIdx.x * a.np + s
                                          : ((uint64_t)f * a.M + p.pred) * a.np + r;
        src[(uint64_t)blockIdx.x * a.np + s] = (int64_t)g;
    }
}

// Debug entry points: the integer stages alone, same device code as k_step.
template <int PPT>
__global__ __launch_bounds__(1024) void k_resample_q(const uint32_t *q, const uint32_t *v,
                                                     uint32_t *anc_out, uint32_t np) {
    __shared__ uint32_t wq[kMaxWaves * 4];
    __shared__ uint32_t mark[PF_MAX_PER_PE_LDS];
    const uint32_t base = blockIdx.x * np;
    uint32_t Qv[PPT], cinc[PPT], anc[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint32_t s = threadIdx.x + k * blockDim.x;
        Qv[k] = (s < np) ? q[base + s] : 0u;
        if (s < np) mark[s] = 0;
    }
    scan_levels<PPT>(Qv, cinc, wq, threadIdx.x);
    __syncthreads();
    const uint32_t T = scan_finish<PPT>(cinc, wq, threadIdx.x);
    mark_offspring<PPT>(Qv, cinc, np, T, v[blockIdx.x], mark, threadIdx.x);
    __syncthreads();
    ancestors_from_marks<PPT>(mark, np, wq, anc, threadIdx.x);
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint32_t j = threadIdx.x * PPT + k;
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

}  // namespace

// k_run<PPT, HALF, LIK> for a context's slots per thread, patch half-width and
// likelihood mode, or NULL when no variant exists (defined in arna_run.hip,
// which is compiled on its own).
void *arna_run_kernel(uint32_t ppt, uint32_t half, uint32_t lik_mode);

