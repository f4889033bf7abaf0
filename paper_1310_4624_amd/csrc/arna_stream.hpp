// The ARNA / RNA iteration with a flexible mapping of PEs to workgroups, for
// the PE sizes at either end of k_step's range:
//   * several PEs per workgroup (P = 2..16 PEs of one filter, each on its own
//     group of whole waves): small PEs share one image tile and one set of
//     barriers, and their log-weights live in LDS;
//   * one PE whose particles do not fit the LDS stage of k_step
//     (PF_MAX_PER_PE_LDS < N_p <= PF_MAX_PER_PE): the log-weights go to a
//     per-context HBM array;
//   * such a PE split over several workgroups, when a context has fewer PEs
//     than compute units (the split kernels at the end of this file: the
//     same passes as three launches).
// The data layout is k_step's (propagated particles plus a 16-bit ancestor
// slot), so the kernels compute the same iteration on the same buffers: Q,
// ancestors and every traced value are k_step's bit for bit, and only the
// FP64 PE sums are added in another order.  Per PE, on its thread group of
// tp threads:
//   pass A (slots t + i tp): the slot's particle -- its own through its
//     ancestor, or pred's slot s_t(pred) (Alg. 3 step 3) -- the step-5
//     normals and propagation, the patch likelihood (LDS tile or frame, as in
//     k_step) and u = lambda + l;
//   pass B (the PE's wave w takes the contiguous slots [w C, (w + 1) C), 64
//     at a time): Q = floor(w Q_max) with w = exp(u - max u), the per-PE FP64
//     sums of step 6, the wave's total of Q;
//   pass C (the same slots): inclusive sums C_i of Q in slot order (one wave
//     scan per 64 slots plus the carry of the earlier ones).  The particles of
//     64 consecutive slots own the consecutive output ranks
//     [first(C_i - Q_i), first(C_i)), first() counting the systematic pointers
//     j T + V below N_p C (step 7); the wave writes those ranks 64 at a time,
//     each lane finding the slot that owns its rank by a binary search over
//     the lanes' first ranks.  These are the ancestors k_step finds from its
//     offspring marks (rank j goes to min { i : N_p C_i > j T + V }), with
//     O(N_p) work however degenerate the weights are;
//   then thread 0 writes the workgroup's PE records (steps 8-9) and, when
//   asked (StepArgs.mout), the last workgroup of the filter computes the
//   once-per-filter master record.
#pragma once

#include "arna_kernels.hpp"

namespace {

constexpr uint32_t kStreamBlock = 1024;   // threads of a streamed PE's workgroup
constexpr uint32_t kMaxPesPerWg = 16;

// Image tile edge of k_step_flex and the split kernels: 32 x 32 pixels, where
// the step kernels load 64 x 64; the workgroups here hold few particles per
// thread (several small PEs, or a PE's segment), for which loading 4096
// pixels costs more than the frame reads of the patches that do not fit a
// smaller tile (with the same result).  Measured on MI355X, us per iteration,
// 64 / 32: at 2^20 particles, 8192 x 128 PEs 64.7 / 55.5 with 4 PEs per
// 256-thread workgroup, 4096 x 256 48.2 / 46.0 with 8 per 512, 1024 x 1024
// 41.1 / 40.0 with 4 per 1024; split, 16 x 65536 40.8 / 38.6, 64 x 16384
// 43.2 / 41.1, 128 x 8192 43.9 / 41.8; one streamed PE per workgroup, 256 x
// 8192 62.0 / 60.6, 512 x 8192 113.6 / 112.3.  Rows are TS + 6 floats apart.
constexpr int kSmallTile = 32;
__host__ __device__ constexpr int tile_pitch(int ts) { return ts + 6; }
static_assert(tile_pitch(kTileCols) == kTilePitch && kTileRows == kTileCols, "square tiles");

struct FlexLds {
    float *tile;       // [TS][tile_pitch(TS)]
    double *wsum;      // [16][6] wave sums (W, W x)
    float *wmax;       // [16] wave maxima of u
    uint32_t *wq;      // [16] wave totals of Q
    uint32_t *flag;    // 1 (+3 padding)
    Prologue *pro;     // [kMaxPesPerWg]
    float *u;          // [P N_p] log-weights (when they stay in LDS)
};
__host__ __device__ constexpr size_t flex_lds_bytes(uint32_t u_slots, int ts) {
    return (size_t)ts * tile_pitch(ts) * sizeof(float) + kMaxWaves * 6 * sizeof(double) +
           kMaxWaves * sizeof(float) + kMaxWaves * sizeof(uint32_t) + 16 +
           kMaxPesPerWg * sizeof(Prologue) + (size_t)u_slots * sizeof(float);
}
template <int TS>
__device__ __forceinline__ FlexLds flex_carve(unsigned char *base) {
    FlexLds l;
    size_t o = 0;
    l.tile = (float *)(base + o);
    o += (size_t)TS * tile_pitch(TS) * sizeof(float);
    l.wsum = (double *)(base + o);
    o += kMaxWaves * 6 * sizeof(double);
    l.wmax = (float *)(base + o);
    o += kMaxWaves * sizeof(float);
    l.wq = (uint32_t *)(base + o);
    o += kMaxWaves * sizeof(uint32_t);
    l.flag = (uint32_t *)(base + o);
    o += 16;
    l.pro = (Prologue *)(base + o);
    o += kMaxPesPerWg * sizeof(Prologue);
    l.u = (float *)(base + o);
    return l;
}

// Fixed-point weight of one slot (the arithmetic of k_step's phase 3).
__device__ __forceinline__ uint32_t stream_q(float u, float lstar, float qmaxf, float &w) {
    w = (lstar == -INFINITY) ? 1.0f : __expf(u - lstar);
    float qf = floorf(w * qmaxf);
    qf = (qf >= 0.f) ? fminf(qf, qmaxf) : 0.f;
    return (uint32_t)qf;
}

// A value the same in every lane of the wave, kept in scalar registers.
__device__ __forceinline__ uint32_t uni(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ float uni(float v) { return __uint_as_float(uni(__float_as_uint(v))); }

// The image tile of a workgroup: TS x TS pixels of z - B around the estimate
// of k-1 moved one step (x + v), zero outside the image; off when the
// estimate is not finite (a PE without mass).
struct TileView {
    int tx0, ty0;
    bool on, inside;
};
template <bool POINT, int TS>
__device__ __forceinline__ TileView load_tile(const StepArgs &a, const double *xh, float *tile,
                                              const uint32_t tid, const uint32_t B) {
    TileView v{0, 0, false, false};
    if (POINT) return v;
    const double cx = xh[0] + xh[2], cy = xh[1] + xh[3];
    if (fabs(cx) < 1e6 && fabs(cy) < 1e6) {   // false for NaN
        v.tx0 = (int)floor(cx + 0.5) - TS / 2;
        v.ty0 = (int)floor(cy + 0.5) - TS / 2;
        v.on = v.tx0 < (int)a.lik.W && v.tx0 + TS > 0 && v.ty0 < (int)a.lik.H && v.ty0 + TS > 0;
        v.inside = v.tx0 >= 0 && v.ty0 >= 0 && v.tx0 + TS <= (int)a.lik.W &&
                   v.ty0 + TS <= (int)a.lik.H;
    }
    if (v.on)
        for (uint32_t idx = tid; idx < (uint32_t)(TS * TS); idx += B) {
            const int uu = v.tx0 + (int)(idx % TS), vv = v.ty0 + (int)(idx / TS);
            const bool in = (unsigned)uu < (unsigned)a.lik.W && (unsigned)vv < (unsigned)a.lik.H;
            tile[(idx / TS) * tile_pitch(TS) + idx % TS] =
                in ? a.lik.img[(size_t)vv * a.lik.W + uu] - a.lik.bg : 0.f;
        }
    return v;
}

// Division by a divisor that is the same in every lane, with one multiply:
// m = floor(2^32 / d) gives floor(n m / 2^32) = floor(n / d) or one less
// (the error n (2^32 - d m) / (d 2^32) is below n / 2^32 < 1), fixed by one
// remainder test.  d = 1 is taken apart (m would not fit).
struct Div32 {
    uint32_t d, m;
};
__device__ __forceinline__ Div32 div32_make(uint32_t d) {
    return Div32{d, d > 1 ? (uint32_t)(0x100000000ull / d) : 0u};
}
__device__ __forceinline__ uint32_t div32(uint32_t n, const Div32 &v) {
    if (v.d == 1) return n;
    uint32_t q = __umulhi(n, v.m);
    if (n - q * v.d >= v.d) ++q;
    return q;
}

// received_from() for N_p <= 65536 in 32-bit arithmetic (every intermediate
// is below N_p^2 <= 2^32) with the divisions by N_p and N_ex as above.
__device__ __forceinline__ uint32_t received_from32(uint32_t s, const Prologue &p, uint32_t np,
                                                    const Div32 &by_np, const Div32 &by_nex) {
    if (p.nex == 0) return kNoSlot;
    const uint32_t sn = s * p.nex;
    const uint32_t t = sn <= p.c_own ? 0u : div32(sn - p.c_own + np - 1, by_np);
    if (t >= p.nex || div32(t * np + p.c_own, by_nex) != s) return kNoSlot;
    return div32(t * np + p.c_pred, by_nex);
}

// The prologue's results, the same in every lane of a wave, to scalar registers.
__device__ __forceinline__ Prologue uniform_prologue(const Prologue *pp) {
    Prologue p = *pp;
    p.pred = uni(p.pred);
    p.nex = uni(p.nex);
    p.c_own = uni(p.c_own);
    p.c_pred = uni(p.c_pred);
    p.lam_own = uni(p.lam_own);
    p.lam_pred = uni(p.lam_pred);
    return p;
}

// Pass A (steps 3-5) over slots s = s0, s0 + step, ... < s1 of PE (f, m):
// the slot's particle (own, through its ancestor, or received), the normals,
// propagation, the likelihood, u = lambda + l to ub[s].  Returns the lane's
// maximum of u.  Called by whole waves (a NaN log-likelihood sets the sticky
// error bit through a wave vote).
template <int HALF, int LIK, int TS>
__device__ __forceinline__ float pass_a(const StepArgs &a, const Prologue &p, uint32_t f,
                                        uint32_t m, uint32_t s0, uint32_t s1, uint32_t step,
                                        float *ub, const float *tile, const TileView &tv) {
    constexpr int P = 2 * HALF + 1;
    constexpr bool POINT = LIK == kLikPoint;
    const uint32_t np = a.np, N = a.N;
    const uint32_t pe_base = (f * a.M + m) * np, pred_base = (f * a.M + p.pred) * np;
    const DebugBufs *D = a.dbg;
    const bool trace = D && D->t_q;
    float umax = -INFINITY;
    bool bad = false;
    const Div32 by_np = div32_make(np), by_nex = div32_make(p.nex ? p.nex : 1u);
#pragma unroll 1
    for (uint32_t s = s0; s < s1; s += step) {
        const uint32_t r = received_from32(s, p, np, by_np, by_nex);
        const uint32_t blk = (r == kNoSlot) ? pe_base : pred_base;   // PE whose slot it takes
        const uint32_t sb = blk + ((r == kNoSlot) ? s : r);          // that resampled slot
        const float lam = (r == kNoSlot) ? p.lam_own : p.lam_pred;
        const uint32_t gsrc = blk + a.ain[sb];                         // its propagated particle
        float x[5], e[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) x[c] = a.pin[(size_t)c * N + gsrc];
        five_normals(philox(m * np + s, a.k, f, kTagProp << 24, a.key0, a.key1), e);
        propagate(x, e, a.dyn);
#pragma unroll
        for (int c = 0; c < 5; ++c) a.pout[(size_t)c * N + pe_base + s] = x[c];
        if (trace) {
            D->t_src[pe_base + s] = (int64_t)sb;
            D->t_lam[pe_base + s] = lam;
#pragma unroll
            for (int c = 0; c < 5; ++c) D->t_prop[(size_t)c * N + pe_base + s] = x[c];
        }
        float ell = 0.f;
        int u0, v0;
        if (POINT) {
            ell = loglik_point(x, a.lik, f);
        } else if (patch_origin<HALF>(x[0], x[1], a.lik.W, a.lik.H, u0, v0)) {
            const int du = u0 - tv.tx0, dv = v0 - tv.ty0;
            if (tv.on && (unsigned)du <= (unsigned)(TS - P) &&
                (unsigned)dv <= (unsigned)(TS - P)) {
                constexpr int TP = tile_pitch(TS);
                const float *pix = tile + dv * TP + du;
                if (LIK == kLikPoisson)
                    ell = patch_loglik_poisson<HALF, kFromTile>(x, u0, v0, pix, TP, a.lik);
                else
                    ell = tv.inside
                              ? patch_loglik<HALF, kFromTileInside>(x, u0, v0, pix, TP, a.lik)
                              : patch_loglik<HALF, kFromTile>(x, u0, v0, pix, TP, a.lik);
            } else if (u0 >= 0 && v0 >= 0 && u0 + P <= (int)a.lik.W && v0 + P <= (int)a.lik.H) {
                const float *pix = a.lik.img + (size_t)v0 * a.lik.W + u0;
                ell = (LIK == kLikPoisson)
                          ? patch_loglik_poisson<HALF, kFromImage>(x, u0, v0, pix, 0, a.lik)
                          : patch_loglik<HALF, kFromImage>(x, u0, v0, pix, 0, a.lik);
            } else {
                ell = (LIK == kLikPoisson)
                          ? patch_loglik_poisson<HALF, kFromImageBorder>(x, u0, v0, a.lik.img, 0,
                                                                          a.lik)
                          : patch_loglik<HALF, kFromImageBorder>(x, u0, v0, a.lik.img, 0, a.lik);
            }
        }
        bad |= (ell != ell);
        const float us = lam + ell;
        umax = fmaxf(umax, us);
        ub[s] = us;
        if (trace) D->t_ell[pe_base + s] = ell;
    }
    if (__any(bad) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(a.err, 1u);
    return umax;
}

// Pass B (step 6 and the totals of step 7) over the contiguous slots
// [c_lo, c_hi) of the PE whose slots start at pe_base, 64 at a time: the
// lane's total of Q and its FP64 sums (W, W x).
__device__ __forceinline__ uint32_t pass_b(const StepArgs &a, const float *ub, uint32_t pe_base,
                                           uint32_t c_lo, uint32_t c_hi, float lstar,
                                           double (&sums)[6]) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const DebugBufs *D = a.dbg;
    const bool trace = D && D->t_q;
    const float qmaxf = (float)a.qmax;
    uint32_t tot = 0;
    for (uint32_t base = c_lo; base < c_hi; base += kWave) {
        const uint32_t s = base + lane;
        if (s < c_hi) {
            float w;
            const uint32_t Q = stream_q(ub[s], lstar, qmaxf, w);
            tot += Q;
            const double wd = (double)w;
            sums[0] += wd;
#pragma unroll
            for (int c = 0; c < 5; ++c)
                sums[1 + c] += wd * (double)a.pout[(size_t)c * a.N + pe_base + s];
            if (trace) D->t_q[pe_base + s] = Q;
        }
    }
    return tot;
}

// Pass C (step 7) over the same slots, by the whole wave: `carry` is the sum
// of Q over the PE's slots before c_lo; writes the ancestors of the output
// ranks these slots own.  T > 0.
__device__ __forceinline__ void pass_c(const StepArgs &a, const float *ub, uint32_t pe_base,
                                       uint32_t c_lo, uint32_t c_hi, float lstar, uint32_t carry,
                                       uint32_t T, uint32_t V) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t np = a.np;
    const DebugBufs *D = a.dbg;
    const bool trace = D && D->t_q;
    const float qmaxf = (float)a.qmax;
    const double inv_T = 1.0 / (double)T;
    for (uint32_t base = c_lo; base < c_hi; base += kWave) {
        const uint32_t s = base + lane;
        float w;
        const uint32_t Q = (s < c_hi) ? stream_q(ub[s], lstar, qmaxf, w) : 0u;
        const uint32_t incl = wave_incl_scan_u32(Q);
        // first rank of this lane's slot; non-decreasing over the lanes
        const uint32_t j0 = first_offspring(carry + incl - Q, np, T, V, inv_T);
        carry += lane63(incl);
        const uint32_t J0 = (uint32_t)__builtin_amdgcn_readlane((int)j0, 0);
        const uint32_t J1 = first_offspring(carry, np, T, V, inv_T);   // wave-uniform
        for (uint32_t r0 = J0; r0 < J1; r0 += kWave) {
            const uint32_t r = r0 + lane;
            // the last lane whose first rank is <= r owns rank r
            uint32_t lo = 0;
#pragma unroll
            for (uint32_t step = kWave / 2; step >= 1; step /= 2) {
                const uint32_t cand = lo + step;
                if ((uint32_t)__shfl((int)j0, (int)cand) <= r) lo = cand;
            }
            if (r < J1) {
                a.aout[pe_base + r] = (uint16_t)(base + lo);
                if (trace) D->t_anc[pe_base + r] = base + lo;
            }
        }
    }
}

// Step 7 when the choices are not drawn: replayed ancestors (test support) or,
// with no weight anywhere, slot 0 for every rank (as k_step's marks give);
// ranks j = j0, j0 + step, ... < j1.
__device__ __forceinline__ void fixed_ancestors(const StepArgs &a, uint32_t pe_base, uint32_t j0,
                                                uint32_t j1, uint32_t step) {
    const DebugBufs *D = a.dbg;
    const bool trace = D && D->t_q;
    for (uint32_t j = j0; j < j1; j += step) {
        const uint32_t anc = a.force_anc ? a.force_anc[pe_base + j] : 0u;
        a.aout[pe_base + j] = (uint16_t)anc;
        if (trace) D->t_anc[pe_base + j] = anc;
    }
}

// ppw PEs of one filter per workgroup (tp = blockDim.x / ppw threads each, a
// multiple of 64; workgroup g of filter f holds PEs g ppw .. g ppw + ppw - 1,
// the last workgroup of a filter possibly fewer).  ULDS: the log-weights stay
// in LDS (ppw N_p floats); else they go to u_hbm [N] (context scratch, fully
// rewritten).  lm_out, if not NULL, receives every PE's log-mass L^(m) beside
// its record ([F M] doubles, contiguous for the master record's reduction).
template <int HALF, int LIK, bool ULDS>
__device__ __forceinline__ void flex_body(const StepArgs &a, float *u_hbm, const uint32_t ppw,
                                          const uint32_t bid, double *lm_out) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr bool POINT = LIK == kLikPoint;
    const uint32_t tid = threadIdx.x;
    const uint32_t M = a.M, np = a.np;
    const uint32_t B = blockDim.x, tp = B / ppw;
    const uint32_t G = (M + ppw - 1) / ppw;   // workgroups per filter
    const uint32_t f = bid / G, m0 = (bid % G) * ppw;
    const uint32_t lane = tid & (kWave - 1), wave = tid / kWave;
    // this thread's PE in the group (whole waves per PE: the same in every
    // lane), its rank in the PE's thread group
    const uint32_t lp = uni(tid / tp), lt = tid - lp * tp;
    const uint32_t wpp = tp / kWave, w_first = lp * wpp;   // the PE's waves
    const uint32_t m = m0 + lp;
    const bool active = m < M;   // the same in every lane of a wave
    const uint32_t pe_base = (f * M + m) * np;
    constexpr int TS = kSmallTile;
    FlexLds L = flex_carve<TS>(smem);
    float *ub = ULDS ? L.u + lp * np : u_hbm + pe_base;
    const DebugBufs *D = a.dbg;
    const bool trace = D && D->t_q;

    // ---- steps 1-2 (the first wave of each PE); the image tile around the
    // estimate of k-1 of the group's first PE (every thread)
    if (active && lt < kWave) {
        if (a.min)
            prologue_master(a, f, m, L.pro + lp, lane);
        else
            prologue_wave(a, f, m, L.pro + lp, lane);
    }
    const TileView tv = load_tile<POINT, TS>(a, a.rin[f * M + m0].xhat, L.tile, tid, B);
    __syncthreads();   // prologues and tile visible

    // ---- pass A (steps 3-5)
    float umax = -INFINITY;
    if (active) {
        const Prologue p = uniform_prologue(L.pro + lp);
        umax = pass_a<HALF, LIK, TS>(a, p, f, m, lt, np, tp, ub, L.tile, tv);
    }
    umax = wave_max_f32(umax);
    if (lane == 0) L.wmax[wave] = umax;
    __syncthreads();   // wave maxima; u and the propagated particles stored
    float lstar = L.wmax[w_first];
    for (uint32_t w = 1; w < wpp; ++w) lstar = fmaxf(lstar, L.wmax[w_first + w]);

    // ---- pass B (step 6 and the totals of step 7)
    const uint32_t wi = wave - w_first;
    const uint32_t chunk = (np + wpp * kWave - 1) / (wpp * kWave) * kWave;
    const uint32_t c_lo = wi * chunk;
    const uint32_t c_hi = active ? (c_lo + chunk < np ? c_lo + chunk : np) : 0u;   // may be <= c_lo
    double sums[6] = {0, 0, 0, 0, 0, 0};
    const uint32_t tot = pass_b(a, ub, pe_base, c_lo, c_hi, lstar, sums);
    {
        const uint32_t wt = lane63(wave_incl_scan_u32(tot));
        if (lane == 0) L.wq[wave] = wt;
        const double t = wave_total6_f64(sums, lane);
        if ((lane & 7u) == 0 && lane < 48) L.wsum[wave * 6 + (lane >> 3)] = t;
    }
    __syncthreads();   // wave totals
    uint32_t carry = 0, T = 0;
    for (uint32_t w = 0; w < wpp; ++w) {
        if (w < wi) carry += L.wq[w_first + w];
        T += L.wq[w_first + w];
    }
    const uint32_t V = mulshift(philox(m, a.k, f, kTagResample << 24, a.key0, a.key1).x, T);

    // ---- pass C (step 7): ancestors of the output ranks
    if (active) {
        if (a.force_anc || T == 0)
            fixed_ancestors(a, pe_base, lt, np, tp);
        else
            pass_c(a, ub, pe_base, c_lo, c_hi, lstar, carry, T, V);
    }

    // ---- steps 8-9: the records of the group's PEs, all by thread 0 (the
    // wave totals they need are in LDS since the last barrier)
    if (tid == 0) {
        for (uint32_t q = 0; q < ppw && m0 + q < M; ++q) {
            const uint32_t mq = m0 + q, wq0 = q * wpp;
            double t6[6] = {0, 0, 0, 0, 0, 0};
            float ls = L.wmax[wq0];
            uint32_t Tq = 0;
            for (uint32_t w = 0; w < wpp; ++w) {
                for (int c = 0; c < 6; ++c) t6[c] += L.wsum[(wq0 + w) * 6 + c];
                ls = fmaxf(ls, L.wmax[wq0 + w]);
                Tq += L.wq[wq0 + w];
            }
            pf_pe_record rec;
            rec.log_mass = (ls == -INFINITY) ? -INFINITY : (double)ls + log(t6[0]);
            for (int c = 0; c < 5; ++c) rec.xhat[c] = t6[1 + c] / t6[0];
            rec.lstar = ls;
            rec.total_q = Tq;
            a.rout[f * M + mq] = rec;
            if (lm_out) lm_out[f * M + mq] = rec.log_mass;
            const Prologue *pq = L.pro + q;
            if (mq == 0) {
                a.nex_used[f] = pq->nex;
                if (a.nex_rec) a.nex_rec[f] = pq->nex;
            }
            if (trace) {
                D->t_pred[f * M + mq] = pq->pred;
                D->t_v[f * M + mq] =
                    mulshift(philox(mq, a.k, f, kTagResample << 24, a.key0, a.key1).x, Tq);
            }
        }
    }
    if (a.mout) {
        // the last workgroup of the filter to publish its records computes the
        // master step of this iteration (records made visible by the fence
        // before the arrival count; the counter is reset for the next one)
        if (tid == 0) {
            __threadfence();
            *L.flag = (atomicAdd(&a.arrive[f], 1u) == G - 1) ? 1u : 0u;
        }
        __syncthreads();
        if (*L.flag) {
            __threadfence();
            master_block(a.rout + (size_t)f * M, M, np, a.mode, a.fixed_nex, a.cutoff_ppm,
                         L.wsum, a.mout + f);
            if (tid == 0) atomicExch(&a.arrive[f], 0u);
        }
    }
}


template <int HALF, int LIK, bool ULDS>
__global__ __launch_bounds__(1024) void k_step_flex(StepArgs a, float *u_hbm, uint32_t ppw,
                                                    double *lm_out) {
    flex_body<HALF, LIK, ULDS>(a, u_hbm, ppw, blockIdx.x, lm_out);
}

// The context of workgroup `bid` in a batched launch: contexts own the
// workgroup ranges [first[i], first[i + 1]).
__device__ __forceinline__ uint32_t batch_context(const uint32_t *first, uint32_t n,
                                                  uint32_t bid) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (first[mid] <= bid)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Several contexts with several PEs per workgroup (or streamed PEs) in one
// launch: context i has arguments args[i], log-weight array u[i] and the
// workgroups [first[i], first[i + 1]); all share ppw and the block size.
template <int HALF, int LIK, bool ULDS>
__global__ __launch_bounds__(1024) void k_step_flex_batch(const StepArgs *args,
                                                          const uint32_t *first, uint32_t n,
                                                          float *const *u, uint32_t ppw) {
    const uint32_t i = batch_context(first, n, blockIdx.x);
    const StepArgs a = args[i];
    flex_body<HALF, LIK, ULDS>(a, u[i], ppw, blockIdx.x - first[i], nullptr);
}

// ---------------------------------------------------------------- split PEs
// A PE beyond the LDS stage split over G workgroups of the same size, each
// taking the S = kSplitSlots consecutive slots [g S, g S + S) of its PE
// (workgroup w is segment g = w mod G of PE w / G).  The three passes become
// three launches, the workgroup boundary replacing the barriers of
// k_step_flex: (1) steps 3-5 and the segment's maximum of u; (2) Q, the FP64
// sums and the wave totals of Q; (3) the carry of every wave from the totals
// of the PE's earlier segments and waves, the ancestors, and the PE record
// (segment 0).  Per-segment results go through the context's SplitBufs.
constexpr uint32_t kSplitBlock = 512;
constexpr uint32_t kSplitSlots = 4 * kSplitBlock;
constexpr uint32_t kSplitWaves = kSplitBlock / 64;

struct SplitBufs {
    float *u;          // [N] log-weights
    float *seg_max;    // [F M G] segment maxima of u
    uint32_t *seg_wq;  // [F M G][kSplitWaves] wave totals of Q
    double *seg_sum;   // [F M G][6] segment sums (W, W x)
    uint32_t G;        // segments per PE
};

__host__ __device__ constexpr size_t split_lds_bytes() { return flex_lds_bytes(0, kSmallTile); }

// The segment's slot range and the PE's maximum of u (from the segment maxima).
struct Segment {
    uint32_t bid, pe, f, m, g, s0, s1, pe_base;   // bid: the segment's workgroup in its context
};
__device__ __forceinline__ Segment segment_of(const StepArgs &a, const SplitBufs &sb,
                                              const uint32_t bid) {
    Segment s;
    s.bid = bid;
    s.pe = bid / sb.G;
    s.g = bid - s.pe * sb.G;
    s.f = s.pe / a.M;
    s.m = s.pe - s.f * a.M;
    s.s0 = s.g * kSplitSlots;
    s.s1 = s.s0 + kSplitSlots < a.np ? s.s0 + kSplitSlots : a.np;
    s.pe_base = s.pe * a.np;
    return s;
}
// (every lane loads at most one segment maximum: G <= 32 = 65536 / 2048)
__device__ __forceinline__ float pe_max_u(const SplitBufs &sb, uint32_t pe) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const float l = lane < sb.G ? sb.seg_max[(size_t)pe * sb.G + lane] : -INFINITY;
    return wave_max_f32(l);
}
constexpr uint32_t kMaxSegments = PF_MAX_PER_PE / kSplitSlots;   // 32

template <int HALF, int LIK>
__device__ __forceinline__ void split_weights_body(const StepArgs &a, const SplitBufs &sb,
                                                   const uint32_t bid) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr bool POINT = LIK == kLikPoint;
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const Segment sg = segment_of(a, sb, bid);
    FlexLds L = flex_carve<kSmallTile>(smem);
    if (wave == 0) prologue_wave(a, sg.f, sg.m, L.pro, lane);
    const TileView tv =
        load_tile<POINT, kSmallTile>(a, a.rin[sg.pe].xhat, L.tile, tid, kSplitBlock);
    __syncthreads();   // prologue and tile visible
    const Prologue p = uniform_prologue(L.pro);
    float umax = pass_a<HALF, LIK, kSmallTile>(a, p, sg.f, sg.m, sg.s0 + tid, sg.s1,
                                              kSplitBlock, sb.u + sg.pe_base, L.tile, tv);
    umax = wave_max_f32(umax);
    if (lane == 0) L.wmax[wave] = umax;
    __syncthreads();
    if (tid == 0) {
        float l = L.wmax[0];
        for (uint32_t w = 1; w < kSplitWaves; ++w) l = fmaxf(l, L.wmax[w]);
        sb.seg_max[sg.bid] = l;
        if (sg.g == 0) {
            if (sg.m == 0) {
                a.nex_used[sg.f] = p.nex;
                if (a.nex_rec) a.nex_rec[sg.f] = p.nex;
            }
            if (a.dbg && a.dbg->t_q) a.dbg->t_pred[sg.pe] = p.pred;
        }
    }
}

// The wave's contiguous share of the segment (64 slots at a time).
__device__ __forceinline__ void wave_chunk(const Segment &sg, uint32_t wave, uint32_t &c_lo,
                                           uint32_t &c_hi) {
    const uint32_t len = sg.s1 - sg.s0;
    const uint32_t chunk = (len + kSplitWaves * kWave - 1) / (kSplitWaves * kWave) * kWave;
    c_lo = sg.s0 + wave * chunk;
    c_hi = c_lo + chunk < sg.s1 ? c_lo + chunk : sg.s1;
}

__device__ __forceinline__ void split_totals_body(const StepArgs &a, const SplitBufs &sb,
                                                  const uint32_t bid) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const Segment sg = segment_of(a, sb, bid);
    FlexLds L = flex_carve<kSmallTile>(smem);
    const float lstar = pe_max_u(sb, sg.pe);
    uint32_t c_lo, c_hi;
    wave_chunk(sg, wave, c_lo, c_hi);
    double sums[6] = {0, 0, 0, 0, 0, 0};
    const uint32_t tot = pass_b(a, sb.u + sg.pe_base, sg.pe_base, c_lo, c_hi, lstar, sums);
    const uint32_t wt = lane63(wave_incl_scan_u32(tot));
    if (lane == 0) sb.seg_wq[(size_t)sg.bid * kSplitWaves + wave] = wt;
    const double s6 = wave_total6_f64(sums, lane);
    if ((lane & 7u) == 0 && lane < 48) L.wsum[wave * 6 + (lane >> 3)] = s6;
    __syncthreads();
    if (tid < 6) {
        double acc = 0;
        for (uint32_t w = 0; w < kSplitWaves; ++w) acc += L.wsum[w * 6 + tid];
        sb.seg_sum[(size_t)sg.bid * 6 + tid] = acc;
    }
}

__device__ __forceinline__ void split_ancestors_body(const StepArgs &a, const SplitBufs &sb,
                                                     const uint32_t bid) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const Segment sg = segment_of(a, sb, bid);
    FlexLds L = flex_carve<kSmallTile>(smem);
    const float lstar = pe_max_u(sb, sg.pe);
    // wave 0: the sum of the wave totals of the PE's earlier segments and of
    // this segment's earlier waves (exclusive prefix in (segment, wave)
    // order), and the total T
    if (wave == 0) {
        constexpr uint32_t kPer = kMaxSegments * kSplitWaves / kWave;   // values per lane
        const uint32_t *wq = sb.seg_wq + (size_t)sg.pe * sb.G * kSplitWaves;
        const uint32_t n = sb.G * kSplitWaves, mine = sg.g * kSplitWaves;
        uint32_t v[kPer];
#pragma unroll
        for (uint32_t j = 0; j < kPer; ++j) {   // all loads in flight before the scans
            const uint32_t i = j * kWave + lane;
            v[j] = i < n ? wq[i] : 0u;
        }
        uint32_t run = 0;
#pragma unroll
        for (uint32_t j = 0; j < kPer; ++j) {
            const uint32_t i = j * kWave + lane;
            const uint32_t incl = wave_incl_scan_u32(v[j]);
            if (i >= mine && i < mine + kSplitWaves) L.wq[i - mine] = run + incl - v[j];
            run += lane63(incl);
        }
        if (lane == 0) *L.flag = run;
    }
    __syncthreads();
    const uint32_t T = *L.flag, carry = L.wq[wave];
    const uint32_t V =
        mulshift(philox(sg.m, a.k, sg.f, kTagResample << 24, a.key0, a.key1).x, T);
    if (a.force_anc || T == 0) {
        fixed_ancestors(a, sg.pe_base, sg.s0 + tid, sg.s1, kSplitBlock);
    } else {
        uint32_t c_lo, c_hi;
        wave_chunk(sg, wave, c_lo, c_hi);
        pass_c(a, sb.u + sg.pe_base, sg.pe_base, c_lo, c_hi, lstar, carry, T, V);
    }
    // steps 8-9: the PE record from the segment sums (lane g loads segment
    // g's, the wave totals them)
    if (sg.g == 0 && wave == 0) {
        double t6[6] = {0, 0, 0, 0, 0, 0};
        if (lane < sb.G)
#pragma unroll
            for (int c = 0; c < 6; ++c) t6[c] = sb.seg_sum[((size_t)sg.pe * sb.G + lane) * 6 + c];
        const double tw = wave_total6_f64(t6, lane);
        if ((lane & 7u) == 0 && lane < 48) L.wsum[lane >> 3] = tw;
    }
    __syncthreads();
    if (sg.g == 0 && tid == 0) {
        double t6[6];
        for (int c = 0; c < 6; ++c) t6[c] = L.wsum[c];
        pf_pe_record rec;
        rec.log_mass = (lstar == -INFINITY) ? -INFINITY : (double)lstar + log(t6[0]);
        for (int c = 0; c < 5; ++c) rec.xhat[c] = t6[1 + c] / t6[0];
        rec.lstar = lstar;
        rec.total_q = T;
        a.rout[sg.pe] = rec;
        if (a.dbg && a.dbg->t_q) a.dbg->t_v[sg.pe] = V;
    }
}


// The three launches of a split iteration, for one context and batched (the
// contexts of a batched launch own the workgroup ranges [first[i],
// first[i + 1]) and have the buffers sb[i]).
template <int HALF, int LIK>
__global__ __launch_bounds__(kSplitBlock) void k_split_weights(StepArgs a, SplitBufs sb) {
    split_weights_body<HALF, LIK>(a, sb, blockIdx.x);
}
__global__ __launch_bounds__(kSplitBlock) void k_split_totals(StepArgs a, SplitBufs sb) {
    split_totals_body(a, sb, blockIdx.x);
}
__global__ __launch_bounds__(kSplitBlock) void k_split_ancestors(StepArgs a, SplitBufs sb) {
    split_ancestors_body(a, sb, blockIdx.x);
}
template <int HALF, int LIK>
__global__ __launch_bounds__(kSplitBlock) void k_split_weights_batch(const StepArgs *args,
                                                                     const uint32_t *first,
                                                                     uint32_t n,
                                                                     const SplitBufs *sb) {
    const uint32_t i = batch_context(first, n, blockIdx.x);
    const StepArgs a = args[i];
    const SplitBufs s = sb[i];
    split_weights_body<HALF, LIK>(a, s, blockIdx.x - first[i]);
}
__global__ __launch_bounds__(kSplitBlock) void k_split_totals_batch(const StepArgs *args,
                                                                    const uint32_t *first,
                                                                    uint32_t n,
                                                                    const SplitBufs *sb) {
    const uint32_t i = batch_context(first, n, blockIdx.x);
    const StepArgs a = args[i];
    const SplitBufs s = sb[i];
    split_totals_body(a, s, blockIdx.x - first[i]);
}
__global__ __launch_bounds__(kSplitBlock) void k_split_ancestors_batch(const StepArgs *args,
                                                                       const uint32_t *first,
                                                                       uint32_t n,
                                                                       const SplitBufs *sb) {
    const uint32_t i = batch_context(first, n, blockIdx.x);
    const StepArgs a = args[i];
    const SplitBufs s = sb[i];
    split_ancestors_body(a, s, blockIdx.x - first[i]);
}

}  // namespace
