// The ARNA / RNA iteration for PEs whose particles do not fit the LDS stage of
// k_step (PF_MAX_PER_PE_LDS < N_p <= PF_MAX_PER_PE): one workgroup of 1024
// threads per PE, as in k_step, with the particles streamed through HBM.  The
// data layout is k_step's (propagated particles plus a 16-bit ancestor slot),
// so the two kernels compute the same iteration on the same buffers.
//
//   pass A (slots t + i B): the slot's particle -- its own through its
//     ancestor, or pred's slot s_t(pred) (Alg. 3 step 3) -- the step-5
//     normals and propagation, the patch likelihood (LDS tile or frame, as in
//     k_step) and u = lambda + l, stored in the context's log-weight array;
//   pass B (wave w takes the contiguous slots [w C, (w + 1) C), 64 at a time):
//     Q = floor(w Q_max) with w = exp(u - max u), the per-PE FP64 sums of
//     step 6, the wave's total of Q;
//   pass C (the same slots): inclusive sums C_i of Q in slot order (one wave
//     scan per 64 slots plus the carry of the earlier ones).  The particles of
//     64 consecutive slots own the consecutive output ranks
//     [first(C_i - Q_i), first(C_i)), first() counting the systematic pointers
//     j T + V below N_p C (step 7); the wave writes those ranks 64 at a time,
//     each lane finding the slot that owns its rank by a binary search over
//     the lanes' first ranks.  These are the ancestors k_step finds from its
//     offspring marks (rank j goes to min { i : N_p C_i > j T + V }), with
//     O(N_p) work however degenerate the weights are;
//   then the PE record (steps 8-9).
// Contexts of this size use neither lineage tags nor the once-per-filter
// master record (M >= 2048), and are never batched.
#pragma once

#include "arna_kernels.hpp"

namespace {

constexpr uint32_t kStreamBlock = 1024;

struct StreamLds {
    float *tile;       // [kTileRows][kTilePitch]
    double *wsum;      // [16][6] wave sums (W, W x)
    float *wmax;       // [16] wave maxima of u
    uint32_t *wq;      // [16] wave totals of Q
    Prologue *pro;     // 1
};
__host__ __device__ constexpr size_t stream_lds_bytes() {
    return (size_t)kTileRows * kTilePitch * sizeof(float) + kMaxWaves * 6 * sizeof(double) +
           kMaxWaves * sizeof(float) + kMaxWaves * sizeof(uint32_t) + 32;
}
__device__ __forceinline__ StreamLds stream_carve(unsigned char *base) {
    StreamLds l;
    size_t o = 0;
    l.tile = (float *)(base + o);
    o += (size_t)kTileRows * kTilePitch * sizeof(float);
    l.wsum = (double *)(base + o);
    o += kMaxWaves * 6 * sizeof(double);
    l.wmax = (float *)(base + o);
    o += kMaxWaves * sizeof(float);
    l.wq = (uint32_t *)(base + o);
    o += kMaxWaves * sizeof(uint32_t);
    l.pro = (Prologue *)(base + o);
    return l;
}

// Fixed-point weight of one slot (the arithmetic of k_step's phase 3).
__device__ __forceinline__ uint32_t stream_q(float u, float lstar, float qmaxf, float &w) {
    w = (lstar == -INFINITY) ? 1.0f : __expf(u - lstar);
    float qf = floorf(w * qmaxf);
    qf = (qf >= 0.f) ? fminf(qf, qmaxf) : 0.f;
    return (uint32_t)qf;
}

// u: [N] log-weights of the iteration (context scratch, fully rewritten).
template <int HALF, int LIK>
__global__ __launch_bounds__(1024) void k_step_stream(StepArgs a, float *u) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int P = 2 * HALF + 1;
    constexpr bool POINT = LIK == kLikPoint;
    const uint32_t tid = threadIdx.x, bid = blockIdx.x;
    const uint32_t M = a.M, np = a.np, N = a.N;
    const uint32_t f = bid / M, m = bid % M;
    const uint32_t B = blockDim.x;
    const uint32_t lane = tid & (kWave - 1), wave = tid / kWave, nwaves = B / kWave;
    StreamLds L = stream_carve(smem);
    const uint32_t pe_base = bid * np;
    const DebugBufs *D = a.dbg;
    const bool trace = D && D->t_q;

    // ---- steps 1-2 (wave 0); the image tile around this PE's estimate of
    // k-1 moved one step (every thread)
    if (wave == 0) {
        if (a.min)
            prologue_master(a, f, m, L.pro, tid);
        else
            prologue_wave(a, f, m, L.pro, tid);
    }
    int tx0 = 0, ty0 = 0;
    bool tile_on = false, tile_inside = false;
    if (!POINT) {
        const double *xh = a.rin[bid].xhat;
        const double cx = xh[0] + xh[2], cy = xh[1] + xh[3];
        if (fabs(cx) < 1e6 && fabs(cy) < 1e6) {   // false for NaN (a PE without mass)
            tx0 = (int)floor(cx + 0.5) - kTileCols / 2;
            ty0 = (int)floor(cy + 0.5) - kTileRows / 2;
            tile_on = tx0 < (int)a.lik.W && tx0 + kTileCols > 0 && ty0 < (int)a.lik.H &&
                      ty0 + kTileRows > 0;
            tile_inside = tx0 >= 0 && ty0 >= 0 && tx0 + kTileCols <= (int)a.lik.W &&
                          ty0 + kTileRows <= (int)a.lik.H;
        }
        if (tile_on)
            for (uint32_t idx = tid; idx < (uint32_t)(kTileRows * kTileCols); idx += B) {
                const int uu = tx0 + (int)(idx % kTileCols), vv = ty0 + (int)(idx / kTileCols);
                const bool in =
                    (unsigned)uu < (unsigned)a.lik.W && (unsigned)vv < (unsigned)a.lik.H;
                L.tile[(idx / kTileCols) * kTilePitch + idx % kTileCols] =
                    in ? a.lik.img[(size_t)vv * a.lik.W + uu] - a.lik.bg : 0.f;
            }
    }
    __syncthreads();   // prologue and tile visible
    const Prologue p = *L.pro;
    const uint32_t pred_base = (f * M + p.pred) * np;

    // ---- pass A (steps 3-5)
    float umax = -INFINITY;
    bool bad = false;
    for (uint32_t s = tid; s < np; s += B) {
        const uint32_t r = received_from(s, p, np);
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
        float ell = 0.f;
        int u0, v0;
        if (POINT) {
            ell = loglik_point(x, a.lik, f);
        } else if (patch_origin<HALF>(x[0], x[1], a.lik.W, a.lik.H, u0, v0)) {
            const int du = u0 - tx0, dv = v0 - ty0;
            if (tile_on && (unsigned)du <= (unsigned)(kTileCols - P) &&
                (unsigned)dv <= (unsigned)(kTileRows - P)) {
                const float *pix = L.tile + dv * kTilePitch + du;
                if (LIK == kLikPoisson)
                    ell = patch_loglik_poisson<HALF, kFromTile>(x, u0, v0, pix, kTilePitch, a.lik);
                else
                    ell = tile_inside ? patch_loglik<HALF, kFromTileInside>(x, u0, v0, pix,
                                                                            kTilePitch, a.lik)
                                      : patch_loglik<HALF, kFromTile>(x, u0, v0, pix, kTilePitch,
                                                                      a.lik);
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
        u[pe_base + s] = us;
        if (trace) {
            D->t_src[pe_base + s] = (int64_t)sb;
            D->t_lam[pe_base + s] = lam;
            D->t_ell[pe_base + s] = ell;
#pragma unroll
            for (int c = 0; c < 5; ++c) D->t_prop[(size_t)c * N + pe_base + s] = x[c];
        }
    }
    if (__any(bad) && lane == 0) atomicOr(a.err, 1u);
    umax = wave_max_f32(umax);
    if (lane == 0) L.wmax[wave] = umax;
    __syncthreads();   // wave maxima; u and the propagated particles stored
    float lstar = L.wmax[0];
    for (uint32_t w = 1; w < nwaves; ++w) lstar = fmaxf(lstar, L.wmax[w]);

    // ---- pass B (step 6 and the totals of step 7)
    const uint32_t chunk = (np + nwaves * kWave - 1) / (nwaves * kWave) * kWave;
    const uint32_t c_lo = wave * chunk;
    const uint32_t c_hi = c_lo + chunk < np ? c_lo + chunk : np;   // may be <= c_lo
    const float qmaxf = (float)a.qmax;
    double sums[6] = {0, 0, 0, 0, 0, 0};
    uint32_t tot = 0;
    for (uint32_t base = c_lo; base < c_hi; base += kWave) {
        const uint32_t s = base + lane;
        if (s < c_hi) {
            float w;
            const uint32_t Q = stream_q(u[pe_base + s], lstar, qmaxf, w);
            tot += Q;
            const double wd = (double)w;
            sums[0] += wd;
#pragma unroll
            for (int c = 0; c < 5; ++c)
                sums[1 + c] += wd * (double)a.pout[(size_t)c * N + pe_base + s];
            if (trace) D->t_q[pe_base + s] = Q;
        }
    }
    {
        const uint32_t wt = lane63(wave_incl_scan_u32(tot));
        if (lane == 0) L.wq[wave] = wt;
        const double t = wave_total6_f64(sums, lane);
        if ((lane & 7u) == 0 && lane < 48) L.wsum[wave * 6 + (lane >> 3)] = t;
    }
    __syncthreads();   // wave totals
    uint32_t carry = 0, T = 0;
    for (uint32_t w = 0; w < nwaves; ++w) {
        if (w < wave) carry += L.wq[w];
        T += L.wq[w];
    }
    const uint32_t V = mulshift(philox(m, a.k, f, kTagResample << 24, a.key0, a.key1).x, T);

    // ---- pass C (step 7): ancestors of the output ranks
    if (a.force_anc) {   // replay of another run's choices (test support)
        for (uint32_t j = tid; j < np; j += B) {
            const uint32_t anc = a.force_anc[pe_base + j];
            a.aout[pe_base + j] = (uint16_t)anc;
            if (trace) D->t_anc[pe_base + j] = anc;
        }
    } else if (T == 0) {   // no weight anywhere: every rank takes slot 0, as in k_step
        for (uint32_t j = tid; j < np; j += B) {
            a.aout[pe_base + j] = 0;
            if (trace) D->t_anc[pe_base + j] = 0;
        }
    } else {
        const double inv_T = 1.0 / (double)T;
        for (uint32_t base = c_lo; base < c_hi; base += kWave) {
            const uint32_t s = base + lane;
            float w;
            const uint32_t Q = (s < c_hi) ? stream_q(u[pe_base + s], lstar, qmaxf, w) : 0u;
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

    // ---- steps 8-9: the PE record
    if (tid == 0) {
        double t6[6] = {0, 0, 0, 0, 0, 0};
        for (uint32_t w = 0; w < nwaves; ++w)
            for (int c = 0; c < 6; ++c) t6[c] += L.wsum[w * 6 + c];
        pf_pe_record rec;
        rec.log_mass = (lstar == -INFINITY) ? -INFINITY : (double)lstar + log(t6[0]);
        for (int c = 0; c < 5; ++c) rec.xhat[c] = t6[1 + c] / t6[0];
        rec.lstar = lstar;
        rec.total_q = T;
        a.rout[bid] = rec;
        if (m == 0) {
            a.nex_used[f] = p.nex;
            if (a.nex_rec) a.nex_rec[f] = p.nex;
        }
        if (trace) {
            D->t_pred[bid] = p.pred;
            D->t_v[bid] = V;
        }
    }
}

}  // namespace
