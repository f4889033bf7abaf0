// arna_adjoint.hpp -- the adjoint (reverse-mode) step of the ARNA filter and
// the final reduction of the gradient.  Included by arna.hip after
// arna_kernels.hpp.
//
// Objective, per filter: J = sum_k (log W_k - log N_p), the filter's estimate
// of log p(z_1..z_K) (steps 9-10 of Alg. 3, with the step-4 renormalization
// the increments chain).  Every discrete choice of the recorded run is held
// fixed -- ring, N_ex, exchanged slots, ancestors, patch origins -- and the
// normals are fixed by their Philox counters, so J is a smooth function of
// theta = (psf_sigma, I0, q); I0 shifts the intensity of every particle of
// the starting state.
//
// Reverse sweep, step k = K .. 1, one workgroup per PE p.  With u_j = lambda_j
// + l_j (step 5 U) and log W^(p)_k = log sum_j exp(u_j) (step 6):
//   ubar_j   = Lbar_p exp(u_j - log W^(p)_k),
//   Lbar_p   = exp(L_p - log W_K) at k = K, else the sum of ubar over the
//              slots of step k + 1 whose carried weight came from PE p (the
//              renormalization terms cancel: sum_p Lbar_p = 1 at every step);
//   xbar_j   = ubar_j grad_x l_j + sum of the adjoints of the resampled slots
//              whose ancestor is j (the ancestors of a PE are sorted, so these
//              are one run of slots, summed in order);
//   the adjoint of slot j's input is F^T xbar_j (NCV: position adjoint adds
//   to the velocity adjoint), written to the slot the input came from (own
//   slot, or pred's sent slot: a bijection, no conflicts);
//   dJ/dsigma += ubar_j dl_j/dsigma;  dJ/dq += xbar_j . n_j / (2 q), n_j the
//   process noise of slot j (proportional to sqrt q), read back from the tape
//   as x_j - F x_in(j).
#pragma once

#include "arna_kernels.hpp"

namespace {

struct AdjArgs {
    const float *xprop;       // [5][N] propagated particles of step k
    const float *xprev;       // [5][N] propagated particles of step k - 1 (the tape's start
                              // state at the first recorded step)
    const uint16_t *ancprev;  // [N] ancestors of step k - 1: slot s of PE p held
                              // xprev[p N_p + ancprev[p N_p + s]] after step k - 1
    const uint16_t *anck;     // [N] ancestors of step k (sorted within each PE)
    const float *rbar_in;     // [5][N] adjoint of the resampled slots of step k; NULL at k = K
    float *rbar_out;          // [5][N] adjoint of the resampled slots of step k - 1
    const double *lbar_in;    // [2][F M] own / received parts of Lbar at step k; NULL at k = K
    double *lbar_out;         // [2][F M] the same for step k - 1
    double *theta;            // [F M][3]: dJ/dsigma, dJ/dq accumulated; the intensity
                              // adjoint this PE wrote (the last sweep step leaves the start's)
    float sigma;              // psf_sigma
    float inv_2q;             // 1 / (2 q)
};

// Dynamic LDS of k_adjoint: the image tile, the adjoints of the PE's
// resampled slots, the receive map, the ancestors and the offspring runs.
__host__ __device__ constexpr size_t adjoint_lds_bytes(uint32_t np) {
    return (size_t)kTileRows * kTilePitch * sizeof(float) + 5 * (size_t)np * sizeof(float) +
           ((size_t)4 * np * sizeof(uint16_t) + 15) / 16 * 16;
}

template <int PPT, int HALF>
__global__ __launch_bounds__(1024) void k_adjoint(StepArgs a, AdjArgs g) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ Prologue pro;
    __shared__ double lbar_sh;
    __shared__ double red[kMaxWaves * 5];
    constexpr int P = 2 * HALF + 1;
    const uint32_t M = a.M, np = a.np, N = a.N;
    const uint32_t f = blockIdx.x / M, m = blockIdx.x % M;
    const uint32_t tid = threadIdx.x, B = blockDim.x;
    const uint32_t lane = tid & (kWave - 1), wave = tid / kWave;
    const uint32_t pe_base = blockIdx.x * np;
    const bool last = g.rbar_in == nullptr;
    float *tile = (float *)smem;
    float *rb = tile + kTileRows * kTilePitch;   // [5][np]
    uint16_t *recv = (uint16_t *)(rb + 5 * (size_t)np);
    uint16_t *ancs = recv + np, *rs = ancs + np, *re = rs + np;

    // ---- phase 0: steps 1-4 of iteration k again (which slots were
    // received, lambda) on wave 0, Lbar of this PE on the next wave; every
    // thread stages the ancestors, the adjoints of its resampled slots and its
    // part of the image tile, centred on this PE's estimate of step k (the
    // mean of its propagated particles).
    if (wave == 0) prologue_wave(a, f, m, &pro, threadIdx.x);
    if (wave == (B > kWave ? 1u : 0u)) {
        if (last) {
            // exp(L_p - log sum_m exp(L_m)) over the records of step k
            const pf_pe_record *R = a.rout + (size_t)f * M;
            double lmax = -INFINITY;
            for (uint32_t i = lane; i < M; i += kWave) lmax = fmax(lmax, R[i].log_mass);
            lmax = wave_max_d(lmax);
            double acc = 0.0;
            if (lmax != -INFINITY)
                for (uint32_t i = lane; i < M; i += kWave) acc += exp(R[i].log_mass - lmax);
            acc = wave_sum(acc);
            if (lane == 0) {
                const double lp = R[m].log_mass;
                lbar_sh = (lmax == -INFINITY || lp == -INFINITY) ? 0.0 : exp(lp - lmax) / acc;
            }
        } else if (lane == 0) {
            lbar_sh = g.lbar_in[blockIdx.x] + g.lbar_in[(size_t)gridDim.x + blockIdx.x];
        }
    }
    int tx0 = 0, ty0 = 0;
    bool tile_on = false;
    {
        const double *xh = a.rout[blockIdx.x].xhat;
        if (B >= 1024 && fabs(xh[0]) < 1e6 && fabs(xh[1]) < 1e6) {   // false for NaN
            tx0 = (int)floor(xh[0] + 0.5) - kTileCols / 2;
            ty0 = (int)floor(xh[1] + 0.5) - kTileRows / 2;
            tile_on = tx0 < a.lik.W && tx0 + kTileCols > 0 && ty0 < a.lik.H && ty0 + kTileRows > 0;
        }
    }
    constexpr int kTileRegs = (kTileRows * kTileCols) / 1024;
    float tv[kTileRegs];
#pragma unroll
    for (int i = 0; i < kTileRegs; ++i) {
        const uint32_t idx = tid + (uint32_t)i * B;
        const int u = tx0 + (int)(idx % kTileCols), v = ty0 + (int)(idx / kTileCols);
        const bool in = tile_on && (unsigned)u < (unsigned)a.lik.W && (unsigned)v < (unsigned)a.lik.H;
        tv[i] = in ? a.lik.img[(size_t)v * a.lik.W + u] - a.lik.bg : 0.f;
    }
    for (uint32_t s = tid; s < np; s += B) {
        recv[s] = 0xFFFF;
        ancs[s] = g.anck[pe_base + s];
        rs[s] = 0;
        re[s] = 0;
    }
    if (!last)
        for (uint32_t s = tid; s < np; s += B)
#pragma unroll
            for (int c = 0; c < 5; ++c) rb[c * np + s] = g.rbar_in[c * N + pe_base + s];
    if (tile_on) {
#pragma unroll
        for (int i = 0; i < kTileRegs; ++i) {
            const uint32_t idx = tid + (uint32_t)i * B;
            tile[(idx / kTileCols) * kTilePitch + idx % kTileCols] = tv[i];
        }
        for (uint32_t idx = tid + kTileRegs * B; idx < (uint32_t)(kTileRows * kTileCols); idx += B) {
            const int u = tx0 + (int)(idx % kTileCols), v = ty0 + (int)(idx / kTileCols);
            const bool in = (unsigned)u < (unsigned)a.lik.W && (unsigned)v < (unsigned)a.lik.H;
            tile[(idx / kTileCols) * kTilePitch + idx % kTileCols] =
                in ? a.lik.img[(size_t)v * a.lik.W + u] - a.lik.bg : 0.f;
        }
    }
    __syncthreads();
    const Prologue p = pro;
    const float lbar = (float)lbar_sh;
    if (p.nex) build_receive_map(recv, p, np, threadIdx.x);
    // runs of equal ancestors: particle i's offspring are slots [rs[i], re[i])
    for (uint32_t s = tid; s < np; s += B) {
        const uint32_t ai = ancs[s];
        if (s == 0 || ancs[s - 1] != ai) rs[ai] = (uint16_t)s;
        if (s == np - 1 || ancs[s + 1] != ai) re[ai] = (uint16_t)(s + 1);
    }
    __syncthreads();

    // ---- phase 1: one propagated particle at a time
    const float logw = (float)a.rout[blockIdx.x].log_mass;
    const uint32_t pred_base = (f * M + p.pred) * np;
    double sums[5] = {0, 0, 0, 0, 0};   // ubar own, ubar received, dJ/dsigma, dJ/dq, Ibar
#pragma unroll 1
    for (int q = 0; q < PPT; ++q) {
        const uint32_t j = tid + q * B;
        if (j >= np) break;
        float x[5], xb[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < 5; ++c) x[c] = g.xprop[c * N + pe_base + j];
        // the input of slot j (own slot, or pred's sent slot): its process
        // noise is n = x - F x_in; loaded now, used after the likelihood
        const uint32_t r = recv[j];
        const uint32_t src_base = (r != 0xFFFFu) ? pred_base : pe_base;
        const uint32_t src = src_base + g.ancprev[src_base + ((r != 0xFFFFu) ? r : j)];
        float xin[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) xin[c] = g.xprev[c * N + src];
        float gl[4] = {0, 0, 0, 0}, ell = 0.f;
        int u0, v0;
        if (patch_origin<HALF>(x[0], x[1], a.lik.W, a.lik.H, u0, v0)) {
            const int du = u0 - tx0, dv = v0 - ty0;
            if (tile_on && (unsigned)du <= (unsigned)(kTileCols - P) &&
                (unsigned)dv <= (unsigned)(kTileRows - P))
                ell = patch_loglik_grad<HALF, true>(x, u0, v0, tile + dv * kTilePitch + du,
                                                    kTilePitch, a.lik, g.sigma, gl);
            else
                ell = patch_loglik_grad<HALF, false>(x, u0, v0, nullptr, 0, a.lik, g.sigma, gl);
        }
        if (!last)   // the adjoints of this particle's offspring (none after the last step)
            for (uint32_t t = rs[j]; t < re[j]; ++t)
#pragma unroll
                for (int c = 0; c < 5; ++c) xb[c] += rb[c * np + t];
        const float lam = (r != 0xFFFFu) ? p.lam_pred : p.lam_own;
        const float ub = (logw == -INFINITY) ? 0.f : lbar * __expf((lam + ell) - logw);
        xb[0] += ub * gl[0];
        xb[1] += ub * gl[1];
        xb[4] += ub * gl[2];
        sums[(r != 0xFFFFu) ? 1 : 0] += (double)ub;
        sums[2] += (double)(ub * gl[3]);
        // process noise of this slot (proportional to sqrt q): x - F x_in
        const float n0 = x[0] - (xin[0] + xin[2]), n2 = x[2] - xin[2];
        const float n1 = x[1] - (xin[1] + xin[3]), n3 = x[3] - xin[3];
        sums[3] += (double)(g.inv_2q * (xb[0] * n0 + xb[2] * n2 + xb[1] * n1 + xb[3] * n3));
        sums[4] += (double)xb[4];
        // adjoint of the input (F^T), to the slot the input came from
        const float in[5] = {xb[0], xb[1], xb[2] + xb[0], xb[3] + xb[1], xb[4]};
        const uint32_t dst = (r != 0xFFFFu) ? pred_base + r : pe_base + j;
#pragma unroll
        for (int c = 0; c < 5; ++c) g.rbar_out[c * N + dst] = in[c];
    }
    block_sum<5>(sums, red);
    if (tid == 0) {
        g.lbar_out[blockIdx.x] = sums[0];
        g.lbar_out[(size_t)gridDim.x + f * M + p.pred] = sums[1];
        g.theta[3 * blockIdx.x] += sums[2];
        g.theta[3 * blockIdx.x + 1] += sums[3];
        g.theta[3 * blockIdx.x + 2] = sums[4];
    }
}

// Per filter: J = sum_k (log sum_m W^(m)_k - log N_p) over the recorded
// records rec[1..K], and the sums over the PEs of the per-PE gradient parts.
// out[f] = (J, dJ/dsigma, dJ/dI0, dJ/dq); with theta == NULL only J.  One
// workgroup of kGradReduceThreads per filter: each wave takes one iteration at
// a time, its lanes the M records (wave reductions, no barrier per
// iteration).
constexpr uint32_t kGradReduceThreads = 1024;
__global__ __launch_bounds__(kGradReduceThreads) void k_grad_reduce(
    const pf_pe_record *rec, uint32_t K, const double *theta, uint32_t M, uint32_t np, uint32_t FM,
    double *out) {
    __shared__ double red[kMaxWaves * 4];
    const uint32_t f = blockIdx.x;
    const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const uint32_t nwaves = blockDim.x / kWave;
    double v[4] = {0, 0, 0, 0};
    for (uint32_t k = 1 + wave; k <= K; k += nwaves) {
        const pf_pe_record *R = rec + (size_t)k * FM + (size_t)f * M;
        double lmax = -INFINITY;
        for (uint32_t i = lane; i < M; i += kWave) lmax = fmax(lmax, R[i].log_mass);
        lmax = wave_max_d(lmax);
        double acc = 0.0;
        if (lmax != -INFINITY)
            for (uint32_t i = lane; i < M; i += kWave) acc += exp(R[i].log_mass - lmax);
        acc = wave_sum(acc);
        if (lane == 0)
            v[0] += (lmax == -INFINITY) ? -INFINITY : lmax + log(acc) - log((double)np);
    }
    if (theta)
        for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) {
            const double *t = theta + 3 * ((size_t)f * M + i);
            v[1] += t[0];
            v[2] += t[2];
            v[3] += t[1];
        }
    block_sum<4>(v, red);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) out[4 * f + c] = (c == 0 || theta) ? v[c] : 0.0;
}

}  // namespace
