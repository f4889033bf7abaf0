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
//   process noise of slot j (proportional to sqrt q).
#pragma once

#include "arna_kernels.hpp"

namespace {

struct AdjArgs {
    const float *xprop;       // [5][N] propagated particles of step k
    const uint16_t *anck;     // [N] ancestors of step k (sorted within each PE)
    const float *rbar_in;     // [5][N] adjoint of the resampled slots of step k; NULL at k = K
    float *rbar_out;          // [5][N] adjoint of the resampled slots of step k - 1
    const double *lbar_in;    // [2][F M] own / received parts of Lbar at step k; NULL at k = K
    double *lbar_out;         // [2][F M] the same for step k - 1
    double *theta;            // [F M][2] accumulated dJ/dsigma, dJ/dq per PE
    float sigma;              // psf_sigma
    float inv_2q;             // 1 / (2 q)
};

template <int PPT, int HALF>
__global__ __launch_bounds__(1024) void k_adjoint(StepArgs a, AdjArgs g) {
    __shared__ Prologue pro;
    __shared__ double lbar_sh;
    __shared__ double red[kMaxWaves * 4];
    __shared__ uint16_t recv[PF_MAX_PER_PE], ancs[PF_MAX_PER_PE];
    __shared__ uint16_t rs[PF_MAX_PER_PE], re[PF_MAX_PER_PE];
    const uint32_t M = a.M, np = a.np, N = a.N;
    const uint32_t f = blockIdx.x / M, m = blockIdx.x % M;
    const uint32_t tid = threadIdx.x, B = blockDim.x;
    const uint32_t lane = tid & (kWave - 1), wave = tid / kWave;
    const uint32_t pe_base = blockIdx.x * np;
    const bool last = g.rbar_in == nullptr;

    // steps 1-4 of iteration k again (which slots were received, lambda),
    // and Lbar of this PE
    if (wave == 0) prologue_wave(a, f, m, &pro);
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
    for (uint32_t s = tid; s < np; s += B) {
        recv[s] = 0xFFFF;
        ancs[s] = g.anck[pe_base + s];
        rs[s] = 0;
        re[s] = 0;
    }
    __syncthreads();
    const Prologue p = pro;
    const double lbar = lbar_sh;
    if (p.nex) build_receive_map(recv, p, np);
    // runs of equal ancestors: particle i's offspring are slots [rs[i], re[i])
    for (uint32_t s = tid; s < np; s += B) {
        const uint32_t ai = ancs[s];
        if (s == 0 || ancs[s - 1] != ai) rs[ai] = (uint16_t)s;
        if (s == np - 1 || ancs[s + 1] != ai) re[ai] = (uint16_t)(s + 1);
    }
    __syncthreads();

    const double logw = a.rout[blockIdx.x].log_mass;
    const uint32_t pred_base = (f * M + p.pred) * np;
    double sums[4] = {0, 0, 0, 0};   // ubar own, ubar received, dJ/dsigma, dJ/dq
#pragma unroll 1
    for (int q = 0; q < PPT; ++q) {
        const uint32_t j = tid + q * B;
        if (j >= np) break;
        float x[5], xb[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < 5; ++c) x[c] = g.xprop[c * N + pe_base + j];
        float gl[4];
        const float ell = patch_loglik_grad<HALF>(x, a.lik, g.sigma, gl);
        if (!last)
            for (uint32_t t = rs[j]; t < re[j]; ++t)
#pragma unroll
                for (int c = 0; c < 5; ++c) xb[c] += g.rbar_in[c * N + pe_base + t];
        const uint32_t r = recv[j];
        const float lam = (r != 0xFFFFu) ? p.lam_pred : p.lam_own;
        const double ub =
            (logw == -INFINITY) ? 0.0 : lbar * exp((double)(lam + ell) - logw);
        const float ubf = (float)ub;
        xb[0] += ubf * gl[0];
        xb[1] += ubf * gl[1];
        xb[4] += ubf * gl[2];
        sums[(r != 0xFFFFu) ? 1 : 0] += ub;
        sums[2] += ub * (double)gl[3];
        // process noise of this slot, sqrt(q) times a fixed combination of normals
        float e[5];
        five_normals(philox(m * np + j, a.k, f, kTagProp << 24, a.key0, a.key1), e);
        const float n0 = a.dyn.a * e[0], n2 = a.dyn.b * e[0] + a.dyn.c * e[1];
        const float n1 = a.dyn.a * e[2], n3 = a.dyn.b * e[2] + a.dyn.c * e[3];
        sums[3] += (double)(g.inv_2q * (xb[0] * n0 + xb[2] * n2 + xb[1] * n1 + xb[3] * n3));
        // adjoint of the input (F^T), to the slot the input came from
        const float in[5] = {xb[0], xb[1], xb[2] + xb[0], xb[3] + xb[1], xb[4]};
        const uint32_t dst = (r != 0xFFFFu) ? pred_base + r : pe_base + j;
#pragma unroll
        for (int c = 0; c < 5; ++c) g.rbar_out[c * N + dst] = in[c];
    }
    block_sum<4>(sums, red);
    if (tid == 0) {
        g.lbar_out[blockIdx.x] = sums[0];
        g.lbar_out[(size_t)gridDim.x + f * M + p.pred] = sums[1];
        g.theta[2 * blockIdx.x] += sums[2];
        g.theta[2 * blockIdx.x + 1] += sums[3];
    }
}

// Per filter: J = sum_k (log sum_m W^(m)_k - log N_p) over the recorded
// records rec[1..K], dJ/dsigma and dJ/dq from the per-PE accumulators, and
// dJ/dI0 = sum of the intensity adjoints of the starting slots.
// out[f] = (J, dJ/dsigma, dJ/dI0, dJ/dq); with theta == NULL only J.
__global__ __launch_bounds__(256) void k_grad_reduce(const pf_pe_record *rec, uint32_t K,
                                                     const double *theta, const float *rbar0,
                                                     uint32_t M, uint32_t np, uint32_t N,
                                                     uint32_t FM, double *out) {
    __shared__ double red[kRedDoubles];
    const uint32_t f = blockIdx.x;
    double J = 0.0;
    for (uint32_t k = 1; k <= K; ++k) {
        const pf_pe_record *R = rec + (size_t)k * FM + (size_t)f * M;
        double lmax = -INFINITY;
        for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) lmax = fmax(lmax, R[i].log_mass);
        lmax = block_max_d(lmax, red);
        double acc[1] = {0.0};
        if (lmax != -INFINITY)
            for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) acc[0] += exp(R[i].log_mass - lmax);
        block_sum<1>(acc, red);
        J += (lmax == -INFINITY) ? -INFINITY : lmax + log(acc[0]) - log((double)np);
    }
    if (!theta) {
        if (threadIdx.x == 0) out[4 * f] = J;
        return;
    }
    double v[3] = {0, 0, 0};
    for (uint32_t i = threadIdx.x; i < M; i += blockDim.x) {
        v[0] += theta[2 * ((size_t)f * M + i)];
        v[2] += theta[2 * ((size_t)f * M + i) + 1];
    }
    const size_t b = (size_t)f * M * np;
    for (size_t i = threadIdx.x; i < (size_t)M * np; i += blockDim.x)
        v[1] += (double)rbar0[4 * (size_t)N + b + i];
    block_sum<3>(v, red);
    if (threadIdx.x == 0) {
        out[4 * f] = J;
        out[4 * f + 1] = v[0];
        out[4 * f + 2] = v[1];
        out[4 * f + 3] = v[2];
    }
}

}  // namespace
