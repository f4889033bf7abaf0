// The once-per-filter master record of Alg. 3 steps 9-10 (Sec. IV-C) for
// contexts with many PEs: the global log-mass log W_k = log sum_m W_k^(m)
// (the renormalization of the next iteration's step 4) and the exchange count
// of Eq. 3 for the next iteration, from PE_eff = (sum_m W^(m))^2 /
// sum_m (W^(m))^2 (Eq. 4).
//
// One workgroup of kMasterThreads threads per filter reads the M log-masses
// its filter's PEs wrote.  Thread t takes PEs t, t + kMasterThreads, ... and
// reduces them in that order, as master_block does with the same block size,
// so the record is bitwise master_block's; but the thread loads all of its
// log-masses into registers before reducing them, so that their latencies
// overlap instead of adding up over the two passes (maximum, then the sum of
// exp(L - max)), and k_step_flex writes the log-masses side by side, so that
// the read is contiguous rather than one 8-byte value per 56-byte record.
// Measured on MI355X (us per launch, one filter, after k_step_flex): two
// passes over the records by 256 threads with the loads issued as needed,
// 5.0 at 512 PEs, 7.8 at 2048, 11.8 at 4096, 19.7 at 8192; this kernel with
// 256 / 512 / 1024 threads, 5.2 / 5.3 / 6.6 at 2048 PEs, 7.8 / 6.1 / 7.7 at
// 4096, 9.9 / 8.1 / 9.3 at 8192.
#pragma once

#include "arna_kernels.hpp"

namespace {

constexpr uint32_t kMasterThreads = 512;
constexpr uint32_t kMasterPerThread = PF_MAX_PE / kMasterThreads;
static_assert(kMasterPerThread * kMasterThreads == PF_MAX_PE, "PF_MAX_PE records per workgroup");

// Master record of filter blockIdx.x from its M <= PER kMasterThreads records
// (block of kMasterThreads threads) to out (if not NULL) and, with row, the
// whole master step of the iteration (Alg. 3 steps 9-10: also x_k = sum_m
// W^(m) x^m / W_k, PE_eff, the increment of log Z, N_ex used, from nex_used)
// to row[f].  With lm (the log-masses [F M] the step wrote beside the
// records) their reads are contiguous: the same values, the same record.  PER
// only sizes the unrolled loads: every PER covering M gives the same record,
// and the record is the same with or without the row (the sums of W and of
// W x^m are reduced component by component in the same order).
template <uint32_t PER>
__global__ __launch_bounds__(kMasterThreads) void k_master(
    const pf_pe_record *rec, const double *lm, MasterRec *out, pf_master_t *row,
    const uint32_t *nex_used, uint64_t step, uint32_t M, uint32_t np, uint32_t mode,
    uint32_t fixed_nex, uint32_t cutoff_ppm) {
    __shared__ double red[kRedDoubles];
    const size_t base = (size_t)blockIdx.x * M;
    const uint32_t tid = threadIdx.x;
    double L[PER];
    if (lm) {
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j) {
            const uint32_t i = tid + j * kMasterThreads;
            L[j] = i < M ? lm[base + i] : -INFINITY;
        }
    } else {
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j) {
            const uint32_t i = tid + j * kMasterThreads;
            L[j] = i < M ? rec[base + i].log_mass : -INFINITY;
        }
    }
    double lmax = -INFINITY;
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) lmax = fmax(lmax, L[j]);
    lmax = block_max_d(lmax, red);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    uint64_t sd[2] = {0, 0};
    if (lmax != -INFINITY) {
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j) {
            if (tid + j * kMasterThreads < M) {
                const double e = exp(L[j] - lmax);
                const uint64_t P = (uint64_t)floor(e * 1048576.0);
                acc[0] += e;
                sd[0] += P;
                sd[1] += P * P;
                L[j] = e;   // (kept for the row)
            }
        }
        if (row) {   // (fully unrolled: every load in flight at once)
#pragma unroll
            for (uint32_t j = 0; j < PER; ++j) {
                const uint32_t i = tid + j * kMasterThreads;
                if (i < M && L[j] > 0.0) {
                    const double *x = rec[base + i].xhat;
#pragma unroll
                    for (int c = 0; c < 5; ++c) acc[1 + c] += L[j] * x[c];
                }
            }
        }
    }
    if (row) {
        block_sum<6>(acc, red);
    } else {
        double a1[1] = {acc[0]};
        block_sum<1>(a1, red);
        acc[0] = a1[0];
    }
    block_sum_u64(sd, (uint64_t *)red);
    if (tid == 0) {
        const uint32_t f = blockIdx.x;
        const double lglob = (lmax == -INFINITY) ? -INFINITY : lmax + log(acc[0]);
        const uint32_t nex_next =
            exchange_count(sd[0], sd[1], M, np, mode, 0, fixed_nex, 0, cutoff_ppm);
        if (out) {
            MasterRec r;
            r.lglob = lglob;
            r.nex_next = nex_next;
            r.pad = 0;
            out[f] = r;
        }
        if (row) {
            pf_master_t o;
            o.log_mass_glob = lglob;
            for (int c = 0; c < 5; ++c) o.xhat[c] = acc[1 + c] / acc[0];
            o.pe_eff = sd[1] ? (double)sd[0] * (double)sd[0] / (double)sd[1] : 0.0;
            o.log_z_inc = lglob - log((double)np);
            o.n_ex = nex_used ? nex_used[f] : 0u;
            o.n_ex_next = nex_next;
            o.step = step;
            row[f] = o;
        }
    }
}

// The master records (out, if not NULL) and master steps (row, if not NULL)
// of F filters of M PEs each on stream s: the smallest unrolling that covers
// M (a short kernel for few PEs).
inline hipError_t launch_master(hipStream_t s, uint32_t F, uint32_t M, uint32_t np,
                                uint32_t mode, uint32_t fixed_nex, uint32_t cutoff_ppm,
                                const pf_pe_record *rec, const double *lm, MasterRec *out,
                                pf_master_t *row = nullptr, const uint32_t *nex_used = nullptr,
                                uint64_t step = 0) {
    (void)hipGetLastError();   // clear errors of earlier, unrelated calls
    const dim3 grid(F), block(kMasterThreads);
    if (M <= 2 * kMasterThreads)
        hipLaunchKernelGGL(k_master<2>, grid, block, 0, s, rec, lm, out, row, nex_used, step, M,
                           np, mode, fixed_nex, cutoff_ppm);
    else if (M <= 8 * kMasterThreads)
        hipLaunchKernelGGL(k_master<8>, grid, block, 0, s, rec, lm, out, row, nex_used, step, M,
                           np, mode, fixed_nex, cutoff_ppm);
    else
        hipLaunchKernelGGL(k_master<kMasterPerThread>, grid, block, 0, s, rec, lm, out, row,
                           nex_used, step, M, np, mode, fixed_nex, cutoff_ppm);
    return hipGetLastError();
}

}  // namespace
