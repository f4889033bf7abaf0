// The once-per-filter master record of Alg. 3 steps 9-10 (Sec. IV-C) for
// contexts with many PEs: the global log-mass log W_k = log sum_m W_k^(m)
// (the normalizer of the next iteration's lambda, Eq. 3) and the exchange
// count that PE_eff = (sum_m W^(m))^2 / sum_m (W^(m))^2 (Eq. 4) gives for the
// next iteration.
//
// One workgroup of kMasterThreads threads per filter reads the M records its
// filter's PEs wrote.  Thread t takes records t, t + kMasterThreads, ... and
// reduces them in that order, as master_block does with the same block size,
// so the record is bitwise master_block's; but the thread loads all of its
// log-masses (at most PF_MAX_PE / kMasterThreads) into registers before
// reducing them, so that their latencies overlap instead of adding up over
// the two passes (maximum, then the sum of exp(L - max)).  Measured on
// MI355X (us per launch, one filter, loads issued as they are needed / all
// first): 512 PEs 5.0 / 5.5, 2048 7.8 / 6.3, 4096 11.8 / 8.2, 8192 19.7 /
// 12.2.  What remains at many PEs is the read of the log-masses, one per
// 56-byte record, by a single compute unit (1024 threads instead of 256:
// 12.0 us at 8192 PEs, and slower below).
#pragma once

#include "arna_kernels.hpp"

namespace {

constexpr uint32_t kMasterThreads = 256;
constexpr uint32_t kMasterPerThread = PF_MAX_PE / kMasterThreads;
static_assert(kMasterPerThread * kMasterThreads == PF_MAX_PE, "PF_MAX_PE records per workgroup");

// Master record of filter blockIdx.x from its M <= PF_MAX_PE records (block
// of kMasterThreads threads).
__global__ __launch_bounds__(kMasterThreads) void k_master(const pf_pe_record *rec,
                                                           MasterRec *out, uint32_t M,
                                                           uint32_t np, uint32_t mode,
                                                           uint32_t fixed_nex,
                                                           uint32_t cutoff_ppm) {
    __shared__ double red[kRedDoubles];
    const pf_pe_record *R = rec + (size_t)blockIdx.x * M;
    const uint32_t tid = threadIdx.x;
    double L[kMasterPerThread];
#pragma unroll
    for (uint32_t j = 0; j < kMasterPerThread; ++j) {
        const uint32_t i = tid + j * kMasterThreads;
        L[j] = i < M ? R[i].log_mass : -INFINITY;
    }
    double lmax = -INFINITY;
#pragma unroll
    for (uint32_t j = 0; j < kMasterPerThread; ++j) lmax = fmax(lmax, L[j]);
    lmax = block_max_d(lmax, red);
    double acc[1] = {0.0};
    uint64_t sd[2] = {0, 0};
    if (lmax != -INFINITY) {
#pragma unroll
        for (uint32_t j = 0; j < kMasterPerThread; ++j) {
            if (tid + j * kMasterThreads < M) {
                const double e = exp(L[j] - lmax);
                const uint64_t P = (uint64_t)floor(e * 1048576.0);
                acc[0] += e;
                sd[0] += P;
                sd[1] += P * P;
            }
        }
    }
    block_sum<1>(acc, red);
    block_sum_u64(sd, (uint64_t *)red);
    if (tid == 0) {
        MasterRec r;
        r.lglob = (lmax == -INFINITY) ? -INFINITY : lmax + log(acc[0]);
        r.nex_next = exchange_count(sd[0], sd[1], M, np, mode, 0, fixed_nex, 0, cutoff_ppm);
        r.pad = 0;
        out[blockIdx.x] = r;
    }
}

}  // namespace
