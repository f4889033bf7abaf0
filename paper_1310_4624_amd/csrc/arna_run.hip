// arna_run.hip -- the multi-iteration launch of the ARNA step (k_run): every
// workgroup stays on its PE for up to 64 iterations, keeping its resampled
// particles in registers, and the PEs of a filter meet at a barrier between
// iterations.  Compiled on its own (with machine-level loop-invariant code
// motion off: hoisting constants out of the iteration loop would hold them in
// registers across the whole loop and spill) and linked into libarna.so.
#include "arna_kernels.hpp"

namespace {

// A StepArgs in the constant address space (the host pass, which only parses
// the kernel, sees a plain pointer: it has no such address space).
#if defined(__HIP_DEVICE_COMPILE__)
typedef const StepArgs __attribute__((address_space(4))) *ConstArgs;
#else
typedef const StepArgs *ConstArgs;
#endif

// Barrier of the M workgroups of one filter.  Every wave waits until its
// memory operations are complete (its stores have reached this die's L2);
// then one thread makes them visible device-wide with an agent-scope release
// (one write-back of the L2 per workgroup rather than one per wave), counts
// the workgroup in, waits for `target` arrivals and makes the other
// workgroups' stores visible here (agent-scope acquire).  Returns false after
// a wait longer than `timeout` (flag: one LDS word).
__device__ __forceinline__ bool filter_barrier(unsigned long long *cnt, unsigned long long target,
                                               unsigned long long timeout, uint32_t *err,
                                               uint32_t *flag, const uint32_t tid) {
    __builtin_amdgcn_s_waitcnt(0);   // all counters zero: this wave's loads and stores done
    __syncthreads();
    if (tid == 0) {
        __hip_atomic_fetch_add(cnt, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long t0 = wall_clock64();
        uint32_t ok = 1u;
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (wall_clock64() - t0 > timeout) {
                ok = 0u;
                atomicOr(err, kErrBarrier);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *flag = ok;
    }
    __syncthreads();
    return *flag != 0u;
}

template <int PPT, int HALF, int LIK>
__global__ __launch_bounds__(1024) void k_run(RunArgs r) {
    extern __shared__ __align__(16) unsigned char smem[];
    // The kernel arguments, the iteration's arguments and the block and wave
    // index pass through empty asm statements every iteration: opaque to the
    // compiler, so nothing is hoisted out of the loop (e.g. the first Philox
    // products of a slot) and held, spilled, in registers for its whole
    // length; everything is read again with scalar loads (constant address
    // space: nothing in the launch writes these arguments).  The thread index
    // is the wave's index, uniform, plus the lane (blockDim.x is a multiple
    // of 64), so it need not stay live in a vector register either.
    typedef const RunArgs __attribute__((address_space(4))) *KernArgs;
    const uint32_t bid = blockIdx.x;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    float xr[PPT][5];
    for (uint32_t i = 0;; ++i) {
        KernArgs kp = (KernArgs)__builtin_amdgcn_kernarg_segment_ptr();
        uint32_t b = bid, w = wv;
        __asm__ volatile("" : "+s"(kp), "+s"(b), "+s"(w));
        ConstArgs ap = (ConstArgs)(uintptr_t)(kp->args + i);
        uint32_t t = w * kWave + __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
        __asm__ volatile("" : "+v"(t));   // else t & 63 folds back to the hoisted lane id
        StepArgs a = *ap;
        // never set for a multi-iteration launch (the host checks); known
        // null here, the code paths they guard drop out
        a.dbg = nullptr;
        a.nex_rec = nullptr;
        a.force_nex = nullptr;
        a.force_anc = nullptr;
        a.min = nullptr;
        a.mout = nullptr;
        a.arrive = nullptr;
        a.traj_prev = nullptr;
        a.lin_in = 0u;
        step_body<PPT, HALF, LIK, true>(a, b, xr, i > 0, t);
        if (i + 1 >= kp->n ||
            !filter_barrier(kp->bar + b / a.M, (unsigned long long)(i + 1) * a.M, kp->timeout,
                            a.err, (uint32_t *)carve(smem, a.np).wmax, t))
            return;
    }
}

template <int PPT, int HALF, int LIK>
void *run_kernel() {
    return reinterpret_cast<void *>(&k_run<PPT, HALF, LIK>);
}

template <int HALF, int LIK>
void *run_kernel_ppt(uint32_t ppt) {
    return ppt == 1 ? run_kernel<1, HALF, LIK>()
                    : (ppt == 2 ? run_kernel<2, HALF, LIK>() : run_kernel<4, HALF, LIK>());
}

}  // namespace

// Variants for the paper's 9 x 9 patch (Gaussian or Poisson pixel noise) and
// for point observations.
void *arna_run_kernel(uint32_t ppt, uint32_t half, uint32_t lik_mode) {
    if (lik_mode == PF_LIK_POINT) return run_kernel_ppt<0, kLikPoint>(ppt);
    if (half != 4) return nullptr;
    if (lik_mode == PF_LIK_POISSON) return run_kernel_ppt<4, kLikPoisson>(ppt);
    return run_kernel_ppt<4, kLikGauss>(ppt);
}
