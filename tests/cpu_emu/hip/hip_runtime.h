// The HIP surface the library's sources use, declared for the CPU emulation
// in emu_rt.cpp (test infrastructure): kernels compile as plain C++ functions
// that every fiber of a workgroup runs; thread and block indices, barriers,
// wave operations, atomics and the runtime calls go to the emulation.
#pragma once
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <math.h>
#include <stdlib.h>
#include <stdio.h>
#include <tuple>
#include <utility>
#include <type_traits>
#include <functional>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static thread_local
#define __align__(n) __attribute__((aligned(n)))

struct dim3 {
    uint32_t x, y, z;
    dim3(uint32_t a = 1, uint32_t b = 1, uint32_t c = 1) : x(a), y(b), z(c) {}
};
struct float2 { float x, y; };
struct float4 { float x, y, z, w; };
static inline float2 make_float2(float a, float b) { return {a, b}; }
static inline float4 make_float4(float a, float b, float c, float d) { return {a, b, c, d}; }

// ---- thread identity of the running fiber
struct EmuIds { dim3 tid, bid, bdim, gdim; uint32_t lane, wave; };
EmuIds &emu_ids();
#define threadIdx (emu_ids().tid)
#define blockIdx (emu_ids().bid)
#define blockDim (emu_ids().bdim)
#define gridDim (emu_ids().gdim)
unsigned char *emu_smem();

// ---- synchronization and wave operations
void emu_syncthreads();
#define __syncthreads() emu_syncthreads()
enum EmuOp { EMU_SHFL = 1, EMU_XOR, EMU_READLANE, EMU_FIRST, EMU_DPP, EMU_ANY };
uint64_t emu_wave_op(int op, uint64_t v, uint64_t par);
template <class T> static inline uint64_t emu_bits(T v) { uint64_t b = 0; memcpy(&b, &v, sizeof(T)); return b; }
template <class T> static inline T emu_from(uint64_t b) { T v; memcpy(&v, &b, sizeof(T)); return v; }
template <class T> static inline T __shfl(T v, int src, int w = 64) { return emu_from<T>(emu_wave_op(EMU_SHFL, emu_bits(v), (uint64_t)(uint32_t)src)); }
template <class T> static inline T __shfl_xor(T v, int m, int w = 64) { return emu_from<T>(emu_wave_op(EMU_XOR, emu_bits(v), (uint64_t)(uint32_t)m)); }
// the sources read the first lane only of values that are the same in every lane
static inline int __builtin_amdgcn_readfirstlane(int v) { return v; }
static inline int __builtin_amdgcn_readlane(int v, int l) { return emu_from<int>(emu_wave_op(EMU_READLANE, emu_bits(v), (uint64_t)(uint32_t)l)); }
static inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int rmask, int bmask, bool bc) {
    uint64_t par = (uint64_t)(uint32_t)old | ((uint64_t)(ctrl & 0xFFF) << 32) | ((uint64_t)(rmask & 0xF) << 44) | ((uint64_t)(bmask & 0xF) << 48) | ((uint64_t)bc << 52);
    return emu_from<int>(emu_wave_op(EMU_DPP, emu_bits(src), par));
}
static inline int __any(int p) { return (int)emu_wave_op(EMU_ANY, p ? 1 : 0, 0); }
static inline uint32_t __builtin_amdgcn_mbcnt_lo(uint32_t m, uint32_t a) { uint32_t l = emu_ids().lane; return a + __builtin_popcount(l >= 32 ? m : (m & ((1u << l) - 1u))); }
static inline uint32_t __builtin_amdgcn_mbcnt_hi(uint32_t m, uint32_t a) { uint32_t l = emu_ids().lane; return a + (l <= 32 ? 0 : __builtin_popcount(m & ((1u << (l - 32)) - 1u))); }
void emu_global_load_lds(const void *g, void *lds, int size);
#define __builtin_amdgcn_global_load_lds(g, l, sz, o, a) emu_global_load_lds((const void *)(g), (void *)(l), sz)
#define __builtin_amdgcn_s_waitcnt(x) ((void)0)
#define __builtin_amdgcn_s_sleep(x) ((void)0)
#define __builtin_amdgcn_fence(o, s) __atomic_thread_fence(__ATOMIC_SEQ_CST)
template <class T> static inline void emu_opaque(T &) {}

// ---- atomics
#define __HIP_MEMORY_SCOPE_AGENT 3
#define __HIP_MEMORY_SCOPE_WORKGROUP 2
#define __HIP_MEMORY_SCOPE_SYSTEM 4
template <class T, class U> static inline T __hip_atomic_fetch_add(T *p, U v, int, int) { return __atomic_fetch_add(p, (T)v, __ATOMIC_SEQ_CST); }
template <class T> static inline T __hip_atomic_load(T *p, int, int) { return __atomic_load_n(p, __ATOMIC_SEQ_CST); }
template <class T, class U> static inline void __hip_atomic_store(T *p, U v, int, int) { __atomic_store_n(p, (T)v, __ATOMIC_SEQ_CST); }
template <class T, class U> static inline T atomicOr(T *p, U v) { return __atomic_fetch_or(p, (T)v, __ATOMIC_SEQ_CST); }
template <class T, class U> static inline T atomicAdd(T *p, U v) { return __atomic_fetch_add(p, (T)v, __ATOMIC_SEQ_CST); }
template <class T, class U> static inline T atomicMax(T *p, U v) {
    T o = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (o < (T)v && !__atomic_compare_exchange_n(p, &o, (T)v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {}
    return o;
}
uint64_t wall_clock64();

// ---- math
static inline uint64_t __umul64hi(uint64_t a, uint64_t b) { return (uint64_t)(((unsigned __int128)a * b) >> 64); }
static inline uint32_t __umulhi(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }
static inline float __builtin_amdgcn_logf(float x) { return log2f(x); }
static inline float __builtin_amdgcn_sqrtf(float x) { return sqrtf(x); }
static inline float __builtin_amdgcn_sinf(float x) { return sinf(6.283185307179586f * x); }
static inline float __builtin_amdgcn_cosf(float x) { return cosf(6.283185307179586f * x); }
static inline int __clz(int x) { return x == 0 ? 32 : __builtin_clz((unsigned)x); }
static inline float __int_as_float(int x) { return emu_from<float>((uint64_t)(uint32_t)x); }
static inline int __float_as_int(float x) { return (int)(uint32_t)emu_bits(x); }
static inline float __uint_as_float(uint32_t x) { return emu_from<float>((uint64_t)x); }
static inline uint32_t __float_as_uint(float x) { return (uint32_t)emu_bits(x); }
static inline int min(int a, int b) { return a < b ? a : b; }
static inline int max(int a, int b) { return a > b ? a : b; }
static inline uint32_t min(uint32_t a, uint32_t b) { return a < b ? a : b; }
static inline uint32_t max(uint32_t a, uint32_t b) { return a > b ? a : b; }

// ---- runtime API
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2, hipErrorLaunchFailure = 719, hipErrorNotSupported = 801 };
typedef struct EmuStream *hipStream_t;
typedef struct EmuEvent *hipEvent_t;
typedef struct EmuGraph *hipGraph_t;
typedef struct EmuGraphExec *hipGraphExec_t;
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyDefault };
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2 };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed };
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };
enum hipDeviceAttribute_t { hipDeviceAttributeCooperativeLaunch, hipDeviceAttributeMultiprocessorCount, hipDeviceAttributeWallClockRate };
struct hipFuncAttributes { size_t localSizeBytes, sharedSizeBytes; int maxThreadsPerBlock, numRegs; };

hipError_t hipMalloc(void **p, size_t n);
template <class T> static inline hipError_t hipMalloc(T **p, size_t n) { return hipMalloc((void **)p, n); }
hipError_t hipFree(void *p);
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t st = nullptr);
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t st = nullptr);
hipError_t hipMemset(void *d, int v, size_t n);
hipError_t hipGetLastError();
hipError_t hipPeekAtLastError();
hipError_t hipDeviceSynchronize();
hipError_t hipStreamSynchronize(hipStream_t);
hipError_t hipStreamCreateWithFlags(hipStream_t *, unsigned);
hipError_t hipStreamDestroy(hipStream_t);
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned);
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode);
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *);
hipError_t hipGraphInstantiate(hipGraphExec_t *, hipGraph_t, void *, char *, size_t);
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t);
hipError_t hipGraphExecDestroy(hipGraphExec_t);
hipError_t hipGraphDestroy(hipGraph_t);
hipError_t hipEventCreate(hipEvent_t *);
hipError_t hipEventCreateWithFlags(hipEvent_t *, unsigned);
hipError_t hipEventDestroy(hipEvent_t);
hipError_t hipEventRecord(hipEvent_t, hipStream_t = nullptr);
hipError_t hipEventSynchronize(hipEvent_t);
hipError_t hipEventElapsedTime(float *, hipEvent_t, hipEvent_t);
hipError_t hipFuncSetAttribute(const void *f, hipFuncAttribute a, int v);
hipError_t hipFuncGetAttributes(hipFuncAttributes *a, const void *f);
hipError_t hipGetDevice(int *d);
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int d);
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *n, const void *f, int b, size_t lds);
hipError_t hipLaunchKernel(const void *f, dim3 g, dim3 b, void **args, size_t lds, hipStream_t s);
hipError_t hipLaunchCooperativeKernel(const void *f, dim3 g, dim3 b, void **args, unsigned lds, hipStream_t s);
hipError_t hipGetSymbolAddress(void **p, const void *sym);
#define HIP_SYMBOL(x) ((const void *)&(x))
template <class T> static inline hipError_t hipFuncSetAttribute(T *f, hipFuncAttribute a, int v) { return hipFuncSetAttribute((const void *)f, a, v); }

// grid execution: body() runs once per thread of every block.  While a
// stream capture is open every launch is recorded (with copies of its
// arguments) instead, and a graph launch runs the recorded launches in order.
hipError_t emu_run_grid(const void *fn, dim3 g, dim3 b, size_t lds, const std::function<void()> &body);
hipError_t emu_launch(const void *fn, dim3 g, dim3 b, size_t lds, std::function<void()> body);
// binds copies of a launch's arguments (given as hipLaunchKernel's void **)
typedef std::function<std::function<void()>(void **)> EmuBinder;
void emu_register_binder(const void *fn, EmuBinder bind);
template <class... P, size_t... I>
static inline std::function<void()> emu_bind(void (*k)(P...), void **a, std::index_sequence<I...>) {
    std::tuple<std::remove_cv_t<std::remove_reference_t<P>>...> t(
        *(std::remove_cv_t<std::remove_reference_t<P>> *)a[I]...);
    return [k, t]() { std::apply(k, t); };
}
template <class... P> static inline void emu_register(void (*k)(P...)) {
    emu_register_binder((const void *)k, [k](void **a) { return emu_bind(k, a, std::index_sequence_for<P...>{}); });
}
template <class... P, class... A>
static inline hipError_t emu_launch_ggl(void (*k)(P...), dim3 g, dim3 b, size_t lds, hipStream_t, A... a) {
    std::tuple<std::remove_cv_t<std::remove_reference_t<P>>...> t(a...);
    return emu_launch((const void *)k, g, b, lds, [k, t]() { std::apply(k, t); });
}
#define hipLaunchKernelGGL(k, g, b, lds, s, ...) emu_launch_ggl(k, dim3(g), dim3(b), lds, s, ##__VA_ARGS__)
template <class... P> static inline void *emu_reg_ret(void (*k)(P...)) { emu_register(k); return (void *)k; }
// a wave-level barrier: every live lane of the wave meets here
static inline void __builtin_amdgcn_wave_barrier() { (void)emu_wave_op(EMU_ANY, 0, 0); }
static inline void __threadfence() { __atomic_thread_fence(__ATOMIC_SEQ_CST); }
template <class T, class U> static inline T atomicExch(T *p, U v) { return __atomic_exchange_n(p, (T)v, __ATOMIC_SEQ_CST); }
