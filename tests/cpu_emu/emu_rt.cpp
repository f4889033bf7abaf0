// CPU emulation of the HIP execution model, for sanitizer runs of the
// library's host code and kernels (test infrastructure, never a product
// path).  Each workgroup runs on one OS thread, its threads as fibers with
// their own stacks; __syncthreads and the wave operations (shuffles, DPP,
// __any, the wave barrier) are scheduling points where the fibers meet.  A
// wave operation completes when every live lane of the wave has reached one;
// lanes that stopped at a different point are reported as a deadlock, which
// is how a wave operation under divergent control flow shows up.  Device
// memory and the LDS block of every workgroup are heap blocks filled with a
// garbage byte, so AddressSanitizer sees every access out of bounds.  Launches
// run to completion when they are enqueued; streams, events and graphs only
// keep the API's shape.
#include "hip/hip_runtime.h"
#include <sys/mman.h>
#include <atomic>
#include <map>
#include <mutex>
#include <thread>
#include <vector>
#include <chrono>
#include <random>
#include <string>
#if defined(__SANITIZE_ADDRESS__)
#include <sanitizer/asan_interface.h>
#include <sanitizer/common_interface_defs.h>
#define EMU_ASAN 1
#else
#define EMU_ASAN 0
#endif

extern "C" void emu_switch(void **save_sp, void *new_sp);
asm(R"(
.text
.globl emu_switch
.type emu_switch,@function
emu_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
.size emu_switch, .-emu_switch
)");

namespace {
constexpr size_t kStack = 512 * 1024;
enum { RUN = 0, WBLOCK = 1, WWAVE = 2, DONE = 3 };
struct Fiber {
    void *sp = nullptr;
    char *stack = nullptr;
    int state = RUN;
    void *fake = nullptr;
    EmuIds ids;
};
struct Wave {
    uint64_t val[64], par[64], res[64];
    void *site[64];
    int op[64];
    int arrived = 0, live = 0;
};
struct Worker {
    std::vector<Fiber> f;
    void *sched_sp = nullptr;
    void *sched_fake = nullptr;
    const void *sched_bottom = nullptr;
    size_t sched_size = 0;
    Wave waves[16];
    uint32_t B = 0, live = 0, block_arrived = 0;
    unsigned char *lds = nullptr;
    const std::function<void()> *body = nullptr;
    Fiber *cur = nullptr;
    EmuIds sched_ids;
};
thread_local Worker *tw = nullptr;
std::mutex g_mu;
std::map<const void *, EmuBinder> &reg() { static std::map<const void *, EmuBinder> r; return r; }
struct Recorded {
    const void *fn;
    dim3 g, b;
    size_t lds;
    std::function<void()> body;
};
bool g_capturing = false;
std::vector<Recorded> g_record;
std::map<const void *, int> &attr() { static std::map<const void *, int> a; return a; }
thread_local hipError_t last_err = hipSuccess;
std::vector<Worker *> g_workers;
int g_fill = 0xFF;   // garbage byte for fresh device memory and LDS

void yield_to_sched() {
    Worker *w = tw;
    Fiber *f = w->cur;
#if EMU_ASAN
    __sanitizer_start_switch_fiber(&f->fake, w->sched_bottom, w->sched_size);
#endif
    emu_switch(&f->sp, w->sched_sp);
#if EMU_ASAN
    __sanitizer_finish_switch_fiber(f->fake, &w->sched_bottom, &w->sched_size);
#endif
}

void fiber_main() {
    Worker *w = tw;
    Fiber *f = w->cur;
#if EMU_ASAN
    __sanitizer_finish_switch_fiber(nullptr, &w->sched_bottom, &w->sched_size);
#endif
    (*w->body)();
    f->state = DONE;
    w->live--;
    w->waves[f->ids.wave].live--;
#if EMU_ASAN
    __sanitizer_start_switch_fiber(nullptr, w->sched_bottom, w->sched_size);
#endif
    void *dummy;
    emu_switch(&dummy, w->sched_sp);
    abort();
}

void compute_wave(Wave &wv, Worker *w, uint32_t wi) {
    // lanes of this wave that are alive and waiting
    int op = 0;
    uint32_t base = wi * 64;
    bool waiting[64] = {};
    int first = -1;
    for (uint32_t l = 0; l < 64 && base + l < w->B; ++l) {
        Fiber &f = w->f[base + l];
        if (f.state == WWAVE) {
            waiting[l] = true;
            if (first < 0) first = (int)l;
            if (op && wv.op[l] != op) {
                fprintf(stderr, "EMU: wave %u mixes wave ops %d and %d\n", wi, op, wv.op[l]);
                abort();
            }
            op = wv.op[l];
        }
    }
    for (uint32_t l = 0; l < 64; ++l) {
        if (!waiting[l]) continue;
        const uint64_t p = wv.par[l];
        uint64_t r = 0;
        switch (op) {
            case EMU_SHFL: {
                uint32_t s = (uint32_t)p & 63u;
                r = wv.val[s];
                if (!waiting[s]) r = 0xDEADBEEFDEADBEEFull;
                break;
            }
            case EMU_XOR: {
                uint32_t s = (l ^ (uint32_t)p) & 63u;
                r = waiting[s] ? wv.val[s] : 0xDEADBEEFDEADBEEFull;
                break;
            }
            case EMU_READLANE: {
                uint32_t s = (uint32_t)p & 63u;
                r = waiting[s] ? wv.val[s] : 0xDEADBEEFDEADBEEFull;
                break;
            }
            case EMU_FIRST: r = wv.val[first]; break;
            case EMU_ANY: {
                r = 0;
                for (uint32_t s = 0; s < 64; ++s)
                    if (waiting[s] && wv.val[s]) r = 1;
                break;
            }
            case EMU_DPP: {
                const uint32_t old = (uint32_t)p;
                const int ctrl = (int)((p >> 32) & 0xFFF), rmask = (int)((p >> 44) & 0xF);
                const uint32_t row = l / 16;
                int src = -1;
                if (ctrl >= 0x111 && ctrl <= 0x11F) {
                    const int n = ctrl - 0x110;
                    if ((int)(l % 16) >= n) src = (int)l - n;
                } else if (ctrl == 0x138) {   // wave_shr:1
                    if (l >= 1) src = (int)l - 1;
                } else if (ctrl == 0x142) {
                    if (row >= 1) src = (int)(row * 16 - 1);
                } else if (ctrl == 0x143) {
                    if (row >= 2) src = 31;
                } else {
                    fprintf(stderr, "EMU: dpp ctrl %x not emulated\n", ctrl);
                    abort();
                }
                if (!((rmask >> row) & 1)) r = old;   // row disabled: keeps old
                else if (src < 0 || !waiting[src]) r = old;
                else r = (uint32_t)wv.val[src];
                break;
            }
            default: fprintf(stderr, "EMU: bad wave op %d\n", op); abort();
        }
        wv.res[l] = r;
    }
    for (uint32_t l = 0; l < 64; ++l)
        if (waiting[l]) w->f[base + l].state = RUN;
    wv.arrived = 0;
}

void run_block(Worker *w, const void *fn, dim3 bid, dim3 bdim, dim3 gdim, size_t lds) {
    const uint32_t B = bdim.x * bdim.y * bdim.z;
    if (w->f.size() < B) {
        size_t old = w->f.size();
        w->f.resize(B);
        for (size_t i = old; i < B; ++i) {
            w->f[i].stack = (char *)mmap(nullptr, kStack, PROT_READ | PROT_WRITE,
                                         MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
            if (w->f[i].stack == MAP_FAILED) { perror("mmap"); abort(); }
        }
    }
    w->B = B;
    w->live = B;
    w->block_arrived = 0;
    for (int i = 0; i < 16; ++i) { w->waves[i].arrived = 0; w->waves[i].live = 0; }
    w->lds = (unsigned char *)malloc(lds ? lds : 1);
    memset(w->lds, g_fill, lds ? lds : 1);
    for (uint32_t t = 0; t < B; ++t) {
        Fiber &f = w->f[t];
        f.state = RUN;
        f.ids.tid = dim3(t % bdim.x, (t / bdim.x) % bdim.y, t / (bdim.x * bdim.y));
        f.ids.bid = bid;
        f.ids.bdim = bdim;
        f.ids.gdim = gdim;
        f.ids.lane = t % 64;
        f.ids.wave = t / 64;
        w->waves[t / 64].live++;
        uint64_t *top = (uint64_t *)(f.stack + kStack);   // 16-aligned
        top[-1] = 0;                                      // fake return address of fiber_main
        top[-2] = (uint64_t)(uintptr_t)&fiber_main;       // where emu_switch returns
        for (int r = 3; r <= 8; ++r) top[-r] = 0;         // rbp rbx r12 r13 r14 r15
        f.sp = (void *)(top - 8);
    }
    for (;;) {
        bool ran = false;
        for (uint32_t t = 0; t < B; ++t) {
            Fiber &f = w->f[t];
            if (f.state != RUN) continue;
            ran = true;
            w->cur = &f;
#if EMU_ASAN
            __sanitizer_start_switch_fiber(&w->sched_fake, f.stack, kStack);
#endif
            emu_switch(&w->sched_sp, f.sp);
#if EMU_ASAN
            __sanitizer_finish_switch_fiber(w->sched_fake, nullptr, nullptr);
#endif
            w->cur = nullptr;
        }
        if (w->live == 0) break;
        bool released = false;
        // wave ops complete when every live lane of the wave waits at one
        for (uint32_t wi = 0; wi * 64 < B; ++wi) {
            Wave &wv = w->waves[wi];
            if (wv.live > 0 && wv.arrived == wv.live) {
                compute_wave(wv, w, wi);
                released = true;
            }
        }
        if (!released && w->block_arrived == w->live) {
            for (uint32_t t = 0; t < B; ++t)
                if (w->f[t].state == WBLOCK) w->f[t].state = RUN;
            w->block_arrived = 0;
            released = true;
        }
        if (!released && !ran) {
            fprintf(stderr, "EMU: deadlock in block (%u,%u) of kernel %p: live %u, at barrier %u\n",
                    bid.x, bid.y, fn, w->live, w->block_arrived);
            for (uint32_t wi = 0; wi * 64 < B; ++wi) {
                fprintf(stderr, "  wave %u: live %d waiting at wave op %d\n", wi, w->waves[wi].live,
                        w->waves[wi].arrived);
                for (uint32_t l = 0; l < 64 && wi * 64 + l < B; ++l)
                    if (w->f[wi * 64 + l].state == WWAVE) {
                        fprintf(stderr, "    lane %u op %d site %p\n", l, w->waves[wi].op[l], w->waves[wi].site[l]);
                        break;
                    }
            }
            fprintf(stderr, "  (wave-op sites are return addresses: subtract the load base from "
                            "/proc/<pid>/maps and use addr2line)\n");
            abort();
        }
    }
    free(w->lds);
    w->lds = nullptr;
}
}  // namespace

EmuIds &emu_ids() {
    Worker *w = tw;
    if (!w || !w->cur) { static thread_local EmuIds host; return host; }
    return w->cur->ids;
}
unsigned char *emu_smem() { return tw->lds; }

void emu_syncthreads() {
    Worker *w = tw;
    w->cur->state = WBLOCK;
    w->block_arrived++;
    yield_to_sched();
}

uint64_t emu_wave_op(int op, uint64_t v, uint64_t par) {
    Worker *w = tw;
    w->waves[w->cur->ids.wave].site[w->cur->ids.lane] = __builtin_return_address(0);
    Fiber *f = w->cur;
    Wave &wv = w->waves[f->ids.wave];
    const uint32_t l = f->ids.lane;
    wv.val[l] = v;
    wv.par[l] = par;
    wv.op[l] = op;
    wv.arrived++;
    f->state = WWAVE;
    yield_to_sched();
    return wv.res[l];
}

void emu_global_load_lds(const void *g, void *lds, int size) {
    Worker *w = tw;
    unsigned char *base = (unsigned char *)lds;
    if (base < w->lds) { fprintf(stderr, "EMU: LDS DMA below the LDS block\n"); abort(); }
    memcpy(base + (size_t)w->cur->ids.lane * size, g, size);
}

uint64_t wall_clock64() {
    return (uint64_t)std::chrono::steady_clock::now().time_since_epoch().count() / 10;
}

void emu_register_binder(const void *fn, EmuBinder bind) { reg()[fn] = std::move(bind); }

hipError_t emu_launch(const void *fn, dim3 g, dim3 b, size_t lds, std::function<void()> body) {
    if (g_capturing) {
        g_record.push_back(Recorded{fn, g, b, lds, std::move(body)});
        return hipSuccess;
    }
    return emu_run_grid(fn, g, b, lds, body);
}

hipError_t emu_run_grid(const void *fn, dim3 g, dim3 b, size_t lds, const std::function<void()> &body) {
    const uint32_t B = b.x * b.y * b.z;
    if (B == 0 || B > 1024 || B % 64) { last_err = hipErrorInvalidValue; return last_err; }
    auto it = attr().find(fn);
    const size_t limit = it != attr().end() && it->second > 65536 ? (size_t)it->second : 65536;
    if (lds > limit || lds > 163840) {
        fprintf(stderr, "EMU: launch with %zu bytes of LDS (limit %zu)\n", lds, limit);
        last_err = hipErrorInvalidValue;
        return last_err;
    }
    const uint64_t nb = (uint64_t)g.x * g.y * g.z;
    static int nthreads = getenv("EMU_THREADS") ? atoi(getenv("EMU_THREADS")) : 8;
    std::atomic<uint64_t> next{0};
    auto work = [&](int wi) {
        Worker *w = g_workers[wi];
        tw = w;
        w->body = &body;
        for (;;) {
            const uint64_t i = next.fetch_add(1);
            if (i >= nb) break;
            dim3 bid((uint32_t)(i % g.x), (uint32_t)((i / g.x) % g.y), (uint32_t)(i / ((uint64_t)g.x * g.y)));
            run_block(w, fn, bid, b, g, lds);
        }
        tw = nullptr;
    };
    {
        std::lock_guard<std::mutex> lk(g_mu);
        while ((int)g_workers.size() < nthreads) g_workers.push_back(new Worker());
    }
    if (nthreads <= 1 || nb == 1) {
        work(0);
    } else {
        std::vector<std::thread> th;
        for (int i = 0; i < nthreads; ++i) th.emplace_back(work, i);
        for (auto &t : th) t.join();
    }
    return hipSuccess;
}

// ---- runtime API
hipError_t hipMalloc(void **p, size_t n) {
    *p = malloc(n ? n : 1);
    if (!*p) return hipErrorOutOfMemory;
    memset(*p, g_fill, n);
    return hipSuccess;
}
hipError_t hipFree(void *p) { free(p); return hipSuccess; }
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) { if (n) memmove(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t) { return hipMemcpy(d, s, n, k); }
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t) { memset(d, v, n); return hipSuccess; }
hipError_t hipMemset(void *d, int v, size_t n) { memset(d, v, n); return hipSuccess; }
hipError_t hipGetLastError() { hipError_t e = last_err; last_err = hipSuccess; return e; }
hipError_t hipPeekAtLastError() { return last_err; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = (hipStream_t) new char[1]; return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { delete[](char *) s; return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) {
    g_capturing = true;
    g_record.clear();
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) {
    g_capturing = false;
    *g = (hipGraph_t) new std::vector<Recorded>(std::move(g_record));
    g_record.clear();
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t g, void *, char *, size_t) {
    *e = (hipGraphExec_t) new std::vector<Recorded>(*(std::vector<Recorded> *)g);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
    for (const Recorded &r : *(std::vector<Recorded> *)e) {
        const hipError_t rc = emu_run_grid(r.fn, r.g, r.b, r.lds, r.body);
        if (rc != hipSuccess) return rc;
    }
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) { delete (std::vector<Recorded> *)e; return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { delete (std::vector<Recorded> *)g; return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e) { *e = (hipEvent_t) new char[1]; return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) { delete[](char *) e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }
hipError_t hipFuncSetAttribute(const void *f, hipFuncAttribute, int v) { attr()[f] = v; return hipSuccess; }
hipError_t hipFuncGetAttributes(hipFuncAttributes *a, const void *) { memset(a, 0, sizeof(*a)); a->localSizeBytes = 1; return hipSuccess; }
hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int) {
    *v = a == hipDeviceAttributeCooperativeLaunch ? 0 : (a == hipDeviceAttributeMultiprocessorCount ? 256 : 100000);
    return hipSuccess;
}
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *n, const void *, int, size_t) { *n = 0; return hipSuccess; }
hipError_t hipLaunchKernel(const void *f, dim3 g, dim3 b, void **args, size_t lds, hipStream_t) {
    auto it = reg().find(f);
    if (it == reg().end()) { fprintf(stderr, "EMU: kernel %p not registered\n", f); abort(); }
    return emu_launch(f, g, b, lds, it->second(args));
}
hipError_t hipLaunchCooperativeKernel(const void *, dim3, dim3, void **, unsigned, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipGetSymbolAddress(void **p, const void *sym) { *p = (void *)sym; return hipSuccess; }

extern "C" void emu_set_fill(int v) { g_fill = v; }
extern "C" float __expf(float x) { return expf(x); }
extern "C" float __logf(float x) { return logf(x); }
