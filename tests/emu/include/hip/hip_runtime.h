// CPU stand-in for the small part of the HIP API the gauge-fixing library
// uses.  TEST INFRASTRUCTURE: it lets the unmodified HIP sources be compiled
// by g++ and run on the host, so that index arithmetic, bounds and barrier
// placement can be checked on a machine without a GPU, with
// AddressSanitizer.  It is never part of the library that runs on the GPU.
//
// Blocks run one after another.  The threads of a block are fibers on one
// host thread (user-space stacks and a small context switch): each runs until
// its next __syncthreads, and once all of them are there the next round
// starts, so a barrier costs two context switches per thread.
#pragma once
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>
#include <random>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
// AMDGPU occupancy attributes carry no meaning on the CPU.
#define amdgpu_waves_per_eu(...) unused
#define __restrict__ __restrict
#define __align__(n) __attribute__((aligned(n)))
// one block runs at a time, so a function-static array is exactly the
// block's shared memory
#define __shared__ static

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

namespace emu {
inline dim3 tidx;
inline dim3 bidx, bdim, gdim;
inline std::vector<unsigned char> dyn_lds;
inline void yield_barrier();
}  // namespace emu

#define threadIdx (emu::tidx)
#define blockIdx (emu::bidx)
#define blockDim (emu::bdim)
#define gridDim (emu::gdim)
#define HIP_DYNAMIC_SHARED(type, var) type* var = reinterpret_cast<type*>(emu::dyn_lds.data());

inline void __syncthreads() { emu::yield_barrier(); }
inline void __threadfence() { std::atomic_thread_fence(std::memory_order_seq_cst); }

// Cross-lane read within a wavefront of 64 threads (ds_bpermute on the GPU).
// Every thread of the block must call it together, as every lane of a
// wavefront does on the GPU where the library uses it.
namespace emu {
inline std::vector<double> shfl_slots;
}
inline double __shfl(double v, int src_lane, int width = 64)
{
    const unsigned t = emu::tidx.x + emu::bdim.x * (emu::tidx.y + emu::bdim.y * emu::tidx.z);
    emu::shfl_slots[t] = v;
    emu::yield_barrier();
    const double r = emu::shfl_slots[(t & ~63u) | (unsigned)(src_lane & (width - 1))];
    emu::yield_barrier();
    return r;
}
inline float __shfl(float v, int src_lane, int width = 64) { return (float)__shfl((double)v, src_lane, width); }

// v_mfma_f64_16x16x4f64 of one wavefront: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; register j of lane l receives
// C + sum_k A[r][k] B[k][c] for r = l / 16 + 4 j, c = l % 16.  Every lane of
// the wavefront must call it (it exchanges values through __shfl).
template <typename V>
inline V __builtin_amdgcn_mfma_f64_16x16x4f64(double a, double b, V c, int, int, int)
{
    const int l = (int)(threadIdx.x & 63);
    double av[4][4], bv[4];
    for (int k = 0; k < 4; ++k) {
        for (int j = 0; j < 4; ++j) av[k][j] = __shfl(a, k * 16 + (l >> 4) + 4 * j);
        bv[k] = __shfl(b, k * 16 + (l & 15));
    }
    for (int j = 0; j < 4; ++j) {
        double s = c[j];
        for (int k = 0; k < 4; ++k) s += av[k][j] * bv[k];
        c[j] = s;
    }
    return c;
}

inline long long __double_as_longlong(double d)
{
    long long r;
    std::memcpy(&r, &d, sizeof r);
    return r;
}
using std::isfinite;
using std::fmax;
using std::fma;
using std::sqrt;

struct alignas(16) double2 {
    double x, y;
};
inline double2 make_double2(double x, double y) { return double2{x, y}; }

inline uint64_t __umul64hi(uint64_t a, uint64_t b) { return (uint64_t)(((unsigned __int128)a * b) >> 64); }

template <typename T>
inline T atomicAdd(T* p, T v)
{
    return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}
inline unsigned long long atomicMax(unsigned long long* p, unsigned long long v)
{
    unsigned long long old = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (old < v && !__atomic_compare_exchange_n(p, &old, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
    }
    return old;
}

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorInvalidValue = 1 };
typedef void* hipStream_t;
typedef struct emu_event* hipEvent_t;
struct emu_event {
    double t;
};
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyHostToHost };
enum { hipStreamNonBlocking = 1, hipHostMallocDefault = 0 };
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };

// Fill value for fresh "device" memory: NaN-like bytes, so reads of
// never-written memory show up in results.
inline hipError_t hipMalloc(void** p, size_t n)
{
    *p = std::malloc(n ? n : 1);
    if (!*p) return hipErrorOutOfMemory;
    std::memset(*p, 0xff, n);
    return hipSuccess;
}
template <typename T>
inline hipError_t hipMalloc(T** p, size_t n) { return hipMalloc(reinterpret_cast<void**>(p), n); }
inline hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned) { return hipMalloc(p, n); }
template <typename T>
inline hipError_t hipHostMalloc(T** p, size_t n, unsigned f) { return hipHostMalloc(reinterpret_cast<void**>(p), n, f); }
inline hipError_t hipHostFree(void* p) { std::free(p); return hipSuccess; }
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { std::memmove(d, s, n); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { std::memmove(d, s, n); return hipSuccess; }
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { std::memset(d, v, n); return hipSuccess; }
inline hipError_t hipMemset(void* d, int v, size_t n) { std::memset(d, v, n); return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = reinterpret_cast<hipStream_t>(0x1); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) { *e = new emu_event{0.0}; return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t)
{
    e->t = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
    return hipSuccess;
}
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) { *ms = (float)((b->t - a->t) * 1e3); return hipSuccess; }
inline hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "emulated HIP error"; }

// Graph capture: launches on a capturing stream are recorded, not run, and a
// graph launch replays them in order.
typedef struct emu_graph* hipGraph_t;
typedef struct emu_graph* hipGraphExec_t;
struct emu_graph {
    std::vector<std::function<void()>> ops;
};
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed };
namespace emu {
inline emu_graph* capturing = nullptr;
}
inline hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode)
{
    emu::capturing = new emu_graph();
    return hipSuccess;
}
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g)
{
    *g = emu::capturing;
    emu::capturing = nullptr;
    return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t* ex, hipGraph_t g, void*, void*, size_t)
{
    *ex = new emu_graph(*g);
    return hipSuccess;
}
inline hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t g) { delete g; return hipSuccess; }
inline hipError_t hipGraphLaunch(hipGraphExec_t g, hipStream_t)
{
    for (auto& op : g->ops) op();
    return hipSuccess;
}
enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount = 1 };
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
// A file-scope device array is an ordinary host array here.
#define HIP_SYMBOL(x) (&(x))
inline hipError_t hipGetSymbolAddress(void** p, const void* symbol)
{
    *p = const_cast<void*>(symbol);
    return hipSuccess;
}
inline hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { *v = 4; return hipSuccess; }

#if defined(__SANITIZE_ADDRESS__)
#include <sanitizer/common_interface_defs.h>
#endif

// Switch stacks: push the callee-saved registers, store the stack pointer in
// *save, load `load` and pop the next context's registers.  A new fiber's
// stack is laid out so that the final `ret` enters emu::fiber_entry.
extern "C" void emu_ctx_switch(void** save, void* load);
asm(R"(
    .text
    .weak emu_ctx_switch
    .type emu_ctx_switch, @function
emu_ctx_switch:
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
    .size emu_ctx_switch, .-emu_ctx_switch
)");

namespace emu {
constexpr size_t kFiberStack = size_t(512) << 10;
struct Fiber {
    void* sp = nullptr;
    char* stack = nullptr;
    int state = 0;              // 0 runnable, 1 at a barrier, 2 finished
    void* asan_fake = nullptr;
};
inline std::vector<Fiber> fibers;
inline void* sched_sp = nullptr;
inline void* sched_fake = nullptr;
inline const void* sched_bottom = nullptr;
inline size_t sched_size = 0;
inline unsigned cur = 0;
inline std::function<void()> body;

inline void asan_start(void** fake, const void* bottom, size_t size)
{
#if defined(__SANITIZE_ADDRESS__)
    __sanitizer_start_switch_fiber(fake, bottom, size);
#else
    (void)fake; (void)bottom; (void)size;
#endif
}
inline void asan_finish(void* fake, const void** bottom, size_t* size)
{
#if defined(__SANITIZE_ADDRESS__)
    __sanitizer_finish_switch_fiber(fake, bottom, size);
#else
    (void)fake; (void)bottom; (void)size;
#endif
}

[[noreturn]] inline void fiber_entry()
{
    asan_finish(nullptr, &sched_bottom, &sched_size);
    body();
    fibers[cur].state = 2;
    asan_start(nullptr, sched_bottom, sched_size);      // this fiber's stack is done with
    emu_ctx_switch(&fibers[cur].sp, sched_sp);
    __builtin_unreachable();
}

inline void yield_barrier()
{
    Fiber& f = fibers[cur];
    f.state = 1;
    asan_start(&f.asan_fake, sched_bottom, sched_size);
    emu_ctx_switch(&f.sp, sched_sp);
    asan_finish(f.asan_fake, nullptr, nullptr);
}

// One launch: blocks in order; the block's threads run as fibers in rounds
// from barrier to barrier.  The LDS is refilled with 0xff before each block,
// as a GPU gives no guarantee about it.
template <typename K, typename... Args>
void launch(K kernel, dim3 grid, dim3 block, size_t lds, Args... args)
{
    const unsigned nth = block.x * block.y * block.z;
    const unsigned nblk = grid.x * grid.y * grid.z;
    gdim = grid;
    bdim = block;
    dyn_lds.assign(lds ? lds : 1, 0xff);
    shfl_slots.assign(nth + 64, 0.0);
    if (fibers.size() < nth) fibers.resize(nth);
    for (unsigned t = 0; t < nth; ++t)
        if (!fibers[t].stack) fibers[t].stack = static_cast<char*>(std::malloc(kFiberStack));
    body = [&] { kernel(args...); };
    // Block order: ascending, or (LGF_EMU_BLOCK_ORDER) reversed or shuffled,
    // so a kernel whose result depends on the order of its blocks shows it.
    std::vector<unsigned> order(nblk);
    for (unsigned k = 0; k < nblk; ++k) order[k] = k;
    if (const char* o = std::getenv("LGF_EMU_BLOCK_ORDER")) {
        if (std::strcmp(o, "reverse") == 0) std::reverse(order.begin(), order.end());
        else if (std::strcmp(o, "shuffle") == 0) std::shuffle(order.begin(), order.end(), std::mt19937(12345u + nblk));
    }
    for (unsigned kk = 0; kk < nblk; ++kk) {
        const unsigned k = order[kk];
        bidx = dim3(k % grid.x, (k / grid.x) % grid.y, k / (grid.x * grid.y));
        std::memset(dyn_lds.data(), 0xff, dyn_lds.size());
        for (unsigned t = 0; t < nth; ++t) {
            Fiber& f = fibers[t];
            uintptr_t top = (reinterpret_cast<uintptr_t>(f.stack) + kFiberStack) & ~uintptr_t(15);
            void** sp = reinterpret_cast<void**>(top - 64);
            for (int r = 0; r < 6; ++r) sp[r] = nullptr;             // r15 .. rbp
            sp[6] = reinterpret_cast<void*>(&fiber_entry);           // ret target
            sp[7] = nullptr;
            f.sp = sp;
            f.state = 0;
        }
        bool live = true;
        while (live) {
            live = false;
            for (unsigned t = 0; t < nth; ++t) {
                Fiber& f = fibers[t];
                if (f.state == 2) continue;
                cur = t;
                tidx = dim3(t % block.x, (t / block.x) % block.y, t / (block.x * block.y));
                f.state = 0;
                asan_start(&sched_fake, f.stack, kFiberStack);
                emu_ctx_switch(&sched_sp, f.sp);
                asan_finish(sched_fake, nullptr, nullptr);
                if (f.state != 2) live = true;
            }
        }
    }
    body = nullptr;
}

template <typename K, typename... Args>
void launch_or_record(K kernel, dim3 grid, dim3 block, size_t lds, Args... args)
{
    if (capturing)
        capturing->ops.push_back([=] { launch(kernel, grid, block, lds, args...); });
    else
        launch(kernel, grid, block, lds, args...);
}
}  // namespace emu

#define hipLaunchKernelGGL(kernel, grid, block, lds, stream, ...) \
    emu::launch_or_record(kernel, grid, block, lds, __VA_ARGS__)
