// Host stand-in for <hip/hip_runtime.h>: lets the integrator kernel sources compile as plain C++
// and run on the CPU, so that they can be checked under AddressSanitizer and
// UndefinedBehaviorSanitizer against the oracle.  Test infrastructure: the GPU library never
// includes it.
//
// What is emulated, and how:
//  * a launch runs one block at a time; each thread of the block is a fiber (ucontext) on one OS
//    thread, so a block's LDS (__shared__ arrays and the dynamic area) is shared by its threads
//    and the run is deterministic;
//  * __syncthreads, the wave barrier and every cross-lane operation (readlane, the DPP row
//    permutations the kernels use, ballot) are meeting points: each fiber writes its operand and
//    yields; once every live fiber of the block has arrived (one round of the scheduler), each
//    reads its source lane.  Meetings alternate between two buffers, so a fiber that has moved on
//    to the next meeting does not overwrite operands others still read.  The scheduler checks
//    that all live fibers arrive at the same meeting (same count, same kind) and aborts with a
//    message otherwise: a cross-lane operation in divergent control flow shows up that way;
//  * a lane that has returned is inactive for ballot;
//  * the hardware reciprocal is the exact one (the kernels refine it by Newton steps);
//  * device memory is host memory.
#pragma once

#include <math.h>
#include <ucontext.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#if defined(__SANITIZE_ADDRESS__)
#include <sanitizer/common_interface_defs.h>
#define EMU_ASAN 1
#endif

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) alignas(n)

using std::isfinite;
using std::isnan;

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct emu_uint3 {
    unsigned x, y, z;
};
inline emu_uint3 threadIdx, blockIdx;
inline dim3 blockDim, gridDim;

typedef int hipError_t;
typedef void *hipStream_t;
constexpr hipError_t hipSuccess = 0;
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize };
inline const char *hipGetErrorString(hipError_t) { return "emulated"; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipGetDevice(int *d) {
    *d = 0;
    return hipSuccess;
}
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipMalloc(void **p, size_t n) {
    *p = std::calloc(n ? n : 1, 1);
    return *p ? hipSuccess : 2;
}
inline hipError_t hipFree(void *p) {
    std::free(p);
    return hipSuccess;
}
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
    std::memcpy(d, s, n);
    return hipSuccess;
}
inline hipError_t hipFuncSetAttribute(const void *, hipFuncAttribute, int) { return hipSuccess; }

namespace emu {

constexpr size_t kStack = size_t(1) << 20;  // bytes of stack per emulated thread

enum Kind { kSync = 1, kExchange = 2, kBallot = 3 };

struct Fiber {
    ucontext_t ctx;
    std::vector<char> stack;
    bool done = false;
    long count = 0;  // meetings passed
    int kind = 0;    // kind of the meeting it waits at
};

struct Sched {
    ucontext_t main;
    std::vector<Fiber> f;
    int cur = -1;
    uint64_t buf[2][1024];
    void (*entry)(void *) = nullptr;
    void *arg = nullptr;
#ifdef EMU_ASAN
    const void *main_bottom = nullptr;
    size_t main_size = 0;
#endif
};

inline Sched *S = nullptr;
inline std::vector<unsigned char> dyn_lds_area;

template <class T>
T *dyn_lds() {
    return reinterpret_cast<T *>(dyn_lds_area.data());
}

// from a fiber back to the scheduler
inline void yield_to_main() {
    Fiber &me = S->f[S->cur];
#ifdef EMU_ASAN
    __sanitizer_start_switch_fiber(nullptr, S->main_bottom, S->main_size);
#endif
    swapcontext(&me.ctx, &S->main);
#ifdef EMU_ASAN
    __sanitizer_finish_switch_fiber(nullptr, nullptr, nullptr);
#endif
}

inline void fiber_entry() {
#ifdef EMU_ASAN
    __sanitizer_finish_switch_fiber(nullptr, &S->main_bottom, &S->main_size);
#endif
    S->entry(S->arg);
    S->f[S->cur].done = true;
    yield_to_main();  // never resumed
}

// wait at a meeting of the given kind; returns the buffer the meeting's operands went to
inline int meet(int kind) {
    Fiber &me = S->f[S->cur];
    const int p = int(me.count & 1);
    me.kind = kind;
    yield_to_main();
    ++me.count;
    return p;
}

inline uint64_t exchange(uint64_t v, int src) {
    const int p = int(S->f[S->cur].count & 1);
    S->buf[p][threadIdx.x] = v;
    meet(kExchange);
    return S->buf[p][src];
}

template <class F, class... A>
void launch(F kernel, dim3 grid, dim3 block, size_t shmem, A... args) {
    if (grid.y != 1 || grid.z != 1 || block.y != 1 || block.z != 1 || block.x > 1024) {
        std::fprintf(stderr, "emulated launch: only 1-D grids of at most 1024 threads\n");
        std::abort();
    }
    if (dyn_lds_area.size() < shmem) dyn_lds_area.assign(shmem, 0);
    auto call = [&] { kernel(args...); };
    using Call = decltype(call);
    Sched sched;
    Sched *prev = S;
    S = &sched;
    sched.entry = [](void *c) { (*static_cast<Call *>(c))(); };
    sched.arg = &call;
    blockDim = block;
    gridDim = grid;
    for (unsigned bx = 0; bx < grid.x; ++bx) {
        blockIdx = emu_uint3{bx, 0, 0};
        sched.f.assign(block.x, Fiber{});
        for (unsigned t = 0; t < block.x; ++t) {
            Fiber &fb = sched.f[t];
            fb.stack.assign(kStack, 0);
            getcontext(&fb.ctx);
            fb.ctx.uc_stack.ss_sp = fb.stack.data();
            fb.ctx.uc_stack.ss_size = kStack;
            fb.ctx.uc_link = nullptr;
            makecontext(&fb.ctx, fiber_entry, 0);
        }
        int live = int(block.x);
        while (live > 0) {
            long count = -1;
            int kind = 0;
            for (unsigned t = 0; t < block.x; ++t) {
                Fiber &fb = sched.f[t];
                if (fb.done) continue;
                sched.cur = int(t);
                threadIdx = emu_uint3{t, 0, 0};
#ifdef EMU_ASAN
                const void *bottom = nullptr;
                __sanitizer_start_switch_fiber(nullptr, fb.stack.data(), kStack);
#endif
                swapcontext(&sched.main, &fb.ctx);
#ifdef EMU_ASAN
                __sanitizer_finish_switch_fiber(nullptr, &bottom, nullptr);
#endif
                if (fb.done) {
                    --live;
                    continue;
                }
                if (count < 0) {
                    count = fb.count;
                    kind = fb.kind;
                } else if (fb.count != count || fb.kind != kind) {
                    std::fprintf(stderr,
                                 "emulated block %u: thread %u waits at meeting %ld (kind %d), others at %ld "
                                 "(kind %d): a cross-lane operation or barrier in divergent control flow\n",
                                 bx, t, fb.count, fb.kind, count, kind);
                    std::abort();
                }
            }
        }
    }
    S = prev;
}

}  // namespace emu

#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) \
    ::emu::launch(kernel, dim3(grid), dim3(block), size_t(shmem), __VA_ARGS__)

inline void __syncthreads() { (void)emu::meet(emu::kSync); }
inline void __builtin_amdgcn_wave_barrier() { (void)emu::meet(emu::kSync); }
#define __builtin_amdgcn_fence(...) ((void)0)

inline int __builtin_amdgcn_readlane(int v, int l) {
    return int(uint32_t(emu::exchange(uint64_t(uint32_t(v)), l)));
}

// the DPP controls the kernels use: quad_perm, row_half_mirror, row_mirror (every source lane
// valid, so `old` and the masks do not matter)
inline int __builtin_amdgcn_update_dpp(int old, int v, int ctrl, int, int, bool) {
    (void)old;
    const int lane = int(threadIdx.x);
    int src;
    if (ctrl < 0x100)
        src = (lane & ~3) | ((ctrl >> (2 * (lane & 3))) & 3);
    else if (ctrl == 0x140)
        src = (lane & ~15) | (15 - (lane & 15));
    else if (ctrl == 0x141)
        src = (lane & ~7) | (7 - (lane & 7));
    else {
        std::fprintf(stderr, "emulated DPP control 0x%x not supported\n", ctrl);
        std::abort();
    }
    return int(uint32_t(emu::exchange(uint64_t(uint32_t(v)), src)));
}

// lanes of the wave that have returned count as inactive
inline unsigned long long __ballot(int pred) {
    const int p = int(emu::S->f[emu::S->cur].count & 1);
    emu::S->buf[p][threadIdx.x] = pred ? 1u : 0u;
    emu::meet(emu::kBallot);
    unsigned long long m = 0;
    const unsigned w0 = threadIdx.x & ~63u;
    for (unsigned l = 0; l < 64 && w0 + l < blockDim.x; ++l)
        if (!emu::S->f[w0 + l].done && emu::S->buf[p][w0 + l]) m |= 1ull << l;
    return m;
}

inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __ffsll(long long x) { return __builtin_ffsll(x); }
inline double __builtin_amdgcn_rcp(double x) { return 1.0 / x; }
inline long long __double_as_longlong(double x) {
    long long r;
    std::memcpy(&r, &x, 8);
    return r;
}
inline double __longlong_as_double(long long x) {
    double r;
    std::memcpy(&r, &x, 8);
    return r;
}
inline unsigned long long atomicAdd(unsigned long long *p, unsigned long long v) {
    const unsigned long long o = *p;
    *p = o + v;
    return o;
}
inline int atomicAdd(int *p, int v) {
    const int o = *p;
    *p = o + v;
    return o;
}
