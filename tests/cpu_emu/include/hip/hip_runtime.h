// Host-only stand-in for <hip/hip_runtime.h>, used by the CPU bounds and
// parity harness under tests/cpu_emu.  TEST INFRASTRUCTURE: the product
// library is always built by hipcc for gfx950; this header lets the very
// same kernel and runtime sources be compiled for the host under
// AddressSanitizer + UndefinedBehaviorSanitizer, so that every memory
// access of every kernel is checked on the CPU before it runs on a GPU.
//
// Execution model: a launch runs its blocks one after another; the threads
// of a block are fibers (own stacks, switched by a few lines of x86-64
// assembly: glibc's swapcontext makes a signal-mask system call on every
// switch, which dominated the run time) that run until they reach a point where
// lanes exchange data -- __syncthreads(), __shfl_xor() or
// __builtin_amdgcn_readfirstlane() -- which act as barriers of the block or
// of the 64-lane wavefront, exactly as lock-step execution would order
// them.  Lanes that have returned no longer take part, like inactive lanes.
// Atomics are plain read-modify-writes (fibers switch only at barriers).
// Stream operations execute immediately; a captured graph records the
// launches (arguments evaluated at capture time) and replays them.
#pragma once

#include <limits.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <functional>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(x) __attribute__((aligned(x)))

struct dim3 {
    unsigned x, y, z;
    constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct int4 {
    int x, y, z, w;
};
inline int4 make_int4(int a, int b, int c, int d) { return int4{a, b, c, d}; }
struct alignas(16) float4 {
    float x, y, z, w;
};

typedef enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorInvalidConfiguration = 9,
    hipErrorInvalidDevice = 101,
    hipErrorStreamCaptureUnsupported = 900,
} hipError_t;

// device symbols are plain host arrays here, so a symbol's device address
// is its own address
#define HIP_SYMBOL(x) (&(x))
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) {
    *p = const_cast<void*>(sym);
    return hipSuccess;
}

inline const char* hipGetErrorString(hipError_t e) {
    switch (e) {
        case hipSuccess: return "hipSuccess";
        case hipErrorInvalidValue: return "hipErrorInvalidValue";
        case hipErrorInvalidConfiguration: return "hipErrorInvalidConfiguration";
        default: return "hipError(emulated)";
    }
}

typedef enum { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
               hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4 } hipMemcpyKind;
typedef enum { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal = 1,
               hipStreamCaptureModeRelaxed = 2 } hipStreamCaptureMode;
#define hipStreamNonBlocking 1

namespace hipemu {

struct Stream { int id; };
struct Graph { std::vector<std::function<void()>> ops; };
struct Event { int id; };

enum State { READY, AT_WAVE_FIRST, AT_WAVE_XOR, AT_WAVE_MFMA, AT_WAVE_BALLOT, AT_BLOCK, DONE };

struct Fiber {
    void* sp = nullptr;   // saved stack pointer while switched out
    char* stack = nullptr;
    int tid = 0;
    State st = READY;
    uint64_t in = 0, out = 0, in2 = 0;
    float acc[16];
    int mask = 0;
    void* asan_fake = nullptr;
};

struct Runtime {
    dim3 grid, block, bidx;
    std::vector<Fiber> fibers;
    void* sched_sp = nullptr;
    Fiber* cur = nullptr;
    const std::function<void()>* body = nullptr;
    Stream* capturing = nullptr;
    Graph* graph = nullptr;
    hipError_t last = hipSuccess;
    const void* sched_bottom = nullptr;
    size_t sched_size = 0;
    long long launches = 0;
};

Runtime& rt();

dim3 thread_idx();
inline dim3 block_idx() { return rt().bidx; }
inline dim3 block_dim() { return rt().block; }
inline dim3 grid_dim() { return rt().grid; }

uint64_t wave_op(State kind, uint64_t v, int mask);
void wave_mfma(uint64_t a, uint64_t b, float acc[16]);
void block_barrier();
void run_grid(dim3 g, dim3 b, const std::function<void()>& fn);

template <typename T>
inline uint64_t pack(T v) {
    uint64_t u = 0;
    memcpy(&u, &v, sizeof(T));
    return u;
}
template <typename T>
inline T unpack(uint64_t u) {
    T v;
    memcpy(&v, &u, sizeof(T));
    return v;
}

template <typename K, typename... A>
inline void launch(void* stream, dim3 g, dim3 b, K k, A... a) {
    Runtime& r = rt();
    if (g.x == 0 || g.y == 0 || g.z == 0 || b.x * b.y * b.z == 0 || b.x * b.y * b.z > 1024) {
        r.last = hipErrorInvalidConfiguration;
        return;
    }
    std::function<void()> fn = [=]() { k(a...); };
    if (r.capturing && static_cast<Stream*>(stream) == r.capturing) {
        r.graph->ops.push_back([g, b, fn]() { run_grid(g, b, fn); });
        return;
    }
    run_grid(g, b, fn);
}

}  // namespace hipemu

#define threadIdx (::hipemu::thread_idx())
#define blockIdx (::hipemu::block_idx())
#define blockDim (::hipemu::block_dim())
#define gridDim (::hipemu::grid_dim())

#define hipLaunchKernelGGL(kern, grid, block, shmem, stream, ...) \
    ::hipemu::launch((void*)(stream), dim3(grid), dim3(block), kern, __VA_ARGS__)

// launch with start/stop events stamped by the dispatch (timing is faked)
template <typename K, typename Ev, typename... A>
inline void hipExtLaunchKernelGGL(K kern, dim3 grid, dim3 block, unsigned shmem, void* stream,
                                  Ev, Ev, unsigned, A... a) {
    (void)shmem;
    ::hipemu::launch(stream, grid, block, kern, a...);
}

inline void __syncthreads() { ::hipemu::block_barrier(); }

inline int __builtin_amdgcn_readfirstlane(int v) {
    return ::hipemu::unpack<int>(::hipemu::wave_op(::hipemu::AT_WAVE_FIRST, ::hipemu::pack(v), 0));
}

// mask of the wavefront's active lanes whose predicate is true (bit = lane)
inline unsigned long long __builtin_amdgcn_ballot_w64(bool v) {
    return ::hipemu::wave_op(::hipemu::AT_WAVE_BALLOT, v ? 1u : 0u, 0);
}

template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
    (void)width;
    return ::hipemu::unpack<T>(::hipemu::wave_op(::hipemu::AT_WAVE_XOR, ::hipemu::pack(v), mask));
}

inline long long wall_clock64() {
    static long long t = 0;
    return t += 7;
}
inline void __builtin_amdgcn_s_waitcnt(int) {}
inline unsigned long long atomicMin(unsigned long long* p, unsigned long long v) {
    unsigned long long old = *p;
    if (v < old) *p = v;
    return old;
}
inline unsigned long long atomicMax(unsigned long long* p, unsigned long long v) {
    unsigned long long old = *p;
    if (v > old) *p = v;
    return old;
}

// v_mfma_f32_32x32x8_bf16: every lane of the wavefront supplies four bf16
// of A (row l % 32, k = 4 (l / 32) + u) and of B (column l % 32, same k);
// lane l's result register r holds row 8 (r / 4) + 4 (l / 32) + r % 4,
// column l % 32.
template <typename V4, typename V16>
inline V16 __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(V4 a, V4 b, V16 c, int, int, int) {
    uint64_t pa = 0, pb = 0;
    for (int u = 0; u < 4; ++u) {
        pa |= (uint64_t)(uint16_t)a[u] << (16 * u);
        pb |= (uint64_t)(uint16_t)b[u] << (16 * u);
    }
    float acc[16];
    for (int r = 0; r < 16; ++r) acc[r] = c[r];
    ::hipemu::wave_mfma(pa, pb, acc);
    for (int r = 0; r < 16; ++r) c[r] = acc[r];
    return c;
}

// v_mfma_f32_32x32x16_bf16 (gfx950): lane l supplies eight bf16 of A (row
// l % 32, k = 8 (l / 32) + u) and of B (column l % 32, same k); the result
// layout is that of the 32x32x8 form.  Emulated as two 32x32x8 products,
// one over u = 0..3 and one over u = 4..7 of every lane, which together
// take every k once.
template <typename V8, typename V16>
inline V16 __builtin_amdgcn_mfma_f32_32x32x16_bf16(V8 a, V8 b, V16 c, int, int, int) {
    float acc[16];
    for (int r = 0; r < 16; ++r) acc[r] = c[r];
    for (int h = 0; h < 2; ++h) {
        uint64_t pa = 0, pb = 0;
        for (int u = 0; u < 4; ++u) {
            const auto ea = a[4 * h + u], eb = b[4 * h + u];
            uint16_t ua, ub;
            memcpy(&ua, &ea, 2);
            memcpy(&ub, &eb, 2);
            pa |= (uint64_t)ua << (16 * u);
            pb |= (uint64_t)ub << (16 * u);
        }
        ::hipemu::wave_mfma(pa, pb, acc);
    }
    for (int r = 0; r < 16; ++r) c[r] = acc[r];
    return c;
}

// Buffer descriptors and raw buffer loads/stores.  The hardware returns
// zero for (and drops) an access beyond the descriptor's size; here such an
// access aborts, so that an indexing mistake cannot hide behind it.
struct HipemuBufferRsrc {
    char* base;
    long long bytes;
};
typedef HipemuBufferRsrc __amdgpu_buffer_rsrc_t;
inline __amdgpu_buffer_rsrc_t __builtin_amdgcn_make_buffer_rsrc(void* p, short, int bytes, int) {
    return HipemuBufferRsrc{static_cast<char*>(p), (long long)bytes};
}
inline char* hipemu_buffer_at(__amdgpu_buffer_rsrc_t r, int off, int soff, int size) {
    const long long o = (long long)(unsigned)off + (long long)(unsigned)soff;
    if (o + size > r.bytes) {
        fprintf(stderr, "hipemu: buffer access at byte %lld (+%d) beyond the descriptor's %lld bytes\n", o,
                size, r.bytes);
        abort();
    }
    return r.base + o;
}
inline unsigned __builtin_amdgcn_raw_buffer_load_b32(__amdgpu_buffer_rsrc_t r, int off, int soff, int) {
    unsigned v;
    memcpy(&v, hipemu_buffer_at(r, off, soff, 4), 4);
    return v;
}
inline unsigned short __builtin_amdgcn_raw_buffer_load_b16(__amdgpu_buffer_rsrc_t r, int off, int soff, int) {
    unsigned short v;
    memcpy(&v, hipemu_buffer_at(r, off, soff, 2), 2);
    return v;
}
inline void __builtin_amdgcn_raw_buffer_store_b32(unsigned v, __amdgpu_buffer_rsrc_t r, int off, int soff, int) {
    memcpy(hipemu_buffer_at(r, off, soff, 4), &v, 4);
}
inline void __builtin_amdgcn_raw_buffer_store_b16(unsigned short v, __amdgpu_buffer_rsrc_t r, int off, int soff,
                                                  int) {
    memcpy(hipemu_buffer_at(r, off, soff, 2), &v, 2);
}

inline int atomicMin(int* p, int v) {
    int old = *p;
    if (v < old) *p = v;
    return old;
}
inline int atomicMax(int* p, int v) {
    int old = *p;
    if (v > old) *p = v;
    return old;
}
inline int atomicAdd(int* p, int v) {
    int old = *p;
    *p = old + v;
    return old;
}
inline float atomicAdd(float* p, float v) {
    float old = *p;
    *p = old + v;
    return old;
}
inline unsigned long long atomicAdd(unsigned long long* p, unsigned long long v) {
    unsigned long long old = *p;
    *p = old + v;
    return old;
}
inline float unsafeAtomicAdd(float* p, float v) {
    float old = *p;
    *p = old + v;
    return old;
}
inline int atomicOr(int* p, int v) {
    int old = *p;
    *p = old | v;
    return old;
}

typedef hipemu::Stream* hipStream_t;
typedef hipemu::Graph* hipGraph_t;
typedef hipemu::Graph* hipGraphExec_t;
typedef hipemu::Event* hipEvent_t;
typedef void* hipGraphNode_t;

struct hipDeviceProp_t {
    char gcnArchName[256];
    int multiProcessorCount;
};
inline hipError_t hipGetDevice(int* d) {
    *d = 0;
    return hipSuccess;
}
inline hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
    strcpy(p->gcnArchName, "host-emulation");
    p->multiProcessorCount = 1;
    return hipSuccess;
}

#define hipDeviceAttributeWallClockRate 1
inline hipError_t hipDeviceGetAttribute(int* v, int, int) {
    *v = 100000;
    return hipSuccess;
}

inline hipError_t hipGetLastError() {
    hipError_t e = hipemu::rt().last;
    hipemu::rt().last = hipSuccess;
    return e;
}
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
    if (n) memcpy(d, s, n);
    return hipSuccess;
}
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) {
    if (n) memset(d, v, n);
    return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
    *s = new hipemu::Stream{1};
    return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) {
    delete s;
    return hipSuccess;
}
inline hipError_t hipEventCreate(hipEvent_t* e) {
    *e = new hipemu::Event{0};
    return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t = nullptr) { return hipSuccess; }
#define hipEventRecordExternal 0x01
inline hipError_t hipEventRecordWithFlags(hipEvent_t, hipStream_t, unsigned) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
    *ms = 1e-3f;
    return hipSuccess;
}
inline hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    hipemu::Runtime& r = hipemu::rt();
    if (r.capturing || !s) return hipErrorStreamCaptureUnsupported;
    r.capturing = s;
    r.graph = new hipemu::Graph();
    return hipSuccess;
}
inline hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
    hipemu::Runtime& r = hipemu::rt();
    if (r.capturing != s) return hipErrorInvalidValue;
    *g = r.graph;
    r.graph = nullptr;
    r.capturing = nullptr;
    return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
    *e = new hipemu::Graph(*g);
    return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
    for (auto& op : e->ops) op();
    return hipSuccess;
}
inline hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
    delete e;
    return hipSuccess;
}
inline hipError_t hipGraphDestroy(hipGraph_t g) {
    delete g;
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// implementation (header-only; one definition through inline functions)
// ---------------------------------------------------------------------------
#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#define HIPEMU_ASAN 1
#endif
#endif
#ifdef HIPEMU_ASAN
extern "C" void __sanitizer_start_switch_fiber(void** fake_stack_save, const void* bottom, size_t size);
extern "C" void __sanitizer_finish_switch_fiber(void* fake_stack_save, const void** bottom_old,
                                                size_t* size_old);
#endif

// Context switch (x86-64 System V): push the callee-saved registers on the
// current stack, store its pointer in *save, load `load` as the stack
// pointer, pop that stack's registers and return into it.  Weak, so that
// every translation unit including this header may define it.
extern "C" void hipemu_switch(void** save, void* load);
__asm__(".text\n"
        ".weak hipemu_switch\n"
        ".type hipemu_switch,@function\n"
        "hipemu_switch:\n"
        "  pushq %rbp\n  pushq %rbx\n  pushq %r12\n  pushq %r13\n  pushq %r14\n  pushq %r15\n"
        "  movq %rsp, (%rdi)\n"
        "  movq %rsi, %rsp\n"
        "  popq %r15\n  popq %r14\n  popq %r13\n  popq %r12\n  popq %rbx\n  popq %rbp\n"
        "  ret\n"
        ".size hipemu_switch, .-hipemu_switch\n");

namespace hipemu {

constexpr size_t kStack = 128 * 1024;

inline Runtime& rt() {
    static Runtime r;
    return r;
}

inline dim3 thread_idx() {
    Runtime& r = rt();
    const int t = r.cur->tid;
    return dim3(t % r.block.x, (t / r.block.x) % r.block.y, t / (r.block.x * r.block.y));
}

// switch from the running fiber back to the scheduler
inline void yield_to_sched(bool finished) {
    Runtime& r = rt();
    Fiber* f = r.cur;
#ifdef HIPEMU_ASAN
    __sanitizer_start_switch_fiber(finished ? nullptr : &f->asan_fake, r.sched_bottom, r.sched_size);
#endif
    hipemu_switch(&f->sp, r.sched_sp);
#ifdef HIPEMU_ASAN
    __sanitizer_finish_switch_fiber(f->asan_fake, nullptr, nullptr);
#endif
    (void)finished;
}

inline void fiber_entry() {
    Runtime& r = rt();
#ifdef HIPEMU_ASAN
    __sanitizer_finish_switch_fiber(nullptr, &r.sched_bottom, &r.sched_size);
#endif
    (*r.body)();
    r.cur->st = DONE;
    yield_to_sched(true);
    abort();  // a finished fiber is never resumed
}

inline uint64_t wave_op(State kind, uint64_t v, int mask) {
    Fiber* f = rt().cur;
    f->st = kind;
    f->in = v;
    f->mask = mask;
    yield_to_sched(false);
    return f->out;
}

inline void wave_mfma(uint64_t a, uint64_t b, float acc[16]) {
    Fiber* f = rt().cur;
    f->st = AT_WAVE_MFMA;
    f->in = a;
    f->in2 = b;
    for (int r = 0; r < 16; ++r) f->acc[r] = acc[r];
    yield_to_sched(false);
    for (int r = 0; r < 16; ++r) acc[r] = f->acc[r];
}

inline void block_barrier() {
    Fiber* f = rt().cur;
    f->st = AT_BLOCK;
    yield_to_sched(false);
}

inline void run_block(const std::function<void()>& fn) {
    Runtime& r = rt();
    const int n = (int)(r.block.x * r.block.y * r.block.z);
    if ((int)r.fibers.size() < n) r.fibers.resize(n);
    r.body = &fn;
    for (int t = 0; t < n; ++t) {
        Fiber& f = r.fibers[t];
        if (!f.stack) f.stack = static_cast<char*>(malloc(kStack));
        f.tid = t;
        f.st = READY;
        f.asan_fake = nullptr;
        // a fresh stack that hipemu_switch "returns" into fiber_entry from:
        // six zero register slots, then the entry address at a 16-byte
        // boundary, so that the entry sees the stack of a function call
        uintptr_t top = (reinterpret_cast<uintptr_t>(f.stack) + kStack) & ~(uintptr_t)15;
        void** slot = reinterpret_cast<void**>(top - 16);
        slot[0] = reinterpret_cast<void*>(&fiber_entry);
        for (int k = 1; k <= 6; ++k) slot[-k] = nullptr;
        f.sp = slot - 6;
    }
    const int nw = (n + 63) / 64;
    for (;;) {
        bool ran = false;
        for (int t = 0; t < n; ++t) {
            Fiber& f = r.fibers[t];
            if (f.st != READY) continue;
            ran = true;
            r.cur = &f;
            void* fake = nullptr;
#ifdef HIPEMU_ASAN
            __sanitizer_start_switch_fiber(&fake, f.stack, kStack);
#endif
            hipemu_switch(&r.sched_sp, f.sp);
#ifdef HIPEMU_ASAN
            __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#endif
        }
        (void)ran;
        bool all_done = true, resolved = false;
        for (int t = 0; t < n; ++t) all_done &= r.fibers[t].st == DONE;
        if (all_done) break;
        for (int w = 0; w < nw; ++w) {
            const int lo = w * 64, hi = lo + 64 < n ? lo + 64 : n;
            int live = 0, first = -1, kindc = 0;
            State kind = READY;
            bool same = true;
            for (int t = lo; t < hi; ++t) {
                const State s = r.fibers[t].st;
                if (s == DONE) continue;
                ++live;
                if (first < 0) { first = t; kind = s; }
                same &= s == kind;
                kindc += (s == AT_WAVE_FIRST || s == AT_WAVE_XOR || s == AT_WAVE_MFMA || s == AT_WAVE_BALLOT);
            }
            if (!live || !same ||
                (kind != AT_WAVE_FIRST && kind != AT_WAVE_XOR && kind != AT_WAVE_MFMA && kind != AT_WAVE_BALLOT))
                continue;
            if (kind == AT_WAVE_MFMA) {
                if (live != 64) {
                    fprintf(stderr, "hipemu: MFMA with inactive lanes\n");
                    abort();
                }
                auto bf = [](uint64_t p, int u) {
                    const uint32_t h = (uint32_t)((p >> (16 * u)) & 0xffffu) << 16;
                    float x;
                    memcpy(&x, &h, 4);
                    return x;
                };
                float Am[32][8], Bm[8][32];
                for (int l = 0; l < 64; ++l)
                    for (int u = 0; u < 4; ++u) {
                        Am[l % 32][4 * (l / 32) + u] = bf(r.fibers[lo + l].in, u);
                        Bm[4 * (l / 32) + u][l % 32] = bf(r.fibers[lo + l].in2, u);
                    }
                for (int l = 0; l < 64; ++l)
                    for (int q = 0; q < 16; ++q) {
                        const int row = 8 * (q / 4) + 4 * (l / 32) + q % 4, col = l % 32;
                        float s = 0.f;
                        for (int k = 0; k < 8; ++k) s += Am[row][k] * Bm[k][col];
                        r.fibers[lo + l].acc[q] += s;
                    }
                for (int t = lo; t < hi; ++t) r.fibers[t].st = READY;
                resolved = true;
                continue;
            }
            uint64_t ballot = 0;
            if (kind == AT_WAVE_BALLOT)
                for (int t = lo; t < hi; ++t)
                    if (r.fibers[t].st != DONE && r.fibers[t].in) ballot |= 1ull << (t - lo);
            for (int t = lo; t < hi; ++t) {
                Fiber& f = r.fibers[t];
                if (f.st == DONE) continue;
                if (kind == AT_WAVE_BALLOT) {
                    f.out = ballot;
                } else if (kind == AT_WAVE_FIRST) {
                    f.out = r.fibers[first].in;
                } else {
                    const int p = lo + ((t - lo) ^ f.mask);
                    if (p >= hi || r.fibers[p].st != AT_WAVE_XOR) {
                        fprintf(stderr, "hipemu: __shfl_xor partner lane %d inactive\n", p);
                        abort();
                    }
                    f.out = r.fibers[p].in;
                }
            }
            for (int t = lo; t < hi; ++t)
                if (r.fibers[t].st != DONE) r.fibers[t].st = READY;
            resolved = true;
        }
        if (resolved) continue;
        bool barrier = true;
        for (int t = 0; t < n; ++t) barrier &= (r.fibers[t].st == DONE || r.fibers[t].st == AT_BLOCK);
        if (barrier) {
            for (int t = 0; t < n; ++t)
                if (r.fibers[t].st == AT_BLOCK) r.fibers[t].st = READY;
            continue;
        }
        fprintf(stderr, "hipemu: lanes wait on different barriers (divergent sync) in block "
                        "(%u,%u,%u)\n", r.bidx.x, r.bidx.y, r.bidx.z);
        abort();
    }
}

inline void run_grid(dim3 g, dim3 b, const std::function<void()>& fn) {
    Runtime& r = rt();
    r.grid = g;
    r.block = b;
    r.launches++;
    for (unsigned z = 0; z < g.z; ++z)
        for (unsigned y = 0; y < g.y; ++y)
            for (unsigned x = 0; x < g.x; ++x) {
                r.bidx = dim3(x, y, z);
                run_block(fn);
            }
}

}  // namespace hipemu
