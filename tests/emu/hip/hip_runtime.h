// CPU emulation of the HIP subset used by the grid, merge and radix-sort
// sources, for tests that run their kernels on the host: the threads of a
// block run as std::threads (blocks one after another), __syncthreads is a
// block barrier, and the wave intrinsics (ballot, shuffles) exchange values
// through a per-wave barrier, so every lane of a wave must reach them
// together, as on the GPU.  Device memory is plain malloc, so a build with
// AddressSanitizer checks every access the kernels make.
#pragma once
#include <atomic>
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define HIP_SYMBOL(x) (&x)
#define amdgpu_waves_per_eu(...)

struct alignas(16) uint4 {
    unsigned x, y, z, w;
};
inline uint4 make_uint4(unsigned x, unsigned y, unsigned z, unsigned w) { return {x, y, z, w}; }

struct dim3 {
    unsigned x = 1, y = 1, z = 1;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
inline thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;

typedef int hipError_t;
typedef void* hipStream_t;
typedef void* hipEvent_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorInvalidValue = 1 };
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyHostToHost, hipMemcpyDefault };

inline hipError_t hipMalloc(void** p, size_t n) { *p = malloc(n); return *p ? hipSuccess : hipErrorOutOfMemory; }
enum { hipHostMallocDefault = 0 };
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned) { return hipMalloc(p, n); }
inline hipError_t hipHostFree(void* p) { free(p); return hipSuccess; }
inline hipError_t hipFree(void* p) { free(p); return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { memset(d, v, n); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) { *e = (void*)1; return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }
// launches run to completion when they are made, so every event has happened
#define hipEventDisableTiming 2u
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = (void*)1; return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }

// ---- block / wave synchronisation
struct EmuWave {
    std::barrier<>* bar;
    uint64_t vals[64];
};
struct EmuBlock {
    std::barrier<>* bar;
    EmuWave* waves;
};
inline thread_local EmuBlock* emu_blk = nullptr;

inline void __syncthreads() { emu_blk->bar->arrive_and_wait(); }
inline unsigned __lane_id() { return threadIdx.x % 64; }
inline EmuWave& emu_wave() { return emu_blk->waves[threadIdx.x / 64]; }
inline unsigned long long __ballot(int pred) {
    EmuWave& W = emu_wave();
    W.vals[__lane_id()] = pred ? 1 : 0;
    W.bar->arrive_and_wait();
    unsigned long long m = 0;
    for (int i = 0; i < 64; ++i)
        if (W.vals[i]) m |= 1ull << i;
    W.bar->arrive_and_wait();
    return m;
}
template <class T>
inline T emu_xchg(T v, unsigned src) {
    static_assert(sizeof(T) <= 8, "shfl");
    EmuWave& W = emu_wave();
    uint64_t u = 0;
    memcpy(&u, &v, sizeof(T));
    W.vals[__lane_id()] = u;
    W.bar->arrive_and_wait();
    uint64_t r = W.vals[src % 64];
    W.bar->arrive_and_wait();
    T out;
    memcpy(&out, &r, sizeof(T));
    return out;
}
template <class T> inline T __shfl(T v, int src, int = 64) { return emu_xchg(v, (unsigned)src); }
template <class T> inline T __shfl_xor(T v, int m, int = 64) { return emu_xchg(v, __lane_id() ^ (unsigned)m); }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __clzll(long long x) { return x ? __builtin_clzll((unsigned long long)x) : 64; }
inline int __ffsll(long long x) { return __builtin_ffsll(x); }
inline int __ffsll(unsigned long long x) { return __builtin_ffsll((long long)x); }
template <class T> inline T __shfl_up(T v, unsigned d, int = 64) {
    const unsigned lane = __lane_id();
    return emu_xchg(v, lane >= d ? lane - d : lane);
}
// AMDGCN builtins the sources call directly
inline unsigned long long __builtin_amdgcn_ballot_w64(bool p) { return __ballot(p); }
inline int __builtin_amdgcn_readlane(int v, int l) { return emu_xchg(v, (unsigned)l); }
// the sources apply it to wave-uniform values only, which every lane holds
inline int __builtin_amdgcn_readfirstlane(int v) { return v; }
inline void __builtin_amdgcn_wave_barrier() { emu_wave().bar->arrive_and_wait(); }
// the hardware square root is accurate to 1 ulp: the emulation errs low by
// one ulp, the side a lower bound built on it must tolerate
inline float __builtin_amdgcn_sqrtf(float x) {
    const float r = std::sqrt(x);
    return (r > 0.f && r < INFINITY) ? std::nextafter(r, 0.f) : r;
}
#define __builtin_amdgcn_fence(order, scope) std::atomic_thread_fence(std::memory_order_seq_cst)
#define __HIP_MEMORY_SCOPE_AGENT 3
#define __HIP_MEMORY_SCOPE_WORKGROUP 2
#define __hip_atomic_load(p, order, scope) __atomic_load_n((p), __ATOMIC_SEQ_CST)
#define __hip_atomic_store(p, v, order, scope) __atomic_store_n((p), (v), __ATOMIC_SEQ_CST)
inline int __float_as_int(float f) { int i; memcpy(&i, &f, 4); return i; }
inline unsigned __float_as_uint(float f) { unsigned i; memcpy(&i, &f, 4); return i; }
inline double __longlong_as_double(long long i) { double d; memcpy(&d, &i, 8); return d; }
inline int __popc(unsigned x) { return __builtin_popcount(x); }

template <class T> inline T atomicAdd(T* p, T v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
template <class T> inline T atomicOr(T* p, T v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
template <class T> inline T atomicAnd(T* p, T v) { return __atomic_fetch_and(p, v, __ATOMIC_SEQ_CST); }
template <class T> inline T atomicMax(T* p, T v) {
    T o = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (o < v && !__atomic_compare_exchange_n(p, &o, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {}
    return o;
}
inline float __double2float_rn(double x) { return (float)x; }
inline float __double2float_ru(double x) { float f = (float)x; if ((double)f < x) f = std::nextafter(f, INFINITY); return f; }
inline float __double2float_rd(double x) { float f = (float)x; if ((double)f > x) f = std::nextafter(f, -INFINITY); return f; }
inline float __int_as_float(int i) { float f; memcpy(&f, &i, 4); return f; }
inline long long __double_as_longlong(double d) { long long i; memcpy(&i, &d, 8); return i; }
using std::isfinite; using std::isnan; using std::floor; using std::fabs; using std::sqrt;
using std::fmin; using std::fmax;
template <class T> inline T max(T a, T b) { return a > b ? a : b; }
template <class T> inline T min(T a, T b) { return a < b ? a : b; }

// ---- launch: blocks in order, the threads of a block concurrently.  One
// host thread per thread of a block serves every block of the launch; a
// barrier separates consecutive blocks (so that LDS, a static array here, is
// not shared by two blocks at once).
extern long emu_launches;
template <class K, class... A>
void emu_launch(K kernel, dim3 g, dim3 b, A... args) {
    ++emu_launches;
    const unsigned nt = b.x;
    const unsigned nw = (nt + 63) / 64;
    std::barrier<> bar(nt), block_end(nt);
    std::vector<std::barrier<>*> wb(nw);
    std::vector<EmuWave> waves(nw);
    for (unsigned w = 0; w < nw; ++w) {
        unsigned lanes = std::min(64u, nt - 64 * w);
        wb[w] = new std::barrier<>(lanes);
        waves[w].bar = wb[w];
    }
    EmuBlock blk{&bar, waves.data()};
    std::vector<std::thread> th;
    th.reserve(nt);
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            threadIdx = dim3(t);
            blockDim = b;
            gridDim = g;
            emu_blk = &blk;
            for (unsigned bx = 0; bx < g.x; ++bx) {
                blockIdx = dim3(bx);
                kernel(args...);
                block_end.arrive_and_wait();
            }
        });
    for (auto& x : th) x.join();
    for (auto* p : wb) delete p;
}
#define hipLaunchKernelGGL(k, g, b, sh, st, ...) emu_launch(k, dim3(g), dim3(b), __VA_ARGS__)
