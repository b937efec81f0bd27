// CPU emulation of the small subset of HIP that the device kernels use, for
// running the kernel source on the host under AddressSanitizer (test
// infrastructure; never part of the library).  Every workgroup runs as real host
// threads (one per work item); workgroups run one after another, so kernel-local
// `__shared__` objects become function statics shared by the threads of the
// workgroup that is running.  A wave of 64 threads has its own barrier for
// shuffles, ballots and wave-level synchronisation.
#pragma once
#include <atomic>
#include <barrier>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <thread>
#include <tuple>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define PXCL_WAVES_PER_EU(...)
#define __shared__ static
#define __HIPCC__ 1

struct dim3 {
    uint32_t x, y, z;
    dim3(uint32_t a = 1, uint32_t b = 1, uint32_t c = 1) : x(a), y(b), z(c) {}
};
struct emu_idx { uint32_t x, y, z; };
struct uint4 { uint32_t x, y, z, w; };
inline thread_local emu_idx threadIdx, blockIdx, blockDim, gridDim;

struct EmuWave {
    std::barrier<> bar{64};
    uint64_t slot[64];
};
struct EmuWG {
    std::unique_ptr<std::barrier<>> bar;
    std::vector<std::unique_ptr<EmuWave>> waves;
};
inline thread_local EmuWG* emu_wg = nullptr;

inline EmuWave& emu_wave() { return *emu_wg->waves[threadIdx.x / 64]; }
inline uint32_t emu_lane() { return threadIdx.x & 63u; }

template <typename T>
inline T emu_read_lane(T v, uint32_t src) {
    static_assert(sizeof(T) <= 8, "lane values");
    EmuWave& w = emu_wave();
    uint64_t b = 0;
    std::memcpy(&b, &v, sizeof(T));
    w.slot[emu_lane()] = b;
    w.bar.arrive_and_wait();
    uint64_t r = w.slot[src & 63u];
    w.bar.arrive_and_wait();
    T out;
    std::memcpy(&out, &r, sizeof(T));
    return out;
}
template <typename T> inline T __shfl(T v, int src, int = 64) { return emu_read_lane(v, uint32_t(src)); }
template <typename T> inline T __shfl_up(T v, unsigned d, int = 64) {
    const uint32_t l = emu_lane();
    T r = emu_read_lane(v, l >= d ? l - d : l);
    return r;
}
template <typename T> inline T __shfl_xor(T v, int m, int = 64) { return emu_read_lane(v, emu_lane() ^ uint32_t(m)); }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline uint64_t __ballot(int pred) {
    EmuWave& w = emu_wave();
    w.slot[emu_lane()] = pred ? 1u : 0u;
    w.bar.arrive_and_wait();
    uint64_t m = 0;
    for (int i = 0; i < 64; ++i) m |= (w.slot[i] ? 1ull : 0ull) << i;
    w.bar.arrive_and_wait();
    return m;
}
inline uint32_t __builtin_amdgcn_readfirstlane(uint32_t v) { return emu_read_lane(v, 0); }
inline void __builtin_amdgcn_wave_barrier() { emu_wave().bar.arrive_and_wait(); }
inline void __builtin_amdgcn_s_barrier() { emu_wg->bar->arrive_and_wait(); }
inline void __builtin_amdgcn_fence(int, const char*, const char* = nullptr) {
    std::atomic_thread_fence(std::memory_order_seq_cst);
}
inline void __builtin_amdgcn_s_waitcnt(int) {}
inline int __popc(uint32_t x) { return __builtin_popcount(x); }
inline float __int_as_float(int x) {
    float f;
    std::memcpy(&f, &x, sizeof(f));
    return f;
}
inline int __ffs(uint32_t x) { return __builtin_ffs(int(x)); }
inline int __ffsll(unsigned long long x) { return __builtin_ffsll((long long)x); }
template <typename T> inline T min(T a, T b) { return a < b ? a : b; }
template <typename T> inline T max(T a, T b) { return a > b ? a : b; }

#define __HIP_MEMORY_SCOPE_WAVEFRONT 1
#define __HIP_MEMORY_SCOPE_WORKGROUP 2
#define __HIP_MEMORY_SCOPE_AGENT 3
#define __HIP_MEMORY_SCOPE_SYSTEM 4
template <typename T> inline T __hip_atomic_load(const T* p, int, int) { return __atomic_load_n(p, __ATOMIC_SEQ_CST); }
template <typename T> inline void __hip_atomic_store(T* p, T v, int, int) { __atomic_store_n(p, v, __ATOMIC_SEQ_CST); }
template <typename T> inline T __hip_atomic_fetch_min(T* p, T v, int, int) {
    T cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (v < cur && !__atomic_compare_exchange_n(p, &cur, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {}
    return cur;
}
template <typename T> inline T __hip_atomic_fetch_add(T* p, T v, int, int) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline uint32_t atomicAdd(uint32_t* p, uint32_t v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline unsigned long long atomicAdd(unsigned long long* p, unsigned long long v) {
    return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}
inline uint64_t atomicAdd(uint64_t* p, uint64_t v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline uint32_t atomicOr(uint32_t* p, uint32_t v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
inline uint64_t atomicCAS(uint64_t* p, uint64_t cmp, uint64_t v) {
    __atomic_compare_exchange_n(p, &cmp, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
    return cmp;
}

// host API subset used by the launch helpers
typedef int hipError_t;
typedef void* hipStream_t;
#define hipSuccess 0
#define hipErrorInvalidValue 1
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void*, int, size_t) {
    *n = 1;
    return hipSuccess;
}

// Run a kernel: workgroups one after another, each as blockDim host threads.
template <typename... P, typename... A>
inline void emu_launch(void (*k)(P...), dim3 grid, dim3 block, A... args_in) {
    const std::tuple<P...> args(static_cast<P>(args_in)...);
    for (uint32_t b = 0; b < grid.x; ++b) {
        EmuWG wg;
        wg.bar = std::make_unique<std::barrier<>>(block.x);
        for (uint32_t w = 0; w < (block.x + 63) / 64; ++w) wg.waves.push_back(std::make_unique<EmuWave>());
        std::vector<std::thread> th;
        th.reserve(block.x);
        for (uint32_t t = 0; t < block.x; ++t)
            th.emplace_back([&, t, b]() {
                threadIdx = {t, 0, 0};
                blockIdx = {b, 0, 0};
                blockDim = {block.x, 1, 1};
                gridDim = {grid.x, 1, 1};
                emu_wg = &wg;
                std::apply(k, args);
            });
        for (auto& x : th) x.join();
    }
}
#define hipLaunchKernelGGL(k, grid, block, shmem, stream, ...) emu_launch(k, dim3(grid), dim3(block), __VA_ARGS__)
