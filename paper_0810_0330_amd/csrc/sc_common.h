// Internal helpers shared by the library's translation units: complex
// arithmetic, wave/block reductions, deterministic split reductions, error
// plumbing and workspace carving.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/seedcg.h"

namespace sc {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
void clear_error();

#define SC_HIP(expr)                                                                  \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess) {                                                       \
            ::sc::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));       \
            return SC_ERR_HIP;                                                        \
        }                                                                             \
    } while (0)

#define SC_LAUNCH_CHECK() SC_HIP(hipGetLastError())

#define SC_ARG(cond, msg)                                                             \
    do {                                                                              \
        if (!(cond)) {                                                                \
            ::sc::set_error(std::string("argument error: ") + (msg));                 \
            return SC_ERR_ARG;                                                        \
        }                                                                             \
    } while (0)

#define SC_TRY(expr)                                                                  \
    do {                                                                              \
        sc_status s_ = (expr);                                                        \
        if (s_ != SC_OK) return s_;                                                   \
    } while (0)

// ---------------------------------------------------------------- complex
template <typename R>
struct cplx {
    R re, im;
};

template <typename R> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };

template <typename R>
__device__ __forceinline__ cplx<R> ld2(const R* p, int64_t idx) {
    auto v = reinterpret_cast<const typename vec2<R>::type*>(p)[idx];
    return {v.x, v.y};
}
template <typename R>
__device__ __forceinline__ void st2(R* p, int64_t idx, cplx<R> c) {
    typename vec2<R>::type v;
    v.x = c.re;
    v.y = c.im;
    reinterpret_cast<typename vec2<R>::type*>(p)[idx] = v;
}

// ---------------------------------------------------------------- reductions
constexpr int kBlock = 256;          // threads per block of the streaming kernels
constexpr int kWaves = kBlock / 64;  // 64-wide wavefronts
// XCDs of the chip: workgroup b of a launch runs on XCD b % kXcd, each with its own L2
constexpr int kXcd = 8;
constexpr int kMaxRedBlocks = 512;   // split-reduction width cap

// v plus the value that DPP control CTRL moves into this lane, in the rows of
// RMASK (plus 0 in the others): one DPP move per 32-bit half, no LDS round trip
template <int CTRL, int RMASK>
__device__ __forceinline__ double dpp_add(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, RMASK, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, RMASK, 0xF, false);
    return v + __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum over the 64 lanes of a wave (all lanes active); every lane gets the
// total.  Pairs, quads, groups of 8 and rows of 16 by DPP lane permutations
// (every lane of a row then holds the row's sum), the four rows by the two row
// broadcasts (lane 63 then holds the total), read back from lane 63.  A fixed
// tree, so the result is deterministic.
__device__ __forceinline__ double wave_sum(double v) {
    v = dpp_add<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v = dpp_add<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v = dpp_add<0x141, 0xF>(v);  // row_half_mirror
    v = dpp_add<0x140, 0xF>(v);  // row_mirror
    v = dpp_add<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), 63);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum over the block; every thread gets the total.  Deterministic: fixed tree.
__device__ __forceinline__ double block_sum(double v, double* sh /* kWaves doubles */) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) t += sh[i];
    return t;
}

// Cross-block reductions without device-scope fences: a producer kernel
// leaves one partial per block (block_partial); every block of a consumer
// kernel adds all of them in index order (sum_partials), so each block gets the
// same, deterministic value.  Kernel boundaries order the two.  (An in-kernel
// last-block scheme needs an agent-scope release per block, which on a
// multi-XCD part writes back the L2 and costs more than the re-summation.)
__device__ __forceinline__ void block_partial(double v, double* part, double* sh) {
    const double b = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = b;
}

__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int G, double* sh) {
    double s = 0.0;
    for (int i = threadIdx.x; i < G; i += blockDim.x) s += part[i];
    return block_sum(s, sh);
}

// 16-byte packs for the streaming kernels (dwordx4 loads and stores)
template <typename R>
struct alignas(16) Pack {
    static constexpr int W = 16 / sizeof(R);
    R v[W];
};
template <typename R>
__device__ __forceinline__ Pack<R> ldp(const R* p, int64_t i) {
    return *reinterpret_cast<const Pack<R>*>(p + i);
}
template <typename R>
__device__ __forceinline__ void stp(R* p, int64_t i, const Pack<R>& v) {
    *reinterpret_cast<Pack<R>*>(p + i) = v;
}

inline int red_grid(int64_t n_items, int per_thread = 16) {
    int64_t g = (n_items + (int64_t)kBlock * per_thread - 1) / ((int64_t)kBlock * per_thread);
    if (g < 1) g = 1;
    if (g > kMaxRedBlocks) g = kMaxRedBlocks;
    return (int)g;
}

// ---------------------------------------------------------------- workspace
struct Carver {
    char* base;
    size_t cap;
    size_t off = 0;
    bool dry;  // size query only
    Carver(void* b, size_t c) : base((char*)b), cap(c), dry(b == nullptr) {}
    // 256-byte aligned carving (absolute addresses; a dry run assumes an aligned base)
    template <typename T>
    T* take(size_t count) {
        const uintptr_t addr = ((uintptr_t)base + off + 255) & ~uintptr_t(255);
        off = addr - (uintptr_t)base;
        T* p = dry ? nullptr : reinterpret_cast<T*>(base + off);
        off += count * sizeof(T);
        return p;
    }
    bool ok() const { return dry || off <= cap; }
};

inline bool is_complex(sc_dtype d) { return d == SC_C64 || d == SC_C128; }
inline bool is_single(sc_dtype d) { return d == SC_C64 || d == SC_R32; }
inline size_t dtype_bytes(sc_dtype d) {
    switch (d) {
        case SC_R64: return 8;
        case SC_C64: return 8;
        case SC_C128: return 16;
        case SC_R32: return 4;
    }
    return 0;
}
inline sc_dtype single_of(sc_dtype d) { return d == SC_C128 ? SC_C64 : (d == SC_R64 ? SC_R32 : d); }
inline sc_dtype double_of(sc_dtype d) { return d == SC_C64 ? SC_C128 : (d == SC_R32 ? SC_R64 : d); }

}  // namespace sc
