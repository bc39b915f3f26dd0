// device.hpp -- wave64 primitives and the counter-based random numbers used
// by every gfx950 kernel of the estimator.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pe {

constexpr int kWave = 64;
constexpr uint16_t kRetired = 0xFFFF;   // degree sentinel of a matched vertex
constexpr double kLn2 = 0.69314718055994530941723212145818;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// ------------------------------------------------------------ address spaces
// A pointer the compiler cannot trace to its allocation (one loaded from an
// argument block) is generic, and its accesses become flat instructions.
// Those count against the LDS wait counter as well as the vector-memory one,
// so every LDS access or cross-lane exchange that waits for its result would
// also wait for all outstanding HBM loads and stores. Device code therefore
// re-types such pointers as global (address space 1) or LDS (3) ones.
// Argument blocks, written by the host before a launch and never by the
// kernels, are read through the constant address space (4): the compiler
// then reads their fields with scalar loads that need not wait for the
// trajectory's own stores, and may keep or re-read them at will.
#if defined(__HIP_DEVICE_COMPILE__)
#define PE_G __attribute__((address_space(1)))
#define PE_L __attribute__((address_space(3)))
#define PE_C __attribute__((address_space(4)))
#else
#define PE_G
#define PE_L
#define PE_C
#endif
constexpr int kAsGlobal = 1, kAsLds = 3;
template <int AS, class T> struct AsPtr { using type = PE_G T *; };
template <class T> struct AsPtr<kAsLds, T> { using type = PE_L T *; };
template <int AS, class T> using as_ptr = typename AsPtr<AS, T>::type;
template <int AS, class T>
__device__ __forceinline__ as_ptr<AS, T> to_as(T *p) { return (as_ptr<AS, T>)p; }
template <class T>
__device__ __forceinline__ PE_G T *gptr(T *p) { return (PE_G T *)p; }
template <class T>
__device__ __forceinline__ const PE_C T *cptr(const T *p) { return (const PE_C T *)p; }
// the same address space with another element type
template <class U, class T>
__device__ __forceinline__ PE_G U *recast(PE_G T *p) { return (PE_G U *)p; }
#if defined(__HIP_DEVICE_COMPILE__)
template <class U, class T>
__device__ __forceinline__ PE_L U *recast(PE_L T *p) { return (PE_L U *)p; }
#endif

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Order this wave's earlier LDS / global accesses before its later ones
// (values are exchanged between lanes of one wave through memory).
__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// Lane src's value in every lane (src must be the same in all lanes); the
// result is wave-uniform, so the compiler may keep it in a scalar register.
template <typename T>
__device__ __forceinline__ T read_lane(T v, int src) {
    if constexpr (sizeof(T) == 8) {
        uint64_t u;
        __builtin_memcpy(&u, &v, 8);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, src);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), src);
        u = ((uint64_t)hi << 32) | lo;
        T r;
        __builtin_memcpy(&r, &u, 8);
        return r;
    } else if constexpr (sizeof(T) == 4) {
        uint32_t u;
        __builtin_memcpy(&u, &v, 4);
        u = (uint32_t)__builtin_amdgcn_readlane((int)u, src);
        T r;
        __builtin_memcpy(&r, &u, 4);
        return r;
    } else {
        return (T)__builtin_amdgcn_readlane((int)v, src);
    }
}

// a value that every lane already holds, made visibly uniform
template <typename T>
__device__ __forceinline__ T uniform(T v) { return read_lane(v, 0); }

// ------------------------------------------------------------ DPP
// Cross-lane data movement by DPP (data-parallel primitives: operands read
// from another lane of the same VGPR in the same VALU instruction), no LDS
// crossbar.  A lane whose source lies outside its row, or whose row is
// masked off, receives `old` (bound_ctrl off).
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ uint32_t dpp(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWS, 0xF, false);
}

// Inclusive scan in lane order for an associative op with identity `id`:
// four shifted steps within each 16-lane row, then the last lane of row 0
// (and of row 2) is added to row 1 (row 3), then lane 31 to rows 2 and 3.
template <typename Op>
__device__ __forceinline__ uint32_t wave_scan_u32(uint32_t x, uint32_t id, Op op) {
    x = op(x, dpp<kRowShr1>(id, x));
    x = op(x, dpp<kRowShr2>(id, x));
    x = op(x, dpp<kRowShr4>(id, x));
    x = op(x, dpp<kRowShr8>(id, x));
    x = op(x, dpp<kRowBcast15, 0xA>(id, x));
    x = op(x, dpp<kRowBcast31, 0xC>(id, x));
    return x;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
    const uint32_t r = wave_scan_u32(x, 0xFFFFFFFFu, [](uint32_t a, uint32_t b) { return b < a ? b : a; });
    return read_lane(r, kWave - 1);
}

// plain comparisons (no fmaxf), so a NaN from another lane never wins
__device__ __forceinline__ float wave_max_f32(float x) {
    const uint32_t r = wave_scan_u32(__float_as_uint(x), __float_as_uint(-__builtin_huge_valf()),
                                     [](uint32_t a, uint32_t b) {
                                         const float fa = __uint_as_float(a), fb = __uint_as_float(b);
                                         return fb > fa ? b : a;
                                     });
    return __uint_as_float(read_lane(r, kWave - 1));
}

__device__ __forceinline__ int32_t wave_max_i32(int32_t x) {
    const uint32_t r = wave_scan_u32((uint32_t)x, 0x80000000u, [](uint32_t a, uint32_t b) {
        return (int32_t)b > (int32_t)a ? b : a;
    });
    return (int32_t)read_lane(r, kWave - 1);
}

// inclusive prefix sum over the 64 lanes in lane order (exact, 64-bit)
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t x) {
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    auto step = [&](uint32_t ylo, uint32_t yhi) {
        const uint32_t s = lo + ylo;
        hi = hi + yhi + (s < lo ? 1u : 0u);
        lo = s;
    };
    step(dpp<kRowShr1>(0u, lo), dpp<kRowShr1>(0u, hi));
    step(dpp<kRowShr2>(0u, lo), dpp<kRowShr2>(0u, hi));
    step(dpp<kRowShr4>(0u, lo), dpp<kRowShr4>(0u, hi));
    step(dpp<kRowShr8>(0u, lo), dpp<kRowShr8>(0u, hi));
    step(dpp<kRowBcast15, 0xA>(0u, lo), dpp<kRowBcast15, 0xA>(0u, hi));
    step(dpp<kRowBcast31, 0xC>(0u, lo), dpp<kRowBcast31, 0xC>(0u, hi));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) { return read_lane(wave_incl_scan_u64(x), kWave - 1); }

// 32-bit inclusive prefix sum, for values whose total over the wave fits
// (integer proposal weights are at most 2^24 + 1, so 64 of them do)
__device__ __forceinline__ uint32_t wave_incl_scan_add_u32(uint32_t x) {
    return wave_scan_u32(x, 0u, [](uint32_t a, uint32_t b) { return a + b; });
}

__device__ __forceinline__ int wave_sum_i32(int x) {
    const uint32_t r = wave_scan_u32((uint32_t)x, 0u, [](uint32_t a, uint32_t b) { return a + b; });
    return (int)read_lane(r, kWave - 1);
}

// float sum in the scan's fixed combination order
__device__ __forceinline__ float wave_sum_f32(float x) {
    const uint32_t r = wave_scan_u32(__float_as_uint(x), 0u, [](uint32_t a, uint32_t b) {
        return __float_as_uint(__uint_as_float(a) + __uint_as_float(b));
    });
    return __uint_as_float(read_lane(r, kWave - 1));
}

// number of set bits of `mask` strictly below this lane
__device__ __forceinline__ int rank_below(uint64_t mask) {
    const int l = lane_id();
    uint64_t below = (l == 0) ? 0ull : (mask & (~0ull >> (64 - l)));
    return __popcll(below);
}


// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32 -> 64-bit products, key bumped by the golden-ratio Weyl constants.
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// 64 random bits for (seed; trajectory k, matrix b, step t, draw d)
__device__ __forceinline__ uint64_t rand64(uint64_t seed, uint32_t k, uint32_t b, uint32_t t, uint32_t d) {
    U4 o = philox4x32_10(U4{k, b, t, d}, (uint32_t)seed, (uint32_t)(seed >> 32));
    return ((uint64_t)o.y << 32) | o.x;
}

// Uniform integer in [0, W), W >= 1, by Lemire's multiply-and-reject method
// (ACM TOMACS 2019); each rejection moves to the next draw index.
__device__ __forceinline__ uint64_t uniform_below(uint64_t seed, uint32_t k, uint32_t b, uint32_t t,
                                                  uint32_t d, uint64_t W) {
    for (;;) {
        const uint64_t x = rand64(seed, k, b, t, d);
        const uint64_t hi = __umul64hi(x, W);
        const uint64_t lo = x * W;
        if (lo < W) {
            const uint64_t thr = (0ull - W) % W;
            if (lo < thr) { ++d; continue; }
        }
        return hi;
    }
}

// SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014) folded over a word
__device__ __forceinline__ uint64_t splitmix_fold(uint64_t h, uint64_t x) {
    uint64_t z = h + 0x9E3779B97F4A7C15ull + x;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace pe
