// Population storage formats in HBM.
//
// Every kernel computes in "shifted" space h_i = f_i - w_i: the moments are
// drho = sum h_i and j = sum e_i h_i (sum w_i = 1, sum w_i e_i = 0), which keeps the
// small deviations from the rest state free of the O(w_i) offset.  The storage trait
// converts between the stored element and h:
//   F64  : stores f (double), computes in double
//   F32  : stores f (float)                 -- the paper's plain single precision
//   F32S : stores h = f - w (float)         -- its round-off minimising formulation
//   BF16S: stores h as bfloat16, FP32 compute
//   F16S : stores h as IEEE half, FP32 compute
// The shifted formats follow the precision subsection of the paper (storing the
// deviation from the rest weights); BF16/F16 halve the bytes per population.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

enum StorageId { ST_F64 = 0, ST_F32 = 1, ST_F32S = 2, ST_BF16S = 3, ST_F16S = 4 };

// Counter-based 32-bit hash (the lowbias32 finaliser of C. Wellons' hash-prospector,
// a published integer mixer) for stochastic rounding draws.
__device__ __forceinline__ uint32_t hash32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// Random bits for stochastic rounding: one hash per node and step seeds Marsaglia's
// xorshift32 (shifts 13, 17, 5); each step gives the random bits of two stored values
// (its high and its low half).  The seed is forced odd so the state is never 0.
struct SrStream {
    uint32_t s;
    __device__ __forceinline__ uint32_t next() {
        s ^= s << 13;
        s ^= s >> 17;
        s ^= s << 5;
        return s;
    }
};
__device__ __forceinline__ SrStream sr_stream(uint32_t node, uint32_t step_key) {
    return SrStream{hash32(node ^ step_key) | 1u};
}

struct StF64 {
    using T = double;  // element in memory
    using C = double;  // compute type
    static constexpr int id = ST_F64;
    static constexpr bool shifted = false;
    static constexpr bool stochastic = false;
    __device__ static __forceinline__ C decode(T v, C w) { return v - w; }
    __device__ static __forceinline__ T encode(C h, C w, uint32_t) { return h + w; }
};

struct StF32 {
    using T = float;
    using C = float;
    static constexpr int id = ST_F32;
    static constexpr bool shifted = false;
    static constexpr bool stochastic = false;
    __device__ static __forceinline__ C decode(T v, C w) { return v - w; }
    __device__ static __forceinline__ T encode(C h, C w, uint32_t) { return h + w; }
};

struct StF32S {
    using T = float;
    using C = float;
    static constexpr int id = ST_F32S;
    static constexpr bool shifted = true;
    static constexpr bool stochastic = false;
    __device__ static __forceinline__ C decode(T v, C) { return v; }
    __device__ static __forceinline__ T encode(C h, C, uint32_t) { return h; }
};

// bfloat16 kept as raw bits: decode is a 16-bit shift, encode rounds to nearest even
// (hardware convert) or stochastically (add 16 random bits below the kept mantissa,
// then truncate; unbiased for finite values).
template <bool SR>
struct StBF16S {
    using T = uint16_t;
    using C = float;
    static constexpr int id = ST_BF16S;
    static constexpr bool shifted = true;
    static constexpr bool stochastic = SR;
    __device__ static __forceinline__ C decode(T v, C) { return __uint_as_float(uint32_t(v) << 16); }
    __device__ static __forceinline__ T encode(C h, C, uint32_t rnd) {
        if constexpr (SR) {
            uint32_t b = __float_as_uint(h);
            return uint16_t((b + (rnd >> 16)) >> 16);
        } else {
            __bf16 r = static_cast<__bf16>(h);
            return __builtin_bit_cast(uint16_t, r);
        }
    }
};

// IEEE half kept as raw bits.  Stochastic rounding rounds |h| up to the next half with
// probability equal to the fraction of a half-ulp step it lies above the one below:
//  - F16 normal range (|h| >= 2^-14): the half keeps 10 of FP32's 23 mantissa bits, so
//    13 random bits are added below the kept ones and the rest truncated; a carry
//    moves into the exponent as it should;
//  - subnormal range: the spacing is 2^-24, so floor(|h| 2^24 + u) 2^-24, u from the
//    top 16 random bits.
// Either result is a half exactly, so the final conversion does not round.
template <bool SR>
struct StF16S {
    using T = uint16_t;
    using C = float;
    static constexpr int id = ST_F16S;
    static constexpr bool shifted = true;
    static constexpr bool stochastic = SR;
    __device__ static __forceinline__ C decode(T v, C) {
        return static_cast<float>(__builtin_bit_cast(_Float16, v));
    }
    __device__ static __forceinline__ T encode(C h, C, uint32_t rnd) {
        if constexpr (SR) {
            const float a = fabsf(h);
            const float up = __uint_as_float((__float_as_uint(a) + (rnd >> 19)) & ~0x1fffu);
            const float sub = floorf(fmaf(a, 0x1p24f, float(rnd >> 16) * 0x1p-16f)) * 0x1p-24f;
            const float q = a >= 0x1p-14f ? up : sub;
            return __builtin_bit_cast(uint16_t, static_cast<_Float16>(copysignf(q, h)));
        } else {
            return __builtin_bit_cast(uint16_t, static_cast<_Float16>(h));
        }
    }
};

}  // namespace lbm
