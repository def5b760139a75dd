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

// Random words for stochastic rounding: one hash per node and step, r0, and for the
// stored value i the Weyl sequence r0 + i * 0x9e3779b9 (the golden-ratio increment; one
// add per value).  Each word is uniform over nodes and steps, which is what makes the
// rounding of every value unbiased; the words of one node are spread evenly over
// [0, 2^32) instead of being independent, which only lowers the variance of sums over
// the node's populations.
__device__ __forceinline__ uint32_t sr_word0(uint32_t node, uint32_t step_key) { return hash32(node ^ step_key); }
__device__ __forceinline__ uint32_t sr_word(uint32_t r0, int i) { return r0 + uint32_t(i) * 0x9e3779b9u; }

// gfx950's stochastic-rounding converts (v_cvt_sr_bf16_f32, v_cvt_sr_f16_f32) round an
// FP32 value up with probability equal to the dropped fraction of an ulp, taking the
// random word as a fraction in [0, 1) from its top bits (an in-bounds probe on the GPU:
// with the dropped fraction exactly 1/2, the word 2^31 rounds up and 2^31 - 1 does not;
// over 65 536 words the mean lands on the value within the sampling noise, for normal
// and subnormal BF16 and F16 results and both signs).
typedef __bf16 sr_bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 sr_f16x2 __attribute__((ext_vector_type(2)));

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

// bfloat16 kept as raw bits: decode is a 16-bit shift, encode rounds to nearest even or
// stochastically (hardware converts of both kinds).
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
            sr_bf16x2 v = {};
            v = __builtin_amdgcn_cvt_sr_bf16_f32(v, h, rnd, false);
            return __builtin_bit_cast(uint16_t, v[0]);
        } else {
            __bf16 r = static_cast<__bf16>(h);
            return __builtin_bit_cast(uint16_t, r);
        }
    }
};

// IEEE half kept as raw bits; encode rounds to nearest even or stochastically (the
// hardware converts; subnormal halves included).
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
            sr_f16x2 v = {};
            v = __builtin_amdgcn_cvt_sr_f16_f32(v, h, rnd, false);
            return __builtin_bit_cast(uint16_t, v[0]);
        } else {
            // The FP32 value is kept as such before the conversion.  The compiler would
            // otherwise fold the conversion into the multiply-add that produced it
            // (v_fma_mix, one rounding straight to F16 instead of FP32 then F16) in some
            // instantiations of a step and not in others, which then differ by an F16 ulp.
            // The empty asm only pins h to a register; it emits no instruction.
            float hr = h;
            asm("" : "+v"(hr));
            return __builtin_bit_cast(uint16_t, static_cast<_Float16>(hr));
        }
    }
};

}  // namespace lbm
