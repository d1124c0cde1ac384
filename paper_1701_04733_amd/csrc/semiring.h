// Device-side semiring arithmetic for the tropical kernels (gfx950).
//
// Semirings of Sec. I, eqs. (1)-(4):  (+) is min (min-plus) or max (max-plus),
// (.) is +.  Conventions used by every kernel:
//
//  float32  (.) is one binary32 add (RN-even, denormals kept, no contraction);
//           (+) is fmin/fmax, which the compiler turns into v_min3_f32 /
//           v_max3_f32 when two terms are folded at once.  The absent value
//           is +inf (min-plus) or -inf (max-plus).
//  int32    (.) is a saturating add (v_add_i32 with clamp).  With every finite
//           operand bounded by |x| <= 2^29-1, a finite sum satisfies
//           |s| <= 2^30-2, while any sum that involves the absent value
//           0x7FFFFFFF (resp. -0x7FFFFFFF) is >= 2^31-2^29 (resp. <= -(2^31-2^29)),
//           so an accumulator is mapped back to the absent value once per
//           output with the threshold 2^30 ("finish" below).  This yields the
//           exact sentinel-absorbing result at no per-term cost.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "btas.h"

namespace btas {

template <int SR, typename T>
struct Ring;

template <>
struct Ring<BTAS_MIN_PLUS, float> {
    __device__ __forceinline__ static float absent() { return __builtin_inff(); }
    __device__ __forceinline__ static float mul(float a, float b) { return a + b; }
    __device__ __forceinline__ static float add(float a, float b) { return __builtin_fminf(a, b); }
    __device__ __forceinline__ static float add3(float a, float b, float c) {
        return __builtin_fminf(__builtin_fminf(a, b), c);
    }
    __device__ __forceinline__ static float finish(float x) { return x; }
};

template <>
struct Ring<BTAS_MAX_PLUS, float> {
    __device__ __forceinline__ static float absent() { return -__builtin_inff(); }
    __device__ __forceinline__ static float mul(float a, float b) { return a + b; }
    __device__ __forceinline__ static float add(float a, float b) { return __builtin_fmaxf(a, b); }
    __device__ __forceinline__ static float add3(float a, float b, float c) {
        return __builtin_fmaxf(__builtin_fmaxf(a, b), c);
    }
    __device__ __forceinline__ static float finish(float x) { return x; }
};

template <>
struct Ring<BTAS_MIN_PLUS, int32_t> {
    __device__ __forceinline__ static int32_t absent() { return BTAS_I32_INF; }
    __device__ __forceinline__ static int32_t mul(int32_t a, int32_t b) {
        return __builtin_elementwise_add_sat(a, b);
    }
    __device__ __forceinline__ static int32_t add(int32_t a, int32_t b) { return a < b ? a : b; }
    __device__ __forceinline__ static int32_t add3(int32_t a, int32_t b, int32_t c) {
        return add(add(a, b), c);
    }
    __device__ __forceinline__ static int32_t finish(int32_t x) {
        return x >= (1 << 30) ? BTAS_I32_INF : x;
    }
};

template <>
struct Ring<BTAS_MAX_PLUS, int32_t> {
    __device__ __forceinline__ static int32_t absent() { return BTAS_I32_NEG_INF; }
    __device__ __forceinline__ static int32_t mul(int32_t a, int32_t b) {
        return __builtin_elementwise_add_sat(a, b);
    }
    __device__ __forceinline__ static int32_t add(int32_t a, int32_t b) { return a > b ? a : b; }
    __device__ __forceinline__ static int32_t add3(int32_t a, int32_t b, int32_t c) {
        return add(add(a, b), c);
    }
    __device__ __forceinline__ static int32_t finish(int32_t x) {
        return x <= -(1 << 30) ? BTAS_I32_NEG_INF : x;
    }
};

template <typename T>
__device__ __forceinline__ uint32_t bits_of(T x) {
    return __builtin_bit_cast(uint32_t, x);
}

}  // namespace btas
