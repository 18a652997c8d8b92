// Shared device-side definitions of libitn (gfx950 / CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef __bf16 bf16_t;
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace itn {

enum Prec { P_F64 = 0, P_F32 = 1, P_BF16 = 2 };

// Operand / accumulator types of one matrix-core precision.
template <int P> struct PT;
template <> struct PT<P_F64> {
  using T = double;
  using Acc = double;
  using AccV = doublex4;
  static constexpr int E16 = 2;  // elements per 16-byte vector
};
template <> struct PT<P_F32> {
  using T = float;
  using Acc = float;
  using AccV = floatx4;
  static constexpr int E16 = 4;
};
template <> struct PT<P_BF16> {
  using T = bf16_t;
  using Acc = float;
  using AccV = floatx4;
  static constexpr int E16 = 8;
};

// Nearest bf16 to a double (ties to even), rounded once.  Narrowing to float
// first and then to bf16 rounds twice and can land one bf16 step off (a
// value just above a bf16 midpoint becomes the midpoint in float, which then
// ties to even).  Narrowing to float with round-to-odd instead (truncate
// toward zero, set the last significand bit when anything was dropped) keeps
// the information the second rounding needs, because float carries more
// than two bits beyond bf16's 8 (Boldo and Melquiond's round-to-odd
// theorem); the float -> bf16 step is the hardware's nearest-even rounding.
__device__ __forceinline__ bf16_t bf16_from_double(double x) {
  float f = (float)x;
  if ((double)f != x && f == f) {
    uint32_t u = __float_as_uint(f);
    if (__builtin_fabs((double)f) > __builtin_fabs(x)) u -= 1u;  // toward zero
    f = __uint_as_float(u | 1u);
  }
  return (bf16_t)f;
}

// Conversions used at load / store boundaries.
template <typename To, typename From> __device__ __forceinline__ To cvt(From x) { return (To)x; }
template <> __device__ __forceinline__ bf16_t cvt<bf16_t, double>(double x) { return bf16_from_double(x); }
template <> __device__ __forceinline__ double cvt<double, bf16_t>(bf16_t x) { return (double)(float)x; }

// Row of element j of lane `lane` in the 16x16 output block of a 16x16xK
// MFMA.  The f32-accumulating instructions place element j at row
// 4*(lane/16)+j; the f64 instruction at row 4*j + lane/16 (both measured on
// gfx950).  The column is lane % 16 for both.
template <int P> __device__ __forceinline__ int acc_row(int lane, int j) {
  if constexpr (P == P_F64) return 4 * j + (lane >> 4);
  else return 4 * (lane >> 4) + j;
}

}  // namespace itn
