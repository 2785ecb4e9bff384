// MFMA building blocks shared by the band factorisation and the solves.
#pragma once

#include "rr_internal.h"

namespace rr {

// 16x16x4 MFMA per precision and the position of accumulator element e of
// lane l (measured on gfx950: f64 puts element e at row l/16 + 4e, f32 at
// row 4(l/16) + e; both at column l%16; operand a is A[l%16][l/16], operand b
// is B[l/16][l%16]).
template <typename R>
struct Mf;
template <>
struct Mf<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int e) { return (l >> 4) + 4 * e; }
};
template <>
struct Mf<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int e) { return 4 * (l >> 4) + e; }
};

// One complex k-step: (are, aim) += (s a) * b with s = -1 when SUB, and a
// conjugated when CA.  A complex product is four real MFMAs.
template <typename R, bool CA, bool SUB>
__device__ __forceinline__ void cmfma(typename Mf<R>::v4& are, typename Mf<R>::v4& aim,
                                      cplx<R> a, cplx<R> b) {
  const R ar = SUB ? -a.re : a.re;
  const R ai = (SUB != CA) ? -a.im : a.im;
  are = Mf<R>::op(ar, b.re, are);
  are = Mf<R>::op(-ai, b.im, are);
  aim = Mf<R>::op(ar, b.im, aim);
  aim = Mf<R>::op(ai, b.re, aim);
}

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return cplx<R>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cplx<R> cinv(cplx<R> a) {
  R d = a.re * a.re + a.im * a.im;
  return cplx<R>{a.re / d, -a.im / d};
}

}  // namespace rr
