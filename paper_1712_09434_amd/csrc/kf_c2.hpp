// kf_c2.hpp -- the Kalman update with compensated (two-float) FP32
// arithmetic for the covariance, used where the prior is nearly diffuse.
#pragma once
#include <hip/hip_runtime.h>

#include "kf_device.hpp"

namespace tpcca {

// A value hi + lo held in two floats (|lo| <= half an ulp of hi), combined by
// the error-free transformations of a sum (Knuth) and of a product (one
// fused multiply-add); every step is FP32 arithmetic.  Used for the
// covariance update of the first Kalman updates of a refit, where the prior
// is nearly diffuse and C - K H C cancels most of the digits of C.
struct F2 {
  float hi, lo;
};
__host__ __device__ __forceinline__ F2 two_sum(float a, float b) {
  const float s = a + b;
  const float bb = s - a;
  return F2{s, (a - (s - bb)) + (b - bb)};
}
__host__ __device__ __forceinline__ F2 quick_two_sum(float a, float b) {   // |a| >= |b| or a == 0
  const float s = a + b;
  return F2{s, b - (s - a)};
}
__host__ __device__ __forceinline__ F2 f2_add(F2 a, F2 b) {
  F2 s = two_sum(a.hi, b.hi);
  const F2 t = two_sum(a.lo, b.lo);
  s = quick_two_sum(s.hi, s.lo + t.hi);
  return quick_two_sum(s.hi, s.lo + t.lo);
}
__host__ __device__ __forceinline__ F2 f2_neg(F2 a) { return F2{-a.hi, -a.lo}; }
__host__ __device__ __forceinline__ F2 f2_mul(F2 a, F2 b) {
  const float p = a.hi * b.hi;
  const float e = fmaf(a.hi, b.hi, -p);
  return quick_two_sum(p, fmaf(a.hi, b.lo, fmaf(a.lo, b.hi, e)));
}
__host__ __device__ __forceinline__ F2 f2_mul(F2 a, float b) {
  const float p = a.hi * b;
  const float e = fmaf(a.hi, b, -p);
  return quick_two_sum(p, fmaf(a.lo, b, e));
}
// 1 / a: the FP32 reciprocal refined by one Newton step on the two-float
// residual 1 - a q.
__host__ __device__ __forceinline__ F2 f2_inv(F2 a) {
  const float q = 1.0f / a.hi;
  const F2 r = f2_add(F2{1.0f, 0.0f}, f2_neg(f2_mul(a, q)));
  return quick_two_sum(q, (r.hi * q));
}

// The Kalman update of update() (same measurement model and expression
// structure), with S, its inverse, the gain and C - K H C in two-float
// arithmetic, each covariance entry rounded once to FP32 at the end; the
// state and chi2 take the rounded gain and inverse.
__host__ __device__ __forceinline__ void update_c2(float p[5], float C[15], float my, float mz, const Model& m,
                                                   float& chi2) {
  const float r0 = my - p[0];
  const float r1 = mz - p[1];
  const F2 S00 = two_sum(C[0], m.vy);
  const F2 S01 = F2{C[1], 0.0f};
  const F2 S11 = two_sum(C[5], m.vz);
  const F2 det = f2_add(f2_mul(S00, S11), f2_neg(f2_mul(S01, S01)));
  const F2 idet = f2_inv(det);
  const F2 I00 = f2_mul(S11, idet);
  const F2 I01 = f2_neg(f2_mul(S01, idet));
  const F2 I11 = f2_mul(S00, idet);
  float row0[5], row1[5];
  F2 K0[5], K1[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) { row0[j] = C[sym(0, j)]; row1[j] = C[sym(1, j)]; }
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    K0[i] = f2_add(f2_mul(I00, row0[i]), f2_mul(I01, row1[i]));
    K1[i] = f2_add(f2_mul(I01, row0[i]), f2_mul(I11, row1[i]));
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) p[i] = p[i] + fmaf(K1[i].hi, r1, K0[i].hi * r0);
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = i; j < 5; ++j) {
      const F2 kr = f2_add(f2_mul(K0[i], row0[j]), f2_mul(K1[i], row1[j]));
      const F2 cn = f2_add(F2{C[sym(i, j)], 0.0f}, f2_neg(kr));
      C[sym(i, j)] = cn.hi + cn.lo;
    }
  chi2 = chi2 + fmaf(r1, fmaf(I11.hi, r1, I01.hi * r0), r0 * fmaf(I01.hi, r1, I00.hi * r0));
}

}  // namespace tpcca
