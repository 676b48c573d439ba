// kf_device.hpp -- FP32 helix transport and Kalman update for gfx950.
//
// Track model (paper, Sec. "Track reconstruction in the TPC": Kalman-filter
// fitting and following of cellular-automaton seeds): state
// p = (y, z, s = sin phi, t = tan lambda, k = q/pT) on planes x = const of
// a sector frame, uniform solenoid, no material.  Every expression below is
// evaluated in exactly this order: the library is built with
// -ffp-contract=off and correctly rounded FP32 division and square root, and
// fused multiply-adds (one rounding) appear only where fmaf is written, so
// the integer decisions taken from these values (which cluster, which row,
// stop or go) are reproducible on any IEEE implementation that evaluates
// the same expressions.
#pragma once
#include <hip/hip_runtime.h>

namespace tpcca {

struct Model {
  float kfac;     // signed curvature per unit q/pT: -c Bz
  float sin_max;
  float vy, vz;   // cluster variances
};

// Packed upper-triangle index of a symmetric 5x5 matrix.
// (Not recursive, so that unrolled loops fold it to a constant: a swap by
// recursion was left as a runtime loop with indexed register reads.)
__host__ __device__ constexpr int sym_upper(int i, int j) {
  return i == 0 ? j : i == 1 ? 4 + j : i == 2 ? 7 + j : i == 3 ? 9 + j : 14;
}
__host__ __device__ constexpr int sym(int i, int j) {
  return i <= j ? sym_upper(i, j) : sym_upper(j, i);
}

// Correctly rounded square root of a finite x that is 0, negative (NaN
// result) or >= 2^-96: the hardware root is within one ulp, and the signs of
// the fused residuals x - s' s of its two neighbours s' pick the rounded
// result.  This is the standard correction without the rescaling of tiny
// inputs, which the callers' arguments never need: 1 - s^2 (one fused
// rounding) for a float s is <= 0 or >= 2^-23 - 2^-48.  (The host build of
// this header, used to run the calibration code on the CPU, takes the
// library square root, which is correctly rounded too.)
__host__ __device__ __forceinline__ float sqrt_rn_normal(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const float s = __builtin_amdgcn_sqrtf(x);
  const float sm = __uint_as_float(__float_as_uint(s) - 1u);
  const float sp = __uint_as_float(__float_as_uint(s) + 1u);
  float r = fmaf(-sm, s, x) <= 0.0f ? sm : s;
  r = fmaf(-sp, s, x) > 0.0f ? sp : r;
  return r;
#else
  return sqrtf(x);
#endif
}

// One step of the helix from the plane x0 to the plane x1.  The sine of the
// direction moves linearly (s1 = s0 + kap dx); the chord rises by
// dx (s0 + s1)/(c0 + c1); the transverse path is the chord (signed like dx)
// times asin(u)/u, u = kap d / 2, taken as its series through u^8; z moves
// by t times that path.  The covariance becomes F C F^T with the exact
// Jacobian F of these expressions.  Returns false, leaving p and C
// untouched, if |s1| would reach sin_max.
__host__ __device__ __forceinline__ bool transport(float p[5], float C[15], float x0, float x1,
                                          const Model& m) {
  const float dx = x1 - x0;
  if (dx == 0.0f) return true;
  const float A1 = 1.0f / 6.0f, A2 = 3.0f / 40.0f, A3 = 5.0f / 112.0f, A4 = 35.0f / 1152.0f;
  const float B1 = 1.0f / 3.0f, B2 = 3.0f / 10.0f, B3 = 15.0f / 56.0f, B4 = 35.0f / 144.0f;
  const float kap = m.kfac * p[4];
  const float s0 = p[2];
  const float f = m.kfac * dx;
  const float s1 = fmaf(kap, dx, s0);
  if (!(fabsf(s1) < m.sin_max)) return false;
  const float c0 = sqrt_rn_normal(fmaf(-s0, s0, 1.0f));
  const float c1 = sqrt_rn_normal(fmaf(-s1, s1, 1.0f));
  const float ss = s0 + s1;
  const float cc = c0 + c1;
  const float icc = 1.0f / cc;   // shared denominator: one division, then products
  const float tn = ss * icc;
  const float dy = dx * tn;
  float d = sqrtf(fmaf(dx, dx, dy * dy));
  if (dx < 0.0f) d = -d;
  const float u = (kap * d) * 0.5f;
  const float u2 = u * u;
  const float g = fmaf(u2, fmaf(u2, fmaf(u2, fmaf(u2, A4, A3), A2), A1), 1.0f);
  const float gp = u * fmaf(u2, fmaf(u2, fmaf(u2, B4, B3), B2), B1);
  const float l = d * g;
  const float i01 = 1.0f / (c0 * c1);   // the two tangents share one division
  const float t0 = (s0 * c1) * i01;
  const float t1 = (s1 * c0) * i01;
  const float dtn_ds = fmaf(tn, t0 + t1, 2.0f) * icc;
  const float dtn_dk = (f * fmaf(tn, t1, 1.0f)) * icc;
  const float a = dx * dtn_ds;
  const float b = dx * dtn_dk;
  const float id = 1.0f / d;
  const float dd_ds = (dy * a) * id;
  const float dd_dk = (dy * b) * id;
  const float du_ds = (kap * dd_ds) * 0.5f;
  const float du_dk = fmaf(m.kfac, d, kap * dd_dk) * 0.5f;
  const float dl_ds = fmaf(dd_ds, g, (d * gp) * du_ds);
  const float dl_dk = fmaf(dd_dk, g, (d * gp) * du_dk);
  const float t = p[3];
  const float c = t * dl_ds;
  const float e = t * dl_dk;
  p[0] = p[0] + dy;
  p[1] = fmaf(t, l, p[1]);
  p[2] = s1;
  const float C00 = C[0], C01 = C[1], C02 = C[2], C03 = C[3], C04 = C[4];
  const float C11 = C[5], C12 = C[6], C13 = C[7], C14 = C[8];
  const float C22 = C[9], C23 = C[10], C24 = C[11];
  const float C33 = C[12], C34 = C[13], C44 = C[14];
  const float T00 = fmaf(b, C04, fmaf(a, C02, C00));
  const float T01 = fmaf(b, C14, fmaf(a, C12, C01));
  const float T02 = fmaf(b, C24, fmaf(a, C22, C02));
  const float T03 = fmaf(b, C34, fmaf(a, C23, C03));
  const float T04 = fmaf(b, C44, fmaf(a, C24, C04));
  const float T11 = fmaf(e, C14, fmaf(l, C13, fmaf(c, C12, C11)));
  const float T12 = fmaf(e, C24, fmaf(l, C23, fmaf(c, C22, C12)));
  const float T13 = fmaf(e, C34, fmaf(l, C33, fmaf(c, C23, C13)));
  const float T14 = fmaf(e, C44, fmaf(l, C34, fmaf(c, C24, C14)));
  const float T22 = fmaf(f, C24, C22);
  const float T23 = fmaf(f, C34, C23);
  const float T24 = fmaf(f, C44, C24);
  C[0] = fmaf(b, T04, fmaf(a, T02, T00));
  C[1] = fmaf(e, T04, fmaf(l, T03, fmaf(c, T02, T01)));
  C[2] = fmaf(f, T04, T02);
  C[3] = T03;
  C[4] = T04;
  C[5] = fmaf(e, T14, fmaf(l, T13, fmaf(c, T12, T11)));
  C[6] = fmaf(f, T14, T12);
  C[7] = T13;
  C[8] = T14;
  C[9] = fmaf(f, T24, T22);
  C[10] = T23;
  C[11] = T24;
  return true;
}

// Kalman update with the cluster (my, mz): H = [I2 0], V = diag(vy, vz).
// Gain from the explicit 2x2 inverse of S = H C H^T + V; chi2 increment
// r^T S^-1 r.
__host__ __device__ __forceinline__ void update(float p[5], float C[15], float my, float mz,
                                       const Model& m, float& chi2) {
  const float r0 = my - p[0];
  const float r1 = mz - p[1];
  const float S00 = C[0] + m.vy;
  const float S01 = C[1];
  const float S11 = C[5] + m.vz;
  const float det = fmaf(S00, S11, -(S01 * S01));
  const float idet = 1.0f / det;
  const float I00 = S11 * idet;
  const float I01 = (-S01) * idet;
  const float I11 = S00 * idet;
  float row0[5], row1[5], K0[5], K1[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) { row0[j] = C[sym(0, j)]; row1[j] = C[sym(1, j)]; }
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    K0[i] = fmaf(row1[i], I01, row0[i] * I00);
    K1[i] = fmaf(row1[i], I11, row0[i] * I01);
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) p[i] = p[i] + fmaf(K1[i], r1, K0[i] * r0);
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = i; j < 5; ++j) C[sym(i, j)] = C[sym(i, j)] - fmaf(K1[i], row1[j], K0[i] * row0[j]);
  chi2 = chi2 + fmaf(r1, fmaf(I11, r1, I01 * r0), r0 * fmaf(I01, r1, I00 * r0));
}

__host__ __device__ __forceinline__ void init_cov(float C[15], float vy, float vz) {
#pragma unroll
  for (int i = 0; i < 15; ++i) C[i] = 0.0f;
  C[0] = vy;
  C[5] = vz;
  C[9] = 0.25f;
  C[12] = 0.25f;
  C[14] = 100.0f;
}

// Direction of the chord from an inner to an outer point.
__host__ __device__ __forceinline__ void chord_dir(float xi, float yi, float zi, float xo, float yo,
                                          float zo, float& s, float& t) {
  const float dX = xo - xi, dY = yo - yi, dZ = zo - zi;
  const float rho = sqrtf(fmaf(dX, dX, dY * dY));
  const float irho = 1.0f / rho;
  s = dY * irho;
  t = dZ * irho;
}

}  // namespace tpcca
