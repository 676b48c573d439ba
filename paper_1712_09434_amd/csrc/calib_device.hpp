// calib_device.hpp -- the calibration correction of one cluster in FP32,
// shared by the tracking input (binning) and the calibration gradient.
//
// Paper, Sec. "Approach for online calibration": tracking consumes
// calibration-transformed clusters; the calibration is computed from
// default-transformed ones and fed back as a new map.  The correction of a
// default-transformed cluster of sector s (side = +1 for the first half of
// the sectors, -1 otherwise; drift length L; D = L - side z the drift
// distance) by theta = (drift-velocity scale delta_s, time offset tau_s,
// 8 x 8 cubic B-spline radial map c_s) is
//   side z' = L - (1 + delta)(D - tau),   x' = x + sum_ab c_ab B_a(xh) B_b(uh),
// xh = (x - x_first)/(x_last - x_first), uh = (y/x + tan a)/(2 tan a), both
// clamped to [0, 1] and taken at the uncorrected (x, y).  In FP32 both are
// evaluated as a correction added to the coordinate, in this order:
//   z' = z + side (tau - delta (D - tau)),
//   x' = x + sum_a Na[a] (sum_b c[fa + a][fb + b] Nb[b])
// over the four non-zero basis functions of each direction (ascending
// indices, each sum from +0), so that theta = 0 leaves a cluster unchanged
// bit for bit.  The tracker's decisions are taken from these values, so the
// order of operations is part of the definition.
#pragma once
#include <hip/hip_runtime.h>

namespace tpcca {

struct CalGeo {
  int S;              // sectors
  float L;            // drift length
  float x_first;      // radial range of the map: first and last pad-row plane
  float x_span;       // x_last - x_first (FP32)
  float tan_a;        // tan of the sector half-opening angle
};

// The four non-zero clamped uniform cubic B-splines (knots
// 0,0,0,0,.2,.4,.6,.8,1,1,1,1) at u, by de Boor's triangular recursion on
// the knot span of u (clamped to [0, 1]; u = 1 takes the last span): they
// are B[first .. first + 3] = N[0 .. 3]; returns first.
__host__ __device__ __forceinline__ int bspline4(float u, float N[4]) {
  u = fminf(fmaxf(u, 0.0f), 1.0f);
  const float kn[12] = {0.f, 0.f, 0.f, 0.f, 0.2f, 0.4f, 0.6f, 0.8f, 1.f, 1.f, 1.f, 1.f};
  int span = 3;
#pragma unroll
  for (int i = 4; i <= 7; ++i) if (u >= kn[i]) span = i;
  N[0] = 1.f; N[1] = 0.f; N[2] = 0.f; N[3] = 0.f;
  float left[4], right[4];
#pragma unroll
  for (int j = 1; j <= 3; ++j) {
    left[j] = u - kn[span + 1 - j];
    right[j] = kn[span + j] - u;
    float saved = 0.f;
#pragma unroll
    for (int r = 0; r < j; ++r) {
      // the two knot differences summed here are at least 0.2 apart
      const float tmp = N[r] / (right[r + 1] + left[j - r]);
      N[r] = saved + right[r + 1] * tmp;
      saved = left[j - r] * tmp;
    }
    N[j] = saved;
  }
  return span - 3;
}

// The corrected (x', z') of a cluster of sector s (map c = the sector's 64
// coefficients), with what the gradient needs: the drift term D - tau, the
// four non-zero basis values of each direction and their first indices.
struct Corrected {
  float x, z, drift;
  float Na[4], Nb[4];
  int fa, fb;
};

__host__ __device__ __forceinline__ Corrected correct_cluster(const CalGeo& g, float delta, float tau,
                                                              const float* c, int s, float x, float y,
                                                              float z) {
  Corrected o;
  const float side = s < g.S / 2 ? 1.0f : -1.0f;
  o.drift = (g.L - side * z) - tau;
  o.z = z + side * (tau - delta * o.drift);
  o.fa = bspline4((x - g.x_first) / g.x_span, o.Na);
  o.fb = bspline4((y / x + g.tan_a) / (2.0f * g.tan_a), o.Nb);
  const float* cm = c + o.fa * 8 + o.fb;
  float acc = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float ra = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) ra += cm[i * 8 + k] * o.Nb[k];
    acc += o.Na[i] * ra;
  }
  o.x = x + acc;
  return o;
}

}  // namespace tpcca
