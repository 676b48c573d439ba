// tpcca_calib.hip -- chi2(theta) of fixed hit lists and its gradient on gfx950.
//
// Paper, Sec. "Approach for online calibration" and Sec. "Overview of HLT
// online calibration": the calibration runs on default-transformed clusters,
// joined to the tracks by the unchanged cluster index, and feeds a new
// transformation map back to tracking.  Here the map is a correction C_theta
// (per-sector drift-velocity scale and time offset, an 8x8 cubic B-spline
// radial displacement map per sector) and the feedback becomes gradient
// descent on the total Kalman-refit chi2 of a frozen track set:
//   1. calibrate the clusters of every hit (FP32);
//   2. one lane per track: forward Kalman refit (outermost hit first, q/pT
//      prior, then the primary vertex as a measured point and an external
//      tan(lambda)), checkpointing the state every K steps and keeping the
//      last segment's and the vertex steps' states; then a hand-written
//      reverse sweep that recomputes each earlier segment from its
//      checkpoint and propagates adjoints through every update and transport
//      (second derivatives of the transport by 3-direction dual numbers);
//   3. per-track FP32 partial derivatives of the 66 parameters of its sector;
//   4. FP64 reduction over tracks in a fixed order (no atomics on floats).
#include <algorithm>

#include "calib_internal.hpp"
#include "kf_c2.hpp"

namespace tpcca {
namespace {

constexpr int TB = 256;

// ------------------------------------------------------------ dual numbers
struct D3 {
  float v, d0, d1, d2;
};
__host__ __device__ __forceinline__ D3 operator+(D3 a, D3 b) { return D3{a.v + b.v, a.d0 + b.d0, a.d1 + b.d1, a.d2 + b.d2}; }
__host__ __device__ __forceinline__ D3 operator-(D3 a, D3 b) { return D3{a.v - b.v, a.d0 - b.d0, a.d1 - b.d1, a.d2 - b.d2}; }
__host__ __device__ __forceinline__ D3 operator-(D3 a) { return D3{-a.v, -a.d0, -a.d1, -a.d2}; }
__host__ __device__ __forceinline__ D3 operator*(D3 a, D3 b) {
  return D3{a.v * b.v, a.d0 * b.v + a.v * b.d0, a.d1 * b.v + a.v * b.d1, a.d2 * b.v + a.v * b.d2};
}
__host__ __device__ __forceinline__ D3 operator*(D3 a, float b) { return D3{a.v * b, a.d0 * b, a.d1 * b, a.d2 * b}; }
__host__ __device__ __forceinline__ D3 operator*(float b, D3 a) { return D3{b * a.v, b * a.d0, b * a.d1, b * a.d2}; }
__host__ __device__ __forceinline__ D3 operator+(D3 a, float b) { return D3{a.v + b, a.d0, a.d1, a.d2}; }
__host__ __device__ __forceinline__ D3 operator+(float b, D3 a) { return D3{b + a.v, a.d0, a.d1, a.d2}; }
__host__ __device__ __forceinline__ D3 operator-(float b, D3 a) { return D3{b - a.v, -a.d0, -a.d1, -a.d2}; }
// The value and the three derivative parts share one reciprocal of the
// denominator (each within an ulp of its own quotient; these duals feed
// the adjoint only, never a state or a decision).
__host__ __device__ __forceinline__ D3 operator/(D3 a, D3 b) {
  const float r = 1.0f / b.v;
  const float q = a.v * r;
  return D3{q, (a.d0 - q * b.d0) * r, (a.d1 - q * b.d1) * r, (a.d2 - q * b.d2) * r};
}
// Square root of a dual: the hardware root and reciprocal root on the
// device (each within an ulp; these duals feed the adjoint only), the
// library root and a division on the host.
__host__ __device__ __forceinline__ D3 dsqrt(D3 a) {
#if defined(__HIP_DEVICE_COMPILE__)
  const float s = __builtin_amdgcn_sqrtf(a.v);
  const float h = 0.5f * __builtin_amdgcn_rsqf(a.v);
#else
  const float s = sqrtf(a.v);
  const float h = 0.5f / s;
#endif
  return D3{s, a.d0 * h, a.d1 * h, a.d2 * h};
}
// Reciprocal of a dual, for a denominator shared by several quotients.
__host__ __device__ __forceinline__ D3 dinv(D3 b) {
  const float r = 1.0f / b.v;
  const float m = -(r * r);
  return D3{r, m * b.d0, m * b.d1, m * b.d2};
}

// The transport's scalar chain (the tracking transport's expressions, its
// quotients by shared reciprocals) in dual numbers over (s0, k, dx): the chord rise dy, the path l and the
// Jacobian entries a = d dy/d s0, b = d dy/d k, ls = d l/d s0,
// lk = d l/d k, each with its derivatives along (s0, k, dx).
struct TDer { D3 dy, l, a, b, ls, lk; };
__host__ __device__ __forceinline__ TDer transport_duals(float s0v, float kv, float dxv, float kfac) {
  const float A1 = 1.0f / 6.0f, A2 = 3.0f / 40.0f, A3 = 5.0f / 112.0f, A4 = 35.0f / 1152.0f;
  const float B1 = 1.0f / 3.0f, B2 = 3.0f / 10.0f, B3 = 15.0f / 56.0f, B4 = 35.0f / 144.0f;
  const D3 s0{s0v, 1.f, 0.f, 0.f}, k{kv, 0.f, 1.f, 0.f}, dx{dxv, 0.f, 0.f, 1.f};
  const D3 kap = kfac * k;
  const D3 f = kfac * dx;
  TDer r;
  const D3 s1 = s0 + kap * dx;
  const D3 c0 = dsqrt(1.0f - s0 * s0);
  const D3 c1 = dsqrt(1.0f - s1 * s1);
  const D3 ss = s0 + s1, cc = c0 + c1;
  const D3 icc = dinv(cc);
  const D3 tn = ss * icc;
  r.dy = dx * tn;
  D3 d = dsqrt(dx * dx + r.dy * r.dy);
  if (dxv < 0.0f) d = -d;
  const D3 u = (kap * d) * 0.5f;
  const D3 u2 = u * u;
  const D3 g = 1.0f + u2 * (A1 + u2 * (A2 + u2 * (A3 + u2 * A4)));
  const D3 gp = u * (B1 + u2 * (B2 + u2 * (B3 + u2 * B4)));
  r.l = d * g;
  const D3 t0 = s0 / c0, t1 = s1 / c1;
  const D3 dtn_ds = (2.0f + tn * (t0 + t1)) * icc;
  const D3 dtn_dk = (f * (1.0f + tn * t1)) * icc;
  r.a = dx * dtn_ds;
  r.b = dx * dtn_dk;
  const D3 id = dinv(d);
  const D3 dd_ds = (r.dy * r.a) * id;
  const D3 dd_dk = (r.dy * r.b) * id;
  const D3 du_ds = (kap * dd_ds) * 0.5f;
  const D3 du_dk = (kfac * d + kap * dd_dk) * 0.5f;
  r.ls = dd_ds * g + (d * gp) * du_ds;
  r.lk = dd_dk * g + (d * gp) * du_dk;
  return r;
}

// ---------------------------------------------------------- small matrices
__host__ __device__ __forceinline__ void unpack(const float c[15], float M[5][5]) {
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) M[i][j] = c[sym(i, j)];
}

// Adjoint of the transport step x -> x + dx at pre-step state (P, C).
// In: gP = d chi2/d P', G = d chi2/d C' (symmetric, packed).  Out: gP, G
// replaced by the adjoints of (P, C); returns d chi2/d dx.
__host__ __device__ float transport_adjoint(const float P[5], const float Cp[15], float dx, float kfac,
                                   float gP[5], float G[15]) {
  const TDer T = transport_duals(P[2], P[4], dx, kfac);
  const float t = P[3];
  const float kap = kfac * P[4];
  float F[5][5] = {};
#pragma unroll
  for (int i = 0; i < 5; ++i) F[i][i] = 1.0f;
  F[0][2] = T.a.v; F[0][4] = T.b.v;
  F[1][2] = t * T.ls.v; F[1][3] = T.l.v; F[1][4] = t * T.lk.v;
  F[2][4] = kfac * dx;
  float Cm[5][5], Gm[5][5];
  unpack(Cp, Cm);
  unpack(G, Gm);
  // M = F C, N = G M; dF = 2 N (only the non-constant entries are needed)
  float M[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      float s = 0.f;
#pragma unroll
      for (int k = 0; k < 5; ++k) s += F[i][k] * Cm[k][j];
      M[i][j] = s;
    }
  auto N = [&](int i, int j) {
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 5; ++k) s += Gm[i][k] * M[k][j];
    return 2.0f * s;
  };
  const float dF02 = N(0, 2), dF04 = N(0, 4), dF12 = N(1, 2), dF13 = N(1, 3), dF14 = N(1, 4), dF24 = N(2, 4);
  // new G = F^T G F
  float GF[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      float s = 0.f;
#pragma unroll
      for (int k = 0; k < 5; ++k) s += Gm[i][k] * F[k][j];
      GF[i][j] = s;
    }
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = i; j < 5; ++j) {
      float s = 0.f;
#pragma unroll
      for (int k = 0; k < 5; ++k) s += F[k][i] * GF[k][j];
      G[sym(i, j)] = s;
    }
  // state adjoint: F^T g, plus the dependence of F on (s0, t, k) and dx
  float ng[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 5; ++i) s += F[i][j] * gP[i];
    ng[j] = s;
  }
  ng[2] += dF02 * T.a.d0 + dF04 * T.b.d0 + dF12 * t * T.ls.d0 + dF13 * T.l.d0 + dF14 * t * T.lk.d0;
  ng[4] += dF02 * T.a.d1 + dF04 * T.b.d1 + dF12 * t * T.ls.d1 + dF13 * T.l.d1 + dF14 * t * T.lk.d1;
  ng[3] += dF12 * T.ls.v + dF14 * T.lk.v;
  float gdx = dF02 * T.a.d2 + dF04 * T.b.d2 + dF12 * t * T.ls.d2 + dF13 * T.l.d2 + dF14 * t * T.lk.d2 +
              dF24 * kfac;
  gdx += gP[0] * T.dy.d2 + gP[1] * t * T.l.d2 + gP[2] * kap;
#pragma unroll
  for (int i = 0; i < 5; ++i) gP[i] = ng[i];
  return gdx;
}

// Adjoint of the (y, z) update at pre-update state (P, C) with measurement m.
// Adds d chi2/d m to gm[2] and replaces (gP, G) by the adjoints of (P, C).
__host__ __device__ void update_adjoint(const float P[5], const float Cp[15], float my, float mz, float vy,
                               float vz, float gP[5], float G[15], float gm[2]) {
  const float r0 = my - P[0], r1 = mz - P[1];
  const float S00 = Cp[0] + vy, S01 = Cp[1], S11 = Cp[5] + vz;
  const float det = S00 * S11 - S01 * S01;
  const float idet = 1.0f / det;
  const float W00 = S11 * idet, W01 = -S01 * idet, W11 = S00 * idet;
  float K[5][2];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const float c0 = Cp[sym(i, 0)], c1 = Cp[sym(i, 1)];
    K[i][0] = c0 * W00 + c1 * W01;
    K[i][1] = c0 * W01 + c1 * W11;
  }
  const float Wr0 = W00 * r0 + W01 * r1, Wr1 = W01 * r0 + W11 * r1;
  float Ktg0 = 0.f, Ktg1 = 0.f;
#pragma unroll
  for (int i = 0; i < 5; ++i) { Ktg0 += K[i][0] * gP[i]; Ktg1 += K[i][1] * gP[i]; }
  const float br0 = 2.0f * Wr0 + Ktg0, br1 = 2.0f * Wr1 + Ktg1;
  float Gm[5][5];
  unpack(G, Gm);
  float GK[5][2];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    float a = 0.f, b = 0.f;
#pragma unroll
    for (int k = 0; k < 5; ++k) { a += Gm[i][k] * K[k][0]; b += Gm[i][k] * K[k][1]; }
    GK[i][0] = a; GK[i][1] = b;
  }
  // bar S = -Wr Wr^T - sym(Ktg Wr^T) + K^T G K
  float KGK00 = 0.f, KGK01 = 0.f, KGK11 = 0.f;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    KGK00 += K[k][0] * GK[k][0];
    KGK01 += K[k][0] * GK[k][1];
    KGK11 += K[k][1] * GK[k][1];
  }
  const float bS00 = -Wr0 * Wr0 - Ktg0 * Wr0 + KGK00;
  const float bS11 = -Wr1 * Wr1 - Ktg1 * Wr1 + KGK11;
  const float bS01 = -Wr0 * Wr1 - 0.5f * (Ktg0 * Wr1 + Ktg1 * Wr0) + KGK01;
  // bar C = G - G K H - H^T K^T G + sym(g v^T) + H^T bar S H,  v = (Wr0, Wr1, 0, 0, 0)
  const float v[5] = {Wr0, Wr1, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = i; j < 5; ++j) {
      float s = Gm[i][j];
      if (j < 2) s -= GK[i][j];
      if (i < 2) s -= GK[j][i];
      s += 0.5f * (gP[i] * v[j] + v[i] * gP[j]);
      if (i < 2 && j < 2) s += (i == 0 && j == 0) ? bS00 : (i == 1 && j == 1) ? bS11 : bS01;
      G[sym(i, j)] = s;
    }
  gm[0] += br0;
  gm[1] += br1;
  gP[0] -= br0;
  gP[1] -= br1;
}

// Adjoint of a scalar update of component q (measurement constant).
__host__ __device__ void update1_adjoint(const float P[5], const float Cp[15], int q, float m, float var,
                                float gP[5], float G[15]) {
  const float S = Cp[sym(q, q)] + var;
  const float W = 1.0f / S;
  const float r = m - P[q];
  float K[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) K[i] = Cp[sym(i, q)] * W;
  const float Wr = W * r;
  float Ktg = 0.f;
#pragma unroll
  for (int i = 0; i < 5; ++i) Ktg += K[i] * gP[i];
  const float br = 2.0f * Wr + Ktg;
  float Gm[5][5];
  unpack(G, Gm);
  float GK[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    float a = 0.f;
#pragma unroll
    for (int k = 0; k < 5; ++k) a += Gm[i][k] * K[k];
    GK[i] = a;
  }
  float KGK = 0.f;
#pragma unroll
  for (int k = 0; k < 5; ++k) KGK += K[k] * GK[k];
  const float bS = -Wr * Wr - Ktg * Wr + KGK;
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = i; j < 5; ++j) {
      float s = Gm[i][j];
      if (j == q) s -= GK[i];
      if (i == q) s -= GK[j];
      const float vi = i == q ? Wr : 0.f, vj = j == q ? Wr : 0.f;
      s += 0.5f * (gP[i] * vj + vi * gP[j]);
      if (i == q && j == q) s += bS;
      G[sym(i, j)] = s;
    }
  gP[q] -= br;
}

// Scalar update of component q (forward).
__host__ __device__ __forceinline__ void update1(float p[5], float C[15], int q, float m, float var, float& chi2) {
  const float S = C[sym(q, q)] + var;
  float row[5], K[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) row[j] = C[sym(q, j)];
  const float r = m - p[q];
#pragma unroll
  for (int i = 0; i < 5; ++i) K[i] = row[i] / S;
#pragma unroll
  for (int i = 0; i < 5; ++i) p[i] = p[i] + K[i] * r;
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = i; j < 5; ++j) C[sym(i, j)] = C[sym(i, j)] - K[i] * row[j];
  chi2 = chi2 + (r * r) / S;
}

__host__ __device__ __forceinline__ void save(float* dst, const float p[5], const float C[15]) {
#pragma unroll
  for (int i = 0; i < 5; ++i) dst[i] = p[i];
#pragma unroll
  for (int i = 0; i < 15; ++i) dst[5 + i] = C[i];
}
__host__ __device__ __forceinline__ void load(const float* src, float p[5], float C[15]) {
#pragma unroll
  for (int i = 0; i < 5; ++i) p[i] = src[i];
#pragma unroll
  for (int i = 0; i < 15; ++i) C[i] = src[5 + i];
}

// ------------------------------------------------------- 1. calibrate hits
__host__ __device__ inline void calib_hit(const CalWs& c, int64_t j) {
  const uint32_t id = c.hit_id[j];
  c.gx[j] = 0.f; c.gy[j] = 0.f; c.gz[j] = 0.f; c.gpt[j] = 0.f;
  if ((int64_t)id >= c.NC || c.csec[id] >= c.S) {
#ifdef __HIP_DEVICE_COMPILE__
    atomicOr(c.err, 1u);
#else
    *c.err |= 1u;
#endif
    c.hx[j] = c.hy[j] = c.hz[j] = 0.f;
    c.bva[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    c.bvb[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    c.bsp[j] = 0;
    c.dzt[j] = 0.f;
    return;
  }
  const int s = c.csec[id];
  const float x = c.cx[id], y = c.cy[id], z = c.cz[id];
  const Corrected k = correct_cluster(c.geo, c.dl[s], c.tau[s], c.map + s * 64, s, x, y, z);
  c.hz[j] = k.z;
  c.dzt[j] = k.drift;
  c.bva[j] = make_float4(k.Na[0], k.Na[1], k.Na[2], k.Na[3]);
  c.bvb[j] = make_float4(k.Nb[0], k.Nb[1], k.Nb[2], k.Nb[3]);
  c.bsp[j] = k.fa | (k.fb << 8) | (1 << 16);
  c.hx[j] = k.x;
  c.hy[j] = y;
}

__global__ __launch_bounds__(TB) void k_cal_hits(CalWs c) {
  for (int64_t j = (int64_t)blockIdx.x * TB + threadIdx.x; j < c.H; j += (int64_t)gridDim.x * TB) calib_hit(c, j);
}

// ------------------------------------------- 2. forward + reverse per track
#ifdef __HIP_DEVICE_COMPILE__
#define SET_ERR(c, v) atomicOr((c).err, (v))
#else
#define SET_ERR(c, v) (*(c).err |= (v))
#endif

// Forward refit with checkpoints, then the reverse sweep, for track t.
__host__ __device__ inline void adjoint_track(const CalWs& c, int64_t t) {
  const int32_t b0 = c.hit_off[t];
  const int nh = c.hit_off[t + 1] - b0;
  float* part = c.part + t * kPart;
  c.tflag[t] = 0;
  c.tndf[t] = 0;
  part[66] = 0.f;
  if (b0 < 0 || nh < 0 || nh > c.R || (int64_t)b0 + nh > c.H) { SET_ERR(c, 2u); return; }
  if (nh < 3) return;
  // k-th processed hit (outermost first) is hit index jk(k)
  auto jk = [&](int k) { return (int64_t)b0 + nh - 1 - k; };
  const Model& m = c.m;
  float p[5], C[15];
  float sdir, tdir;
  const int64_t j0 = jk(0), j2 = jk(2);
  chord_dir(c.hx[j2], c.hy[j2], c.hz[j2], c.hx[j0], c.hy[j0], c.hz[j0], sdir, tdir);
  p[0] = c.hy[j0]; p[1] = c.hz[j0]; p[2] = sdir; p[3] = tdir; p[4] = c.k_prior[t];
  init_cov(C, m.vy, m.vz);
  if (!(fabsf(sdir) < m.sin_max)) return;
  float* ck = c.ckpt + t * (int64_t)c.nck * 20;
  float* sg = c.seg + t * (int64_t)c.nseg * 20;
  // a hit step's slot holds its state before and after the transport, so
  // the reverse sweep takes the transported state as kept, not recomputed
  float* tl = sg + (int64_t)c.K * 40;   // the steps to the vertex
  float chi2 = 0.f;
  bool ok = true;
  float xc = c.hx[j0];
  // the reverse sweep starts with the last segment of steps: its pre-step
  // states are kept here, so that segment is not recomputed (with K >= the
  // step count there is one segment and no recomputation at all)
  const int k1_last = 1 + ((nh - 2) / c.K) * c.K;
  // each step's hit is loaded one step ahead (the last step reloads its own)
  float nx = c.hx[jk(1)], ny = c.hy[jk(1)], nz = c.hz[jk(1)];
  for (int k = 1; k < nh; ++k) {
    if ((k - 1) % c.K == 0) save(ck + ((k - 1) / c.K) * 20, p, C);
    if (k >= k1_last) save(sg + (k - k1_last) * 40, p, C);
    const float hx = nx, hy = ny, hz = nz;
    const int64_t jn = jk(k + 1 < nh ? k + 1 : k);
    nx = c.hx[jn]; ny = c.hy[jn]; nz = c.hz[jn];
    if (!transport(p, C, xc, hx, m)) { ok = false; break; }
    if (k >= k1_last) save(sg + (k - k1_last) * 40 + 20, p, C);
    if (k <= kFirstC2) update_c2(p, C, hy, hz, m, chi2);
    else update(p, C, hy, hz, m, chi2);
    xc = hx;
  }
  if (!ok) return;
  // vertex and external tan(lambda)
  const bool uv = c.use_vertex && c.use_vertex[t];
  const bool ue = uv && c.ext_tgl;
  int flag = 1;
  int nsub = 0;
  const float x_last = xc;
  if (uv) {
    nsub = (int)ceilf(x_last / 10.0f);
    bool vok = nsub <= kTail - 2 && nsub >= 1;
    float q[5], Q[15];
#pragma unroll
    for (int i = 0; i < 5; ++i) q[i] = p[i];
#pragma unroll
    for (int i = 0; i < 15; ++i) Q[i] = C[i];
    // each pre-step state of the tail is kept for the reverse sweep
    float xv = x_last;
    for (int s = 0; vok && s < nsub; ++s) {
      save(tl + s * 20, q, Q);
      const float xt = 10.0f * (float)(nsub - 1 - s);
      if (!transport(q, Q, xv, xt, m)) { vok = false; break; }
      xv = xt;
    }
    if (vok) {
      save(tl + nsub * 20, q, Q);                  // before the vertex update
      float c2 = chi2;
      update(q, Q, 0.0f, 0.0f, Model{m.kfac, m.sin_max, c.sv2, c.sv2}, c2);
      if (ue) update1(q, Q, 3, c.ext_tgl[t], c.st2, c2);
      chi2 = c2;
      flag = 2;
    }
  }
  c.tflag[t] = flag;
  c.tndf[t] = 2 * nh - 5 + (flag == 2 ? 2 + (ue ? 1 : 0) : 0);
  part[66] = chi2;
  // ---------------------------------------------------------- reverse
  float gP[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, G[15];
#pragma unroll
  for (int i = 0; i < 15; ++i) G[i] = 0.f;
  if (flag == 2) {
    // the tail's states were kept by the forward pass
    float q[5], Q[15];
    load(tl + nsub * 20, q, Q);
    if (ue) {
      float dummy = 0.f;
      update(q, Q, 0.0f, 0.0f, Model{m.kfac, m.sin_max, c.sv2, c.sv2}, dummy);
      update1_adjoint(q, Q, 3, c.ext_tgl[t], c.st2, gP, G);
      load(tl + nsub * 20, q, Q);
    }
    float gm[2] = {0.f, 0.f};
    update_adjoint(q, Q, 0.0f, 0.0f, c.sv2, c.sv2, gP, G, gm);
    for (int s = nsub - 1; s >= 0; --s) {
      load(tl + s * 20, q, Q);
      const float xf = s == 0 ? x_last : 10.0f * (float)(nsub - s);
      const float xt = 10.0f * (float)(nsub - 1 - s);
      const float gdx = transport_adjoint(q, Q, xt - xf, m.kfac, gP, G);
      if (s == 0) c.gpt[jk(nh - 1)] -= gdx;
    }
  }
  // hit steps, segment by segment from the last
  const int nsteps = nh - 1;
  for (int sgi = (nsteps - 1) / c.K; sgi >= 0; --sgi) {
    const int k1 = 1 + sgi * c.K;
    const int k2 = min(nsteps, k1 + c.K - 1);
    float q[5], Q[15];
    load(ck + sgi * 20, q, Q);
    float xv = c.hx[jk(k1 - 1)];
    float dummy = 0.f;
    float nx = c.hx[jk(k1)], ny = c.hy[jk(k1)], nz = c.hz[jk(k1)];
    for (int k = k1; k <= k2 && k1 != k1_last; ++k) {
      save(sg + (k - k1) * 40, q, Q);
      const float hx = nx, hy = ny, hz = nz;
      const int64_t jn = jk(k < k2 ? k + 1 : k);
      nx = c.hx[jn]; ny = c.hy[jn]; nz = c.hz[jn];
      transport(q, Q, xv, hx, m);
      save(sg + (k - k1) * 40 + 20, q, Q);
      if (k <= kFirstC2) update_c2(q, Q, hy, hz, m, dummy);
      else update(q, Q, hy, hz, m, dummy);
      xv = hx;
    }
    // the hit values of the step are loaded one step ahead; gy and gz of a
    // hit are still zero (set with the calibrated hits) when its step is
    // reached, each hit ending one step, so they are written, not updated
    float xt_n = c.hx[jk(k2)], yt_n = c.hy[jk(k2)], zt_n = c.hz[jk(k2)], xf_n = c.hx[jk(k2 - 1)];
    // the saved states of the step are loaded one step ahead as well
    float a_n[5], A_n[15], b_n[5], B_n[15];
    load(sg + (k2 - k1) * 40, a_n, A_n);
    load(sg + (k2 - k1) * 40 + 20, b_n, B_n);
    for (int k = k2; k >= k1; --k) {
      const int64_t j = jk(k);
      float a[5], A[15], b[5], B[15];
#pragma unroll
      for (int i = 0; i < 5; ++i) { a[i] = a_n[i]; b[i] = b_n[i]; }
#pragma unroll
      for (int i = 0; i < 15; ++i) { A[i] = A_n[i]; B[i] = B_n[i]; }
      load(sg + (k > k1 ? k - 1 - k1 : 0) * 40, a_n, A_n);
      load(sg + (k > k1 ? k - 1 - k1 : 0) * 40 + 20, b_n, B_n);
      const float xt = xt_n, yt = yt_n, zt = zt_n, xf = xf_n;
      // the next step (k - 1) ends on hit k - 1 and starts from hit k - 2
      const int64_t jq = jk(k - 1), jr = jk(k >= 2 ? k - 2 : 0);
      xt_n = xf; yt_n = c.hy[jq]; zt_n = c.hz[jq]; xf_n = c.hx[jr];
      float gm[2] = {0.f, 0.f};
      update_adjoint(b, B, yt, zt, m.vy, m.vz, gP, G, gm);
      c.gy[j] = 0.0f + gm[0];
      c.gz[j] = 0.0f + gm[1];
      // the step's dx-derivative is kept whole (at the hit it ends on); the
      // map partials weight it by the change of the basis product between
      // its two hits, which avoids forming the difference of two large,
      // nearly equal step derivatives per hit
      c.gx[j] = transport_adjoint(a, A, xt - xf, m.kfac, gP, G);
    }
  }
  // initial state: (y, z) of the outermost hit, direction from the chord
  {
    c.gy[j0] += gP[0];
    c.gz[j0] += gP[1];
    const float dX = c.hx[j0] - c.hx[j2], dY = c.hy[j0] - c.hy[j2], dZ = c.hz[j0] - c.hz[j2];
    const float rho = sqrtf(fmaf(dX, dX, dY * dY));   // as the forward chord_dir
    const float r3 = rho * rho * rho;
    const float gs = gP[2], gt = gP[3];
    const float gdX = gs * (-dY * dX / r3) + gt * (-dZ * dX / r3);
    const float gdY = gs * (dX * dX / r3) + gt * (-dZ * dY / r3);
    const float gdZ = gt / rho;
    c.gpt[j0] += gdX; c.gpt[j2] -= gdX;
    c.gy[j0] += gdY; c.gy[j2] -= gdY;
    c.gz[j0] += gdZ; c.gz[j2] -= gdZ;
  }
}

// One lane per track, one wave per workgroup: a call has a few thousand
// tracks, so this spreads their waves over as many compute units (and their
// vector memory paths) as there are waves, rather than four to a unit.
constexpr int TA = 64;
__global__ __launch_bounds__(TA) void k_cal_adjoint(CalWs c) {
  for (int64_t t = (int64_t)blockIdx.x * TA + threadIdx.x; t < c.T; t += (int64_t)gridDim.x * TA) adjoint_track(c, t);
}

// ------------------------------------------ 3. per-track parameter partials
// One wave per track: lane l owns map coefficient (l / 8, l % 8); lanes 0
// and 1 also own the drift scale and the time offset.  Sums run over the
// track's hits in order (FP32).
__host__ __device__ inline void partials_lane(const CalWs& c, int64_t t, int l) {
  float* part = c.part + t * kPart;
  const int32_t b0 = c.hit_off[t];
  const int nh = c.hit_off[t + 1] - b0;
  float acc = 0.f, accd = 0.f;
  if (c.tflag[t] > 0) {
    const uint32_t id0 = c.hit_id[b0];
    int s = (int64_t)id0 < c.NC ? c.csec[id0] : 0;
    if (s >= c.S) s = 0;   // flagged as an error by k_cal_hits
    const float side = s < c.S / 2 ? 1.0f : -1.0f;
    const float dl = c.dl[s];
    const int a = l >> 3, b = l & 7;
    // this lane's basis product at each hit from the four non-zero values
    // of each direction stored per hit (the same floats as the full basis):
    // each lane loads its own component of the hit's two records (0 where
    // its coefficient lies outside the hit's support; such lanes load the
    // first component, all lanes then read one cache line), the hit's other
    // values are the same for every lane of the track
    const float kd = l == 0 ? -side : side * (1.0f + dl);
    // basis product at hit i+1 (the next hit outward), carried down the loop
    float w_next = 0.f;
#pragma unroll 8
    for (int i = nh - 1; i >= 0; --i) {
      const int64_t j = b0 + i;
      const int32_t sp = c.bsp[j];
      const int ka = a - (sp & 0xFF), kb = b - ((sp >> 8) & 0xFF);
      const bool ina = (unsigned)ka < 4u, inb = (unsigned)kb < 4u;
      const float xa = ((const float*)(c.bva + j))[ina ? ka : 0];
      const float xb = ((const float*)(c.bvb + j))[inb ? kb : 0];
      const float gxj = c.gx[j], gpj = c.gpt[j], gzj = c.gz[j], dz = c.dzt[j];
      const float wj = (ina ? xa : 0.0f) * (inb ? xb : 0.0f);
      // drift scale (lane 0) and time offset (lane 1), valid hits only
      const float td = l == 0 ? dz : 1.0f;
      if (l < 2 && (sp >> 16) != 0) accd += gzj * (kd * td);
      if (i < nh - 1) acc += gxj * (wj - w_next);
      acc += gpj * wj;
      w_next = wj;
    }
  }
  part[2 + l] = acc;
  if (l < 2) part[l] = accd;
  if (l == 0 && c.flag_out) c.flag_out[t] = c.tflag[t] | (nh < kMinAccurateHits ? TPCCA_TRK_SHORT : 0);
}

__global__ __launch_bounds__(64) void k_cal_partials(CalWs c) { partials_lane(c, blockIdx.x, threadIdx.x); }

// --------------------------------------------- 4. FP64 fixed-order reduction
// chunk[ch][s*66 + p] = sum over the tracks of chunk ch (ascending) in sector s
// of part[t][p]; chunk[ch][S*66] = sum of the chunk's chi2.
__global__ __launch_bounds__(TB) void k_cal_chunks(CalWs c) {
  __shared__ int s_sec[kChunk];
  // the chunk's tracks listed by sector, ascending within each, so that
  // each sum visits only its sector's tracks, in the same order as a scan
  // of the whole chunk
  __shared__ int s_list[kChunk];
  __shared__ int s_first[kMaxSectors + 1];
  __shared__ unsigned long long s_ndf;
  const int64_t t0 = (int64_t)blockIdx.x * kChunk;
  if (threadIdx.x == 0) s_ndf = 0ull;
  const int64_t nt = (c.T - t0) < kChunk ? (c.T - t0) : (int64_t)kChunk;
  for (int i = threadIdx.x; i < kChunk; i += TB) {
    int s = -1;
    if (i < nt && c.tflag[t0 + i] > 0) {
      const uint32_t id = c.hit_id[c.hit_off[t0 + i]];
      s = (int64_t)id < c.NC ? c.csec[id] : 0;
      if (s >= c.S) s = 0;   // flagged as an error by k_cal_hits
    }
    s_sec[i] = s;
  }
  __syncthreads();
  // each entry's rank among the earlier entries of its sector (broadcast
  // LDS reads), the sectors' counts, their prefix, then the lists
  for (int q = threadIdx.x; q <= c.S; q += TB) s_first[q] = 0;
  __syncthreads();
  int rank[kChunk / TB];
#pragma unroll
  for (int u = 0; u < kChunk / TB; ++u) {
    const int i = threadIdx.x + u * TB;
    const int si = s_sec[i];
    int rk = 0;
    if (si >= 0) {
      for (int k = 0; k < i; ++k) rk += s_sec[k] == si ? 1 : 0;
      atomicAdd(&s_first[si + 1], 1);
    }
    rank[u] = rk;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int q = 0; q < c.S; ++q) s_first[q + 1] += s_first[q];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kChunk / TB; ++u) {
    const int i = threadIdx.x + u * TB;
    if (s_sec[i] >= 0) s_list[s_first[s_sec[i]] + rank[u]] = i;
  }
  __syncthreads();
  const int nq = c.S * kNPar + 1;
  double* out = c.chunk + (int64_t)blockIdx.x * nq;
  // the terms are loaded kU at a time (indices clamped into the list) and
  // added one by one in list order, so the loads of a batch are in flight
  // together while the sum is the same as the plain sequential loop
  constexpr int kU = 16;
  for (int q = threadIdx.x; q < nq; q += TB) {
    double acc = 0.0;
    if (q == c.S * kNPar) {
      for (int i = 0; i < nt; i += kU) {
        float v[kU];
        bool ok[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int iu = i + u < nt ? i + u : i;
          ok[u] = i + u < nt && s_sec[iu] >= 0;
          v[u] = c.part[(t0 + iu) * kPart + 66];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) acc = ok[u] ? acc + (double)v[u] : acc;
      }
    } else {
      const int s = q / kNPar, p = q % kNPar;
      const int k0 = s_first[s], k1 = s_first[s + 1];
      for (int k = k0; k < k1; k += kU) {
        float v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) v[u] = c.part[(t0 + s_list[k + u < k1 ? k + u : k]) * kPart + p];
#pragma unroll
        for (int u = 0; u < kU; ++u) acc = k + u < k1 ? acc + (double)v[u] : acc;
      }
    }
    out[q] = acc;
  }
  // ndf: the chunk's integer sum first, then one global atomic per chunk
  unsigned long long nd = 0ull;
  for (int i = threadIdx.x; i < nt; i += TB)
    if (c.tflag[t0 + i] > 0) nd += (unsigned long long)c.tndf[t0 + i];
  if (nd) atomicAdd(&s_ndf, nd);
  __syncthreads();
  if (threadIdx.x == 0 && s_ndf) atomicAdd(c.ndf_sum, s_ndf);
}

__global__ __launch_bounds__(TB) void k_cal_final(CalWs c, int64_t nchunk) {
  const int nq = c.S * kNPar + 1;
  for (int q = blockIdx.x * TB + threadIdx.x; q < nq; q += gridDim.x * TB) {
    double acc = 0.0;
    for (int64_t ch = 0; ch < nchunk; ++ch) acc += c.chunk[ch * nq + q];
    c.out[q] = acc;
    if (c.g_dl && q < nq - 1) {
      const int s = q / kNPar, p = q - s * kNPar;
      if (p == 0) c.g_dl[s] = acc;
      else if (p == 1) c.g_tau[s] = acc;
      else c.g_map[(int64_t)s * 64 + (p - 2)] = acc;
    }
  }
}

__global__ void k_cal_zero(CalWs c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) { *c.ndf_sum = 0ull; *c.err = 0u; }
}

}  // namespace

hipError_t run_calib(const CalWs& c, hipStream_t st) {
  // every array the kernels touch must be set before anything is launched
  const void* need[] = {c.hit_off, c.hit_id, c.k_prior, c.cx, c.cy, c.cz, c.csec, c.dl, c.tau, c.map,
                        c.hx, c.hy, c.hz, c.gx, c.gy, c.gz, c.gpt, c.bva, c.bvb, c.bsp, c.dzt,
                        c.part, c.tflag, c.tndf, c.ckpt,
                        c.seg, c.chunk, c.out, c.ndf_sum, c.err};
  for (const void* p : need)
    if (!p) return hipErrorInvalidValue;
  if (c.K < 1 || c.nseg < 2 * c.K + kTail || c.nck < (c.R - 1 + c.K - 1) / c.K + 1) return hipErrorInvalidValue;
  k_cal_zero<<<1, 64, 0, st>>>(c);
  const unsigned bh = (unsigned)std::min<int64_t>(std::max<int64_t>((c.H + TB - 1) / TB, 1), 65536);
  k_cal_hits<<<bh, TB, 0, st>>>(c);
  const unsigned bt = (unsigned)std::min<int64_t>(std::max<int64_t>((c.T + TA - 1) / TA, 1), 65536);
  k_cal_adjoint<<<bt, TA, 0, st>>>(c);
  if (c.T > 0) k_cal_partials<<<dim3((unsigned)c.T), 64, 0, st>>>(c);
  const int64_t nchunk = (c.T + kChunk - 1) / kChunk;
  if (nchunk > 0) k_cal_chunks<<<dim3((unsigned)nchunk), TB, 0, st>>>(c);
  k_cal_final<<<dim3((unsigned)((c.S * kNPar + 1 + TB - 1) / TB)), TB, 0, st>>>(c, nchunk);
  return hipGetLastError();
}

}  // namespace tpcca
