// tpcca_its.hip -- ITS standalone tracking on gfx950.
//
// Paper, Sec. "Fast ITS standalone tracking": the primary vertex is where
// most lines through pairs of clusters of the two innermost (pixel) layers
// converge; tracklets are pixel-cluster pairs seen under nearly the same
// angles from the vertex; a Kalman filter initialised from the vertex and
// the pair, the vertex taken as a measured point, follows each tracklet
// outward, taking on the outer layers the cluster closest to the
// extrapolation under a strict chi2 cut, multiple scattering from the
// average material of each layer; at least four clusters, never two
// consecutive layers without one; the outward state is kept and an inward
// fit gives the state at the vertex region.  Sec. "Luminous region
// estimation based on ITS tracking": tracks propagated to the beam line, a
// linear fit of the point of least distance, bi-square outlier weights.
// The library's reading of the rules and constants is in tpcca.h.
//
// Kernels (one event per call; clusters are few, tens of thousands):
// cluster preparation and per-stave counts, stave offsets, stave lists;
// pair histogram (thread per layer-0 cluster over the three layer-1 staves
// around its azimuth), peak, fixed-point mean; tracklet candidates (best of
// each layer-0 cluster in registers, best of each layer-1 cluster by a
// 64-bit atomic minimum of (score bits, id)), mutual pairs compacted in id
// order; following and inward fit (lane per tracklet); vertex fit (one
// workgroup, fixed-order FP64 reductions).
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.hpp"

struct tpcca_its_ctx {
  int device = 0;
  tpcca_its_geometry g{};
  tpcca_its_params P{};
  std::string err;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  float* tab = nullptr;          // device stave tables
};

namespace tpcca {
namespace {

constexpr int TB = 256;
constexpr int kLayers = 6;
constexpr int kStaves = 64;      // per layer, at most
constexpr int kBins = 4096;      // vertexer histogram bins, at most

// Geometry tables in device memory (FP32 values of FP64 expressions):
// stave centre cos/sin and wedge boundary cos/sin per layer.
struct ItsTab {
  float ca[kLayers][kStaves], sa[kLayers][kStaves];
  float bc[kLayers][kStaves + 1], bs[kLayers][kStaves + 1];
};

struct ItsWs {
  int64_t n, cap;
  const float* x;
  const float* y;
  const float* z;
  const int8_t* layer;
  const int16_t* stave;
  const ItsTab* tab;
  float r[kLayers], hz[kLayers], xx0[kLayers], vy[kLayers], vz[kLayers], kms[kLayers];
  int ns[kLayers];
  Model m;
  tpcca_its_params P;
  int nbins;
  // work
  float* cX;                 // [n] global position and radius (FP32)
  float* cY;
  float* cR;
  uint32_t* scount;          // [6 * 64 + 1] clusters per stave -> offsets
  uint32_t* scur;            // [6 * 64] fill cursors
  uint32_t* slist;           // [n] cluster ids by stave
  uint32_t* hist;            // [nbins]
  unsigned long long* vsum;  // [4]: pairs, pairs in the mean, fixed-point sum, error bits
  float* vzd;                // [2]: vertex z, found flag
  int32_t* vpeak;            // [1]
  unsigned long long* best0; // [n] (score bits << 32) | layer-1 id
  unsigned long long* best1; // [n] (score bits << 32) | layer-0 id
  uint32_t* tflag;           // [n + 1] mutual pair at a layer-0 cluster -> offsets
  double* vw;                // [cap] vertex-fit weights
  double* vres;              // [8]: vertex (3), sum of weights, tracks used, ok
  // outputs
  tpcca_its_tracks o;
};

__device__ __forceinline__ int sidx(int l, int k) { return l * kStaves + k; }

__device__ __forceinline__ bool valid_cluster(const ItsWs& w, int64_t i) {
  const int l = w.layer[i], k = w.stave[i];
  return l >= 0 && l < kLayers && k >= 0 && k < w.ns[l] && isfinite(w.x[i]) && isfinite(w.y[i]) &&
         isfinite(w.z[i]);
}

__global__ __launch_bounds__(TB) void k_its_prep(ItsWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i >= w.n) return;
  const int l = w.layer[i], k = w.stave[i];
  const float x = w.x[i], y = w.y[i];
  if (!valid_cluster(w, i)) {
    atomicOr(&w.vsum[3], 1ull);
    w.cX[i] = 0.0f; w.cY[i] = 0.0f; w.cR[i] = 0.0f;
    return;
  }
  const float ca = w.tab->ca[l][k], sa = w.tab->sa[l][k];
  const float X = x * ca - y * sa;
  const float Y = x * sa + y * ca;
  w.cX[i] = X;
  w.cY[i] = Y;
  w.cR[i] = sqrtf(X * X + Y * Y);
  atomicAdd(&w.scount[sidx(l, k)], 1u);
}

// stave offsets (one workgroup of 512 threads: 384 staves)
__global__ __launch_bounds__(512) void k_its_soff(ItsWs w) {
  __shared__ uint32_t s[kLayers * kStaves];
  const int t = threadIdx.x;
  if (t < kLayers * kStaves) s[t] = w.scount[t];
  __syncthreads();
  if (t == 0) {
    uint32_t acc = 0;
    for (int j = 0; j < kLayers * kStaves; ++j) {
      const uint32_t c = s[j];
      s[j] = acc;
      acc += c;
    }
    w.scount[kLayers * kStaves] = acc;
  }
  __syncthreads();
  if (t < kLayers * kStaves) { w.scount[t] = s[t]; w.scur[t] = s[t]; }
}

__global__ __launch_bounds__(TB) void k_its_fill(ItsWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i >= w.n) return;
  if (!valid_cluster(w, i)) return;
  w.slist[atomicAdd(&w.scur[sidx(w.layer[i], w.stave[i])], 1u)] = (uint32_t)i;
}

// The layer-1 stave whose wedge holds the direction (X, Y), searched from a
// stave of the same angular position on layer lf.
__device__ __forceinline__ int wedge_of(const ItsWs& w, int l, int lf, int kf, float X, float Y) {
  const int ns = w.ns[l];
  int k = ((2 * kf + 1) * ns) / (2 * w.ns[lf]);
  for (int it = 0; it < 4; ++it) {
    const bool lo = w.tab->bc[l][k] * Y - w.tab->bs[l][k] * X >= 0.0f;
    const bool hi = w.tab->bc[l][k + 1] * Y - w.tab->bs[l][k + 1] * X < 0.0f;
    if (lo && hi) break;
    k = lo ? (k + 1) % ns : (k + ns - 1) % ns;
  }
  return k;
}

// Visits every layer-1 cluster of the three staves around a layer-0
// cluster's azimuth (every pair within a window narrower than a stave).
template <class F>
__device__ __forceinline__ void for_l1(const ItsWs& w, int64_t i0, F f) {
  const int k0 = w.stave[i0];
  const int kc = wedge_of(w, 1, 0, k0, w.cX[i0], w.cY[i0]);
  const int ns = w.ns[1];
  for (int d = -1; d <= 1; ++d) {
    const int k = (kc + d + ns) % ns;
    if (d != 0 && (k == kc || (d == 1 && k == (kc + ns - 1) % ns))) continue;   // (fewer than 3 staves)
    const uint32_t a = w.scount[sidx(1, k)], b = w.scount[sidx(1, k) + 1];
    for (uint32_t j = a; j < b; ++j) f((int64_t)w.slist[j]);
  }
}

__device__ __forceinline__ bool spd_pair(const ItsWs& w, int64_t a, int64_t b, float sphi, float& cross) {
  const float Xa = w.cX[a], Ya = w.cY[a], Xb = w.cX[b], Yb = w.cY[b];
  cross = Xa * Yb - Ya * Xb;
  const float dot = Xa * Xb + Ya * Yb;
  return dot > 0.0f && fabsf(cross) <= sphi * (w.cR[a] * w.cR[b]);
}

__device__ __forceinline__ float zline(const ItsWs& w, int64_t a, int64_t b) {
  const float za = w.z[a], zb = w.z[b], ra = w.cR[a], rb = w.cR[b];
  return za - ra * ((zb - za) / (rb - ra));
}

__device__ __forceinline__ int bin_of(const ItsWs& w, float zv) {
  const float u = (zv + w.P.vtx_range) / w.P.vtx_bin;
  if (!(u >= 0.0f) || !(u < (float)w.nbins)) return -1;
  return (int)floorf(u);
}

__global__ __launch_bounds__(TB) void k_its_vpairs(ItsWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i >= w.n || w.layer[i] != 0 || w.vsum[3] != 0ull) return;
  uint32_t cnt = 0;
  for_l1(w, i, [&](int64_t j) {
    float cr;
    if (!spd_pair(w, i, j, w.P.vtx_sin_phi, cr)) return;
    const int b = bin_of(w, zline(w, i, j));
    if (b < 0) return;
    atomicAdd(&w.hist[b], 1u);
    ++cnt;
  });
  if (cnt) atomicAdd(&w.vsum[0], (unsigned long long)cnt);
}

// fullest bin (ties: lower), one workgroup
__global__ __launch_bounds__(TB) void k_its_vpeak(ItsWs w) {
  __shared__ unsigned long long s[TB];
  unsigned long long best = 0ull;
  for (int b = threadIdx.x; b < w.nbins; b += TB) {
    const uint32_t c = w.hist[b];
    // key: count high, inverted bin low, so the maximum prefers the lower bin
    const unsigned long long key = c ? ((unsigned long long)c << 32) | (uint32_t)(0xFFFFFFFFu - (uint32_t)b) : 0ull;
    best = key > best ? key : best;
  }
  s[threadIdx.x] = best;
  __syncthreads();
  for (int d = TB / 2; d > 0; d >>= 1) {
    if (threadIdx.x < d && s[threadIdx.x + d] > s[threadIdx.x]) s[threadIdx.x] = s[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) w.vpeak[0] = s[0] ? (int32_t)(0xFFFFFFFFu - (uint32_t)(s[0] & 0xFFFFFFFFull)) : -1;
}

__global__ __launch_bounds__(TB) void k_its_vsum(ItsWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  const int pk = w.vpeak[0];
  if (i >= w.n || w.layer[i] != 0 || pk < 0 || w.vsum[3] != 0ull) return;
  unsigned long long cnt = 0ull, q = 0ull;
  for_l1(w, i, [&](int64_t j) {
    float cr;
    if (!spd_pair(w, i, j, w.P.vtx_sin_phi, cr)) return;
    const float zv = zline(w, i, j);
    const int b = bin_of(w, zv);
    if (b < 0 || b < pk - 1 || b > pk + 1) return;
    q += (unsigned long long)(long long)rintf(zv * 65536.0f);   // (two's complement sums)
    ++cnt;
  });
  if (cnt) {
    atomicAdd(&w.vsum[1], cnt);
    atomicAdd(&w.vsum[2], q);
  }
}

__global__ void k_its_vfinal(ItsWs w) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const unsigned long long n = w.vsum[1];
  if (w.vpeak[0] >= 0 && n > 0ull) {
    const long long q = (long long)w.vsum[2];
    w.vzd[0] = (float)((double)q / (double)n / 65536.0);
    w.vzd[1] = 1.0f;
  } else {
    w.vzd[0] = 0.0f;
    w.vzd[1] = 0.0f;
  }
}

__global__ __launch_bounds__(TB) void k_its_tl(ItsWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i >= w.n || w.layer[i] != 0 || w.vsum[3] != 0ull) return;
  const float vz = w.vzd[0];
  const float itp2 = 1.0f / (w.P.trk_sin_phi * w.P.trk_sin_phi);
  const float itt2 = 1.0f / (w.P.trk_dtgl * w.P.trk_dtgl);
  const float ra = w.cR[i], za = w.z[i];
  unsigned long long best = ~0ull;
  for_l1(w, i, [&](int64_t j) {
    float cr;
    if (!spd_pair(w, i, j, w.P.trk_sin_phi, cr)) return;
    const float rb = w.cR[j];
    const float dt = (w.z[j] - vz) / rb - (za - vz) / ra;
    if (!(fabsf(dt) <= w.P.trk_dtgl)) return;
    const float sp = cr / (ra * rb);
    const float sc = (sp * sp) * itp2 + (dt * dt) * itt2;
    const unsigned long long hi = (unsigned long long)__float_as_uint(sc) << 32;
    best = min(best, hi | (uint32_t)j);
    atomicMin(&w.best1[j], hi | (uint32_t)i);
  });
  w.best0[i] = best;
}

__global__ __launch_bounds__(TB) void k_its_tlflag(ItsWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i >= w.n) return;
  uint32_t f = 0u;
  if (w.layer[i] == 0 && w.vsum[3] == 0ull) {
    const unsigned long long b = w.best0[i];
    if (b != ~0ull) {
      const uint32_t j = (uint32_t)(b & 0xFFFFFFFFull);
      f = (uint32_t)(w.best1[j] & 0xFFFFFFFFull) == (uint32_t)i ? 1u : 0u;
    }
  }
  w.tflag[i] = f;
}

__global__ __launch_bounds__(TB) void k_its_tlcompact(ItsWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i >= w.n) return;
  const uint32_t a = w.tflag[i], b = w.tflag[i + 1];
  if (b == a || (int64_t)a >= w.cap) return;
  w.o.tl0[a] = (int32_t)i;
  w.o.tl1[a] = (int32_t)(w.best0[i] & 0xFFFFFFFFull);
}

// Rotation of a state at plane x into a frame turned by the angle with
// cosine ca and sine sa (the point (x ca + y sa, -x sa + y ca), sin phi' =
// s ca - c sa, covariance J C J^T with the Jacobian at the fixed new
// plane).  False if |sin phi'| reaches sin_max.
__device__ bool rotate_frame(float& x, float p[5], float C[15], float ca, float sa, const Model& m) {
  const float s = p[2];
  const float c = sqrtf(1.0f - s * s);
  const float s2 = s * ca - c * sa;
  if (!(fabsf(s2) < m.sin_max)) return false;
  const float c2 = sqrtf(1.0f - s2 * s2);
  const float kap = m.kfac * p[4];
  const float x2 = x * ca + p[0] * sa;
  const float y2 = -(x * sa) + p[0] * ca;
  float J[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) J[i][j] = 0.0f;
  J[0][0] = ca - (s2 / c2) * sa;
  J[1][0] = -(p[3] / c2) * sa;
  J[1][1] = 1.0f;
  J[2][0] = -kap * sa;
  J[2][2] = ca + sa * (s / c);
  J[3][3] = 1.0f;
  J[4][4] = 1.0f;
  float T[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k < 5; ++k) acc = acc + J[i][k] * C[sym(k, j)];
      T[i][j] = acc;
    }
  float Cn[15];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = i; j < 5; ++j) {
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k < 5; ++k) acc = acc + T[i][k] * J[j][k];
      Cn[sym(i, j)] = acc;
    }
#pragma unroll
  for (int i = 0; i < 15; ++i) C[i] = Cn[i];
  x = x2;
  p[0] = y2;
  p[2] = s2;
  return true;
}

// Multiple scattering in a layer's average material: two independent
// deflections of variance theta0^2 perpendicular to the direction give
// var(sin phi) = theta0^2 cos^2 phi / cos^2 lambda, var(tan lambda) =
// theta0^2 / cos^4 lambda, var(q/pT) = theta0^2 (q/pT)^2 tan^2 lambda and
// cov(tan lambda, q/pT) = theta0^2 (q/pT) tan lambda / cos^2 lambda; theta0
// by Highland (beta = 1) for the path x/X0 / (cos lambda cos phi), with the
// logarithmic factor kms at normal incidence.
__device__ __forceinline__ void its_ms(float p[5], float C[15], float xx0, float kms) {
  const float s = p[2], t = p[3], k = p[4];
  const float t2 = 1.0f + t * t;
  const float c2 = 1.0f - s * s;
  const float path = xx0 * sqrtf(t2 / c2);
  const float pin = (k * k) / t2;
  const float hl = 0.0136f;
  const float th2 = (((hl * hl) * pin) * path) * (kms * kms);
  const float kt = k * t;
  C[sym(2, 2)] = C[sym(2, 2)] + th2 * (c2 * t2);
  C[sym(3, 3)] = C[sym(3, 3)] + th2 * (t2 * t2);
  C[sym(3, 4)] = C[sym(3, 4)] + th2 * (t2 * kt);
  C[sym(4, 4)] = C[sym(4, 4)] + th2 * (kt * kt);
}

__device__ __forceinline__ void frame_turn(const ItsTab* tb, int lt, int kt, int lf, int kf, float& dca, float& dsa) {
  dca = tb->ca[lt][kt] * tb->ca[lf][kf] + tb->sa[lt][kt] * tb->sa[lf][kf];
  dsa = tb->sa[lt][kt] * tb->ca[lf][kf] - tb->ca[lt][kt] * tb->sa[lf][kf];
}

// Following and inward fit of one tracklet (lane per tracklet).
__global__ __launch_bounds__(64) void k_its_follow(ItsWs w) {
  const int64_t t = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int64_t T = std::min<int64_t>((int64_t)w.tflag[w.n], w.cap);
  if (t >= T) return;
  const ItsTab* tb = w.tab;
  const int64_t ia = w.o.tl0[t], ib = w.o.tl1[t];
  const float vz = w.vzd[0];
  Model m = w.m;
  const float ax = w.x[ia], ay = w.y[ia], az = w.z[ia];
  const int ka = w.stave[ia], kb = w.stave[ib];
  const float ca0 = tb->ca[0][ka], sa0 = tb->sa[0][ka];
  const float BX = w.cX[ib], BY = w.cY[ib];
  const float bx = BX * ca0 + BY * sa0, by = -(BX * sa0) + BY * ca0;
  const float la = sqrtf(ax * ax + ay * ay), lb = sqrtf(bx * bx + by * by);
  const float ex = bx - ax, ey = by - ay, lab = sqrtf(ex * ex + ey * ey);
  const float crs = ax * by - ay * bx;
  const float kap = (2.0f * crs) / ((la * lb) * lab);
  const float dl = (kap * la) * 0.5f;
  const float cd = sqrtf(1.0f - dl * dl);
  float p[5], C[15];
  p[0] = 0.0f;
  p[1] = vz;
  p[2] = (ay / la) * cd - (ax / la) * dl;
  p[3] = (w.z[ib] - az) / lab;
  p[4] = kap / m.kfac;
#pragma unroll
  for (int i = 0; i < 15; ++i) C[i] = 0.0f;
  C[sym(0, 0)] = w.P.sigma_vy * w.P.sigma_vy;
  C[sym(1, 1)] = w.P.sigma_vz * w.P.sigma_vz;
  C[sym(2, 2)] = 1e-2f;
  C[sym(3, 3)] = 1e-2f;
  C[sym(4, 4)] = 1.0f;
  float chi2 = 0.0f, xc = 0.0f;
  int kst[kLayers] = {-1, -1, -1, -1, -1, -1};
  int32_t cl[kLayers] = {-1, -1, -1, -1, -1, -1};
  bool alive = fabsf(p[2]) < m.sin_max;
  int lc = -1, kc = -1, ncl = 0, miss = 0;
  bool rejected = false;
  for (int l = 0; l < 2 && alive; ++l) {
    const int64_t h = l == 0 ? ia : ib;
    const int kh = l == 0 ? ka : kb;
    if (l == 1) {
      float dca, dsa;
      frame_turn(tb, 1, kh, 0, kc, dca, dsa);
      if (!rotate_frame(xc, p, C, dca, dsa, m)) { alive = false; break; }
    }
    const float hx = w.x[h];
    if (!transport(p, C, xc, hx, m)) { alive = false; break; }
    xc = hx;
    m.vy = w.vy[l]; m.vz = w.vz[l];
    update(p, C, w.y[h], w.z[h], m, chi2);
    its_ms(p, C, w.xx0[l], w.kms[l]);
    cl[l] = (int32_t)h;
    kst[l] = kh;
    lc = l; kc = kh;
    ++ncl;
  }
  for (int l = 2; l < kLayers && alive; ++l) {
    float pp[5], CC[15];
#pragma unroll
    for (int i = 0; i < 5; ++i) pp[i] = p[i];
#pragma unroll
    for (int i = 0; i < 15; ++i) CC[i] = C[i];
    if (!transport(pp, CC, xc, w.r[l], m)) { alive = false; break; }
    const float X = w.r[l] * tb->ca[lc][kc] - pp[0] * tb->sa[lc][kc];
    const float Y = w.r[l] * tb->sa[lc][kc] + pp[0] * tb->ca[lc][kc];
    const int k = wedge_of(w, l, lc, kc, X, Y);
    float dca, dsa;
    frame_turn(tb, l, k, lc, kc, dca, dsa);
    if (!rotate_frame(xc, p, C, dca, dsa, m)) { alive = false; break; }
    if (!transport(p, C, xc, w.r[l], m)) { alive = false; break; }
    xc = w.r[l];
    lc = l; kc = k; kst[l] = k;
    const float isy = 1.0f / (C[0] + w.vy[l]), isz = 1.0f / (C[5] + w.vz[l]);
    float bchi = w.P.chi2_cut;
    int32_t bid = -1;
    const uint32_t a = w.scount[sidx(l, k)], b = w.scount[sidx(l, k) + 1];
    for (uint32_t j = a; j < b; ++j) {
      const int32_t id = (int32_t)w.slist[j];
      const float dy = w.y[id] - p[0], dz = w.z[id] - p[1];
      const float ch = (dy * dy) * isy + (dz * dz) * isz;
      if (ch < bchi || (ch == bchi && (bid < 0 || id < bid))) { bchi = ch; bid = id; }
    }
    if (bid >= 0) {
      m.vy = w.vy[l]; m.vz = w.vz[l];
      update(p, C, w.y[bid], w.z[bid], m, chi2);
      cl[l] = bid;
      ++ncl;
      miss = 0;
    } else if (++miss >= 2) {
      rejected = true;
      break;
    }
    its_ms(p, C, w.xx0[l], w.kms[l]);
  }
  const int missing_tail = kLayers - 1 - lc;
  if (lc < 1 || miss + missing_tail >= 2) rejected = true;
  int32_t* cls = w.o.cls + t * 6;
  if (rejected || ncl < w.P.min_clusters) {
    w.o.ok[t] = 0;
    w.o.in_ok[t] = 0;
    w.o.ncls[t] = 0;
    w.o.chi2[t] = 0.0f;
    w.o.out_layer[t] = -1; w.o.out_stave[t] = -1; w.o.in_stave[t] = -1;
#pragma unroll
    for (int i = 0; i < 6; ++i) cls[i] = -1;
    return;
  }
  w.o.ok[t] = 1;
  w.o.ncls[t] = ncl;
  w.o.chi2[t] = chi2;
  w.o.out_layer[t] = lc;
  w.o.out_stave[t] = kc;
  w.o.out_x[t] = xc;
#pragma unroll
  for (int i = 0; i < 6; ++i) cls[i] = cl[i];
#pragma unroll
  for (int i = 0; i < 5; ++i) w.o.out_p[t * 5 + i] = p[i];
#pragma unroll
  for (int i = 0; i < 15; ++i) w.o.out_cov[t * 15 + i] = C[i];
  // inward, no vertex point
  float q[5], Q[15], dummy = 0.0f;
#pragma unroll
  for (int i = 0; i < 5; ++i) q[i] = p[i];
#pragma unroll
  for (int i = 0; i < 15; ++i) Q[i] = C[i] * w.P.cov_scale_in;
  float xq = xc;
  bool iok = true;
  for (int l = lc; l >= 0 && iok; --l) {
    if (l < lc) {
      float dca, dsa;
      frame_turn(tb, l, kst[l], l + 1, kst[l + 1], dca, dsa);
      if (!rotate_frame(xq, q, Q, dca, dsa, m)) { iok = false; break; }
      if (!transport(q, Q, xq, w.r[l], m)) { iok = false; break; }
      xq = w.r[l];
    }
    if (cl[l] >= 0) {
      m.vy = w.vy[l]; m.vz = w.vz[l];
      update(q, Q, w.y[cl[l]], w.z[cl[l]], m, dummy);
    }
    its_ms(q, Q, w.xx0[l], w.kms[l]);
  }
  if (iok && transport(q, Q, xq, 0.0f, m)) {
    w.o.in_ok[t] = 1;
    w.o.in_stave[t] = kst[0];
#pragma unroll
    for (int i = 0; i < 5; ++i) w.o.in_p[t * 5 + i] = q[i];
#pragma unroll
    for (int i = 0; i < 15; ++i) w.o.in_cov[t * 15 + i] = Q[i];
  } else {
    w.o.in_ok[t] = 0;
    w.o.in_stave[t] = -1;
  }
}

// Vertex fit: one workgroup; per solve, each thread sums its tracks (t =
// tid, tid + TB, ...) and the partial sums are added by a fixed tree, so the
// result does not depend on timing.
__global__ __launch_bounds__(TB) void k_its_vfit(ItsWs w) {
  __shared__ double s[10][TB];
  __shared__ double V[3];
  __shared__ int good;
  const int tid = threadIdx.x;
  const int64_t T = std::min<int64_t>((int64_t)w.tflag[w.n], w.cap);
  const ItsTab* tb = w.tab;
  int64_t nt = 0;
  for (int64_t t = tid; t < T; t += TB) {
    const bool use = w.o.ok[t] && w.o.in_ok[t];
    w.vw[t] = use ? 1.0 : 0.0;
  }
  // tracks entering the fit (block count)
  {
    int c = 0;
    for (int64_t t = tid; t < T; t += TB) c += (w.o.ok[t] && w.o.in_ok[t]) ? 1 : 0;
    s[0][tid] = (double)c;
    __syncthreads();
    for (int d = TB / 2; d > 0; d >>= 1) {
      if (tid < d) s[0][tid] += s[0][tid + d];
      __syncthreads();
    }
    nt = (int64_t)s[0][0];
    __syncthreads();
  }
  if (tid == 0) { good = nt >= 2 ? 1 : 0; V[0] = V[1] = V[2] = 0.0; }
  __syncthreads();
  double nused = 0.0, sumw = 0.0;
  auto line = [&](int64_t t, double Pp[3], double d[3], double& s2) {
    const int k = w.o.in_stave[t];
    const double ca = tb->ca[0][k], sa = tb->sa[0][k];
    const double yy = w.o.in_p[t * 5 + 0], zz = w.o.in_p[t * 5 + 1];
    const double sn = w.o.in_p[t * 5 + 2], tt = w.o.in_p[t * 5 + 3];
    const double cc = sqrt(1.0 - sn * sn), nn = sqrt(1.0 + tt * tt);
    Pp[0] = -(yy * sa); Pp[1] = yy * ca; Pp[2] = zz;
    d[0] = (cc * ca - sn * sa) / nn; d[1] = (cc * sa + sn * ca) / nn; d[2] = tt / nn;
    s2 = 0.5 * ((double)w.o.in_cov[t * 15 + 0] + (double)w.o.in_cov[t * 15 + 5]);
  };
  for (int it = 0; it < w.P.fit_iters && good; ++it) {
    double a[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // A (6) and b (3)
    for (int64_t t = tid; t < T; t += TB) {
      const double wt = w.vw[t];
      if (!(w.o.ok[t] && w.o.in_ok[t])) continue;
      double Pp[3], d[3], s2;
      line(t, Pp, d, s2);
      const double f = wt / s2;
      double M[3][3];
      for (int r = 0; r < 3; ++r)
        for (int c2 = 0; c2 < 3; ++c2) M[r][c2] = (r == c2 ? 1.0 : 0.0) - d[r] * d[c2];
      a[0] += f * M[0][0]; a[1] += f * M[0][1]; a[2] += f * M[0][2];
      a[3] += f * M[1][1]; a[4] += f * M[1][2]; a[5] += f * M[2][2];
      for (int r = 0; r < 3; ++r) a[6 + r] += f * (M[r][0] * Pp[0] + M[r][1] * Pp[1] + M[r][2] * Pp[2]);
    }
    for (int j = 0; j < 9; ++j) s[j][tid] = a[j];
    __syncthreads();
    for (int d = TB / 2; d > 0; d >>= 1) {
      if (tid < d)
        for (int j = 0; j < 9; ++j) s[j][tid] += s[j][tid + d];
      __syncthreads();
    }
    if (tid == 0) {
      const double a00 = s[0][0], a01 = s[1][0], a02 = s[2][0], a11 = s[3][0], a12 = s[4][0], a22 = s[5][0];
      const double b0 = s[6][0], b1 = s[7][0], b2 = s[8][0];
      const double c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22, c02 = a01 * a12 - a02 * a11;
      const double det = a00 * c00 + a01 * c01 + a02 * c02;
      if (!(fabs(det) > 0.0)) {
        good = 0;
      } else {
        const double c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12, c22 = a00 * a11 - a01 * a01;
        V[0] = (c00 * b0 + c01 * b1 + c02 * b2) / det;
        V[1] = (c01 * b0 + c11 * b1 + c12 * b2) / det;
        V[2] = (c02 * b0 + c12 * b1 + c22 * b2) / det;
      }
    }
    __syncthreads();
    if (!good) break;
    double nu = 0.0, sw = 0.0;
    for (int64_t t = tid; t < T; t += TB) {
      if (!(w.o.ok[t] && w.o.in_ok[t])) continue;
      double Pp[3], d[3], s2;
      line(t, Pp, d, s2);
      const double u0 = V[0] - Pp[0], u1 = V[1] - Pp[1], u2 = V[2] - Pp[2];
      const double pr = u0 * d[0] + u1 * d[1] + u2 * d[2];
      const double e0 = u0 - pr * d[0], e1 = u1 - pr * d[1], e2 = u2 - pr * d[2];
      const double D = sqrt((e0 * e0 + e1 * e1 + e2 * e2) / s2) / (double)w.P.tukey_c;
      const double wt = D < 1.0 ? (1.0 - D * D) * (1.0 - D * D) : 0.0;
      w.vw[t] = wt;
      nu += wt > 0.0 ? 1.0 : 0.0;
      sw += wt;
    }
    s[0][tid] = nu;
    s[1][tid] = sw;
    __syncthreads();
    for (int d = TB / 2; d > 0; d >>= 1) {
      if (tid < d) { s[0][tid] += s[0][tid + d]; s[1][tid] += s[1][tid + d]; }
      __syncthreads();
    }
    nused = s[0][0];
    sumw = s[1][0];
    __syncthreads();
  }
  if (tid == 0) {
    w.vres[0] = V[0]; w.vres[1] = V[1]; w.vres[2] = V[2];
    w.vres[3] = sumw; w.vres[4] = nused; w.vres[5] = good ? 1.0 : 0.0;
  }
}

__global__ void k_its_init(ItsWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i < kLayers * kStaves + 1) w.scount[i] = 0u;
  if (i < w.nbins) w.hist[i] = 0u;
  if (i < 4) w.vsum[i] = 0ull;
  if (i < w.n) w.best1[i] = ~0ull;
}

inline unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>((n + TB - 1) / TB, 1); }

hipError_t run_its(const ItsWs& w, hipStream_t st) {
  const unsigned g = grid_for(w.n);
  const int64_t ninit = std::max<int64_t>(std::max<int64_t>(w.n, w.nbins), kLayers * kStaves + 1);
  k_its_init<<<grid_for(ninit), TB, 0, st>>>(w);
  k_its_prep<<<g, TB, 0, st>>>(w);
  k_its_soff<<<1, 512, 0, st>>>(w);
  k_its_fill<<<g, TB, 0, st>>>(w);
  k_its_vpairs<<<g, TB, 0, st>>>(w);
  k_its_vpeak<<<1, TB, 0, st>>>(w);
  k_its_vsum<<<g, TB, 0, st>>>(w);
  k_its_vfinal<<<1, 64, 0, st>>>(w);
  k_its_tl<<<g, TB, 0, st>>>(w);
  k_its_tlflag<<<g, TB, 0, st>>>(w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_exclusive_u32(w.tflag, w.tflag, w.n, (uint32_t*)(w.vres + 8), st);
  if (e != hipSuccess) return e;
  k_its_tlcompact<<<g, TB, 0, st>>>(w);
  k_its_follow<<<(unsigned)std::max<int64_t>((w.cap + 63) / 64, 1), 64, 0, st>>>(w);
  k_its_vfit<<<1, TB, 0, st>>>(w);
  return hipGetLastError();
}

int its_fail(tpcca_its_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

}  // namespace
}  // namespace tpcca

using namespace tpcca;

extern "C" {

void tpcca_its_default_params(tpcca_its_params* p) {
  if (!p) return;
  p->vtx_sin_phi = 0.03f;
  p->vtx_bin = 0.1f;
  p->vtx_range = 20.0f;
  p->trk_sin_phi = 0.03f;
  p->trk_dtgl = 0.025f;
  p->chi2_cut = 12.0f;
  p->sigma_vy = 0.005f;
  p->sigma_vz = 0.02f;
  p->sin_max = 0.99f;
  p->min_clusters = 4;
  p->tukey_c = 4.685f;
  p->fit_iters = 8;
  p->cov_scale_in = 100.0f;
}

int tpcca_its_create(const tpcca_its_geometry* g, tpcca_its_ctx** out) {
  if (!g || !out) return TPCCA_E_INVALID;
  *out = nullptr;
  if (g->n_layers != kLayers || !(g->bz > 0.0f || g->bz < 0.0f)) return TPCCA_E_INVALID;
  for (int l = 0; l < kLayers; ++l) {
    if (g->n_staves[l] < 1 || g->n_staves[l] > kStaves || !(g->radius[l] > 0.0f) || !(g->half_z[l] > 0.0f) ||
        !(g->x_over_x0[l] > 0.0f) || !(g->sigma_y[l] > 0.0f) || !(g->sigma_z[l] > 0.0f))
      return TPCCA_E_INVALID;
    if (l > 0 && !(g->radius[l] > g->radius[l - 1])) return TPCCA_E_INVALID;
  }
  tpcca_its_ctx* c = new (std::nothrow) tpcca_its_ctx();
  if (!c) return TPCCA_E_NOMEM;
  c->g = *g;
  tpcca_its_default_params(&c->P);
  const float wmax = (float)std::sin(2.0 * M_PI / (double)g->n_staves[1]);
  if (!(c->P.vtx_sin_phi < wmax) || !(c->P.trk_sin_phi < wmax)) { delete c; return TPCCA_E_INVALID; }
  if (hipGetDevice(&c->device) != hipSuccess) { (void)hipGetLastError(); delete c; return TPCCA_E_DEVICE; }
  ItsTab tab{};
  for (int l = 0; l < kLayers; ++l) {
    const double d = 2.0 * M_PI / (double)g->n_staves[l];
    for (int k = 0; k < g->n_staves[l]; ++k) {
      tab.ca[l][k] = (float)std::cos((k + 0.5) * d);
      tab.sa[l][k] = (float)std::sin((k + 0.5) * d);
    }
    for (int j = 0; j <= g->n_staves[l]; ++j) {
      tab.bc[l][j] = (float)std::cos(j * d);
      tab.bs[l][j] = (float)std::sin(j * d);
    }
  }
  if (hipMalloc((void**)&c->tab, sizeof(ItsTab)) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return TPCCA_E_NOMEM;
  }
  if (hipMemcpy(c->tab, &tab, sizeof(ItsTab), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(c->tab);
    delete c;
    return TPCCA_E_DEVICE;
  }
  *out = c;
  return TPCCA_OK;
}

int tpcca_its_set_params(tpcca_its_ctx* c, const tpcca_its_params* p) {
  if (!c || !p) return TPCCA_E_INVALID;
  const int nb = (int)std::lrint(2.0 * (double)p->vtx_range / (double)p->vtx_bin);
  if (!(p->vtx_sin_phi > 0.0f && p->vtx_sin_phi < 0.1f) || !(p->vtx_bin > 0.0f) || !(p->vtx_range > 0.0f) ||
      nb < 1 || nb > kBins || !(p->trk_sin_phi > 0.0f && p->trk_sin_phi < 0.1f) || !(p->trk_dtgl > 0.0f) ||
      !(p->chi2_cut > 0.0f) || !(p->sigma_vy > 0.0f) || !(p->sigma_vz > 0.0f) ||
      !(p->sin_max > 0.0f && p->sin_max < 1.0f) || p->min_clusters < 2 || p->min_clusters > kLayers ||
      !(p->tukey_c > 0.0f) || p->fit_iters < 1 || p->fit_iters > 100 || !(p->cov_scale_in >= 1.0f))
    return its_fail(c, TPCCA_E_INVALID, "invalid ITS parameters");
  // the pair windows must be narrower than a layer-1 stave (the pair search
  // scans the stave around a cluster's azimuth and its two neighbours)
  const float wmax = (float)std::sin(2.0 * M_PI / (double)c->g.n_staves[1]);
  if (!(p->vtx_sin_phi < wmax) || !(p->trk_sin_phi < wmax))
    return its_fail(c, TPCCA_E_INVALID, "pair windows wider than a layer-1 stave");
  c->P = *p;
  return TPCCA_OK;
}

int tpcca_its_track(tpcca_its_ctx* c, const tpcca_its_clusters* cl, tpcca_its_tracks* o) {
  if (!c) return TPCCA_E_INVALID;
  if (!cl || !o) return its_fail(c, TPCCA_E_INVALID, "null clusters or output");
  const int64_t n = cl->n;
  if (n < 0 || n >= ((int64_t)1 << 31)) return its_fail(c, TPCCA_E_INVALID, "bad cluster count");
  if (n > 0 && (!cl->x || !cl->y || !cl->z || !cl->layer || !cl->stave))
    return its_fail(c, TPCCA_E_INVALID, "null cluster array");
  if (o->cap < 0 || (o->cap > 0 && (!o->tl0 || !o->tl1 || !o->ok || !o->cls || !o->ncls || !o->chi2 ||
                                    !o->out_layer || !o->out_stave || !o->out_x || !o->out_p ||
                                    !o->out_cov || !o->in_ok || !o->in_stave || !o->in_p || !o->in_cov)))
    return its_fail(c, TPCCA_E_INVALID, "null output array");
  hipError_t he = hipSetDevice(c->device);
  if (he != hipSuccess) return its_fail(c, TPCCA_E_DEVICE, "hipSetDevice");
  hipStream_t st = (hipStream_t)cl->stream;
  const int nbins = (int)std::lrint(2.0 * (double)c->P.vtx_range / (double)c->P.vtx_bin);
  const int64_t cap = o->cap;
  // workspace
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t at = off; off += (bytes + 255) & ~(size_t)255; return at; };
  const int64_t nn = std::max<int64_t>(n, 1);
  const size_t oX = take(4 * nn), oY = take(4 * nn), oR = take(4 * nn);
  const size_t ocnt = take(4 * (kLayers * kStaves + 1)), ocur = take(4 * kLayers * kStaves);
  const size_t olist = take(4 * nn), ohist = take(4 * nbins), ovsum = take(8 * 4), ovz = take(8), opk = take(8);
  const size_t ob0 = take(8 * nn), ob1 = take(8 * nn), oflag = take(4 * (nn + 1));
  const size_t ovw = take(8 * std::max<int64_t>(cap, 1));
  const size_t ovres = take(8 * 8 + 4 * (2 * (nn / 1024 + 2)) + 64);
  if (off > c->arena_bytes) {
    if (c->arena) { (void)hipFree(c->arena); c->arena = nullptr; c->arena_bytes = 0; }
    if (hipMalloc((void**)&c->arena, off + off / 4) != hipSuccess) {
      (void)hipGetLastError();
      return its_fail(c, TPCCA_E_NOMEM, "ITS workspace allocation failed");
    }
    c->arena_bytes = off + off / 4;
  }
  char* b = c->arena;
  ItsWs w{};
  w.n = n; w.cap = cap;
  w.x = cl->x; w.y = cl->y; w.z = cl->z; w.layer = cl->layer; w.stave = cl->stave;
  w.tab = (const ItsTab*)c->tab;
  for (int l = 0; l < kLayers; ++l) {
    w.r[l] = c->g.radius[l]; w.hz[l] = c->g.half_z[l]; w.xx0[l] = c->g.x_over_x0[l];
    w.vy[l] = c->g.sigma_y[l] * c->g.sigma_y[l]; w.vz[l] = c->g.sigma_z[l] * c->g.sigma_z[l];
    w.kms[l] = (float)(1.0 + 0.038 * std::log((double)c->g.x_over_x0[l]));
    w.ns[l] = c->g.n_staves[l];
  }
  w.m.kfac = -(float)((double)2.99792458e-3) * c->g.bz;
  w.m.sin_max = c->P.sin_max;
  w.m.vy = 0.0f; w.m.vz = 0.0f;
  w.P = c->P;
  w.nbins = nbins;
  w.cX = (float*)(b + oX); w.cY = (float*)(b + oY); w.cR = (float*)(b + oR);
  w.scount = (uint32_t*)(b + ocnt); w.scur = (uint32_t*)(b + ocur); w.slist = (uint32_t*)(b + olist);
  w.hist = (uint32_t*)(b + ohist); w.vsum = (unsigned long long*)(b + ovsum); w.vzd = (float*)(b + ovz);
  w.vpeak = (int32_t*)(b + opk);
  w.best0 = (unsigned long long*)(b + ob0); w.best1 = (unsigned long long*)(b + ob1);
  w.tflag = (uint32_t*)(b + oflag); w.vw = (double*)(b + ovw); w.vres = (double*)(b + ovres);
  w.o = *o;
  // an empty capacity still hands the kernels valid pointers
  if (cap == 0) {
    w.o.tl0 = w.o.tl1 = w.o.ok = w.o.ncls = w.o.out_layer = w.o.out_stave = w.o.in_ok = w.o.in_stave = (int32_t*)b;
    w.o.cls = (int32_t*)b;
    w.o.chi2 = w.o.out_x = w.o.out_p = w.o.out_cov = w.o.in_p = w.o.in_cov = (float*)b;
  }
  if (n == 0) {
    w.x = w.y = w.z = (const float*)b; w.layer = (const int8_t*)b; w.stave = (const int16_t*)b;
  }
  he = run_its(w, st);
  if (he != hipSuccess) return its_fail(c, TPCCA_E_DEVICE, std::string("ITS kernels: ") + hipGetErrorString(he));
  unsigned long long vs[4] = {0, 0, 0, 0};
  float vz[2] = {0, 0};
  int32_t pk = -1;
  uint32_t T = 0;
  double vr[6] = {0, 0, 0, 0, 0, 0};
  he = hipMemcpyAsync(vs, w.vsum, sizeof(vs), hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipMemcpyAsync(vz, w.vzd, sizeof(vz), hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipMemcpyAsync(&pk, w.vpeak, 4, hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipMemcpyAsync(&T, w.tflag + n, 4, hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipMemcpyAsync(vr, w.vres, sizeof(vr), hipMemcpyDeviceToHost, st);
  if (he == hipSuccess && o->hist)
    he = hipMemcpyAsync(o->hist, w.hist, 4 * (size_t)nbins, hipMemcpyDeviceToDevice, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) return its_fail(c, TPCCA_E_DEVICE, std::string("ITS results: ") + hipGetErrorString(he));
  if (vs[3]) return its_fail(c, TPCCA_E_INVALID, "a cluster has a bad layer or stave or a non-finite coordinate");
  o->n_tracklets = n > 0 ? (int64_t)T : 0;
  if (o->n_tracklets > cap) return its_fail(c, TPCCA_E_CAPACITY, "more tracklets than the output holds");
  o->n_pairs = (int64_t)vs[0];
  o->peak = pk;
  o->vz = vz[0];
  o->vz_ok = vz[1] != 0.0f ? 1 : 0;
  o->vertex[0] = vr[0]; o->vertex[1] = vr[1]; o->vertex[2] = vr[2];
  o->vfit_sumw = vr[3];
  o->vfit_n = (int32_t)vr[4];
  o->vfit_ok = vr[5] != 0.0 ? 1 : 0;
  return TPCCA_OK;
}

const char* tpcca_its_last_error(const tpcca_its_ctx* c) { return c ? c->err.c_str() : "null context"; }

void tpcca_its_destroy(tpcca_its_ctx* c) {
  if (!c) return;
  if (c->arena) (void)hipFree(c->arena);
  if (c->tab) (void)hipFree(c->tab);
  delete c;
}

}  // extern "C"
