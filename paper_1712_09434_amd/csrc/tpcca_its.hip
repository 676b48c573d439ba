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
// One call covers any number of events (ITS events are small: one event per
// call would leave the chip idle and pay the launches per event).  Kernels:
// gather of the events' clusters with their global positions and per-stave
// counts; stave offsets; stave records (global x, y, radius, z for the pair
// tests; local y, z, id for the cluster search) and the ordered layer-0
// list; pair histogram per event (eight lanes per layer-0 cluster share the
// records of the three layer-1 staves around its azimuth, each loading eight
// at a time; the histogram privatised in LDS), peak, fixed-point mean;
// tracklet candidates (best of each layer-0 cluster by a group minimum, best
// of each layer-1 cluster by a 64-bit atomic minimum of (score bits, id)); mutual pairs compacted in
// id order; following and inward fit (four lanes per tracklet sharing the
// cluster search); vertex fit (one workgroup per event, fixed-order FP64
// reductions).  Every event's results equal those of a call on that event
// alone.
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
  char* hpin = nullptr;          // pinned staging of the per-call tables and results
  size_t hpin_bytes = 0;
};

namespace tpcca {
namespace {

constexpr int TB = 256;
constexpr int kLayers = 6;
constexpr int kStaves = 64;      // per layer, at most
constexpr int kBins = 4096;      // vertexer histogram bins, at most
constexpr int kPerEv = kLayers * kStaves;   // stave slots per event

// Geometry tables in device memory (FP32 values of FP64 expressions):
// stave centre cos/sin and wedge boundary cos/sin per layer.
struct ItsTab {
  float ca[kLayers][kStaves], sa[kLayers][kStaves];
  float bc[kLayers][kStaves + 1], bs[kLayers][kStaves + 1];
};

struct ItsEvIn {
  const float* x;
  const float* y;
  const float* z;
  const int8_t* layer;
  const int16_t* stave;
  int64_t off;             // first global cluster of the event
};

struct ItsWs {
  int E;
  int64_t n;               // clusters of all events
  const ItsEvIn* ev;       // [E + 1] (off of entry E: n)
  tpcca_its_tracks* out;   // [E] the callers' outputs (device copy of the structs)
  const ItsTab* tab;
  float r[kLayers], xx0[kLayers], vy[kLayers], vz[kLayers], kms[kLayers];
  int ns[kLayers];
  Model m;
  tpcca_its_params P;
  int nbins;
  // clusters of all events (global order = event-major input order)
  float* cx;
  float* cy;
  float* cz;
  int8_t* cl;
  int16_t* ck;
  int32_t* cev;
  float* cX;               // global position and radius (FP32)
  float* cY;
  float* cR;
  uint32_t* err;           // [1] bit 0: a bad layer / stave or a non-finite coordinate
  uint32_t* scnt;          // [E * kPerEv + 1] clusters per (event, layer, stave) -> offsets
  uint32_t* scur;          // [E * kPerEv] fill cursors
  uint32_t* slist;         // [n] cluster ids by stave
  float4* sA;              // [n] by stave: global X, Y, radius, z (pair tests)
  float4* sB;              // [n] by stave: local y, z, id bits (cluster search)
  uint32_t* l0f;           // [n + 1] layer-0 indicator -> offsets
  uint32_t* l0list;        // [n] layer-0 clusters in id order
  uint32_t* hist;          // [E * nbins]
  unsigned long long* vsum;   // [E * 4]: pairs, pairs in the mean, fixed-point sum
  float* vzd;              // [E * 2]: vertex z, found flag
  int32_t* vpeak;          // [E]
  unsigned long long* best0;  // [n] (score bits << 32) | layer-1 id
  unsigned long long* best1;  // [n] (score bits << 32) | layer-0 id
  uint32_t* tflag;         // [n + 1] mutual pair at a layer-0 cluster -> offsets
  int32_t* tl0;            // [n] global tracklet list: layer-0 id, layer-1 id, event
  int32_t* tl1;
  int32_t* tev;
  uint32_t* toff;          // [E + 1] first tracklet of each event
  double* vw;              // [n] vertex-fit weights
  double* vres;            // [E * 8]: vertex (3), sum of weights, tracks used, ok
  uint32_t* part;          // scan partial sums
};

__device__ __forceinline__ int sidx(int e, int l, int k) { return (e * kLayers + l) * kStaves + k; }

// Largest e with ev[e].off <= i.
__device__ __forceinline__ int event_of(const ItsWs& w, int64_t i) {
  int lo = 0, hi = w.E - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (w.ev[mid].off <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(TB) void k_its_init(ItsWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i < (int64_t)w.E * kPerEv + 1) w.scnt[i] = 0u;
  if (i < (int64_t)w.E * w.nbins) w.hist[i] = 0u;
  if (i < (int64_t)w.E * 4) w.vsum[i] = 0ull;
  if (i < w.n) w.best1[i] = ~0ull;
  if (i == 0) w.err[0] = 0u;
}

__global__ __launch_bounds__(TB) void k_its_gather(ItsWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i >= w.n) return;
  const int e = event_of(w, i);
  const ItsEvIn& v = w.ev[e];
  const int64_t j = i - v.off;
  const int l = v.layer[j], k = v.stave[j];
  const float x = v.x[j], y = v.y[j], z = v.z[j];
  w.cx[i] = x; w.cy[i] = y; w.cz[i] = z; w.cl[i] = (int8_t)l; w.ck[i] = (int16_t)k; w.cev[i] = e;
  const bool ok = l >= 0 && l < kLayers && k >= 0 && k < w.ns[l] && isfinite(x) && isfinite(y) && isfinite(z);
  w.l0f[i] = ok && l == 0 ? 1u : 0u;
  if (!ok) {
    atomicOr(w.err, 1u);
    w.cX[i] = 0.0f; w.cY[i] = 0.0f; w.cR[i] = 0.0f;
    w.cl[i] = -1;   // (skipped by the later kernels)
    return;
  }
  const float ca = w.tab->ca[l][k], sa = w.tab->sa[l][k];
  const float X = x * ca - y * sa;
  const float Y = x * sa + y * ca;
  w.cX[i] = X;
  w.cY[i] = Y;
  w.cR[i] = sqrtf(X * X + Y * Y);
  atomicAdd(&w.scnt[sidx(e, l, k)], 1u);
}

__global__ __launch_bounds__(TB) void k_its_cursors(ItsWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i < (int64_t)w.E * kPerEv) w.scur[i] = w.scnt[i];
}

__global__ __launch_bounds__(TB) void k_its_fill(ItsWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i >= w.n || w.cl[i] < 0) return;
  const int l = w.cl[i];
  const uint32_t pos = atomicAdd(&w.scur[sidx(w.cev[i], l, w.ck[i])], 1u);
  w.slist[pos] = (uint32_t)i;
  w.sA[pos] = make_float4(w.cX[i], w.cY[i], w.cR[i], w.cz[i]);
  w.sB[pos] = make_float4(w.cy[i], w.cz[i], __uint_as_float((uint32_t)i), 0.0f);
  if (l == 0) w.l0list[w.l0f[i]] = (uint32_t)i;
}

// The stave of layer l whose wedge holds the direction (X, Y), searched
// from the stave of the same angular position as stave kf of layer lf.
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

// Lanes per layer-0 cluster in the pair kernels and per tracklet in the
// following (fewer: each lane also repeats the tracklet's Kalman steps): the
// records a cluster or tracklet visits are split over them.
constexpr int kGrp = 8;
constexpr int kGrpF = 4;   // lanes per tracklet in the following

template <int G = kGrp>
__device__ __forceinline__ unsigned long long grp_min(unsigned long long v) {
#pragma unroll
  for (int d = 1; d < G; d <<= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)(v & 0xFFFFFFFFull), d, G);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), d, G);
    const unsigned long long o = ((unsigned long long)hi << 32) | lo;
    v = o < v ? o : v;
  }
  return v;
}

// Sum over the group (integers: any order gives the same result).
__device__ __forceinline__ unsigned long long grp_sum(unsigned long long v) {
#pragma unroll
  for (int d = 1; d < kGrp; d <<= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)(v & 0xFFFFFFFFull), d, kGrp);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), d, kGrp);
    v += ((unsigned long long)hi << 32) | lo;
  }
  return v;
}

// One layer-0 cluster per group of kGrp lanes, in id order.
struct L0 {
  bool ok;
  float X, Y, R, z;
  int k, e;
  uint32_t id;
};
__device__ __forceinline__ L0 l0_cluster(const ItsWs& w, int64_t t) {
  L0 c{};
  c.ok = t < (int64_t)w.l0f[w.n] && w.err[0] == 0u;
  if (!c.ok) return c;
  c.id = w.l0list[t];
  c.X = w.cX[c.id]; c.Y = w.cY[c.id]; c.R = w.cR[c.id]; c.z = w.cz[c.id];
  c.k = w.ck[c.id];
  c.e = w.cev[c.id];
  return c;
}

// Visits every layer-1 cluster record of the event's three staves around a
// layer-0 cluster's azimuth (every pair within a window narrower than a
// stave), lane gl of the group taking every kGrp-th record, the records of
// a chunk loaded together: f(record, list position).
constexpr int kChunk = 8;
template <class F>
__device__ __forceinline__ void for_l1(const ItsWs& w, const L0& c, int gl, F f) {
  const int kc = wedge_of(w, 1, 0, c.k, c.X, c.Y);
  const int ns = w.ns[1];
  for (int d = -1; d <= 1; ++d) {
    const int k = (kc + d + ns) % ns;
    if (d != 0 && (k == kc || (d == 1 && k == (kc + ns - 1) % ns))) continue;   // (fewer than 3 staves)
    const uint32_t a = w.scnt[sidx(c.e, 1, k)], b = w.scnt[sidx(c.e, 1, k) + 1];
    for (uint32_t j0 = a + (uint32_t)gl; j0 < b; j0 += kChunk * kGrp) {
      float4 r[kChunk];
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        const uint32_t j = j0 + (uint32_t)(u * kGrp);
        r[u] = w.sA[j < b ? j : a];
      }
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        const uint32_t j = j0 + (uint32_t)(u * kGrp);
        if (j < b) f(r[u], j);
      }
    }
  }
}

// Layer-0 clusters per workgroup of the pair kernels.
constexpr int kPerWg = TB / kGrp;

__device__ __forceinline__ bool spd_pair(const L0& a, const float4& b, float sphi, float& cross) {
  cross = a.X * b.y - a.Y * b.x;
  const float dot = a.X * b.x + a.Y * b.y;
  return dot > 0.0f && fabsf(cross) <= sphi * (a.R * b.z);
}

__device__ __forceinline__ float zline(const L0& a, const float4& b) {
  return a.z - a.R * ((b.w - a.z) / (b.z - a.R));
}

__device__ __forceinline__ int bin_of(const ItsWs& w, float zv) {
  const float u = (zv + w.P.vtx_range) / w.P.vtx_bin;
  if (!(u >= 0.0f) || !(u < (float)w.nbins)) return -1;
  return (int)floorf(u);
}

// Pair histogram.  The pairs of an event crowd into the few bins around its
// vertex: the bins of the workgroup's first event are privatised in LDS
// (one global atomic per non-empty bin), other events' go straight to the
// global histogram.
__global__ __launch_bounds__(TB) void k_its_vpairs(ItsWs w) {
  __shared__ uint32_t h[kBins];
  __shared__ unsigned long long s_n;
  const int64_t t0 = (int64_t)blockIdx.x * kPerWg;
  const L0 f = l0_cluster(w, t0);
  if (!f.ok) return;   // (workgroup-uniform: no layer-0 cluster from here on)
  const int e0 = f.e;
  for (int bb = threadIdx.x; bb < w.nbins; bb += TB) h[bb] = 0u;
  if (threadIdx.x == 0) s_n = 0ull;
  const int gl = threadIdx.x % kGrp;
  const L0 c = l0_cluster(w, t0 + threadIdx.x / kGrp);
  __syncthreads();
  if (c.ok) {
    unsigned long long cnt = 0ull;
    for_l1(w, c, gl, [&](const float4& b, uint32_t) {
      float cr;
      if (!spd_pair(c, b, w.P.vtx_sin_phi, cr)) return;
      const int bin = bin_of(w, zline(c, b));
      if (bin < 0) return;
      if (c.e == e0) atomicAdd(&h[bin], 1u);
      else atomicAdd(&w.hist[(int64_t)c.e * w.nbins + bin], 1u);
      ++cnt;
    });
    cnt = grp_sum(cnt);
    // the pair count of the workgroup's first event is summed in LDS first
    if (gl == 0 && cnt) {
      if (c.e == e0) atomicAdd(&s_n, cnt);
      else atomicAdd(&w.vsum[c.e * 4 + 0], cnt);
    }
  }
  __syncthreads();
  for (int bb = threadIdx.x; bb < w.nbins; bb += TB)
    if (h[bb]) atomicAdd(&w.hist[(int64_t)e0 * w.nbins + bb], h[bb]);
  if (threadIdx.x == 0 && s_n) atomicAdd(&w.vsum[e0 * 4 + 0], s_n);
}

// fullest bin of each event (ties: lower), one workgroup per event
__global__ __launch_bounds__(TB) void k_its_vpeak(ItsWs w) {
  __shared__ unsigned long long s[TB];
  const int e = blockIdx.x;
  const uint32_t* hist = w.hist + (int64_t)e * w.nbins;
  unsigned long long best = 0ull;
  for (int b = threadIdx.x; b < w.nbins; b += TB) {
    const uint32_t c = hist[b];
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
  if (threadIdx.x == 0) w.vpeak[e] = s[0] ? (int32_t)(0xFFFFFFFFu - (uint32_t)(s[0] & 0xFFFFFFFFull)) : -1;
}

// Pairs in the peak's three bins: count and fixed-point sum of their z, the
// workgroup's first event summed in LDS first (one global atomic each per
// workgroup; the event counters of a batch share a few cache lines).
__global__ __launch_bounds__(TB) void k_its_vsum(ItsWs w) {
  __shared__ unsigned long long s_n, s_q;
  const int64_t t0 = (int64_t)blockIdx.x * kPerWg;
  const L0 f = l0_cluster(w, t0);
  if (!f.ok) return;   // (workgroup-uniform)
  const int e0 = f.e;
  if (threadIdx.x == 0) { s_n = 0ull; s_q = 0ull; }
  __syncthreads();
  const L0 c = l0_cluster(w, t0 + threadIdx.x / kGrp);
  const int gl = threadIdx.x % kGrp;
  const int pk = c.ok ? w.vpeak[c.e] : -1;
  if (pk >= 0) {   // (group-uniform)
    unsigned long long cnt = 0ull, q = 0ull;
    for_l1(w, c, gl, [&](const float4& b, uint32_t) {
      float cr;
      if (!spd_pair(c, b, w.P.vtx_sin_phi, cr)) return;
      const float zv = zline(c, b);
      const int bin = bin_of(w, zv);
      if (bin < 0 || bin < pk - 1 || bin > pk + 1) return;
      q += (unsigned long long)(long long)rintf(zv * 65536.0f);   // (two's complement sums)
      ++cnt;
    });
    cnt = grp_sum(cnt);
    q = grp_sum(q);
    if (gl == 0 && cnt) {
      if (c.e == e0) {
        atomicAdd(&s_n, cnt);
        atomicAdd(&s_q, q);
      } else {
        atomicAdd(&w.vsum[c.e * 4 + 1], cnt);
        atomicAdd(&w.vsum[c.e * 4 + 2], q);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && s_n) {
    atomicAdd(&w.vsum[e0 * 4 + 1], s_n);
    atomicAdd(&w.vsum[e0 * 4 + 2], s_q);
  }
}

__global__ __launch_bounds__(TB) void k_its_vfinal(ItsWs w) {
  const int e = blockIdx.x * TB + threadIdx.x;
  if (e >= w.E) return;
  const unsigned long long n = w.vsum[e * 4 + 1];
  if (w.vpeak[e] >= 0 && n > 0ull) {
    const long long q = (long long)w.vsum[e * 4 + 2];
    w.vzd[e * 2] = (float)((double)q / (double)n / 65536.0);
    w.vzd[e * 2 + 1] = 1.0f;
  } else {
    w.vzd[e * 2] = 0.0f;
    w.vzd[e * 2 + 1] = 0.0f;
  }
}

__global__ __launch_bounds__(TB) void k_its_tl(ItsWs w) {
  const L0 c = l0_cluster(w, (int64_t)blockIdx.x * kPerWg + threadIdx.x / kGrp);
  const int gl = threadIdx.x % kGrp;
  if (!c.ok) return;   // (group-uniform)
  const float vz = w.vzd[c.e * 2];
  const float itp2 = 1.0f / (w.P.trk_sin_phi * w.P.trk_sin_phi);
  const float itt2 = 1.0f / (w.P.trk_dtgl * w.P.trk_dtgl);
  unsigned long long best = ~0ull;
  for_l1(w, c, gl, [&](const float4& b, uint32_t pos) {
    float cr;
    if (!spd_pair(c, b, w.P.trk_sin_phi, cr)) return;
    const float dt = (b.w - vz) / b.z - (c.z - vz) / c.R;
    if (!(fabsf(dt) <= w.P.trk_dtgl)) return;
    const float sp = cr / (c.R * b.z);
    const float sc = (sp * sp) * itp2 + (dt * dt) * itt2;
    const unsigned long long hi = (unsigned long long)__float_as_uint(sc) << 32;
    const uint32_t j = w.slist[pos];
    best = min(best, hi | j);
    atomicMin(&w.best1[j], hi | c.id);
  });
  best = grp_min(best);
  if (gl == 0) w.best0[c.id] = best;
}

__global__ __launch_bounds__(TB) void k_its_tlflag(ItsWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i >= w.n) return;
  uint32_t f = 0u;
  if (w.cl[i] == 0 && w.err[0] == 0u) {
    const unsigned long long b = w.best0[i];
    if (b != ~0ull) {
      const uint32_t j = (uint32_t)(b & 0xFFFFFFFFull);
      f = (uint32_t)(w.best1[j] & 0xFFFFFFFFull) == (uint32_t)i ? 1u : 0u;
    }
  }
  w.tflag[i] = f;
}

// Tracklets in id order (events in order): the global list, the event's
// first tracklet, and the callers' lists (event-local ids).
__global__ __launch_bounds__(TB) void k_its_tlcompact(ItsWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i < w.E + 1) w.toff[i] = w.tflag[i < w.E ? w.ev[i].off : w.n];
  if (i >= w.n) return;
  const uint32_t a = w.tflag[i], b = w.tflag[i + 1];
  if (b == a) return;
  const int e = w.cev[i];
  const uint32_t j = (uint32_t)(w.best0[i] & 0xFFFFFFFFull);
  w.tl0[a] = (int32_t)i;
  w.tl1[a] = (int32_t)j;
  w.tev[a] = e;
  const int64_t off = w.ev[e].off;
  const int64_t t = (int64_t)a - (int64_t)w.tflag[off];
  const tpcca_its_tracks& o = w.out[e];
  if (t < o.cap) {
    o.tl0[t] = (int32_t)(i - off);
    o.tl1[t] = (int32_t)((int64_t)j - off);
  }
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

// Following and inward fit of one tracklet by a group of kGrpF lanes: every
// lane of the group evaluates the same state (the same expressions, so the
// same values), the cluster search of a layer is split over the lanes and
// its result is the group minimum of (chi2 bits, id); lane 0 writes.

__global__ __launch_bounds__(64) void k_its_follow(ItsWs w) {
  const int64_t a = (int64_t)blockIdx.x * (64 / kGrpF) + threadIdx.x / kGrpF;
  const int gl = threadIdx.x % kGrpF;
  if (a >= (int64_t)w.tflag[w.n]) return;   // (the whole group)
  const int e = w.tev[a];
  const int64_t t = a - (int64_t)w.toff[e];
  const tpcca_its_tracks& o = w.out[e];
  if (t >= o.cap) return;
  const int64_t off = w.ev[e].off;
  const ItsTab* tb = w.tab;
  const int64_t ia = w.tl0[a], ib = w.tl1[a];
  const float vz = w.vzd[e * 2];
  Model m = w.m;
  const float ax = w.cx[ia], ay = w.cy[ia], az = w.cz[ia];
  const int ka = w.ck[ia], kb = w.ck[ib];
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
  p[3] = (w.cz[ib] - az) / lab;
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
    const float hx = w.cx[h];
    if (!transport(p, C, xc, hx, m)) { alive = false; break; }
    xc = hx;
    m.vy = w.vy[l]; m.vz = w.vz[l];
    update(p, C, w.cy[h], w.cz[h], m, chi2);
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
    const float cut = w.P.chi2_cut;
    unsigned long long best = ~0ull;
    const uint32_t sa = w.scnt[sidx(e, l, k)], sb = w.scnt[sidx(e, l, k) + 1];
    constexpr int kU = 4;
    for (uint32_t j0 = sa + (uint32_t)gl; j0 < sb; j0 += kU * kGrpF) {
      float4 rc[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const uint32_t j = j0 + (uint32_t)(u * kGrpF);
        rc[u] = w.sB[j < sb ? j : sa];
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (j0 + (uint32_t)(u * kGrpF) >= sb) continue;
        const float dy = rc[u].x - p[0], dz = rc[u].y - p[1];
        const float ch = (dy * dy) * isy + (dz * dz) * isz;
        if (ch <= cut) best = min(best, ((unsigned long long)__float_as_uint(ch) << 32) | __float_as_uint(rc[u].z));
      }
    }
    best = grp_min<kGrpF>(best);
    const int32_t bid = best == ~0ull ? -1 : (int32_t)(best & 0xFFFFFFFFull);
    if (bid >= 0) {
      m.vy = w.vy[l]; m.vz = w.vz[l];
      update(p, C, w.cy[bid], w.cz[bid], m, chi2);
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
  if (gl != 0) return;   // (the group's results are identical; lane 0 writes)
  int32_t* cls = o.cls + t * 6;
  if (rejected || ncl < w.P.min_clusters) {
    o.ok[t] = 0;
    o.in_ok[t] = 0;
    o.ncls[t] = 0;
    o.chi2[t] = 0.0f;
    o.out_layer[t] = -1; o.out_stave[t] = -1; o.in_stave[t] = -1;
#pragma unroll
    for (int i = 0; i < 6; ++i) cls[i] = -1;
    return;
  }
  o.ok[t] = 1;
  o.ncls[t] = ncl;
  o.chi2[t] = chi2;
  o.out_layer[t] = lc;
  o.out_stave[t] = kc;
  o.out_x[t] = xc;
#pragma unroll
  for (int i = 0; i < 6; ++i) cls[i] = cl[i] >= 0 ? (int32_t)(cl[i] - off) : -1;
#pragma unroll
  for (int i = 0; i < 5; ++i) o.out_p[t * 5 + i] = p[i];
#pragma unroll
  for (int i = 0; i < 15; ++i) o.out_cov[t * 15 + i] = C[i];
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
      update(q, Q, w.cy[cl[l]], w.cz[cl[l]], m, dummy);
    }
    its_ms(q, Q, w.xx0[l], w.kms[l]);
  }
  if (iok && transport(q, Q, xq, 0.0f, m)) {
    o.in_ok[t] = 1;
    o.in_stave[t] = kst[0];
#pragma unroll
    for (int i = 0; i < 5; ++i) o.in_p[t * 5 + i] = q[i];
#pragma unroll
    for (int i = 0; i < 15; ++i) o.in_cov[t * 15 + i] = Q[i];
  } else {
    o.in_ok[t] = 0;
    o.in_stave[t] = -1;
  }
}

// Vertex fit: one 512-thread workgroup per event.  Thread tid owns tracks
// tid + k * TBV (k < kVReg) and keeps their lines (point, direction,
// variance) and weights in registers for all solves; tracks past kVReg TBV
// are recomputed from memory in each pass.  Per solve each thread sums its
// tracks in order, the waves sum their lanes by a fixed butterfly and thread
// 0 adds the waves in order, so the result does not depend on timing.
constexpr int TBV = 512;
constexpr int kVReg = 4;

struct VLine { double P[3], d[3], s2; };

__device__ __forceinline__ VLine its_line(const ItsTab* tb, const tpcca_its_tracks& o, int64_t t) {
  VLine L;
  const int k = o.in_stave[t];
  const double ca = tb->ca[0][k], sa = tb->sa[0][k];
  const double yy = o.in_p[t * 5 + 0], zz = o.in_p[t * 5 + 1];
  const double sn = o.in_p[t * 5 + 2], tt = o.in_p[t * 5 + 3];
  const double cc = sqrt(1.0 - sn * sn), nn = sqrt(1.0 + tt * tt);
  L.P[0] = -(yy * sa); L.P[1] = yy * ca; L.P[2] = zz;
  L.d[0] = (cc * ca - sn * sa) / nn; L.d[1] = (cc * sa + sn * ca) / nn; L.d[2] = tt / nn;
  L.s2 = 0.5 * ((double)o.in_cov[t * 15 + 0] + (double)o.in_cov[t * 15 + 5]);
  return L;
}

// A[0..5] (xx, xy, xz, yy, yz, zz) and b[0..2] += the track's weighted terms
__device__ __forceinline__ void vfit_acc(const VLine& L, double wgt, double acc[9]) {
  const double f = wgt / L.s2;
  double M[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c2 = 0; c2 < 3; ++c2) M[r][c2] = (r == c2 ? 1.0 : 0.0) - L.d[r] * L.d[c2];
  acc[0] += f * M[0][0]; acc[1] += f * M[0][1]; acc[2] += f * M[0][2];
  acc[3] += f * M[1][1]; acc[4] += f * M[1][2]; acc[5] += f * M[2][2];
#pragma unroll
  for (int r = 0; r < 3; ++r) acc[6 + r] += f * (M[r][0] * L.P[0] + M[r][1] * L.P[1] + M[r][2] * L.P[2]);
}

__device__ __forceinline__ double bisquare(const VLine& L, const double V[3], double c) {
  const double u0 = V[0] - L.P[0], u1 = V[1] - L.P[1], u2 = V[2] - L.P[2];
  const double pr = u0 * L.d[0] + u1 * L.d[1] + u2 * L.d[2];
  const double e0 = u0 - pr * L.d[0], e1 = u1 - pr * L.d[1], e2 = u2 - pr * L.d[2];
  const double D = sqrt((e0 * e0 + e1 * e1 + e2 * e2) / L.s2) / c;
  return D < 1.0 ? (1.0 - D * D) * (1.0 - D * D) : 0.0;
}

__device__ __forceinline__ double shfl_xor_d(double v, int m) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)(u & 0xFFFFFFFFull), m, 64);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(u >> 32), m, 64);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sums of n values over the workgroup, returned to every thread (s: LDS of
// n * TBV / 64 doubles, out: LDS of n doubles).
template <int N>
__device__ __forceinline__ void vfit_sum(double v[N], double* s, double* out) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1)
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] += shfl_xor_d(v[j], m);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int j = 0; j < N; ++j) s[j * (TBV / 64) + wv] = v[j];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double a = 0.0;
      for (int q = 0; q < TBV / 64; ++q) a += s[j * (TBV / 64) + q];
      out[j] = a;
    }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = out[j];
  __syncthreads();   // (s and out are reused by the next sum)
}

__global__ __launch_bounds__(TBV) void k_its_vfit(ItsWs w) {
  __shared__ double s[9 * (TBV / 64)];
  __shared__ double out[9];
  __shared__ double V[3];
  __shared__ int good;
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  const tpcca_its_tracks& o = w.out[e];
  const int64_t T = std::min<int64_t>((int64_t)(w.toff[e + 1] - w.toff[e]), o.cap);
  double* vw = w.vw + w.toff[e];
  const ItsTab* tb = w.tab;
  VLine L[kVReg];
  double wr[kVReg];
  bool use[kVReg];
  double c1[1] = {0.0};
#pragma unroll
  for (int k = 0; k < kVReg; ++k) {
    const int64_t t = tid + (int64_t)k * TBV;
    use[k] = t < T && o.ok[t] && o.in_ok[t];
    if (use[k]) L[k] = its_line(tb, o, t);
    wr[k] = use[k] ? 1.0 : 0.0;
    c1[0] += use[k] ? 1.0 : 0.0;
  }
  for (int64_t t = tid + (int64_t)kVReg * TBV; t < T; t += TBV) {
    const bool u = o.ok[t] && o.in_ok[t];
    vw[t] = u ? 1.0 : 0.0;
    c1[0] += u ? 1.0 : 0.0;
  }
  vfit_sum<1>(c1, s, out);
  if (tid == 0) { good = c1[0] >= 2.0 ? 1 : 0; V[0] = V[1] = V[2] = 0.0; }
  __syncthreads();
  double nused = 0.0, sumw = 0.0;
  for (int it = 0; it < w.P.fit_iters && good; ++it) {
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < kVReg; ++k)
      if (use[k]) vfit_acc(L[k], wr[k], acc);
    for (int64_t t = tid + (int64_t)kVReg * TBV; t < T; t += TBV)
      if (o.ok[t] && o.in_ok[t]) vfit_acc(its_line(tb, o, t), vw[t], acc);
    vfit_sum<9>(acc, s, out);
    if (tid == 0) {
      const double a00 = acc[0], a01 = acc[1], a02 = acc[2], a11 = acc[3], a12 = acc[4], a22 = acc[5];
      const double b0 = acc[6], b1 = acc[7], b2 = acc[8];
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
    const double Vl[3] = {V[0], V[1], V[2]};
    double nw[2] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kVReg; ++k)
      if (use[k]) {
        wr[k] = bisquare(L[k], Vl, (double)w.P.tukey_c);
        nw[0] += wr[k] > 0.0 ? 1.0 : 0.0;
        nw[1] += wr[k];
      }
    for (int64_t t = tid + (int64_t)kVReg * TBV; t < T; t += TBV)
      if (o.ok[t] && o.in_ok[t]) {
        const double wt = bisquare(its_line(tb, o, t), Vl, (double)w.P.tukey_c);
        vw[t] = wt;
        nw[0] += wt > 0.0 ? 1.0 : 0.0;
        nw[1] += wt;
      }
    vfit_sum<2>(nw, s, out);
    nused = nw[0];
    sumw = nw[1];
  }
  if (tid == 0) {
    double* r = w.vres + e * 8;
    r[0] = V[0]; r[1] = V[1]; r[2] = V[2];
    r[3] = sumw; r[4] = nused; r[5] = good ? 1.0 : 0.0;
  }
}

inline unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>((n + TB - 1) / TB, 1); }

hipError_t run_its(const ItsWs& w, hipStream_t st) {
  const unsigned g = grid_for(w.n);
  const int64_t ns = (int64_t)w.E * kPerEv;
  const int64_t ninit = std::max<int64_t>(std::max<int64_t>(w.n, (int64_t)w.E * w.nbins), std::max<int64_t>(ns + 1, 4 * w.E));
  k_its_init<<<grid_for(ninit), TB, 0, st>>>(w);
  k_its_gather<<<g, TB, 0, st>>>(w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_exclusive_u32(w.scnt, w.scnt, ns, w.part, st);
  if (e != hipSuccess) return e;
  e = scan_exclusive_u32(w.l0f, w.l0f, w.n, w.part, st);
  if (e != hipSuccess) return e;
  k_its_cursors<<<grid_for(ns), TB, 0, st>>>(w);
  k_its_fill<<<g, TB, 0, st>>>(w);
  const unsigned gg = grid_for(w.n * kGrp);   // (kGrp lanes per layer-0 cluster)
  k_its_vpairs<<<gg, TB, 0, st>>>(w);
  k_its_vpeak<<<(unsigned)w.E, TB, 0, st>>>(w);
  k_its_vsum<<<gg, TB, 0, st>>>(w);
  k_its_vfinal<<<grid_for(w.E), TB, 0, st>>>(w);
  k_its_tl<<<gg, TB, 0, st>>>(w);
  k_its_tlflag<<<g, TB, 0, st>>>(w);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_exclusive_u32(w.tflag, w.tflag, w.n, w.part, st);
  if (e != hipSuccess) return e;
  k_its_tlcompact<<<grid_for(std::max<int64_t>(w.n, w.E + 1)), TB, 0, st>>>(w);
  k_its_follow<<<(unsigned)std::max<int64_t>((w.n + 64 / kGrpF - 1) / (64 / kGrpF), 1), 64, 0, st>>>(w);
  k_its_vfit<<<(unsigned)w.E, TBV, 0, st>>>(w);
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

int tpcca_its_track_batch(tpcca_its_ctx* c, int32_t E, const tpcca_its_clusters* ev, tpcca_its_tracks* outs) {
  if (!c) return TPCCA_E_INVALID;
  if (E < 1 || !ev || !outs) return its_fail(c, TPCCA_E_INVALID, "need events and outputs");
  int64_t n = 0;
  for (int e = 0; e < E; ++e) {
    const tpcca_its_clusters& k = ev[e];
    if (k.n < 0 || (k.n > 0 && (!k.x || !k.y || !k.z || !k.layer || !k.stave)))
      return its_fail(c, TPCCA_E_INVALID, "event " + std::to_string(e) + ": null cluster array or bad size");
    if (k.stream != ev[0].stream) return its_fail(c, TPCCA_E_INVALID, "all events must share one stream");
    const tpcca_its_tracks& o = outs[e];
    if (o.cap < 0 || (o.cap > 0 && (!o.tl0 || !o.tl1 || !o.ok || !o.cls || !o.ncls || !o.chi2 || !o.out_layer ||
                                    !o.out_stave || !o.out_x || !o.out_p || !o.out_cov || !o.in_ok ||
                                    !o.in_stave || !o.in_p || !o.in_cov)))
      return its_fail(c, TPCCA_E_INVALID, "event " + std::to_string(e) + ": null output array");
    n += k.n;
  }
  if (n >= ((int64_t)1 << 31)) return its_fail(c, TPCCA_E_INVALID, "more than 2^31 clusters in one call");
  hipError_t he = hipSetDevice(c->device);
  if (he != hipSuccess) return its_fail(c, TPCCA_E_DEVICE, "hipSetDevice");
  hipStream_t st = (hipStream_t)ev[0].stream;
  const int nbins = (int)std::lrint(2.0 * (double)c->P.vtx_range / (double)c->P.vtx_bin);
  // workspace
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t at = off; off += (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255; return at; };
  const int64_t nn = std::max<int64_t>(n, 1);
  const int64_t ns = (int64_t)E * kPerEv;
  // the event and output tables back to back (one upload), the per-event
  // results back to back (one download)
  const size_t up_ev = sizeof(ItsEvIn) * (E + 1), up_bytes = up_ev + sizeof(tpcca_its_tracks) * E;
  const size_t r_vsum = 0, r_vres = r_vsum + 8 * 4 * (size_t)E, r_vzd = r_vres + 8 * 8 * (size_t)E;
  const size_t r_pk = r_vzd + 8 * (size_t)E, r_toff = r_pk + 4 * (size_t)E, r_err = r_toff + 4 * ((size_t)E + 1);
  const size_t res_bytes = r_err + 8;
  const size_t o_up = take(up_bytes), o_res = take(res_bytes);
  const size_t o_cx = take(4 * nn), o_cy = take(4 * nn), o_cz = take(4 * nn), o_cl = take(nn), o_ck = take(2 * nn);
  const size_t o_cev = take(4 * nn), o_X = take(4 * nn), o_Y = take(4 * nn), o_R = take(4 * nn);
  const size_t o_scnt = take(4 * (ns + 1)), o_scur = take(4 * ns), o_slist = take(4 * nn);
  const size_t o_sA = take(16 * nn), o_sB = take(16 * nn), o_l0f = take(4 * (nn + 1)), o_l0l = take(4 * nn);
  const size_t o_hist = take(4 * (int64_t)E * nbins);
  const size_t o_b0 = take(8 * nn), o_b1 = take(8 * nn), o_tf = take(4 * (nn + 1));
  const size_t o_tl0 = take(4 * nn), o_tl1 = take(4 * nn), o_tev = take(4 * nn);
  const size_t o_vw = take(8 * nn);
  const size_t o_part = take(4 * (2 * (std::max<int64_t>(nn, ns) / 1024 + 2)));
  if (off > c->arena_bytes) {
    if (c->arena) { (void)hipFree(c->arena); c->arena = nullptr; c->arena_bytes = 0; }
    if (hipMalloc((void**)&c->arena, off + off / 4) != hipSuccess) {
      (void)hipGetLastError();
      return its_fail(c, TPCCA_E_NOMEM, "ITS workspace allocation failed");
    }
    c->arena_bytes = off + off / 4;
  }
  if (std::max(up_bytes, res_bytes) > c->hpin_bytes) {
    if (c->hpin) { (void)hipHostFree(c->hpin); c->hpin = nullptr; c->hpin_bytes = 0; }
    const size_t hb = std::max(up_bytes, res_bytes) * 2;
    if (hipHostMalloc((void**)&c->hpin, hb) != hipSuccess) {
      (void)hipGetLastError();
      c->hpin = nullptr;
      return its_fail(c, TPCCA_E_NOMEM, "ITS staging allocation failed");
    }
    c->hpin_bytes = hb;
  }
  char* b = c->arena;
  // per-event tables (the input pointers of an empty event still point at
  // valid memory; they are never read)
  ItsEvIn* tin = (ItsEvIn*)c->hpin;
  tpcca_its_tracks* tout = (tpcca_its_tracks*)(c->hpin + up_ev);
  std::copy(outs, outs + E, tout);
  int64_t acc = 0;
  for (int e = 0; e < E; ++e) {
    const tpcca_its_clusters& k = ev[e];
    tin[e] = ItsEvIn{k.n ? k.x : (const float*)b, k.n ? k.y : (const float*)b, k.n ? k.z : (const float*)b,
                     k.n ? k.layer : (const int8_t*)b, k.n ? k.stave : (const int16_t*)b, acc};
    acc += k.n;
    if (tout[e].cap == 0) {   // (valid pointers for the kernels' checks)
      tpcca_its_tracks& o = tout[e];
      o.tl0 = o.tl1 = o.ok = o.ncls = o.out_layer = o.out_stave = o.in_ok = o.in_stave = o.cls = (int32_t*)b;
      o.chi2 = o.out_x = o.out_p = o.out_cov = o.in_p = o.in_cov = (float*)b;
    }
  }
  tin[E] = ItsEvIn{nullptr, nullptr, nullptr, nullptr, nullptr, acc};
  ItsWs w{};
  w.E = E; w.n = n;
  w.ev = (const ItsEvIn*)(b + o_up);
  w.out = (tpcca_its_tracks*)(b + o_up + up_ev);
  w.tab = (const ItsTab*)c->tab;
  for (int l = 0; l < kLayers; ++l) {
    w.r[l] = c->g.radius[l]; w.xx0[l] = c->g.x_over_x0[l];
    w.vy[l] = c->g.sigma_y[l] * c->g.sigma_y[l]; w.vz[l] = c->g.sigma_z[l] * c->g.sigma_z[l];
    w.kms[l] = (float)(1.0 + 0.038 * std::log((double)c->g.x_over_x0[l]));
    w.ns[l] = c->g.n_staves[l];
  }
  w.m.kfac = -(float)((double)2.99792458e-3) * c->g.bz;
  w.m.sin_max = c->P.sin_max;
  w.m.vy = 0.0f; w.m.vz = 0.0f;
  w.P = c->P;
  w.nbins = nbins;
  w.cx = (float*)(b + o_cx); w.cy = (float*)(b + o_cy); w.cz = (float*)(b + o_cz);
  w.cl = (int8_t*)(b + o_cl); w.ck = (int16_t*)(b + o_ck); w.cev = (int32_t*)(b + o_cev);
  w.cX = (float*)(b + o_X); w.cY = (float*)(b + o_Y); w.cR = (float*)(b + o_R);
  w.err = (uint32_t*)(b + o_res + r_err); w.scnt = (uint32_t*)(b + o_scnt); w.scur = (uint32_t*)(b + o_scur);
  w.slist = (uint32_t*)(b + o_slist); w.sA = (float4*)(b + o_sA); w.sB = (float4*)(b + o_sB);
  w.l0f = (uint32_t*)(b + o_l0f); w.l0list = (uint32_t*)(b + o_l0l);
  w.hist = (uint32_t*)(b + o_hist); w.vsum = (unsigned long long*)(b + o_res + r_vsum);
  w.vzd = (float*)(b + o_res + r_vzd); w.vpeak = (int32_t*)(b + o_res + r_pk);
  w.best0 = (unsigned long long*)(b + o_b0); w.best1 = (unsigned long long*)(b + o_b1);
  w.tflag = (uint32_t*)(b + o_tf); w.tl0 = (int32_t*)(b + o_tl0); w.tl1 = (int32_t*)(b + o_tl1);
  w.tev = (int32_t*)(b + o_tev); w.toff = (uint32_t*)(b + o_res + r_toff);
  w.vw = (double*)(b + o_vw); w.vres = (double*)(b + o_res + r_vres); w.part = (uint32_t*)(b + o_part);
  he = hipMemcpyAsync(b + o_up, c->hpin, up_bytes, hipMemcpyHostToDevice, st);
  if (he == hipSuccess) he = run_its(w, st);
  if (he != hipSuccess) {
    (void)hipStreamSynchronize(st);
    return its_fail(c, TPCCA_E_DEVICE, std::string("ITS kernels: ") + hipGetErrorString(he));
  }
  // (the upload has been read by the kernels once the stream passes them:
  // the staging buffer takes the results now)
  he = hipMemcpyAsync(c->hpin, b + o_res, res_bytes, hipMemcpyDeviceToHost, st);
  for (int e = 0; e < E && he == hipSuccess; ++e)
    if (outs[e].hist)
      he = hipMemcpyAsync(outs[e].hist, w.hist + (int64_t)e * nbins, 4 * (size_t)nbins, hipMemcpyDeviceToDevice, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) return its_fail(c, TPCCA_E_DEVICE, std::string("ITS results: ") + hipGetErrorString(he));
  const unsigned long long* vs = (const unsigned long long*)(c->hpin + r_vsum);
  const double* vr = (const double*)(c->hpin + r_vres);
  const float* vz = (const float*)(c->hpin + r_vzd);
  const int32_t* pk = (const int32_t*)(c->hpin + r_pk);
  const uint32_t* toff = (const uint32_t*)(c->hpin + r_toff);
  const uint32_t err = *(const uint32_t*)(c->hpin + r_err);
  if (err) return its_fail(c, TPCCA_E_INVALID, "a cluster has a bad layer or stave or a non-finite coordinate");
  bool fits = true;
  for (int e = 0; e < E; ++e) {
    tpcca_its_tracks& o = outs[e];
    o.n_tracklets = (int64_t)(toff[e + 1] - toff[e]);
    fits = fits && o.n_tracklets <= o.cap;
    o.n_pairs = (int64_t)vs[4 * e];
    o.peak = pk[e];
    o.vz = vz[2 * e];
    o.vz_ok = vz[2 * e + 1] != 0.0f ? 1 : 0;
    o.vertex[0] = vr[8 * e]; o.vertex[1] = vr[8 * e + 1]; o.vertex[2] = vr[8 * e + 2];
    o.vfit_sumw = vr[8 * e + 3];
    o.vfit_n = (int32_t)vr[8 * e + 4];
    o.vfit_ok = vr[8 * e + 5] != 0.0 ? 1 : 0;
  }
  if (!fits) return its_fail(c, TPCCA_E_CAPACITY, "more tracklets than an event's output holds");
  return TPCCA_OK;
}

int tpcca_its_track(tpcca_its_ctx* c, const tpcca_its_clusters* cl, tpcca_its_tracks* o) {
  if (!c) return TPCCA_E_INVALID;
  if (!cl || !o) return its_fail(c, TPCCA_E_INVALID, "null clusters or output");
  return tpcca_its_track_batch(c, 1, cl, o);
}

const char* tpcca_its_last_error(const tpcca_its_ctx* c) { return c ? c->err.c_str() : "null context"; }

void tpcca_its_destroy(tpcca_its_ctx* c) {
  if (!c) return;
  if (c->arena) (void)hipFree(c->arena);
  if (c->tab) (void)hipFree(c->tab);
  if (c->hpin) (void)hipHostFree(c->hpin);
  delete c;
}

}  // extern "C"
