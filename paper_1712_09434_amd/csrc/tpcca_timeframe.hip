// tpcca_timeframe.hip -- slicing of continuous-readout time frames on gfx950.
//
// Paper, Sec. "Track reconstruction in the TPC": with continuous readout the
// TPC delivers time frames of overlapping collisions; they can be sliced
// along the time (beam) axis, the slices processed individually and the
// track segments merged afterwards.  A cluster of a frame carries its
// readout time tau (cm of drift since the frame start) instead of z.  The
// library's reading: slice s = floor(tau / D) (FP32 quotient), no overlap;
// inside its slice a cluster is tracked with z' = side (L - (tau - s D)),
// which is z shifted by a constant per collision, so every track stays a
// helix; segments are taken to frame coordinates z_tf = side (L - tau).
//
// Kernels: per-workgroup slice histograms (LDS), one exclusive scan over
// (slice, workgroup), a stable scatter into slice order (ranks within a wave
// by matching the slice bits over ballots, waves of a workgroup in order),
// and after the per-slice tracking the gather of every slice's tracks into
// one contiguous segment set in frame coordinates.
#include "timeframe_internal.hpp"

namespace tpcca {
namespace {

constexpr int TB = 256;
constexpr int kRounds = kTfBlock / TB;

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << (threadIdx.x & 63)) - 1ull; }

// Slice of a readout time; false for a non-finite or negative tau or one
// past the last slice.
__device__ __forceinline__ bool slice_of(float tau, float D, int n_slices, int& s) {
  const float q = tau / D;
  if (!(q >= 0.0f) || !(q < (float)n_slices)) return false;
  s = (int)floorf(q);
  return s < n_slices;
}

__global__ __launch_bounds__(TB) void k_tf_count(TfSlice a) {
  __shared__ uint32_t h[kTfMaxSlices];
  for (int s = threadIdx.x; s < a.n_slices; s += TB) h[s] = 0u;
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * kTfBlock;
  float tv[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = b0 + r * TB + threadIdx.x;
    tv[r] = i < a.n ? a.tau[i] : 0.0f;
  }
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = b0 + r * TB + threadIdx.x;
    if (i < a.n) {
      int s = 0;
      if (slice_of(tv[r], a.D, a.n_slices, s)) atomicAdd(&h[s], 1u);
      else atomicOr(a.err, 1u);
    }
  }
  __syncthreads();
  for (int s = threadIdx.x; s < a.n_slices; s += TB) a.cnt[(int64_t)s * a.nb + blockIdx.x] = h[s];
}

// Stable scatter: the workgroup's clusters in frame order go to the scanned
// (slice, workgroup) offsets; within a round of TB clusters each wave ranks
// its lanes among those of the same slice, and the waves take their places
// in order from running per-slice cursors in LDS.
__global__ __launch_bounds__(TB) void k_tf_scatter(TfSlice a) {
  __shared__ uint32_t run[kTfMaxSlices];
  for (int s = threadIdx.x; s < a.n_slices; s += TB) run[s] = a.cnt[(int64_t)s * a.nb + blockIdx.x];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int nbits = 0;
  while ((1 << nbits) < a.n_slices) ++nbits;
  const int64_t b0 = (int64_t)blockIdx.x * kTfBlock;
  float tv[kRounds], xv[kRounds], yv[kRounds];
  int16_t rv[kRounds];
  uint8_t sv[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = b0 + r * TB + threadIdx.x;
    const int64_t k = i < a.n ? i : 0;
    tv[r] = a.tau[k]; xv[r] = a.x[k]; yv[r] = a.y[k]; rv[r] = a.row[k]; sv[r] = a.sector[k];
  }
  __syncthreads();
  const float L = a.L, D = a.D;
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = b0 + r * TB + threadIdx.x;
    int s = 0;
    const bool ok = i < a.n && slice_of(tv[r], D, a.n_slices, s);
    // lanes of this wave with the same slice: agree on every bit
    uint64_t m = __ballot(ok);
    for (int b = 0; b < nbits; ++b) {
      const bool bit = ok && ((s >> b) & 1);
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(m & lanemask_lt());
    const bool last = ok && (m >> lane) == 1ull;   // the group's highest lane
    const float side = (int)sv[r] < a.half ? 1.0f : -1.0f;
    for (int q = 0; q < TB / 64; ++q) {
      if (wv == q && ok) {
        const uint32_t pos = run[s] + rank;
        if (last) run[s] = pos + 1u;
        const float t1 = (float)s * D;
        a.sx[pos] = xv[r];
        a.sy[pos] = yv[r];
        a.sz[pos] = side * (L - (tv[r] - t1));
        a.srow[pos] = rv[r];
        a.ssec[pos] = sv[r];
        a.sid[pos] = (uint32_t)i;
      }
      __syncthreads();
    }
    if (i < a.n) a.ztf[i] = side * (L - tv[r]);
  }
}

__global__ void k_tf_offsets(TfSlice a) {
  for (int s = threadIdx.x; s <= a.n_slices; s += blockDim.x) a.soff[s] = a.cnt[(int64_t)s * a.nb];
}

// Largest e in [0, E) whose range starts at or before v (the slices holding
// nothing share their start with the next one).
__device__ __forceinline__ int find_range(const TfRange* tab, int E, int64_t v, bool hits) {
  int lo = 0, hi = E - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t st = hits ? tab[mid].hout : tab[mid].tout;
    if (st <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(TB) void k_tf_segs(TfGather g) {
  const int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (t == 0) g.ohoff[g.T] = (int32_t)g.H;
  if (t >= g.T) return;
  const int e = find_range(g.tab, g.E, t, false);
  const TfRange r = g.tab[e];
  const int64_t j = t - r.tout, src = r.tcap + j;
  const uint8_t sec = g.isec[src];
  const float shift = (float)e * g.D;
  g.osec[t] = sec;
  g.oxref[t] = g.ixref[src];
#pragma unroll
  for (int k = 0; k < 5; ++k) g.op[t * 5 + k] = g.ip[src * 5 + k];
  const float p1 = g.ip[src * 5 + 1];
  g.op[t * 5 + 1] = (int)sec < g.half ? p1 - shift : p1 + shift;
#pragma unroll
  for (int k = 0; k < 15; ++k) g.ocov[t * 15 + k] = g.icov[src * 15 + k];
  g.ochi2[t] = g.ichi2[src];
  g.ondf[t] = g.indf[src];
  g.ohoff[t] = (int32_t)(r.hout + g.ihoff[r.hoff + j]);
  g.oslice[t] = e;
}

__global__ __launch_bounds__(TB) void k_tf_hits(TfGather g) {
  const int64_t h = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (h >= g.H) return;
  const int e = find_range(g.tab, g.E, h, true);
  const TfRange r = g.tab[e];
  const uint32_t local = g.ihid[r.hcap + (h - r.hout)];
  g.ohid[h] = g.sid[r.coff + local];
}

inline unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>((n + TB - 1) / TB, 1); }

}  // namespace

hipError_t tf_slice(const TfSlice& a, uint32_t* scan_part, hipStream_t st) {
  const unsigned nb = (unsigned)std::max<int64_t>(a.nb, 1);
  k_tf_count<<<nb, TB, 0, st>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_exclusive_u32(a.cnt, a.cnt, (int64_t)a.n_slices * a.nb, scan_part, st);
  if (e != hipSuccess) return e;
  k_tf_scatter<<<nb, TB, 0, st>>>(a);
  k_tf_offsets<<<1, 256, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t tf_gather(const TfGather& g, hipStream_t st) {
  k_tf_segs<<<grid_for(g.T), TB, 0, st>>>(g);
  if (g.H > 0) k_tf_hits<<<grid_for(g.H), TB, 0, st>>>(g);
  return hipGetLastError();
}

}  // namespace tpcca
