// tpcca_kernels.hip -- the tracking path on gfx950.
//
// Paper, Sec. "Track reconstruction in the TPC": cellular-automaton seeding
// with one thread per cluster, Kalman-filter following with one thread per
// track, every sector independent.  Here every (event, sector) pair is an
// independent unit, so one launch of each phase covers all events of a
// batch.  Phases:
//   a1 binning    count per (event, sector, row) -> scan -> bucket -> per
//                 row: sort by id in LDS, canonical SoA, 2-D (z, y) grid
//   a2 links      one lane per cluster, windows on the adjacent rows' grids
//   a3/a4         reciprocal-link cleaning, start and seed flags, wave ballot
//                 compaction in canonical (event, sector, row, id) order
//   a5 tracklets  one lane per seed: chain fit, upward and downward
//                 following with grid searches
//   a6 selection  64-bit atomicMax ownership per cluster
//   a7 final fit  outermost-to-innermost Kalman refit of the owned hits,
//                 ordered compaction into the caller's flat buffers
#include <algorithm>

#include "internal.hpp"
#include "kf_c2.hpp"

namespace tpcca {
namespace {

constexpr int TB = 256;
constexpr int kXcd = 8;   // accelerator complex dies (each with its own L2) of the chip
constexpr int kBackRows = 32;   // longest transport (rows) back to a seed's first row
constexpr int kRefillMin = 16;  // waiting lanes that make a wave take new seeds

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// Exclusive scan over a 256-thread block; *tot receives the block total.
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t* tot) {
  __shared__ uint32_t s_w[TB / 64];
  const uint32_t inc = wave_incl_scan(v);
  const int wid = threadIdx.x >> 6;
  if (lane_id() == 63) s_w[wid] = inc;
  __syncthreads();
  uint32_t base = 0, total = 0;
#pragma unroll
  for (int i = 0; i < TB / 64; ++i) {
    const uint32_t t = s_w[i];
    if (i < wid) base += t;
    total += t;
  }
  __syncthreads();
  *tot = total;
  return base + inc - v;
}

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// ---------------------------------------------------------------- utilities
__global__ void k_fill(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) p[i] = v;
}

// Two ranges cleared by one launch.
__global__ void k_zero2(uint32_t* __restrict__ p, int64_t n, uint32_t* __restrict__ q, int64_t m) {
  for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n + m; i += (int64_t)gridDim.x * TB) {
    if (i < n) p[i] = 0u;
    else q[i - n] = 0u;
  }
}

// Exclusive scans, out[n] = total (out may equal in).  Up to two arrays of
// the same length are scanned by the same launches (blockIdx.y selects the
// array): one workgroup each when n <= kScanSmall, else reduce / partials /
// down-sweep over tiles of 1024.
struct ScanArgs {
  const uint32_t* in[2];
  uint32_t* out[2];
  int ind[2];   // 1: scan the indicator (value > 0) of the input instead of the value
};
__device__ __forceinline__ uint32_t scan_in(const ScanArgs& a, int y, uint32_t v) {
  return a.ind[y] ? (v > 0u ? 1u : 0u) : v;
}
constexpr int kScanNT = 1024;                        // threads of a one-workgroup scan
constexpr int64_t kScanSmall = 4 * 4 * kScanNT;      // at most four tiles of 4 x kScanNT

// Size classes of row units.  The row and link kernels come in variants by
// row size; with few row units (RU <= kScanSmall, e.g. one event) each
// variant's launch covers every row unit and skips the others, with many
// (batches of events) the binning builds one list per variant and the
// variants other than the wave-per-unit ones run over their list only, so
// that the hundreds of thousands of mostly tiny units of a batch do not
// each cost a workgroup launch in every variant.
constexpr uint32_t kTiny = 64;         // clusters of a row unit handled by one wave, one per lane
constexpr uint32_t kWaveRow = 256;     // clusters of a row unit handled by one wave, four per lane
constexpr uint32_t kSmallSlab = 256;   // neighbour rows staged in the small-LDS link variant
constexpr uint32_t kSlab = 896;        // clusters of one row staged in LDS (3 workgroups per CU fit)
__host__ __device__ inline bool ru_lists(int64_t RU) { return RU > kScanSmall; }
// 0: k_rows_tiny (empty units too), 1: k_rows_wave, 2: k_rows<false>, 3: k_rows<true>
__device__ __forceinline__ int rows_class(uint32_t n) {
  return n <= kTiny ? 0 : n <= kWaveRow ? 1 : n <= 4u * TB ? 2 : 3;
}
// -1: nothing to do (empty), 0/1/2: k_links<kTiny>, <kSmallSlab>, <kSlab>
// (the last also writes the no-link entries of edge rows and over-full units)
__device__ __forceinline__ int links_class(uint32_t n, uint32_t nd, uint32_t nu, bool inner) {
  if (n == 0) return -1;
  if (!inner || n > (uint32_t)kMaxRow) return 2;
  return (nd <= kTiny && nu <= kTiny) ? 0 : (nd <= kSmallSlab && nu <= kSmallSlab) ? 1 : 2;
}
// Workgroups of a list-driven launch (each loops over list entries).
constexpr unsigned kListGrid = 2048, kListGridBig = 1024;

// Exclusive scan over a kScanNT-thread block; *tot receives the block total.
__device__ uint32_t block_excl_scan_big(uint32_t v, uint32_t* tot) {
  __shared__ uint32_t s_w[kScanNT / 64];
  const uint32_t inc = wave_incl_scan(v);
  const int wid = threadIdx.x >> 6;
  if (lane_id() == 63) s_w[wid] = inc;
  __syncthreads();
  uint32_t base = 0, total = 0;
#pragma unroll
  for (int i = 0; i < kScanNT / 64; ++i) {
    const uint32_t t = s_w[i];
    if (i < wid) base += t;
    total += t;
  }
  __syncthreads();
  *tot = total;
  return base + inc - v;
}

__global__ __launch_bounds__(kScanNT) void k_scan_small(ScanArgs a, int64_t n) {
  const uint32_t* in = a.in[blockIdx.x];
  uint32_t* out = a.out[blockIdx.x];
  const uint32_t n32 = (uint32_t)n;   // n <= kScanSmall
  // tiles of four coalesced values per thread with a running carry; past
  // the end a thread reads element 0 and drops it (no branch around loads)
  uint32_t carry = 0;
  for (uint32_t t0 = 0; t0 < n32; t0 += 4u * kScanNT) {
    const uint32_t base = t0 + 4u * threadIdx.x;
    uint32_t v[4], sum = 0;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      const uint32_t x = scan_in(a, blockIdx.x, in[base + j < n32 ? base + j : 0u]);
      v[j] = base + j < n32 ? x : 0u;
      sum += v[j];
    }
    uint32_t tot;
    uint32_t ex = carry + block_excl_scan_big(sum, &tot);
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      if (base + j < n32) out[base + j] = ex;
      ex += v[j];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) out[n32] = carry;
}

// Row-unit offsets in one workgroup (RU <= kScanSmall): scans the counts
// into ru_off and the cell capacities (grid_cells(count) + 1, computed here)
// into cell_base, then clears the counts for their second use as the
// scatter's fill cursors.
__global__ __launch_bounds__(kScanNT) void k_scan_rows(Ws w) {
  const uint32_t n32 = (uint32_t)w.RU;
  uint32_t carry0 = 0, carry1 = 0;
  for (uint32_t t0 = 0; t0 < n32; t0 += 4u * kScanNT) {
    const uint32_t base = t0 + 4u * threadIdx.x;
    uint32_t v0[4], v1[4], s0 = 0, s1 = 0;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      const uint32_t x = w.ru_count[base + j < n32 ? base + j : 0u];
      v0[j] = base + j < n32 ? x : 0u;
      v1[j] = base + j < n32 ? grid_cells(x) + 1u : 0u;
      s0 += v0[j];
      s1 += v1[j];
    }
    uint32_t tot0, tot1;
    uint32_t e0 = carry0 + block_excl_scan_big(s0, &tot0);
    uint32_t e1 = carry1 + block_excl_scan_big(s1, &tot1);
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      if (base + j < n32) {
        w.ru_off[base + j] = e0;
        w.cell_base[base + j] = e1;
        w.ru_count[base + j] = 0u;
      }
      e0 += v0[j];
      e1 += v1[j];
    }
    carry0 += tot0;
    carry1 += tot1;
  }
  if (threadIdx.x == 0) { w.ru_off[n32] = carry0; w.cell_base[n32] = carry1; }
}

__global__ __launch_bounds__(TB) void k_scan_reduce(ScanArgs a, int64_t n, uint32_t* __restrict__ part,
                                                    int64_t pstride) {
  const uint32_t* in = a.in[blockIdx.y];
  part += blockIdx.y * pstride;
  const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) if (base + j < n) s += scan_in(a, blockIdx.y, in[base + j]);
  uint32_t tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(TB) void k_scan_parts(uint32_t* __restrict__ part, int64_t np, int64_t pstride) {
  part += blockIdx.x * pstride;
  uint32_t carry = 0;
  for (int64_t b = 0; b < np; b += TB) {
    const int64_t i = b + threadIdx.x;
    const uint32_t v = i < np ? part[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan(v, &tot);
    if (i < np) part[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) part[np] = carry;
}

__global__ __launch_bounds__(TB) void k_scan_down(ScanArgs a, int64_t n, const uint32_t* __restrict__ part,
                                                  int64_t np, int64_t pstride) {
  const uint32_t* in = a.in[blockIdx.y];
  uint32_t* out = a.out[blockIdx.y];
  part += blockIdx.y * pstride;
  const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
  uint32_t v[4], s = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) { v[j] = base + j < n ? scan_in(a, blockIdx.y, in[base + j]) : 0u; s += v[j]; }
  uint32_t tot;
  uint32_t ex = block_excl_scan(s, &tot) + (blockIdx.x < np ? part[blockIdx.x] : 0u);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (base + j < n) out[base + j] = ex;
    ex += v[j];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = part[np];
}

// Exclusive scans of narr (1 or 2) arrays of n values; part holds
// 2 (n / 1024 + 2) values.
hipError_t scan_arrays(ScanArgs a, int narr, int64_t n, uint32_t* part, hipStream_t st) {
  if (n <= kScanSmall) {
    k_scan_small<<<dim3((unsigned)narr), dim3(kScanNT), 0, st>>>(a, n);
    return hipGetLastError();
  }
  const int64_t np = (n + 1023) / 1024;
  const int64_t ps = np + 2;
  k_scan_reduce<<<dim3((unsigned)np, (unsigned)narr), dim3(TB), 0, st>>>(a, n, part, ps);
  k_scan_parts<<<dim3((unsigned)narr), TB, 0, st>>>(part, np, ps);
  k_scan_down<<<dim3((unsigned)np, (unsigned)narr), dim3(TB), 0, st>>>(a, n, part, np, ps);
  return hipGetLastError();
}

hipError_t scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* part, hipStream_t st) {
  ScanArgs a{{in, in}, {out, out}, {0, 0}};
  return scan_arrays(a, 1, n, part, st);
}

// ind0: the first array is scanned as the indicator of its values.
hipError_t scan_u32x2(const uint32_t* in0, uint32_t* out0, const uint32_t* in1, uint32_t* out1, int64_t n,
                      uint32_t* part, hipStream_t st, int ind0 = 0) {
  ScanArgs a{{in0, in1}, {out0, out1}, {ind0, 0}};
  return scan_arrays(a, 2, n, part, st);
}

inline unsigned blocks_for(int64_t n, int64_t cap = 1 << 16) {
  int64_t b = (n + TB - 1) / TB;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

// A multiple of kXcd workgroups (at most 2^14) for kernels that split their
// work by XCD.
inline unsigned xcd_blocks(int64_t n) {
  const int64_t b = blocks_for(n, 1 << 14);
  return (unsigned)((b + kXcd - 1) / kXcd * kXcd);
}

// ------------------------------------------------------------- a1: binning
// Raw fields of one input cluster, then its validation and row unit.  The
// binning kernels take kGroup clusters per thread at a time and issue all
// their loads before the first is used.
struct RawCl { float x, y, z; int r, s; };

__device__ __forceinline__ RawCl load_cluster(const EventIn& E, int64_t l) {
  return RawCl{E.x[l], E.y[l], E.z[l], (int)E.row[l], (int)E.sector[l]};
}

__device__ __forceinline__ bool check_cluster(const Ws& w, const RawCl& c, int e, int64_t l, uint32_t& ru,
                                              float4& v) {
  if (!(isfinite(c.x) && isfinite(c.y) && isfinite(c.z)) || c.r < 0 || c.r >= w.R || c.s >= w.S) return false;
  ru = ((uint32_t)e * (uint32_t)w.S + (uint32_t)c.s) * (uint32_t)w.R + (uint32_t)c.r;
  v = make_float4(c.x, c.y, c.z, __uint_as_float((uint32_t)l));
  return true;
}

constexpr int kGroup = 4;
// threads of the binning workgroups: a chunk's clusters and bins are spread
// over sixteen waves, so the few hundred chunks of a large event still keep
// several waves on every SIMD
constexpr int TBB = 1024;

// f(ok, ru, v) for every cluster of the chunk [c0, c1) of event e taken by
// this thread (stride TBB), kGroup at a time.
template <class F>
__device__ __forceinline__ void for_chunk(const Ws& w, int64_t c0, int64_t c1, int e, F&& f) {
  const EventIn& E = w.ev[e];
  for (int64_t g0 = c0 + threadIdx.x; g0 < c1; g0 += (int64_t)kGroup * TBB) {
    RawCl c[kGroup];
#pragma unroll
    for (int k = 0; k < kGroup; ++k) {
      const int64_t g = g0 + (int64_t)k * TBB;
      if (g < c1) c[k] = load_cluster(E, g - E.base);
    }
#pragma unroll
    for (int k = 0; k < kGroup; ++k) {
      const int64_t g = g0 + (int64_t)k * TBB;
      if (g >= c1) continue;
      uint32_t ru = 0;
      float4 v;
      const bool ok = check_cluster(w, c[k], e, g - E.base, ru, v);
      f(ok, ru, v);
    }
  }
}

// Binning histograms are privatised in LDS per chunk (up to kChunkCl
// clusters of one event, from the host's chunk table): the bins are the
// event's row units.  Count: one global atomic per non-empty bin.  Scatter:
// one global range reservation per non-empty bin, then LDS ranks.
constexpr int kLdsBins = 8192;

__global__ __launch_bounds__(TBB) void k_count(Ws w) {
  __shared__ uint32_t s_h[kLdsBins];
  const ChunkIn ch = w.chunk[blockIdx.x];
  if (ch.c0 >= ch.c1) return;
  const int64_t c0 = ch.c0, c1 = ch.c1;
  const int e = ch.e;
  const uint32_t per = (uint32_t)w.S * (uint32_t)w.R;
  const bool lds = per <= (uint32_t)kLdsBins;
  const uint32_t rb = (uint32_t)e * per;
  if (lds) for (uint32_t b = threadIdx.x; b < per; b += TBB) s_h[b] = 0u;
  __syncthreads();
  for_chunk(w, c0, c1, e, [&](bool ok, uint32_t ru, const float4&) {
    if (!ok) { atomicOr(&w.flags[F_ERR], ERR_INVALID); return; }
    if (lds && ru - rb < per) atomicAdd(&s_h[ru - rb], 1u);
    else atomicAdd(&w.ru_count[ru], 1u);
  });
  __syncthreads();
  if (lds)
    for (uint32_t b = threadIdx.x; b < per; b += TBB)
      if (s_h[b]) atomicAdd(&w.ru_count[rb + b], s_h[b]);
}

// Appends v to a list (forward from 0, or backward from cap - 1) for every
// lane with p: one atomic per wave.  The order of the entries is not
// defined; every consumer's results are independent of it.
__device__ __forceinline__ void list_push(bool p, uint32_t v, uint32_t* ctr, uint32_t* list, bool backward,
                                          int64_t cap) {
  const uint64_t m = __ballot(p);
  if (m == 0ull) return;
  const int leader = __ffsll((unsigned long long)m) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(ctr, (uint32_t)__popcll(m));
  base = (uint32_t)__shfl((int)base, leader, 64);
  if (p) {
    const uint32_t k = base + (uint32_t)__popcll(m & lanemask_lt());
    list[backward ? cap - 1 - (int64_t)k : (int64_t)k] = v;
  }
}

// cells + 1 offsets per row unit; with many row units also the lists of the
// row and link variants (from the counts, before they are reused as cursors)
__global__ void k_cell_caps(Ws w) {
  const bool lists = ru_lists(w.RU);
  for (int64_t b0 = (int64_t)blockIdx.x * TB; b0 < w.RU; b0 += (int64_t)gridDim.x * TB) {
    const int64_t ru = b0 + threadIdx.x;
    const bool ok = ru < w.RU;
    const uint32_t n = ok ? w.ru_count[ru] : 0u;
    if (ok) w.cell_cap[ru] = grid_cells(n) + 1u;
    if (!lists) continue;
    const int r = ok ? (int)(ru % w.R) : 0;
    const bool inner = r >= 1 && r <= w.R - 2;
    const uint32_t nd = ok && inner ? w.ru_count[ru - 1] : 0u, nu = ok && inner ? w.ru_count[ru + 1] : 0u;
    const int rc = rows_class(n), lc = links_class(n, nd, nu, inner);
    list_push(ok && rc == 1, (uint32_t)ru, &w.flags[F_LROWS1], w.ru_rows, false, w.RU);
    list_push(ok && rc == 2, (uint32_t)ru, &w.flags[F_LROWS2], w.ru_rows, true, w.RU);
    list_push(ok && rc == 3, (uint32_t)ru, &w.flags[F_LROWS3], w.ru_big, false, w.RU);
    list_push(ok && lc == 1, (uint32_t)ru, &w.flags[F_LLINKS1], w.ru_links, false, w.RU);
    list_push(ok && lc == 2, (uint32_t)ru, &w.flags[F_LLINKS2], w.ru_links, true, w.RU);
  }
}

// ru_count is reused as the global fill cursor (zeroed after the scans).
// Each cluster travels with its coordinates and event-local id, so the row
// kernel reads its row unit contiguously instead of gathering from the
// (arbitrarily ordered) input.
__global__ __launch_bounds__(TBB) void k_scatter(Ws w) {
  __shared__ uint32_t s_h[kLdsBins];
  const ChunkIn ch = w.chunk[blockIdx.x];
  if (ch.c0 >= ch.c1) return;
  const int64_t c0 = ch.c0, c1 = ch.c1;
  const int e = ch.e;
  const uint32_t per = (uint32_t)w.S * (uint32_t)w.R;
  const bool lds = per <= (uint32_t)kLdsBins;
  const uint32_t rb = (uint32_t)e * per;
  if (lds) {
    for (uint32_t b = threadIdx.x; b < per; b += TBB) s_h[b] = 0u;
    __syncthreads();
    for_chunk(w, c0, c1, e, [&](bool ok, uint32_t ru, const float4&) {
      if (ok && ru - rb < per) atomicAdd(&s_h[ru - rb], 1u);
    });
    __syncthreads();
    // range reservations: the returning atomics of a thread's bins are all
    // issued before their results are stored
    constexpr int kPer = kLdsBins / TBB;
    uint32_t got[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const uint32_t b = threadIdx.x + (uint32_t)i * TBB;
      const uint32_t n = b < per ? s_h[b] : 0u;
      got[i] = n ? atomicAdd(&w.ru_count[rb + b], n) : 0u;
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const uint32_t b = threadIdx.x + (uint32_t)i * TBB;
      if (b < per) s_h[b] = got[i];
    }
    __syncthreads();
  }
  for_chunk(w, c0, c1, e, [&](bool ok, uint32_t ru, const float4& v) {
    if (!ok) return;
    const uint32_t k = (lds && ru - rb < per) ? atomicAdd(&s_h[ru - rb], 1u) : atomicAdd(&w.ru_count[ru], 1u);
    float4 o = v;
    if (w.cal) {
      // the installed calibration, applied on the way into the row buckets:
      // every later step sees only corrected clusters (the row is kept)
      const int s = (int)((ru / (uint32_t)w.R) % (uint32_t)w.S);
      const int S = w.S;
      const Corrected c = correct_cluster(w.cal_geo, w.cal[s], w.cal[S + s], w.cal + 2 * S + s * 64, s, v.x,
                                          v.y, v.z);
      o.x = c.x;
      o.z = c.z;
    }
    w.tmp4[w.ru_off[ru] + k] = o;
  });
}

__device__ __forceinline__ uint32_t cell_coord(float v, float v0, float inv, uint32_t nc) {
  float t = (v - v0) * inv;
  t = fminf(fmaxf(t, 0.0f), (float)(nc - 1u));
  return (uint32_t)t;
}

__device__ __forceinline__ uint32_t cell_of(const GridParams& G, float y, float z) {
  return cell_coord(z, G.z0, G.inv_bz, G.nz) * G.ny + cell_coord(y, G.y0, G.inv_by, G.ny);
}

// Search grid of a row unit of n clusters with the given bounding box: about
// grid_cells(n) cells of equal shape over the box (one cell if the box is
// degenerate or n < 4).
__device__ __forceinline__ GridParams make_grid(uint32_t n, uint32_t cbase, uint32_t off, float ymin, float ymax,
                                                float zmin, float zmax) {
  const uint32_t cap = grid_cells(n);
  uint32_t nz = 1, ny = 1;
  float dz = zmax - zmin, dy = ymax - ymin;
  if (!(n > 0)) { zmin = 0.f; ymin = 0.f; dz = 0.f; dy = 0.f; }
  if (n >= 4 && dz > 0.0f && dy > 0.0f) {
    const float a = sqrtf((dz * dy) / (float)cap);
    nz = (uint32_t)fminf(fmaxf(dz / a, 1.0f), (float)cap);
    ny = (uint32_t)fminf(fmaxf(dy / a, 1.0f), (float)(cap / nz));
  }
  GridParams G;
  G.cell_base = cbase; G.nz = nz; G.ny = ny; G.z0 = zmin; G.y0 = ymin;
  G.inv_bz = dz > 0.0f ? (float)nz / dz : 0.0f;
  G.inv_by = dy > 0.0f ? (float)ny / dy : 0.0f;
  G.base = off;
  G.off_plane = 0u;
  return G;
}

// One block per row unit: the row unit's (x, y, z, id) entries sorted by id
// in LDS (bitonic on the ids, carrying the entry's slot), canonical SoA
// written in that order, then a uniform 2-D grid over the row's bounding box
// with about two clusters per cell, filled by an LDS counting sort.
// Ordering of LDS accesses between the lanes of one wave (the wave's LDS
// operations complete in order; this waits for them and keeps the compiler
// from moving accesses across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row units of at most 64 clusters (most units of small events): one wave
// each, four per workgroup, no workgroup barrier.  Lane k holds the k-th
// entry: the ids are sorted by a bitonic network over lane shuffles, the
// coordinates follow by a gather from the lane that held them; the grid is
// built as in k_rows with a per-wave LDS histogram.  Same results as k_rows.
__global__ __launch_bounds__(TB) void k_rows_tiny(Ws w) {
  __shared__ uint32_t s_h[TB / 64][kCellsPerCluster * kTiny + 2];
  const int wv = threadIdx.x >> 6, lane = lane_id();
  const int64_t ru = (int64_t)blockIdx.x * (TB / 64) + wv;
  if (ru >= w.RU) return;
  const uint32_t off = w.ru_off[ru];
  const uint32_t n = w.ru_off[ru + 1] - off;
  if (n > kTiny) return;
  const uint32_t cbase = w.cell_base[ru];
  uint32_t* hist = s_h[wv];
  float x0 = 0.f, y0 = 0.f, z0 = 0.f;
  uint32_t key = 0xFFFFFFFFu, slot = (uint32_t)lane;
  if ((uint32_t)lane < n) {
    const float4 v = w.tmp4[off + lane];
    x0 = v.x; y0 = v.y; z0 = v.z; key = __float_as_uint(v.w);
  }
  uint32_t npad = 2;
  while (npad < n) npad <<= 1;
  for (uint32_t kk = 2; kk <= npad; kk <<= 1) {
    for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
      const uint32_t o = (uint32_t)__shfl_xor((int)key, (int)j, 64);
      const uint32_t os = (uint32_t)__shfl_xor((int)slot, (int)j, 64);
      const bool lower = ((uint32_t)lane & j) == 0, asc = ((uint32_t)lane & kk) == 0;
      const uint32_t lo = lower ? key : o, hi = lower ? o : key;
      if (asc ? lo > hi : lo < hi) { key = o; slot = os; }
    }
  }
  const float x = __shfl(x0, (int)slot, 64), y = __shfl(y0, (int)slot, 64), z = __shfl(z0, (int)slot, 64);
  const bool mine = (uint32_t)lane < n;
  if (mine) {
    w.cx[off + lane] = x; w.cy[off + lane] = y; w.cz[off + lane] = z;
    w.cid[off + lane] = key; w.cru[off + lane] = (uint32_t)ru;
  }
  float ymin = mine ? y : INFINITY, ymax = mine ? y : -INFINITY;
  float zmin = mine ? z : INFINITY, zmax = mine ? z : -INFINITY;
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    ymin = fminf(ymin, __shfl_xor(ymin, d, 64)); ymax = fmaxf(ymax, __shfl_xor(ymax, d, 64));
    zmin = fminf(zmin, __shfl_xor(zmin, d, 64)); zmax = fmaxf(zmax, __shfl_xor(zmax, d, 64));
  }
  // grid parameters: every lane computes the same values, lane 0 stores them
  GridParams G = make_grid(n, cbase, off, ymin, ymax, zmin, zmax);
  G.off_plane = __ballot(mine && x != w.row_x[ru % w.R]) ? 1u : 0u;
  if (lane == 0) w.grid[ru] = G;
  const uint32_t nc = G.nz * G.ny;
  for (uint32_t c = lane; c <= nc; c += 64) hist[c] = 0u;
  wave_sync();
  const uint32_t cell = mine ? cell_of(G, y, z) : 0u;
  if (mine) atomicAdd(&hist[cell], 1u);
  wave_sync();
  uint32_t carry = 0;
  for (uint32_t c0 = 0; c0 < nc; c0 += 64) {
    const uint32_t c = c0 + lane;
    const uint32_t v = c < nc ? hist[c] : 0u;
    const uint32_t inc = wave_incl_scan(v);
    if (c < nc) { hist[c] = carry + inc - v; w.cell_off[cbase + c] = (uint16_t)(carry + inc - v); }
    carry += (uint32_t)__shfl((int)inc, 63, 64);
  }
  if (lane == 0) w.cell_off[cbase + nc] = (uint16_t)n;
  wave_sync();
  if (mine) {
    const uint32_t pos = atomicAdd(&hist[cell], 1u);
    w.gbuf[off + pos] = make_float4(y, z, x, __uint_as_float(off + lane));
    w.grec[off + pos] = SearchRec{y, z, off + lane};
  }
}

// Row units of kTiny < n <= kWaveRow clusters: one wave each, four per
// workgroup, no workgroup barrier.  Lane l holds entries 4l .. 4l+3; the
// bitonic sort on the ids swaps registers for partners in the same lane and
// uses shuffles otherwise, then every sorted entry's coordinates are read
// from its original slot; the grid is built with a per-wave LDS histogram.
// Same results as k_rows.
__global__ __launch_bounds__(TB) void k_rows_wave(Ws w) {
  __shared__ uint32_t s_h[TB / 64][kCellsPerCluster * kWaveRow + 2];
  const int wv = threadIdx.x >> 6, lane = lane_id();
  uint32_t* hist = s_h[wv];
  auto unit = [&](const int64_t ru) {
    const uint32_t off = w.ru_off[ru];
    const uint32_t n = w.ru_off[ru + 1] - off;
    if (rows_class(n) != 1) return;
    const uint32_t cbase = w.cell_base[ru];
    uint32_t K[4], V[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t i = 4u * lane + k;
      K[k] = i < n ? __float_as_uint(w.tmp4[off + i].w) : 0xFFFFFFFFu;
      V[k] = i;
    }
    auto cs = [&](int k0, int k1, uint32_t kk) {   // registers k0 < k1 of this lane
      const bool asc = ((4u * lane + k0) & kk) == 0;
      if (asc ? K[k0] > K[k1] : K[k0] < K[k1]) {
        const uint32_t t = K[k0]; K[k0] = K[k1]; K[k1] = t;
        const uint32_t u = V[k0]; V[k0] = V[k1]; V[k1] = u;
      }
    };
    uint32_t npad = 2;
    while (npad < n) npad <<= 1;
    for (uint32_t kk = 2; kk <= npad; kk <<= 1) {
      for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
        if (j == 1) {
          cs(0, 1, kk); cs(2, 3, kk);
        } else if (j == 2) {
          cs(0, 2, kk); cs(1, 3, kk);
        } else {
          uint32_t O[4], OV[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            O[k] = (uint32_t)__shfl_xor((int)K[k], (int)(j >> 2), 64);
            OV[k] = (uint32_t)__shfl_xor((int)V[k], (int)(j >> 2), 64);
          }
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const uint32_t i = 4u * lane + k;
            const bool lower = (i & j) == 0, asc = (i & kk) == 0;
            const uint32_t lo = lower ? K[k] : O[k], hi = lower ? O[k] : K[k];
            if (asc ? lo > hi : lo < hi) { K[k] = O[k]; V[k] = OV[k]; }
          }
        }
      }
    }
    float px[4], py[4], pz[4];
    float ymin = INFINITY, ymax = -INFINITY, zmin = INFINITY, zmax = -INFINITY;
    const float xr = w.row_x[ru % w.R];
    bool offp = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t i = 4u * lane + k;
      px[k] = py[k] = pz[k] = 0.f;
      if (i < n) {
        const float4 v = w.tmp4[off + V[k]];
        px[k] = v.x; py[k] = v.y; pz[k] = v.z;
        w.cx[off + i] = v.x; w.cy[off + i] = v.y; w.cz[off + i] = v.z;
        w.cid[off + i] = K[k]; w.cru[off + i] = (uint32_t)ru;
        ymin = fminf(ymin, v.y); ymax = fmaxf(ymax, v.y); zmin = fminf(zmin, v.z); zmax = fmaxf(zmax, v.z);
        offp = offp || v.x != xr;
      }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
      ymin = fminf(ymin, __shfl_xor(ymin, d, 64)); ymax = fmaxf(ymax, __shfl_xor(ymax, d, 64));
      zmin = fminf(zmin, __shfl_xor(zmin, d, 64)); zmax = fmaxf(zmax, __shfl_xor(zmax, d, 64));
    }
    // every lane computes the same grid, lane 0 stores it
    GridParams G = make_grid(n, cbase, off, ymin, ymax, zmin, zmax);
    G.off_plane = __ballot(offp) ? 1u : 0u;
    if (lane == 0) w.grid[ru] = G;
    const uint32_t nc = G.nz * G.ny;
    for (uint32_t c = lane; c <= nc; c += 64) hist[c] = 0u;
    wave_sync();
    uint32_t cell[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      cell[k] = 4u * lane + k < n ? cell_of(G, py[k], pz[k]) : 0u;
      if (4u * lane + k < n) atomicAdd(&hist[cell[k]], 1u);
    }
    wave_sync();
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < nc; c0 += 64) {
      const uint32_t c = c0 + lane;
      const uint32_t v = c < nc ? hist[c] : 0u;
      const uint32_t inc = wave_incl_scan(v);
      if (c < nc) { hist[c] = carry + inc - v; w.cell_off[cbase + c] = (uint16_t)(carry + inc - v); }
      carry += (uint32_t)__shfl((int)inc, 63, 64);
    }
    if (lane == 0) w.cell_off[cbase + nc] = (uint16_t)n;
    wave_sync();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t i = 4u * lane + k;
      if (i < n) {
        const uint32_t pos = atomicAdd(&hist[cell[k]], 1u);
        w.gbuf[off + pos] = make_float4(py[k], pz[k], px[k], __uint_as_float(off + i));
        w.grec[off + pos] = SearchRec{py[k], pz[k], off + i};
      }
    }
  };
  if (!ru_lists(w.RU)) {
    const int64_t ru = (int64_t)blockIdx.x * (TB / 64) + wv;
    if (ru < w.RU) unit(ru);
    return;
  }
  const uint32_t cnt = w.flags[F_LROWS1];
  for (uint32_t i = blockIdx.x * (TB / 64) + wv; i < cnt; i += gridDim.x * (TB / 64)) {
    unit(w.ru_rows[i]);
    wave_sync();   // the histogram is reused by the next unit
  }
}

// Two instantiations: row units of kWaveRow < n <= 4 TB clusters (small LDS,
// so many workgroups share a CU) and larger ones (LDS for kMaxRow ids).  With few row
// units a launch covers every unit and skips those of the other sizes; with
// many its workgroups loop over the class's list.
template <bool kLarge>
__global__ __launch_bounds__(TB) void k_rows(Ws w) {
  constexpr uint32_t kIds = kLarge ? (uint32_t)kMaxRow : 4u * TB;
  constexpr uint32_t kCells = kLarge ? (uint32_t)kMaxCells : kCellsPerCluster * 4u * TB + 1u;   // grid_cells(n) bound
  __shared__ uint32_t s_ids[kIds];
  // slots (16 bit) during the sort, then the cell histogram
  __shared__ uint32_t s_aux[(kCells + 1) > kIds / 2 ? (kCells + 1) : kIds / 2];
  __shared__ float s_red[4][TB / 64];
  __shared__ uint32_t s_off[TB / 64];
  __shared__ GridParams s_gp;
  uint16_t* s_slot = (uint16_t*)s_aux;
  uint32_t* s_hist = s_aux;
  // one row unit (workgroup-uniform); called once per unit of the launch
  auto unit = [&](const int64_t ru) {
    const uint32_t off = w.ru_off[ru];
    const uint32_t n = w.ru_off[ru + 1] - off;
    const uint32_t cbase = w.cell_base[ru];
    const int tid = threadIdx.x;
    if (rows_class(n) != (kLarge ? 3 : 2)) return;   // (smaller units: k_rows_tiny, k_rows_wave)
    if (n > (uint32_t)kMaxRow) {
      if (tid == 0) {
        atomicOr(&w.flags[F_ERR], ERR_LIMIT);
        GridParams G{cbase, 1u, 1u, 0.f, 0.f, 0.f, 0.f, off, 1u};
        w.grid[ru] = G;
        w.cell_off[cbase] = 0;
        w.cell_off[cbase + 1] = 0;
      }
      // every per-position array still gets a defined entry (its own position
      // in the grid copy), so later kernels stay in bounds until the error is
      // reported
      const float nan = __int_as_float(0x7fc00000);
      for (uint32_t k = tid; k < n; k += TB) {
        w.cx[off + k] = nan; w.cy[off + k] = nan; w.cz[off + k] = nan;
        w.cid[off + k] = 0u; w.cru[off + k] = (uint32_t)ru;
        w.gbuf[off + k] = make_float4(nan, nan, nan, __uint_as_float(off + k));
        w.grec[off + k] = SearchRec{nan, nan, off + k};
      }
      return;
    }
    // Rows of up to 4 TB clusters (all but extreme ones) are sorted in
    // registers: thread t holds sorted positions 4t .. 4t+3; bitonic stages
    // whose partner is in the same thread swap registers, partners in the
    // same wave come by shuffles, and only the stages across waves (partner
    // distance >= 256) go through LDS.  Their coordinates then stay in
    // registers for the grid passes.
    const bool fast = !kLarge;
    uint32_t K[4], V[4];
    float px[4], py[4], pz[4];
    float ymin = INFINITY, ymax = -INFINITY, zmin = INFINITY, zmax = -INFINITY;
    const float xr = w.row_x[ru % w.R];
    bool offp = false;
    if (fast) {
  #pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t i = 4u * tid + k;
        K[k] = i < n ? __float_as_uint(w.tmp4[off + i].w) : 0xFFFFFFFFu;
        V[k] = i;
      }
      auto cs = [&](int k0, int k1, uint32_t kk) {   // registers k0 < k1 of this thread
        const bool asc = ((4u * tid + k0) & kk) == 0;
        if (asc ? K[k0] > K[k1] : K[k0] < K[k1]) {
          const uint32_t t = K[k0]; K[k0] = K[k1]; K[k1] = t;
          const uint32_t u = V[k0]; V[k0] = V[k1]; V[k1] = u;
        }
      };
      // stages up to the row's power-of-two size only: the entries past it are
      // all padding (equal maxima), already in order
      uint32_t npad = 2;
      while (npad < n) npad <<= 1;
      for (uint32_t kk = 2; kk <= npad; kk <<= 1) {
        for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
          if (j == 1) {
            cs(0, 1, kk); cs(2, 3, kk);
          } else if (j == 2) {
            cs(0, 2, kk); cs(1, 3, kk);
          } else {
            uint32_t O[4], OV[4];
            if (j < 256) {
  #pragma unroll
              for (int k = 0; k < 4; ++k) {
                O[k] = (uint32_t)__shfl_xor((int)K[k], (int)(j >> 2), 64);
                OV[k] = (uint32_t)__shfl_xor((int)V[k], (int)(j >> 2), 64);
              }
            } else {
              __syncthreads();
  #pragma unroll
              for (int k = 0; k < 4; ++k) { s_ids[4u * tid + k] = K[k]; s_slot[4u * tid + k] = (uint16_t)V[k]; }
              __syncthreads();
  #pragma unroll
              for (int k = 0; k < 4; ++k) { O[k] = s_ids[(4u * tid + k) ^ j]; OV[k] = s_slot[(4u * tid + k) ^ j]; }
            }
  #pragma unroll
            for (int k = 0; k < 4; ++k) {
              const uint32_t i = 4u * tid + k;
              const bool lower = (i & j) == 0, asc = (i & kk) == 0;
              const uint32_t lo = lower ? K[k] : O[k], hi = lower ? O[k] : K[k];
              if (asc ? lo > hi : lo < hi) { K[k] = O[k]; V[k] = OV[k]; }
            }
          }
        }
      }
  #pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t i = 4u * tid + k;
        if (i < n) {
          const float4 v = w.tmp4[off + V[k]];
          px[k] = v.x; py[k] = v.y; pz[k] = v.z;
          w.cx[off + i] = v.x; w.cy[off + i] = v.y; w.cz[off + i] = v.z;
          w.cid[off + i] = K[k]; w.cru[off + i] = (uint32_t)ru;
          ymin = fminf(ymin, v.y); ymax = fmaxf(ymax, v.y); zmin = fminf(zmin, v.z); zmax = fmaxf(zmax, v.z);
          offp = offp || v.x != xr;
        }
      }
    } else {
      uint32_t npad = 2;
      while (npad < n) npad <<= 1;
      for (uint32_t k = tid; k < npad; k += TB) {
        s_ids[k] = k < n ? __float_as_uint(w.tmp4[off + k].w) : 0xFFFFFFFFu;
        s_slot[k] = (uint16_t)k;
      }
      __syncthreads();
      for (uint32_t kk = 2; kk <= npad; kk <<= 1) {
        for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
          for (uint32_t i = tid; i < npad; i += TB) {
            const uint32_t ixj = i ^ j;
            if (ixj > i) {
              const uint32_t a = s_ids[i], b = s_ids[ixj];
              const bool asc = (i & kk) == 0;
              if ((a > b) == asc) {
                s_ids[i] = b; s_ids[ixj] = a;
                const uint16_t t = s_slot[i]; s_slot[i] = s_slot[ixj]; s_slot[ixj] = t;
              }
            }
          }
          __syncthreads();
        }
      }
      for (uint32_t k = tid; k < n; k += TB) {
        const float4 v = w.tmp4[off + s_slot[k]];
        const float x = v.x, y = v.y, z = v.z;
        w.cx[off + k] = x; w.cy[off + k] = y; w.cz[off + k] = z;
        w.cid[off + k] = s_ids[k]; w.cru[off + k] = (uint32_t)ru;
        ymin = fminf(ymin, y); ymax = fmaxf(ymax, y); zmin = fminf(zmin, z); zmax = fmaxf(zmax, z);
        offp = offp || x != xr;
      }
    }
  #pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
      ymin = fminf(ymin, __shfl_xor(ymin, d, 64)); ymax = fmaxf(ymax, __shfl_xor(ymax, d, 64));
      zmin = fminf(zmin, __shfl_xor(zmin, d, 64)); zmax = fmaxf(zmax, __shfl_xor(zmax, d, 64));
    }
    const bool offw = __ballot(offp) != 0ull;
    if (lane_id() == 0) {
      s_red[0][tid >> 6] = ymin; s_red[1][tid >> 6] = ymax; s_red[2][tid >> 6] = zmin; s_red[3][tid >> 6] = zmax;
      s_off[tid >> 6] = offw ? 1u : 0u;
    }
    __syncthreads();
    if (tid == 0) {
      uint32_t o = s_off[0];
      for (int i = 1; i < TB / 64; ++i) {
        ymin = fminf(ymin, s_red[0][i]); ymax = fmaxf(ymax, s_red[1][i]);
        zmin = fminf(zmin, s_red[2][i]); zmax = fmaxf(zmax, s_red[3][i]);
        o |= s_off[i];
      }
      GridParams G = make_grid(n, cbase, off, ymin, ymax, zmin, zmax);
      G.off_plane = o;
      s_gp = G;
      w.grid[ru] = G;
    }
    __syncthreads();
    const GridParams G = s_gp;
    const uint32_t nc = G.nz * G.ny;
    for (uint32_t c = tid; c <= nc; c += TB) s_hist[c] = 0u;
    __syncthreads();
    if (fast) {
  #pragma unroll
      for (int k = 0; k < 4; ++k)
        if (4u * tid + k < n) atomicAdd(&s_hist[cell_of(G, py[k], pz[k])], 1u);
    } else {
      // the canonical entries were written by this same thread (same k
      // stride): re-read them, coalesced
      for (uint32_t k = tid; k < n; k += TB) atomicAdd(&s_hist[cell_of(G, w.cy[off + k], w.cz[off + k])], 1u);
    }
    __syncthreads();
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < nc; c0 += TB) {
      const uint32_t c = c0 + tid;
      const uint32_t v = c < nc ? s_hist[c] : 0u;
      uint32_t tot;
      const uint32_t ex = block_excl_scan(v, &tot) + carry;
      if (c < nc) { s_hist[c] = ex; w.cell_off[cbase + c] = (uint16_t)ex; }
      carry += tot;
    }
    if (tid == 0) w.cell_off[cbase + nc] = (uint16_t)n;
    __syncthreads();
    if (fast) {
  #pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t i = 4u * tid + k;
        if (i < n) {
          const uint32_t slot = atomicAdd(&s_hist[cell_of(G, py[k], pz[k])], 1u);
          w.gbuf[off + slot] = make_float4(py[k], pz[k], px[k], __uint_as_float(off + i));
          w.grec[off + slot] = SearchRec{py[k], pz[k], off + i};
        }
      }
    } else {
      for (uint32_t k = tid; k < n; k += TB) {
        const float x = w.cx[off + k], y = w.cy[off + k], z = w.cz[off + k];
        const uint32_t slot = atomicAdd(&s_hist[cell_of(G, y, z)], 1u);
        w.gbuf[off + slot] = make_float4(y, z, x, __uint_as_float(off + k));
        w.grec[off + slot] = SearchRec{y, z, off + k};
      }
    }
  };
  if (!ru_lists(w.RU)) {
    unit(blockIdx.x);
    return;
  }
  const uint32_t cnt = w.flags[kLarge ? F_LROWS3 : F_LROWS2];
  for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
    unit(kLarge ? w.ru_big[i] : w.ru_rows[w.RU - 1 - (int64_t)i]);
    __syncthreads();   // LDS is reused by the next unit
  }
}

// Cell rectangle [iz0, iz1] x [iy0, iy1] covering |y - yq| <= wy, |z - zq| <= wz
// (the margin absorbs the rounding of the bounds; the exact test is done per
// candidate).
struct CellBox { uint32_t iz0, iz1, iy0, iy1; };
__device__ __forceinline__ CellBox cell_box(const GridParams& G, float yq, float zq, float wy, float wz) {
  const float m = 1e-3f;
  CellBox b;
  b.iz0 = cell_coord(zq - wz - m, G.z0, G.inv_bz, G.nz);
  b.iz1 = cell_coord(zq + wz + m, G.z0, G.inv_bz, G.nz);
  b.iy0 = cell_coord(yq - wy - m, G.y0, G.inv_by, G.ny);
  b.iy1 = cell_coord(yq + wy + m, G.y0, G.inv_by, G.ny);
  return b;
}

// ---------------------------------------------------------- a2: neighbours
// For the middle cluster i: the (down, up) pair on rows r-1 / r+1 inside the
// windows minimising the deviation of i from the chord d-u, accepted iff the
// score <= link_cut, ties by smaller up id then smaller down id (canonical
// positions are ordered like ids within a row).  D/U: the grid-ordered
// entries of the two rows; Dc/Uc: their cell start offsets (index into D/U).
template <class F4, class U32>
__device__ __forceinline__ void find_pair(const Ws& w, float xi, float yi, float zi,
                                          const GridParams& Gd, F4 D4, U32 Dc,
                                          const GridParams& Gu, F4 U4, U32 Uc,
                                          int32_t& bu, int32_t& bd) {
  const float WY = w.P.win_y, WZ = w.P.win_z, IWY = w.P.inv_var_y, IWZ = w.P.inv_var_z;
  const float CUT = w.P.link_cut;
  const CellBox bdn = cell_box(Gd, yi, zi, WY, WZ);
  const CellBox bup = cell_box(Gu, yi, zi, WY, WZ);
  bool have = false;
  float bs = 0.0f;
  bu = -1; bd = -1;
  for (uint32_t izd = bdn.iz0; izd <= bdn.iz1; ++izd) {
    const uint32_t cd0 = izd * Gd.ny;
    const uint32_t kd1 = Dc[cd0 + bdn.iy1 + 1];
    for (uint32_t kd = Dc[cd0 + bdn.iy0]; kd < kd1; ++kd) {
      const float4 D = D4[kd];
      if (!(fabsf(D.x - yi) <= WY && fabsf(D.y - zi) <= WZ)) continue;
      const int32_t pd = (int32_t)__float_as_uint(D.w);
      for (uint32_t izu = bup.iz0; izu <= bup.iz1; ++izu) {
        const uint32_t cu0 = izu * Gu.ny;
        const uint32_t ku1 = Uc[cu0 + bup.iy1 + 1];
        for (uint32_t ku = Uc[cu0 + bup.iy0]; ku < ku1; ++ku) {
          const float4 U = U4[ku];
          if (!(fabsf(U.x - yi) <= WY && fabsf(U.y - zi) <= WZ)) continue;
          const float wgt = (xi - D.z) / (U.z - D.z);
          const float ey = yi - fmaf(U.x - D.x, wgt, D.x);
          const float ez = zi - fmaf(U.y - D.y, wgt, D.y);
          const float score = fmaf(ez * ez, IWZ, (ey * ey) * IWY);
          if (!(score <= CUT)) continue;
          const int32_t pu = (int32_t)__float_as_uint(U.w);
          const bool better = !have || score < bs || (score == bs && (pu < bu || (pu == bu && pd < bd)));
          if (better) { have = true; bs = score; bu = pu; bd = pd; }
        }
      }
    }
  }
}

constexpr int kCand = 15;          // passing candidates per side kept per lane

// Window scan of one row's box: indices (into D4) of the entries within the
// windows, at most kCand; returns the count, or kCand + 1 on overflow.
template <class F4, class U32>
__device__ __forceinline__ int collect(const GridParams& G, F4 D4, U32 Dc, float yi, float zi, float WY,
                                       float WZ, uint16_t* out) {
  const CellBox b = cell_box(G, yi, zi, WY, WZ);
  int n = 0;
  for (uint32_t iz = b.iz0; iz <= b.iz1; ++iz) {
    const uint32_t c0 = iz * G.ny;
    const uint32_t k0 = Dc[c0 + b.iy0], k1 = Dc[c0 + b.iy1 + 1];
    // four entries read before any is tested
    for (uint32_t k = k0; k < k1; k += 4) {
      float4 D[4];
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j)
        if (k + j < k1) D[j] = D4[k + j];
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j) {
        if (k + j < k1 && fabsf(D[j].x - yi) <= WY && fabsf(D[j].y - zi) <= WZ) {
          if (n < kCand) out[n] = (uint16_t)(k + j);
          ++n;
        }
      }
    }
  }
  return n <= kCand ? n : kCand + 1;
}

// Pairs of one lane's two candidate lists, same arithmetic and tie-break as
// find_pair (the one-wave and small-slab variants; every pair reads its up
// candidate from LDS).  The interpolation weight depends only on the two x
// coordinates, so the quotient of the previous pair is reused when they
// repeat (clusters on their row planes).
template <class F4>
__device__ __forceinline__ void best_pair(const Ws& w, float xi, float yi, float zi, F4 D4, const uint16_t* ld,
                                          int nd, F4 U4, const uint16_t* lu, int nu, int32_t& bu,
                                          int32_t& bd) {
  const float IWY = w.P.inv_var_y, IWZ = w.P.inv_var_z, CUT = w.P.link_cut;
  bu = -1; bd = -1;
  if (nu == 0) return;
  // (bs, bu, bd) starts at (CUT, INT32_MAX, INT32_MAX): the first pair with
  // score <= CUT replaces it, later ones must beat the best so far (a NaN
  // score fails every comparison)
  float bs = CUT;
  int32_t ku = INT32_MAX, kd = INT32_MAX;
  auto take = [&](float score, int32_t pu, int32_t pd) {
    if (score < bs || (score == bs && (pu < ku || (pu == ku && pd < kd)))) { bs = score; ku = pu; kd = pd; }
  };
  // the last quotient and the x coordinates it was taken for
  float wx_d = 0.0f, wx_u = 0.0f, wq = 0.0f;
  bool wk = false;
  for (int i = 0; i < nd; ++i) {
    const float4 D = D4[ld[i]];
    const int32_t pd = (int32_t)__float_as_uint(D.w);
    for (int j = 0; j < nu; ++j) {
      const float4 U = U4[lu[j]];
      if (!(wk && D.z == wx_d && U.z == wx_u)) {
        wq = (xi - D.z) / (U.z - D.z);
        wx_d = D.z; wx_u = U.z; wk = true;
      }
      const float ey = yi - fmaf(U.x - D.x, wq, D.x);
      const float ez = zi - fmaf(U.y - D.y, wq, D.y);
      take(fmaf(ez * ez, IWZ, (ey * ey) * IWY), (int32_t)__float_as_uint(U.w), pd);
    }
  }
  if (ku != INT32_MAX) { bu = ku; bd = kd; }
}

// The pairs of a wave's lanes scored by all 64 lanes, same arithmetic and
// tie-break as find_pair.  Lane l (has: a cluster whose lists fit) owns
// cd_l cu_l pairs, listed in lane order and, within a lane, down-major; the
// list is cut into 64 contiguous ranges, one per lane, so a wave runs about
// its mean pair count instead of its lanes' largest candidate counts.  A lane
// keeps the least key of the pairs it scored for the current owner and folds
// it into the owner's LDS word (atomic minimum) when it moves on.  The key
// is (score bits, up offset, down offset) in 32 + 10 + 10 bits: a score that
// passes the cut is >= 0, so its bits order like its value, and the offsets
// of the neighbour rows' canonical positions (rows of at most kSlab entries)
// order like the positions, so the least key is find_pair's choice.  Called
// by all lanes of the wave; ld_w/lu_w/key_w: the wave's slices of the
// candidate lists and of the key words.
constexpr unsigned long long kNoKey = ~0ull;
static_assert(kSlab <= 1024u, "row offsets in the pair key take 10 bits");

__device__ __forceinline__ void wave_pairs(const Ws& w, bool has, float xi, float yi, float zi, uint32_t cd,
                                           uint32_t cu, const float4* D4, const float4* U4, const uint16_t* ld_w,
                                           const uint16_t* lu_w, unsigned long long* key_w, uint32_t offd,
                                           uint32_t offu, int32_t& bu, int32_t& bd) {
  const float IWY = w.P.inv_var_y, IWZ = w.P.inv_var_z, CUT = w.P.link_cut;
  const int lane = lane_id();
  const uint32_t cnt = has ? cd * cu : 0u;
  const uint32_t incl = wave_incl_scan(cnt);
  const uint32_t P = (uint32_t)__shfl((int)incl, 63, 64);
  bu = -1; bd = -1;
  if (P == 0u) return;   // (uniform)
  key_w[lane] = kNoKey;
  wave_sync();
  const uint64_t owners = __ballot(cnt > 0u);
  uint32_t t = (uint32_t)(((uint64_t)lane * P) >> 6);
  const uint32_t t1 = (uint32_t)(((uint64_t)(lane + 1) * P) >> 6);
  // owner of pair t (< P): the lowest lane whose inclusive count exceeds t
  int o = 0;
#pragma unroll
  for (int st = 32; st > 0; st >>= 1) {
    const uint32_t v = (uint32_t)__shfl((int)incl, o + st - 1, 64);
    if (v <= t) o += st;
  }
  // the owner's cluster, up count and pair range (shuffles by every lane)
  float oxi, oyi, ozi;
  uint32_t ocu, oend;
  auto fetch = [&](int src) {
    oxi = __shfl(xi, src, 64);
    oyi = __shfl(yi, src, 64);
    ozi = __shfl(zi, src, 64);
    ocu = (uint32_t)__shfl((int)cu, src, 64);
    oend = (uint32_t)__shfl((int)incl, src, 64);
  };
  fetch(o);
  const uint32_t ocnt = (uint32_t)__shfl((int)cnt, o, 64);
  uint32_t i = 0, j = 0;
  if (t < t1) {
    const uint32_t rel = t - (oend - ocnt);
    i = rel / ocu;
    j = rel - i * ocu;
  }
  unsigned long long best = kNoKey;
  // the interpolation quotient of the last pair, reused while the three x
  // coordinates repeat (clusters on their row planes)
  float wx_i = 0.0f, wx_d = 0.0f, wx_u = 0.0f, wq = 0.0f;
  bool wk = false;
  const uint32_t steps = (P + 63u) >> 6;   // the longest range
  for (uint32_t k = 0; k < steps; ++k) {
    const bool act = t < t1;
    if (act) {
      const float4 D = D4[ld_w[kCand * o + (int)i]];
      const float4 U = U4[lu_w[kCand * o + (int)j]];
      if (!(wk && oxi == wx_i && D.z == wx_d && U.z == wx_u)) {
        wq = (oxi - D.z) / (U.z - D.z);
        wx_i = oxi; wx_d = D.z; wx_u = U.z; wk = true;
      }
      const float ey = oyi - fmaf(U.x - D.x, wq, D.x);
      const float ez = ozi - fmaf(U.y - D.y, wq, D.y);
      const float score = fmaf(ez * ez, IWZ, (ey * ey) * IWY);
      if (score <= CUT) {
        const unsigned long long key = ((unsigned long long)__float_as_uint(score) << 20) |
                                       ((unsigned long long)(__float_as_uint(U.w) - offu) << 10) |
                                       (unsigned long long)(__float_as_uint(D.w) - offd);
        best = key < best ? key : best;
      }
      ++t;
      if (++j == ocu) { j = 0; ++i; }
    }
    const bool fold = act && (t == oend || t == t1);
    if (fold && best != kNoKey) atomicMin(&key_w[o], best);
    if (fold) best = kNoKey;
    // the range goes on into the next owner (a later lane with pairs)
    const bool next = act && t == oend && t < t1;
    if (__ballot(next) != 0ull) {
      const int on = next ? __ffsll((unsigned long long)(owners & ~((2ull << o) - 1ull))) - 1 : o;
      fetch(on);
      if (next) { o = on; i = 0; j = 0; }
    }
  }
  wave_sync();
  const unsigned long long b = key_w[lane];
  if (has && b != kNoKey) {
    bu = (int32_t)(offu + (uint32_t)((b >> 10) & 1023ull));
    bd = (int32_t)(offd + (uint32_t)(b & 1023ull));
  }
}

// One block per row unit: the grids of rows r-1 and r+1 (entries and cell
// offsets) are staged in LDS when each holds at most kSlab clusters.  Lanes
// take the row's clusters in grid (cell) order, so the lanes of a wave are
// spatial neighbours with similar candidate counts.  A lane first collects
// the down and up candidates inside the windows (two flat scans), then the
// pairs are scored: by the lane itself in the two smaller variants, by all
// lanes of the wave in the slab variant (wave_pairs); nested scanning would
// make a wave run the product of its lanes' largest candidate counts.
// Results do not depend on the order.
//
// Three instantiations by the size of the neighbour rows: up to kTiny
// clusters (one wave per row unit, four per workgroup, wave-level ordering),
// up to kSmallSlab (workgroup per row unit, half the LDS) and the rest
// (896-cluster slab).  With few row units each launch covers every unit and
// skips those of the other kinds; with many the two workgroup variants loop
// over their class's list.
template <uint32_t kS, uint32_t kG>
__global__ __launch_bounds__(TB) void k_links(Ws w) {
  constexpr uint32_t kNG = TB / kG;   // row units per workgroup
  constexpr int kClass = kS == kTiny ? 0 : kS == kSmallSlab ? 1 : 2;
  // one spare slot at the end of each array takes the staging stores of
  // slots past a row's end (never read)
  constexpr uint32_t kSpareE = kS, kSpareC = kCellsPerCluster * kS + 2;
  __shared__ float4 s_d[kNG][kS + 1], s_u[kNG][kS + 1];
  // cell offsets relative to the slab (< kS): 16 bit; a row of <= kS
  // clusters has at most kCellsPerCluster kS + 1 cells
  __shared__ uint16_t s_cd[kNG][kSpareC + 1], s_cu[kNG][kSpareC + 1];
  __shared__ uint16_t s_ld[kCand * TB], s_lu[kCand * TB];
  // per-lane best pair keys of the wave-level pair scoring (slab variant)
  __shared__ unsigned long long s_key[kClass == 2 ? TB : 1];
  const uint32_t g = threadIdx.x / kG, gt = threadIdx.x % kG;
  // one row unit (uniform over its kG threads); called once per unit of the launch
  auto unit = [&](const int64_t ru) {
    if (ru >= w.RU) return;
    const int r = (int)(ru % w.R);
    const bool inner = r >= 1 && r <= w.R - 2;
    // every row offset and both neighbour grids in one round of loads
    const int64_t rdn = inner ? ru - 1 : ru, rup = inner ? ru + 1 : ru;
    const uint32_t offd = w.ru_off[rdn], off = w.ru_off[ru], offu = w.ru_off[ru + 1];
    const uint32_t endu = w.ru_off[inner ? ru + 2 : ru + 1];
    const GridParams Gd = w.grid[rdn], Gu = w.grid[rup];
    const uint32_t n = offu - off;
    if (n == 0) return;
    // edge rows have no links; an over-full row unit (reported as an error) gets none either
    if (!inner || n > (uint32_t)kMaxRow) {
      if (kClass == 2)   // (written by one of the instantiations)
        for (uint32_t k = gt; k < n; k += kG) { w.up[off + k] = -1; w.dn[off + k] = -1; }
      return;
    }
    const uint32_t nd = off - offd, nu = endu - offu;
    const int cls = links_class(n, nd, nu, true);
    if (cls != kClass) return;
    const bool lds = nd <= kS && nu <= kS;
    float4* sd = s_d[g];
    float4* su = s_u[g];
    uint16_t* scd = s_cd[g];
    uint16_t* scu = s_cu[g];
    // this thread's own clusters (grid order) for its first rounds, read now
    // so that they arrive with the staged rows
    constexpr int kOwn = 4;   // (the slab variant's rounds shift through four)
    float4 mine[kOwn];
  #pragma unroll
    for (int i = 0; i < kOwn; ++i) {
      const uint32_t k = gt + kG * i;
      mine[i] = w.gbuf[off + (k < n ? k : 0u)];   // (used only if k < n)
    }
    if (lds) {
      // all of a thread's staging loads are issued before the first LDS store
      // (one memory round trip instead of one per loop iteration); slots past
      // a row's end load an entry known to exist (this row's first entry, the
      // row's first cell offset) and store it to the spare slot, so that
      // neither the loads nor the stores need a branch
      constexpr int kE = (int)((kS + kG - 1) / kG);                          // entries per thread
      constexpr int kC = (int)((kCellsPerCluster * kS + 1 + kG) / kG);      // cell offsets per thread
      const uint32_t ncd = Gd.nz * Gd.ny, ncu = Gu.nz * Gu.ny;
  #pragma unroll
      for (int j = 0; j < kE; ++j) {
        const uint32_t i = gt + kG * (uint32_t)j;
        const float4 a = w.gbuf[i < nd ? offd + i : off];
        const float4 b = w.gbuf[i < nu ? offu + i : off];
        sd[i < nd ? i : kSpareE] = a;
        su[i < nu ? i : kSpareE] = b;
      }
  #pragma unroll
      for (int j = 0; j < kC; ++j) {
        const uint32_t i = gt + kG * (uint32_t)j;
        const uint16_t a = w.cell_off[Gd.cell_base + (i <= ncd ? i : 0u)];
        const uint16_t b = w.cell_off[Gu.cell_base + (i <= ncu ? i : 0u)];
        scd[i <= ncd ? i : kSpareC] = a;
        scu[i <= ncu ? i : kSpareC] = b;
      }
      if (kG == TB) __syncthreads(); else wave_sync();
    }
    uint16_t* ld = s_ld + kCand * threadIdx.x;
    uint16_t* lu = s_lu + kCand * threadIdx.x;
    const float WY = w.P.win_y, WZ = w.P.win_z;
    auto link = [&](const float4& me) {
      const uint32_t p = __float_as_uint(me.w);
      const float xi = me.z, yi = me.x, zi = me.y;
      int32_t bu = -1, bd = -1;
      if (lds) {
        const int cd = collect(Gd, (const float4*)sd, (const uint16_t*)scd, yi, zi, WY, WZ, ld);
        const int cu = cd > 0 ? collect(Gu, (const float4*)su, (const uint16_t*)scu, yi, zi, WY, WZ, lu) : 0;
        if (cd <= kCand && cu <= kCand)
          best_pair(w, xi, yi, zi, (const float4*)sd, ld, cd, (const float4*)su, lu, cu, bu, bd);
        else
          find_pair(w, xi, yi, zi, Gd, (const float4*)sd, (const uint16_t*)scd, Gu, (const float4*)su,
                    (const uint16_t*)scu, bu, bd);
      } else {
        find_pair(w, xi, yi, zi, Gd, w.gbuf + offd, w.cell_off + Gd.cell_base, Gu, w.gbuf + offu,
                  w.cell_off + Gu.cell_base, bu, bd);
      }
      w.up[p] = bu;
      w.dn[p] = bd;
    };
    if constexpr (kClass == 2) {
      if (lds) {
        // rounds of the wave's 64 clusters: candidate lists per lane, then
        // the wave's pairs scored by all its lanes; a lane whose lists
        // overflow takes find_pair afterwards
        const uint32_t wb = gt & ~63u;
        const uint16_t* ld_w = s_ld + kCand * (threadIdx.x & ~63u);
        const uint16_t* lu_w = s_lu + kCand * (threadIdx.x & ~63u);
        unsigned long long* key_w = s_key + (threadIdx.x & ~63u);
        // the prefetched clusters move down one slot per round (an array
        // indexed by the round would be placed in scratch memory)
        float4 m0 = mine[0], m1 = mine[1], m2 = mine[2], m3 = mine[3];
        for (uint32_t i = 0; wb + kG * i < n; ++i) {
          const uint32_t k = gt + kG * i;
          const bool has = k < n;
          float4 me = m0;
          if (i >= (uint32_t)kOwn) me = w.gbuf[off + (has ? k : 0u)];
          m0 = m1; m1 = m2; m2 = m3;
          const float xi = me.z, yi = me.x, zi = me.y;
          int cd = 0, cu = 0;
          if (has) {
            cd = collect(Gd, (const float4*)sd, (const uint16_t*)scd, yi, zi, WY, WZ, ld);
            cu = cd > 0 ? collect(Gu, (const float4*)su, (const uint16_t*)scu, yi, zi, WY, WZ, lu) : 0;
          }
          const bool fb = has && (cd > kCand || cu > kCand);
          int32_t bu, bd;
          wave_pairs(w, has && !fb, xi, yi, zi, (uint32_t)cd, (uint32_t)cu, (const float4*)sd, (const float4*)su,
                     ld_w, lu_w, key_w, offd, offu, bu, bd);
          if (fb)
            find_pair(w, xi, yi, zi, Gd, (const float4*)sd, (const uint16_t*)scd, Gu, (const float4*)su,
                      (const uint16_t*)scu, bu, bd);
          if (has) {
            const uint32_t p = __float_as_uint(me.w);
            w.up[p] = bu;
            w.dn[p] = bd;
          }
        }
        return;
      }
    }
  #pragma unroll
    for (int i = 0; i < kOwn; ++i)
      if (gt + kG * i < n) link(mine[i]);
    for (uint32_t k = gt + kG * kOwn; k < n; k += kG) link(w.gbuf[off + k]);
  };
  if (kNG != 1 || !ru_lists(w.RU)) {
    unit((int64_t)blockIdx.x * kNG + g);
    return;
  }
  const uint32_t cnt = w.flags[kClass == 2 ? F_LLINKS2 : F_LLINKS1];
  for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
    unit(kClass == 2 ? w.ru_links[w.RU - 1 - (int64_t)i] : w.ru_links[i]);
    __syncthreads();   // LDS is reused by the next unit
  }
}

// ------------------------------------------------------- a3/a4: clean/start
// Keep a link only if reciprocated (from the raw arrays).  Start hit: kept up
// link, no kept down link.  Seed: start hit whose chain reaches
// min_seed_hits clusters.  Optional taps map positions to cluster ids.
__global__ __launch_bounds__(TB) void k_clean(Ws w) {
  __shared__ uint32_t s_cnt[2][TB / 64];
  const int64_t p = (int64_t)blockIdx.x * TB + threadIdx.x;
  bool start = false, seed = false;
  if (p < w.N) {
    // independent loads first, then both reciprocity gathers together
    // (a missing link reads the cluster's own entry, which is not used)
    const int32_t u = w.up[p], d = w.dn[p];
    const float x = w.cx[p], y = w.cy[p], z = w.cz[p];
    const int32_t du = w.dn[u >= 0 ? u : (int32_t)p];
    const int32_t ud = w.up[d >= 0 ? d : (int32_t)p];
    const int32_t cu = (u >= 0 && du == (int32_t)p) ? u : -1;
    const int32_t cd = (d >= 0 && ud == (int32_t)p) ? d : -1;
    w.cup[p] = cu;
    w.cdn[p] = cd;
    w.cpk[p] = make_float4(x, y, z, __int_as_float(cu));
    start = cu >= 0 && cd < 0;
    if (start) {
      int L = 2;
      int32_t q = cu;
      while (L < w.P.min_seed_hits) {
        const int32_t nu = w.up[q];
        if (nu < 0 || w.dn[nu] != q) break;
        q = nu;
        ++L;
      }
      seed = L >= w.P.min_seed_hits;
    }
    w.flag[p] = (uint8_t)((start ? 1 : 0) | (seed ? 2 : 0));
    if (w.taps) {
      const int e = (int)(w.cru[p] / ((uint32_t)w.S * (uint32_t)w.R));
      const EventOut& O = w.out[e];
      const uint32_t id = w.cid[p];
      if (O.dbg_up) O.dbg_up[id] = u >= 0 ? (int32_t)w.cid[u] : -1;
      if (O.dbg_dn) O.dbg_dn[id] = d >= 0 ? (int32_t)w.cid[d] : -1;
      if (O.dbg_cup) O.dbg_cup[id] = cu >= 0 ? (int32_t)w.cid[cu] : -1;
      if (O.dbg_cdn) O.dbg_cdn[id] = cd >= 0 ? (int32_t)w.cid[cd] : -1;
    }
  }
  const uint64_t bs = __ballot(start), bq = __ballot(seed);
  if (lane_id() == 0) { s_cnt[0][threadIdx.x >> 6] = (uint32_t)__popcll(bs); s_cnt[1][threadIdx.x >> 6] = (uint32_t)__popcll(bq); }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = 0, b = 0;
    for (int i = 0; i < TB / 64; ++i) { a += s_cnt[0][i]; b += s_cnt[1][i]; }
    w.blk_start[blockIdx.x] = a;
    w.blk_seed[blockIdx.x] = b;
  }
}

// Ordered compaction: block offset (scanned) + wave offset + ballot rank.
__global__ __launch_bounds__(TB) void k_compact(Ws w) {
  __shared__ uint32_t s_cnt[2][TB / 64];
  const int64_t p = (int64_t)blockIdx.x * TB + threadIdx.x;
  const uint8_t f = p < w.N ? w.flag[p] : (uint8_t)0;
  const bool start = f & 1, seed = (f >> 1) & 1;
  const uint64_t bs = __ballot(start), bq = __ballot(seed);
  const int wid = threadIdx.x >> 6;
  if (lane_id() == 0) { s_cnt[0][wid] = (uint32_t)__popcll(bs); s_cnt[1][wid] = (uint32_t)__popcll(bq); }
  __syncthreads();
  uint32_t os = w.blk_start[blockIdx.x], oq = w.blk_seed[blockIdx.x];
  for (int i = 0; i < wid; ++i) { os += s_cnt[0][i]; oq += s_cnt[1][i]; }
  const uint64_t lt = lanemask_lt();
  if (start) w.starts[os + (uint32_t)__popcll(bs & lt)] = (uint32_t)p;
  if (seed) w.seeds[oq + (uint32_t)__popcll(bq & lt)] = (uint32_t)p;
}

// Counts and per-event (and, for seeds, per-sector) ranges of the start and
// seed lists: entry i of a list writes the boundaries between its
// predecessor's unit and its own (all entries in parallel).
__global__ __launch_bounds__(TB) void k_ev_offsets(Ws w) {
  const uint32_t ns = w.blk_seed[w.nb], nst = w.blk_start[w.nb];
  const int64_t g0 = (int64_t)blockIdx.x * TB + threadIdx.x, gs = (int64_t)gridDim.x * TB;
  if (g0 == 0) { w.flags[F_NSEEDS] = ns; w.flags[F_NSTARTS] = nst; }
  const int64_t nsu = (int64_t)w.E * w.S;
  for (int64_t i = g0; i <= ns; i += gs) {
    const int64_t cur = i < ns ? (int64_t)(w.cru[w.seeds[i]] / (uint32_t)w.R) : nsu;
    const int64_t prev = i > 0 ? (int64_t)(w.cru[w.seeds[i - 1]] / (uint32_t)w.R) : -1;
    for (int64_t u = prev + 1; u <= cur; ++u) w.seed_su_off[u] = (uint32_t)i;
    const int64_t ce = i < ns ? cur / w.S : w.E, pe = i > 0 ? prev / w.S : -1;
    for (int64_t e = pe + 1; e <= ce; ++e) w.seed_ev_off[e] = (uint32_t)i;
  }
  const uint32_t per = (uint32_t)w.S * (uint32_t)w.R;
  for (int64_t i = g0; i <= nst; i += gs) {
    const int64_t ce = i < nst ? (int64_t)(w.cru[w.starts[i]] / per) : w.E;
    const int64_t pe = i > 0 ? (int64_t)(w.cru[w.starts[i - 1]] / per) : -1;
    for (int64_t e = pe + 1; e <= ce; ++e) w.start_ev_off[e] = (uint32_t)i;
  }
}

__global__ __launch_bounds__(TB) void k_start_tap(Ws w) {
  const uint32_t nst = w.flags[F_NSTARTS];
  const uint32_t per = (uint32_t)w.S * (uint32_t)w.R;
  for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < nst; i += (int64_t)gridDim.x * TB) {
    const uint32_t p = w.starts[i];
    const int e = (int)(w.cru[p] / per);
    const EventOut& O = w.out[e];
    if (O.dbg_start) O.dbg_start[i - w.start_ev_off[e]] = w.cid[p];
  }
}

// ----------------------------------------------------------- a5: tracklets
struct Found { int32_t pos; float y, z; };

// Closest cluster of row unit ru to the predicted (y, z):
// d = dy^2/(Cyy + sy^2) + dz^2/(Czz + sz^2) <= chi2_ext, minimum (d, id).
// The candidates are the 12-byte (y, z, canonical position) search records
// (the winner's x is read from the canonical arrays only in row units with
// clusters off the row plane).  The cell ranges of the box's first two z
// rows are read together, then their entries in chunks of eight loads issued
// before any is tested, so a step waits for memory twice rather than once
// per candidate.  The result does not depend on the order the candidates
// are visited in.
__device__ __forceinline__ Found search_row(const Ws& w, const GridParams& G, const float p[5],
                                            const float C[15]) {
  const float sy2 = C[0] + w.m.vy, sz2 = C[5] + w.m.vz;
  const float isy = 1.0f / sy2, isz = 1.0f / sz2;
  const float CUT = w.P.chi2_ext;
  // the window only bounds the cells scanned: the hardware square root
  // (1 ulp) is enough under the 1e-4 relative and 1e-3 cm margins, which
  // keep the scanned cells a superset of every cluster passing the cut
  const float wy = 3.0f * __builtin_amdgcn_sqrtf(sy2) * 1.0001f;
  const float wz = 3.0f * __builtin_amdgcn_sqrtf(sz2) * 1.0001f;
  const CellBox b = cell_box(G, p[0], p[1], wy, wz);
  // (bd, pos) starts at (CUT, INT32_MAX): the first candidate with d <= CUT
  // replaces it, later ones must beat the best so far, so no separate test
  // of the cut (a NaN distance fails every comparison)
  Found best{INT32_MAX, 0.f, 0.f};
  float bd = CUT;
  auto consider = [&](const SearchRec& c) {
    const float dY = c.y - p[0], dZ = c.z - p[1];
    const float d = fmaf(dZ * dZ, isz, (dY * dY) * isy);
    const int32_t pos = (int32_t)c.pos;
    if (d < bd || (d == bd && pos < best.pos)) { best = Found{pos, c.y, c.z}; bd = d; }
  };
  const uint32_t nzr = b.iz1 - b.iz0 + 1;
  const uint32_t c0a = G.cell_base + b.iz0 * G.ny;
  const uint32_t c0b = c0a + G.ny;
  const uint32_t ka0 = G.base + w.cell_off[c0a + b.iy0], ka1 = G.base + w.cell_off[c0a + b.iy1 + 1];
  uint32_t kb0 = 0, kb1 = 0;
  if (nzr > 1) { kb0 = G.base + w.cell_off[c0b + b.iy0]; kb1 = G.base + w.cell_off[c0b + b.iy1 + 1]; }
  // entries of the two ranges as one sequence t = 0 .. na + nb - 1
  const uint32_t na = ka1 - ka0, nt = na + (kb1 - kb0);
  constexpr uint32_t kChunk = 8;
  for (uint32_t t0 = 0; t0 < nt; t0 += kChunk) {
    SearchRec c[kChunk];
#pragma unroll
    for (uint32_t j = 0; j < kChunk; ++j) {
      const uint32_t t = t0 + j;
      if (t < nt) c[j] = w.grec[t < na ? ka0 + t : kb0 + (t - na)];
    }
#pragma unroll
    for (uint32_t j = 0; j < kChunk; ++j)
      if (t0 + j < nt) consider(c[j]);
  }
  for (uint32_t iz = 2; iz < nzr; ++iz) {
    const uint32_t cz = G.cell_base + (b.iz0 + iz) * G.ny;
    const uint32_t k0 = G.base + w.cell_off[cz + b.iy0], k1 = G.base + w.cell_off[cz + b.iy1 + 1];
    for (uint32_t k = k0; k < k1; k += 4) {
      SearchRec c[4];
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j)
        if (k + j < k1) c[j] = w.grec[k + j];
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j)
        if (k + j < k1) consider(c[j]);
    }
  }
  if (best.pos == INT32_MAX) best.pos = -1;
  return best;
}

struct Acc { float tan_a, z_max; };

__device__ __forceinline__ bool accepted(float X, const Acc& a, const float p[5]) {
  const float lim = X * a.tan_a;
  return !(fabsf(p[0]) > lim || fabsf(p[1]) > a.z_max);
}

// Tracklet construction as a per-lane state machine: every loop iteration
// advances each lane by one row step, whatever phase it is in, so the lanes
// of a wave stay converged on the common transport.  Phases:
//   CHAIN  fit the next cluster of the seed's chain (no search);
//   UP     transport to the next row plane, acceptance, search, update;
//   BACK   transport back to the seed's first row, at most kBackRows rows
//          per step, no updates;
//   DOWN   as UP, downward from the row below the seed.
// A lane that finishes writes its tracklet and takes the next seed from a
// device counter (one atomic per wave).  The seed list is split into kXcd
// contiguous ranges with a counter each; a workgroup starts on the range of
// its XCD and moves on to the others once that one is used up.
enum : int { ST_CHAIN = 0, ST_UP = 1, ST_BACK = 2, ST_DOWN = 3, ST_DONE = 4, ST_IDLE = 5 };

__global__ __launch_bounds__(TB) void k_tracklets(Ws w) {
  __shared__ float sX[256];
  for (int r = threadIdx.x; r < w.R; r += TB) sX[r] = w.row_x[r];
  __syncthreads();
  const Acc acc{w.tan_a, w.z_max};
  const uint32_t ns = w.flags[F_NSEEDS];
  // when the lanes of the lower workgroups already outnumber the seeds they
  // take (and, by refills, finish) them all: this one has nothing to do
  if ((int64_t)blockIdx.x * TB >= (int64_t)ns) return;
  const int R = w.R;
  int phase = ST_IDLE;
  int64_t s = -1;
  int32_t* hits = nullptr;
  int32_t h0 = 0, nxt = -1;
  int r0 = 0, r = 0, rstate = 0, rlo = 0, rhi = 0, nhits = 0, gap = 0;
  uint32_t rubase = 0;
  float p[5], C[15], xc = 0.f;
  uint32_t iters = 0;
  int nupd = 0;   // Kalman updates of the current seed (the first three are compensated)
  // the record of the next chain cluster (nxt), loaded one step ahead
  float4 cn = make_float4(0.f, 0.f, 0.f, 0.f);
  // hit slots are written through a four-row buffer (rows are visited in
  // order within a phase), one 16-byte store per full group of four rows
  int32_t wb0 = 0, wb1 = 0, wb2 = 0, wb3 = 0;
  int wbase = -1;
  uint32_t wmask = 0;
  const int64_t bstride = (int64_t)w.seed_cap * 8;   // between the bands of one seed
  auto flush = [&]() {
    int32_t* q = hits + (int64_t)(wbase >> 3) * bstride + (wbase & 7);
    if (wmask == 0xFu) {
      *(int4*)q = make_int4(wb0, wb1, wb2, wb3);
    } else if (wmask) {
      if (wmask & 1u) q[0] = wb0;
      if (wmask & 2u) q[1] = wb1;
      if (wmask & 4u) q[2] = wb2;
      if (wmask & 8u) q[3] = wb3;
    }
    wmask = 0;
  };
  auto put = [&](int row, int32_t v) {
    const int b = row & ~3;
    if (b != wbase) { flush(); wbase = b; }
    const int q = row & 3;
    // value selects, not a store through a selected pointer: the latter
    // would put the buffer in scratch memory
    wb0 = q == 0 ? v : wb0;
    wb1 = q == 1 ? v : wb1;
    wb2 = q == 2 ? v : wb2;
    wb3 = q == 3 ? v : wb3;
    wmask |= 1u << q;
  };
  // seed range of this workgroup's XCD (workgroups are dispatched to the
  // XCDs round-robin), so that each XCD's L2 holds the grids of its sectors
  int rx = (int)(blockIdx.x % kXcd), tries = 0;
  while (true) {
    // every lane's steps are bounded (rows only move one way per phase), so
    // this cap is never reached by a correct kernel; it turns a defect into
    // an error instead of a hang
    if (++iters > (1u << 22)) { atomicOr(&w.flags[F_ERR], ERR_STUCK); break; }
    // finished lanes publish their tracklet and take new seeds
    if (phase == ST_DONE) {
      flush();
      wbase = -1;
      float* st = w.tl_state + s * kTl;
#pragma unroll
      for (int i = 0; i < 5; ++i) st[i] = p[i];
#pragma unroll
      for (int i = 0; i < 15; ++i) st[5 + i] = C[i];
      w.tl_nhits[s] = nhits;
      w.tl_range[s] = rlo | (rhi << 16);
      w.tl_key[s] = ((uint64_t)(uint32_t)nhits << 40) | ((uint64_t)(255 - r0) << 32) |
                    (uint64_t)(0xFFFFFFFFu - w.cid[h0]);
      phase = ST_IDLE;
    }
    bool want = phase == ST_IDLE && s != -2;
    uint64_t wm = __ballot(want);
    // refills stall the whole wave (counter, atomic, seed set-up): take new
    // seeds only once a quarter of the lanes wait, or no lane is working
    if (__popcll(wm) < kRefillMin && __ballot(phase != ST_IDLE) != 0ull) wm = 0ull;
    while (wm) {
      const uint32_t lo = (uint32_t)(((uint64_t)ns * (uint32_t)rx) / kXcd);
      const uint32_t hi = (uint32_t)(((uint64_t)ns * (uint32_t)(rx + 1)) / kXcd);
      uint32_t* ctr = &w.flags[F_SEEDCTR + rx];
      // a fresh (L2-bypassing) read first: exhausted ranges cost no atomic
      uint32_t base = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (base < hi - lo) {
        const int leader = __ffsll((unsigned long long)wm) - 1;
        if (lane_id() == leader) base = atomicAdd(ctr, (uint32_t)__popcll(wm));
        base = __shfl(base, leader, 64);
        if (want) {
          const uint64_t mine = (uint64_t)lo + base + (uint32_t)__popcll(wm & lanemask_lt());
          if (mine < hi) {
            want = false;
            s = (int64_t)mine;
            h0 = (int32_t)w.seeds[s];
            const uint32_t ru0 = w.cru[h0];
            r0 = (int)(ru0 % (uint32_t)R);
            rubase = ru0 - (uint32_t)r0;
            hits = w.tl_hits + s * 8;
            const float4 a0 = w.cpk[h0];
            const int32_t h1 = __float_as_int(a0.w);
            const float4 a1 = w.cpk[h1];
            const int32_t h2 = __float_as_int(a1.w);
            const float4 a2 = w.cpk[h2];
            float sdir, tdir;
            const float x0 = a0.x, y0 = a0.y, z0 = a0.z;
            chord_dir(x0, y0, z0, a2.x, a2.y, a2.z, sdir, tdir);
            p[0] = y0; p[1] = z0; p[2] = sdir; p[3] = tdir; p[4] = 0.0f;
            init_cov(C, w.m.vy, w.m.vz);
            nupd = 0;
            rlo = rhi = rstate = r0;
            xc = x0;
            if (fabsf(sdir) < w.m.sin_max) {
              put(r0, h0);
              nhits = 1;
              nxt = h1;
              cn = a1;
              phase = ST_CHAIN;
            } else {
              nhits = 0;
              phase = ST_DONE;
            }
          }
        }
      }
      wm = __ballot(want);
      if (wm) {
        // this range is used up: take seeds from the next one
        if (++tries >= kXcd) {
          if (want) s = -2;   // every range is used up: no more work for this lane
          break;
        }
        rx = (rx + 1) % kXcd;
      }
    }
    if (__ballot(phase != ST_IDLE) == 0ull) break;
    if (phase == ST_DONE || phase == ST_IDLE) continue;
    // one row step: every active lane transports once (the target plane
    // depends on the phase), then the phase's own work follows
    const bool chain = phase == ST_CHAIN;
    const bool search = phase == ST_UP || phase == ST_DOWN;
    float X, my = 0.0f, mz = 0.0f;
    int32_t cnx = -1;
    GridParams G;
    if (chain) {
      X = cn.x; my = cn.y; mz = cn.z; cnx = __float_as_int(cn.w);
    } else {
      X = sX[r];
    }
    if (search) G = w.grid[rubase + (uint32_t)r];
    bool go = transport(p, C, xc, X, w.m);
    bool upd = false, wrote = false;
    if (chain) {
      upd = go;
    } else if (search && go) {
      xc = X;
      rstate = r;
      go = accepted(X, acc, p);
      if (go) {
        const Found h = search_row(w, G, p, C);
        if (h.pos >= 0) {
          float hx = X;
          if (G.off_plane) hx = w.cx[h.pos];
          if (hx != X) {
            go = transport(p, C, X, hx, w.m);
            if (go) xc = hx;
          }
          if (go) {
            my = h.y; mz = h.z;
            upd = true;
            put(r, h.pos);
            ++nhits;
            gap = 0;
            wrote = true;
          }
        } else {
          put(r, -1);
          ++gap;
          wrote = true;
        }
        if (wrote) go = gap <= w.P.max_gap;
      }
    }
    if (upd) {
      float dummy = 0.0f;
      if (nupd < TPCCA_GRAD_C2_UPDATES) update_c2(p, C, my, mz, w.m, dummy);
      else update(p, C, my, mz, w.m, dummy);
      ++nupd;
    }
    if (chain) {
      if (!go) {
        nhits = 0; rlo = rhi = r0; phase = ST_DONE;
      } else {
        ++rstate;
        put(rstate, nxt);
        ++nhits;
        xc = X;
        nxt = cnx;
        if (nxt < 0) {
          rhi = rstate;
          gap = 0;
          r = rstate + 1;
          phase = r < R ? ST_UP : ST_BACK;
          if (phase == ST_BACK) r = max(r0, rstate - kBackRows);
        }
      }
    } else if (phase == ST_BACK) {
      if (!go) {
        phase = ST_DONE;
      } else {
        xc = X;
        if (r == r0) {
          gap = 0;
          r = r0 - 1;
          phase = r >= 0 ? ST_DOWN : ST_DONE;
        } else {
          r = max(r0, r - kBackRows);
        }
      }
    } else if (phase == ST_UP) {
      if (wrote) rhi = r;
      if (go && r + 1 < R) {
        ++r;
      } else {
        if (rstate > r0) {
          r = max(r0, rstate - kBackRows);
          phase = ST_BACK;
        } else {
          gap = 0;
          r = r0 - 1;
          phase = r >= 0 ? ST_DOWN : ST_DONE;
        }
      }
    } else {
      if (wrote) rlo = r;
      if (go && r - 1 >= 0) --r; else phase = ST_DONE;
    }
    // the next chain record, loaded now so that it is there when the next
    // step's transport needs its plane
    if (phase == ST_CHAIN) cn = w.cpk[nxt];
  }
}

// ----------------------------------------------------------- a6: selection
// Ownership by bands of kBandRows pad rows of one (event, sector): tracklets
// of different sectors never share a cluster, so the workgroup of a band
// scans its sector's tracklets (four lanes per tracklet, one per row) and
// takes the key maximum of each of the band's clusters with LDS atomics,
// then writes the band's owners out in order.  A band with more than
// kBandCap clusters uses global atomics on the (zeroed) owner array instead.
constexpr int kBandRows = 8;
constexpr int kBandCap = 6144;
// threads of an ownership workgroup: 1024 where the sectors hold many
// tracklets (short chains of dependent loads per thread), TB for batches of
// small events (few tracklets per band, many workgroups)
constexpr int TBO = 1024;

__global__ __launch_bounds__(TBO) void k_owner(Ws w) {
  const uint32_t nt = blockDim.x;   // (TBO for events of many tracklets, TB otherwise)
  __shared__ unsigned long long s_own[kBandCap];
  const int nband = (w.R + kBandRows - 1) / kBandRows;
  const int64_t su = blockIdx.x / nband;
  const int r_lo = (int)(blockIdx.x % nband) * kBandRows;
  const int r_hi = min(r_lo + kBandRows, w.R) - 1;
  const uint32_t c0 = w.ru_off[su * w.R + r_lo], c1 = w.ru_off[su * w.R + r_hi + 1];
  const uint32_t nc = c1 - c0;
  const bool lds = nc <= (uint32_t)kBandCap;
  // every cluster lies in one band, whose workgroup alone takes its
  // maxima: in LDS or, for bands above the LDS capacity, by global atomics
  // on entries this workgroup clears
  if (lds)
    for (uint32_t i = threadIdx.x; i < nc; i += nt) s_own[i] = 0ull;
  else
    for (uint32_t i = threadIdx.x; i < nc; i += nt) w.owner[c0 + i] = 0ull;
  __syncthreads();
  // one thread per tracklet: the band's eight hit slots are two aligned
  // 16-byte loads, and the band's slots of consecutive tracklets are
  // contiguous (hit_slot), so a wave reads them in whole lines
  static_assert(kBandRows == 8, "two int4 of hit slots per band");
  const uint32_t s0 = w.seed_su_off[su], s1 = w.seed_su_off[su + 1];
  constexpr int kUn = 2;   // passes whose loads are issued together
  for (uint32_t sb = s0; sb < s1; sb += nt * kUn) {
    int32_t rg[kUn], nh[kUn];
    int4 hh[kUn], hh2[kUn];
    unsigned long long key[kUn];
    bool ok[kUn];
#pragma unroll
    for (int u = 0; u < kUn; ++u) {
      const uint32_t s = sb + u * nt + threadIdx.x;
      ok[u] = s < s1;
      const uint32_t sc = ok[u] ? s : s0;
      rg[u] = w.tl_range[sc];
      nh[u] = w.tl_nhits[sc];
      const int32_t* hb = w.tl_hits + hit_slot(w.seed_cap, sc, r_lo);   // (r_lo: a band's first row)
      hh[u] = *(const int4*)hb;
      hh2[u] = *(const int4*)(hb + 4);
      key[u] = w.tl_key[sc];
    }
#pragma unroll
    for (int u = 0; u < kUn; ++u) {
      if (!ok[u] || nh[u] < w.P.min_hits) continue;
      const int rlo = rg[u] & 0xFFFF, rhi = rg[u] >> 16;
      const int32_t hq[8] = {hh[u].x, hh[u].y, hh[u].z, hh[u].w, hh2[u].x, hh2[u].y, hh2[u].z, hh2[u].w};
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int r = r_lo + q;
        const int32_t h = hq[q];
        if (r > r_hi || r < rlo || r > rhi || h < 0) continue;
        if (lds) atomicMax(&s_own[(uint32_t)h - c0], key[u]);
        else if (w.owner[h] < key[u]) atomicMax((unsigned long long*)&w.owner[h], key[u]);
      }
    }
  }
  __syncthreads();
  // the band's maxima are final: every tracklet of the sector gets the mask
  // of the band's rows whose hit it owns (its key is the maximum there),
  // written beside those of the neighbouring tracklets
  uint8_t* mk = w.own_mask + (int64_t)(r_lo >> 3) * w.seed_cap;
  for (uint32_t s = s0 + threadIdx.x; s < s1; s += nt) {
    const int32_t rg = w.tl_range[s];
    const int nh = w.tl_nhits[s];
    const int32_t* hb = w.tl_hits + hit_slot(w.seed_cap, s, r_lo);
    const int4 a = *(const int4*)hb, b = *(const int4*)(hb + 4);
    const unsigned long long key = w.tl_key[s];
    uint32_t m = 0;
    if (nh >= w.P.min_hits) {
      const int rlo = rg & 0xFFFF, rhi = rg >> 16;
      const int32_t hq[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int r = r_lo + q;
        const int32_t h = hq[q];
        if (r > r_hi || r < rlo || r > rhi || h < 0) continue;
        // (bands above the LDS capacity: the maxima are this workgroup's
        // atomics, read past the compute unit's cache)
        const unsigned long long mx =
            lds ? s_own[(uint32_t)h - c0] : __hip_atomic_load(&w.owner[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (mx == key) m |= 1u << q;
      }
    }
    mk[s] = (uint8_t)m;
  }
}

// ------------------------------------------------ a6/a7: accept + final fit
// Acceptance: count the hits a tracklet owns (outermost first), keep them as
// a compact list tl_own[s][0..cnt) and flag the tracklet if it owns at least
// min_hits and owned_num/owned_den of its hits.  One wave per tracklet: 64
// rows per pass from the outermost down, compacted with a ballot.
__global__ __launch_bounds__(TB) void k_accept(Ws w) {
  // half a wave (32 lanes) per tracklet, two tracklets per wave in flight;
  // the tracklets of one XCD's seed range go to that XCD's workgroups
  const uint32_t ns = w.flags[F_NSEEDS];
  const int lane = lane_id(), hl = lane & 31;
  const uint64_t half = (lane < 32) ? 0x00000000FFFFFFFFull : 0xFFFFFFFF00000000ull;
  const uint32_t x = blockIdx.x % kXcd;
  const int64_t lo = (int64_t)(((uint64_t)ns * x) / kXcd), hi = (int64_t)(((uint64_t)ns * (x + 1)) / kXcd);
  const int64_t first = lo + (int64_t)(blockIdx.x / kXcd) * (TB / 32) + (threadIdx.x >> 5);
  const int64_t stride = (int64_t)(gridDim.x / kXcd) * (TB / 32);
  for (int64_t s = first; s < hi; s += stride) {
    uint32_t acc = 0, cnt = 0;
    // the two are loaded together (one memory round trip): no branch
    // around the rest, whose loads and stores are predicated on ok instead
    const int nh = w.tl_nhits[s];
    const int32_t rg = w.tl_range[s];
    const bool ok = nh >= w.P.min_hits;
    const int rlo = rg & 0xFFFF, rhi = rg >> 16;
    const int32_t* hits = w.tl_hits + s * 8;
    const int64_t bstride = (int64_t)w.seed_cap * 8;
    const uint8_t* mk = w.own_mask + s;
    int32_t* own = w.tl_own + s * w.R;
    // a list spans at most eight passes of 32 rows (<= 255 rows): read all
    // hit slots and the owned-row masks of their bands, then compact pass
    // by pass
    constexpr int kPass = 8;
    int32_t h[kPass];
    uint32_t mb[kPass];
#pragma unroll
    for (int c = 0; c < kPass; ++c) {
      const int r = rhi - hl - 32 * c;
      const bool in = ok && r >= rlo;
      h[c] = in ? hits[(int64_t)(r >> 3) * bstride + (r & 7)] : -1;
      mb[c] = in ? ((uint32_t)mk[(int64_t)(r >> 3) * w.seed_cap] >> (r & 7)) & 1u : 0u;
    }
#pragma unroll
    for (int c = 0; c < kPass; ++c) {
      const bool mine = h[c] >= 0 && mb[c] != 0u;
      const uint64_t m = __ballot(mine) & half;
      if (mine) own[cnt + (uint32_t)__popcll(m & lanemask_lt())] = h[c];
      cnt += (uint32_t)__popcll(m);
    }
    acc = (ok && (int)cnt >= w.P.min_hits && (int64_t)w.P.owned_den * cnt >= (int64_t)w.P.owned_num * nh) ? 1u : 0u;
    if (hl == 0) {
      w.acc_flag[s] = acc;
      w.own_cnt[s] = acc ? cnt : 0u;
    }
  }
  // slots past the seed count (scanned with the others)
  for (int64_t s = (int64_t)ns + (int64_t)blockIdx.x * TB + threadIdx.x; s < w.seed_cap;
       s += (int64_t)gridDim.x * TB) {
    w.acc_flag[s] = 0u;
    w.own_cnt[s] = 0u;
  }
}

__global__ __launch_bounds__(TB) void k_acc_list(Ws w) {
  for (int64_t s = (int64_t)blockIdx.x * TB + threadIdx.x; s < w.seed_cap; s += (int64_t)gridDim.x * TB) {
    const uint32_t a = w.acc_off[s];
    if (w.acc_off[s + 1] != a) w.acc_list[a] = (uint32_t)s;
  }
}

// Final fit of every accepted tracklet (dense over the accepted list):
// outermost owned hit first, direction from the chord to the hit two
// positions inward, q/pT prior from following; the next hit's coordinates
// are loaded while the current step computes.
__global__ __launch_bounds__(TB) void k_refit(Ws w) {
  const uint32_t na = w.acc_off[w.seed_cap];
  for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < na; i += (int64_t)gridDim.x * TB) {
    const int64_t s = w.acc_list[i];
    const int32_t* own = w.tl_own + s * w.R;
    const uint32_t cnt = w.own_cnt[s];
    float p[5], C[15], sdir, tdir;
    const int32_t o0 = own[0], o2 = own[2];
    const float4 c0 = w.cpk[o0], c2 = w.cpk[o2];
    const float xo = c0.x, yo = c0.y, zo = c0.z;
    chord_dir(c2.x, c2.y, c2.z, xo, yo, zo, sdir, tdir);
    const float kpr = w.tl_state[s * kTl + 4];
    p[0] = yo; p[1] = zo; p[2] = sdir; p[3] = tdir; p[4] = kpr;
    init_cov(C, w.m.vy, w.m.vz);
    float chi2 = 0.0f;
    bool ok = fabsf(sdir) < w.m.sin_max;
    float xc = xo;
    // hit records are read four steps ahead of their use and hit indices
    // eight steps ahead, so loads overlap the filter steps.  The loop is
    // unrolled by four with one register slot per step: a slot is refilled
    // right after its use, and no register moves (which would wait for the
    // loads in flight) rotate the slots.
    float4 q0 = w.cpk[own[1]];
    float4 q1 = w.cpk[2 < cnt ? own[2] : o0];
    float4 q2 = w.cpk[3 < cnt ? own[3] : o0];
    float4 q3 = w.cpk[4 < cnt ? own[4] : o0];
    int32_t j0 = own[5 < cnt ? 5u : 0u], j1 = own[6 < cnt ? 6u : 0u];
    int32_t j2 = own[7 < cnt ? 7u : 0u], j3 = own[8 < cnt ? 8u : 0u];
    // (past the list's end a slot is refilled from the first hit, never
    // used: loads made by every step, whether its hit exists or not, leave
    // no register to merge after them)
    // The refill is issued after the step's arithmetic, when the slot's old
    // value is dead, so it lands in the same registers.
    auto step = [&](float4& q, int32_t& j, uint32_t k) {
      if (ok && k < cnt) {
        if (transport(p, C, xc, q.x, w.m)) {
          if (k <= (uint32_t)TPCCA_GRAD_C2_UPDATES) update_c2(p, C, q.y, q.z, w.m, chi2);
          else update(p, C, q.y, q.z, w.m, chi2);
          xc = q.x;
        } else {
          ok = false;
        }
      }
      q = w.cpk[k + 4 < cnt ? j : o0];
      j = own[k + 8 < cnt ? k + 8 : 0u];
    };
    for (uint32_t k = 1; ok && k < cnt; k += 4) {
      step(q0, j0, k);
      step(q1, j1, k + 1);
      step(q2, j2, k + 2);
      step(q3, j3, k + 3);
    }
    if (ok) {
      float* rf = w.rf + s * kRf;
      rf[0] = xc;
#pragma unroll
      for (int q = 0; q < 5; ++q) rf[1 + q] = p[q];
#pragma unroll
      for (int q = 0; q < 15; ++q) rf[6 + q] = C[q];
      rf[21] = chi2;
      rf[22] = kpr;
    } else {
      w.own_cnt[s] = 0u;          // a failed fit produces no track
    }
  }
}


// Per-event totals and the capacity check.
__global__ __launch_bounds__(TB) void k_totals(Ws w) {
  __shared__ int s_fit;
  if (threadIdx.x == 0) s_fit = 1;
  __syncthreads();
  for (int e = threadIdx.x; e < w.E; e += TB) {
    const uint32_t b = w.seed_ev_off[e], en = w.seed_ev_off[e + 1];
    const int64_t nt = (int64_t)w.trk_flag[en] - (int64_t)w.trk_flag[b];
    const int64_t nh = (int64_t)w.hit_cnt[en] - (int64_t)w.hit_cnt[b];
    w.ev_res[e * 4 + 0] = nt;
    w.ev_res[e * 4 + 1] = nh;
    w.ev_res[e * 4 + 2] = (int64_t)w.start_ev_off[e + 1] - (int64_t)w.start_ev_off[e];
    const EventOut& O = w.out[e];
    const bool fit = nt <= O.cap_tracks && nh <= O.cap_hits;
    w.ev_res[e * 4 + 3] = fit ? 1 : 0;
    if (!fit) atomicAnd(&s_fit, 0);
  }
  __syncthreads();
  const bool go = s_fit && w.flags[F_ERR] == 0u;
  if (threadIdx.x == 0) w.flags[F_FITS] = go ? 1u : 0u;
  if (go)
    for (int e = threadIdx.x; e < w.E; e += TB)
      w.out[e].hit_off[w.ev_res[e * 4 + 0]] = (int32_t)w.ev_res[e * 4 + 1];
}

// One wave per accepted tracklet (the ordered accepted list; those whose
// fit failed are skipped): scalars spread over the lanes, the hit list
// written in whole cache lines (innermost first).
__global__ __launch_bounds__(TB) void k_write(Ws w) {
  if (w.flags[F_FITS] == 0u) return;
  const uint32_t na = w.acc_off[w.seed_cap];
  const int lane = lane_id();
  const int64_t nw = (int64_t)gridDim.x * (TB / 64);
  for (int64_t i = (int64_t)blockIdx.x * (TB / 64) + (threadIdx.x >> 6); i < na; i += nw) {
    const int64_t s = w.acc_list[i];
    // everything indexed by s in one round trip
    const uint32_t t0 = w.trk_flag[s], t1 = w.trk_flag[s + 1];
    const uint32_t c0 = w.hit_cnt[s], c1 = w.hit_cnt[s + 1];
    const int32_t h0 = (int32_t)w.seeds[s];
    if (t1 == t0) continue;
    const uint32_t vsec = w.cru[h0] / (uint32_t)w.R;
    const int e = (int)(vsec / (uint32_t)w.S);
    const EventOut& O = w.out[e];
    // offsets within the event (a single event starts at zero)
    uint32_t j = t0, o = c0;
    if (w.E > 1) {
      const uint32_t sb = w.seed_ev_off[e];
      j = t0 - w.trk_flag[sb];
      o = c0 - w.hit_cnt[sb];
    }
    const uint32_t n = c1 - c0;
    const float* rf = w.rf + s * kRf;
    if (lane < 5) O.p[j * 5 + lane] = rf[1 + lane];
    else if (lane < 20) O.cov[j * 15 + (lane - 5)] = rf[6 + (lane - 5)];
    else if (lane == 20) O.x_ref[j] = rf[0];
    else if (lane == 21) O.chi2[j] = rf[21];
    else if (lane == 22) { if (O.k_prior) O.k_prior[j] = rf[22]; }
    else if (lane == 23) O.sector[j] = (uint8_t)(vsec % (uint32_t)w.S);
    else if (lane == 24) O.ndf[j] = 2 * (int32_t)n - 5;
    else if (lane == 25) O.hit_off[j] = (int32_t)o;
    const int32_t* own = w.tl_own + s * w.R;
    for (uint32_t q = lane; q < n; q += 64) O.hit_id[o + q] = w.cid[own[n - 1 - q]];
  }
}

}  // namespace

// Exclusive scan of n values into out[0 .. n] (out[n] = total); part holds
// 2 (n / 1024 + 2) values.
hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* part, hipStream_t st) {
  return scan_u32(in, out, n, part, st);
}

// Persistent grid of the tracklet kernel: one lane per possible seed (the
// workgroups past the actual seed count leave at once), or the tuned value.
unsigned tracklet_grid(const Ws& w) {
  if (w.tracklet_grid > 0) return (unsigned)w.tracklet_grid;
  return blocks_for(w.seed_cap, 1 << 16);
}

namespace {
// FP32 building blocks of the bit-exact contract, elementwise, compiled with
// the flags of the tracking kernels: op 0 sqrt_rn_normal(a), 1 a / b,
// 2 1 / a, 3 sqrtf(a).
__global__ __launch_bounds__(TB) void k_fp32_probe(int op, int64_t n, const float* __restrict__ a,
                                                   const float* __restrict__ b, float* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
    const float x = a[i];
    float r;
    if (op == 0) r = sqrt_rn_normal(x);
    else if (op == 1) r = x / b[i];
    else if (op == 2) r = 1.0f / x;
    else r = sqrtf(x);
    out[i] = r;
  }
}
}  // namespace

hipError_t fp32_probe(int op, int64_t n, const float* a, const float* b, float* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_fp32_probe<<<blocks_for(n, 1 << 14), TB, 0, st>>>(op, n, a, b, out);
  return hipGetLastError();
}

hipError_t fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_fill<<<blocks_for(n, 4096), TB, 0, st>>>(p, v, n);
  return hipGetLastError();
}

hipError_t run_pipeline(const Ws& w, hipStream_t st, const PhaseEvents* pe) {
  hipError_t e;
#define TPCCA_CHECK(x) do { if ((e = (x)) != hipSuccess) return e; } while (0)
#define TPCCA_MARK(i) do { if (pe) TPCCA_CHECK(hipEventRecord(pe->ev[i], st)); } while (0)
  TPCCA_MARK(PH_ZERO);
  k_zero2<<<blocks_for(F_COUNT + w.RU, 4096), TB, 0, st>>>(w.flags, F_COUNT, w.ru_count, w.RU);
  TPCCA_CHECK(hipGetLastError());
  TPCCA_MARK(PH_COUNT);
  const unsigned nchunk = (unsigned)chunk_cap(w.N, w.E);
  k_count<<<nchunk, TBB, 0, st>>>(w);
  TPCCA_CHECK(hipGetLastError());
  TPCCA_MARK(PH_SCAN);
  if (w.RU <= kScanSmall) {
    k_scan_rows<<<1, kScanNT, 0, st>>>(w);
    TPCCA_CHECK(hipGetLastError());
  } else {
    k_cell_caps<<<blocks_for(w.RU), TB, 0, st>>>(w);
    TPCCA_CHECK(scan_u32x2(w.ru_count, w.ru_off, w.cell_cap, w.cell_base, w.RU, w.scan_tmp, st));
    TPCCA_CHECK(fill_u32(w.ru_count, 0u, w.RU, st));
  }
  TPCCA_MARK(PH_SCATTER);
  k_scatter<<<nchunk, TBB, 0, st>>>(w);
  TPCCA_MARK(PH_ROWS);
  const bool lists = ru_lists(w.RU);
  const unsigned g_all = (unsigned)w.RU;
  const unsigned g_mid = lists ? std::min(g_all, kListGrid) : g_all, g_big = lists ? std::min(g_all, kListGridBig) : g_all;
  const unsigned g_wave = (unsigned)((w.RU + TB / 64 - 1) / (TB / 64));
  k_rows_tiny<<<g_wave, TB, 0, st>>>(w);
  k_rows_wave<<<lists ? std::min(g_wave, kListGrid) : g_wave, TB, 0, st>>>(w);
  k_rows<false><<<g_mid, TB, 0, st>>>(w);
  k_rows<true><<<g_big, TB, 0, st>>>(w);
  TPCCA_CHECK(hipGetLastError());
  const unsigned nbN = (unsigned)w.nb;
  TPCCA_MARK(PH_LINKS);
  k_links<kTiny, 64><<<g_wave, TB, 0, st>>>(w);
  k_links<kSmallSlab, TB><<<g_mid, TB, 0, st>>>(w);
  k_links<kSlab, TB><<<g_big, TB, 0, st>>>(w);
  TPCCA_MARK(PH_CLEAN);
  k_clean<<<nbN, TB, 0, st>>>(w);
  TPCCA_MARK(PH_COMPACT);
  TPCCA_CHECK(scan_u32x2(w.blk_start, w.blk_start, w.blk_seed, w.blk_seed, w.nb, w.scan_tmp, st));
  k_compact<<<nbN, TB, 0, st>>>(w);
  k_ev_offsets<<<blocks_for(w.N / 2 + 2, 4096), TB, 0, st>>>(w);
  if (w.taps) k_start_tap<<<blocks_for(w.N / 2 + 1, 2048), TB, 0, st>>>(w);
  TPCCA_CHECK(hipGetLastError());
  TPCCA_MARK(PH_TRACKLETS);
  k_tracklets<<<tracklet_grid(w), TB, 0, st>>>(w);
  TPCCA_CHECK(hipGetLastError());
  TPCCA_MARK(PH_OWNER);
  k_owner<<<(unsigned)((int64_t)w.E * w.S * ((w.R + kBandRows - 1) / kBandRows)),
             w.N / std::max(w.E, 1) >= ((int64_t)1 << 20) ? TBO : TB, 0, st>>>(w);
  TPCCA_MARK(PH_REFIT);
  k_accept<<<xcd_blocks(w.seed_cap * 32), TB, 0, st>>>(w);
  TPCCA_CHECK(scan_u32(w.acc_flag, w.acc_off, w.seed_cap, w.scan_tmp, st));
  k_acc_list<<<blocks_for(w.seed_cap, 4096), TB, 0, st>>>(w);
  k_refit<<<blocks_for(w.seed_cap / 4 + 1, 4096), TB, 0, st>>>(w);
  TPCCA_MARK(PH_OUTPUT);
  // track offsets (indicator of a fitted track) and hit offsets (owned
  // count) from the owned counts, by the same launches
  TPCCA_CHECK(scan_u32x2(w.own_cnt, w.trk_flag, w.own_cnt, w.hit_cnt, w.seed_cap, w.scan_tmp, st, 1));
  k_totals<<<1, TB, 0, st>>>(w);
  k_write<<<blocks_for(w.seed_cap * 16, 1 << 13), TB, 0, st>>>(w);
  TPCCA_CHECK(hipGetLastError());
  TPCCA_MARK(PH_N);
#undef TPCCA_MARK
#undef TPCCA_CHECK
  return hipSuccess;
}

}  // namespace tpcca
