// tpcca_merge.hip -- sector track merger on gfx950.
//
// Paper, Sec. "Track reconstruction in the TPC": the TPC sectors are tracked
// independently and their track segments are merged afterwards; the final
// refit of the merged tracks runs on the GPU.  Rules (the paper gives none;
// these are the library's reading): a segment's exit state is its fitted
// state transported to its outermost hit; a pair (inner a, outer b) in
// adjacent wedges of one side is a candidate if a's last pad row is below
// b's first and a's outermost hit lies within merge_dist of b's innermost
// hit (transverse and z); its match chi2 compares a's exit state, rotated
// into b's frame and transported to b's reference plane, with b's state
// under the summed covariance; links are mutual best pairs under
// chi2_merge; chains of linked segments are refitted as one track, the
// state rotated into the next inner segment's frame at each boundary.  In
// a time frame (slice indices given) two segments of one sector from
// neighbouring slices are candidates too, under the same row and distance
// conditions, and share the frame (no rotation).
//
// Kernels, one lane per segment unless noted: exit states and hit ends,
// segments listed by sector, candidate search (each outer segment scans the
// two neighbouring sectors' lists, and its own in a time frame; keys (chi2
// bits, index) taken by atomic
// minimum, so the result does not depend on the scan order), mutual links,
// chain walk and merged refit (lane per chain head), output offsets
// (exclusive scans), output writing (lane per chain head).
#include <algorithm>

#include "kf_c2.hpp"
#include "merge_internal.hpp"

namespace tpcca {
namespace {

constexpr int TB = 256;
constexpr unsigned long long kNone = ~0ull;

// Rotation of a state at plane x into a frame turned by the angle with
// cosine ca and sine sa about z (tracks move outward in x, so cos phi > 0):
// the point (x ca + y sa, -x sa + y ca), sin phi' = s ca - c sa; covariance
// J C J^T with the Jacobian at the fixed new plane (dy'/dy = ca - tan phi'
// sa, dz'/dy = -(t / cos phi') sa, ds'/dy = -kap sa, ds'/ds = ca + sa s/c;
// z, tan lambda, q/pT kept).  False if |sin phi'| reaches sin_max.
__device__ bool rotate_state(float& x, float p[5], float C[15], float ca, float sa, const Model& m) {
  const float s = p[2];
  const float c = sqrtf(fmaf(-s, s, 1.0f));
  const float s2 = s * ca - c * sa;
  if (!(fabsf(s2) < m.sin_max)) return false;
  const float c2 = sqrtf(fmaf(-s2, s2, 1.0f));
  const float kap = m.kfac * p[4];
  float J[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) J[i][j] = i == j ? 1.0f : 0.0f;
  J[0][0] = ca - (s2 / c2) * sa;
  J[1][0] = -(p[3] / c2) * sa;
  J[2][0] = -kap * sa;
  J[2][2] = ca + sa * (s / c);
  float T[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k < 5; ++k) acc += J[i][k] * C[sym(k, j)];
      T[i][j] = acc;
    }
  float Cn[15];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = i; j < 5; ++j) {
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k < 5; ++k) acc += T[i][k] * J[j][k];
      Cn[sym(i, j)] = acc;
    }
#pragma unroll
  for (int i = 0; i < 15; ++i) C[i] = Cn[i];
  const float x2 = x * ca + p[0] * sa;
  p[0] = -(x * sa) + p[0] * ca;
  p[2] = s2;
  x = x2;
  return true;
}

// d^T M^-1 d by the Cholesky factor of M scaled to a unit diagonal (the
// five parameters differ by orders of magnitude in their variances).
__device__ bool match_chi2(const float d[5], const float M[15], float& chi2) {
  float is[5], e[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const float v = M[sym(i, i)];
    if (!(v > 0.0f)) return false;
    is[i] = 1.0f / sqrtf(v);
    e[i] = d[i] * is[i];
  }
  float L[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      float acc = i == j ? 1.0f : M[sym(i, j)] * is[i] * is[j];
#pragma unroll
      for (int k = 0; k < j; ++k) acc -= L[i][k] * L[j][k];
      if (i == j) {
        if (!(acc > 0.0f)) return false;
        L[i][i] = sqrtf(acc);
      } else {
        L[i][j] = acc / L[j][j];
      }
    }
  float w[5];
  chi2 = 0.0f;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    float acc = e[i];
#pragma unroll
    for (int k = 0; k < i; ++k) acc -= L[i][k] * w[k];
    w[i] = acc / L[i][i];
    chi2 += w[i] * w[i];
  }
  return true;
}

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << (threadIdx.x & 63)) - 1ull; }

// Turn (sign of the adjacent-wedge angle) from the frame of wedge wa to that
// of wedge wb: +1 if wb follows wa counter-clockwise.
__device__ __forceinline__ float turn_sign(int wa, int wb, int NW) { return wb == (wa + 1) % NW ? 1.0f : -1.0f; }

__global__ __launch_bounds__(TB) void k_mrg_init(MergeWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i < (int64_t)w.S * w.nsl) { w.sec_cnt[i] = 0u; w.sec_cur[i] = 0u; }
  if (i < 4) w.err[i] = 0u;
  if (i < w.T) {
    w.best_in[i] = kNone;
    w.best_out[i] = kNone;
    w.link[i] = -1;
    w.inner[i] = -1;
    w.flags[i] = 0u;
  }
}

// (Sector, slice) histogram of a workgroup's segments in LDS, one global
// atomic per non-empty bin (the segments of a workgroup share few bins);
// with more bins than kSecBins, global atomics per segment.
constexpr int kSecBins = 256;

__device__ __forceinline__ uint32_t sec_bin(const MergeWs& w, int64_t i, int s) {
  return (uint32_t)s * (uint32_t)w.nsl + (uint32_t)(w.slice ? w.slice[i] : 0);
}

__global__ __launch_bounds__(TB) void k_mrg_ends(MergeWs w) {
  __shared__ uint32_t s_h[kSecBins];
  s_h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i < w.T) {
    const int32_t b0 = w.hit_off[i], b1 = w.hit_off[i + 1];
    const int s = w.sector[i];
    bool good = !(b0 < 0 || b1 - b0 < 3 || b1 - b0 > w.R || (int64_t)b1 > w.H || s >= w.S);
    if (!good) atomicOr(&w.err[0], 1u);
    uint32_t hf = 0, hl = 0;
    if (good) {
      hf = w.hit_id[b0];
      hl = w.hit_id[b1 - 1];
      if ((int64_t)hf >= w.NC || (int64_t)hl >= w.NC) { atomicOr(&w.err[0], 2u); good = false; }
    }
    if (good) {
      w.first[i] = make_float4(w.cx[hf], w.cy[hf], w.cz[hf], __int_as_float((int)w.crow[hf]));
      const float xo = w.cx[hl];
      w.last[i] = make_float4(xo, w.cy[hl], w.cz[hl], __int_as_float((int)w.crow[hl]));
      const uint32_t bin = sec_bin(w, i, s);
      if (w.S * w.nsl <= kSecBins) atomicAdd(&s_h[bin], 1u);
      else atomicAdd(&w.sec_cnt[bin], 1u);
      float p[5], C[15];
#pragma unroll
      for (int k = 0; k < 5; ++k) p[k] = w.p[i * 5 + k];
#pragma unroll
      for (int k = 0; k < 15; ++k) C[k] = w.cov[i * 15 + k];
      uint32_t f = 2u;                      // a well-formed segment
      if (transport(p, C, w.x_ref[i], xo, w.m)) {
        float* e = w.ex + i * 24;
        e[0] = xo;
#pragma unroll
        for (int k = 0; k < 5; ++k) e[1 + k] = p[k];
#pragma unroll
        for (int k = 0; k < 15; ++k) e[6 + k] = C[k];
        f = 3u;                             // ... with an exit state
      }
      w.flags[i] = f;
    }
  }
  __syncthreads();
  if (threadIdx.x < w.S * w.nsl && w.S * w.nsl <= kSecBins && s_h[threadIdx.x])
    atomicAdd(&w.sec_cnt[threadIdx.x], s_h[threadIdx.x]);
}

// Every well-formed segment takes a slot of its (sector, slice) list (the
// bins' offsets are the exclusive scan of the counts; a range per bin and
// workgroup, ranks in LDS) and writes there what the candidate search tests
// first: its outermost hit, last row and exit flag.
__global__ __launch_bounds__(TB) void k_mrg_secfill(MergeWs w) {
  __shared__ uint32_t s_h[kSecBins];
  const bool lds = w.S * w.nsl <= kSecBins;
  s_h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  const bool good = i < w.T && (w.flags[i] & 2u);
  const uint32_t bin = good ? sec_bin(w, i, (int)w.sector[i]) : 0u;
  uint32_t rank = 0;
  if (good) rank = lds ? atomicAdd(&s_h[bin], 1u) : atomicAdd(&w.sec_cur[bin], 1u);
  __syncthreads();
  if (lds && threadIdx.x < w.S * w.nsl && s_h[threadIdx.x])
    s_h[threadIdx.x] = atomicAdd(&w.sec_cur[threadIdx.x], s_h[threadIdx.x]);
  __syncthreads();
  if (good) {
    const uint32_t pos = w.sec_cnt[bin] + (lds ? s_h[bin] : 0u) + rank;
    const float4 l = w.last[i];
    const int sl = w.slice ? w.slice[i] : 0;   // (0 <= slice < 2^22, checked by the caller)
    w.sec_list[pos] = (uint32_t)i;
    w.srec[pos] = make_float4(l.x, l.y, l.z,
                              __int_as_float((sl << 9) | (__float_as_int(l.w) << 1) | (int)(w.flags[i] & 1u)));
  }
}

// Candidate search of outer segment b over the lists of the two
// neighbouring wedges of its side (and, in a time frame, of its own sector
// for segments of the neighbouring slices): one wave per b, its lanes taking
// every 64th record (the cheap tests on the record first), the best
// candidate the minimum of the lanes' (chi2 bits, index) keys.
__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)(v & 0xFFFFFFFFull), d, 64);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), d, 64);
    const unsigned long long o = ((unsigned long long)hi << 32) | lo;
    v = o < v ? o : v;
  }
  return v;
}

// Each (sector, slice) list of at most kZSort records sorted by the z of the
// outermost hit (bitonic in LDS on (z order bits, slot)), so that the
// candidate search reads only the part inside the z window; longer lists
// are copied as they are and scanned whole.
constexpr int kZSort = 2048;
constexpr int TBZ = 1024;

__global__ __launch_bounds__(TBZ) void k_mrg_zsort(MergeWs w) {
  __shared__ unsigned long long s_k[kZSort];
  const uint32_t bin = blockIdx.x;
  const uint32_t k0 = w.sec_cnt[bin], n = w.sec_cnt[bin + 1] - k0;
  if (n > (uint32_t)kZSort) {
    for (uint32_t i = threadIdx.x; i < n; i += TBZ) {
      w.zrec[k0 + i] = w.srec[k0 + i];
      w.zlist[k0 + i] = w.sec_list[k0 + i];
    }
    if (threadIdx.x == 0) w.zsorted[bin] = 0;
    return;
  }
  if (threadIdx.x == 0) w.zsorted[bin] = 1;
  if (n == 0) return;
  uint32_t npad = 1;
  while (npad < n) npad <<= 1;
  for (uint32_t i = threadIdx.x; i < npad; i += TBZ) {
    unsigned long long key = ~0ull;
    if (i < n) {
      // order-preserving bits of the float (negatives reversed below positives)
      const uint32_t u = __float_as_uint(w.srec[k0 + i].z);
      const uint32_t m = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
      key = ((unsigned long long)m << 32) | i;
    }
    s_k[i] = key;
  }
  __syncthreads();
  for (uint32_t kk = 2; kk <= npad; kk <<= 1) {
    for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < npad; i += TBZ) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const unsigned long long x = s_k[i], y = s_k[ixj];
          if ((x > y) == ((i & kk) == 0)) { s_k[i] = y; s_k[ixj] = x; }
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t i = threadIdx.x; i < n; i += TBZ) {
    const uint32_t src = (uint32_t)(s_k[i] & 0xFFFFFFFFull);
    w.zrec[k0 + i] = w.srec[k0 + src];
    w.zlist[k0 + i] = w.sec_list[k0 + src];
  }
}

__global__ __launch_bounds__(TB) void k_mrg_pairs(MergeWs w) {
  // records that pass the cheap tests, collected per wave and then tested
  // in full one per lane (the full test is long; survivors are few and
  // scattered over the lanes)
  __shared__ uint32_t s_cand[TB / 64][64];
  __shared__ uint8_t s_dir[TB / 64][64];
  const int wv = threadIdx.x >> 6;
  const int64_t b = (int64_t)blockIdx.x * (TB / 64) + wv;
  const int lane = threadIdx.x & 63;
  if (b >= w.T || w.err[0] != 0u || !(w.flags[b] & 2u) || w.NW < 3) return;
  const int sb = w.sector[b];
  const int wb = sb % w.NW, side0 = sb - wb;
  const float4 hb = w.first[b];
  const int rlo_b = __float_as_int(hb.w);
  const float xb = w.x_ref[b];
  const int slb = w.slice ? w.slice[b] : 0;
  unsigned long long best = kNone;
  int cnt = 0;                        // wave-uniform
  auto flush = [&]() {
    __builtin_amdgcn_wave_barrier();
    if (lane < cnt) {
      const uint32_t k = s_cand[wv][lane];
      const int dir = s_dir[wv][lane];
      const int wa = dir == 1 ? (wb + 1) % w.NW : (wb + w.NW - 1) % w.NW;
      const float sa = turn_sign(wa, wb, w.NW) * w.sa, ca = w.ca;
      const uint32_t a = w.zlist[k];
      const float* e = w.ex + (int64_t)a * 24;
      float x = e[0], q[5], Q[15];
#pragma unroll
      for (int j = 0; j < 5; ++j) q[j] = e[1 + j];
#pragma unroll
      for (int j = 0; j < 15; ++j) Q[j] = e[6 + j];
      float chi = 0.0f;
      bool ok = dir == 2 || rotate_state(x, q, Q, ca, sa, w.m);   // (one frame within a sector)
      if (ok) ok = transport(q, Q, x, xb, w.m);
      if (ok) {
        float d[5], M[15];
#pragma unroll
        for (int j = 0; j < 5; ++j) d[j] = q[j] - w.p[b * 5 + j];
#pragma unroll
        for (int j = 0; j < 15; ++j) M[j] = Q[j] + w.cov[b * 15 + j];
        ok = match_chi2(d, M, chi) && chi <= w.chi2_merge;
      }
      if (ok) {
        const unsigned long long cb = (unsigned long long)__float_as_uint(chi) << 32;
        best = min(best, cb | a);
        atomicMin(&w.best_out[a], cb | (unsigned long long)b);
      }
    }
    __builtin_amdgcn_wave_barrier();
    cnt = 0;
  };
  const int ndir = w.slice ? 3 : 2;
  // hit ends outside [zlo, zhi] fail the window test (the margin covers the
  // rounding of the bounds and of the test's difference)
  const float zlo = (hb.z - w.merge_dist) - 0.01f, zhi = (hb.z + w.merge_dist) + 0.01f;
  // the list of bin for direction dir: in a z-sorted list, from the last of
  // 64 evenly spaced probes below zlo up to the first chunk wholly above zhi
  auto scan = [&](int dir, float ca, float sa, uint32_t bin) {
    uint32_t k0 = w.sec_cnt[bin];
    const uint32_t k1 = w.sec_cnt[bin + 1];
    if (k0 >= k1) return;
    const bool zs = w.zsorted[bin] != 0;
    if (zs) {
      const uint32_t step = (k1 - k0 + 63) / 64;
      const uint32_t at = k0 + (uint32_t)lane * step;
      const int c = __popcll(__ballot(at < k1 && w.zrec[at].z < zlo));
      if (c > 0) k0 += (uint32_t)(c - 1) * step;
    }
    for (uint32_t kb = k0; kb < k1; kb += 64) {
      const uint32_t k = kb + (uint32_t)lane;
      bool pass = false, inside = false;
      if (k < k1) {
        const float4 ha = w.zrec[k];
        inside = !(ha.z > zhi);
        const int bits = __float_as_int(ha.w);
        const int dsl = (bits >> 9) - slb;
        if ((bits & 1) && ((bits >> 1) & 0xFF) < rlo_b && (dir < 2 || dsl == 1 || dsl == -1)) {
          const float xa = ha.x * ca + ha.y * sa, ya = -(ha.x * sa) + ha.y * ca;
          const float dX = xa - hb.x, dY = ya - hb.y;
          const float dr = sqrtf(dX * dX + dY * dY);
          pass = dr <= w.merge_dist && fabsf(ha.z - hb.z) <= w.merge_dist;
        }
      }
      const uint64_t mask = __ballot(pass);
      const bool stop = zs && __ballot(inside) == 0ull;   // (sorted: all later records lie above)
      const int np = __popcll(mask);
      if (np > 0) {
        if (cnt + np > 64) flush();
        if (pass) {
          const int slot = cnt + __popcll(mask & lanemask_lt());
          s_cand[wv][slot] = k;
          s_dir[wv][slot] = (uint8_t)dir;
        }
        cnt += np;
      }
      if (stop) break;
    }
  };
  for (int dir = 0; dir < ndir; ++dir) {
    // 0, 1: the preceding and following wedge of the side; 2: the own sector
    const int wa = dir == 0 ? (wb + w.NW - 1) % w.NW : dir == 1 ? (wb + 1) % w.NW : wb;
    const uint32_t s0 = (uint32_t)(side0 + wa) * (uint32_t)w.nsl;
    const float sa = dir == 2 ? 0.0f : turn_sign(wa, wb, w.NW) * w.sa, ca = dir == 2 ? 1.0f : w.ca;
    if (!w.prune) {
      for (int sl = 0; sl < w.nsl; ++sl) scan(dir, ca, sa, s0 + (uint32_t)sl);
      continue;
    }
    // hit ends two or more slices apart are more than a slice length apart
    // in the frame's z, outside the window: only the neighbouring slices
    // (and, across wedges, the own one) are scanned
    for (int ds = -1; ds <= 1; ++ds) {
      const int sl = slb + ds;
      if ((dir == 2 && ds == 0) || sl < 0 || sl >= w.nsl) continue;
      scan(dir, ca, sa, s0 + (uint32_t)sl);
    }
  }
  if (cnt > 0) flush();
  best = wave_min_u64(best);
  if (lane == 0) w.best_in[b] = best;
}

__global__ __launch_bounds__(TB) void k_mrg_links(MergeWs w) {
  const int64_t a = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (a >= w.T) return;
  const unsigned long long bo = w.best_out[a];
  int32_t l = -1;
  if (bo != kNone) {
    const uint32_t b = (uint32_t)(bo & 0xFFFFFFFFull);
    const unsigned long long bi = w.best_in[b];
    if (bi != kNone && (uint32_t)(bi & 0xFFFFFFFFull) == (uint32_t)a) {
      l = (int32_t)b;
      w.inner[b] = (int32_t)a;
    }
  }
  w.link[a] = l;
  if (w.o_link) w.o_link[a] = l;
}

// Chain of head i (a segment without an inner partner): every segment's
// head, place and preceding hits; the head's counts (its segments as they
// are, until the refit succeeds); chains of two or more listed for the refit.
__global__ __launch_bounds__(TB) void k_mrg_chains(MergeWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i >= w.T) return;
  if (w.inner[i] >= 0 || w.err[0] != 0u) { w.emit[i] = 0u; w.hemit[i] = 0u; return; }
  uint32_t n = 0, hits = 0;
  // (rows increase strictly along a chain, so it has at most R segments)
  for (int32_t c = (int32_t)i; c >= 0 && n <= (uint32_t)w.R; c = w.link[c]) {
    w.head[c] = (int32_t)i;
    w.tpos[c] = n;
    w.hpos[c] = hits;
    ++n;
    hits += (uint32_t)(w.hit_off[c + 1] - w.hit_off[c]);
  }
  w.nseg[i] = n;
  w.emit[i] = n;
  w.hemit[i] = hits;
  if (n > 1) w.rlist[atomicAdd(&w.err[3], 1u)] = (uint32_t)i;
}

// The total of a scanned count array (v[T]) into its result word.
__global__ void k_mrg_total(const uint32_t* __restrict__ v, int64_t T, uint32_t* __restrict__ tot) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *tot = v[T];
}

// One wave per segment: its hit ids copied to their place in the output
// (the chain's hits, innermost segment first).
__global__ __launch_bounds__(TB) void k_mrg_hits(MergeWs w) {
  const int64_t c = (int64_t)blockIdx.x * (TB / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= w.T || w.err[0] != 0u) return;
  const uint32_t h = w.hemit[w.head[c]] + w.hpos[c];
  const int32_t b0 = w.hit_off[c], nh = w.hit_off[c + 1] - b0;
  for (int32_t k = lane; k < nh; k += 64) w.o_hit_id[h + (uint32_t)k] = w.hit_id[b0 + k];
}

// Merged refit of a listed chain, from its outermost hit inward over the
// chain's hit ids as written to the output (innermost segment first, so read
// backwards): ids are loaded eight steps ahead, coordinates four steps
// ahead, a ring of four slots per kind (past the chain's first hit the
// loads repeat it and are never used).  At each segment boundary the state
// is rotated into the next inner segment's frame; that segment's sector and
// hit count, and the index of the one inside it, are loaded a segment ahead,
// so a lane crossing a boundary does not stop its wave for dependent loads.
__global__ __launch_bounds__(64) void k_mrg_refit(MergeWs w) {
  const int64_t q = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (q >= (int64_t)w.err[3]) return;
  const int32_t i = (int32_t)w.rlist[q];
  const uint32_t* ids = w.o_hit_id + w.hemit[i];
  int32_t c = i;
  while (w.link[c] >= 0) c = w.link[c];
  // the chain's hits at positions 0 .. n-1 (inner to outer); the outermost
  // segment c covers the last nc of them
  const int32_t n = (int32_t)(w.hemit[i + 1] - w.hemit[i]);
  int32_t seg_lo = n - (w.hit_off[c + 1] - w.hit_off[c]);
  // the current segment's sector; the next inner segment (na), its sector and
  // hit count, and the segment inside it (nna); past the chain's innermost
  // segment the loads repeat the current one and are never used
  int sec_c = w.sector[c];
  int32_t na = w.inner[c];
  int32_t sa = na >= 0 ? na : c;
  int sec_a = w.sector[sa];
  int32_t len_a = w.hit_off[sa + 1] - w.hit_off[sa];
  int32_t nna = w.inner[sa];
  const Model& m = w.m;
  auto X = [&](uint32_t id) { return make_float4(w.cx[id], w.cy[id], w.cz[id], 0.0f); };
  const float4 r0 = X(ids[n - 1]), r2 = X(ids[n - 3]);
  float p[5], C[15], s, t;
  chord_dir(r2.x, r2.y, r2.z, r0.x, r0.y, r0.z, s, t);
  p[0] = r0.y; p[1] = r0.z; p[2] = s; p[3] = t; p[4] = w.p[c * 5 + 4];
  init_cov(C, m.vy, m.vz);
  float chi2 = 0.0f, xc = r0.x;
  bool ok = fabsf(s) < m.sin_max;
  int nupd = 0;
  auto at = [&](int32_t k) { return k >= 0 ? k : 0; };
  // ring slots: coordinates of hits k, k-1, k-2, k-3; ids of hits k-4 .. k-7
  int32_t k = n - 2;
  float4 c0 = X(ids[at(k)]), c1 = X(ids[at(k - 1)]), c2 = X(ids[at(k - 2)]), c3 = X(ids[at(k - 3)]);
  uint32_t j0 = ids[at(k - 4)], j1 = ids[at(k - 5)], j2 = ids[at(k - 6)], j3 = ids[at(k - 7)];
  auto step = [&](float4& cs, uint32_t& js) {
    if (ok && k >= 0) {
      if (k < seg_lo) {
        // entering the next inner segment (its frame, unless it lies in the
        // same sector: a neighbouring slice of a time frame)
        const int wc = sec_c % w.NW, wa = sec_a % w.NW;
        if (sec_a != sec_c && !rotate_state(xc, p, C, w.ca, turn_sign(wc, wa, w.NW) * w.sa, m))
          ok = false;
        c = na;
        sec_c = sec_a;
        seg_lo -= len_a;
        na = nna;
        sa = na >= 0 ? na : c;
        sec_a = w.sector[sa];
        len_a = w.hit_off[sa + 1] - w.hit_off[sa];
        nna = w.inner[sa];
      }
      if (ok && !transport(p, C, xc, cs.x, m)) ok = false;
      if (ok) {
        if (nupd < TPCCA_GRAD_C2_UPDATES) update_c2(p, C, cs.y, cs.z, m, chi2);
        else update(p, C, cs.y, cs.z, m, chi2);
        ++nupd;
        xc = cs.x;
      }
    }
    cs = X(js);
    js = ids[at(k - 8)];
    --k;
  };
  while (ok && k >= 0) {
    step(c0, j0);
    step(c1, j1);
    step(c2, j2);
    step(c3, j3);
  }
  if (ok) {
    w.emit[i] = 1u;
    float* r = w.rec + (int64_t)i * 24;
    r[0] = xc;
#pragma unroll
    for (int kk = 0; kk < 5; ++kk) r[1 + kk] = p[kk];
#pragma unroll
    for (int kk = 0; kk < 15; ++kk) r[6 + kk] = C[kk];
    r[21] = chi2;
  }
}

// Lane per segment: the track records -- the segment's own, or, for the
// head of a refitted chain, the merged track; the output's final offset.
__global__ __launch_bounds__(TB) void k_mrg_tracks(MergeWs w) {
  const int64_t c = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (c == 0) w.o_hit_off[w.emit[w.T]] = (int32_t)w.hemit[w.T];
  if (c >= w.T || w.err[0] != 0u) return;
  const int32_t i = w.head[c];
  const uint32_t t0 = w.emit[i], ne = w.emit[i + 1] - t0;
  const uint32_t h = w.hemit[i] + w.hpos[c];
  if (ne == 1u && w.nseg[i] > 1u) {
    if (c != i) return;
    const float* r = w.rec + (int64_t)i * 24;
    w.o_sector[t0] = w.sector[i];
    w.o_x_ref[t0] = r[0];
#pragma unroll
    for (int k = 0; k < 5; ++k) w.o_p[t0 * 5 + k] = r[1 + k];
#pragma unroll
    for (int k = 0; k < 15; ++k) w.o_cov[t0 * 15 + k] = r[6 + k];
    w.o_chi2[t0] = r[21];
    w.o_ndf[t0] = 2 * (int32_t)(w.hemit[i + 1] - w.hemit[i]) - 5;
    w.o_hit_off[t0] = (int32_t)h;
    return;
  }
  const uint32_t t = t0 + w.tpos[c];
  w.o_sector[t] = w.sector[c];
  w.o_x_ref[t] = w.x_ref[c];
#pragma unroll
  for (int k = 0; k < 5; ++k) w.o_p[t * 5 + k] = w.p[c * 5 + k];
#pragma unroll
  for (int k = 0; k < 15; ++k) w.o_cov[t * 15 + k] = w.cov[c * 15 + k];
  w.o_chi2[t] = w.chi2[c];
  w.o_ndf[t] = w.ndf[c];
  w.o_hit_off[t] = (int32_t)h;
}

}  // namespace

hipError_t run_merge(const MergeWs& w, hipStream_t st) {
  const void* need[] = {w.sector, w.x_ref, w.p, w.cov, w.chi2, w.ndf, w.hit_off, w.hit_id, w.cx, w.cy, w.cz,
                        w.crow, w.ex, w.first, w.last, w.flags, w.sec_cnt, w.sec_cur, w.sec_list, w.srec, w.zrec, w.zlist, w.zsorted,
                        w.best_in, w.best_out, w.link, w.inner, w.emit, w.hemit, w.head, w.tpos, w.hpos, w.nseg,
                        w.rlist, w.rec, w.err, w.scan_part, w.o_sector, w.o_x_ref, w.o_p, w.o_cov, w.o_chi2, w.o_ndf,
                        w.o_hit_off, w.o_hit_id};
  for (const void* q : need)
    if (!q) return hipErrorInvalidValue;
  if (w.S > kMaxSectors || w.S > kSecBins || w.nsl < 1 || w.T >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const int64_t nbin = (int64_t)w.S * w.nsl;
  const int64_t n0 = std::max<int64_t>(std::max<int64_t>(w.T, nbin), 4);
  k_mrg_init<<<(unsigned)((n0 + TB - 1) / TB), TB, 0, st>>>(w);
  const unsigned g = (unsigned)std::max<int64_t>((w.T + TB - 1) / TB, 1);
  const unsigned gw = (unsigned)std::max<int64_t>((w.T + TB / 64 - 1) / (TB / 64), 1);
  if (w.T > 0) {
    k_mrg_ends<<<g, TB, 0, st>>>(w);
    const hipError_t es = scan_exclusive_u32(w.sec_cnt, w.sec_cnt, nbin, w.scan_part, st);
    if (es != hipSuccess) return es;
    k_mrg_secfill<<<g, TB, 0, st>>>(w);
    k_mrg_zsort<<<(unsigned)nbin, TBZ, 0, st>>>(w);
    k_mrg_pairs<<<gw, TB, 0, st>>>(w);
    k_mrg_links<<<g, TB, 0, st>>>(w);
    k_mrg_chains<<<g, TB, 0, st>>>(w);
  }
  // hit offsets of the chains (they do not depend on the refit), the hits,
  // the refit (one lane per listed chain: at most T / 2 of them), then the
  // track offsets and records
  hipError_t e = scan_exclusive_u32(w.hemit, w.hemit, w.T, w.scan_part, st);
  if (e != hipSuccess) return e;
  k_mrg_total<<<1, 64, 0, st>>>(w.hemit, w.T, w.err + 2);
  if (w.T > 0) {
    k_mrg_hits<<<gw, TB, 0, st>>>(w);
    k_mrg_refit<<<(unsigned)((w.T / 2 + 64) / 64), 64, 0, st>>>(w);
  }
  e = scan_exclusive_u32(w.emit, w.emit, w.T, w.scan_part, st);
  if (e != hipSuccess) return e;
  k_mrg_total<<<1, 64, 0, st>>>(w.emit, w.T, w.err + 1);
  k_mrg_tracks<<<g, TB, 0, st>>>(w);
  return hipGetLastError();
}

}  // namespace tpcca
