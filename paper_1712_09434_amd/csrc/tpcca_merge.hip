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
// state rotated into the next inner segment's frame at each boundary.
//
// Kernels, one lane per segment unless noted: exit states and hit ends,
// segments listed by sector, candidate search (each outer segment scans the
// two neighbouring sectors' lists; keys (chi2 bits, index) taken by atomic
// minimum, so the result does not depend on the scan order), mutual links,
// chain walk and merged refit (lane per chain head), output offsets (one
// workgroup), output writing (lane per chain head).
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

// Turn (sign of the adjacent-wedge angle) from the frame of wedge wa to that
// of wedge wb: +1 if wb follows wa counter-clockwise.
__device__ __forceinline__ float turn_sign(int wa, int wb, int NW) { return wb == (wa + 1) % NW ? 1.0f : -1.0f; }

__global__ __launch_bounds__(TB) void k_mrg_exit(MergeWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i < w.S) w.sec_cnt[i] = 0u;
  if (i < w.T) {
    w.best_in[i] = kNone;
    w.best_out[i] = kNone;
    w.link[i] = -1;
    w.inner[i] = -1;
    w.flags[i] = 0u;
  }
}

__global__ __launch_bounds__(TB) void k_mrg_ends(MergeWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i >= w.T) return;
  const int32_t b0 = w.hit_off[i], b1 = w.hit_off[i + 1];
  const int s = w.sector[i];
  if (b0 < 0 || b1 - b0 < 3 || b1 - b0 > w.R || (int64_t)b1 > w.H || s >= w.S) { atomicOr(&w.err[0], 1u); return; }
  const uint32_t hf = w.hit_id[b0], hl = w.hit_id[b1 - 1];
  if ((int64_t)hf >= w.NC || (int64_t)hl >= w.NC) { atomicOr(&w.err[0], 2u); return; }
  w.flags[i] = 2u;                        // a well-formed segment
  w.first[i] = make_float4(w.cx[hf], w.cy[hf], w.cz[hf], __int_as_float((int)w.crow[hf]));
  w.last[i] = make_float4(w.cx[hl], w.cy[hl], w.cz[hl], __int_as_float((int)w.crow[hl]));
  atomicAdd(&w.sec_cnt[s], 1u);
  float p[5], C[15];
#pragma unroll
  for (int k = 0; k < 5; ++k) p[k] = w.p[i * 5 + k];
#pragma unroll
  for (int k = 0; k < 15; ++k) C[k] = w.cov[i * 15 + k];
  const float xo = w.cx[hl];
  if (transport(p, C, w.x_ref[i], xo, w.m)) {
    float* e = w.ex + i * 24;
    e[0] = xo;
#pragma unroll
    for (int k = 0; k < 5; ++k) e[1 + k] = p[k];
#pragma unroll
    for (int k = 0; k < 15; ++k) e[6 + k] = C[k];
    w.flags[i] = 3u;                      // ... with an exit state
  }
}

// Segments listed by sector: offsets (one thread; at most 254 sectors), then
// every segment takes a slot of its sector.
__global__ void k_mrg_secscan(MergeWs w) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint32_t acc = 0;
  for (int s = 0; s < w.S; ++s) {
    const uint32_t n = w.sec_cnt[s];
    w.sec_cnt[s] = acc;
    w.sec_cur[s] = acc;
    acc += n;
  }
  w.sec_cnt[w.S] = acc;
}

__global__ __launch_bounds__(TB) void k_mrg_secfill(MergeWs w) {
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (i >= w.T) return;
  const int s = w.sector[i];
  if (s >= w.S) return;
  w.sec_list[atomicAdd(&w.sec_cur[s], 1u)] = (uint32_t)i;
}

// Candidate search of outer segment b over the segments of the two
// neighbouring wedges of its side.
__global__ __launch_bounds__(TB) void k_mrg_pairs(MergeWs w) {
  const int64_t b = (int64_t)blockIdx.x * TB + threadIdx.x;
  if (b >= w.T || w.err[0] != 0u || !(w.flags[b] & 2u)) return;
  const int sb = w.sector[b];
  if (w.NW < 3) return;
  const int wb = sb % w.NW, side0 = sb - wb;
  const float4 hb = w.first[b];
  const int rlo_b = __float_as_int(hb.w);
  const float xb = w.x_ref[b];
  float pb[5], Cb[15];
#pragma unroll
  for (int k = 0; k < 5; ++k) pb[k] = w.p[b * 5 + k];
#pragma unroll
  for (int k = 0; k < 15; ++k) Cb[k] = w.cov[b * 15 + k];
  unsigned long long best = kNone;
  for (int dir = 0; dir < 2; ++dir) {
    const int wa = dir == 0 ? (wb + w.NW - 1) % w.NW : (wb + 1) % w.NW;
    const int sa_ = side0 + wa;
    const float sgn = turn_sign(wa, wb, w.NW);
    const float sa = sgn * w.sa, ca = w.ca;
    const uint32_t k0 = w.sec_cnt[sa_], k1 = w.sec_cnt[sa_ + 1];
    for (uint32_t k = k0; k < k1; ++k) {
      const uint32_t a = w.sec_list[k];
      if (!(w.flags[a] & 1u)) continue;
      const float4 ha = w.last[a];
      if (!(__float_as_int(ha.w) < rlo_b)) continue;
      const float xa = ha.x * ca + ha.y * sa, ya = -(ha.x * sa) + ha.y * ca;
      const float dX = xa - hb.x, dY = ya - hb.y;
      const float dr = sqrtf(dX * dX + dY * dY);
      if (!(dr <= w.merge_dist && fabsf(ha.z - hb.z) <= w.merge_dist)) continue;
      const float* e = w.ex + (int64_t)a * 24;
      float x = e[0], q[5], Q[15];
#pragma unroll
      for (int j = 0; j < 5; ++j) q[j] = e[1 + j];
#pragma unroll
      for (int j = 0; j < 15; ++j) Q[j] = e[6 + j];
      if (!rotate_state(x, q, Q, ca, sa, w.m)) continue;
      if (!transport(q, Q, x, xb, w.m)) continue;
      float d[5], M[15], chi;
#pragma unroll
      for (int j = 0; j < 5; ++j) d[j] = q[j] - pb[j];
#pragma unroll
      for (int j = 0; j < 15; ++j) M[j] = Q[j] + Cb[j];
      if (!match_chi2(d, M, chi) || !(chi <= w.chi2_merge)) continue;
      const unsigned long long cb = (unsigned long long)__float_as_uint(chi) << 32;
      best = min(best, cb | a);
      atomicMin(&w.best_out[a], cb | (unsigned long long)b);
    }
  }
  w.best_in[b] = best;
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

// Chain of head i (a segment without an inner partner): its output tracks
// and hits, and for a chain of two or more segments the merged refit.
__global__ __launch_bounds__(64) void k_mrg_chains(MergeWs w) {
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (i >= w.T) return;
  if (w.inner[i] >= 0 || w.err[0] != 0u) { w.emit[i] = 0u; w.hemit[i] = 0u; return; }
  int n = 1;
  int32_t c = (int32_t)i;
  uint32_t hits = (uint32_t)(w.hit_off[i + 1] - w.hit_off[i]);
  while (w.link[c] >= 0 && n <= w.S) {
    c = w.link[c];
    ++n;
    hits += (uint32_t)(w.hit_off[c + 1] - w.hit_off[c]);
  }
  w.hemit[i] = hits;
  if (n == 1) { w.emit[i] = 1u; return; }
  // merged refit, from the outermost hit of the outermost segment c inward
  const Model& m = w.m;
  int32_t b0 = w.hit_off[c], hi = w.hit_off[c + 1] - 1;
  const uint32_t h0 = w.hit_id[hi], h2 = w.hit_id[hi - 2];
  float p[5], C[15], s, t;
  chord_dir(w.cx[h2], w.cy[h2], w.cz[h2], w.cx[h0], w.cy[h0], w.cz[h0], s, t);
  p[0] = w.cy[h0]; p[1] = w.cz[h0]; p[2] = s; p[3] = t; p[4] = w.p[c * 5 + 4];
  init_cov(C, m.vy, m.vz);
  float chi2 = 0.0f, xc = w.cx[h0];
  bool ok = fabsf(s) < m.sin_max;
  int nupd = 0;
  --hi;
  while (ok) {
    for (; hi >= b0; --hi) {
      const uint32_t h = w.hit_id[hi];
      const float hx = w.cx[h];
      if (!transport(p, C, xc, hx, m)) { ok = false; break; }
      if (nupd < TPCCA_GRAD_C2_UPDATES) update_c2(p, C, w.cy[h], w.cz[h], m, chi2);
      else update(p, C, w.cy[h], w.cz[h], m, chi2);
      ++nupd;
      xc = hx;
    }
    if (!ok || c == (int32_t)i) break;
    const int32_t a = w.inner[c];
    const int wc = w.sector[c] % w.NW, wa = w.sector[a] % w.NW;
    if (!rotate_state(xc, p, C, w.ca, turn_sign(wc, wa, w.NW) * w.sa, m)) { ok = false; break; }
    c = a;
    b0 = w.hit_off[c];
    hi = w.hit_off[c + 1] - 1;
  }
  w.emit[i] = ok ? 1u : (uint32_t)n;
  if (ok) {
    float* r = w.rec + i * 24;
    r[0] = xc;
#pragma unroll
    for (int k = 0; k < 5; ++k) r[1 + k] = p[k];
#pragma unroll
    for (int k = 0; k < 15; ++k) r[6 + k] = C[k];
    r[21] = chi2;
  }
}

// Exclusive scans of emit and hemit over the segments (one workgroup of
// 1024 threads, each a contiguous block); totals at [T]; the output's final
// hit offset.
constexpr int kScanT = 1024;
__global__ __launch_bounds__(kScanT) void k_mrg_scan(MergeWs w) {
  __shared__ uint32_t se[kScanT], sh[kScanT];
  const int64_t per = (w.T + kScanT - 1) / kScanT;
  const int64_t i0 = (int64_t)threadIdx.x * per, i1 = min<int64_t>(i0 + per, w.T);
  uint32_t ae = 0, ah = 0;
  for (int64_t i = i0; i < i1; ++i) { ae += w.emit[i]; ah += w.hemit[i]; }
  se[threadIdx.x] = ae;
  sh[threadIdx.x] = ah;
  __syncthreads();
  for (int d = 1; d < kScanT; d <<= 1) {
    const uint32_t ve = threadIdx.x >= (unsigned)d ? se[threadIdx.x - d] : 0u;
    const uint32_t vh = threadIdx.x >= (unsigned)d ? sh[threadIdx.x - d] : 0u;
    __syncthreads();
    se[threadIdx.x] += ve;
    sh[threadIdx.x] += vh;
    __syncthreads();
  }
  uint32_t oe = threadIdx.x ? se[threadIdx.x - 1] : 0u, oh = threadIdx.x ? sh[threadIdx.x - 1] : 0u;
  for (int64_t i = i0; i < i1; ++i) {
    const uint32_t e = w.emit[i], h = w.hemit[i];
    w.emit[i] = oe;
    w.hemit[i] = oh;
    oe += e;
    oh += h;
  }
  if (threadIdx.x == kScanT - 1) {
    w.emit[w.T] = se[kScanT - 1];
    w.hemit[w.T] = sh[kScanT - 1];
    w.err[1] = se[kScanT - 1];
    w.err[2] = sh[kScanT - 1];
    w.o_hit_off[se[kScanT - 1]] = (int32_t)sh[kScanT - 1];
  }
}

__device__ void copy_hits(const MergeWs& w, int32_t c, uint32_t h) {
  const int32_t b0 = w.hit_off[c], b1 = w.hit_off[c + 1];
  for (int32_t k = b0; k < b1; ++k) w.o_hit_id[h + (uint32_t)(k - b0)] = w.hit_id[k];
}

__global__ __launch_bounds__(64) void k_mrg_write(MergeWs w) {
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (i >= w.T || w.inner[i] >= 0 || w.err[0] != 0u) return;
  uint32_t t = w.emit[i], h = w.hemit[i];
  const uint32_t ne = w.emit[i + 1] - t;
  if (ne == 1u && w.link[i] >= 0) {
    // merged chain
    const float* r = w.rec + i * 24;
    w.o_sector[t] = w.sector[i];
    w.o_x_ref[t] = r[0];
#pragma unroll
    for (int k = 0; k < 5; ++k) w.o_p[t * 5 + k] = r[1 + k];
#pragma unroll
    for (int k = 0; k < 15; ++k) w.o_cov[t * 15 + k] = r[6 + k];
    w.o_chi2[t] = r[21];
    w.o_ndf[t] = 2 * (int32_t)(w.hemit[i + 1] - h) - 5;
    w.o_hit_off[t] = (int32_t)h;
    for (int32_t c = (int32_t)i; c >= 0; c = w.link[c]) {
      copy_hits(w, c, h);
      h += (uint32_t)(w.hit_off[c + 1] - w.hit_off[c]);
    }
    return;
  }
  // single segment, or a chain whose refit failed: its segments as they are
  for (int32_t c = (int32_t)i; c >= 0; c = w.link[c]) {
    w.o_sector[t] = w.sector[c];
    w.o_x_ref[t] = w.x_ref[c];
#pragma unroll
    for (int k = 0; k < 5; ++k) w.o_p[t * 5 + k] = w.p[c * 5 + k];
#pragma unroll
    for (int k = 0; k < 15; ++k) w.o_cov[t * 15 + k] = w.cov[c * 15 + k];
    w.o_chi2[t] = w.chi2[c];
    w.o_ndf[t] = w.ndf[c];
    w.o_hit_off[t] = (int32_t)h;
    copy_hits(w, c, h);
    h += (uint32_t)(w.hit_off[c + 1] - w.hit_off[c]);
    ++t;
  }
}

__global__ void k_mrg_zero(MergeWs w) {
  if (threadIdx.x < 4 && blockIdx.x == 0) w.err[threadIdx.x] = 0u;
}

}  // namespace

hipError_t run_merge(const MergeWs& w, hipStream_t st) {
  const void* need[] = {w.sector, w.x_ref, w.p, w.cov, w.chi2, w.ndf, w.hit_off, w.hit_id, w.cx, w.cy, w.cz,
                        w.crow, w.ex, w.first, w.last, w.flags, w.sec_cnt, w.sec_cur, w.sec_list, w.best_in,
                        w.best_out, w.link, w.inner, w.emit, w.hemit, w.rec, w.err, w.o_sector, w.o_x_ref,
                        w.o_p, w.o_cov, w.o_chi2, w.o_ndf, w.o_hit_off, w.o_hit_id};
  for (const void* q : need)
    if (!q) return hipErrorInvalidValue;
  if (w.S > kMaxSectors || w.T >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  k_mrg_zero<<<1, 64, 0, st>>>(w);
  const int64_t n0 = std::max<int64_t>(w.T, w.S);
  const unsigned g0 = (unsigned)std::max<int64_t>((n0 + TB - 1) / TB, 1);
  k_mrg_exit<<<g0, TB, 0, st>>>(w);
  if (w.T > 0) {
    const unsigned g = (unsigned)((w.T + TB - 1) / TB), g64 = (unsigned)((w.T + 63) / 64);
    k_mrg_ends<<<g, TB, 0, st>>>(w);
    k_mrg_secscan<<<1, 64, 0, st>>>(w);
    k_mrg_secfill<<<g, TB, 0, st>>>(w);
    k_mrg_pairs<<<g, TB, 0, st>>>(w);
    k_mrg_links<<<g, TB, 0, st>>>(w);
    k_mrg_chains<<<g64, 64, 0, st>>>(w);
  }
  k_mrg_scan<<<1, kScanT, 0, st>>>(w);
  if (w.T > 0) k_mrg_write<<<(unsigned)((w.T + 63) / 64), 64, 0, st>>>(w);
  return hipGetLastError();
}

}  // namespace tpcca
