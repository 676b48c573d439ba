// oracle.cpp -- plain CPU oracle of the per-sector TPC track finder.
//
// TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked
// against.  It shares no code with the GPU path.  Linear scans over row
// lists, no grids, no blocking, one tracklet at a time.
//
// The paper (Sec. "Track reconstruction in the TPC") fixes the structure:
// cellular-automaton seeding of short chains of hits, then Kalman-filter
// fitting and following, sectors processed independently, one worker per
// cluster (seeding) and per track (following).  It states no constant and no
// rule beyond that; every rule below is a reading, listed in the design
// notes with its pin.  Units: cm, tesla, GeV.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fPIC -shared (no fast-math;
// FP32 expressions are evaluated exactly as written, IEEE round-to-nearest).
#include "tpcca_oracle.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <vector>

namespace {

// Longest transport (in pad rows) on the way back from the last row reached
// upward to the seed's first row.
constexpr int kBackRows = 32;

// ---------------------------------------------------------------------------
// Reverse-mode tape scalar (FP64).  Every operation records its local
// partial derivatives; backprop() accumulates adjoints in reverse order.
struct Tape {
  struct Node { int a, b; double da, db; };
  std::vector<Node> nodes;
  std::vector<double> adj;
  int add(int a, double da, int b, double db) {
    if (a < 0 && b < 0) return -1;
    nodes.push_back({a, b, da, db});
    return (int)nodes.size() - 1;
  }
  int leaf() { nodes.push_back({-1, -1, 0.0, 0.0}); return (int)nodes.size() - 1; }
  void backprop(int out) {
    adj.assign(nodes.size(), 0.0);
    if (out < 0) return;
    adj[out] = 1.0;
    for (int i = out; i >= 0; --i) {
      const Node& n = nodes[i];
      if (adj[i] == 0.0) continue;
      if (n.a >= 0) adj[n.a] += n.da * adj[i];
      if (n.b >= 0) adj[n.b] += n.db * adj[i];
    }
  }
  void clear() { nodes.clear(); adj.clear(); }
};
Tape* g_tape = nullptr;

struct Var {
  double v; int i;
  Var() : v(0.0), i(-1) {}
  Var(double x) : v(x), i(-1) {}                 // NOLINT: constants convert implicitly
  static Var leaf(double x) { Var r(x); r.i = g_tape->leaf(); return r; }
};
inline Var mk(double v, int a, double da, int b, double db) {
  Var r(v); r.i = g_tape ? g_tape->add(a, da, b, db) : -1; return r;
}
inline Var operator+(Var a, Var b) { return mk(a.v + b.v, a.i, 1.0, b.i, 1.0); }
inline Var operator-(Var a, Var b) { return mk(a.v - b.v, a.i, 1.0, b.i, -1.0); }
inline Var operator-(Var a) { return mk(-a.v, a.i, -1.0, -1, 0.0); }
inline Var operator*(Var a, Var b) { return mk(a.v * b.v, a.i, b.v, b.i, a.v); }
inline Var operator/(Var a, Var b) { double q = a.v / b.v; return mk(q, a.i, 1.0 / b.v, b.i, -q / b.v); }
inline bool operator<(Var a, Var b) { return a.v < b.v; }
inline bool operator<=(Var a, Var b) { return a.v <= b.v; }
inline bool operator>(Var a, Var b) { return a.v > b.v; }
inline bool operator==(Var a, Var b) { return a.v == b.v; }
inline bool operator!=(Var a, Var b) { return a.v != b.v; }

inline float Sqrt(float x) { return std::sqrt(x); }
inline double Sqrt(double x) { return std::sqrt(x); }
inline Var Sqrt(Var x) { double s = std::sqrt(x.v); return mk(s, x.i, 0.5 / s, -1, 0.0); }
inline float Abs(float x) { return std::fabs(x); }
inline double Abs(double x) { return std::fabs(x); }
inline Var Abs(Var x) { return x.v < 0 ? -x : x; }
// Fused multiply-add a*b + c with one rounding (the FP32 parity mode takes it
// at exactly the places the GPU code does); on the tape an ordinary product
// and sum.
inline float Fma(float a, float b, float c) { return std::fma(a, b, c); }
inline double Fma(double a, double b, double c) { return std::fma(a, b, c); }
inline Var Fma(Var a, Var b, Var c) { return a * b + c; }
inline double val(float x) { return x; }
inline double val(double x) { return x; }
inline double val(Var x) { return x.v; }

// ---------------------------------------------------------------------------
// Packed symmetric 5x5 covariance, upper triangle row by row.
inline int ix(int i, int j) {
  if (i > j) std::swap(i, j);
  static const int base[5] = {0, 5, 9, 12, 14};
  return base[i] + (j - i);
}

template <class R> struct Model {
  R kfac;        // curvature per unit q/pT: -c * Bz
  R sin_max;
  R vy, vz;      // measurement variances
};

template <class R> Model<R> make_model(const orc_geometry& g, const orc_params& P) {
  Model<R> m;
  m.kfac = -R((double)2.99792458e-3) * R(g.bz);
  m.sin_max = R(P.sin_max);
  m.vy = R(P.sigma_y) * R(P.sigma_y);
  m.vz = R(P.sigma_z) * R(P.sigma_z);
  return m;
}

// Transport of state p = (y, z, s = sin phi, t = tan lambda, k = q/pT) from
// the plane x0 to the plane x1 along a helix in a uniform field.  With the
// signed curvature kap = kfac * k: s1 = s0 + kap*dx; the transverse chord
// rises by dy = dx * (s0 + s1)/(c0 + c1) (tangent of the mean direction,
// exact for a circle); the transverse arc is d * asin(u)/u with d the chord
// length carrying the sign of dx (inward steps have negative path length)
// and u = kap*d/2, asin(u)/u taken as its Maclaurin series to u^8; z
// advances by t times the arc.  F is the exact Jacobian of these formulas;
// the covariance becomes F C F^T (no process noise: no material).
template <class R>
bool transport(R p[5], R C[15], R x0, R x1, const Model<R>& m, R* Fout = nullptr) {
  R dx = x1 - x0;
  if (dx == R(0.0)) {
    if (Fout) { for (int i = 0; i < 25; ++i) Fout[i] = R(0.0); for (int i = 0; i < 5; ++i) Fout[i * 6] = R(1.0); }
    return true;
  }
  const R A1 = R(1.0) / R(6.0), A2 = R(3.0) / R(40.0), A3 = R(5.0) / R(112.0), A4 = R(35.0) / R(1152.0);
  const R B1 = R(1.0) / R(3.0), B2 = R(3.0) / R(10.0), B3 = R(15.0) / R(56.0), B4 = R(35.0) / R(144.0);
  R kap = m.kfac * p[4];
  R s0 = p[2];
  R f = m.kfac * dx;                      // d s1 / d k
  R s1 = Fma(kap, dx, s0);
  if (!(Abs(s1) < m.sin_max)) return false;
  R c0 = Sqrt(Fma(-s0, s0, R(1.0)));
  R c1 = Sqrt(Fma(-s1, s1, R(1.0)));
  R ss = s0 + s1;
  R cc = c0 + c1;
  R icc = R(1.0) / cc;                    // shared denominator: one division, then products
  R tn = ss * icc;
  R dy = dx * tn;
  R d = Sqrt(Fma(dx, dx, dy * dy));       // chord length, signed like dx
  if (dx < R(0.0)) d = -d;
  R u = (kap * d) * R(0.5);
  R u2 = u * u;
  R g = Fma(u2, Fma(u2, Fma(u2, Fma(u2, A4, A3), A2), A1), R(1.0));
  R gp = u * Fma(u2, Fma(u2, Fma(u2, B4, B3), B2), B1);   // d(asin(u)/u)/du
  R l = d * g;
  R i01 = R(1.0) / (c0 * c1);              // the two tangents share one division
  R t0 = (s0 * c1) * i01;
  R t1 = (s1 * c0) * i01;
  R dtn_ds = Fma(tn, t0 + t1, R(2.0)) * icc;
  R dtn_dk = (f * Fma(tn, t1, R(1.0))) * icc;
  R a = dx * dtn_ds;                       // d dy / d s0
  R b = dx * dtn_dk;                       // d dy / d k
  R id = R(1.0) / d;
  R dd_ds = (dy * a) * id;
  R dd_dk = (dy * b) * id;
  R du_ds = (kap * dd_ds) * R(0.5);
  R du_dk = Fma(m.kfac, d, kap * dd_dk) * R(0.5);
  R dl_ds = Fma(dd_ds, g, (d * gp) * du_ds);
  R dl_dk = Fma(dd_dk, g, (d * gp) * du_dk);
  R t = p[3];
  R c = t * dl_ds;                         // d z1 / d s0
  R e = t * dl_dk;                         // d z1 / d k
  p[0] = p[0] + dy;
  p[1] = Fma(t, l, p[1]);
  p[2] = s1;
  // F = [[1,0,a,0,b],[0,1,c,l,e],[0,0,1,0,f],[0,0,0,1,0],[0,0,0,0,1]]
  R C00 = C[0], C01 = C[1], C02 = C[2], C03 = C[3], C04 = C[4];
  R C11 = C[5], C12 = C[6], C13 = C[7], C14 = C[8];
  R C22 = C[9], C23 = C[10], C24 = C[11];
  R C33 = C[12], C34 = C[13], C44 = C[14];
  // T = F C (rows 0, 1, 2; rows 3 and 4 equal those of C)
  R T00 = Fma(b, C04, Fma(a, C02, C00));
  R T01 = Fma(b, C14, Fma(a, C12, C01));
  R T02 = Fma(b, C24, Fma(a, C22, C02));
  R T03 = Fma(b, C34, Fma(a, C23, C03));
  R T04 = Fma(b, C44, Fma(a, C24, C04));
  R T11 = Fma(e, C14, Fma(l, C13, Fma(c, C12, C11)));
  R T12 = Fma(e, C24, Fma(l, C23, Fma(c, C22, C12)));
  R T13 = Fma(e, C34, Fma(l, C33, Fma(c, C23, C13)));
  R T14 = Fma(e, C44, Fma(l, C34, Fma(c, C24, C14)));
  R T22 = Fma(f, C24, C22);
  R T23 = Fma(f, C34, C23);
  R T24 = Fma(f, C44, C24);
  // C' = T F^T
  C[0] = Fma(b, T04, Fma(a, T02, T00));
  C[1] = Fma(e, T04, Fma(l, T03, Fma(c, T02, T01)));
  C[2] = Fma(f, T04, T02);
  C[3] = T03;
  C[4] = T04;
  C[5] = Fma(e, T14, Fma(l, T13, Fma(c, T12, T11)));
  C[6] = Fma(f, T14, T12);
  C[7] = T13;
  C[8] = T14;
  C[9] = Fma(f, T24, T22);
  C[10] = T23;
  C[11] = T24;
  // C33, C34, C44 unchanged
  if (Fout) {
    for (int i = 0; i < 25; ++i) Fout[i] = R(0.0);
    for (int i = 0; i < 5; ++i) Fout[i * 6] = R(1.0);
    Fout[2] = a; Fout[4] = b; Fout[7] = c; Fout[8] = l; Fout[9] = e; Fout[14] = f;
  }
  return true;
}

// Kalman update with a (y, z) measurement, H = [I2 0], V = diag(vy, vz).
template <class R>
void kf_update(R p[5], R C[15], R my, R mz, R vy, R vz, R& chi2) {
  R r0 = my - p[0];
  R r1 = mz - p[1];
  R S00 = C[0] + vy;
  R S01 = C[1];
  R S11 = C[5] + vz;
  R det = Fma(S00, S11, -(S01 * S01));
  R idet = R(1.0) / det;
  R I00 = S11 * idet;
  R I01 = (-S01) * idet;
  R I11 = S00 * idet;
  R row0[5], row1[5];
  for (int j = 0; j < 5; ++j) { row0[j] = C[ix(0, j)]; row1[j] = C[ix(1, j)]; }
  R K0[5], K1[5];
  for (int i = 0; i < 5; ++i) {
    K0[i] = Fma(row1[i], I01, row0[i] * I00);
    K1[i] = Fma(row1[i], I11, row0[i] * I01);
  }
  for (int i = 0; i < 5; ++i) p[i] = p[i] + Fma(K1[i], r1, K0[i] * r0);
  for (int i = 0; i < 5; ++i)
    for (int j = i; j < 5; ++j) C[ix(i, j)] = C[ix(i, j)] - Fma(K1[i], row1[j], K0[i] * row0[j]);
  chi2 = chi2 + Fma(r1, Fma(I11, r1, I01 * r0), r0 * Fma(I01, r1, I00 * r0));
}

// The first Kalman updates of a fit, whose prior is nearly diffuse (q/pT
// variance 100): there C - K H C cancels most of the digits of C, and in
// FP32 the plain update leaves some tracks' covariance off by orders of
// magnitude.  In FP32 this update computes S, its inverse, the gain and
// C - K H C in compensated arithmetic: each value a pair hi + lo of floats
// (|lo| at most half an ulp of hi), sums by Knuth's error-free two-sum,
// products by one fused multiply-add for the rounding error, the inverse by
// one Newton step on the pair residual 1 - a q; each covariance entry is
// rounded once at the end, the state and chi2 take the rounded gain and
// inverse.  In FP64 (and on the tape) it is the plain update.
struct F2 { float hi, lo; };
inline F2 f2_two_sum(float a, float b) {
  const float s = a + b;
  const float bb = s - a;
  return F2{s, (a - (s - bb)) + (b - bb)};
}
inline F2 f2_quick(float a, float b) {           // |a| >= |b| or a == 0
  const float s = a + b;
  return F2{s, b - (s - a)};
}
inline F2 f2_add(F2 a, F2 b) {
  F2 s = f2_two_sum(a.hi, b.hi);
  const F2 t = f2_two_sum(a.lo, b.lo);
  s = f2_quick(s.hi, s.lo + t.hi);
  return f2_quick(s.hi, s.lo + t.lo);
}
inline F2 f2_neg(F2 a) { return F2{-a.hi, -a.lo}; }
inline F2 f2_mul(F2 a, F2 b) {
  const float p = a.hi * b.hi;
  const float e = std::fma(a.hi, b.hi, -p);
  return f2_quick(p, std::fma(a.hi, b.lo, std::fma(a.lo, b.hi, e)));
}
inline F2 f2_mul(F2 a, float b) {
  const float p = a.hi * b;
  const float e = std::fma(a.hi, b, -p);
  return f2_quick(p, std::fma(a.lo, b, e));
}
inline F2 f2_inv(F2 a) {
  const float q = 1.0f / a.hi;
  const F2 r = f2_add(F2{1.0f, 0.0f}, f2_neg(f2_mul(a, q)));
  return f2_quick(q, r.hi * q);
}

template <class R>
void kf_update_first(R p[5], R C[15], R my, R mz, R vy, R vz, R& chi2) {
  kf_update(p, C, my, mz, vy, vz, chi2);
}
template <>
void kf_update_first<float>(float p[5], float C[15], float my, float mz, float vy, float vz, float& chi2) {
  const float r0 = my - p[0];
  const float r1 = mz - p[1];
  const F2 S00 = f2_two_sum(C[0], vy);
  const F2 S01 = F2{C[1], 0.0f};
  const F2 S11 = f2_two_sum(C[5], vz);
  const F2 det = f2_add(f2_mul(S00, S11), f2_neg(f2_mul(S01, S01)));
  const F2 idet = f2_inv(det);
  const F2 I00 = f2_mul(S11, idet);
  const F2 I01 = f2_neg(f2_mul(S01, idet));
  const F2 I11 = f2_mul(S00, idet);
  float row0[5], row1[5];
  F2 K0[5], K1[5];
  for (int j = 0; j < 5; ++j) { row0[j] = C[ix(0, j)]; row1[j] = C[ix(1, j)]; }
  for (int i = 0; i < 5; ++i) {
    K0[i] = f2_add(f2_mul(I00, row0[i]), f2_mul(I01, row1[i]));
    K1[i] = f2_add(f2_mul(I01, row0[i]), f2_mul(I11, row1[i]));
  }
  for (int i = 0; i < 5; ++i) p[i] = p[i] + std::fma(K1[i].hi, r1, K0[i].hi * r0);
  for (int i = 0; i < 5; ++i)
    for (int j = i; j < 5; ++j) {
      const F2 kr = f2_add(f2_mul(K0[i], row0[j]), f2_mul(K1[i], row1[j]));
      const F2 cn = f2_add(F2{C[ix(i, j)], 0.0f}, f2_neg(kr));
      C[ix(i, j)] = cn.hi + cn.lo;
    }
  chi2 = chi2 + std::fma(r1, std::fma(I11.hi, r1, I01.hi * r0), r0 * std::fma(I01.hi, r1, I00.hi * r0));
}
// Updates 1 .. kFirstUpdates of a fit take kf_update_first.
constexpr int kFirstUpdates = 3;

// Kalman update with a scalar measurement of state component q.
template <class R>
void kf_update1(R p[5], R C[15], int q, R m, R v, R& chi2) {
  R S = C[ix(q, q)] + v;
  R rowq[5];
  for (int j = 0; j < 5; ++j) rowq[j] = C[ix(q, j)];
  R r = m - p[q];
  R K[5];
  for (int i = 0; i < 5; ++i) K[i] = rowq[i] / S;
  for (int i = 0; i < 5; ++i) p[i] = p[i] + K[i] * r;
  for (int i = 0; i < 5; ++i)
    for (int j = i; j < 5; ++j) C[ix(i, j)] = C[ix(i, j)] - K[i] * rowq[j];
  chi2 = chi2 + (r * r) / S;
}

template <class R> void init_cov(R C[15], const orc_params& P) {
  for (int i = 0; i < 15; ++i) C[i] = R(0.0);
  C[0] = R(P.sigma_y) * R(P.sigma_y);
  C[5] = R(P.sigma_z) * R(P.sigma_z);
  C[9] = R(0.25);
  C[12] = R(0.25);
  C[14] = R(100.0);
}

// Direction from the chord between an inner hit (xi,yi,zi) and an outer hit
// (xo,yo,zo): s = dy/rho, t = dz/rho with rho the transverse chord length.
template <class R>
void chord_dir(R xi, R yi, R zi, R xo, R yo, R zo, R& s, R& t) {
  R dX = xo - xi, dY = yo - yi, dZ = zo - zi;
  R rho = Sqrt(Fma(dX, dX, dY * dY));
  R irho = R(1.0) / rho;
  s = dY * irho;
  t = dZ * irho;
}

// Final fit of an ordered hit list (outermost first): state initialised at
// the outermost hit, direction from the chord to the hit two positions
// inward, q/pT from the prior k0; then transport + update hit by hit.
template <class R>
bool fit_hits(const Model<R>& m, const orc_params& P, int n, const R* x, const R* y, const R* z,
              R k0, R p[5], R C[15], R& chi2, R& xcur) {
  if (n < 3) return false;
  R s, t;
  chord_dir(x[2], y[2], z[2], x[0], y[0], z[0], s, t);
  p[0] = y[0]; p[1] = z[0]; p[2] = s; p[3] = t; p[4] = k0;
  init_cov(C, P);
  chi2 = R(0.0);
  if (!(Abs(s) < m.sin_max)) return false;
  xcur = x[0];
  for (int h = 1; h < n; ++h) {
    if (!transport(p, C, xcur, x[h], m)) return false;
    if (h <= kFirstUpdates) kf_update_first(p, C, y[h], z[h], m.vy, m.vz, chi2);
    else kf_update(p, C, y[h], z[h], m.vy, m.vz, chi2);
    xcur = x[h];
  }
  return true;
}

// ---------------------------------------------------------------------------
// The per-sector pipeline.
template <class R> struct Pipeline {
  const orc_geometry& g;
  const orc_params& P;
  Model<R> m;
  int64_t n;
  std::vector<R> x, y, z;
  std::vector<int> row, sec;
  std::vector<R> X;                               // row planes
  std::vector<std::vector<int64_t>> rows;         // ids per (sector,row), ascending id
  std::vector<int64_t> up, dn, cup, cdn;

  Pipeline(const orc_geometry& g_, const orc_params& P_) : g(g_), P(P_), m(make_model<R>(g_, P_)) {}

  int ru(int s, int r) const { return s * g.n_rows + r; }

  // Neighbour finding for a middle cluster i on row r (1 <= r <= n_rows-2):
  // among down candidates d on row r-1 and up candidates u on row r+1 inside
  // the (y, z) windows, the pair whose middle point deviates least from the
  // straight chord d-u.  Score = ey^2/(1.5 sy^2) + ez^2/(1.5 sz^2) with
  // (ey, ez) the deviation of i from the chord at x_i; accepted iff <= cut;
  // ties broken by smaller up id, then smaller down id.
  void find_neighbours(int64_t i) {
    int s = sec[i], r = row[i];
    up[i] = dn[i] = -1;
    if (r < 1 || r > g.n_rows - 2) return;
    const R WY = R(P.win_y), WZ = R(P.win_z), IWY = R(P.inv_var_y), IWZ = R(P.inv_var_z), CUT = R(P.link_cut);
    bool have = false;
    R bs = R(0.0);
    int64_t bu = -1, bd = -1;
    for (int64_t d : rows[ru(s, r - 1)]) {
      if (!(Abs(y[d] - y[i]) <= WY && Abs(z[d] - z[i]) <= WZ)) continue;
      for (int64_t u : rows[ru(s, r + 1)]) {
        if (!(Abs(y[u] - y[i]) <= WY && Abs(z[u] - z[i]) <= WZ)) continue;
        R w = (x[i] - x[d]) / (x[u] - x[d]);
        R ey = y[i] - Fma(y[u] - y[d], w, y[d]);
        R ez = z[i] - Fma(z[u] - z[d], w, z[d]);
        R score = Fma(ez * ez, IWZ, (ey * ey) * IWY);
        if (!(score <= CUT)) continue;
        bool better = !have || score < bs || (score == bs && (u < bu || (u == bu && d < bd)));
        if (better) { have = true; bs = score; bu = u; bd = d; }
      }
    }
    if (have) { up[i] = bu; dn[i] = bd; }
  }

  // Search row r of sector s for the cluster closest to the predicted
  // (y, z): d = dy^2/(Cyy+sy^2) + dz^2/(Czz+sz^2) <= chi2_ext, minimum
  // (d, id).  Returns -1 if none.
  int64_t search(int s, int r, const R p[5], const R C[15]) const {
    R sy2 = C[0] + m.vy, sz2 = C[5] + m.vz;
    R isy = R(1.0) / sy2, isz = R(1.0) / sz2;
    const R CUT = R(P.chi2_ext);
    int64_t best = -1;
    R bd = R(0.0);
    for (int64_t h : rows[ru(s, r)]) {
      R dY = y[h] - p[0], dZ = z[h] - p[1];
      R d = Fma(dZ * dZ, isz, (dY * dY) * isy);
      if (!(d <= CUT)) continue;
      if (best < 0 || d < bd || (d == bd && h < best)) { best = h; bd = d; }
    }
    return best;
  }

  bool accepted_here(int r, const R p[5]) const {
    R lim = X[r] * R(g.tan_half_angle);
    return !(Abs(p[0]) > lim || Abs(p[1]) > R(g.z_max));
  }

  struct Tracklet {
    int64_t start = -1;
    int32_t nhits = 0, rlo = 0, rhi = 0;
    uint64_t key = 0;
    std::vector<int64_t> hits;
    R p[5], C[15];
  };

  // One following step on row r (used by both directions).  Returns false
  // when following must stop.
  bool follow_row(int s, int r, R p[5], R C[15], R& xc, int& rstate, Tracklet& T, int& gap,
                  bool& wrote) {
    wrote = false;
    if (!transport(p, C, xc, X[r], m)) return false;
    xc = X[r];
    rstate = r;
    if (!accepted_here(r, p)) return false;
    int64_t h = search(s, r, p, C);
    if (h >= 0) {
      if (x[h] != X[r]) {
        if (!transport(p, C, X[r], x[h], m)) return false;
        xc = x[h];
      }
      R dummy = R(0.0);
      kf_update(p, C, y[h], z[h], m.vy, m.vz, dummy);
      T.hits[r] = h;
      T.nhits++;
      gap = 0;
    } else {
      T.hits[r] = -1;
      gap++;
    }
    wrote = true;
    return gap <= P.max_gap;
  }

  // Tracklet construction from a chain head (one independent unit).
  Tracklet build(int64_t head) {
    Tracklet T;
    T.start = head;
    T.hits.assign(g.n_rows, -1);
    std::vector<int64_t> chain;
    for (int64_t h = head; h >= 0; h = cup[h]) chain.push_back(h);
    int s = sec[head], r0 = row[head];
    T.rlo = T.rhi = r0;
    // seed: position at the head, direction from the chord to the second successor
    R p[5], C[15];
    R sdir, tdir;
    int64_t h0 = chain[0], h2 = chain[2];
    chord_dir(x[h0], y[h0], z[h0], x[h2], y[h2], z[h2], sdir, tdir);
    p[0] = y[h0]; p[1] = z[h0]; p[2] = sdir; p[3] = tdir; p[4] = R(0.0);
    init_cov(C, P);
    for (int i = 0; i < 5; ++i) T.p[i] = p[i];
    for (int i = 0; i < 15; ++i) T.C[i] = C[i];
    if (!(Abs(sdir) < m.sin_max)) { T.nhits = 0; return T; }
    T.hits[r0] = h0;
    T.nhits = 1;
    R xc = x[h0];
    R dummy = R(0.0);
    for (size_t j = 1; j < chain.size(); ++j) {
      int64_t h = chain[j];
      if (!transport(p, C, xc, x[h], m)) { T.nhits = 0; T.hits.assign(g.n_rows, -1); return T; }
      if ((int)j <= kFirstUpdates) kf_update_first(p, C, y[h], z[h], m.vy, m.vz, dummy);
      else kf_update(p, C, y[h], z[h], m.vy, m.vz, dummy);
      T.hits[row[h]] = h;
      T.nhits++;
      xc = x[h];
    }
    int rstate = row[chain.back()];
    T.rhi = rstate;
    // upward following
    int gap = 0;
    for (int r = rstate + 1; r < g.n_rows; ++r) {
      bool wrote;
      bool go = follow_row(s, r, p, C, xc, rstate, T, gap, wrote);
      if (wrote) T.rhi = r;
      if (!go) break;
    }
    // back to the head row without updates, in transports of at most
    // kBackRows rows (no measurement in between, and without material a
    // helix step composes exactly), then downward following
    bool ok = true;
    for (int r = rstate; r > r0;) {
      r = std::max(r0, r - kBackRows);
      if (!transport(p, C, xc, X[r], m)) { ok = false; break; }
      xc = X[r];
    }
    if (ok) {
      gap = 0;
      int rs = r0;
      for (int r = r0 - 1; r >= 0; --r) {
        bool wrote;
        bool go = follow_row(s, r, p, C, xc, rs, T, gap, wrote);
        if (wrote) T.rlo = r;
        if (!go) break;
      }
    }
    for (int i = 0; i < 5; ++i) T.p[i] = p[i];
    for (int i = 0; i < 15; ++i) T.C[i] = C[i];
    // selection key: more hits first, then the lower start row, then the
    // smaller start id (the start row makes equal-length tracklets grown from
    // different chains of one track independent of the input order)
    T.key = ((uint64_t)(uint32_t)T.nhits << 40) | ((uint64_t)(255 - r0) << 32) |
            (uint64_t)(0xFFFFFFFFu - (uint32_t)head);
    return T;
  }
};

template <class R>
orc_result* run_pipeline(const orc_geometry& g, const orc_params& P, int64_t n, const double* xin,
                         const double* yin, const double* zin, const int16_t* rowin,
                         const uint8_t* secin, const uint8_t* mask) {
  Pipeline<R> pl(g, P);
  pl.n = n;
  pl.x.resize(n); pl.y.resize(n); pl.z.resize(n); pl.row.resize(n); pl.sec.resize(n);
  pl.X.resize(g.n_rows);
  for (int r = 0; r < g.n_rows; ++r) pl.X[r] = R(g.row_x[r]);
  pl.rows.assign((size_t)g.n_sectors * g.n_rows, {});
  for (int64_t i = 0; i < n; ++i) {
    pl.x[i] = R(xin[i]); pl.y[i] = R(yin[i]); pl.z[i] = R(zin[i]);
    pl.row[i] = rowin[i]; pl.sec[i] = secin[i];
    if (mask && !mask[secin[i]]) continue;
    pl.rows[pl.ru(secin[i], rowin[i])].push_back(i);        // ascending id by construction
  }
  pl.up.assign(n, -1); pl.dn.assign(n, -1); pl.cup.assign(n, -1); pl.cdn.assign(n, -1);
  auto active = [&](int64_t i) { return !mask || mask[pl.sec[i]]; };
  for (int64_t i = 0; i < n; ++i) if (active(i)) pl.find_neighbours(i);
  // link cleaning: keep a link only if it is reciprocated (from the raw arrays)
  for (int64_t i = 0; i < n; ++i) {
    int64_t u = pl.up[i], d = pl.dn[i];
    pl.cup[i] = (u >= 0 && pl.dn[u] == i) ? u : -1;
    pl.cdn[i] = (d >= 0 && pl.up[d] == i) ? d : -1;
  }
  // start hits in (sector, row, id) order
  std::vector<int64_t> starts;
  for (const auto& lst : pl.rows)
    for (int64_t i : lst)
      if (pl.cup[i] >= 0 && pl.cdn[i] < 0) starts.push_back(i);
  // seeds = heads of chains of at least min_seed_hits
  std::vector<typename Pipeline<R>::Tracklet> tl;
  for (int64_t h : starts) {
    int L = 0;
    for (int64_t q = h; q >= 0; q = pl.cup[q]) ++L;
    if (L < P.min_seed_hits) continue;
    tl.push_back(pl.build(h));
  }
  // selection: owner(h) = max key over the valid tracklets containing h
  std::vector<uint64_t> owner(n, 0);
  for (auto& T : tl) {
    if (T.nhits < P.min_hits) continue;
    for (int r = 0; r < g.n_rows; ++r) {
      int64_t h = T.hits[r];
      if (h >= 0) owner[h] = std::max(owner[h], T.key);
    }
  }
  orc_result* res = (orc_result*)std::calloc(1, sizeof(orc_result));
  res->n = n;
  auto cp64 = [](const std::vector<int64_t>& v) {
    int64_t* p = (int64_t*)std::malloc(sizeof(int64_t) * (v.size() + 1));
    if (!v.empty()) std::memcpy(p, v.data(), sizeof(int64_t) * v.size());
    return p;
  };
  res->up = cp64(pl.up); res->dn = cp64(pl.dn); res->cup = cp64(pl.cup); res->cdn = cp64(pl.cdn);
  res->n_starts = (int64_t)starts.size(); res->starts = cp64(starts);
  int64_t ns = (int64_t)tl.size();
  res->n_seeds = ns;
  res->seed_start = (int64_t*)std::malloc(sizeof(int64_t) * (ns + 1));
  res->seed_nhits = (int32_t*)std::malloc(sizeof(int32_t) * (ns + 1));
  res->seed_key = (uint64_t*)std::malloc(sizeof(uint64_t) * (ns + 1));
  res->seed_rlo = (int32_t*)std::malloc(sizeof(int32_t) * (ns + 1));
  res->seed_rhi = (int32_t*)std::malloc(sizeof(int32_t) * (ns + 1));
  res->seed_hits = (int64_t*)std::malloc(sizeof(int64_t) * (ns * g.n_rows + 1));
  res->seed_state = (double*)std::malloc(sizeof(double) * (ns * 20 + 1));
  for (int64_t k = 0; k < ns; ++k) {
    auto& T = tl[k];
    res->seed_start[k] = T.start; res->seed_nhits[k] = T.nhits; res->seed_key[k] = T.key;
    res->seed_rlo[k] = T.rlo; res->seed_rhi[k] = T.rhi;
    for (int r = 0; r < g.n_rows; ++r) res->seed_hits[k * g.n_rows + r] = T.hits[r];
    for (int i = 0; i < 5; ++i) res->seed_state[k * 20 + i] = val(T.p[i]);
    for (int i = 0; i < 15; ++i) res->seed_state[k * 20 + 5 + i] = val(T.C[i]);
  }
  // acceptance and final fit
  std::vector<int64_t> tseed, hoff{0}, hids;
  std::vector<int32_t> tsec, tndf;
  std::vector<double> txref, tp, tcov, tchi2;
  for (int64_t k = 0; k < ns; ++k) {
    auto& T = tl[k];
    if (T.nhits < P.min_hits) continue;
    std::vector<int64_t> own;                      // outermost first
    for (int r = g.n_rows - 1; r >= 0; --r) {
      int64_t h = T.hits[r];
      if (h >= 0 && owner[h] == T.key) own.push_back(h);
    }
    int no = (int)own.size();
    if (!(no >= P.min_hits && (int64_t)P.owned_den * no >= (int64_t)P.owned_num * T.nhits)) continue;
    std::vector<R> hx(no), hy(no), hz(no);
    for (int j = 0; j < no; ++j) { hx[j] = pl.x[own[j]]; hy[j] = pl.y[own[j]]; hz[j] = pl.z[own[j]]; }
    R p[5], C[15], chi2, xcur;
    if (!fit_hits(pl.m, P, no, hx.data(), hy.data(), hz.data(), T.p[4], p, C, chi2, xcur)) continue;
    tseed.push_back(k);
    tsec.push_back(pl.sec[T.start]);
    txref.push_back(val(xcur));
    for (int i = 0; i < 5; ++i) tp.push_back(val(p[i]));
    for (int i = 0; i < 15; ++i) tcov.push_back(val(C[i]));
    tchi2.push_back(val(chi2));
    tndf.push_back(2 * no - 5);
    for (int j = no - 1; j >= 0; --j) hids.push_back(own[j]);   // ascending row
    hoff.push_back((int64_t)hids.size());
  }
  int64_t nt = (int64_t)tseed.size();
  res->n_tracks = nt;
  res->trk_seed = cp64(tseed);
  res->trk_sector = (int32_t*)std::malloc(sizeof(int32_t) * (nt + 1));
  res->trk_ndf = (int32_t*)std::malloc(sizeof(int32_t) * (nt + 1));
  res->trk_xref = (double*)std::malloc(sizeof(double) * (nt + 1));
  res->trk_chi2 = (double*)std::malloc(sizeof(double) * (nt + 1));
  res->trk_p = (double*)std::malloc(sizeof(double) * (5 * nt + 1));
  res->trk_cov = (double*)std::malloc(sizeof(double) * (15 * nt + 1));
  for (int64_t t = 0; t < nt; ++t) {
    res->trk_sector[t] = tsec[t]; res->trk_ndf[t] = tndf[t];
    res->trk_xref[t] = txref[t]; res->trk_chi2[t] = tchi2[t];
  }
  if (nt) {
    std::memcpy(res->trk_p, tp.data(), sizeof(double) * 5 * nt);
    std::memcpy(res->trk_cov, tcov.data(), sizeof(double) * 15 * nt);
  }
  res->hit_off = cp64(hoff);
  res->hit_ids = cp64(hids);
  return res;
}

// ---------------------------------------------------------------------------
// Sector track merger.  The paper processes the TPC sectors independently
// and merges their track segments afterwards (Sec. "Track reconstruction in
// the TPC"); its rules are not given, so every rule below is a reading.
//
// Rotation of a state from the frame of one sector into a frame turned by
// dalpha about z (ca = cos dalpha, sa = sin dalpha).  The point (x, y) of
// the track becomes (x ca + y sa, -x sa + y ca); the direction angle drops
// by dalpha, so s' = s ca - c sa with c = +sqrt(1 - s^2) (tracks move
// outward in x); z, tan(lambda) and q/pT are unchanged.  The new state
// lives on the plane x' of the rotated point.  Its covariance is J C J^T
// with J the Jacobian at that fixed plane: a shift dy of the old point
// moves the new point by (sa, ca) dy, and bringing it back to the plane x'
// along the track (slope tan phi' = s'/c' in y, t/c' in z, curvature kap in
// s) gives
//   dy'/dy = ca - (s'/c') sa,  dz'/dy = -(t/c') sa,  ds'/dy = -kap sa,
//   ds'/ds = ca + sa s/c,  and 1 on the diagonal for z, t, k.
template <class R>
bool rotate_state(R& x, R p[5], R C[15], R ca, R sa, const Model<R>& m, R* Jout = nullptr) {
  const R s = p[2];
  const R c = Sqrt(R(1.0) - s * s);
  const R s2 = s * ca - c * sa;
  if (!(Abs(s2) < m.sin_max)) return false;
  const R c2 = Sqrt(R(1.0) - s2 * s2);
  const R kap = m.kfac * p[4];
  const R x2 = x * ca + p[0] * sa;
  const R y2 = -(x * sa) + p[0] * ca;
  R J[25];
  for (int i = 0; i < 25; ++i) J[i] = R(0.0);
  J[0 * 5 + 0] = ca - (s2 / c2) * sa;
  J[1 * 5 + 0] = -(p[3] / c2) * sa;
  J[1 * 5 + 1] = R(1.0);
  J[2 * 5 + 0] = -kap * sa;
  J[2 * 5 + 2] = ca + sa * (s / c);
  J[3 * 5 + 3] = R(1.0);
  J[4 * 5 + 4] = R(1.0);
  R T[25], Cn[15];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      R acc = R(0.0);
      for (int k = 0; k < 5; ++k) acc = acc + J[i * 5 + k] * C[ix(k, j)];
      T[i * 5 + j] = acc;
    }
  for (int i = 0; i < 5; ++i)
    for (int j = i; j < 5; ++j) {
      R acc = R(0.0);
      for (int k = 0; k < 5; ++k) acc = acc + T[i * 5 + k] * J[j * 5 + k];
      Cn[ix(i, j)] = acc;
    }
  for (int i = 0; i < 15; ++i) C[i] = Cn[i];
  x = x2;
  p[0] = y2;
  p[2] = s2;
  if (Jout) for (int i = 0; i < 25; ++i) Jout[i] = J[i];
  return true;
}

// Centre angle of a sector's frame (R-1: wedge w = s mod 18 centred at
// (w + 1/2) 20 degrees), and the turn from frame a to frame b in (-pi, pi].
double sector_alpha(int s, int n_sectors) {
  const int nw = n_sectors / 2;
  return ((s % nw) + 0.5) * (2.0 * M_PI / nw);
}
double frame_turn(int sa, int sb, int n_sectors) {
  double d = sector_alpha(sb, n_sectors) - sector_alpha(sa, n_sectors);
  while (d > M_PI) d -= 2.0 * M_PI;
  while (d <= -M_PI) d += 2.0 * M_PI;
  return d;
}

// Match chi2 of two 5-vectors' difference under the covariance M (packed):
// Delta^T M^-1 Delta by Cholesky decomposition.  Returns false if M is not
// positive definite.
bool match_chi2(const double d[5], const double M[15], double& chi2) {
  double L[5][5] = {};
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j <= i; ++j) {
      double acc = M[ix(i, j)];
      for (int k = 0; k < j; ++k) acc -= L[i][k] * L[j][k];
      if (i == j) {
        if (!(acc > 0.0)) return false;
        L[i][i] = std::sqrt(acc);
      } else {
        L[i][j] = acc / L[j][j];
      }
    }
  double w[5];
  chi2 = 0.0;
  for (int i = 0; i < 5; ++i) {
    double acc = d[i];
    for (int k = 0; k < i; ++k) acc -= L[i][k] * w[k];
    w[i] = acc / L[i][i];
    chi2 += w[i] * w[i];
  }
  return true;
}

// The merger on one event (FP64), in the order of the rules:
//  1. exit state of every segment: its state at the innermost hit transported
//     (in its own frame) to the plane of its outermost hit's x;
//  2. a pair (a inner, b outer) is a candidate iff a and b lie in sectors of
//     the same side whose wedges are adjacent, a's last pad row is below b's
//     first, and a's outermost hit lies within merge_dist of b's innermost
//     hit both in the transverse plane and in z; in a time frame (slice
//     indices given) also a pair in the same sector whose slices are
//     neighbours, under the same row and distance conditions (no rotation);
//  3. its match chi2: a's exit state rotated into b's frame and transported
//     to b's reference plane, compared with b's state: Delta^T (C_a + C_b)^-1
//     Delta over the five parameters; a candidate is valid iff the rotation
//     and transport succeed and chi2 <= chi2_merge;
//  4. every segment takes its best valid partner on each side (smallest
//     chi2, ties by the smaller segment index); a link a -> b is kept iff b
//     is a's best outer and a is b's best inner partner;
//  5. links form chains (a segment has at most one inner and one outer
//     partner, rows increase along a chain); each chain of two or more
//     segments is refitted as one track (refit_chain); chains whose refit
//     fails stay split into their segments.
// Output in the order of the segments: a segment without an inner link
// emits its chain (or, if unmerged, itself); the others are emitted with
// their chain.
template <class R>
bool refit_chain(const orc_geometry& g, const orc_params& P, const Model<R>& m,
                 const std::vector<int>& chain, const std::vector<int>& sec,
                 const std::vector<std::vector<int64_t>>& hits, const double* x, const double* y,
                 const double* z, R k0, R p[5], R C[15], R& chi2, R& xref);

struct MergeOut {
  std::vector<int> link, best_in, best_out;
  std::vector<double> chi_in, chi_in2, chi_out, chi_out2;
  // merged tracks
  std::vector<int64_t> head;
  std::vector<int32_t> sector, ndf;
  std::vector<double> xref, p, cov, chi2;
  std::vector<int64_t> hit_off, hit_ids;
};

MergeOut merge_segments(const orc_geometry& g, const orc_params& P, const double* x, const double* y,
                        const double* z, const int16_t* row, int64_t nseg, const int32_t* ssec,
                        const double* sxref, const double* sp, const double* scov, const double* schi2,
                        const int64_t* soff, const int64_t* sids, const int32_t* sslice) {
  const Model<double> m = make_model<double>(g, P);
  const int S = g.n_sectors, NW = S / 2;
  const double INF = std::numeric_limits<double>::infinity();
  std::vector<std::vector<int64_t>> hits(nseg);
  std::vector<int> sec(nseg), rlo(nseg), rhi(nseg);
  std::vector<bool> has_exit(nseg, false);
  std::vector<double> ex(nseg), ep((size_t)nseg * 5), ec((size_t)nseg * 15);
  for (int64_t i = 0; i < nseg; ++i) {
    hits[i].assign(sids + soff[i], sids + soff[i + 1]);
    sec[i] = ssec[i];
    rlo[i] = row[hits[i].front()];
    rhi[i] = row[hits[i].back()];
    // 1. exit state
    double q[5], Q[15];
    for (int k = 0; k < 5; ++k) q[k] = sp[i * 5 + k];
    for (int k = 0; k < 15; ++k) Q[k] = scov[i * 15 + k];
    const double xo = x[hits[i].back()];
    if (transport(q, Q, sxref[i], xo, m)) {
      has_exit[i] = true;
      ex[i] = xo;
      for (int k = 0; k < 5; ++k) ep[i * 5 + k] = q[k];
      for (int k = 0; k < 15; ++k) ec[i * 15 + k] = Q[k];
    }
  }
  MergeOut o;
  o.link.assign(nseg, -1);
  o.best_in.assign(nseg, -1); o.best_out.assign(nseg, -1);
  o.chi_in.assign(nseg, INF); o.chi_in2.assign(nseg, INF);
  o.chi_out.assign(nseg, INF); o.chi_out2.assign(nseg, INF);
  auto offer = [&](int& best, double& bchi, double& bchi2, int cand, double chi) {
    if (chi < bchi || (chi == bchi && cand < best)) {
      bchi2 = bchi;
      bchi = chi;
      best = cand;
    } else if (chi < bchi2) {
      bchi2 = chi;
    }
  };
  for (int64_t a = 0; a < nseg; ++a) {
    if (!has_exit[a]) continue;
    for (int64_t b = 0; b < nseg; ++b) {
      // 2. candidate
      const bool same_side = (sec[a] < NW) == (sec[b] < NW);
      const int wa = sec[a] % NW, wb = sec[b] % NW;
      const bool adjacent = (wb == (wa + 1) % NW) || (wa == (wb + 1) % NW);
      const bool slices = sec[a] == sec[b] && sslice != nullptr && std::abs(sslice[a] - sslice[b]) == 1;
      if (!((same_side && adjacent) || slices) || !(rhi[a] < rlo[b])) continue;
      const double turn = slices ? 0.0 : frame_turn(sec[a], sec[b], S);
      const double ca = std::cos(turn), sa = std::sin(turn);
      const int64_t ha = hits[a].back(), hb = hits[b].front();
      const double xa = x[ha] * ca + y[ha] * sa, ya = -(x[ha] * sa) + y[ha] * ca;
      const double dr = std::sqrt((xa - x[hb]) * (xa - x[hb]) + (ya - y[hb]) * (ya - y[hb]));
      if (!(dr <= P.merge_dist && std::fabs(z[ha] - z[hb]) <= P.merge_dist)) continue;
      // 3. match chi2
      double xx = ex[a], q[5], Q[15];
      for (int k = 0; k < 5; ++k) q[k] = ep[a * 5 + k];
      for (int k = 0; k < 15; ++k) Q[k] = ec[a * 15 + k];
      if (!slices && !rotate_state(xx, q, Q, ca, sa, m)) continue;
      if (!transport(q, Q, xx, sxref[b], m)) continue;
      double d[5], M[15], chi;
      for (int k = 0; k < 5; ++k) d[k] = q[k] - sp[b * 5 + k];
      for (int k = 0; k < 15; ++k) M[k] = Q[k] + scov[b * 15 + k];
      if (!match_chi2(d, M, chi) || !(chi <= P.chi2_merge)) continue;
      // 4. best partners
      offer(o.best_out[a], o.chi_out[a], o.chi_out2[a], (int)b, chi);
      offer(o.best_in[b], o.chi_in[b], o.chi_in2[b], (int)a, chi);
    }
  }
  std::vector<int> inner(nseg, -1);
  for (int64_t a = 0; a < nseg; ++a) {
    const int b = o.best_out[a];
    if (b >= 0 && o.best_in[b] == a) { o.link[a] = b; inner[b] = (int)a; }
  }
  // 5. chains and their refit
  o.hit_off.push_back(0);
  auto emit_one = [&](int i) {
    o.head.push_back(i);
    o.sector.push_back(sec[i]);
    o.xref.push_back(sxref[i]);
    for (int k = 0; k < 5; ++k) o.p.push_back(sp[i * 5 + k]);
    for (int k = 0; k < 15; ++k) o.cov.push_back(scov[i * 15 + k]);
    o.chi2.push_back(schi2[i]);
    o.ndf.push_back(2 * (int)hits[i].size() - 5);
    for (int64_t h : hits[i]) o.hit_ids.push_back(h);
    o.hit_off.push_back((int64_t)o.hit_ids.size());
  };
  for (int64_t i = 0; i < nseg; ++i) {
    if (inner[i] >= 0) continue;
    std::vector<int> chain{(int)i};
    while (o.link[chain.back()] >= 0) chain.push_back(o.link[chain.back()]);
    if (chain.size() == 1) { emit_one((int)i); continue; }
    double p[5], C[15], chi2, xr;
    const double k0 = sp[(size_t)chain.back() * 5 + 4];
    if (!refit_chain(g, P, m, chain, sec, hits, x, y, z, k0, p, C, chi2, xr)) {
      for (int c : chain) emit_one(c);
      continue;
    }
    o.head.push_back(i);
    o.sector.push_back(sec[i]);
    o.xref.push_back(xr);
    for (int k = 0; k < 5; ++k) o.p.push_back(p[k]);
    for (int k = 0; k < 15; ++k) o.cov.push_back(C[k]);
    o.chi2.push_back(chi2);
    int64_t n = 0;
    for (int c : chain) {
      for (int64_t h : hits[c]) o.hit_ids.push_back(h);
      n += (int64_t)hits[c].size();
    }
    o.ndf.push_back(2 * (int)n - 5);
    o.hit_off.push_back((int64_t)o.hit_ids.size());
  }
  return o;
}

// Refit of a chain of segments (innermost first) as one track: the final fit
// of the selection step over all its hits, outermost first (state at the
// outermost hit, direction from the chord to the hit two positions inward,
// q/pT prior k0, initial covariance as there), crossing each segment
// boundary by rotating the state into the next inner segment's frame;
// result at the innermost hit.
template <class R>
bool refit_chain(const orc_geometry& g, const orc_params& P, const Model<R>& m,
                 const std::vector<int>& chain, const std::vector<int>& sec,
                 const std::vector<std::vector<int64_t>>& hits, const double* x, const double* y,
                 const double* z, R k0, R p[5], R C[15], R& chi2, R& xref) {
  const int S = g.n_sectors;
  // outermost segment's hits, outermost first
  int ci = (int)chain.size() - 1;
  const std::vector<int64_t>* hl = &hits[chain[ci]];
  int hi = (int)hl->size() - 1;
  if (hi < 2) return false;
  auto X = [&](int64_t h) { return R(x[h]); };
  auto Y = [&](int64_t h) { return R(y[h]); };
  auto Z = [&](int64_t h) { return R(z[h]); };
  const int64_t h0 = (*hl)[hi], h2 = (*hl)[hi - 2];
  R s, t;
  chord_dir(X(h2), Y(h2), Z(h2), X(h0), Y(h0), Z(h0), s, t);
  p[0] = Y(h0); p[1] = Z(h0); p[2] = s; p[3] = t; p[4] = k0;
  init_cov(C, P);
  chi2 = R(0.0);
  if (!(Abs(s) < m.sin_max)) return false;
  R xc = X(h0);
  --hi;
  while (true) {
    for (; hi >= 0; --hi) {
      const int64_t h = (*hl)[hi];
      if (!transport(p, C, xc, X(h), m)) return false;
      kf_update(p, C, Y(h), Z(h), m.vy, m.vz, chi2);
      xc = X(h);
    }
    if (ci == 0) break;
    // into the frame of the next inner segment
    // (segments of one sector from neighbouring slices share the frame)
    const double turn = frame_turn(sec[chain[ci]], sec[chain[ci - 1]], S);
    if (sec[chain[ci]] != sec[chain[ci - 1]] &&
        !rotate_state(xc, p, C, R(std::cos(turn)), R(std::sin(turn)), m))
      return false;
    --ci;
    hl = &hits[chain[ci]];
    hi = (int)hl->size() - 1;
  }
  xref = xc;
  return true;
}

// ---------------------------------------------------------------------------
// Calibration correction (applied to default-transformed clusters):
//  drift: with side = +1 for A-side sectors (first half), -1 otherwise,
//         side*z' = L - (1 + delta_s) * (L - side*z - tau_s);
//  radial: x' = x + sum_ab c[s][a][b] B_a(xh) B_b(uh) with xh = (x - x_first)
//         / (x_last - x_first), uh = (y/x + tanA)/(2 tanA), both clamped to
//         [0, 1] and evaluated at the uncorrected (x, y).
// B_a: the 8 clamped uniform cubic B-splines (knots 0,0,0,0,.2,.4,.6,.8,1,1,1,1).
void bspline8(double u, double B[8]) {
  static const double t[12] = {0, 0, 0, 0, 0.2, 0.4, 0.6, 0.8, 1, 1, 1, 1};
  if (u < 0.0) u = 0.0;
  if (u > 1.0) u = 1.0;
  double N[11];
  for (int i = 0; i < 11; ++i) N[i] = (t[i] <= u && u < t[i + 1]) ? 1.0 : 0.0;
  if (u >= 1.0) N[7] = 1.0;
  for (int p = 1; p <= 3; ++p) {
    for (int i = 0; i < 11 - p; ++i) {
      double a = (t[i + p] > t[i]) ? (u - t[i]) / (t[i + p] - t[i]) : 0.0;
      double b = (t[i + p + 1] > t[i + 1]) ? (t[i + p + 1] - u) / (t[i + p + 1] - t[i + 1]) : 0.0;
      N[i] = a * N[i] + b * N[i + 1];
    }
  }
  for (int i = 0; i < 8; ++i) B[i] = N[i];
}

template <class R>
void calib_point(const orc_geometry& g, int s, double x, double y, double z, const R* th, R& xo,
                 R& zo) {
  int half = g.n_sectors / 2;
  double side = s < half ? 1.0 : -1.0;
  double L = g.z_max;
  const R& dl = th[s];
  const R& tau = th[g.n_sectors + s];
  zo = R(side) * (R(L) - (R(1.0) + dl) * (R(L - side * z) - tau));
  double x0 = g.row_x[0], x1 = g.row_x[g.n_rows - 1];
  double ta = g.tan_half_angle;
  double Ba[8], Bb[8];
  bspline8((x - x0) / (x1 - x0), Ba);
  bspline8((y / x + ta) / (2.0 * ta), Bb);
  const R* c = th + 2 * g.n_sectors + (size_t)s * 64;
  R acc = R(x);
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b) {
      double w = Ba[a] * Bb[b];
      if (w != 0.0) acc = acc + c[a * 8 + b] * R(w);
    }
  xo = acc;
}

// The same correction as the tracker applies it to its FP32 input, every
// operation rounded to FP32 in this order (no contraction):
//   z' = z + side (tau - delta (D - tau)),  D = L - side z
//        (side z' = L - (1 + delta)(D - tau) rearranged so that the small
//        correction is added to z: theta = 0 leaves z unchanged);
//   x' = x + sum_a Na[a] (sum_b c[fa + a][fb + b] Nb[b])  over the four
//        non-zero basis functions of each direction, ascending indices,
//        each sum starting at +0;
// with the basis values from de Boor's triangular recursion on the knot
// span of the clamped argument.
static void bspline_nonzero32(float u, int& first, float N[4]) {
  static const float U[12] = {0.f, 0.f, 0.f, 0.f, 0.2f, 0.4f, 0.6f, 0.8f, 1.f, 1.f, 1.f, 1.f};
  u = std::min(std::max(u, 0.0f), 1.0f);
  int i = 3;                              // span: U[i] <= u < U[i+1]; the last one for u = 1
  while (i < 7 && u >= U[i + 1]) ++i;
  float left[4], right[4];
  N[0] = 1.0f;
  for (int j = 1; j <= 3; ++j) {
    left[j] = u - U[i + 1 - j];
    right[j] = U[i + j] - u;
    float saved = 0.0f;
    for (int r = 0; r < j; ++r) {
      const float temp = N[r] / (right[r + 1] + left[j - r]);
      N[r] = saved + right[r + 1] * temp;
      saved = left[j - r] * temp;
    }
    N[j] = saved;
  }
  first = i - 3;
}

void calib_point32(const orc_geometry& g, int s, float x, float y, float z, const float* th, float& xo,
                   float& zo) {
  const int S = g.n_sectors;
  const float side = s < S / 2 ? 1.0f : -1.0f;
  const float L = g.z_max;
  const float dl = th[s], tau = th[S + s];
  const float D = L - side * z;
  zo = z + side * (tau - dl * (D - tau));
  const float xf = g.row_x[0], xl = g.row_x[g.n_rows - 1];
  const float ta = g.tan_half_angle;
  float Na[4], Nb[4];
  int fa, fb;
  bspline_nonzero32((x - xf) / (xl - xf), fa, Na);
  bspline_nonzero32((y / x + ta) / (2.0f * ta), fb, Nb);
  const float* c = th + 2 * S + (size_t)s * 64;
  float d = 0.0f;
  for (int a = 0; a < 4; ++a) {
    float inner = 0.0f;
    for (int b = 0; b < 4; ++b) inner = inner + c[(fa + a) * 8 + (fb + b)] * Nb[b];
    d = d + Na[a] * inner;
  }
  xo = x + d;
}

// Calibration objective of one track (see orc_calib_chi2).
// Returns 0 if the hit fit fails, 1 if only the hits were used (vertex terms
// off, or the transport to the beam axis left the sin(phi) range), 2 if the
// vertex (and, if enabled, the external tan(lambda)) were added.
template <class R>
int track_objective(const orc_geometry& g, const orc_params& P, const Model<R>& m, int nh,
                    const R* hx, const R* hy, const R* hz, R k0, bool use_vtx, bool use_ext,
                    R ext_tgl, R& chi2) {
  (void)g;
  R p[5], C[15], xcur;
  if (!fit_hits(m, P, nh, hx, hy, hz, k0, p, C, chi2, xcur)) return 0;
  if (!use_vtx) return 1;
  // sub-stepped transport to the beam axis at x = 0 (planes at multiples of 10 cm)
  R q[5], Q[15];
  for (int i = 0; i < 5; ++i) q[i] = p[i];
  for (int i = 0; i < 15; ++i) Q[i] = C[i];
  int mstep = (int)std::ceil(val(xcur) / 10.0) - 1;
  R xc = xcur;
  for (int k = mstep; k >= 0; --k) {
    R xt = R(10.0 * k);
    if (!transport(q, Q, xc, xt, m)) return 1;         // vertex terms skipped
    xc = xt;
  }
  R sv2 = R(P.sigma_vertex) * R(P.sigma_vertex);
  kf_update(q, Q, R(0.0), R(0.0), sv2, sv2, chi2);
  if (use_ext) kf_update1(q, Q, 3, ext_tgl, R(P.sigma_tgl) * R(P.sigma_tgl), chi2);
  return 2;
}


// ===========================================================================
// ITS standalone tracking (paper, Sec. "Fast ITS standalone tracking" and
// Sec. "Luminous region estimation based on ITS tracking"; reading R-26).
// Six layers of flat staves around the beam axis; every decision in FP32
// with the expressions written here (the GPU library evaluates the same
// ones), the vertex fit in FP64.

struct ItsGeo {
  int L = 0;
  float r[6], hz[6], xx0[6], vy[6], vz[6], kms[6];
  int ns[6];
  std::vector<float> ca[6], sa[6];   // stave centre angle (k + 1/2) 2 pi / n
  std::vector<float> bc[6], bs[6];   // wedge boundary angle j 2 pi / n, j = 0 .. n
  Model<float> m;
};

ItsGeo its_geo(const orc_its_geometry& g, const orc_its_params& P) {
  ItsGeo G;
  G.L = g.n_layers;
  for (int l = 0; l < G.L; ++l) {
    G.r[l] = g.radius[l]; G.hz[l] = g.half_z[l]; G.xx0[l] = g.x_over_x0[l];
    G.vy[l] = g.sigma_y[l] * g.sigma_y[l]; G.vz[l] = g.sigma_z[l] * g.sigma_z[l];
    G.ns[l] = g.n_staves[l];
    // Highland's logarithmic factor at normal incidence (a per-layer constant)
    G.kms[l] = (float)(1.0 + 0.038 * std::log((double)g.x_over_x0[l]));
    const double d = 2.0 * M_PI / (double)g.n_staves[l];
    for (int k = 0; k < G.ns[l]; ++k) {
      G.ca[l].push_back((float)std::cos((k + 0.5) * d));
      G.sa[l].push_back((float)std::sin((k + 0.5) * d));
    }
    for (int j = 0; j <= G.ns[l]; ++j) {
      G.bc[l].push_back((float)std::cos(j * d));
      G.bs[l].push_back((float)std::sin(j * d));
    }
  }
  G.m.kfac = -(float)((double)2.99792458e-3) * g.bz;
  G.m.sin_max = P.sin_max;
  G.m.vy = 0.0f;
  G.m.vz = 0.0f;
  return G;
}

// Multiple scattering in the average material of a layer (thin layer, no
// energy loss): two independent small deflections of variance theta0^2
// perpendicular to the direction change phi by d1 / cos(lambda) and lambda
// by d2, hence var(sin phi) = theta0^2 cos^2 phi / cos^2 lambda, var(tan
// lambda) = theta0^2 / cos^4 lambda, var(q/pT) = theta0^2 (q/pT)^2 tan^2
// lambda, cov(tan lambda, q/pT) = theta0^2 (q/pT) tan lambda / cos^2 lambda.
// theta0 by Highland's formula for beta = 1 with the path through the
// stave, x/X0 / (cos lambda cos phi), the logarithmic factor taken at
// normal incidence.
void its_ms(float p[5], float C[15], float xx0, float kms) {
  const float s = p[2], t = p[3], k = p[4];
  const float t2 = 1.0f + t * t;
  const float c2 = 1.0f - s * s;
  const float path = xx0 * Sqrt(t2 / c2);
  const float pin = (k * k) / t2;
  const float hl = 0.0136f;
  const float th2 = (((hl * hl) * pin) * path) * (kms * kms);
  const float kt = k * t;
  C[ix(2, 2)] = C[ix(2, 2)] + th2 * (c2 * t2);
  C[ix(3, 3)] = C[ix(3, 3)] + th2 * (t2 * t2);
  C[ix(3, 4)] = C[ix(3, 4)] + th2 * (t2 * kt);
  C[ix(4, 4)] = C[ix(4, 4)] + th2 * (kt * kt);
}

struct ItsCl {
  float x, y, z, X, Y, r;
  int l, k;
};

struct ItsOut {
  std::vector<int64_t> hist;
  int64_t npairs = 0, qn = 0, qsum = 0;
  int peak = -1, vz_ok = 0;
  float vz = 0.0f;
  std::vector<int32_t> tl0, tl1;
  std::vector<int32_t> ok, cls, ncls, ostave, olayer, istave, iok;
  std::vector<float> chi2, ox, op, oc, ip, ic;
  double V[3] = {0, 0, 0};
  double sumw = 0.0;
  int nused = 0, vfit_ok = 0;
};

// SPD pair test (vertexer and tracklets): the two clusters lie within the
// azimuth window seen from the beam axis (|sin dphi| <= sphi, same side).
inline bool spd_pair(const ItsCl& a, const ItsCl& b, float sphi, float& cross) {
  cross = a.X * b.Y - a.Y * b.X;
  const float dot = a.X * b.X + a.Y * b.Y;
  return dot > 0.0f && Abs(cross) <= sphi * (a.r * b.r);
}

ItsOut its_run(const orc_its_geometry& g, const orc_its_params& P, int64_t n, const float* x, const float* y,
               const float* z, const int8_t* layer, const int16_t* stave) {
  const ItsGeo G = its_geo(g, P);
  ItsOut o;
  std::vector<ItsCl> c(n);
  std::vector<std::vector<int32_t>> lists(6 * 64);   // clusters per (layer, stave), ascending id
  std::vector<int32_t> L0, L1;
  for (int64_t i = 0; i < n; ++i) {
    ItsCl& q = c[i];
    q.x = x[i]; q.y = y[i]; q.z = z[i]; q.l = layer[i]; q.k = stave[i];
    const float ca = G.ca[q.l][q.k], sa = G.sa[q.l][q.k];
    q.X = q.x * ca - q.y * sa;
    q.Y = q.x * sa + q.y * ca;
    q.r = Sqrt(q.X * q.X + q.Y * q.Y);
    lists[q.l * 64 + q.k].push_back((int32_t)i);
    if (q.l == 0) L0.push_back((int32_t)i);
    if (q.l == 1) L1.push_back((int32_t)i);
  }
  // 1. vertexer: z where the SPD pair lines cross the beam axis, histogram
  // peak (ties: lower bin), then the mean over the peak bin and its two
  // neighbours in fixed point (2^-16 cm)
  const int nb = (int)std::lrint(2.0 * (double)P.vtx_range / (double)P.vtx_bin);
  o.hist.assign(nb, 0);
  auto zline = [&](const ItsCl& a, const ItsCl& b) { return a.z - a.r * ((b.z - a.z) / (b.r - a.r)); };
  auto bin_of = [&](float zv) {
    const float u = (zv + P.vtx_range) / P.vtx_bin;
    if (!(u >= 0.0f) || !(u < (float)nb)) return -1;
    return (int)std::floor(u);
  };
  for (int32_t i0 : L0)
    for (int32_t i1 : L1) {
      float cr;
      if (!spd_pair(c[i0], c[i1], P.vtx_sin_phi, cr)) continue;
      const int b = bin_of(zline(c[i0], c[i1]));
      if (b < 0) continue;
      ++o.hist[b];
      ++o.npairs;
    }
  int64_t best = 0;
  for (int b = 0; b < nb; ++b)
    if (o.hist[b] > best) { best = o.hist[b]; o.peak = b; }
  if (o.peak >= 0) {
    for (int32_t i0 : L0)
      for (int32_t i1 : L1) {
        float cr;
        if (!spd_pair(c[i0], c[i1], P.vtx_sin_phi, cr)) continue;
        const float zv = zline(c[i0], c[i1]);
        const int b = bin_of(zv);
        if (b < 0 || b < o.peak - 1 || b > o.peak + 1) continue;
        o.qsum += (int64_t)std::rint(zv * 65536.0f);
        ++o.qn;
      }
    o.vz = (float)((double)o.qsum / (double)o.qn / 65536.0);
    o.vz_ok = 1;
  }
  const float vz = o.vz;
  // 2. tracklets: mutual best SPD pairs seen under nearly the same angles
  // from the vertex (beam axis at the origin, z = vz)
  const float itp2 = 1.0f / (P.trk_sin_phi * P.trk_sin_phi), itt2 = 1.0f / (P.trk_dtgl * P.trk_dtgl);
  std::vector<std::pair<float, int32_t>> b0(n, {INFINITY, -1}), b1(n, {INFINITY, -1});
  auto better = [](std::pair<float, int32_t>& cur, float sc, int32_t id) {
    if (sc < cur.first || (sc == cur.first && id < cur.second)) cur = {sc, id};
  };
  for (int32_t i0 : L0)
    for (int32_t i1 : L1) {
      const ItsCl &a = c[i0], &b = c[i1];
      float cr;
      if (!spd_pair(a, b, P.trk_sin_phi, cr)) continue;
      const float dt = (b.z - vz) / b.r - (a.z - vz) / a.r;
      if (!(Abs(dt) <= P.trk_dtgl)) continue;
      const float sp = cr / (a.r * b.r);
      const float sc = (sp * sp) * itp2 + (dt * dt) * itt2;
      better(b0[i0], sc, i1);
      better(b1[i1], sc, i0);
    }
  for (int32_t i0 : L0) {   // (L0 in ascending id)
    const int32_t i1 = b0[i0].second;
    if (i1 >= 0 && b1[i1].second == i0) { o.tl0.push_back(i0); o.tl1.push_back(i1); }
  }
  // 3. following, one tracklet at a time
  const int64_t T = (int64_t)o.tl0.size();
  o.ok.assign(T, 0); o.cls.assign(T * 6, -1); o.ncls.assign(T, 0); o.ostave.assign(T, -1);
  o.olayer.assign(T, -1); o.istave.assign(T, -1); o.iok.assign(T, 0);
  o.chi2.assign(T, 0.0f); o.ox.assign(T, 0.0f); o.op.assign(T * 5, 0.0f); o.oc.assign(T * 15, 0.0f);
  o.ip.assign(T * 5, 0.0f); o.ic.assign(T * 15, 0.0f);
  const Model<float>& m = G.m;
  for (int64_t t = 0; t < T; ++t) {
    const ItsCl &a = c[o.tl0[t]], &b = c[o.tl1[t]];
    // initial state at the beam axis (x = 0 in the frame of a's stave): the
    // vertex as the measured point, direction and q/pT from the circle
    // through the axis and the two SPD clusters
    const float ca0 = G.ca[0][a.k], sa0 = G.sa[0][a.k];
    const float bx = b.X * ca0 + b.Y * sa0, by = -(b.X * sa0) + b.Y * ca0;
    const float la = Sqrt(a.x * a.x + a.y * a.y), lb = Sqrt(bx * bx + by * by);
    const float ex = bx - a.x, ey = by - a.y, lab = Sqrt(ex * ex + ey * ey);
    const float crs = a.x * by - a.y * bx;
    const float kap = (2.0f * crs) / ((la * lb) * lab);
    const float dl = (kap * la) * 0.5f;
    const float cd = Sqrt(1.0f - dl * dl);
    float p[5], C[15];
    p[0] = 0.0f;
    p[1] = vz;
    p[2] = (a.y / la) * cd - (a.x / la) * dl;
    p[3] = (b.z - a.z) / lab;
    p[4] = kap / m.kfac;
    for (int i = 0; i < 15; ++i) C[i] = 0.0f;
    C[ix(0, 0)] = P.sigma_vy * P.sigma_vy;
    C[ix(1, 1)] = P.sigma_vz * P.sigma_vz;
    C[ix(2, 2)] = 1e-2f;
    C[ix(3, 3)] = 1e-2f;
    C[ix(4, 4)] = 1.0f;
    float chi2 = 0.0f, xc = 0.0f;
    int kst[6] = {-1, -1, -1, -1, -1, -1};
    int32_t cl[6] = {-1, -1, -1, -1, -1, -1};
    bool alive = Abs(p[2]) < m.sin_max;
    int lc = -1, kc = -1, ncl = 0, miss = 0;
    bool rejected = false;
    // the tracklet's SPD clusters
    for (int l = 0; l < 2 && alive; ++l) {
      const ItsCl& h = l == 0 ? a : b;
      if (l == 1) {
        const float dca = G.ca[1][h.k] * G.ca[0][kc] + G.sa[1][h.k] * G.sa[0][kc];
        const float dsa = G.sa[1][h.k] * G.ca[0][kc] - G.ca[1][h.k] * G.sa[0][kc];
        if (!rotate_state(xc, p, C, dca, dsa, m)) { alive = false; break; }
      }
      if (!transport(p, C, xc, h.x, m)) { alive = false; break; }
      xc = h.x;
      kf_update(p, C, h.y, h.z, G.vy[l], G.vz[l], chi2);
      its_ms(p, C, G.xx0[l], G.kms[l]);
      cl[l] = l == 0 ? o.tl0[t] : o.tl1[t];
      kst[l] = h.k;
      lc = l; kc = h.k;
      ++ncl;
    }
    for (int l = 2; l < G.L && alive; ++l) {
      // the stave whose wedge holds the prediction on the plane at r_l
      // parallel to the current stave
      float pp[5], CC[15];
      for (int i = 0; i < 5; ++i) pp[i] = p[i];
      for (int i = 0; i < 15; ++i) CC[i] = C[i];
      if (!transport(pp, CC, xc, G.r[l], m)) { alive = false; break; }
      const float X = G.r[l] * G.ca[lc][kc] - pp[0] * G.sa[lc][kc];
      const float Y = G.r[l] * G.sa[lc][kc] + pp[0] * G.ca[lc][kc];
      const int ns = G.ns[l];
      int k = ((2 * kc + 1) * ns) / (2 * G.ns[lc]);
      for (int it = 0; it < 4; ++it) {
        const bool lo = G.bc[l][k] * Y - G.bs[l][k] * X >= 0.0f;
        const bool hi = G.bc[l][k + 1] * Y - G.bs[l][k + 1] * X < 0.0f;
        if (lo && hi) break;
        k = lo ? (k + 1) % ns : (k + ns - 1) % ns;
      }
      const float dca = G.ca[l][k] * G.ca[lc][kc] + G.sa[l][k] * G.sa[lc][kc];
      const float dsa = G.sa[l][k] * G.ca[lc][kc] - G.ca[l][k] * G.sa[lc][kc];
      if (!rotate_state(xc, p, C, dca, dsa, m)) { alive = false; break; }
      if (!transport(p, C, xc, G.r[l], m)) { alive = false; break; }
      xc = G.r[l];
      lc = l; kc = k; kst[l] = k;
      // closest cluster of the stave under the chi2 cut (ties: lower id)
      const float isy = 1.0f / (C[0] + G.vy[l]), isz = 1.0f / (C[5] + G.vz[l]);
      float bchi = P.chi2_cut;
      int32_t bid = -1;
      for (int32_t id : lists[l * 64 + k]) {
        const float dy = c[id].y - p[0], dz = c[id].z - p[1];
        const float ch = (dy * dy) * isy + (dz * dz) * isz;
        if (ch < bchi || (ch == bchi && (bid < 0 || id < bid))) { bchi = ch; bid = id; }
      }
      if (bid >= 0) {
        kf_update(p, C, c[bid].y, c[bid].z, G.vy[l], G.vz[l], chi2);
        cl[l] = bid;
        ++ncl;
        miss = 0;
      } else if (++miss >= 2) {
        rejected = true;
        break;
      }
      its_ms(p, C, G.xx0[l], G.kms[l]);
    }
    // layers not reached count as missing
    const int missing_tail = G.L - 1 - lc;
    if (lc < 1 || miss + missing_tail >= 2) rejected = true;
    if (rejected || ncl < P.min_clusters) continue;
    o.ok[t] = 1;
    o.ncls[t] = ncl;
    o.chi2[t] = chi2;
    o.olayer[t] = lc;
    o.ostave[t] = kc;
    o.ox[t] = xc;
    for (int i = 0; i < 6; ++i) o.cls[t * 6 + i] = cl[i];
    for (int i = 0; i < 5; ++i) o.op[t * 5 + i] = p[i];
    for (int i = 0; i < 15; ++i) o.oc[t * 15 + i] = C[i];
    // 4. inward: from the outward state (covariance scaled up) back over
    // the track's clusters to the beam axis, no vertex point
    float q[5], Q[15], dummy = 0.0f;
    for (int i = 0; i < 5; ++i) q[i] = p[i];
    for (int i = 0; i < 15; ++i) Q[i] = C[i] * P.cov_scale_in;
    float xq = xc;
    bool iok = true;
    for (int l = lc; l >= 0 && iok; --l) {
      if (l < lc) {
        const int kf = kst[l + 1], kt = kst[l];
        const float dca = G.ca[l][kt] * G.ca[l + 1][kf] + G.sa[l][kt] * G.sa[l + 1][kf];
        const float dsa = G.sa[l][kt] * G.ca[l + 1][kf] - G.ca[l][kt] * G.sa[l + 1][kf];
        if (!rotate_state(xq, q, Q, dca, dsa, m)) { iok = false; break; }
        if (!transport(q, Q, xq, G.r[l], m)) { iok = false; break; }
        xq = G.r[l];
      }
      if (cl[l] >= 0) kf_update(q, Q, c[cl[l]].y, c[cl[l]].z, G.vy[l], G.vz[l], dummy);
      its_ms(q, Q, G.xx0[l], G.kms[l]);
    }
    if (iok && transport(q, Q, xq, 0.0f, m)) {
      o.iok[t] = 1;
      o.istave[t] = kst[0];
      for (int i = 0; i < 5; ++i) o.ip[t * 5 + i] = q[i];
      for (int i = 0; i < 15; ++i) o.ic[t * 15 + i] = Q[i];
    }
  }
  // 5. vertex: the point of least weighted squared distance to the tracks'
  // straight-line extrapolations at the beam axis, Tukey bi-square weights
  // on the normalised distance, fit_iters solves (FP64)
  std::vector<double> PX, PY, PZ, DX, DY, DZ, S2, W;
  for (int64_t t = 0; t < T; ++t) {
    if (!o.ok[t] || !o.iok[t]) continue;
    const double ca = G.ca[0][o.istave[t]], sa = G.sa[0][o.istave[t]];
    const double yy = o.ip[t * 5 + 0], zz = o.ip[t * 5 + 1], s = o.ip[t * 5 + 2], tt = o.ip[t * 5 + 3];
    const double cc = std::sqrt(1.0 - s * s), nn = std::sqrt(1.0 + tt * tt);
    PX.push_back(-(yy * sa)); PY.push_back(yy * ca); PZ.push_back(zz);
    DX.push_back((cc * ca - s * sa) / nn); DY.push_back((cc * sa + s * ca) / nn); DZ.push_back(tt / nn);
    S2.push_back(0.5 * ((double)o.ic[t * 15 + 0] + (double)o.ic[t * 15 + 5]));
    W.push_back(1.0);
  }
  const size_t nt = PX.size();
  if (nt >= 2) {
    bool good = true;
    for (int it = 0; it < P.fit_iters && good; ++it) {
      double A[6] = {0, 0, 0, 0, 0, 0}, bv[3] = {0, 0, 0};   // A: xx, xy, xz, yy, yz, zz
      for (size_t i = 0; i < nt; ++i) {
        const double f = W[i] / S2[i];
        const double d[3] = {DX[i], DY[i], DZ[i]}, Pp[3] = {PX[i], PY[i], PZ[i]};
        double M[3][3];
        for (int r = 0; r < 3; ++r)
          for (int cc2 = 0; cc2 < 3; ++cc2) M[r][cc2] = (r == cc2 ? 1.0 : 0.0) - d[r] * d[cc2];
        A[0] += f * M[0][0]; A[1] += f * M[0][1]; A[2] += f * M[0][2];
        A[3] += f * M[1][1]; A[4] += f * M[1][2]; A[5] += f * M[2][2];
        for (int r = 0; r < 3; ++r) bv[r] += f * (M[r][0] * Pp[0] + M[r][1] * Pp[1] + M[r][2] * Pp[2]);
      }
      // 3x3 symmetric solve by Cramer's rule
      const double a00 = A[0], a01 = A[1], a02 = A[2], a11 = A[3], a12 = A[4], a22 = A[5];
      const double c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22, c02 = a01 * a12 - a02 * a11;
      const double det = a00 * c00 + a01 * c01 + a02 * c02;
      if (!(std::fabs(det) > 0.0)) { good = false; break; }
      const double c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12, c22 = a00 * a11 - a01 * a01;
      o.V[0] = (c00 * bv[0] + c01 * bv[1] + c02 * bv[2]) / det;
      o.V[1] = (c01 * bv[0] + c11 * bv[1] + c12 * bv[2]) / det;
      o.V[2] = (c02 * bv[0] + c12 * bv[1] + c22 * bv[2]) / det;
      o.nused = 0;
      o.sumw = 0.0;
      for (size_t i = 0; i < nt; ++i) {
        const double u[3] = {o.V[0] - PX[i], o.V[1] - PY[i], o.V[2] - PZ[i]};
        const double pr = u[0] * DX[i] + u[1] * DY[i] + u[2] * DZ[i];
        const double e0 = u[0] - pr * DX[i], e1 = u[1] - pr * DY[i], e2 = u[2] - pr * DZ[i];
        const double D = std::sqrt((e0 * e0 + e1 * e1 + e2 * e2) / S2[i]) / (double)P.tukey_c;
        W[i] = D < 1.0 ? (1.0 - D * D) * (1.0 - D * D) : 0.0;
        if (W[i] > 0.0) ++o.nused;
        o.sumw += W[i];
      }
    }
    o.vfit_ok = good ? 1 : 0;
  }
  return o;
}

}  // namespace

// ===========================================================================
extern "C" {

void orc_default_params(orc_params* p) {
  p->win_y = 2.0f;
  p->win_z = 2.2f;
  p->inv_var_y = (float)(1.0 / (1.5 * 0.1 * 0.1));
  p->inv_var_z = (float)(1.0 / (1.5 * 0.15 * 0.15));
  p->link_cut = 16.0f;
  p->chi2_ext = 9.0f;
  p->max_gap = 8;
  p->min_seed_hits = 5;
  p->min_hits = 10;
  p->owned_num = 9;
  p->owned_den = 10;
  p->sin_max = 0.99f;
  p->sigma_y = 0.1f;
  p->sigma_z = 0.15f;
  p->sigma_vertex = 0.01f;
  p->sigma_tgl = 1e-3f;
  p->chi2_merge = 50.0f;
  p->merge_dist = 20.0f;
}

int orc_transport(int precision, const double pin[5], const double Cin[15], double x0, double x1,
                  double bz, double sin_max, double out_p[5], double out_C[15], double F[25]) {
  orc_geometry g{};
  g.bz = (float)bz;
  orc_params P;
  orc_default_params(&P);
  P.sin_max = (float)sin_max;
  if (precision == 32) {
    Model<float> m = make_model<float>(g, P);
    m.sin_max = (float)sin_max;
    float p[5], C[15], Fl[25];
    for (int i = 0; i < 5; ++i) p[i] = (float)pin[i];
    for (int i = 0; i < 15; ++i) C[i] = (float)Cin[i];
    if (!transport<float>(p, C, (float)x0, (float)x1, m, Fl)) return 0;
    for (int i = 0; i < 5; ++i) out_p[i] = p[i];
    for (int i = 0; i < 15; ++i) out_C[i] = C[i];
    if (F) for (int i = 0; i < 25; ++i) F[i] = Fl[i];
    return 1;
  }
  Model<double> m;
  m.kfac = -2.99792458e-3 * bz;
  m.sin_max = sin_max;
  double p[5], C[15], Fl[25];
  for (int i = 0; i < 5; ++i) p[i] = pin[i];
  for (int i = 0; i < 15; ++i) C[i] = Cin[i];
  if (!transport<double>(p, C, x0, x1, m, Fl)) return 0;
  for (int i = 0; i < 5; ++i) out_p[i] = p[i];
  for (int i = 0; i < 15; ++i) out_C[i] = C[i];
  if (F) for (int i = 0; i < 25; ++i) F[i] = Fl[i];
  return 1;
}

void orc_kf_update(int precision, const double pin[5], const double Cin[15], double my, double mz,
                   double vy, double vz, double out_p[5], double out_C[15], double* dchi2) {
  if (precision == 32) {
    float p[5], C[15], c2 = 0.0f;
    for (int i = 0; i < 5; ++i) p[i] = (float)pin[i];
    for (int i = 0; i < 15; ++i) C[i] = (float)Cin[i];
    kf_update<float>(p, C, (float)my, (float)mz, (float)vy, (float)vz, c2);
    for (int i = 0; i < 5; ++i) out_p[i] = p[i];
    for (int i = 0; i < 15; ++i) out_C[i] = C[i];
    *dchi2 = c2;
    return;
  }
  double p[5], C[15], c2 = 0.0;
  for (int i = 0; i < 5; ++i) p[i] = pin[i];
  for (int i = 0; i < 15; ++i) C[i] = Cin[i];
  kf_update<double>(p, C, my, mz, vy, vz, c2);
  for (int i = 0; i < 5; ++i) out_p[i] = p[i];
  for (int i = 0; i < 15; ++i) out_C[i] = C[i];
  *dchi2 = c2;
}

void orc_kf_update1(int precision, const double pin[5], const double Cin[15], int q, double m,
                    double v, double out_p[5], double out_C[15], double* dchi2) {
  if (precision == 32) {
    float p[5], C[15], c2 = 0.0f;
    for (int i = 0; i < 5; ++i) p[i] = (float)pin[i];
    for (int i = 0; i < 15; ++i) C[i] = (float)Cin[i];
    kf_update1<float>(p, C, q, (float)m, (float)v, c2);
    for (int i = 0; i < 5; ++i) out_p[i] = p[i];
    for (int i = 0; i < 15; ++i) out_C[i] = C[i];
    *dchi2 = c2;
    return;
  }
  double p[5], C[15], c2 = 0.0;
  for (int i = 0; i < 5; ++i) p[i] = pin[i];
  for (int i = 0; i < 15; ++i) C[i] = Cin[i];
  kf_update1<double>(p, C, q, m, v, c2);
  for (int i = 0; i < 5; ++i) out_p[i] = p[i];
  for (int i = 0; i < 15; ++i) out_C[i] = C[i];
  *dchi2 = c2;
}

int orc_fit_hits(int precision, const orc_geometry* g, const orc_params* P, int32_t n,
                 const double* x, const double* y, const double* z, double k0, double pout[5],
                 double Cout[15], double* chi2out) {
  if (precision == 32) {
    Model<float> m = make_model<float>(*g, *P);
    std::vector<float> hx(n), hy(n), hz(n);
    for (int i = 0; i < n; ++i) { hx[i] = (float)x[i]; hy[i] = (float)y[i]; hz[i] = (float)z[i]; }
    float p[5], C[15], c2, xc;
    if (!fit_hits<float>(m, *P, n, hx.data(), hy.data(), hz.data(), (float)k0, p, C, c2, xc)) return 0;
    for (int i = 0; i < 5; ++i) pout[i] = p[i];
    for (int i = 0; i < 15; ++i) Cout[i] = C[i];
    *chi2out = c2;
    return 1;
  }
  Model<double> m;
  m.kfac = -2.99792458e-3 * (double)g->bz;
  m.sin_max = P->sin_max;
  m.vy = (double)P->sigma_y * (double)P->sigma_y;
  m.vz = (double)P->sigma_z * (double)P->sigma_z;
  double p[5], C[15], c2, xc;
  if (!fit_hits<double>(m, *P, n, x, y, z, k0, p, C, c2, xc)) return 0;
  for (int i = 0; i < 5; ++i) pout[i] = p[i];
  for (int i = 0; i < 15; ++i) Cout[i] = C[i];
  *chi2out = c2;
  return 1;
}

int orc_track(int precision, const orc_geometry* g, const orc_params* P, int64_t n, const double* x,
              const double* y, const double* z, const int16_t* row, const uint8_t* sector,
              const uint8_t* sector_mask, orc_result** out) {
  if (precision == 32)
    *out = run_pipeline<float>(*g, *P, n, x, y, z, row, sector, sector_mask);
  else
    *out = run_pipeline<double>(*g, *P, n, x, y, z, row, sector, sector_mask);
  return 0;
}

void orc_result_free(orc_result* r) {
  if (!r) return;
  void* ptrs[] = {r->up, r->dn, r->cup, r->cdn, r->starts, r->seed_start, r->seed_nhits,
                  r->seed_key, r->seed_rlo, r->seed_rhi, r->seed_hits, r->seed_state, r->trk_seed,
                  r->trk_sector, r->trk_xref, r->trk_p, r->trk_cov, r->trk_chi2, r->trk_ndf,
                  r->hit_off, r->hit_ids};
  for (void* p : ptrs) std::free(p);
  std::free(r);
}

void orc_calib_apply(const orc_geometry* g, int64_t n, const uint8_t* sector, const double* x,
                     const double* y, const double* z, const double* theta, double* xo,
                     double* zo) {
  for (int64_t i = 0; i < n; ++i) calib_point<double>(*g, sector[i], x[i], y[i], z[i], theta, xo[i], zo[i]);
}

int orc_rotate(int precision, double x, const double p[5], const double C[15], double dalpha, double bz,
               double sin_max, double* out_x, double out_p[5], double out_C[15], double J[25]) {
  orc_geometry g{};
  g.bz = (float)bz;
  orc_params P{};
  orc_default_params(&P);
  P.sin_max = (float)sin_max;
  if (precision == 32) {
    Model<float> m = make_model<float>(g, P);
    m.sin_max = (float)sin_max;
    float xx = (float)x, q[5], Q[15], Jf[25];
    for (int i = 0; i < 5; ++i) q[i] = (float)p[i];
    for (int i = 0; i < 15; ++i) Q[i] = (float)C[i];
    if (!rotate_state(xx, q, Q, (float)std::cos(dalpha), (float)std::sin(dalpha), m, Jf)) return 0;
    *out_x = xx;
    for (int i = 0; i < 5; ++i) out_p[i] = q[i];
    for (int i = 0; i < 15; ++i) out_C[i] = Q[i];
    for (int i = 0; i < 25; ++i) J[i] = Jf[i];
    return 1;
  }
  Model<double> m = make_model<double>(g, P);
  m.sin_max = sin_max;
  double xx = x, q[5], Q[15];
  for (int i = 0; i < 5; ++i) q[i] = p[i];
  for (int i = 0; i < 15; ++i) Q[i] = C[i];
  if (!rotate_state(xx, q, Q, std::cos(dalpha), std::sin(dalpha), m, J)) return 0;
  *out_x = xx;
  for (int i = 0; i < 5; ++i) out_p[i] = q[i];
  for (int i = 0; i < 15; ++i) out_C[i] = Q[i];
  return 1;
}

int orc_merge(const orc_geometry* g, const orc_params* P, int64_t n_clusters, const double* x,
              const double* y, const double* z, const int16_t* row, int64_t n_seg,
              const int32_t* seg_sector, const double* seg_xref, const double* seg_p,
              const double* seg_cov, const double* seg_chi2, const int64_t* seg_hit_off,
              const int64_t* seg_hit_ids, const int32_t* seg_slice, int32_t* link, int32_t* best_in,
              double* chi_in, double* chi_in2, int32_t* best_out, double* chi_out, double* chi_out2,
              orc_result** out) {
  (void)n_clusters;
  MergeOut o = merge_segments(*g, *P, x, y, z, row, n_seg, seg_sector, seg_xref, seg_p, seg_cov, seg_chi2,
                              seg_hit_off, seg_hit_ids, seg_slice);
  for (int64_t i = 0; i < n_seg; ++i) {
    link[i] = o.link[i]; best_in[i] = o.best_in[i]; best_out[i] = o.best_out[i];
    chi_in[i] = o.chi_in[i]; chi_in2[i] = o.chi_in2[i]; chi_out[i] = o.chi_out[i]; chi_out2[i] = o.chi_out2[i];
  }
  orc_result* r = (orc_result*)std::calloc(1, sizeof(orc_result));
  const int64_t nt = (int64_t)o.head.size();
  r->n_tracks = nt;
  auto c64 = [](const std::vector<int64_t>& v) {
    int64_t* q = (int64_t*)std::malloc(sizeof(int64_t) * std::max<size_t>(v.size(), 1));
    std::memcpy(q, v.data(), sizeof(int64_t) * v.size());
    return q;
  };
  auto cd = [](const std::vector<double>& v) {
    double* q = (double*)std::malloc(sizeof(double) * std::max<size_t>(v.size(), 1));
    std::memcpy(q, v.data(), sizeof(double) * v.size());
    return q;
  };
  auto c32 = [](const std::vector<int32_t>& v) {
    int32_t* q = (int32_t*)std::malloc(sizeof(int32_t) * std::max<size_t>(v.size(), 1));
    std::memcpy(q, v.data(), sizeof(int32_t) * v.size());
    return q;
  };
  r->trk_seed = c64(o.head);
  r->trk_sector = c32(o.sector);
  r->trk_xref = cd(o.xref);
  r->trk_p = cd(o.p);
  r->trk_cov = cd(o.cov);
  r->trk_chi2 = cd(o.chi2);
  r->trk_ndf = c32(o.ndf);
  r->hit_off = c64(o.hit_off);
  r->hit_ids = c64(o.hit_ids);
  *out = r;
  return 0;
}

void orc_calib_apply32(const orc_geometry* g, int64_t n, const uint8_t* sector, const float* x,
                       const float* y, const float* z, const float* theta, float* xo, float* zo) {
  for (int64_t i = 0; i < n; ++i) calib_point32(*g, sector[i], x[i], y[i], z[i], theta, xo[i], zo[i]);
}

int orc_calib_chi2(const orc_geometry* g, const orc_params* P, int64_t n_clusters, const double* x,
                   const double* y, const double* z, const uint8_t* sector, int64_t n_tracks,
                   const int64_t* hit_off, const int64_t* hit_ids, const double* k0,
                   const double* ext_tgl, const uint8_t* use_vertex, const double* theta,
                   double* chi2_out, int64_t* ndf_out, double* trk_chi2, double* grad) {
  (void)n_clusters;
  const int npar = 2 * g->n_sectors + 64 * g->n_sectors;
  if (grad) for (int i = 0; i < npar; ++i) grad[i] = 0.0;
  double total = 0.0;
  int64_t ndf = 0;
  Tape tape;
  for (int64_t t = 0; t < n_tracks; ++t) {
    int64_t b = hit_off[t], e = hit_off[t + 1];
    int nh = (int)(e - b);
    bool uv = use_vertex && use_vertex[t];
    bool ue = uv && ext_tgl != nullptr;
    double c2v = 0.0;
    int ok;
    if (!grad) {
      Model<double> m;
      m.kfac = -2.99792458e-3 * (double)g->bz;
      m.sin_max = P->sin_max;
      m.vy = (double)P->sigma_y * (double)P->sigma_y;
      m.vz = (double)P->sigma_z * (double)P->sigma_z;
      std::vector<double> hx(nh), hy(nh), hz(nh);
      for (int j = 0; j < nh; ++j) {                 // outermost first
        int64_t c = hit_ids[e - 1 - j];
        calib_point<double>(*g, sector[c], x[c], y[c], z[c], theta, hx[j], hz[j]);
        hy[j] = y[c];
      }
      double c2 = 0.0;
      ok = track_objective<double>(*g, *P, m, nh, hx.data(), hy.data(), hz.data(), k0[t], uv, ue,
                                   ue ? ext_tgl[t] : 0.0, c2);
      c2v = c2;
    } else {
      g_tape = &tape;
      tape.clear();
      int s = sector[hit_ids[b]];
      std::vector<Var> th(npar);
      for (int i = 0; i < npar; ++i) th[i] = Var(theta[i]);
      std::vector<int> leaves;
      auto mkleaf = [&](int i) { th[i] = Var::leaf(theta[i]); leaves.push_back(i); };
      mkleaf(s);
      mkleaf(g->n_sectors + s);
      for (int k = 0; k < 64; ++k) mkleaf(2 * g->n_sectors + s * 64 + k);
      Model<Var> m;
      m.kfac = Var(-2.99792458e-3 * (double)g->bz);
      m.sin_max = Var((double)P->sin_max);
      m.vy = Var((double)P->sigma_y * (double)P->sigma_y);
      m.vz = Var((double)P->sigma_z * (double)P->sigma_z);
      std::vector<Var> hx(nh), hy(nh), hz(nh);
      for (int j = 0; j < nh; ++j) {
        int64_t c = hit_ids[e - 1 - j];
        calib_point<Var>(*g, sector[c], x[c], y[c], z[c], th.data(), hx[j], hz[j]);
        hy[j] = Var(y[c]);
      }
      Var c2(0.0);
      ok = track_objective<Var>(*g, *P, m, nh, hx.data(), hy.data(), hz.data(), Var(k0[t]), uv, ue,
                                Var(ue ? ext_tgl[t] : 0.0), c2);
      c2v = c2.v;
      if (ok) {
        tape.backprop(c2.i);
        for (int i : leaves) grad[i] += tape.adj[th[i].i];
      }
      g_tape = nullptr;
    }
    if (!ok) c2v = 0.0;
    if (trk_chi2) trk_chi2[t] = c2v;
    if (ok) {
      total += c2v;
      ndf += 2 * nh - 5 + (ok == 2 ? 2 + (ue ? 1 : 0) : 0);
    }
  }
  *chi2_out = total;
  *ndf_out = ndf;
  return 0;
}


void orc_its_default_params(orc_its_params* p) {
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

int orc_its(const orc_its_geometry* g, const orc_its_params* P, int64_t n, const float* x, const float* y,
            const float* z, const int8_t* layer, const int16_t* stave, int64_t* hist, int64_t* meta, float* vz,
            int32_t* tl0, int32_t* tl1, int32_t* ok, int32_t* cls, int32_t* ncls, float* chi2,
            int32_t* olayer, int32_t* ostave, float* ox, float* op, float* oc, int32_t* iok, int32_t* istave,
            float* ip, float* ic, double* vfit, int32_t* vfit_n) {
  ItsOut o = its_run(*g, *P, n, x, y, z, layer, stave);
  for (size_t b = 0; b < o.hist.size(); ++b) hist[b] = o.hist[b];
  meta[0] = o.npairs; meta[1] = o.peak; meta[2] = o.qn; meta[3] = o.qsum; meta[4] = (int64_t)o.tl0.size();
  meta[5] = o.vz_ok; meta[6] = o.vfit_ok;
  *vz = o.vz;
  const size_t T = o.tl0.size();
  for (size_t t = 0; t < T; ++t) {
    tl0[t] = o.tl0[t]; tl1[t] = o.tl1[t]; ok[t] = o.ok[t]; ncls[t] = o.ncls[t]; chi2[t] = o.chi2[t];
    olayer[t] = o.olayer[t]; ostave[t] = o.ostave[t]; ox[t] = o.ox[t]; iok[t] = o.iok[t]; istave[t] = o.istave[t];
    for (int i = 0; i < 6; ++i) cls[t * 6 + i] = o.cls[t * 6 + i];
    for (int i = 0; i < 5; ++i) { op[t * 5 + i] = o.op[t * 5 + i]; ip[t * 5 + i] = o.ip[t * 5 + i]; }
    for (int i = 0; i < 15; ++i) { oc[t * 15 + i] = o.oc[t * 15 + i]; ic[t * 15 + i] = o.ic[t * 15 + i]; }
  }
  vfit[0] = o.V[0]; vfit[1] = o.V[1]; vfit[2] = o.V[2]; vfit[3] = o.sumw;
  *vfit_n = o.nused;
  return 0;
}

int orc_its_ms(const orc_its_geometry* g, int layer, const float p[5], float C[15]) {
  orc_its_params P;
  orc_its_default_params(&P);
  const ItsGeo G = its_geo(*g, P);
  float q[5];
  for (int i = 0; i < 5; ++i) q[i] = p[i];
  its_ms(q, C, G.xx0[layer], G.kms[layer]);
  return 0;
}

}  // extern "C"
