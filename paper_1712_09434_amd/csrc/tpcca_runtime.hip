// tpcca_runtime.hip -- host side of libtpcca: the C ABI of include/tpcca.h.
//
// One context per geometry and stream user.  The context owns a single
// device arena (grown on demand, never shrunk) that holds every
// intermediate array of the tracking path, plus staging for host-memory
// inputs and outputs.  Errors are reported by return code and message;
// nothing throws or aborts across the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "calib_internal.hpp"
#include "internal.hpp"
#include "merge_internal.hpp"
#include "timeframe_internal.hpp"

using namespace tpcca;

namespace {

// Scratch of tpcca_refit_grad_noalloc, which allocates nothing: a file-scope
// device array.  Each GPU the library runs on holds its own copy, at its own
// address, until the process ends.  In host code `scratch` names only a
// host-side stand-in: every host use goes through the device address that
// hipGetSymbolAddress returned for the GPU (scratch_address).
constexpr size_t kNoAllocScratchBytes = (size_t)TPCCA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `dev`, looked up once per device with
// that device current (the caller has made it current).
hipError_t scratch_address(int dev, char** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

struct tpcca_ctx {
  int device = 0;
  int S = 0, R = 0;
  float tan_a = 0.f, z_max = 0.f, bz = 0.f;
  float* row_x_d = nullptr;
  float row_x_first = 0.f, row_x_last = 0.f;   // the map's radial range
  tpcca_params P{};
  std::string err;
  // arena
  char* arena = nullptr;
  size_t arena_bytes = 0;
  // staging for host-memory inputs / outputs
  char* stage = nullptr;
  size_t stage_bytes = 0;
  // pinned host memory for the per-call tables and the result words, so
  // their copies are asynchronous
  char* hpin = nullptr;
  size_t hpin_bytes = 0;
  bool hpin_busy = false;         // copies from/to it may still be queued (a call failed midway)
  hipStream_t hpin_stream = nullptr;
  Ws w{};
  // last tracking call (debug tap)
  bool last_ok = false;
  int64_t last_nseeds = 0;
  // refit_grad scratch
  char* gscratch = nullptr;
  size_t gscratch_bytes = 0;
  // sector merger scratch
  char* mscratch = nullptr;
  size_t mscratch_bytes = 0;
  // time-frame workspace (slices, per-slice tracks, the segment set)
  char* tfscratch = nullptr;
  size_t tfscratch_bytes = 0;
  // installed calibration of the tracking input (device, 66 S floats), or off
  float* cal_d = nullptr;
  bool cal_on = false;
  // device address of the static scratch of tpcca_refit_grad_noalloc on
  // this context's GPU (null, with the reason, if the lookup failed)
  char* noalloc_scratch = nullptr;
  std::string noalloc_err;
  // tuning
  tpcca_tuning tune{160, 0, 0};
  // captured tracking graph and the workspace shape it was captured for
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  struct GraphKey {
    int64_t N = -1;
    int E = 0;
    char* arena = nullptr;
    hipStream_t st = nullptr;
    tpcca_params P{};
    int tracklet_grid = 0;
    int taps = 0;
    const float* cal = nullptr;
  } gkey;
  // phase timing
  bool timing = false;
  PhaseEvents pe{};
  double phase_ms[PH_N] = {};
  int64_t timed_calls = 0;
};

namespace {

int fail(tpcca_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(tpcca_ctx* c, hipError_t e, const char* where) {
  return fail(c, TPCCA_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

Model make_model(float bz, const tpcca_params& P) {
  Model m;
  m.kfac = -((float)2.99792458e-3) * bz;
  m.sin_max = P.sin_max;
  m.vy = P.sigma_y * P.sigma_y;
  m.vz = P.sigma_z * P.sigma_z;
  return m;
}

size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

// The geometry of the calibration correction of a context.
CalGeo cal_geo(const tpcca_ctx* c) {
  return CalGeo{c->S, c->z_max, c->row_x_first, c->row_x_last - c->row_x_first, c->tan_a};
}


struct Layout {
  size_t off = 0;
  template <class T> size_t take(int64_t n) { size_t o = off; off += al(sizeof(T) * (size_t)std::max<int64_t>(n, 1)); return o; }
};

// Lay out every workspace array for N clusters in E events.  With base ==
// nullptr only the size is computed.
size_t layout_ws(Ws& w, char* base, int64_t N, int E, int S, int R, int min_seed) {
  Layout L;
  w.E = E; w.S = S; w.R = R; w.N = N;
  w.Rh = (R + 7) & ~7;
  w.RU = (int64_t)E * S * R;
  w.seed_cap = N / std::max(min_seed, 1) + 1;
  w.nb = std::max<int64_t>(1, (N + 255) / 256);
  const int64_t RU = w.RU, SC = w.seed_cap;
  const int64_t scan_n = std::max<int64_t>(std::max<int64_t>(RU, w.nb), SC) + 1;
  // flags, then the per-event results: one download after the pipeline
  // (the host staging buffer repeats this placement)
  size_t o_flags = L.take<uint32_t>(F_COUNT);
  size_t o_res = L.take<int64_t>((int64_t)E * 4);
  size_t o_ruc = L.take<uint32_t>(RU), o_ruo = L.take<uint32_t>(RU + 1);
  size_t o_cc = L.take<uint32_t>(RU), o_cb = L.take<uint32_t>(RU + 1);
  size_t o_grid = L.take<GridParams>(RU);
  size_t o_lr = L.take<uint32_t>(RU), o_ll = L.take<uint32_t>(RU), o_lb = L.take<uint32_t>(RU);
  size_t o_tmp = L.take<float4>(N);
  size_t o_cx = L.take<float>(N), o_cy = L.take<float>(N), o_cz = L.take<float>(N);
  size_t o_cid = L.take<uint32_t>(N), o_cru = L.take<uint32_t>(N);
  size_t o_gbuf = L.take<float4>(N), o_grec = L.take<SearchRec>(N);
  size_t o_coff = L.take<uint16_t>(kCellsPerCluster * N + 2 * RU + 1);
  size_t o_up = L.take<int32_t>(N), o_dn = L.take<int32_t>(N), o_cup = L.take<int32_t>(N), o_cdn = L.take<int32_t>(N);
  size_t o_cpk = L.take<float4>(N);
  size_t o_flag = L.take<uint8_t>(N);
  size_t o_bs = L.take<uint32_t>(w.nb + 1), o_bq = L.take<uint32_t>(w.nb + 1);
  size_t o_scan = L.take<uint32_t>(2 * (scan_n / 1024 + 2) + 4);
  size_t o_starts = L.take<uint32_t>(N / 2 + 1), o_seeds = L.take<uint32_t>(SC);
  size_t o_seo = L.take<uint32_t>(E + 1), o_steo = L.take<uint32_t>(E + 1);
  size_t o_ssu = L.take<uint32_t>((int64_t)E * S + 1);
  size_t o_tln = L.take<int32_t>(SC), o_tlr = L.take<int32_t>(SC);
  size_t o_tlk = L.take<uint64_t>(SC), o_tls = L.take<float>(SC * kTl), o_tlh = L.take<int32_t>(SC * ((R + 7) & ~7));
  size_t o_own = L.take<uint64_t>(N), o_omask = L.take<uint8_t>(SC * ((R + 7) / 8));
  size_t o_tlo = L.take<int32_t>(SC * R);
  size_t o_acf = L.take<uint32_t>(SC + 1), o_aco = L.take<uint32_t>(SC + 1);
  size_t o_acl = L.take<uint32_t>(SC), o_occ = L.take<uint32_t>(SC + 1);
  size_t o_rf = L.take<float>(SC * kRf);
  size_t o_tf = L.take<uint32_t>(SC + 1), o_hc = L.take<uint32_t>(SC + 1);
  // event, output and chunk tables back to back: one upload per call (the
  // host staging buffer repeats this placement)
  size_t o_ev = L.take<EventIn>(E), o_out = L.take<EventOut>(E);
  size_t o_chunk = L.take<ChunkIn>(chunk_cap(N, E));
  if (base) {
    w.flags = (uint32_t*)(base + o_flags);
    w.ru_count = (uint32_t*)(base + o_ruc); w.ru_off = (uint32_t*)(base + o_ruo);
    w.cell_cap = (uint32_t*)(base + o_cc); w.cell_base = (uint32_t*)(base + o_cb);
    w.grid = (GridParams*)(base + o_grid);
    w.ru_rows = (uint32_t*)(base + o_lr); w.ru_links = (uint32_t*)(base + o_ll);
    w.ru_big = (uint32_t*)(base + o_lb);
    w.tmp4 = (float4*)(base + o_tmp);
    w.cx = (float*)(base + o_cx); w.cy = (float*)(base + o_cy); w.cz = (float*)(base + o_cz);
    w.cid = (uint32_t*)(base + o_cid); w.cru = (uint32_t*)(base + o_cru);
    w.gbuf = (float4*)(base + o_gbuf); w.grec = (SearchRec*)(base + o_grec); w.cell_off = (uint16_t*)(base + o_coff);
    w.up = (int32_t*)(base + o_up); w.dn = (int32_t*)(base + o_dn);
    w.cup = (int32_t*)(base + o_cup); w.cdn = (int32_t*)(base + o_cdn);
    w.cpk = (float4*)(base + o_cpk);
    w.flag = (uint8_t*)(base + o_flag);
    w.blk_start = (uint32_t*)(base + o_bs); w.blk_seed = (uint32_t*)(base + o_bq);
    w.scan_tmp = (uint32_t*)(base + o_scan);
    w.starts = (uint32_t*)(base + o_starts); w.seeds = (uint32_t*)(base + o_seeds);
    w.seed_ev_off = (uint32_t*)(base + o_seo); w.start_ev_off = (uint32_t*)(base + o_steo);
    w.seed_su_off = (uint32_t*)(base + o_ssu);
    w.tl_nhits = (int32_t*)(base + o_tln); w.tl_range = (int32_t*)(base + o_tlr);
    w.tl_key = (uint64_t*)(base + o_tlk); w.tl_state = (float*)(base + o_tls);
    w.tl_hits = (int32_t*)(base + o_tlh);
    w.owner = (uint64_t*)(base + o_own); w.own_mask = (uint8_t*)(base + o_omask);
    w.tl_own = (int32_t*)(base + o_tlo);
    w.acc_flag = (uint32_t*)(base + o_acf); w.acc_off = (uint32_t*)(base + o_aco);
    w.acc_list = (uint32_t*)(base + o_acl); w.own_cnt = (uint32_t*)(base + o_occ);
    w.rf = (float*)(base + o_rf);
    w.trk_flag = (uint32_t*)(base + o_tf); w.hit_cnt = (uint32_t*)(base + o_hc);
    w.ev_res = (int64_t*)(base + o_res);
    w.ev = (const EventIn*)(base + o_ev);
    w.chunk = (const ChunkIn*)(base + o_chunk);
    w.out = (const EventOut*)(base + o_out);
  }
  return L.off;
}

int ensure_arena(tpcca_ctx* c, size_t need) {
  if (need <= c->arena_bytes) return TPCCA_OK;
  if (c->arena) { (void)hipFree(c->arena); c->arena = nullptr; c->arena_bytes = 0; }
  size_t want = need + need / 4;
  hipError_t e = hipMalloc((void**)&c->arena, want);
  if (e != hipSuccess) {
    c->arena = nullptr;
    (void)hipGetLastError();
    return fail(c, TPCCA_E_NOMEM, "device workspace allocation of " + std::to_string(want) + " bytes failed");
  }
  c->arena_bytes = want;
  return TPCCA_OK;
}

int ensure_pinned(tpcca_ctx* c, size_t need) {
  if (need <= c->hpin_bytes) return TPCCA_OK;
  if (c->hpin) { (void)hipHostFree(c->hpin); c->hpin = nullptr; c->hpin_bytes = 0; }
  const size_t want = need + need / 2;
  hipError_t e = hipHostMalloc((void**)&c->hpin, want, hipHostMallocDefault);
  if (e != hipSuccess) {
    c->hpin = nullptr;
    (void)hipGetLastError();
    return fail(c, TPCCA_E_NOMEM, "pinned host allocation failed");
  }
  c->hpin_bytes = want;
  return TPCCA_OK;
}

int ensure_stage(tpcca_ctx* c, size_t need) {
  if (need <= c->stage_bytes) return TPCCA_OK;
  if (c->stage) { (void)hipFree(c->stage); c->stage = nullptr; c->stage_bytes = 0; }
  hipError_t e = hipMalloc((void**)&c->stage, need);
  if (e != hipSuccess) {
    c->stage = nullptr;
    (void)hipGetLastError();
    return fail(c, TPCCA_E_NOMEM, "staging allocation failed");
  }
  c->stage_bytes = need;
  return TPCCA_OK;
}

int check_params(const tpcca_params* p) {
  if (!(p->win_y > 0 && p->win_z > 0 && p->inv_var_y > 0 && p->inv_var_z > 0 && p->link_cut > 0 &&
        p->chi2_ext > 0 && p->max_gap >= 0 && p->min_seed_hits >= 3 && p->min_hits >= 3 &&
        p->owned_num >= 0 && p->owned_den > 0 && p->sin_max > 0 && p->sin_max < 1 &&
        p->sigma_y > 0 && p->sigma_z > 0 && p->sigma_vertex > 0 && p->sigma_tgl > 0 &&
        p->chi2_merge > 0 && p->merge_dist > 0))
    return TPCCA_E_INVALID;
  return TPCCA_OK;
}

struct HostOut {   // where host-memory outputs of an event are staged on the device
  bool host = false;
  int64_t tcap = 0, hcap = 0, n = 0;
  size_t o_sector, o_xref, o_p, o_cov, o_chi2, o_ndf, o_kp, o_hoff, o_hid, o_up, o_dn, o_cup, o_cdn, o_start;
};

}  // namespace

extern "C" {

void tpcca_default_params(tpcca_params* p) {
  if (!p) return;
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

int tpcca_create(const tpcca_geometry* g, const tpcca_field* f, tpcca_ctx** out) {
  if (!out) return TPCCA_E_INVALID;
  *out = nullptr;
  if (!g || !f || !g->row_x) return TPCCA_E_INVALID;
  if (g->n_sectors <= 0 || (g->n_sectors & 1) || g->n_sectors > kMaxSectors || g->n_rows < 3 || g->n_rows > 255)
    return TPCCA_E_INVALID;
  for (int r = 0; r < g->n_rows; ++r) {
    if (!std::isfinite(g->row_x[r]) || g->row_x[r] <= 0.0f) return TPCCA_E_INVALID;
    if (r > 0 && !(g->row_x[r] > g->row_x[r - 1])) return TPCCA_E_INVALID;
  }
  if (!(g->tan_half_angle > 0 && g->z_max > 0 && std::isfinite(f->bz_tesla))) return TPCCA_E_INVALID;
  tpcca_ctx* c = new (std::nothrow) tpcca_ctx();
  if (!c) return TPCCA_E_NOMEM;
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) { (void)hipGetLastError(); delete c; return TPCCA_E_DEVICE; }
  c->S = g->n_sectors; c->R = g->n_rows;
  c->tan_a = g->tan_half_angle; c->z_max = g->z_max; c->bz = f->bz_tesla;
  tpcca_default_params(&c->P);
  c->row_x_first = g->row_x[0];
  c->row_x_last = g->row_x[g->n_rows - 1];
  e = hipMalloc((void**)&c->row_x_d, sizeof(float) * g->n_rows);
  if (e == hipSuccess) e = hipMemcpy(c->row_x_d, g->row_x, sizeof(float) * g->n_rows, hipMemcpyHostToDevice);
  if (e != hipSuccess) { (void)hipGetLastError(); if (c->row_x_d) (void)hipFree(c->row_x_d); delete c; return TPCCA_E_DEVICE; }
  // the static scratch of the allocation-free gradient: its address on this
  // device (the device is current); only that entry point needs it
  e = scratch_address(c->device, &c->noalloc_scratch);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    c->noalloc_scratch = nullptr;
    c->noalloc_err = hipGetErrorString(e);
  }
  *out = c;
  return TPCCA_OK;
}

int tpcca_set_params(tpcca_ctx* c, const tpcca_params* p) {
  if (!c || !p) return TPCCA_E_INVALID;
  if (check_params(p) != TPCCA_OK) return fail(c, TPCCA_E_INVALID, "invalid parameter values");
  c->P = *p;
  return TPCCA_OK;
}

int tpcca_get_params(const tpcca_ctx* c, tpcca_params* p) {
  if (!c || !p) return TPCCA_E_INVALID;
  *p = c->P;
  return TPCCA_OK;
}

int tpcca_set_calib(tpcca_ctx* c, const tpcca_calib* cal) {
  if (!c) return TPCCA_E_INVALID;
  if (!cal) { c->cal_on = false; return TPCCA_OK; }
  if (!cal->drift_scale || !cal->time_offset || !cal->map) return fail(c, TPCCA_E_INVALID, "null calibration arrays");
  if (cal->mem != TPCCA_MEM_HOST && cal->mem != TPCCA_MEM_DEVICE) return fail(c, TPCCA_E_INVALID, "bad mem kind");
  hipError_t he = hipSetDevice(c->device);
  if (he != hipSuccess) return hip_fail(c, he, "hipSetDevice");
  const int S = c->S;
  std::vector<float> th((size_t)S * 66);
  const hipMemcpyKind k = cal->mem == TPCCA_MEM_HOST ? hipMemcpyHostToHost : hipMemcpyDeviceToHost;
  he = hipMemcpy(th.data(), cal->drift_scale, sizeof(float) * S, k);
  if (he == hipSuccess) he = hipMemcpy(th.data() + S, cal->time_offset, sizeof(float) * S, k);
  if (he == hipSuccess) he = hipMemcpy(th.data() + 2 * S, cal->map, sizeof(float) * 64 * S, k);
  if (he != hipSuccess) return hip_fail(c, he, "calibration read");
  for (float v : th)
    if (!std::isfinite(v)) return fail(c, TPCCA_E_INVALID, "non-finite calibration value");
  if (!c->cal_d) {
    he = hipMalloc((void**)&c->cal_d, sizeof(float) * th.size());
    if (he != hipSuccess) { c->cal_d = nullptr; (void)hipGetLastError(); return fail(c, TPCCA_E_NOMEM, "calibration buffer allocation failed"); }
  }
  he = hipMemcpy(c->cal_d, th.data(), sizeof(float) * th.size(), hipMemcpyHostToDevice);
  if (he != hipSuccess) return hip_fail(c, he, "calibration upload");
  c->cal_on = true;
  return TPCCA_OK;
}

const char* tpcca_last_error(const tpcca_ctx* c) { return c ? c->err.c_str() : "null context"; }

int tpcca_set_phase_timing(tpcca_ctx* c, int on) {
  if (!c) return TPCCA_E_INVALID;
  if (on && !c->pe.ev[0]) {
    // timing only (read after the call's stream synchronisation): no
    // system-scope fence, so recording an event between two kernels does not
    // write back and invalidate the caches under the next one
    for (int i = 0; i <= PH_N; ++i) {
      hipError_t e = hipEventCreateWithFlags(&c->pe.ev[i], hipEventDisableSystemFence);
      if (e != hipSuccess) return hip_fail(c, e, "hipEventCreate");
    }
  }
  c->timing = on != 0;
  for (int i = 0; i < PH_N; ++i) c->phase_ms[i] = 0.0;
  c->timed_calls = 0;
  return TPCCA_OK;
}

int tpcca_phase_times(const tpcca_ctx* c, int32_t cap, const char** names, double* total_ms,
                      int64_t* calls) {
  if (!c) return TPCCA_E_INVALID;
  if (calls) *calls = c->timed_calls;
  for (int i = 0; i < PH_N && i < cap; ++i) {
    if (names) names[i] = kPhaseNames[i];
    if (total_ms) total_ms[i] = c->phase_ms[i];
  }
  return PH_N;
}

void tpcca_destroy(tpcca_ctx* c) {
  if (!c) return;
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  for (int i = 0; i <= PH_N; ++i)
    if (c->pe.ev[i]) (void)hipEventDestroy(c->pe.ev[i]);
  if (c->arena) (void)hipFree(c->arena);
  if (c->stage) (void)hipFree(c->stage);
  if (c->hpin) (void)hipHostFree(c->hpin);
  if (c->gscratch) (void)hipFree(c->gscratch);
  if (c->cal_d) (void)hipFree(c->cal_d);
  if (c->mscratch) (void)hipFree(c->mscratch);
  if (c->tfscratch) (void)hipFree(c->tfscratch);
  if (c->row_x_d) (void)hipFree(c->row_x_d);
  delete c;
}

int tpcca_track_batch(tpcca_ctx* c, int32_t E, const tpcca_clusters* ev, tpcca_tracks* out) {
  if (!c) return TPCCA_E_INVALID;
  c->last_ok = false;
  if (E <= 0 || !ev || !out) return fail(c, TPCCA_E_INVALID, "need n_events > 0, events and outputs");
  if (check_params(&c->P) != TPCCA_OK) return fail(c, TPCCA_E_INVALID, "invalid parameters");
  hipStream_t st = (hipStream_t)ev[0].stream;
  int64_t N = 0;
  for (int e = 0; e < E; ++e) {
    const tpcca_clusters& k = ev[e];
    if (k.n < 0 || (k.n > 0 && (!k.x || !k.y || !k.z || !k.row || !k.sector)))
      return fail(c, TPCCA_E_INVALID, "event " + std::to_string(e) + ": null array or negative size");
    if (k.mem != TPCCA_MEM_HOST && k.mem != TPCCA_MEM_DEVICE) return fail(c, TPCCA_E_INVALID, "bad mem kind");
    if (k.stream != ev[0].stream) return fail(c, TPCCA_E_INVALID, "all events must share one stream");
    N += k.n;
    const tpcca_tracks& o = out[e];
    if (o.mem != TPCCA_MEM_HOST && o.mem != TPCCA_MEM_DEVICE) return fail(c, TPCCA_E_INVALID, "bad output mem kind");
    if (o.cap_tracks < 0 || o.cap_hits < 0 || !o.hit_off)
      return fail(c, TPCCA_E_INVALID, "event " + std::to_string(e) + ": negative capacity or null hit_off");
    if (o.cap_tracks > 0 && (!o.sector || !o.x_ref || !o.p || !o.cov || !o.chi2 || !o.ndf))
      return fail(c, TPCCA_E_INVALID, "event " + std::to_string(e) + ": null track array");
    if (o.cap_hits > 0 && !o.hit_id) return fail(c, TPCCA_E_INVALID, "null hit_id");
  }
  if (N >= (int64_t)1 << 31) return fail(c, TPCCA_E_INVALID, "more than 2^31 clusters in one call");
  hipError_t he = hipSetDevice(c->device);
  if (he != hipSuccess) return hip_fail(c, he, "hipSetDevice");

  Ws w{};
  const size_t need = layout_ws(w, nullptr, N, E, c->S, c->R, c->P.min_seed_hits);
  int rc = ensure_arena(c, need);
  if (rc) return rc;
  layout_ws(w, c->arena, N, E, c->S, c->R, c->P.min_seed_hits);
  w.row_x = c->row_x_d;
  w.m = make_model(c->bz, c->P);
  w.P = c->P;
  w.tan_a = c->tan_a;
  w.z_max = c->z_max;
  w.tracklet_grid = c->tune.tracklet_grid;
  w.cal = c->cal_on ? c->cal_d : nullptr;
  w.cal_geo = cal_geo(c);
  w.taps = 0;
  for (int e = 0; e < E; ++e)
    if (out[e].dbg_up || out[e].dbg_dn || out[e].dbg_cup || out[e].dbg_cdn || out[e].dbg_start) w.taps = 1;

  // staging: host inputs and host outputs
  std::vector<HostOut> ho(E);
  size_t soff = 0;
  auto take = [&](size_t b) { size_t o = soff; soff += al(std::max<size_t>(b, 1)); return o; };
  std::vector<size_t> in_off(E, 0);
  for (int e = 0; e < E; ++e)
    if (ev[e].mem == TPCCA_MEM_HOST && ev[e].n > 0) in_off[e] = take((size_t)ev[e].n * 15);
  for (int e = 0; e < E; ++e) {
    const tpcca_tracks& o = out[e];
    HostOut& h = ho[e];
    if (o.mem != TPCCA_MEM_HOST) continue;
    h.host = true;
    h.n = ev[e].n;
    h.tcap = std::min<int64_t>(o.cap_tracks, ev[e].n / std::max(c->P.min_seed_hits, 1) + 1);
    h.hcap = std::min<int64_t>(o.cap_hits, ev[e].n);
    h.o_sector = take(h.tcap); h.o_xref = take(4 * h.tcap); h.o_p = take(20 * h.tcap);
    h.o_cov = take(60 * h.tcap); h.o_chi2 = take(4 * h.tcap); h.o_ndf = take(4 * h.tcap);
    h.o_kp = take(4 * h.tcap); h.o_hoff = take(4 * (h.tcap + 1)); h.o_hid = take(4 * h.hcap);
    h.o_up = take(4 * h.n); h.o_dn = take(4 * h.n); h.o_cup = take(4 * h.n); h.o_cdn = take(4 * h.n);
    h.o_start = take(4 * h.n);
  }
  if (soff > 0) { rc = ensure_stage(c, soff); if (rc) return rc; }
  char* sb = c->stage;

  // per-call tables and result words in pinned host memory (a call that
  // failed after queueing copies may have left them in flight)
  if (c->hpin_busy) {
    (void)hipStreamSynchronize(c->hpin_stream);
    (void)hipGetLastError();
    c->hpin_busy = false;
  }
  const size_t nchunk = (size_t)chunk_cap(N, E);
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t p_ein = 0, p_eout = al(p_ein + sizeof(EventIn) * E), p_chunk = al(p_eout + sizeof(EventOut) * E);
  const size_t p_flags = al(p_chunk + sizeof(ChunkIn) * nchunk), p_res = al(p_flags + sizeof(uint32_t) * F_COUNT);
  rc = ensure_pinned(c, p_res + sizeof(int64_t) * 4 * E);
  if (rc) return rc;
  EventIn* ein = (EventIn*)(c->hpin + p_ein);
  EventOut* eout = (EventOut*)(c->hpin + p_eout);
  ChunkIn* chunks = (ChunkIn*)(c->hpin + p_chunk);
  uint32_t* flags = (uint32_t*)(c->hpin + p_flags);
  int64_t* res = (int64_t*)(c->hpin + p_res);
  int64_t base = 0;
  for (int e = 0; e < E; ++e) {
    const tpcca_clusters& k = ev[e];
    EventIn& I = ein[e];
    I.base = base; I.n = k.n;
    if (k.mem == TPCCA_MEM_HOST && k.n > 0) {
      char* p = sb + in_off[e];
      he = hipMemcpyAsync(p, k.x, 4 * k.n, hipMemcpyHostToDevice, st);
      if (he == hipSuccess) he = hipMemcpyAsync(p + 4 * k.n, k.y, 4 * k.n, hipMemcpyHostToDevice, st);
      if (he == hipSuccess) he = hipMemcpyAsync(p + 8 * k.n, k.z, 4 * k.n, hipMemcpyHostToDevice, st);
      if (he == hipSuccess) he = hipMemcpyAsync(p + 12 * k.n, k.row, 2 * k.n, hipMemcpyHostToDevice, st);
      if (he == hipSuccess) he = hipMemcpyAsync(p + 14 * k.n, k.sector, k.n, hipMemcpyHostToDevice, st);
      if (he != hipSuccess) return hip_fail(c, he, "input upload");
      I.x = (const float*)p; I.y = (const float*)(p + 4 * k.n); I.z = (const float*)(p + 8 * k.n);
      I.row = (const int16_t*)(p + 12 * k.n); I.sector = (const uint8_t*)(p + 14 * k.n);
    } else {
      I.x = k.x; I.y = k.y; I.z = k.z; I.row = k.row; I.sector = k.sector;
    }
    base += k.n;
    const tpcca_tracks& o = out[e];
    EventOut& O = eout[e];
    O.cap_tracks = o.cap_tracks; O.cap_hits = o.cap_hits;
    if (ho[e].host) {
      const HostOut& h = ho[e];
      O.cap_tracks = h.tcap; O.cap_hits = h.hcap;
      O.sector = (uint8_t*)(sb + h.o_sector); O.x_ref = (float*)(sb + h.o_xref); O.p = (float*)(sb + h.o_p);
      O.cov = (float*)(sb + h.o_cov); O.chi2 = (float*)(sb + h.o_chi2); O.ndf = (int32_t*)(sb + h.o_ndf);
      O.k_prior = o.k_prior ? (float*)(sb + h.o_kp) : nullptr;
      O.hit_off = (int32_t*)(sb + h.o_hoff); O.hit_id = (uint32_t*)(sb + h.o_hid);
      O.dbg_up = o.dbg_up ? (int32_t*)(sb + h.o_up) : nullptr;
      O.dbg_dn = o.dbg_dn ? (int32_t*)(sb + h.o_dn) : nullptr;
      O.dbg_cup = o.dbg_cup ? (int32_t*)(sb + h.o_cup) : nullptr;
      O.dbg_cdn = o.dbg_cdn ? (int32_t*)(sb + h.o_cdn) : nullptr;
      O.dbg_start = o.dbg_start ? (uint32_t*)(sb + h.o_start) : nullptr;
    } else {
      O.sector = o.sector; O.x_ref = o.x_ref; O.p = o.p; O.cov = o.cov; O.chi2 = o.chi2; O.ndf = o.ndf;
      O.k_prior = o.k_prior; O.hit_off = o.hit_off; O.hit_id = o.hit_id;
      O.dbg_up = o.dbg_up; O.dbg_dn = o.dbg_dn; O.dbg_cup = o.dbg_cup; O.dbg_cdn = o.dbg_cdn;
      O.dbg_start = o.dbg_start;
    }
  }
  // binning chunks never span two events (the table has a fixed length for
  // given N and E, so a captured graph stays valid; surplus entries are empty)
  {
    size_t q = 0;
    for (int e = 0; e < E; ++e)
      for (int64_t c0 = ein[e].base; c0 < ein[e].base + ein[e].n; c0 += kChunkCl)
        chunks[q++] = ChunkIn{c0, std::min<int64_t>(c0 + kChunkCl, ein[e].base + ein[e].n), e, 0};
    for (; q < nchunk; ++q) chunks[q] = ChunkIn{0, 0, 0, 0};
  }
  c->hpin_busy = true;
  c->hpin_stream = st;
  // the three tables in one copy: same placement on both sides
  he = hipMemcpyAsync((void*)w.ev, ein, p_chunk + sizeof(ChunkIn) * nchunk, hipMemcpyHostToDevice, st);
  if (he != hipSuccess) return hip_fail(c, he, "table upload");

  if (c->tune.use_graph && !c->timing && st != nullptr) {
    const bool same = c->gexec && c->gkey.N == N && c->gkey.E == E && c->gkey.arena == c->arena &&
                      c->gkey.st == st && c->gkey.tracklet_grid == c->tune.tracklet_grid &&
                      c->gkey.taps == w.taps && c->gkey.cal == w.cal &&
                      std::memcmp(&c->gkey.P, &c->P, sizeof(tpcca_params)) == 0;
    if (!same) {
      if (c->gexec) { (void)hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
      if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
      he = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
      if (he != hipSuccess) return hip_fail(c, he, "graph capture");
      hipError_t le = run_pipeline(w, st, nullptr);
      he = hipStreamEndCapture(st, &c->graph);
      if (le != hipSuccess) return hip_fail(c, le, "kernel launch (capture)");
      if (he != hipSuccess) return hip_fail(c, he, "graph capture");
      he = hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0);
      if (he != hipSuccess) { c->gexec = nullptr; return hip_fail(c, he, "graph instantiate"); }
      c->gkey.N = N; c->gkey.E = E; c->gkey.arena = c->arena; c->gkey.st = st;
      c->gkey.P = c->P; c->gkey.tracklet_grid = c->tune.tracklet_grid; c->gkey.taps = w.taps;
      c->gkey.cal = w.cal;
    }
    he = hipGraphLaunch(c->gexec, st);
    if (he != hipSuccess) return hip_fail(c, he, "graph launch");
  } else {
    he = run_pipeline(w, st, c->timing ? &c->pe : nullptr);
    if (he != hipSuccess) return hip_fail(c, he, "kernel launch");
  }
  // flags and per-event results in one copy: same placement on both sides
  he = hipMemcpyAsync(flags, w.flags, (p_res - p_flags) + sizeof(int64_t) * 4 * E, hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) return hip_fail(c, he, "tracking");
  c->hpin_busy = false;
  if (c->timing) {
    for (int i = 0; i < PH_N; ++i) {
      float ms = 0.f;
      he = hipEventElapsedTime(&ms, c->pe.ev[i], c->pe.ev[i + 1]);
      if (he != hipSuccess) return hip_fail(c, he, "phase timing");
      c->phase_ms[i] += ms;
    }
    c->timed_calls++;
  }
  if (flags[F_ERR] & ERR_STUCK) return fail(c, TPCCA_E_DEVICE, "tracklet kernel exceeded its iteration bound");
  if (flags[F_ERR] & ERR_INVALID) return fail(c, TPCCA_E_INVALID, "non-finite coordinate or row/sector out of range");
  if (flags[F_ERR] & ERR_LIMIT)
    return fail(c, TPCCA_E_LIMIT, "a pad row holds more than " + std::to_string(kMaxRow) + " clusters");
  bool fits = true;
  for (int e = 0; e < E; ++e) {
    out[e].n_tracks = res[e * 4 + 0];
    out[e].n_hits = res[e * 4 + 1];
    out[e].n_start = res[e * 4 + 2];
    fits &= res[e * 4 + 0] <= out[e].cap_tracks && res[e * 4 + 1] <= out[e].cap_hits;
  }
  c->last_ok = true;
  c->last_nseeds = flags[F_NSEEDS];
  c->w = w;
  if (!fits || flags[F_FITS] == 0u) return fail(c, TPCCA_E_CAPACITY, "output capacity too small");
  // host-memory outputs
  for (int e = 0; e < E; ++e) {
    if (!ho[e].host) continue;
    const HostOut& h = ho[e];
    tpcca_tracks& o = out[e];
    const int64_t nt = o.n_tracks, nh = o.n_hits, n = h.n;
    struct Cp { void* dst; size_t src; size_t bytes; };
    std::vector<Cp> cps = {
        {o.sector, h.o_sector, (size_t)nt}, {o.x_ref, h.o_xref, 4 * (size_t)nt}, {o.p, h.o_p, 20 * (size_t)nt},
        {o.cov, h.o_cov, 60 * (size_t)nt}, {o.chi2, h.o_chi2, 4 * (size_t)nt}, {o.ndf, h.o_ndf, 4 * (size_t)nt},
        {o.k_prior, h.o_kp, 4 * (size_t)nt}, {o.hit_off, h.o_hoff, 4 * (size_t)(nt + 1)},
        {o.hit_id, h.o_hid, 4 * (size_t)nh}, {o.dbg_up, h.o_up, 4 * (size_t)n}, {o.dbg_dn, h.o_dn, 4 * (size_t)n},
        {o.dbg_cup, h.o_cup, 4 * (size_t)n}, {o.dbg_cdn, h.o_cdn, 4 * (size_t)n},
        {o.dbg_start, h.o_start, 4 * (size_t)o.n_start}};
    for (const Cp& cp : cps) {
      if (!cp.dst || cp.bytes == 0) continue;
      he = hipMemcpyAsync(cp.dst, sb + cp.src, cp.bytes, hipMemcpyDeviceToHost, st);
      if (he != hipSuccess) return hip_fail(c, he, "output download");
    }
  }
  he = hipStreamSynchronize(st);
  if (he != hipSuccess) return hip_fail(c, he, "output download");
  return TPCCA_OK;
}

int tpcca_track(tpcca_ctx* c, const tpcca_clusters* k, tpcca_tracks* out) {
  if (!c) return TPCCA_E_INVALID;
  if (!k || !out) return fail(c, TPCCA_E_INVALID, "null clusters or output");
  return tpcca_track_batch(c, 1, k, out);
}

int tpcca_debug_tracklets(tpcca_ctx* c, int64_t cap, int64_t* n_seeds, uint32_t* seed_start,
                          int32_t* seed_nhits, int32_t* seed_hits, float* seed_state) {
  if (!c || !n_seeds) return TPCCA_E_INVALID;
  if (!c->last_ok) return fail(c, TPCCA_E_INVALID, "no successful tracking call to inspect");
  const Ws& w = c->w;
  const int64_t ns = c->last_nseeds;
  *n_seeds = ns;
  if (cap < ns) return fail(c, TPCCA_E_CAPACITY, "seed capacity too small");
  if (ns == 0) return TPCCA_OK;
  std::vector<uint32_t> seeds(ns), cid(w.N);
  std::vector<int32_t> nh(ns), hits((size_t)ns * w.Rh);   // [band][seed][8] for the first ns seeds
  std::vector<float> state((size_t)ns * kTl);
  hipError_t he = hipMemcpy(seeds.data(), w.seeds, 4 * ns, hipMemcpyDeviceToHost);
  if (he == hipSuccess) he = hipMemcpy(cid.data(), w.cid, 4 * w.N, hipMemcpyDeviceToHost);
  if (he == hipSuccess) he = hipMemcpy(nh.data(), w.tl_nhits, 4 * ns, hipMemcpyDeviceToHost);
  if (he == hipSuccess)
    he = hipMemcpy2D(hits.data(), 32 * (size_t)ns, w.tl_hits, 32 * (size_t)w.seed_cap, 32 * (size_t)ns,
                     (size_t)(w.Rh / 8), hipMemcpyDeviceToHost);
  if (he == hipSuccess) he = hipMemcpy(state.data(), w.tl_state, 4 * (size_t)ns * kTl, hipMemcpyDeviceToHost);
  std::vector<int32_t> rng(ns);
  if (he == hipSuccess) he = hipMemcpy(rng.data(), w.tl_range, 4 * ns, hipMemcpyDeviceToHost);
  if (he != hipSuccess) return hip_fail(c, he, "debug download");
  for (int64_t s = 0; s < ns; ++s) {
    if (seed_start) seed_start[s] = cid[seeds[s]];
    if (seed_nhits) seed_nhits[s] = nh[s];
    if (seed_hits) {
      const int rlo = rng[s] & 0xFFFF, rhi = rng[s] >> 16;
      for (int r = 0; r < w.R; ++r) {
        const int32_t h = hits[(size_t)hit_slot(ns, s, r)];
        seed_hits[(size_t)s * w.R + r] = (nh[s] > 0 && r >= rlo && r <= rhi && h >= 0) ? (int32_t)cid[h] : -1;
      }
    }
    if (seed_state) std::memcpy(seed_state + (size_t)s * kTl, state.data() + (size_t)s * kTl, sizeof(float) * kTl);
  }
  return TPCCA_OK;
}

int tpcca_debug_fp32(int32_t op, int64_t n, const float* a, const float* b, float* out, void* stream) {
  if (op < 0 || op > 3 || n < 0) return TPCCA_E_INVALID;
  if (n > 0 && (!a || !out || (op == 1 && !b))) return TPCCA_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  hipError_t he = fp32_probe(op, n, a, b, out, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) { (void)hipGetLastError(); return TPCCA_E_DEVICE; }
  return TPCCA_OK;
}

int tpcca_set_tuning(tpcca_ctx* c, const tpcca_tuning* t) {
  if (!c || !t) return TPCCA_E_INVALID;
  if (t->ckpt_every < 1 || t->ckpt_every > 160 || t->tracklet_grid < 0 || t->use_graph < 0 || t->use_graph > 1)
    return fail(c, TPCCA_E_INVALID, "invalid tuning values");
  c->tune = *t;
  return TPCCA_OK;
}

int tpcca_get_tuning(const tpcca_ctx* c, tpcca_tuning* t) {
  if (!c || !t) return TPCCA_E_INVALID;
  *t = c->tune;
  return TPCCA_OK;
}

}  // extern "C"

namespace {

// Where the arrays of one gradient call live in its scratch (byte offsets
// from the scratch base), for T tracks, H hits, NC clusters, S sectors, R
// pad rows and checkpoint stride K; host inputs get staged copies.
struct GradLayout {
  int K = 0, nck = 0, nseg = 0;
  size_t o_hx = 0, o_hy = 0, o_hz = 0, o_gx = 0, o_gy = 0, o_gz = 0, o_gpt = 0;
  size_t o_bva = 0, o_bvb = 0, o_bsp = 0, o_dzt = 0;
  size_t o_part = 0, o_tf = 0, o_tn = 0, o_ck = 0, o_sg = 0, o_chunk = 0, o_out = 0, o_ndf = 0, o_err = 0;
  size_t o_off = 0, o_ids = 0, o_kp = 0, o_ext = 0, o_uv = 0;
  size_t o_cx = 0, o_cy = 0, o_cz = 0, o_cs = 0, o_th = 0;
  size_t o_flag = 0;       // staged per-track flags for a host track_flag
  size_t bytes = 0;
};

GradLayout grad_layout(int64_t T, int64_t H, int64_t NC, int S, int R, int K, bool th, bool kh, bool ch,
                       bool fh) {
  GradLayout g;
  g.K = K;
  g.nck = (R - 1 + K - 1) / K + 1;
  g.nseg = 2 * K + kTail;
  const int nq = S * kNPar + 1;
  const int64_t nchunk = (T + kChunk - 1) / kChunk;
  Layout L;
  g.o_hx = L.take<float>(H); g.o_hy = L.take<float>(H); g.o_hz = L.take<float>(H);
  g.o_gx = L.take<float>(H); g.o_gy = L.take<float>(H); g.o_gz = L.take<float>(H); g.o_gpt = L.take<float>(H);
  g.o_bva = L.take<float4>(H); g.o_bvb = L.take<float4>(H); g.o_bsp = L.take<int32_t>(H);
  g.o_dzt = L.take<float>(H);
  g.o_part = L.take<float>(T * kPart);
  g.o_tf = L.take<int32_t>(T); g.o_tn = L.take<int32_t>(T);
  g.o_ck = L.take<float>(T * g.nck * 20); g.o_sg = L.take<float>(T * g.nseg * 20);
  // the total chi2 (last entry of out), ndf and the error word are read
  // back together: keep them adjacent
  g.o_chunk = L.take<double>(nchunk * nq); g.o_out = L.take<double>(nq);
  g.o_ndf = L.take<unsigned long long>(1); g.o_err = L.take<uint32_t>(1);
  if (th) {
    g.o_off = L.take<int32_t>(T + 1); g.o_ids = L.take<uint32_t>(H); g.o_kp = L.take<float>(T);
    g.o_ext = L.take<float>(T); g.o_uv = L.take<uint8_t>(T);
  }
  if (kh) { g.o_cx = L.take<float>(NC); g.o_cy = L.take<float>(NC); g.o_cz = L.take<float>(NC); g.o_cs = L.take<uint8_t>(NC); }
  if (ch) g.o_th = L.take<float>(S * 66);
  if (fh) g.o_flag = L.take<int32_t>(T);
  g.bytes = L.off;
  return g;
}

// Argument checks shared by the gradient entry points.
int grad_args(tpcca_ctx* c, const tpcca_tracks* t, const tpcca_calib* cal, const tpcca_grad* g) {
  if (!t || !cal || !g || !t->clusters) return fail(c, TPCCA_E_INVALID, "null tracks, clusters, calib or grad");
  const tpcca_clusters& k = *t->clusters;
  const int64_t T = t->n_tracks, NC = k.n;
  if (T < 0 || NC < 0) return fail(c, TPCCA_E_INVALID, "negative sizes");
  if (T >= ((int64_t)1 << 31) || NC >= ((int64_t)1 << 32)) return fail(c, TPCCA_E_INVALID, "too many tracks or clusters");
  if (T > 0 && (!t->hit_off || !t->hit_id || !t->k_prior)) return fail(c, TPCCA_E_INVALID, "null hit_off/hit_id/k_prior");
  if (NC > 0 && (!k.x || !k.y || !k.z || !k.sector)) return fail(c, TPCCA_E_INVALID, "null cluster arrays");
  if (!cal->drift_scale || !cal->time_offset || !cal->map) return fail(c, TPCCA_E_INVALID, "null calibration arrays");
  if (!g->d_drift_scale || !g->d_time_offset || !g->d_map) return fail(c, TPCCA_E_INVALID, "null gradient arrays");
  for (int mk : {t->mem, k.mem, cal->mem, g->mem})
    if (mk != TPCCA_MEM_HOST && mk != TPCCA_MEM_DEVICE) return fail(c, TPCCA_E_INVALID, "bad mem kind");
  return TPCCA_OK;
}

// Bind the workspace of a gradient call to scratch base b (laid out by gl)
// and to the caller's arrays; host inputs are copied into the scratch on
// stream st.
hipError_t grad_bind(const tpcca_ctx* c, CalWs& w, char* b, const GradLayout& gl, const tpcca_tracks* t,
                     const tpcca_calib* cal, const tpcca_grad* g, int64_t H, hipStream_t st) {
  const tpcca_clusters& k = *t->clusters;
  const int S = c->S;
  const int64_t T = t->n_tracks, NC = k.n;
  w = CalWs{};
  w.S = S; w.R = c->R;
  w.geo = cal_geo(c);
  w.m = make_model(c->bz, c->P);
  w.sv2 = c->P.sigma_vertex * c->P.sigma_vertex;
  w.st2 = c->P.sigma_tgl * c->P.sigma_tgl;
  w.K = gl.K; w.nck = gl.nck; w.nseg = gl.nseg;
  w.T = T; w.H = H; w.NC = NC;
  auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0 || !src) return hipSuccess;
    return hipMemcpyAsync(b + off, src, bytes, hipMemcpyHostToDevice, st);
  };
  hipError_t he = hipSuccess;
  if (t->mem == TPCCA_MEM_HOST) {
    if (he == hipSuccess) he = up(gl.o_off, t->hit_off, 4 * (T + 1));
    if (he == hipSuccess) he = up(gl.o_ids, t->hit_id, 4 * H);
    if (he == hipSuccess) he = up(gl.o_kp, t->k_prior, 4 * T);
    if (he == hipSuccess) he = up(gl.o_ext, t->ext_tgl, 4 * T);
    if (he == hipSuccess) he = up(gl.o_uv, t->use_vertex, T);
    w.hit_off = (const int32_t*)(b + gl.o_off); w.hit_id = (const uint32_t*)(b + gl.o_ids);
    w.k_prior = (const float*)(b + gl.o_kp);
    w.ext_tgl = t->ext_tgl ? (const float*)(b + gl.o_ext) : nullptr;
    w.use_vertex = t->use_vertex ? (const uint8_t*)(b + gl.o_uv) : nullptr;
  } else {
    w.hit_off = t->hit_off; w.hit_id = t->hit_id; w.k_prior = t->k_prior;
    w.ext_tgl = t->ext_tgl; w.use_vertex = t->use_vertex;
  }
  if (k.mem == TPCCA_MEM_HOST) {
    if (he == hipSuccess) he = up(gl.o_cx, k.x, 4 * NC);
    if (he == hipSuccess) he = up(gl.o_cy, k.y, 4 * NC);
    if (he == hipSuccess) he = up(gl.o_cz, k.z, 4 * NC);
    if (he == hipSuccess) he = up(gl.o_cs, k.sector, NC);
    w.cx = (const float*)(b + gl.o_cx); w.cy = (const float*)(b + gl.o_cy); w.cz = (const float*)(b + gl.o_cz);
    w.csec = (const uint8_t*)(b + gl.o_cs);
  } else {
    w.cx = k.x; w.cy = k.y; w.cz = k.z; w.csec = k.sector;
  }
  if (cal->mem == TPCCA_MEM_HOST) {
    if (he == hipSuccess) he = up(gl.o_th, cal->drift_scale, 4 * S);
    if (he == hipSuccess) he = up(gl.o_th + 4 * S, cal->time_offset, 4 * S);
    if (he == hipSuccess) he = up(gl.o_th + 8 * S, cal->map, 4 * 64 * S);
    w.dl = (const float*)(b + gl.o_th); w.tau = (const float*)(b + gl.o_th + 4 * S);
    w.map = (const float*)(b + gl.o_th + 8 * S);
  } else {
    w.dl = cal->drift_scale; w.tau = cal->time_offset; w.map = cal->map;
  }
  w.hx = (float*)(b + gl.o_hx); w.hy = (float*)(b + gl.o_hy); w.hz = (float*)(b + gl.o_hz);
  w.gx = (float*)(b + gl.o_gx); w.gy = (float*)(b + gl.o_gy); w.gz = (float*)(b + gl.o_gz);
  w.gpt = (float*)(b + gl.o_gpt);
  w.bva = (float4*)(b + gl.o_bva); w.bvb = (float4*)(b + gl.o_bvb); w.bsp = (int32_t*)(b + gl.o_bsp);
  w.dzt = (float*)(b + gl.o_dzt);
  w.part = (float*)(b + gl.o_part); w.tflag = (int32_t*)(b + gl.o_tf); w.tndf = (int32_t*)(b + gl.o_tn);
  w.ckpt = (float*)(b + gl.o_ck); w.seg = (float*)(b + gl.o_sg);
  w.chunk = (double*)(b + gl.o_chunk); w.out = (double*)(b + gl.o_out);
  w.ndf_sum = (unsigned long long*)(b + gl.o_ndf); w.err = (uint32_t*)(b + gl.o_err);
  // device gradient arrays and flags are written by the kernels themselves
  if (g->mem == TPCCA_MEM_DEVICE) {
    w.g_dl = g->d_drift_scale; w.g_tau = g->d_time_offset; w.g_map = g->d_map;
    w.flag_out = g->track_flag;
  } else if (g->track_flag) {
    w.flag_out = (int32_t*)(b + gl.o_flag);
  }
  return he;
}

// The error word of a finished gradient call.
int grad_err(tpcca_ctx* c, uint32_t err) {
  if (err & 1u) return fail(c, TPCCA_E_INVALID, "hit id or sector out of range");
  if (err & 2u) return fail(c, TPCCA_E_INVALID, "a track has more hits than pad rows");
  return TPCCA_OK;
}

// The merger on T segments with H hits (checked by the caller) whose hit
// ids index NC clusters (cx, cy, cz, crow); slice: the segments' time-frame
// slices or null.  Device memory throughout.
// slice: each segment's time-frame slice (null for one event); nsl slices
// of length slice_len along the readout time.
int merge_core(tpcca_ctx* c, const tpcca_tracks* seg, const float* cx, const float* cy, const float* cz,
               const int16_t* crow, int64_t NC, const int32_t* slice, int nsl, float slice_len, int64_t H,
               tpcca_tracks* out, int32_t* seg_link, hipStream_t st) {
  const int64_t T = seg->n_tracks;
  hipError_t he;
  // the merged output has at most as many tracks, and exactly as many hits
  if (out->cap_tracks < T || out->cap_hits < H) {
    out->n_tracks = T;
    out->n_hits = H;
    return fail(c, TPCCA_E_CAPACITY, "merged output needs n_tracks and n_hits of the segments");
  }
  if ((T > 0 && (!out->sector || !out->x_ref || !out->p || !out->cov || !out->chi2 || !out->ndf)) ||
      (H > 0 && !out->hit_id))
    return fail(c, TPCCA_E_INVALID, "null output array");
  Layout L;
  const size_t o_ex = L.take<float>(T * 24), o_first = L.take<float4>(T), o_last = L.take<float4>(T);
  const int64_t nbin = (int64_t)c->S * (slice ? nsl : 1);
  const size_t o_flags = L.take<uint32_t>(T), o_cnt = L.take<uint32_t>(nbin + 1), o_cur = L.take<uint32_t>(nbin);
  const size_t o_list = L.take<uint32_t>(T), o_bi = L.take<unsigned long long>(T), o_bo = L.take<unsigned long long>(T);
  const size_t o_link = L.take<int32_t>(T), o_inner = L.take<int32_t>(T), o_emit = L.take<uint32_t>(T + 1);
  const size_t o_hemit = L.take<uint32_t>(T + 1), o_rec = L.take<float>(T * 24), o_err = L.take<uint32_t>(4);
  const size_t o_srec = L.take<float4>(T), o_head = L.take<int32_t>(T), o_tpos = L.take<uint32_t>(T);
  const size_t o_hpos = L.take<uint32_t>(T), o_nseg = L.take<uint32_t>(T), o_rlist = L.take<uint32_t>(T);
  const size_t o_part = L.take<uint32_t>(2 * (std::max<int64_t>(T, nbin) / 1024 + 2));
  const size_t o_zrec = L.take<float4>(T), o_zlist = L.take<uint32_t>(T), o_zs = L.take<uint8_t>(nbin);
  if (L.off > c->mscratch_bytes) {
    if (c->mscratch) { (void)hipFree(c->mscratch); c->mscratch = nullptr; c->mscratch_bytes = 0; }
    he = hipMalloc((void**)&c->mscratch, L.off + L.off / 4);
    if (he != hipSuccess) { c->mscratch = nullptr; (void)hipGetLastError(); return fail(c, TPCCA_E_NOMEM, "merger scratch allocation failed"); }
    c->mscratch_bytes = L.off + L.off / 4;
  }
  char* b = c->mscratch;
  MergeWs w{};
  w.T = T; w.H = H; w.S = c->S; w.NW = c->S / 2; w.R = c->R; w.NC = NC;
  w.m = make_model(c->bz, c->P);
  w.chi2_merge = c->P.chi2_merge;
  w.merge_dist = c->P.merge_dist;
  const double turn = 2.0 * M_PI / (double)w.NW;
  w.ca = (float)std::cos(turn);
  w.sa = (float)std::sin(turn);
  w.sector = seg->sector; w.x_ref = seg->x_ref; w.p = seg->p; w.cov = seg->cov; w.chi2 = seg->chi2;
  w.ndf = seg->ndf; w.hit_off = seg->hit_off; w.hit_id = seg->hit_id;
  w.cx = cx; w.cy = cy; w.cz = cz; w.crow = crow; w.slice = slice;
  w.nsl = slice ? nsl : 1;
  w.prune = slice && nsl > 1 && w.merge_dist < 0.5f * slice_len ? 1 : 0;
  w.ex = (float*)(b + o_ex); w.first = (float4*)(b + o_first); w.last = (float4*)(b + o_last);
  w.flags = (uint32_t*)(b + o_flags); w.sec_cnt = (uint32_t*)(b + o_cnt); w.sec_cur = (uint32_t*)(b + o_cur);
  w.sec_list = (uint32_t*)(b + o_list);
  w.best_in = (unsigned long long*)(b + o_bi); w.best_out = (unsigned long long*)(b + o_bo);
  w.link = (int32_t*)(b + o_link); w.inner = (int32_t*)(b + o_inner);
  w.emit = (uint32_t*)(b + o_emit); w.hemit = (uint32_t*)(b + o_hemit);
  w.rec = (float*)(b + o_rec); w.err = (uint32_t*)(b + o_err);
  w.srec = (float4*)(b + o_srec); w.head = (int32_t*)(b + o_head); w.tpos = (uint32_t*)(b + o_tpos);
  w.hpos = (uint32_t*)(b + o_hpos); w.nseg = (uint32_t*)(b + o_nseg); w.rlist = (uint32_t*)(b + o_rlist);
  w.scan_part = (uint32_t*)(b + o_part);
  w.zrec = (float4*)(b + o_zrec); w.zlist = (uint32_t*)(b + o_zlist); w.zsorted = (uint8_t*)(b + o_zs);
  w.o_sector = out->sector; w.o_x_ref = out->x_ref; w.o_p = out->p; w.o_cov = out->cov; w.o_chi2 = out->chi2;
  w.o_ndf = out->ndf; w.o_hit_off = out->hit_off; w.o_hit_id = out->hit_id; w.o_link = seg_link;
  // an empty call still passes valid pointers to the kernels' checks
  if (T == 0) {
    w.sector = w.o_sector = (uint8_t*)b; w.x_ref = w.o_x_ref = (float*)b; w.p = w.o_p = (float*)b;
    w.cov = w.o_cov = (float*)b; w.chi2 = w.o_chi2 = (float*)b; w.ndf = w.o_ndf = (int32_t*)b;
    w.hit_id = w.o_hit_id = (uint32_t*)b;
  }
  if (NC == 0) { w.cx = w.cy = w.cz = (const float*)b; w.crow = (const int16_t*)b; }
  he = run_merge(w, st);
  if (he != hipSuccess) return hip_fail(c, he, "merger kernels");
  uint32_t res[4] = {0, 0, 0, 0};
  he = hipMemcpyAsync(res, w.err, sizeof(res), hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) return hip_fail(c, he, "merger");
  if (res[0] & 1u) return fail(c, TPCCA_E_INVALID, "a segment has fewer than 3 or more than n_rows hits, or a bad sector");
  if (res[0] & 2u) return fail(c, TPCCA_E_INVALID, "hit id out of range");
  out->n_tracks = res[1];
  out->n_hits = res[2];
  return TPCCA_OK;
}

}  // namespace

extern "C" {

int tpcca_refit_grad(tpcca_ctx* c, const tpcca_tracks* t, const tpcca_calib* cal, tpcca_grad* g) {
  if (!c) return TPCCA_E_INVALID;
  int rc = grad_args(c, t, cal, g);
  if (rc != TPCCA_OK) return rc;
  const tpcca_clusters& k = *t->clusters;
  const int64_t T = t->n_tracks, NC = k.n;
  const int S = c->S;
  hipError_t he = hipSetDevice(c->device);
  if (he != hipSuccess) return hip_fail(c, he, "hipSetDevice");
  hipStream_t st = (hipStream_t)k.stream;
  // the hit count and the results are read back through pinned host memory
  // (a call that failed after queueing copies may have left them in flight)
  if (c->hpin_busy) {
    (void)hipStreamSynchronize(c->hpin_stream);
    (void)hipGetLastError();
    c->hpin_busy = false;
  }
  const int nq = S * kNPar + 1;
  const size_t r_bytes = al(sizeof(double) * nq) + al(sizeof(unsigned long long)) + sizeof(uint32_t);
  rc = ensure_pinned(c, r_bytes);
  if (rc != TPCCA_OK) return rc;
  // number of hits
  int32_t H32 = 0;
  if (T > 0) {
    if (t->mem == TPCCA_MEM_HOST) {
      H32 = t->hit_off[T];
      if (t->hit_off[0] != 0) return fail(c, TPCCA_E_INVALID, "hit_off[0] must be 0");
    } else {
      int32_t* ends = (int32_t*)c->hpin;
      c->hpin_busy = true;
      c->hpin_stream = st;
      he = hipMemcpyAsync(&ends[0], t->hit_off, 4, hipMemcpyDeviceToHost, st);
      if (he == hipSuccess) he = hipMemcpyAsync(&ends[1], t->hit_off + T, 4, hipMemcpyDeviceToHost, st);
      if (he == hipSuccess) he = hipStreamSynchronize(st);
      if (he != hipSuccess) return hip_fail(c, he, "hit_off read");
      c->hpin_busy = false;
      if (ends[0] != 0) return fail(c, TPCCA_E_INVALID, "hit_off[0] must be 0");
      H32 = ends[1];
    }
  }
  const int64_t H = H32;
  if (H < 0) return fail(c, TPCCA_E_INVALID, "negative hit count");
  const GradLayout gl = grad_layout(T, H, NC, S, c->R, c->tune.ckpt_every, t->mem == TPCCA_MEM_HOST,
                                    k.mem == TPCCA_MEM_HOST, cal->mem == TPCCA_MEM_HOST,
                                    g->mem == TPCCA_MEM_HOST && g->track_flag);
  if (gl.bytes > c->gscratch_bytes) {
    if (c->gscratch) { (void)hipFree(c->gscratch); c->gscratch = nullptr; c->gscratch_bytes = 0; }
    he = hipMalloc((void**)&c->gscratch, gl.bytes + gl.bytes / 4);
    if (he != hipSuccess) { c->gscratch = nullptr; (void)hipGetLastError(); return fail(c, TPCCA_E_NOMEM, "gradient scratch allocation failed"); }
    c->gscratch_bytes = gl.bytes + gl.bytes / 4;
  }
  CalWs w{};
  he = grad_bind(c, w, c->gscratch, gl, t, cal, g, H, st);
  if (he != hipSuccess) return hip_fail(c, he, "input upload");
  he = run_calib(w, st);
  if (he != hipSuccess) return hip_fail(c, he, "gradient kernels");
  // sums, ndf and the error word in one copy (adjacent in the layout)
  c->hpin_busy = true;
  c->hpin_stream = st;
  he = hipMemcpyAsync(c->hpin, w.out, r_bytes, hipMemcpyDeviceToHost, st);
  if (he == hipSuccess && g->mem == TPCCA_MEM_HOST && g->track_flag && T > 0)
    he = hipMemcpyAsync(g->track_flag, w.flag_out, sizeof(int32_t) * (size_t)T, hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) return hip_fail(c, he, "gradient");
  c->hpin_busy = false;
  const double* out = (const double*)c->hpin;
  const unsigned long long ndf = *(const unsigned long long*)(c->hpin + (gl.o_ndf - gl.o_out));
  const uint32_t err = *(const uint32_t*)(c->hpin + (gl.o_err - gl.o_out));
  rc = grad_err(c, err);
  if (rc != TPCCA_OK) return rc;
  g->chi2 = out[S * kNPar];
  g->ndf = (int64_t)ndf;
  if (g->mem == TPCCA_MEM_HOST) {
    for (int s = 0; s < S; ++s) {
      g->d_drift_scale[s] = out[s * kNPar + 0];
      g->d_time_offset[s] = out[s * kNPar + 1];
      for (int q = 0; q < 64; ++q) g->d_map[(size_t)s * 64 + q] = out[s * kNPar + 2 + q];
    }
  }
  return TPCCA_OK;
}

int tpcca_merge(tpcca_ctx* c, const tpcca_tracks* seg, tpcca_tracks* out, int32_t* seg_link) {
  if (!c) return TPCCA_E_INVALID;
  if (!seg || !out || !seg->clusters) return fail(c, TPCCA_E_INVALID, "null segments, output or clusters");
  const tpcca_clusters& k = *seg->clusters;
  const int64_t T = seg->n_tracks, NC = k.n;
  if (T < 0 || NC < 0 || T >= ((int64_t)1 << 31)) return fail(c, TPCCA_E_INVALID, "bad sizes");
  if (seg->mem != TPCCA_MEM_DEVICE || k.mem != TPCCA_MEM_DEVICE || out->mem != TPCCA_MEM_DEVICE)
    return fail(c, TPCCA_E_INVALID, "the merger takes device memory only");
  if (!seg->hit_off || (T > 0 && (!seg->sector || !seg->x_ref || !seg->p || !seg->cov || !seg->chi2 || !seg->ndf ||
                                  !seg->hit_id)))
    return fail(c, TPCCA_E_INVALID, "null segment array");
  if (NC > 0 && (!k.x || !k.y || !k.z || !k.row)) return fail(c, TPCCA_E_INVALID, "null cluster array");
  if (!out->hit_off || out->cap_tracks < 0 || out->cap_hits < 0) return fail(c, TPCCA_E_INVALID, "bad output");
  hipError_t he = hipSetDevice(c->device);
  if (he != hipSuccess) return hip_fail(c, he, "hipSetDevice");
  hipStream_t st = (hipStream_t)k.stream;
  int32_t ends[2] = {0, 0};
  if (T > 0) {
    he = hipMemcpyAsync(&ends[0], seg->hit_off, 4, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipMemcpyAsync(&ends[1], seg->hit_off + T, 4, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return hip_fail(c, he, "hit_off read");
    if (ends[0] != 0 || ends[1] < 0) return fail(c, TPCCA_E_INVALID, "hit_off must start at 0");
  }
  return merge_core(c, seg, k.x, k.y, k.z, k.row, NC, nullptr, 1, 0.0f, ends[1], out, seg_link, st);
}

int tpcca_track_timeframe(tpcca_ctx* c, const tpcca_clusters* fr, float slice_len, int32_t n_slices,
                          tpcca_tracks* merged, tpcca_tracks* segs, int32_t* seg_slice, int32_t* seg_link) {
  if (!c) return TPCCA_E_INVALID;
  if (!fr || !merged) return fail(c, TPCCA_E_INVALID, "null frame or output");
  const int64_t n = fr->n;
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(c, TPCCA_E_INVALID, "bad cluster count");
  if (fr->mem != TPCCA_MEM_DEVICE || merged->mem != TPCCA_MEM_DEVICE || (segs && segs->mem != TPCCA_MEM_DEVICE))
    return fail(c, TPCCA_E_INVALID, "time-frame tracking takes device memory only");
  if (n > 0 && (!fr->x || !fr->y || !fr->z || !fr->row || !fr->sector))
    return fail(c, TPCCA_E_INVALID, "null cluster array");
  if (!(slice_len > 0.0f) || !(slice_len <= 2.0f * c->z_max))
    return fail(c, TPCCA_E_INVALID, "slice length outside (0, 2 z_max]");
  if (n_slices < 1 || n_slices > kTfMaxSlices) return fail(c, TPCCA_E_INVALID, "n_slices outside [1, 1024]");
  if (!merged->hit_off || merged->cap_tracks < 0 || merged->cap_hits < 0 ||
      (segs && (!segs->hit_off || segs->cap_tracks < 0 || segs->cap_hits < 0)))
    return fail(c, TPCCA_E_INVALID, "bad output");
  if (check_params(&c->P) != TPCCA_OK) return fail(c, TPCCA_E_INVALID, "invalid parameters");
  hipError_t he = hipSetDevice(c->device);
  if (he != hipSuccess) return hip_fail(c, he, "hipSetDevice");
  hipStream_t st = (hipStream_t)fr->stream;
  const int E = n_slices;
  const int64_t nb = std::max<int64_t>((n + kTfBlock - 1) / kTfBlock, 1);
  const int64_t TC = n / std::max(c->P.min_hits, 1) + E;     // tracks of all slices, at most
  const int64_t ncnt = (int64_t)E * nb;
  Layout L;
  const size_t o_cnt = L.take<uint32_t>(ncnt + 1), o_part = L.take<uint32_t>(2 * (ncnt / 1024 + 2));
  const size_t o_err = L.take<uint32_t>(4), o_soff = L.take<uint32_t>(E + 1);
  const size_t o_sx = L.take<float>(n), o_sy = L.take<float>(n), o_sz = L.take<float>(n);
  const size_t o_srow = L.take<int16_t>(n), o_ssec = L.take<uint8_t>(n), o_sid = L.take<uint32_t>(n);
  const size_t o_ztf = L.take<float>(n);
  const size_t o_isec = L.take<uint8_t>(TC), o_ixr = L.take<float>(TC), o_ip = L.take<float>(TC * 5);
  const size_t o_icov = L.take<float>(TC * 15), o_ichi = L.take<float>(TC), o_indf = L.take<int32_t>(TC);
  const size_t o_ihoff = L.take<int32_t>(TC + E), o_ihid = L.take<uint32_t>(n);
  const size_t o_osec = L.take<uint8_t>(TC), o_oxr = L.take<float>(TC), o_op = L.take<float>(TC * 5);
  const size_t o_ocov = L.take<float>(TC * 15), o_ochi = L.take<float>(TC), o_ondf = L.take<int32_t>(TC);
  const size_t o_ohoff = L.take<int32_t>(TC + 1), o_ohid = L.take<uint32_t>(n), o_osl = L.take<int32_t>(TC);
  const size_t o_tab = L.take<TfRange>(E + 1);
  if (L.off > c->tfscratch_bytes) {
    if (c->tfscratch) { (void)hipFree(c->tfscratch); c->tfscratch = nullptr; c->tfscratch_bytes = 0; }
    he = hipMalloc((void**)&c->tfscratch, L.off + L.off / 4);
    if (he != hipSuccess) {
      c->tfscratch = nullptr;
      (void)hipGetLastError();
      return fail(c, TPCCA_E_NOMEM, "time-frame workspace allocation failed");
    }
    c->tfscratch_bytes = L.off + L.off / 4;
  }
  char* b = c->tfscratch;
  // 1. slices (counts, scan, stable scatter, offsets)
  TfSlice a{};
  a.n = n; a.x = fr->x; a.y = fr->y; a.tau = fr->z; a.row = fr->row; a.sector = fr->sector;
  a.D = slice_len; a.L = c->z_max; a.n_slices = E; a.half = c->S / 2; a.S = c->S; a.nb = nb;
  a.cnt = (uint32_t*)(b + o_cnt); a.err = (uint32_t*)(b + o_err); a.soff = (uint32_t*)(b + o_soff);
  a.sx = (float*)(b + o_sx); a.sy = (float*)(b + o_sy); a.sz = (float*)(b + o_sz);
  a.srow = (int16_t*)(b + o_srow); a.ssec = (uint8_t*)(b + o_ssec); a.sid = (uint32_t*)(b + o_sid);
  a.ztf = (float*)(b + o_ztf);
  std::vector<uint32_t> soff(E + 1, 0u);
  uint32_t terr = 0;
  if (n > 0) {
    he = fill_u32(a.err, 0u, 4, st);
    if (he == hipSuccess) he = tf_slice(a, (uint32_t*)(b + o_part), st);
    if (he == hipSuccess) he = hipMemcpyAsync(soff.data(), a.soff, sizeof(uint32_t) * (E + 1), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipMemcpyAsync(&terr, a.err, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return hip_fail(c, he, "time-frame slicing");
    if (terr) return fail(c, TPCCA_E_INVALID, "a readout time is not finite or lies outside the slices");
  }
  // 2. every slice tracked as one event of a batch (without the installed
  // calibration: its drift terms need the collision time)
  std::vector<tpcca_clusters> cls(E);
  std::vector<tpcca_tracks> trs(E);
  std::vector<int64_t> tcap(E + 1, 0);
  for (int e = 0; e < E; ++e) {
    const int64_t ne = (int64_t)soff[e + 1] - soff[e], co = soff[e];
    tcap[e + 1] = tcap[e] + ne / std::max(c->P.min_hits, 1) + 1;
    tpcca_clusters& k = cls[e];
    k = tpcca_clusters{};
    k.n = ne; k.x = a.sx + co; k.y = a.sy + co; k.z = a.sz + co; k.row = a.srow + co; k.sector = a.ssec + co;
    k.mem = TPCCA_MEM_DEVICE; k.stream = fr->stream;
    tpcca_tracks& o = trs[e];
    o = tpcca_tracks{};
    o.cap_tracks = tcap[e + 1] - tcap[e]; o.cap_hits = ne;
    o.sector = (uint8_t*)(b + o_isec) + tcap[e]; o.x_ref = (float*)(b + o_ixr) + tcap[e];
    o.p = (float*)(b + o_ip) + tcap[e] * 5; o.cov = (float*)(b + o_icov) + tcap[e] * 15;
    o.chi2 = (float*)(b + o_ichi) + tcap[e]; o.ndf = (int32_t*)(b + o_indf) + tcap[e];
    o.hit_off = (int32_t*)(b + o_ihoff) + tcap[e] + e; o.hit_id = (uint32_t*)(b + o_ihid) + co;
    o.mem = TPCCA_MEM_DEVICE;
  }
  const bool cal = c->cal_on;
  c->cal_on = false;
  int rc = tpcca_track_batch(c, E, cls.data(), trs.data());
  c->cal_on = cal;
  if (rc != TPCCA_OK) return rc;
  // 3. the segment set in frame coordinates
  std::vector<TfRange> tab(E + 1);
  int64_t T = 0, H = 0;
  for (int e = 0; e <= E; ++e) {
    TfRange& r = tab[e];
    r.tcap = tcap[std::min(e, E)]; r.hoff = r.tcap + e; r.hcap = soff[e]; r.coff = soff[e];
    r.tout = T; r.hout = H;
    if (e < E) { T += trs[e].n_tracks; H += trs[e].n_hits; }
  }
  if (merged->cap_tracks < T || merged->cap_hits < H || (segs && (segs->cap_tracks < T || segs->cap_hits < H))) {
    merged->n_tracks = T; merged->n_hits = H;
    if (segs) { segs->n_tracks = T; segs->n_hits = H; }
    return fail(c, TPCCA_E_CAPACITY, "outputs need the segments' track and hit counts");
  }
  TfGather g{};
  g.E = E; g.half = c->S / 2; g.D = slice_len; g.T = T; g.H = H;
  g.tab = (const TfRange*)(b + o_tab);
  g.isec = (const uint8_t*)(b + o_isec); g.ixref = (const float*)(b + o_ixr); g.ip = (const float*)(b + o_ip);
  g.icov = (const float*)(b + o_icov); g.ichi2 = (const float*)(b + o_ichi); g.indf = (const int32_t*)(b + o_indf);
  g.ihoff = (const int32_t*)(b + o_ihoff); g.ihid = (const uint32_t*)(b + o_ihid); g.sid = a.sid;
  g.osec = (uint8_t*)(b + o_osec); g.oxref = (float*)(b + o_oxr); g.op = (float*)(b + o_op);
  g.ocov = (float*)(b + o_ocov); g.ochi2 = (float*)(b + o_ochi); g.ondf = (int32_t*)(b + o_ondf);
  g.ohoff = (int32_t*)(b + o_ohoff); g.ohid = (uint32_t*)(b + o_ohid); g.oslice = (int32_t*)(b + o_osl);
  he = hipMemcpyAsync(b + o_tab, tab.data(), sizeof(TfRange) * (E + 1), hipMemcpyHostToDevice, st);
  if (he == hipSuccess) he = tf_gather(g, st);
  if (he == hipSuccess && segs) {
    auto cp = [&](void* dst, const void* src, size_t bytes) {
      if (he == hipSuccess && bytes) he = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
    };
    if (T > 0 && (!segs->sector || !segs->x_ref || !segs->p || !segs->cov || !segs->chi2 || !segs->ndf))
      return fail(c, TPCCA_E_INVALID, "null segment output array");
    if (H > 0 && !segs->hit_id) return fail(c, TPCCA_E_INVALID, "null segment hit_id");
    cp(segs->sector, g.osec, (size_t)T); cp(segs->x_ref, g.oxref, 4 * (size_t)T);
    cp(segs->p, g.op, 20 * (size_t)T); cp(segs->cov, g.ocov, 60 * (size_t)T);
    cp(segs->chi2, g.ochi2, 4 * (size_t)T); cp(segs->ndf, g.ondf, 4 * (size_t)T);
    cp(segs->hit_off, g.ohoff, 4 * (size_t)(T + 1)); cp(segs->hit_id, g.ohid, 4 * (size_t)H);
  }
  if (he == hipSuccess && seg_slice && T > 0)
    he = hipMemcpyAsync(seg_slice, g.oslice, 4 * (size_t)T, hipMemcpyDeviceToDevice, st);
  if (he != hipSuccess) return hip_fail(c, he, "time-frame segment set");
  if (segs) { segs->n_tracks = T; segs->n_hits = H; }
  // 4. the merger over slices and sectors, on the frame coordinates
  tpcca_tracks view{};
  view.n_tracks = T; view.n_hits = H;
  view.sector = g.osec; view.x_ref = g.oxref; view.p = g.op; view.cov = g.ocov; view.chi2 = g.ochi2;
  view.ndf = g.ondf; view.hit_off = g.ohoff; view.hit_id = g.ohid; view.mem = TPCCA_MEM_DEVICE;
  // (the tab upload above reads host memory that lives until here: the merger synchronises the stream)
  return merge_core(c, &view, fr->x, fr->y, a.ztf, fr->row, n, g.oslice, E, slice_len, H, merged, seg_link, st);
}

int tpcca_refit_grad_noalloc(tpcca_ctx* c, const tpcca_tracks* t, const tpcca_calib* cal, tpcca_grad* g) {
  if (!c) return TPCCA_E_INVALID;
  int rc = grad_args(c, t, cal, g);
  if (rc != TPCCA_OK) return rc;
  const tpcca_clusters& k = *t->clusters;
  if (t->mem != TPCCA_MEM_DEVICE || k.mem != TPCCA_MEM_DEVICE || cal->mem != TPCCA_MEM_DEVICE ||
      g->mem != TPCCA_MEM_DEVICE)
    return fail(c, TPCCA_E_INVALID, "the allocation-free gradient takes device memory only");
  if (!c->noalloc_scratch)
    return fail(c, TPCCA_E_DEVICE, "the device address of the static gradient scratch is unknown: " + c->noalloc_err);
  const int64_t T = t->n_tracks, NC = k.n;
  const int S = c->S;
  hipError_t he = hipSetDevice(c->device);
  if (he != hipSuccess) return hip_fail(c, he, "hipSetDevice");
  hipStream_t st = (hipStream_t)k.stream;
  // the hit count, read into host stack memory
  int32_t ends[2] = {0, 0};
  if (T > 0) {
    he = hipMemcpyAsync(&ends[0], t->hit_off, 4, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipMemcpyAsync(&ends[1], t->hit_off + T, 4, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return hip_fail(c, he, "hit_off read");
    if (ends[0] != 0) return fail(c, TPCCA_E_INVALID, "hit_off[0] must be 0");
    if (ends[1] < 0) return fail(c, TPCCA_E_INVALID, "negative hit count");
  }
  const int64_t H = ends[1];
  // the largest checkpoint stride up to the tuned one whose layout fits
  // (results do not depend on the stride)
  GradLayout gl;
  int K = c->tune.ckpt_every;
  for (; K >= 1; --K) {
    gl = grad_layout(T, H, NC, S, c->R, K, false, false, false, false);
    if (gl.bytes <= kNoAllocScratchBytes) break;
  }
  if (K < 1)
    return fail(c, TPCCA_E_LIMIT, std::to_string(T) + " tracks with " + std::to_string(H) +
                                      " hits need more than the " + std::to_string(kNoAllocScratchBytes >> 20) +
                                      " MiB of static gradient scratch at every checkpoint stride");
  CalWs w{};
  he = grad_bind(c, w, c->noalloc_scratch, gl, t, cal, g, H, st);
  if (he != hipSuccess) return hip_fail(c, he, "workspace");
  he = run_calib(w, st);
  if (he != hipSuccess) return hip_fail(c, he, "gradient kernels");
  // the total chi2 (last entry of out), ndf and the error word are adjacent
  const size_t from = gl.o_out + sizeof(double) * (size_t)(S * kNPar);
  const size_t span = gl.o_err + sizeof(uint32_t) - from;
  alignas(8) unsigned char res[1024];
  static_assert(sizeof(double) + 256 + 256 + sizeof(uint32_t) <= sizeof(res), "result words");
  if (span > sizeof(res)) return fail(c, TPCCA_E_DEVICE, "result layout");
  he = hipMemcpyAsync(res, c->noalloc_scratch + from, span, hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) return hip_fail(c, he, "gradient");
  double chi2;
  unsigned long long ndf;
  uint32_t err;
  std::memcpy(&chi2, res, sizeof(double));
  std::memcpy(&ndf, res + (gl.o_ndf - from), sizeof(ndf));
  std::memcpy(&err, res + (gl.o_err - from), sizeof(err));
  rc = grad_err(c, err);
  if (rc != TPCCA_OK) return rc;
  g->chi2 = chi2;
  g->ndf = (int64_t)ndf;
  return TPCCA_OK;
}

}  // extern "C"
