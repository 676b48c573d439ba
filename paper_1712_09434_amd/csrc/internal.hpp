// internal.hpp -- device workspace layout shared by the kernels and the host
// runtime of libtpcca (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tpcca.h"
#include "calib_device.hpp"
#include "kf_device.hpp"

namespace tpcca {

constexpr int kMaxRow = TPCCA_MAX_ROW_CLUSTERS;   // clusters per (sector, row) handled in LDS
constexpr int kMaxSectors = 254;                  // sectors of a geometry, at most
constexpr int kMaxCells = kMaxRow / 2 + 1;        // grid cells per (sector, row), at most

// Cells of a row unit's search grid for n clusters: kCellsPerCluster per
// cluster (window searches then scan ~2 candidates), capped at kMaxCells.
constexpr uint32_t kCellsPerCluster = 2;
__host__ __device__ inline uint32_t grid_cells(uint32_t n) {
  const uint32_t c = kCellsPerCluster * n + 1u;
  return c < (uint32_t)kMaxCells ? c : (uint32_t)kMaxCells;
}

// Flags / counters in device memory.
enum : int {
  F_ERR = 0,        // error bits (below)
  F_NSEEDS = 1,     // number of seeds
  F_NSTARTS = 2,    // number of start hits
  F_FITS = 3,       // 1 if every event's outputs fit their capacities
  F_LROWS1 = 4,     // list lengths of the row-unit size classes (many row units only):
  F_LROWS2 = 5,     //   row kernels' wave, workgroup and large classes (also F_LROWS3),
  F_LLINKS1 = 6,    //   link kernels' small-slab and slab classes
  F_LLINKS2 = 7,
  F_SEEDCTR = 8,    // work counters of the tracklet kernel, one per seed range (8)
  F_LROWS3 = 16,
  F_COUNT = 20
};
enum : uint32_t { ERR_INVALID = 1u, ERR_LIMIT = 2u, ERR_STUCK = 4u };

// Per-(event, sector, row) search grid: cells of a uniform 2-D (z, y) grid
// over the row's bounding box; cell (iz, iy) = cell_base + iz * ny + iy.
struct alignas(16) GridParams {
  uint32_t cell_base;
  uint32_t nz, ny;
  float z0, y0, inv_bz, inv_by;
  uint32_t base;        // the row unit's first entry in the grid-ordered arrays
  uint32_t off_plane;   // 1: some cluster of the row unit has x other than the row's plane
};

// Grid-ordered record of the tracklet search: (y, z, canonical position).
struct SearchRec {
  float y, z;
  uint32_t pos;
};

struct EventIn {
  const float* x;
  const float* y;
  const float* z;
  const int16_t* row;
  const uint8_t* sector;
  int64_t base;     // first global cluster index of the event
  int64_t n;
};

// Binning chunk: kChunkCl consecutive clusters of one event (the last chunk
// of an event is shorter; unused table entries are empty).
constexpr int kChunkCl = 8192;
struct ChunkIn {
  int64_t c0, c1;   // global cluster range
  int32_t e;        // event
  int32_t pad;
};
inline int64_t chunk_cap(int64_t N, int E) { return N / kChunkCl + E + 1; }

struct EventOut {
  uint8_t* sector;
  float* x_ref;
  float* p;
  float* cov;
  float* chi2;
  int32_t* ndf;
  float* k_prior;
  int32_t* hit_off;
  uint32_t* hit_id;
  int32_t* dbg_up;
  int32_t* dbg_dn;
  int32_t* dbg_cup;
  int32_t* dbg_cdn;
  uint32_t* dbg_start;
  int64_t cap_tracks, cap_hits;
};

// Per-seed refit record (floats): x_ref, p[5], cov[15], chi2, k_prior.
constexpr int kRf = 23;
// Per-seed tracklet state (floats): p[5], cov[15].
constexpr int kTl = 20;

struct Ws {
  // sizes
  int E, S, R;          // events, sectors per event, rows
  int Rh;               // hit-slot rows of a tracklet: R rounded up to a band of 8
  int64_t N;            // clusters (all events)
  int64_t RU;           // row units = E * S * R
  int64_t seed_cap;     // capacity of seed arrays (>= N / min_seed_hits)
  int64_t nb;           // blocks of 256 over N
  // tables
  const EventIn* ev;
  const EventOut* out;
  const float* row_x;   // [R]
  Model m;
  tpcca_params P;
  float tan_a, z_max;   // acceptance: |y| <= x tan_a, |z| <= z_max
  int tracklet_grid;    // workgroups of the tracklet kernel (0 = automatic)
  int taps;             // 1 if some event of the call asks for link or start-hit taps
  const float* cal;     // installed calibration [S delta][S tau][S][8][8] (device), or null
  CalGeo cal_geo;       // geometry of the correction
  uint32_t* flags;      // [F_COUNT]
  const ChunkIn* chunk; // [chunk_cap(N, E)] binning chunks, empty entries past the last
  // binning
  uint32_t* ru_count;   // [RU]
  uint32_t* ru_off;     // [RU + 1]
  uint32_t* cell_cap;   // [RU] cells + 1 per row unit, then scanned -> cell base [RU + 1]
  uint32_t* cell_base;  // [RU + 1]
  GridParams* grid;     // [RU]
  uint32_t* ru_rows;    // [RU] row units of the wave row class from the front, workgroup class from the back
  uint32_t* ru_big;     // [RU] row units of the large row class
  uint32_t* ru_links;   // [RU] same for the small-slab and slab link classes
  float4* tmp4;         // [N] (x, y, z, event-local id bits), bucketed by row unit
  // canonical SoA: (event, sector, row, id) order
  float* cx;
  float* cy;
  float* cz;
  uint32_t* cid;        // event-local cluster id
  uint32_t* cru;        // row unit
  // grid-ordered copy for window searches: (y, z, x, canonical position)
  float4* gbuf;         // [N]
  SearchRec* grec;      // [N] the same entries without x (the tracklet search's records)
  uint16_t* cell_off;   // [kCellsPerCluster N + 2 RU + 1] (grid_cells + 1 per row unit), relative to the
                        // row unit's first entry (rows hold at most TPCCA_MAX_ROW_CLUSTERS < 2^16)
  // links (canonical positions)
  int32_t* up;
  int32_t* dn;
  int32_t* cup;
  float4* cpk;          // [N] (x, y, z, cleaned up-link bits): one load per chain step
  int32_t* cdn;
  uint8_t* flag;        // bit0 start, bit1 seed
  uint32_t* blk_start;  // [nb + 1]
  uint32_t* blk_seed;   // [nb + 1]
  uint32_t* scan_tmp;   // scan partials
  uint32_t* starts;     // [N / 2 + 1] canonical positions
  uint32_t* seeds;      // [seed_cap]
  uint32_t* seed_ev_off;   // [E + 1]
  uint32_t* seed_su_off;   // [E * S + 1] seeds per (event, sector)
  uint32_t* start_ev_off;  // [E + 1]
  // tracklets
  int32_t* tl_nhits;    // [seed_cap]
  int32_t* tl_range;    // [seed_cap] rlo | rhi << 16
  uint64_t* tl_key;     // [seed_cap]
  float* tl_state;      // [seed_cap * kTl]
  int32_t* tl_hits;     // [Rh / 8][seed_cap][8]: band-major hit slots (hit_slot())
  uint64_t* owner;      // [N] (bands above the LDS capacity only)
  uint8_t* own_mask;    // [Rh / 8][seed_cap]: rows of a band whose hit the tracklet owns
  int32_t* tl_own;      // [seed_cap * R] owned hits of accepted tracklets, outermost first
  uint32_t* acc_flag;   // [seed_cap + 1]
  uint32_t* acc_off;    // [seed_cap + 1] scanned acc_flag
  uint32_t* acc_list;   // [seed_cap] accepted seeds
  uint32_t* own_cnt;    // [seed_cap] owned hits of accepted and fitted tracklets
  // selection / refit / output
  float* rf;            // [seed_cap * kRf]
  uint32_t* trk_flag;   // [seed_cap + 1] -> scanned in place
  uint32_t* hit_cnt;    // [seed_cap + 1] -> scanned in place
  int64_t* ev_res;      // [E * 4]: n_tracks, n_hits, n_start, fits
};

// Phase boundaries of one tracking call; events are recorded on the
// caller's stream between the kernels when timing is enabled.
enum Phase : int {
  PH_ZERO = 0, PH_COUNT, PH_SCAN, PH_SCATTER, PH_ROWS, PH_LINKS, PH_CLEAN, PH_COMPACT,
  PH_TRACKLETS, PH_OWNER, PH_REFIT, PH_OUTPUT, PH_N
};
static const char* const kPhaseNames[PH_N] = {
    "zero", "count", "scan", "scatter", "rows", "links", "clean", "compact",
    "tracklets", "owner", "refit", "output"};

struct PhaseEvents {
  hipEvent_t ev[PH_N + 1];
};

// Host-side launchers (tpcca_kernels.hip).
hipError_t run_pipeline(const Ws& w, hipStream_t st, const PhaseEvents* pe = nullptr);
hipError_t fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
// Hit slot of seed s at pad row r: rows in bands of 8, each band holding
// the 8 slots of every seed in turn (a band's slots of consecutive seeds are
// contiguous; four rows of one band are one aligned 16-byte group).
__host__ __device__ inline int64_t hit_slot(int64_t seed_cap, int64_t s, int r) {
  return ((int64_t)(r >> 3) * seed_cap + s) * 8 + (r & 7);
}

hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* part, hipStream_t st);
hipError_t fp32_probe(int op, int64_t n, const float* a, const float* b, float* out, hipStream_t st);

}  // namespace tpcca
