// timeframe_internal.hpp -- workspace of time-frame tracking (not ABI).
#pragma once
#include "internal.hpp"

namespace tpcca {

constexpr int kTfBlock = 1024;        // clusters per workgroup of the slicing kernels
constexpr int kTfMaxSlices = 1024;
static_assert(kTfMaxSlices == TPCCA_TF_MAX_SLICES, "slice limit of the ABI");

// Slicing of a frame: slice s = floor(tau / D) (FP32 quotient), stable
// partition of the clusters by slice, z' = side (L - (tau - s D)) per
// cluster in slice order, z_tf = side (L - tau) in frame order.
struct TfSlice {
  int64_t n;
  const float* x;
  const float* y;
  const float* tau;
  const int16_t* row;
  const uint8_t* sector;
  float D, L;
  int n_slices, half, S;
  int64_t nb;            // workgroups of kTfBlock clusters
  uint32_t* cnt;         // [n_slices * nb + 1] per (slice, workgroup) counts, then their exclusive scan
  uint32_t* err;         // [1] bit 0: non-finite tau or a slice outside [0, n_slices)
  uint32_t* soff;        // [n_slices + 1] first cluster of each slice (slice order)
  float* sx;             // [n] slice order
  float* sy;
  float* sz;             // z'
  int16_t* srow;
  uint8_t* ssec;
  uint32_t* sid;         // frame index of each slice-order cluster
  float* ztf;            // [n] frame order
};

// Per-slice tracking outputs (capacity layout) to one contiguous segment
// set in frame coordinates.
struct TfRange {
  int64_t tcap;          // first track slot of the slice in the per-slice buffers
  int64_t hoff;          // first hit_off entry of the slice (tcap + slice index)
  int64_t hcap;          // first hit slot of the slice
  int64_t tout, hout;    // first track and hit of the slice in the contiguous set
  int64_t coff;          // first cluster of the slice (slice order)
};

struct TfGather {
  int E;                 // slices
  int half;
  float D;
  int64_t T, H;          // segments, hits
  const TfRange* tab;    // [E + 1] (tout / hout of entry E: the totals)
  const uint8_t* isec;
  const float* ixref;
  const float* ip;
  const float* icov;
  const float* ichi2;
  const int32_t* indf;
  const int32_t* ihoff;
  const uint32_t* ihid;
  const uint32_t* sid;
  uint8_t* osec;
  float* oxref;
  float* op;
  float* ocov;
  float* ochi2;
  int32_t* ondf;
  int32_t* ohoff;        // [T + 1]
  uint32_t* ohid;
  int32_t* oslice;
};

hipError_t tf_slice(const TfSlice& a, uint32_t* scan_part, hipStream_t st);
hipError_t tf_gather(const TfGather& g, hipStream_t st);

}  // namespace tpcca
