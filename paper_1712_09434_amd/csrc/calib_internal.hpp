// calib_internal.hpp -- workspace of the calibration gradient (not ABI).
#pragma once
#include "calib_device.hpp"
#include "internal.hpp"

namespace tpcca {

constexpr int kPart = 68;                       // per-track partials: 66 parameters, chi2, pad
constexpr int kNPar = TPCCA_NPAR_PER_SECTOR;    // 66 per sector
constexpr int kChunk = 256;                     // tracks per first-level reduction chunk
constexpr int kTail = 28;                       // state slots of the steps to the vertex (<= kTail - 2 steps)
constexpr int kFirstC2 = TPCCA_GRAD_C2_UPDATES;   // hit updates 1..kFirstC2 of a refit in two-float arithmetic
constexpr int kMinAccurateHits = TPCCA_GRAD_MIN_HITS;

struct CalWs {
  int S, R;
  CalGeo geo;              // the correction's geometry (drift length, radial range, sector angle)
  Model m;
  float sv2, st2;          // vertex and external tan(lambda) variances
  int K;                   // checkpoint stride (hit steps)
  int nck, nseg;           // checkpoints and state slots per track: 2K for a segment of hit
                           // steps (each step's state before and after its transport),
                           // then kTail for the steps to the vertex
  int64_t T, H, NC;        // tracks, hits, clusters
  const int32_t* hit_off;
  const uint32_t* hit_id;
  const float* k_prior;
  const float* ext_tgl;    // may be null
  const uint8_t* use_vertex;  // may be null
  const float* cx;
  const float* cy;
  const float* cz;
  const uint8_t* csec;
  const float* dl;
  const float* tau;
  const float* map;
  float* hx;
  float* hy;
  float* hz;
  float* gx;               // [H] dx-derivative of the step ending at the hit
  float* gy;
  float* gz;
  float* gpt;              // [H] x-adjoint point terms (seed chord, vertex hop)
  float4* bva;             // [H] the four non-zero x-direction B-splines at the hit
  float4* bvb;             // [H] the four non-zero y/x-direction B-splines at the hit
  int32_t* bsp;            // [H] index of the first of each four: x in bits 0-7, y/x in 8-15
  float* dzt;              // [H] drift term (L - side z) - tau of the hit (0 if invalid)
  float* part;             // [T][kPart]
  int32_t* tflag;          // [T] 0 failed, 1 hits only, 2 with vertex terms
  int32_t* tndf;           // [T]
  int32_t* flag_out;       // [T] per-track status for the caller (may be null)
  float* ckpt;             // [T][nck][20]
  float* seg;              // [T][nseg][20]
  double* chunk;           // [nchunk][S*66 + 1]
  double* out;             // [S*66 + 1]: per sector (delta, tau, map[64]), then chi2
  double* g_dl;            // device gradient outputs [S], [S], [S][64]; null for host outputs
  double* g_tau;
  double* g_map;
  unsigned long long* ndf_sum;
  uint32_t* err;
};

hipError_t run_calib(const CalWs& c, hipStream_t st);

}  // namespace tpcca
