/*
 * tpcca.h -- C ABI of the MI355X (gfx950) TPC cellular-automaton + Kalman
 * track finder.
 *
 * Source of the method: Rohr et al., "Online Reconstruction and Calibration
 * with feed back loop in the ALICE High Level Trigger" (arXiv:1712.09434).
 *   - Sec. "Track reconstruction in the TPC": a cellular automaton builds
 *     seeds of a handful of hits (five to ten); a Kalman filter then fits and
 *     follows them; one GPU thread per cluster during the cellular automaton
 *     and one per track during following; sectors are processed individually
 *     and their segments merged afterwards; several events share one GPU.
 *   - Sec. "Approach for online calibration" and Sec. "Overview of HLT online
 *     calibration": tracking consumes calibration-transformed clusters; the
 *     calibration consumes default-transformed clusters joined to the tracks
 *     by the unchanged cluster index, and feeds a new map back.
 *   - Sec. "A flat data structure": tracks are shipped as flat, pointer-free
 *     buffers; a TPC track carries at most one cluster per pad row (159).
 *
 * Conventions shared by every call:
 *   - Lengths in cm, field in tesla, momenta in GeV.  Sector-local frame:
 *     x along the sector centre line, y across it, z along the beam.
 *   - A track state is p = (y, z, sin phi, tan lambda, q/pT) at the plane
 *     x = x_ref; its covariance is the packed upper triangle of the 5x5
 *     matrix, row by row (15 floats).
 *   - Cluster ids are positions in the caller's input arrays (0-based, per
 *     event).  They never change between tracking and calibration.
 *   - Buffers are owned by the caller.  `mem` says whether the pointers of a
 *     struct are host (TPCCA_MEM_HOST) or device (TPCCA_MEM_DEVICE) memory.
 *     The library owns only the context and its device workspace, which
 *     grows on demand and is released by tpcca_destroy.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *     Every call returns after the stream has finished the call's work, so
 *     host and device outputs are valid on return.  One context per
 *     concurrently used stream / host thread.
 *   - Return codes: TPCCA_OK, or a negative TPCCA_E_* code; nothing aborts
 *     and nothing throws across this boundary.  tpcca_last_error() gives the
 *     message of the last failure on a context.
 */
#ifndef TPCCA_H
#define TPCCA_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define TPCCA_OK 0
#define TPCCA_E_INVALID (-1)   /* null pointer, bad size, NaN/inf coordinate, row or sector out of range */
#define TPCCA_E_CAPACITY (-2)  /* outputs too small: required sizes written to n_tracks / n_hits */
#define TPCCA_E_DEVICE (-3)    /* HIP runtime error */
#define TPCCA_E_NOMEM (-4)     /* device workspace allocation failed */
#define TPCCA_E_LIMIT (-5)     /* a fixed limit exceeded: a pad row of one sector holds more than
                                  TPCCA_MAX_ROW_CLUSTERS clusters, or a call needs more than the
                                  static scratch of tpcca_refit_grad_noalloc */

#define TPCCA_MEM_HOST 0
#define TPCCA_MEM_DEVICE 1

#define TPCCA_MAX_ROW_CLUSTERS 8192
#define TPCCA_NPAR_PER_SECTOR 66   /* drift scale, time offset, 8x8 radial map */

typedef struct tpcca_ctx tpcca_ctx;

/* Detector geometry (host memory).  n_sectors even: the first half are the
 * z >= 0 (A-side) sectors, the second half the C-side ones.  row_x holds the
 * n_rows pad-row plane positions, strictly increasing. */
typedef struct {
  int32_t n_sectors;        /* 36 */
  int32_t n_rows;           /* 159, at most 255 */
  const float* row_x;       /* [n_rows], cm */
  float tan_half_angle;     /* tan of the sector half-opening angle (10 deg) */
  float z_max;              /* drift length L, cm (250) */
} tpcca_geometry;

/* Uniform solenoid field along z. */
typedef struct {
  float bz_tesla;           /* 0.5 */
} tpcca_field;

/* Tunable constants.  The paper states none of them; the defaults are this
 * library's reading (tpcca_default_params).  */
typedef struct {
  float win_y, win_z;        /* neighbour windows |dy| <= win_y, |dz| <= win_z (2.0, 2.2) */
  float inv_var_y, inv_var_z;/* 1/(1.5 sigma^2) for the midpoint deviation score */
  float link_cut;            /* accept a (down, up) pair iff score <= link_cut (16) */
  float chi2_ext;            /* row search: dy^2/Syy + dz^2/Szz <= chi2_ext (9) */
  int32_t max_gap;           /* stop following after more than max_gap empty rows (8) */
  int32_t min_seed_hits;     /* minimum chain length of a seed (5) */
  int32_t min_hits;          /* minimum hits of a tracklet and a track (10) */
  int32_t owned_num, owned_den; /* accept iff owned_den*owned >= owned_num*n_hits (9, 10) */
  float sin_max;             /* |sin phi| limit of every transport step (0.99) */
  float sigma_y, sigma_z;    /* cluster errors (0.1, 0.15) */
  float sigma_vertex;        /* primary-vertex pseudo-measurement error (0.01) */
  float sigma_tgl;           /* external tan(lambda) error (1e-3) */
  float chi2_merge;          /* segment merging: a pair's match chi2 at most this (50) */
  float merge_dist;          /* segment merging: outer hit of the inner segment within this
                                transverse and z distance of the inner hit of the outer one (20 cm) */
} tpcca_params;

/* Clusters of one event: structure of arrays, n entries each. */
typedef struct {
  int64_t n;
  const float* x;           /* sector-local x (cm); the pad-row plane for an undistorted cluster */
  const float* y;
  const float* z;
  const int16_t* row;       /* pad row, [0, n_rows) */
  const uint8_t* sector;    /* [0, n_sectors) */
  int32_t mem;              /* TPCCA_MEM_HOST or TPCCA_MEM_DEVICE */
  void* stream;             /* hipStream_t the work is enqueued on */
} tpcca_clusters;

/* Track output of one event (flat, pointer-free as shipped), and the input
 * of tpcca_refit_grad.  All arrays are caller-owned, in memory `mem`.
 * Tracks are ordered by their start hit (sector, pad row, cluster id); the
 * hits of a track are in ascending pad row. */
typedef struct {
  int64_t cap_tracks, cap_hits;   /* in: capacities of the arrays below */
  int64_t n_tracks, n_hits;       /* out: counts (required sizes on TPCCA_E_CAPACITY) */
  uint8_t* sector;                /* [cap_tracks] */
  float* x_ref;                   /* [cap_tracks] x of the innermost hit */
  float* p;                       /* [cap_tracks][5] state at x_ref */
  float* cov;                     /* [cap_tracks][15] */
  float* chi2;                    /* [cap_tracks] */
  int32_t* ndf;                   /* [cap_tracks] 2*n_hits - 5 */
  float* k_prior;                 /* [cap_tracks] q/pT at the end of following (optional, NULL = off) */
  int32_t* hit_off;               /* [cap_tracks + 1] */
  uint32_t* hit_id;               /* [cap_hits] cluster ids */
  /* optional parity taps of the seeding steps (NULL = off), indexed by cluster id */
  int32_t* dbg_up;                /* [n] raw up link (cluster id or -1) */
  int32_t* dbg_dn;                /* [n] raw down link */
  int32_t* dbg_cup;               /* [n] cleaned up link */
  int32_t* dbg_cdn;               /* [n] cleaned down link */
  uint32_t* dbg_start;            /* [n] start hits in (sector, row, id) order */
  int64_t n_start;                /* out: number of start hits (valid if dbg_start) */
  /* refit_grad inputs (ignored by tracking) */
  const tpcca_clusters* clusters; /* default-transformed clusters hit_id refers to */
  const float* ext_tgl;           /* [n_tracks] external tan(lambda) (NULL = none) */
  const uint8_t* use_vertex;      /* [n_tracks] 1: add vertex + external terms */
  int32_t mem;
} tpcca_tracks;

/* Calibration parameters theta (FP32): per sector drift-velocity scale
 * delta, time offset tau (cm) and an 8x8 radial displacement map (cm). */
typedef struct {
  const float* drift_scale;       /* [n_sectors] */
  const float* time_offset;       /* [n_sectors] */
  const float* map;               /* [n_sectors][8][8] */
  int32_t mem;
} tpcca_calib;

/* d chi2 / d theta (FP64, deterministic reduction over tracks). */
typedef struct {
  double chi2;                    /* out: total chi2 */
  int64_t ndf;                    /* out */
  double* d_drift_scale;          /* [n_sectors] */
  double* d_time_offset;          /* [n_sectors] */
  double* d_map;                  /* [n_sectors][8][8] */
  int32_t* track_flag;            /* [n_tracks] optional (NULL = off): per-track status, see
                                     TPCCA_TRK_* */
  int32_t mem;
} tpcca_grad;

/* Per-track status of a gradient call (track_flag): the low two bits say
 * what entered chi2, the next bit whether the track lies outside the
 * accuracy domain of the FP32 per-track gradient. */
#define TPCCA_TRK_NOT_FITTED 0    /* fewer than 3 hits, or a transport reached |sin phi| >= sin_max */
#define TPCCA_TRK_HITS 1          /* the hits only (no vertex requested, or its transport refused) */
#define TPCCA_TRK_VERTEX 2        /* the hits, the vertex and (if given) the external tan(lambda) */
#define TPCCA_TRK_SHORT 4         /* fewer than TPCCA_GRAD_MIN_HITS hits (see tpcca_refit_grad) */
#define TPCCA_GRAD_MIN_HITS 40

/* Launch tuning (no effect on results).  ckpt_every: Kalman states kept
 * every that many hit steps by the gradient's forward pass (1..160, default
 * 160); the reverse sweep recomputes the states of each segment but the last
 * from its checkpoint, so at the default (at least a track's step count) no
 * state is recomputed, for 348 x 80 bytes of state per track (each hit
 * step keeps its state before and after the transport);
 * tracklet_grid: workgroups of the persistent tracklet kernel, 0 =
 * automatic; use_graph: 1 = capture the kernel sequence of a tracking call
 * in a hipGraph the first time a workspace shape is seen on a non-null
 * stream and replay it afterwards (default 0). */
typedef struct {
  int32_t ckpt_every;
  int32_t tracklet_grid;
  int32_t use_graph;
} tpcca_tuning;

/* Default constants (host call, no context needed). */
void tpcca_default_params(tpcca_params* p);

/* Create a context for one geometry and field (Sec. "Track reconstruction
 * in the TPC": the tracker is configured once per run).  Copies the row
 * table to the device.  Returns TPCCA_E_INVALID for a bad geometry
 * (n_sectors not even, n_rows not in [3, 255], row_x not increasing,
 * non-positive sizes), TPCCA_E_DEVICE if no HIP device is usable. */
int tpcca_create(const tpcca_geometry* geom, const tpcca_field* field, tpcca_ctx** out);

/* Replace the constants (validated: positive windows, cuts, sigmas,
 * 0 < sin_max < 1, min_seed_hits >= 3, min_hits >= 3). */
int tpcca_set_params(tpcca_ctx* ctx, const tpcca_params* p);
int tpcca_get_params(const tpcca_ctx* ctx, tpcca_params* p);

/* Track one event (Sec. "Track reconstruction in the TPC"): binning per
 * (sector, pad row), neighbour finding on adjacent pad rows, link cleaning,
 * start hits, Kalman tracklet construction, selection and final fit, every
 * sector independent.  On TPCCA_E_CAPACITY the required sizes are in
 * out->n_tracks / out->n_hits and nothing else is written. */
int tpcca_track(tpcca_ctx* ctx, const tpcca_clusters* clusters, tpcca_tracks* out);

/* Install (or, with calib = NULL, remove) a calibration correction of the
 * tracking input (Sec. "Track reconstruction in the TPC": components
 * chained on the GPU so that no data crosses PCIe between them; Sec.
 * "Approach for online calibration": tracking consumes calibration-
 * transformed clusters, the calibration feeds a new map back).  While
 * installed, every tracking call of the context corrects each cluster of
 * sector s on the device, inside binning, before anything else reads it:
 *   z' = z + side (tau_s - delta_s (D - tau_s)),  D = L - side z,
 *   x' = x + sum_a Na (sum_b c_s[a][b] Nb)  (four non-zero cubic B-splines of
 *        each direction at the uncorrected (x, y), as tpcca_refit_grad),
 * in FP32 in exactly this order (side = +1 for the first half of the
 * sectors, -1 otherwise; L = z_max); the pad row is kept.  The library
 * copies theta (host or device memory per calib->mem, read synchronously:
 * device arrays must be complete) into its own device buffer; later changes
 * of the caller's arrays have no effect until the next call.  Returns
 * TPCCA_E_INVALID for null arrays, a bad mem kind or a non-finite value,
 * TPCCA_E_NOMEM if the buffer cannot be allocated. */
int tpcca_set_calib(tpcca_ctx* ctx, const tpcca_calib* calib);

/* Track n_events events together (Sec. "Track reconstruction in the TPC":
 * several events processed concurrently on one GPU to fill it).  Event e is
 * described by events[e] and written to out[e]; the result of every event is
 * identical to tpcca_track on that event alone.  All events must use the
 * same stream.  If any event overflows, every out[e] gets its required sizes
 * and nothing else is written. */
int tpcca_track_batch(tpcca_ctx* ctx, int32_t n_events, const tpcca_clusters* events,
                      tpcca_tracks* out);

/* Sector track merger (Sec. "Track reconstruction in the TPC": sectors are
 * tracked independently and their segments merged afterwards; the refit of
 * the merged tracks runs on the GPU).  segments: the output of tpcca_track
 * for one event (n_tracks, sector, x_ref, p, cov, chi2, ndf, hit_off,
 * hit_id) with segments->clusters the event's clusters (x, y, z, row);
 * all device memory.  Two segments are joined when they continue each
 * other across the boundary of adjacent wedges of one side: the inner one
 * ends on a lower pad row than the outer one starts, its outermost hit lies
 * within params.merge_dist (cm, transverse and z) of the outer one's
 * innermost hit, and its state, transported to its outermost hit, rotated
 * into the outer segment's frame and transported to that segment's
 * reference plane, matches the outer segment's state with
 * Delta^T (C_in + C_out)^-1 Delta <= params.chi2_merge; each segment keeps
 * its best such partner on each side and a link needs both ends to agree.
 * Each chain of linked segments is refitted as one track (outermost hit
 * first, the state rotated into the next segment's frame at each boundary,
 * q/pT prior = the outermost segment's, result at the innermost hit, ndf =
 * 2 n - 5; FP32, the first TPCCA_GRAD_C2_UPDATES updates compensated); a
 * chain whose refit fails stays split.  Output (merged, device memory):
 * tracks in the order of the segments, a chain where its innermost segment
 * was, sector = that segment's, hits innermost segment first (ascending pad
 * row); unmerged segments are copied unchanged.  The output needs
 * cap_tracks >= segments->n_tracks and cap_hits >= the segments' hits (else
 * TPCCA_E_CAPACITY with those sizes in n_tracks / n_hits); on return
 * n_tracks / n_hits hold the merged counts.  seg_link (optional, device,
 * [segments->n_tracks]) receives each segment's outer partner or -1.
 * TPCCA_E_INVALID for host memory, null arrays, a segment with fewer than
 * 3 hits, a bad sector or hit id. */
int tpcca_merge(tpcca_ctx* ctx, const tpcca_tracks* segments, tpcca_tracks* merged, int32_t* seg_link);

/* Time-frame tracking (Sec. "Track reconstruction in the TPC": with
 * continuous readout the TPC delivers time frames of overlapping
 * collisions; a frame is sliced along the time axis, the slices are tracked
 * individually and their track segments merged afterwards).
 * frame: the clusters of one time frame, device memory: x, y, row, sector
 * as for tpcca_track; z holds tau, the readout time since the frame start
 * in drift-length units (cm): for a cluster at z of a collision at time c,
 * tau = c + z_max - side z (side = +1 in the first half of the sectors, -1
 * in the second).  Cluster ids are frame indices.
 * slice_len D (cm, 0 < D <= 2 z_max) and n_slices (1 .. TPCCA_TF_MAX_SLICES):
 * the slice of a cluster is s = floor(tau / D) (FP32 quotient) and must lie
 * in [0, n_slices); slices do not overlap.
 * Each slice is tracked as one event of a batch (tpcca_track_batch) on its
 * clusters in ascending frame order with z' = side (z_max - (tau - s D))
 * (FP32, in that order) in place of z; the segments are taken to frame
 * coordinates (hit ids = frame indices; the z of the state shifted by
 * -side s D, so that a cluster's z is side (z_max - tau)) and merged as by
 * tpcca_merge, where two segments of one sector from neighbouring slices are
 * candidates too (same frame, no rotation).  The installed calibration is
 * not applied (its drift terms need the collision time).
 * Outputs, device memory: merged (required): the merged tracks in frame
 * coordinates, as tpcca_merge writes them; segments (optional, NULL = not
 * returned): the per-slice tracks in frame coordinates, slices ascending;
 * seg_slice, seg_link (optional, [segments]): each segment's slice and outer
 * merge partner (-1 if none).  Both track outputs need cap_tracks >= the
 * number of segments and cap_hits >= their hits; at most n / min_hits +
 * n_slices tracks and n hits.  Otherwise TPCCA_E_CAPACITY with the required
 * counts in n_tracks / n_hits (the tracking was done; only the outputs are
 * missing).  TPCCA_E_INVALID for host memory, null arrays, a bad slice
 * length or count, a non-finite tau or one outside the slices; the errors
 * of tpcca_track otherwise. */
#define TPCCA_TF_MAX_SLICES 1024
int tpcca_track_timeframe(tpcca_ctx* ctx, const tpcca_clusters* frame, float slice_len, int32_t n_slices,
                          tpcca_tracks* merged, tpcca_tracks* segments, int32_t* seg_slice, int32_t* seg_link);

/* Calibration objective and gradient (Sec. "Approach for online
 * calibration"; Sec. "Overview of HLT online calibration"): apply the
 * correction theta to the default-transformed clusters tracks->clusters,
 * refit the fixed hit lists of `tracks` (outermost hit first, q/pT prior
 * tracks->k_prior), add the primary vertex as a measured point and the
 * external tan(lambda) where use_vertex is set, and return the total chi2,
 * its ndf and d chi2/d theta (FP32 per track, FP64 deterministic reduction).
 * tracks->hit_id / hit_off / k_prior / ext_tgl / use_vertex are read for
 * tracks->n_tracks tracks; all of them, the clusters, calib and grad arrays
 * must share one `mem` kind per struct.  Device gradient arrays are written
 * by the kernels, so after an error found on the device (a hit id or sector
 * out of range, more hits than pad rows) they may hold partial values.
 *
 * Accuracy.  Each track is refitted and differentiated in FP32; the first
 * TPCCA_GRAD_C2_UPDATES Kalman updates of a refit, where the nearly
 * diffuse prior makes C - K H C cancel most digits of C, compute the gain
 * and the covariance update in compensated two-float arithmetic (FP32
 * operations only).  For tracks of at least TPCCA_GRAD_MIN_HITS hits the
 * gradient over a calibration set then agrees with exact arithmetic to
 * about 1e-4 (relative, per parameter group).  Shorter tracks are
 * ill-conditioned in FP32: their map gradient is a sum of large per-hit
 * terms that nearly cancel (a common shift of the hits along the track is
 * absorbed by its parameters), and for short, strongly curved segments or
 * long extrapolations to the vertex single tracks can be off by percents.
 * They are computed and summed like the others and reported with
 * TPCCA_TRK_SHORT in track_flag; a calibration set should leave them out. */
#define TPCCA_GRAD_C2_UPDATES 3
int tpcca_refit_grad(tpcca_ctx* ctx, const tpcca_tracks* tracks, const tpcca_calib* calib,
                     tpcca_grad* out);

/* tpcca_refit_grad for callers that cannot allocate memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same results, bit for bit, but its scratch is a
 * static device array of TPCCA_NOALLOC_SCRATCH_BYTES that the library
 * holds on every GPU it runs on until the process ends, and the call makes
 * no device or pinned-host allocation (it does synchronise the stream and
 * read the hit count and the result words into host stack memory).
 * Differences from tpcca_refit_grad:
 *   - tracks, clusters, calib and grad must all be device memory
 *     (TPCCA_MEM_DEVICE), else TPCCA_E_INVALID;
 *   - the checkpoint stride is the largest one up to the tuned ckpt_every
 *     whose workspace fits the scratch (results do not depend on it); if
 *     none fits, TPCCA_E_LIMIT and nothing runs.  Per track the workspace
 *     is 68 bytes per hit plus 5.5 KB (stride 9-12) to 28 KB (stride 160)
 *     of kept states: for tracks of 130 hits the scratch holds about 3,600
 *     of them at stride 160 and about 9,300 at the most compact stride;
 *   - every call on a GPU, from any context, uses that GPU's one array:
 *     calls that overlap in time on one GPU (two streams, two threads)
 *     race and give wrong results.  The array keeps the last call's
 *     contents; each call clears what it needs cleared itself;
 *   - TPCCA_E_DEVICE if the array's device address could not be found
 *     when the context was created. */
#define TPCCA_NOALLOC_SCRATCH_BYTES (128ll << 20)
int tpcca_refit_grad_noalloc(tpcca_ctx* ctx, const tpcca_tracks* tracks, const tpcca_calib* calib,
                             tpcca_grad* out);

/* Debug tap of the last tpcca_track call (host memory): the tracklet of
 * every seed (chain head with at least min_seed_hits links), in start
 * order.  seed_hits is [cap][n_rows] cluster ids or -1; state is
 * [cap][20] (p then cov after following).  Fails with TPCCA_E_CAPACITY if
 * cap is too small (required size in *n_seeds). */
int tpcca_debug_tracklets(tpcca_ctx* ctx, int64_t cap, int64_t* n_seeds, uint32_t* seed_start,
                          int32_t* seed_nhits, int32_t* seed_hits, float* seed_state);

/* Test tap of the FP32 arithmetic the bit-exact decisions rest on (the
 * library's reading of the paper's tracking: integer decisions taken from
 * FP32 values that any IEEE implementation of the same expressions
 * reproduces).  Evaluates, elementwise on the device with the tracking
 * kernels' compile flags, op 0: the correctly rounded square root used for
 * cosines (argument 0, negative, or >= 2^-96), 1: a[i] / b[i], 2: 1 / a[i],
 * 3: the correctly rounded sqrtf(a[i]).  a, b, out are device arrays of n
 * floats (b only for op 1), owned by the caller; work is enqueued on
 * `stream` and finished on return.  TPCCA_E_INVALID for a bad op, size or
 * null pointer, TPCCA_E_DEVICE for a HIP error.  No context needed. */
int tpcca_debug_fp32(int32_t op, int64_t n, const float* a, const float* b, float* out, void* stream);

/* Replace / read the launch tuning of a context (results never change). */
int tpcca_set_tuning(tpcca_ctx* ctx, const tpcca_tuning* t);
int tpcca_get_tuning(const tpcca_ctx* ctx, tpcca_tuning* t);

/* Per-phase timing of tracking calls (HIP events recorded on the caller's
 * stream between the kernels).  tpcca_set_phase_timing(ctx, 1) enables it
 * and clears the accumulators; tpcca_phase_times writes up to cap phase
 * names (static strings) and their accumulated milliseconds, and the number
 * of timed calls; it returns the number of phases. */
int tpcca_set_phase_timing(tpcca_ctx* ctx, int on);
int tpcca_phase_times(const tpcca_ctx* ctx, int32_t cap, const char** names, double* total_ms,
                      int64_t* calls);

const char* tpcca_last_error(const tpcca_ctx* ctx);
void tpcca_destroy(tpcca_ctx* ctx);

/* ---- ITS standalone tracking (Sec. "Fast ITS standalone tracking" and
 * Sec. "Luminous region estimation based on ITS tracking": a fast tracker
 * of the six-layer inner silicon detector for calibration and for the
 * luminous region, and a vertex fit with outlier rejection).
 * Detector: layer l (0 .. 5, innermost first) is a polygon of n_staves[l]
 * flat staves around the beam axis; stave k lies in the plane at distance
 * radius[l] from the axis whose normal points at azimuth (k + 1/2) 2 pi /
 * n_staves[l] and covers |y| <= radius tan(pi / n_staves), |z| <= half_z.
 * Clusters are given in their stave's frame (x = radius, y across, z along
 * the beam); the beam axis is x = y = 0.
 * Steps of one event (all FP32, the vertex fit FP64; the integer decisions
 * are reproducible from the written expressions):
 *   1. SPD vertexer: every layer-0/layer-1 pair with |sin dphi| <=
 *      vtx_sin_phi (same side) gives the z where its line crosses the axis;
 *      histogram of vtx_bin bins over [-vtx_range, vtx_range); the vertex z
 *      is the mean over the fullest bin (ties: lower) and its two
 *      neighbours, summed in fixed point (2^-16 cm);
 *   2. tracklets: layer-0/layer-1 pairs with |sin dphi| <= trk_sin_phi and
 *      |d(dz/dr)| <= trk_dtgl seen from the vertex; a tracklet is a mutual
 *      best pair by (sin dphi / trk_sin_phi)^2 + (d / trk_dtgl)^2 (ties:
 *      lower cluster id), tracklets ordered by their layer-0 cluster id;
 *   3. following: a Kalman filter from the vertex as a measured point
 *      (sigma_vy, sigma_vz) through the tracklet's clusters, then on layers
 *      2 .. 5 the closest cluster of the predicted stave with chi2 <=
 *      chi2_cut; multiple scattering in each layer's average material
 *      (x_over_x0, Highland); a track needs min_clusters clusters and never
 *      two consecutive layers without one;
 *   4. inward fit: from the outward state (covariance times cov_scale_in)
 *      over the track's clusters to the beam axis (x = 0);
 *   5. vertex: the point of least weighted squared distance to the tracks'
 *      straight-line extrapolations at the axis, Tukey bi-square weights
 *      with cut tukey_c on the distance over its error, fit_iters solves. */
typedef struct {
  int32_t n_layers;                  /* 6 */
  float radius[6], half_z[6];        /* cm */
  float x_over_x0[6];                /* average material per layer (radiation lengths) */
  float sigma_y[6], sigma_z[6];      /* cluster resolution, cm */
  int32_t n_staves[6];               /* 1 .. 64 */
  float bz;                          /* tesla */
} tpcca_its_geometry;

typedef struct {
  float vtx_sin_phi, vtx_bin, vtx_range;   /* 0.03, 0.1 cm, 20 cm */
  float trk_sin_phi, trk_dtgl;             /* 0.03, 0.025 */
  float chi2_cut;                          /* 12 */
  float sigma_vy, sigma_vz;                /* 0.005, 0.02 cm */
  float sin_max;                           /* 0.99 */
  int32_t min_clusters;                    /* 4 */
  float tukey_c;                           /* 4.685 */
  int32_t fit_iters;                       /* 8 */
  float cov_scale_in;                      /* 100 */
} tpcca_its_params;

/* One event's clusters, device memory only; ids are positions. */
typedef struct {
  int64_t n;
  const float* x;
  const float* y;
  const float* z;
  const int8_t* layer;
  const int16_t* stave;
  void* stream;
} tpcca_its_clusters;

/* Results of one event.  Arrays (device memory, caller-owned) hold one entry
 * per tracklet (capacity cap; at most the layer-0 clusters); the scalars
 * are written by the call. */
typedef struct {
  int64_t cap;                 /* in: entries of the arrays below */
  int64_t n_tracklets;         /* out (required capacity on TPCCA_E_CAPACITY) */
  int32_t* tl0;                /* [cap] layer-0 cluster id */
  int32_t* tl1;                /* [cap] layer-1 cluster id */
  int32_t* ok;                 /* [cap] 1: accepted track */
  int32_t* cls;                /* [cap][6] cluster id per layer or -1 */
  int32_t* ncls;               /* [cap] */
  float* chi2;                 /* [cap] outward chi2 */
  int32_t* out_layer;          /* [cap] last layer of the outward fit */
  int32_t* out_stave;          /* [cap] its stave */
  float* out_x;                /* [cap] its plane */
  float* out_p;                /* [cap][5] outward state (for matching with the TPC) */
  float* out_cov;              /* [cap][15] */
  int32_t* in_ok;              /* [cap] 1: the inward fit reached the axis */
  int32_t* in_stave;           /* [cap] layer-0 stave of the inward state's frame */
  float* in_p;                 /* [cap][5] state at x = 0 */
  float* in_cov;               /* [cap][15] */
  uint32_t* hist;              /* optional [bins] vertexer histogram (NULL = not returned) */
  /* out: vertexer and vertex fit */
  int64_t n_pairs;             /* SPD pairs in the histogram */
  int32_t peak;                /* fullest bin, -1 if none */
  int32_t vz_ok;
  float vz;
  int32_t vfit_ok;
  int32_t vfit_n;              /* tracks with non-zero weight */
  double vertex[3];
  double vfit_sumw;
} tpcca_its_tracks;

typedef struct tpcca_its_ctx tpcca_its_ctx;
void tpcca_its_default_params(tpcca_its_params* p);
/* TPCCA_E_INVALID for a bad geometry (n_layers != 6, staves outside 1 ..
 * 64, non-positive sizes, radii not increasing). */
int tpcca_its_create(const tpcca_its_geometry* geom, tpcca_its_ctx** out);
int tpcca_its_set_params(tpcca_its_ctx* ctx, const tpcca_its_params* p);
/* TPCCA_E_INVALID for null arrays, non-finite coordinates or a layer /
 * stave out of range; TPCCA_E_CAPACITY (required count in n_tracklets)
 * when the arrays hold fewer than the tracklets. */
int tpcca_its_track(tpcca_its_ctx* ctx, const tpcca_its_clusters* cl, tpcca_its_tracks* out);
/* n_events events in one pass over the chip (ITS events are small; the
 * paper's data-parallel processing of many events at once): events[e] and
 * outs[e] as in tpcca_its_track, ids local to each event, every event's
 * results equal to those of tpcca_its_track on that event alone.  All
 * events name the same stream (TPCCA_E_INVALID otherwise); the call returns
 * after the stream has finished the work.  Fewer than 2^31 clusters in all.
 * On TPCCA_E_CAPACITY every event's n_tracklets holds its required count;
 * on any error no event's results are valid. */
int tpcca_its_track_batch(tpcca_its_ctx* ctx, int32_t n_events, const tpcca_its_clusters* events,
                          tpcca_its_tracks* outs);
const char* tpcca_its_last_error(const tpcca_its_ctx* ctx);
void tpcca_its_destroy(tpcca_its_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
