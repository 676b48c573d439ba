/*
 * tpcca_oracle.h -- C interface of the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that
 * the GPU library is checked against.  It shares no code and no header with
 * the GPU path.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.
 *
 * Method (paper, Sec. "Track reconstruction in the TPC"): per-sector
 * cellular-automaton seeding (neighbour finding between clusters on adjacent
 * pad rows, link cleaning, start hits of chains), Kalman-filter tracklet
 * construction and following, tracklet selection and a final Kalman refit.
 * Calibration semantics (Sec. "Approach for online calibration" and
 * Sec. "Overview of HLT online calibration"): the calibration consumes
 * default-transformed clusters joined to the tracks by the unchanged
 * cluster index; here that becomes a chi2(theta) objective with gradient.
 *
 * Every floating-point routine exists in three instantiations: FP32
 * (decision parity with the GPU: same expressions, no contraction), FP64
 * (physics reference) and an FP64 reverse-mode tape type (exact gradient of
 * the FP64 objective).
 */
#ifndef TPCCA_ORACLE_H
#define TPCCA_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_sectors, n_rows;
  const float* row_x;        /* [n_rows] pad-row plane positions, cm */
  float tan_half_angle;      /* sector half-opening tan(10 deg) */
  float z_max;               /* drift length, cm */
  float bz;                  /* solenoid field, tesla */
} orc_geometry;

typedef struct {
  float win_y, win_z;        /* neighbour window half-widths, cm */
  float inv_var_y, inv_var_z;/* 1/(1.5 sigma^2) of the midpoint deviation */
  float link_cut;            /* neighbour score cut */
  float chi2_ext;            /* per-row search cut in tracklet following */
  int32_t max_gap;           /* consecutive empty rows tolerated */
  int32_t min_seed_hits;     /* minimum chain length of a seed */
  int32_t min_hits;          /* minimum hits of a tracklet / track */
  int32_t owned_num, owned_den; /* accept iff den*owned >= num*n_hits */
  float sin_max;             /* |sin phi| limit of the transport */
  float sigma_y, sigma_z;    /* cluster errors, cm */
  float sigma_vertex;        /* vertex pseudo-measurement error, cm */
  float sigma_tgl;           /* external tan(lambda) error */
  float chi2_merge;          /* segment merging: accept a pair iff its match chi2 <= chi2_merge */
  float merge_dist;          /* segment merging: outer hit of the inner segment within this
                                transverse and z distance (cm) of the inner hit of the outer one */
} orc_params;

void orc_default_params(orc_params* p);

/* One transport step x0 -> x1 of state p=(y,z,sin phi,tan lambda,q/pT) and
 * covariance C (upper triangle, 15).  precision is 32 or 64.  Writes the
 * propagated state, covariance and the 5x5 Jacobian (row-major).  Returns 1
 * on success, 0 if |sin phi| would reach sin_max (outputs untouched). */
int orc_transport(int precision, const double p[5], const double C[15], double x0, double x1,
                  double bz, double sin_max, double out_p[5], double out_C[15], double F[25]);

/* One Kalman update with measurement (my, mz), variances (vy, vz).  Writes
 * the filtered state, covariance and the chi2 increment. */
void orc_kf_update(int precision, const double p[5], const double C[15], double my, double mz,
                   double vy, double vz, double out_p[5], double out_C[15], double* dchi2);

/* One Kalman update with a scalar measurement m of state component q
 * (0..4) with variance v (the external tan(lambda) of the calibration
 * objective).  Writes the filtered state, covariance and chi2 increment. */
void orc_kf_update1(int precision, const double p[5], const double C[15], int q, double m,
                    double v, double out_p[5], double out_C[15], double* dchi2);

/* Final fit of an ordered hit list (outermost first): the track refit of the
 * selection step.  Returns 1 on success. */
int orc_fit_hits(int precision, const orc_geometry* g, const orc_params* P, int32_t n,
                 const double* x, const double* y, const double* z, double k0,
                 double p[5], double C[15], double* chi2);

typedef struct {
  int64_t n;                                 /* clusters */
  int64_t *up, *dn;                          /* raw links, cluster ids or -1 */
  int64_t *cup, *cdn;                        /* cleaned links */
  int64_t n_starts; int64_t* starts;         /* all chain heads, (sector,row,id) order */
  int64_t n_seeds;                           /* heads with chain length >= min_seed_hits */
  int64_t* seed_start;                       /* [n_seeds] head cluster id */
  int32_t* seed_nhits;                       /* [n_seeds] tracklet hits (0 if the seed fit failed) */
  uint64_t* seed_key;                        /* [n_seeds] selection key */
  int32_t *seed_rlo, *seed_rhi;              /* row range written */
  int64_t* seed_hits;                        /* [n_seeds * n_rows] cluster id per row or -1 */
  double* seed_state;                        /* [n_seeds * 20]: p[5] then C[15] after following */
  int64_t n_tracks;
  int64_t* trk_seed;                         /* index into the seed arrays */
  int32_t* trk_sector;
  double *trk_xref, *trk_p, *trk_cov, *trk_chi2;   /* [n], [5n], [15n], [n] */
  int32_t* trk_ndf;
  int64_t* hit_off;                          /* [n_tracks + 1] */
  int64_t* hit_ids;                          /* ascending row within a track */
} orc_result;

/* Full per-sector pipeline.  Coordinates are given in FP64 and rounded to
 * the working precision.  sector_mask (optional, [n_sectors]) selects the
 * sectors to process; clusters of other sectors get no links.  Returns 0. */
int orc_track(int precision, const orc_geometry* g, const orc_params* P, int64_t n,
              const double* x, const double* y, const double* z, const int16_t* row,
              const uint8_t* sector, const uint8_t* sector_mask, orc_result** out);
void orc_result_free(orc_result* r);

/* ---- sector track merger (FP64) --------------------------------------------
 * Joins the per-sector track segments of one event that continue each other
 * across the boundary of two adjacent sectors on the same side (see
 * merge_segments for the rules), and refits each joined chain.  Segments are
 * given as the tracking output: sector, x_ref, p[5], cov[15] at the
 * innermost hit, hit lists (cluster ids, ascending row) indexing the
 * clusters (x, y, z, row).  Outputs: link[i] = the outer partner of segment
 * i or -1; per segment the best inner / outer candidate, its match chi2 and
 * the second-best chi2 (inf if none) -- what decides each link; and the
 * merged tracks in out (trk_seed = the index of the chain's innermost
 * segment, sector, x_ref, p, cov, chi2, ndf, hit lists innermost segment
 * first).  seg_slice (NULL for one event): the time-frame slice of each
 * segment; then segments of one sector from neighbouring slices are
 * candidates as well (same frame, no rotation).  Returns 0. */
int orc_merge(const orc_geometry* g, const orc_params* P, int64_t n_clusters, const double* x,
              const double* y, const double* z, const int16_t* row, int64_t n_seg,
              const int32_t* seg_sector, const double* seg_xref, const double* seg_p,
              const double* seg_cov, const double* seg_chi2, const int64_t* seg_hit_off,
              const int64_t* seg_hit_ids, const int32_t* seg_slice, int32_t* link, int32_t* best_in,
              double* chi_in, double* chi_in2, int32_t* best_out, double* chi_out, double* chi_out2,
              orc_result** out);

/* Rotation of a state at plane x from the frame of one sector to a frame
 * turned by dalpha (radians) about z: writes the new plane, state,
 * covariance and the 5x5 Jacobian (row-major).  Returns 1 on success, 0 if
 * |sin phi| in the new frame would reach sin_max.  precision 32 or 64. */
int orc_rotate(int precision, double x, const double p[5], const double C[15], double dalpha, double bz,
               double sin_max, double* out_x, double out_p[5], double out_C[15], double J[25]);

/* ---- calibration (FP64) ---------------------------------------------------
 * theta layout: [0,36) drift scale delta, [36,72) time offset tau (cm),
 * [72, 72+36*64) radial map c[s][a][b] (cm). */
enum { ORC_NPAR = 36 + 36 + 36 * 64 };

/* Apply the calibration correction to default-transformed clusters. */
void orc_calib_apply(const orc_geometry* g, int64_t n, const uint8_t* sector, const double* x,
                     const double* y, const double* z, const double* theta, double* xo,
                     double* zo);

/* The same correction in FP32 as the tracker applies it to its input
 * (corrections added to the coordinates; see calib_point32 for the order of
 * operations).  theta in FP32, same layout. */
void orc_calib_apply32(const orc_geometry* g, int64_t n, const uint8_t* sector, const float* x,
                       const float* y, const float* z, const float* theta, float* xo, float* zo);

/* chi2(theta) of fixed hit lists: refit over the hits (outermost first), then
 * optionally the primary vertex as a measured point and an external
 * tan(lambda).  hit_ids[hit_off[t]..hit_off[t+1]) index the clusters in
 * ascending row order; k0[t] is the frozen q/pT prior; use_vertex[t] enables
 * the vertex and external terms of track t (ext_tgl may be NULL).
 * Writes the total chi2 and ndf, per-track chi2 (optional) and, if grad is
 * not NULL, d chi2 / d theta by reverse-mode differentiation. */
int orc_calib_chi2(const orc_geometry* g, const orc_params* P, int64_t n_clusters,
                   const double* x, const double* y, const double* z, const uint8_t* sector,
                   int64_t n_tracks, const int64_t* hit_off, const int64_t* hit_ids,
                   const double* k0, const double* ext_tgl, const uint8_t* use_vertex,
                   const double* theta, double* chi2, int64_t* ndf, double* trk_chi2,
                   double* grad);

/* ---- ITS standalone tracking (paper, Sec. "Fast ITS standalone tracking"
 * and Sec. "Luminous region estimation based on ITS tracking"; reading R-26)
 * Six layers of flat staves around the beam axis (stave k of layer l: the
 * plane at distance radius[l] whose normal points at (k + 1/2) 2 pi /
 * n_staves[l]); clusters in stave-local (x, y, z).  Steps: SPD vertexer
 * (z histogram of the lines through layer-0/layer-1 pairs, peak, fixed-point
 * mean), tracklets (mutual best layer-0/layer-1 pairs in azimuth and dip
 * from the vertex), Kalman following outward from the vertex as a measured
 * point with multiple scattering per layer (closest cluster of the
 * predicted stave under chi2_cut; at least min_clusters clusters, never two
 * consecutive layers missing), inward Kalman fit to the beam axis, vertex
 * fit with Tukey bi-square weights.  FP32 except the vertex fit (FP64). */
typedef struct {
  int32_t n_layers;          /* 6 */
  float radius[6], half_z[6], x_over_x0[6], sigma_y[6], sigma_z[6];
  int32_t n_staves[6];       /* at most 64 */
  float bz;
} orc_its_geometry;

typedef struct {
  float vtx_sin_phi;         /* SPD pair azimuth window |sin dphi| (vertexer) */
  float vtx_bin, vtx_range;  /* z histogram bin and half range, cm */
  float trk_sin_phi;         /* tracklet azimuth window */
  float trk_dtgl;            /* tracklet dip window (dz/dr from the vertex) */
  float chi2_cut;            /* track-to-cluster chi2 cut in following */
  float sigma_vy, sigma_vz;  /* vertex measurement errors, cm */
  float sin_max;
  int32_t min_clusters;      /* clusters of an accepted track */
  float tukey_c;             /* bi-square cut of the normalised distance */
  int32_t fit_iters;         /* vertex-fit solves */
  float cov_scale_in;        /* inward fit: outward covariance times this */
} orc_its_params;

void orc_its_default_params(orc_its_params* p);

/* One event.  Outputs (caller-allocated): hist[bins], meta[7] = (SPD pairs,
 * peak bin, pairs in the mean, their fixed-point sum, tracklets, vertex z
 * found, vertex fit found), vz; per tracklet t (at most the layer-0
 * clusters): tl0/tl1 (cluster ids), ok, cls[6] (id per layer or -1), ncls,
 * chi2, outward layer/stave/x/p[5]/cov[15], inward ok/stave/p[5]/cov[15]
 * at x = 0; vfit[4] = (x, y, z, sum of weights), vfit_n tracks with weight
 * > 0.  Returns 0. */
int orc_its(const orc_its_geometry* g, const orc_its_params* P, int64_t n, const float* x, const float* y,
            const float* z, const int8_t* layer, const int16_t* stave, int64_t* hist, int64_t* meta, float* vz,
            int32_t* tl0, int32_t* tl1, int32_t* ok, int32_t* cls, int32_t* ncls, float* chi2,
            int32_t* olayer, int32_t* ostave, float* ox, float* op, float* oc, int32_t* iok, int32_t* istave,
            float* ip, float* ic, double* vfit, int32_t* vfit_n);

/* The multiple-scattering covariance increment of one layer (FP32). */
int orc_its_ms(const orc_its_geometry* g, int layer, const float p[5], float C[15]);

#ifdef __cplusplus
}
#endif
#endif
