/*
 * tpc_oracle.h -- plain, slow, FP64 CPU reference of the TPC sector tracker
 * (Rohr et al., "ALICE HLT TPC Tracking of Pb-Pb Events on GPUs").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the oracle that the GPU path is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * All floating-point work is done in double precision.  Inputs are the same
 * FP32 cluster coordinates the GPU path reads, widened exactly to double.
 *
 * Conventions: cm, GeV, Tesla.  A track state at local x is
 *   p = (y, z, sin(phi), tan(lambda), q/pT)
 * with phi the direction angle to the local x axis (cos(phi) > 0) and
 * curvature kappa = 0.00299792458 * Bz * q/pT (1/cm); d(phi)/ds = -kappa.
 *
 * Every function returns 0 on success and a negative value on bad arguments.
 * All pointers are host pointers owned by the caller.
 */
#ifndef TPC_ORACLE_H
#define TPC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Tunable constants of the method.  alpha (chi^2-suppression factor, section
 * 3.1) and min_clusters (shortest sector track, section 5) come from the paper;
 * the paper gives no values for the others. */
typedef struct {
  double sigma_y, sigma_z;      /* cluster resolution (cm) */
  double nf_win_y, nf_win_z;    /* neighbour search window (cm) */
  double nf_chi2_max;           /* straight-line cut of the neighbours finder */
  int32_t min_seed_len;         /* shortest link chain that becomes a tracklet */
  int32_t seed_window;          /* the seed uses the first min(m, seed_window) chain clusters */
  double chi2_gate;             /* per-cluster chi^2 gate of the extension */
  int32_t max_miss;             /* extension stops after more consecutive misses */
  double max_sinphi;            /* |sin(phi)| limit of the propagation */
  double alpha, beta;           /* cluster weight w = n (alpha - (chi2/ndf)/beta) */
  int32_t min_clusters;         /* pre-cut and final cut on the cluster count */
  double min_pt;                /* low-momentum cut (GeV), ignored when Bz == 0 */
  double prior_sinphi, prior_tanl, prior_qpt;   /* initial variances */
} orc_params;

typedef struct {
  int32_t n_rows;               /* pad rows per sector (159) */
  const float* row_x;           /* [n_rows] local x of each row, increasing */
  float tan_half_angle;         /* tan(10 deg): |y| <= x*tan_half_angle */
  float z_max;                  /* drift length (cm) */
} orc_geometry;

typedef struct {
  int32_t n_sectors;            /* sector slots in this event */
  const int32_t* sector_id;     /* [n_sectors] physical sector of each slot */
  int64_t n_clusters;
  const float* y;               /* [n_clusters] local y */
  const float* z;               /* [n_clusters] z */
  const int32_t* row_offsets;   /* [n_sectors*n_rows + 1] */
} orc_event;

typedef struct {
  int32_t cap_tracks, cap_track_clusters;   /* in: capacities */
  int32_t n_tracks, n_track_clusters;       /* out: sizes (also when too small) */
  double* track_par;    /* [cap_tracks][8]: x, y, z, sinphi, tanl, qpt, chi2, ndf */
  int32_t* track_meta;  /* [cap_tracks][4]: sector_id, n_clusters, first, seed_id */
  int32_t* track_cluster;   /* [cap_track_clusters] cluster indices, row-ascending */
  int32_t* cluster_track;   /* [n_clusters] track index or -1 */
} orc_tracks;

/* Per-tracklet results of the construction step (arrays of n_tracklets). */
typedef struct {
  int32_t* hits;        /* [n_tracklets][n_rows]: cluster per row or -1 */
  int32_t* row_lo;      /* innermost collected row */
  int32_t* row_hi;      /* outermost collected row */
  int32_t* n;           /* collected clusters; 0 marks a dropped tracklet */
  double* chi2;         /* chi^2 of the final (inward) fit */
  int32_t* ndf;         /* 2n - 5 */
  double* par;          /* [n_tracklets][6]: x, y, z, sinphi, tanl, qpt at row_lo */
} orc_tracklets;

void orc_params_default(orc_params* p);

/* Whole method on one event.  Sectors are independent and are spread over
 * n_threads threads (<= 0: one).  Returns 1 if the track capacities are too
 * small (sizes are still reported, nothing else is written). */
int orc_track_event(const orc_event* ev, const orc_geometry* geo, double bz,
                    const orc_params* prm, orc_tracks* out, int n_threads);

/* ---- global tracking (section 5) ----------------------------------------
 * Prolongation of sector tracks that leave their sector through a side edge
 * into the neighbouring sector (reading in tpc_oracle.c).  Prolongations are
 * ordered by (track index, end) and each holds the free clusters it owns. */
typedef struct {
  int32_t cap, cap_clusters;   /* in: capacities */
  int32_t n, n_clusters;       /* out: sizes (also when too small) */
  double* par;      /* [cap][8]: x, y, z, sinphi, tanl, qpt at the last collected
                       cluster, in the frame of the sector entered; chi2; ndf */
  int32_t* meta;    /* [cap][5]: track index, end (0 inner, 1 outer), sector_id
                       entered, n_clusters, first */
  int32_t* cluster; /* [cap_clusters]: cluster indices in the order met */
} orc_prolongations;

/* orc_track_event, then the prolongation of its tracks.  Returns 1 if a
 * capacity is too small (sizes reported). */
int orc_track_event_global(const orc_event* ev, const orc_geometry* geo, double bz,
                           const orc_params* prm, orc_tracks* out,
                           orc_prolongations* pro, int n_threads);

/* ---- track merger with refit ---------------------------------------------
 * Joins the sector tracks of one particle (outer end of one to the inner end
 * of a track in a neighbouring or membrane-partner sector) and refits every
 * joined track from its cluster list alone (reading in tpc_oracle.c). */
typedef struct {
  int32_t cap, cap_clusters;   /* in: capacities */
  int32_t n, n_clusters;       /* out: sizes (also when too small) */
  double* par;        /* [cap][8]: x, y, z, sinphi, tanl, qpt at the innermost fitted
                         cluster (frame of its sector), chi2, ndf (0: refit failed) */
  int32_t* meta;      /* [cap][5]: sector_id of that frame, tracks joined, n_clusters,
                         first, first track of the chain */
  int32_t* cluster;   /* [cap_clusters]: clusters in path order */
  int32_t* track_merged;  /* [cap_tracks of the tracks]: joined track of each track */
} orc_merged;

/* orc_track_event_global (pro may be NULL: no prolongations), then the
 * merger.  Joined tracks are ordered by their first track.  Returns 1 if a
 * capacity is too small. */
int orc_track_event_merged(const orc_event* ev, const orc_geometry* geo, double bz,
                           const orc_params* prm, double merge_chi2, orc_tracks* out,
                           orc_prolongations* pro, orc_merged* mrg, int n_threads);

/* The merger's refit of cluster lists: list i is clusters[offsets[i] ..
 * offsets[i+1]) in path order; par [n_lists][8] as orc_merged.par,
 * frame_sector [n_lists] (may be NULL) the sector_id of par's frame or -1. */
int orc_refit(const orc_event* ev, const orc_geometry* geo, double bz, const orc_params* prm,
              int32_t n_lists, const int32_t* offsets, const int32_t* clusters, double* par,
              int32_t* frame_sector);

/* Rotation of a state (and covariance, may be NULL) at x into a frame turned
 * by d radians.  Returns 1 if the direction would not point along the new
 * x axis. */
int orc_rotate(double x, const double* st, const double* cov, double d, double bz,
               double* x_out, double* st_out, double* cov_out);

/* ---- individual steps, for stage-by-stage checks ---------------------- */

/* Neighbours finder (section 1): up/dn links of every cluster, -1 = none. */
int orc_neighbours(const orc_event* ev, const orc_geometry* geo,
                   const orc_params* prm, int32_t* up, int32_t* dn);

/* Straight-line chi^2 of cluster c with lower neighbour d and upper neighbour
 * u (event-global indices).  Returns a negative value if d/c/u are not on
 * consecutive rows of one sector. */
double orc_nf_chi2(const orc_event* ev, const orc_geometry* geo,
                   const orc_params* prm, int32_t d, int32_t c, int32_t u);

/* Evolution step (section 1): keep reciprocal links only. */
int orc_evolve(int64_t n_clusters, const int32_t* up, const int32_t* dn,
               int32_t* up2, int32_t* dn2);

/* Chain starts with at least min_seed_len clusters, in increasing index order.
 * Returns the number of seeds, or -1 if it exceeds cap. */
int64_t orc_seeds(const orc_event* ev, const orc_geometry* geo,
                  const orc_params* prm, const int32_t* up2, const int32_t* dn2,
                  int32_t* seeds, int64_t cap);

/* Tracklet construction (section 1) of the given seeds along the given links. */
int orc_construct(const orc_event* ev, const orc_geometry* geo, double bz,
                  const orc_params* prm, const int32_t* up2,
                  int64_t n_seeds, const int32_t* seeds, orc_tracklets* tl);

/* Weights, cluster assignment and selection (sections 1 and 3.1).  qpt is
 * tl->par[.][5].  weights (may be NULL) replaces the computed cluster weight
 * of each tracklet, so that a caller can decide the ownership with weights
 * evaluated in another precision.  owner[c] = index of the owning tracklet or
 * -1; keep[t] = 1 for the tracklets that become tracks. */
int orc_select(const orc_event* ev, const orc_geometry* geo, double bz,
               const orc_params* prm, int64_t n_tl, const int32_t* ids,
               const orc_tracklets* tl, const double* weights, int32_t* owner,
               int32_t* keep);

/* ---- fit pieces on explicit double-precision hits (tests only) ---------- */

/* Exact helix step of state st (5) and covariance cov (5x5 row-major) from x1
 * to x2.  Writes the Jacobian (5x5, may be NULL).  Returns 0, or 1 when
 * |sin(phi)| would exceed max_sinphi (state unchanged). */
int orc_propagate(double x1, double* st, double* cov, double x2, double bz,
                  double max_sinphi, double* jac);

/* Fit of a fixed list of hits (x increasing) the way a tracklet made of one
 * link chain covering them is fitted: three-point seed, outward filter,
 * inward refit (the seed from the first seed_window hits).  Outputs the state and covariance at x[0], chi^2, ndf.
 * Returns 0, or 1 if the propagation left |sin(phi)| <= max_sinphi. */
int orc_fit_hits(int32_t n, const double* x, const double* y, const double* z,
                 double bz, const orc_params* prm, double* st, double* cov,
                 double* chi2, int32_t* ndf);

#ifdef __cplusplus
}
#endif
#endif /* TPC_ORACLE_H */
