/*
 * tpc_track.h -- C ABI of the MI355X (gfx950) TPC sector tracker.
 *
 * Method: Rohr et al., "ALICE HLT TPC Tracking of Pb-Pb Events on GPUs".
 * Section 1 defines the steps run here, all on the GPU in hand-written HIP:
 *   neighbours finder -> evolution step -> chains of one-to-one links ->
 *   tracklet construction (Kalman fit, extrapolation, chi^2 condition,
 *   refit) -> tracklet selection.
 * Section 3.1 defines the cluster weight w = n (alpha - chi^2/beta) that
 * decides which tracklet keeps a shared cluster; section 3.2 the sorted track
 * output; section 5 the 30-cluster minimum of a sector track.
 *
 * Conventions
 *  - Units cm, GeV, Tesla.  Sector-local frame: x along the sector's centre
 *    line (pad rows at fixed x), y across it, z along the beam.
 *  - Track state at a row: (y, z, sin phi, tan lambda, q/pT), phi the angle
 *    to the local x axis.  Curvature kappa = 0.00299792458 * Bz * q/pT.
 *  - Clusters of an event are one structure-of-arrays, sorted by
 *    (sector slot, row); the order inside a row is free.  Cluster indices in
 *    every output are event-global int32 indices into that array.
 *  - The device path computes in FP32, except the Kalman filter's covariance
 *    and gain, which are FP64 (a diffuse q/pT prior makes the FP32 covariance
 *    update lose precision on low-pT tracks).
 *
 * Pointers: every array inside tpc_event and tpc_tracks is DEVICE memory on
 * the context's GPU; tpc_geometry.row_x, tpc_params and the size fields
 * tpc_tracks.n_tracks / n_track_clusters are HOST memory.  The caller owns
 * all of them; the library keeps no pointer after a call returns.
 *
 * Errors: every call returns TPC_OK (0) or a TPC_ERR_* code and never throws;
 * tpc_last_error() gives a message for the calling thread.
 *
 * Threads: a context may be used by one thread at a time.  Calls that share
 * a context are serialised by the caller.
 */
#ifndef TPC_TRACK_H
#define TPC_TRACK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TPC_OK = 0,
  TPC_ERR_INVALID_ARG = 1, /* bad sizes, null pointers, bad offsets or params */
  TPC_ERR_CAPACITY = 2,    /* output arrays too small; required sizes written */
  TPC_ERR_OOM = 3,         /* device memory beyond the context budget */
  TPC_ERR_DEVICE = 4,      /* a HIP call failed */
  TPC_ERR_OVERFLOW = 5,    /* internal tracklet buffer too small after retry */
  TPC_ERR_BUSY = 6         /* server: event not admitted now, try again */
};

#define TPC_MAX_ROWS 160

typedef struct tpc_ctx tpc_ctx;

/* Pad-row geometry of one sector (section 1: 159 rows per sector). */
typedef struct {
  int32_t n_rows;        /* rows per sector, 3 .. TPC_MAX_ROWS */
  const float* row_x;    /* HOST [n_rows]: local x of each row, strictly increasing */
  float tan_half_angle;  /* sector half opening: a row spans |y| <= x*tan_half_angle */
  float z_max;           /* drift length: |z| <= z_max */
} tpc_geometry;

/* One event (section 1: 2 x 18 trapezoidal sectors tracked independently). */
typedef struct {
  int32_t n_sectors;          /* sector slots in this event (1 .. 4096) */
  const int32_t* sector_id;   /* DEVICE [n_sectors]: physical sector of each slot,
                                 copied to the output only */
  int64_t n_clusters;         /* 0 .. 2^31 - 1 */
  const float* y;             /* DEVICE [n_clusters] local y */
  const float* z;             /* DEVICE [n_clusters] z */
  const int32_t* row_offsets; /* DEVICE [n_sectors*n_rows + 1]: row (s, r) holds
                                 clusters [off[s*n_rows + r], off[s*n_rows + r + 1]);
                                 off[0] = 0, off[last] = n_clusters, non-decreasing.
                                 Violations are detected on the device and return
                                 TPC_ERR_INVALID_ARG. */
} tpc_event;

/* Constants of the method.  alpha = 6 (section 3.1) and min_clusters = 30
 * (section 5) are the paper's; it gives no values for the others. */
typedef struct {
  float sigma_y, sigma_z;   /* cluster resolution (cm) */
  float nf_win_y, nf_win_z; /* neighbours finder: |dy|, |dz| window on rows k+-1 */
  float nf_chi2_max;        /* neighbours finder: straight-line chi^2 cut */
  int32_t min_seed_len;     /* shortest chain of one-to-one links used as a seed */
  int32_t seed_window;      /* the seed circle uses the first, middle and last of the
                               first min(m, seed_window) chain clusters (>= 2) */
  float chi2_gate;          /* construction: chi^2 condition for collecting a cluster */
  int32_t max_miss;         /* construction: stop after more consecutive empty rows */
  float max_sinphi;         /* construction: |sin phi| limit */
  float alpha, beta;        /* weight w = n (alpha - (chi2/ndf)/beta) */
  int32_t min_clusters;     /* pre-cut for competing and final cut on owned clusters */
  float min_pt;             /* low-momentum cut (GeV), not applied when Bz == 0 */
  float prior_sinphi, prior_tanl, prior_qpt; /* initial variances of the fit */
  int32_t max_tracklets;    /* tracklet reservation, 0 = automatic (grown on overflow) */
} tpc_params;

/* Caller-allocated outputs. */
typedef struct {
  int32_t cap_tracks;          /* rows of track_par / track_meta */
  int32_t cap_track_clusters;  /* length of track_cluster */
  int32_t* n_tracks;           /* HOST out: number of tracks (also on CAPACITY) */
  int32_t* n_track_clusters;   /* HOST out: clusters in all tracks (also on CAPACITY) */
  float* track_par;            /* DEVICE [cap_tracks][8]: x, y, z, sinphi, tanl, q/pT
                                  at the innermost collected cluster, chi2, ndf */
  int32_t* track_meta;         /* DEVICE [cap_tracks][4]: sector_id, n_clusters,
                                  first (offset into track_cluster), seed id */
  int32_t* track_cluster;      /* DEVICE [cap_track_clusters]: cluster indices,
                                  row-ascending per track */
  int32_t* cluster_track;      /* DEVICE [n_clusters]: track index or -1 */
} tpc_tracks;

/* Fill p with the default constants. */
void tpc_params_default(tpc_params* p);

/* Host-only argument checks of tpc_track_event (sizes, pointers, geometry,
 * parameters); touches no device memory and needs no GPU.  Device-side
 * checks (offsets, non-finite coordinates) happen in tpc_track_event. */
int tpc_validate(const tpc_event* ev, const tpc_geometry* geo, const tpc_params* params);

/* Create a context on HIP device `device` that may hold up to
 * hbm_budget_bytes of scratch memory (0 = no limit).  Scratch is allocated on
 * first use and grows as needed. */
int tpc_ctx_create(int device, size_t hbm_budget_bytes, tpc_ctx** out);
void tpc_ctx_destroy(tpc_ctx* ctx);

/* Track one event (sections 1, 3.1, 3.2).  All kernels are enqueued on
 * hip_stream (a hipStream_t, NULL = default stream); the call returns after
 * the stream has finished this event, with tracks sorted by (sector slot,
 * seed id) and each track's clusters in row order.
 * Returns TPC_ERR_CAPACITY with *n_tracks / *n_track_clusters set when the
 * outputs are too small (their contents are then unspecified). */
int tpc_track_event(tpc_ctx* ctx, const tpc_event* ev, const tpc_geometry* geo, float bz_tesla,
                    const tpc_params* params, tpc_tracks* out, void* hip_stream);

/* ---- allocation-free variant ----------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * tpc_track_event with the same arguments, outputs and results, except that
 * its scratch is a static array of TPC_NOALLOC_SCRATCH_BYTES per GPU (held
 * by the library until the process ends, its address resolved by
 * tpc_ctx_create) instead of the context's arena: the call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine).  The scratch of an
 * event is about 130 B per cluster (a central event of 1.33 M clusters:
 * about 175 MB); an event whose scratch does not fit returns TPC_ERR_OOM.
 * Every call on a GPU shares that GPU's array, so calls that overlap on one
 * GPU (from different contexts or streams) race: serialise them. */
#define TPC_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int tpc_track_event_noalloc(tpc_ctx* ctx, const tpc_event* ev, const tpc_geometry* geo,
                            float bz_tesla, const tpc_params* params, tpc_tracks* out,
                            void* hip_stream);

/* Track n_events events in one launch sequence (sections 1, 3.1, 3.2): the
 * events' sectors are tracked side by side and each event's tracks, cluster
 * lists and cluster->track map are written to its own outputs[i], exactly as
 * tpc_track_event would write them for that event alone (indices are the
 * event's own).  events[i] and outputs[i] follow the rules of
 * tpc_track_event.  Returns TPC_ERR_CAPACITY if any event's outputs are too
 * small (every event's sizes are written; contents of those events are
 * unspecified), TPC_ERR_INVALID_ARG if any event is invalid. */
int tpc_track_batch(tpc_ctx* ctx, const tpc_event* events, int n_events, const tpc_geometry* geo,
                    float bz_tesla, const tpc_params* params, tpc_tracks* outputs,
                    void* hip_stream);

/* ---- global tracking (section 5) ----------------------------------------
 * A sector track needs min_clusters clusters, so a short piece of a track
 * beyond a sector edge is not found by the sector tracker.  Global tracking
 * prolongs the ends of the sector tracks that leave their sector through a
 * side edge: the end state is rotated into the neighbouring sector's frame
 * and the construction continues there on the clusters no sector track owns.
 * Reading of the paper's short description:
 *   - both ends of every track are tried: the inner one from the inward fit
 *     at its innermost cluster, the outer one from the outward filter at its
 *     outermost cluster; helix steps away from the track through the own
 *     sector's rows (no search) find the row where it leaves the trapezoid
 *     (first/last row, |sin phi| > max_sinphi or |z| > z_max: no
 *     prolongation);
 *   - the neighbour is the sector on that side in the same half of the
 *     2 x 18 layout (sector_id 0-17 and 18-35; index +1 mod 18 for y > 0,
 *     -1 for y < 0), the event's first slot with that id; slots with other
 *     ids are not prolonged;
 *   - the state at the last row inside is rotated by one sector width
 *     (2 atan(tan_half_angle)) and the extension continues from the first
 *     row beyond its x, in the same direction, with the construction's
 *     chi^2 gate and miss limit, taking only clusters whose cluster_track is
 *     -1;
 *   - a cluster collected by several prolongations goes to the one with the
 *     smallest (seed id, end); a prolongation is reported if it owns at
 *     least one cluster.
 * Sector tracks and cluster_track are exactly those of tpc_track_event. */
typedef struct {
  int32_t cap;            /* rows of par / meta */
  int32_t cap_clusters;   /* length of cluster */
  int32_t* n;             /* HOST out: number of prolongations (also on CAPACITY) */
  int32_t* n_clusters;    /* HOST out: clusters owned by them (also on CAPACITY) */
  float* par;             /* DEVICE [cap][8]: x, y, z, sinphi, tanl, q/pT at the last
                             collected cluster, in the frame of the sector entered;
                             chi2 of its updates; ndf = 2 x clusters collected */
  int32_t* meta;          /* DEVICE [cap][5]: track index, end (0 inner, 1 outer),
                             sector_id entered, n_clusters owned, first (offset
                             into cluster) */
  int32_t* cluster;       /* DEVICE [cap_clusters]: owned clusters in the order
                             collected (away from the track) */
} tpc_prolongations;

/* tpc_track_event followed by global tracking.  Prolongations are ordered by
 * (track index, end).  Returns TPC_ERR_CAPACITY with the sizes set when the
 * track or the prolongation outputs are too small (*pro->n and
 * *pro->n_clusters are 0 when the tracks did not fit). */
int tpc_track_event_global(tpc_ctx* ctx, const tpc_event* ev, const tpc_geometry* geo,
                           float bz_tesla, const tpc_params* params, tpc_tracks* out,
                           tpc_prolongations* pro, void* hip_stream);

/* ---- track merger with refit (section 1: the merger follows the sector
 * tracker; section 3.3: it refits each track from its cluster list, so the
 * same clusters give the same fit whatever the sector tracker computed).
 * Reading of the paper, which describes no more:
 *   - the outer end of track A (outward filter at its outermost cluster) is
 *     joined to the inner end of track B (inward fit at its innermost
 *     cluster) in a side neighbour of A's sector or in its membrane partner
 *     (same index, other half of the 2 x 18 layout), if B's innermost cluster
 *     is farther from the beam axis than A's outermost: A's end, rotated into
 *     B's frame and propagated to B's x, and B's end are independent, so
 *     chi^2 = d^T (C_A + C_B)^-1 d over the five parameters; A and B are
 *     linked if chi^2 <= merge_chi2 and each is the other's best candidate
 *     (smallest chi^2, then smallest track index); links form chains (a
 *     closed one starts at its smallest track);
 *   - a joined track's list in path order: the inner prolongation of its
 *     first track (reversed), each track's own clusters, the outer
 *     prolongation of its last track (prolongations only with global
 *     tracking);
 *   - the refit (also tpc_refit): seed circle of the first run of >= 3
 *     consecutive clusters of one sector with increasing rows (first, middle,
 *     last of its first min(m, seed_window)), outward Kalman filter to the end
 *     of the list, inward fit from the last cluster with a fresh covariance
 *     over the whole list; between sectors the state is rotated by whole
 *     sector widths; a cluster whose step fails is skipped; fewer than three
 *     fitted clusters, or a list over several sectors with an id outside
 *     0-35, fail (par zero). */
typedef struct {
  int32_t cap;            /* rows of par / meta */
  int32_t cap_clusters;   /* length of cluster */
  int32_t* n;             /* HOST out: joined tracks (also on CAPACITY) */
  int32_t* n_clusters;    /* HOST out: clusters in their lists (also on CAPACITY) */
  float* par;             /* DEVICE [cap][8]: x, y, z, sinphi, tanl, q/pT at the innermost
                             fitted cluster, in the frame of sector meta[0]; chi2; ndf
                             (0 = the refit failed) */
  int32_t* meta;          /* DEVICE [cap][5]: sector_id of par's frame, tracks joined,
                             n_clusters, first (offset into cluster), first track */
  int32_t* cluster;       /* DEVICE [cap_clusters]: cluster lists in path order */
  int32_t* track_merged;  /* DEVICE [cap_tracks of the tracks]: joined track of each track */
} tpc_merged;

/* tpc_track_event (and global tracking if pro is not NULL), then the merger.
 * Joined tracks are ordered by their first track.  TPC_ERR_CAPACITY with the
 * sizes set when an output is too small (later stages report 0 then). */
int tpc_track_event_merged(tpc_ctx* ctx, const tpc_event* ev, const tpc_geometry* geo,
                           float bz_tesla, const tpc_params* params, float merge_chi2,
                           tpc_tracks* out, tpc_prolongations* pro, tpc_merged* mrg,
                           void* hip_stream);

/* The merger's refit of caller-given cluster lists of an event: list i is
 * clusters[offsets[i] .. offsets[i+1]) (DEVICE offsets [n_lists + 1], DEVICE
 * clusters [n_entries]; offsets are clamped to [0, n_entries], cluster
 * indices outside the event fail that list).  par (DEVICE [n_lists][8]) and
 * frame_sector (DEVICE [n_lists], may be NULL: sector_id of par's frame, -1
 * if the refit failed) as in tpc_merged.  The event is validated as in
 * tpc_track_event. */
int tpc_refit(tpc_ctx* ctx, const tpc_event* ev, const tpc_geometry* geo, float bz_tesla,
              const tpc_params* params, int32_t n_lists, int32_t n_entries,
              const int32_t* offsets, const int32_t* clusters, float* par,
              int32_t* frame_sector, void* hip_stream);

/* Stage-by-stage access for checks (same kernels as tpc_track_event).
 * Runs the neighbours finder and the evolution step and copies the link
 * arrays into DEVICE buffers of n_clusters int32 each (any may be NULL):
 * up/dn before evolution, up2/dn2 after it. */
int tpc_debug_links(tpc_ctx* ctx, const tpc_event* ev, const tpc_geometry* geo,
                    const tpc_params* params, int32_t* up, int32_t* dn, int32_t* up2,
                    int32_t* dn2, void* hip_stream);

/* Runs the path up to tracklet construction and copies the tracklets into
 * DEVICE buffers: seeds [cap] (start cluster of each tracklet, increasing),
 * hits [cap][n_rows] (cluster per row or -1, valid on [row_lo, row_hi]),
 * row_lo, row_hi, n (0 = dropped), ndf [cap] int32, chi2 [cap] float,
 * par [cap][6] float (x, y, z, sinphi, tanl, q/pT).  *n_tracklets (HOST)
 * receives the count; TPC_ERR_CAPACITY if it exceeds cap. */
int tpc_debug_tracklets(tpc_ctx* ctx, const tpc_event* ev, const tpc_geometry* geo,
                        float bz_tesla, const tpc_params* params, int32_t cap,
                        int32_t* n_tracklets, int32_t* seeds, int32_t* hits, int32_t* row_lo,
                        int32_t* row_hi, int32_t* n, int32_t* ndf, float* chi2, float* par,
                        void* hip_stream);

/* ---- tuning --------------------------------------------------------------
 * Knobs that change speed, never results (every setting gives bitwise the
 * same outputs). */
typedef struct {
  int32_t use_graph;        /* tpc_track_batch captures its launch sequence in a HIP
                               graph and replays it for later batches of the same
                               shape (number of events, sector slots, capacity) */
  int32_t construct_blocks; /* tracklet-construction grid in workgroups of 64 lanes,
                               rounded up to a multiple of 8 (one share per XCD);
                               0 = sized from the tracklet reservation; a smaller
                               grid makes workgroups loop over the work */
  float bin_occupancy;      /* target clusters per bin of the per-row search grids
                               (1 .. 64; a row never gets more bins than clusters) */
  int32_t construct_schedule; /* 0 = one lane per tracklet, each at its own row,
                                 tracklets taken from a queue;
                                 1 = row-synchronous: a workgroup walks the rows of
                                 one sector in lockstep for up to 64 of its
                                 tracklets, the searched row staged in LDS */
  int32_t construct_lanes;    /* lane schedule: lanes of each 64-lane wave that take
                                 tracklets (1 .. 64); fewer lanes per wave shorten
                                 each wave's steps at the cost of more waves;
                                 0 = automatic (one per 16k clusters up to 0.3 M,
                                 at least 1, then with the square root of the
                                 clusters: 24 at 0.5 M, 40 at 1.3 M, 64 from 4 M) */
  int32_t nf_stage;           /* neighbours finder's LDS stage: 1 = rows of up to 512
                                 clusters, 12 window candidates per lane and row
                                 (five workgroups per CU); 2 = rows of up to 1024
                                 clusters, 32 candidates, eight waves (two per CU);
                                 3 = rows of
                                 up to 256 clusters, one wave per row slot (fourteen
                                 per CU), and one wave per row slot for the grid,
                                 evolution and seed kernels too; larger rows take the
                                 global-memory search;
                                 0 = automatic (2 when the event or batch averages
                                 more than 320 clusters per row, 3 when a batch of
                                 32768 row slots or more averages fewer than 128,
                                 else 1) */
  int32_t own_order;          /* selection's launch order: 1 = every sector's first
                                 workgroups first; 2 = a sector's workgroups one
                                 after another (they share its tracklets' rows in
                                 the caches); 0 = automatic (2 for more than 144
                                 sectors of 64k clusters or more on average, else 1) */
} tpc_tuning;
void tpc_tuning_default(tpc_tuning* t);
int tpc_ctx_set_tuning(tpc_ctx* ctx, const tpc_tuning* t);
/* Number of HIP-graph replays done by this context (for checks). */
int tpc_ctx_graph_launches(tpc_ctx* ctx, int64_t* n);

/* ---- measurement -------------------------------------------------------
 * Kernels of one event are numbered 0 .. tpc_kernel_count()-1 in launch
 * order; tpc_kernel_name(i) names them.  With a non-zero mask, later calls
 * record a HIP event pair on the call's stream around each selected kernel
 * (bit i = kernel i) and add the elapsed time to per-kernel totals. */
int tpc_kernel_count(void);
const char* tpc_kernel_name(int i);
int tpc_ctx_set_timing(tpc_ctx* ctx, uint32_t kernel_mask);
/* Totals since the last reset: kernel_ms / kernel_launches [tpc_kernel_count()]
 * and work[5] = events, tracklets, constructor helix steps, Kalman updates,
 * candidate clusters tested (any pointer may be NULL). */
int tpc_ctx_get_stats(tpc_ctx* ctx, double* kernel_ms, int64_t* kernel_launches, int64_t* work);
int tpc_ctx_reset_stats(tpc_ctx* ctx);

/* ---- serving -------------------------------------------------------------
 * Continuous batching.  Events arrive one by one in HOST memory; an event is
 * admitted when its device footprint (about 160 B per cluster) fits the
 * budget still free, is staged and uploaded at once, and is tracked by the
 * next free worker together with every other uploaded event (at most
 * max_batch; an event that finds a worker idle is tracked alone by the
 * per-event path of tpc_track_event, without the batch's gather and scatter).  n_workers workers, each with its own context and stream, keep
 * that many batches in flight, so uploads, tracking and downloads of
 * different events overlap.  Each event's tracks are exactly those
 * tpc_track_event gives it alone.  One worker with max_batch = 1 is the
 * plain one-event-at-a-time path. */
typedef struct tpc_server tpc_server;
typedef struct {
  int32_t device;
  size_t hbm_budget_bytes;  /* admission budget for resident events */
  int32_t max_batch;        /* events per launch sequence (>= 1) */
  int32_t n_workers;        /* launch sequences in flight (1 .. 16) */
  int32_t use_graph;        /* replay captured launch sequences */
  int32_t keep_results;     /* copy tracks back for tpc_server_fetch */
} tpc_server_config;
typedef struct {
  uint64_t tag;
  int32_t status;           /* TPC_OK or the error of the event's batch */
  int32_t n_tracks, n_track_clusters;
  double t_submit, t_done;  /* tpc_server_now() clock: submit entry, results on host */
} tpc_server_done;
void tpc_server_config_default(tpc_server_config* cfg);
int tpc_server_create(const tpc_server_config* cfg, const tpc_geometry* geo, float bz_tesla,
                      const tpc_params* params, tpc_server** out);
/* host_event: the fields of tpc_event, all HOST pointers (copied before return).
 * TPC_ERR_BUSY: not admitted now (try again after completions). */
int tpc_server_submit(tpc_server* srv, const tpc_event* host_event, uint64_t tag);
/* Up to max finished events (waits up to timeout_ms for the first one). */
int tpc_server_poll(tpc_server* srv, tpc_server_done* done, int max, int* n_done,
                    int timeout_ms);
/* Copies a polled event's results into HOST buffers sized by its counts
 * (track_par [n][8], track_meta [n][4], track_cluster, cluster_track
 * [n_clusters]; any may be NULL) and releases them. */
int tpc_server_fetch(tpc_server* srv, uint64_t tag, float* track_par, int32_t* track_meta,
                     int32_t* track_cluster, int32_t* cluster_track);
int tpc_server_stats(tpc_server* srv, int64_t* batches, int64_t* events, size_t* resident_bytes);
double tpc_server_now(void);
const char* tpc_server_last_error(void);
void tpc_server_destroy(tpc_server* srv);

/* Message of the last failed call on this thread ("" if none). */
const char* tpc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TPC_TRACK_H */
