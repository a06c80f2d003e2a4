// Internal interface between the host runtime (tpc_runtime.cpp) and the
// kernels (tpc_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tpc_track.h"

namespace tpc {

// Per-call constants, passed by value as a kernel argument (no copies needed).
struct KParams {
  float row_x[TPC_MAX_ROWS];
  int32_t n_rows;
  float tan_half, z_max, bz, k_curv;  // k_curv = 0.00299792458 * bz
  float sigma_y, sigma_z, sy2, sz2;
  float nf_win_y, nf_win_z, nf_chi2_max;
  int32_t min_seed_len;
  int32_t seed_window;
  float chi2_gate;
  int32_t max_miss;
  float max_sinphi;
  float alpha, beta;
  int32_t min_clusters;
  float max_qpt;  // 1 / min_pt
  float prior_sinphi, prior_tanl, prior_qpt;
  float bin_occupancy;     // target clusters per search-grid bin
  int32_t construct_blocks;  // constructor grid (0 = sized from the reservation)
  int32_t construct_schedule;  // 0 = one lane per tracklet, 1 = row-synchronous
  int32_t nf_stage;            // neighbours finder's LDS stage: 1 = 512 clusters, four waves;
                               // 2 = 1024 clusters; 3 = 256 clusters, one wave per row slot
  int32_t row_wave;            // grid, evolution and seed kernels: one wave per row slot
  int32_t construct_lanes;     // lane schedule: lanes of a wave that take tracklets
  int32_t own_chunk;           // selection: clusters per LDS chunk of a sector (speed only)
  int32_t own_by_sector;       // selection: a sector's workgroups consecutive in launch order
  int32_t n_cu;                // compute units of the device (launch sizing only)
  int32_t expect_tl;           // tracklets expected (launch sizing only)
  float rot_c, rot_s;          // cos, sin of one sector width (global tracking)
  float rot_tab[18][2];        // cos, sin of k sector widths, k = -9 .. 8 at [k + 9]
  float merge_chi2;            // track merger: chi^2(5) cut of a join
};

struct DevEvent {
  const float* y;
  const float* z;
  const int32_t* ro;
  const int32_t* sector_id;
  int32_t n_sectors;
  int32_t n_clusters;
  const int32_t* n_dev;  // if set, the cluster count is read here (graph replays)
};

// One cluster in grid order: coordinates and event index in one 16-byte load.
struct __attribute__((aligned(16))) GridRec {
  float y, z;
  int32_t id, pad;
};

// Per-row search grid: clusters of a row counting-sorted into ny x nz bins.
struct RowGrid {
  float y0, z0, iby, ibz;
  int32_t ny, nz, bin_base, n;
};

enum Counter {
  C_ERR = 0,        // error bits
  C_NONFINITE = 1,  // clusters with a non-finite coordinate
  C_SEEDS = 2,      // tracklets found (may exceed the reservation)
  C_TRACKS = 3,
  C_TRACK_CLUSTERS = 4,
  C_STEPS = 5,      // constructor: helix steps taken
  C_UPDATES = 6,    // constructor: Kalman updates
  C_CANDS = 7,      // constructor: candidate clusters tested against the gate
  C_QUEUE = 8,      // constructor: next tracklet to hand out, one per XCD group (8..15)
  C_COUNT = 16
};
enum ErrBits { E_OFFSETS = 1, E_NONFINITE = 2, E_TL_OVERFLOW = 4, E_CAPACITY = 8 };

constexpr int kHitStride = 160;  // per-tracklet row slots (>= n_rows, padded)
constexpr int kEndStride = 40;   // floats per tracklet end state (x, 5 state, flag, pad, 15 FP64 cov, pad)
constexpr int kLayoutSectors = 36;  // 2 x 18 sectors: ids 0-17 and 18-35

// Device scratch of one event.
struct Scratch {
  int32_t* counters;       // [C_COUNT]
  RowGrid* grid;           // [R]
  int32_t* bins;           // [N + R + 1]
  GridRec* g_rec;          // [N] grid order: y, z, event index
  int32_t *up, *dn;        // [N]
  int32_t *up2, *dn2;      // [N]
  uint8_t* start;          // [N]
  unsigned long long* own; // [N] owner key per cluster
  int32_t* row_cnt;        // [R + 1] seeds per row, then exclusive offsets
  int32_t* row_part;       // [R / kRowSpan + 1] sums of spans of row_cnt
  int32_t cap_tl;          // tracklet reservation T
  int32_t* seeds;          // [T]
  int32_t* seed_rs;        // [T]
  int32_t* hits;           // [T * kHitStride]
  float2* hit_yz;          // [T * kHitStride] coordinates of collected clusters
  int32_t *row_lo, *row_hi, *n, *ndf;  // [T]
  float* chi2;             // [T]
  float* par;              // [T * 6]
  unsigned long long* key; // [T]
  int32_t *owned, *kept;   // [T]
  int32_t *trk_idx, *trk_off; // [T]
  int32_t* span_sum;       // [2 * spans]: kept / owned sums per span of tracklets
  float* ends;             // [T][2][kEndStride] inner / outer end states, or null
                           // (recorded only for global tracking)
};

// Device scratch of global tracking (section 5): one prolongation slot per
// (tracklet, end), slot = 2 * tracklet + end.
struct GlobalScratch {
  int32_t* counters;   // [C_COUNT]: C_SEEDS = slots, C_TRACKS / C_TRACK_CLUSTERS = output
                       // prolongations / clusters, C_ERR copied from the sector tracker
  int32_t* p2s;        // [kLayoutSectors] first slot of each physical sector, or -1
  int32_t* claim;      // [N] smallest slot that collected the cluster
  int32_t* n;          // [2T] clusters collected (0 = no prolongation)
  int32_t* nslot;      // [2T] sector slot entered
  float* par;          // [2T][8] x, state at the last collected cluster, chi2, ndf
  int32_t* hit;        // [2T][kHitStride] clusters in the order met
  int32_t* act;        // [2T] slots of the kept tracklets, in track order
  int32_t *owned, *kept, *idx, *off;  // [2T] clusters owned, reported, output index/offset
  int32_t* span_sum;   // scan partials
};

// Device scratch of the track merger, indexed by track (at most T tracks).
struct MergeScratch {
  int32_t* counters;    // [C_COUNT]: C_SEEDS = tracks, C_TRACKS / C_TRACK_CLUSTERS = joined
                        // tracks / clusters, C_ERR from the sector tracker
  int32_t* first;       // [S + 1] first track of each sector slot
  float4* sum;          // [T][2] inner end of each track: x, y, tanl, q/pT; var tanl, var
                        // q/pT, radius, valid
  int32_t *next, *best; // [T]
  unsigned long long* prev_key;  // [T] best predecessor: chi^2 bits << 32 | track
  int32_t* prev;        // [T]
  int32_t *cnt, *nseg, *kept, *idx, *off;  // [T] per chain head
  int32_t* span_sum;
  int32_t* loff;        // [T + 1] offsets of the joined tracks' lists
  int32_t* rowslot;     // [N] row slot of each cluster (refit)
  float4* rec;          // [cap_rec] list entries gathered for the refit: y, z, row slot
  int32_t cap_rec;
};

struct MergeOutputs {
  int32_t cap, cap_clusters;
  float* par;           // [cap][8]
  int32_t* meta;        // [cap][5]: frame sector id, tracks joined, n_clusters, first, first track
  int32_t* cluster;     // [cap_clusters]
  int32_t* track_merged;  // [tracks]
};

struct ProOutputs {
  int32_t cap, cap_clusters;
  float* par;        // [cap][8]
  int32_t* meta;     // [cap][5]: track, end, sector id, n_clusters, first
  int32_t* cluster;  // [cap_clusters]
};

struct Outputs {
  int32_t cap_tracks, cap_track_clusters;
  float* track_par;
  int32_t* track_meta;
  int32_t* track_cluster;
  int32_t* cluster_track;
};

// One event of a batch: the caller's device arrays and outputs, and where the
// event sits in the concatenated batch.
struct BatchEventDesc {
  const float* y;
  const float* z;
  const int32_t* ro;
  const int32_t* sector_id;
  int32_t n_clusters, n_sectors;
  int32_t cbase, sbase;  // first cluster / first sector slot of the event in the batch
  float* track_par;
  int32_t* track_meta;
  int32_t* track_cluster;
  int32_t* cluster_track;
  int32_t cap_tracks, cap_track_clusters;
};

// Device buffers of a batch: the concatenated event and its outputs.
struct BatchBuffers {
  float* y;
  float* z;
  int32_t* ro;          // [S*n_rows + 1]
  int32_t* sector_id;   // [S]
  float* par;           // [cap_tracks][8]
  int32_t* meta;        // [cap_tracks][4]
  int32_t* tcl;         // [N]
  int32_t* ctr;         // [N]
  int32_t cap_tracks;
  int32_t* ev_counts;   // [E][2]: tracks, track clusters of each event
  BatchEventDesc* desc; // [E]
  int32_t* hdr;         // [4]: total clusters of the batch (read by graph replays)
};

// Clears the counters, then gathers the events (so that it can flag bad offsets).
hipError_t enqueue_batch_gather(const BatchBuffers& bb, const Scratch& sc, int n_events,
                                int n_rows, int n_total, int s_total, hipStream_t st);
hipError_t enqueue_batch_scatter(const BatchBuffers& bb, const Scratch& sc, int n_events,
                                 hipStream_t st);

// Static scratch of the allocation-free entry point (one array per device).
constexpr size_t kStaticScratchBytes = TPC_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
// Resolves the array's address on `device`, which must be current; once per
// device, later calls return at once.
hipError_t static_scratch_init(int device);
// The device address of the array on `device`, or null before static_scratch_init.
void* static_scratch(int device);

size_t scratch_bytes(int64_t n_clusters, int64_t n_rowslots, int64_t cap_tl);
// Global tracking: the end states (Scratch::ends) and GlobalScratch.
size_t global_bytes(int64_t n_clusters, int64_t cap_tl);
void global_carve(void* base, int64_t n_clusters, int64_t cap_tl, float** ends,
                  GlobalScratch* gs);
void scratch_carve(void* base, int64_t n_clusters, int64_t n_rowslots, int64_t cap_tl,
                   Scratch* sc);

// Kernels of one event, in launch order (index into timing tables).
enum KernelId {
  K_ZERO, K_GRID, K_NF, K_EVO, K_SCAN_ROWS, K_SEED_WRITE, K_CONSTRUCT, K_OWN,
  K_TL_REDUCE, K_TL_SCAN, K_OUTPUT,
  // global tracking
  K_PRO_INIT, K_ENDS, K_PROLONG, K_PRO_OWN, K_PRO_REDUCE, K_PRO_SCAN, K_PRO_OUTPUT,
  // track merger with refit
  K_MRG_INIT, K_MRG_MATCH, K_MRG_LINK, K_MRG_CHAIN, K_MRG_REDUCE, K_MRG_SCAN, K_MRG_WRITE,
  K_ROWMAP, K_REFIT_GATHER, K_REFIT, K_NUM
};
extern const char* const kKernelNames[K_NUM];

// Optional HIP events recorded around selected kernels (mask bit = KernelId).
struct KernelTimer {
  uint32_t mask = 0;
  hipEvent_t ev[K_NUM][2] = {};
};

// Stage groups; each enqueues its kernels on `st` and returns the first error.
enum Stage { STAGE_GRID = 0, STAGE_LINKS = 1, STAGE_SEEDS = 2, STAGE_TRACKLETS = 3, STAGE_ALL = 4 };
hipError_t enqueue_event(const DevEvent& ev, const KParams& kp, const Scratch& sc,
                         const Outputs& out, int upto, hipStream_t st,
                         const KernelTimer* timer = nullptr, bool zero_counters = true);
// Global tracking after enqueue_event(STAGE_ALL) with Scratch::ends set:
// prolongs the event's tracks (reads the tracker's cluster_track output);
// with po == nullptr only the end states are prepared (for the merger).
// part: 0 = the end states only, 1 = the prolongations only, -1 = both.
hipError_t enqueue_global(const DevEvent& ev, const KParams& kp, const Scratch& sc,
                          const Outputs& out, const GlobalScratch& gs, const ProOutputs* po,
                          hipStream_t st, const KernelTimer* timer = nullptr, int part = -1);
// The track merger with refit, after enqueue_global; po as given to it.
size_t merge_bytes(int64_t n_clusters, int64_t n_sectors, int64_t cap_tl, int64_t cap_rec);
void merge_carve(void* base, int64_t n_clusters, int64_t n_sectors, int64_t cap_tl,
                 int64_t cap_rec, MergeScratch* ms);
// part: 0 = the joins (need only the end states, so they may run beside the
// prolongations), 1 = chains, lists and refits (need the prolongations),
// -1 = both.
hipError_t enqueue_merge(const DevEvent& ev, const KParams& kp, const Scratch& sc,
                         const Outputs& out, const GlobalScratch& gs, const ProOutputs* po,
                         const MergeScratch& ms, const MergeOutputs& mo, hipStream_t st,
                         const KernelTimer* timer = nullptr, int part = -1);
// The merger's refit of caller-given cluster lists (after STAGE_GRID, which
// validates the event): list i = clusters[offsets[i] .. offsets[i+1]),
// offsets clamped to [0, n_entries].
hipError_t enqueue_refit(const DevEvent& ev, const KParams& kp, const Scratch& sc,
                         const MergeScratch& ms, int32_t n_lists, int32_t n_entries,
                         const int32_t* offsets, const int32_t* clusters, float* par,
                         int32_t* frame, hipStream_t st, const KernelTimer* timer = nullptr);

}  // namespace tpc
