// Host runtime of the C ABI (include/tpc_track.h): argument validation,
// device scratch arena, launch of the per-event kernel sequence, overflow
// retry and error reporting.  No exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "tpc_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(TPC_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

struct tpc_ctx {
  int device = 0;
  int n_cu = 0;             // compute units of the device
  size_t budget = 0;        // 0 = unlimited
  void* arena = nullptr;
  size_t arena_bytes = 0;
  int32_t* h_counters = nullptr;  // pinned: sector tracker's, global tracking's, merger's counters
  void* glob_arena = nullptr;     // global tracking scratch
  size_t glob_bytes = 0;
  // the merger's joins run beside the prolongations on a second stream
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  double seen_ratio = 0.0;     // tracklets per cluster of the last call (launch sizing)
  double learned_ratio = 0.0;  // tracklets per cluster learned from overflows: the
                               // reservation scales with the event (or batch) size
  tpc::KernelTimer timer;   // HIP events around selected kernels
  bool timer_ready = false;
  double kernel_ms[tpc::K_NUM] = {};
  int64_t kernel_launches[tpc::K_NUM] = {};
  int64_t work[5] = {};     // events, tracklets, helix steps, updates, candidates
  // batches
  void* batch_arena = nullptr;
  size_t batch_bytes = 0;
  void* h_batch = nullptr;  // pinned: descriptors out, per-event counts back
  size_t h_batch_bytes = 0;
  tpc_tuning tuning{};  // set by tpc_ctx_create (tpc_tuning_default)
  // captured batch launch sequence and what it was captured for
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  uint64_t graph_key = 0;
  int64_t graph_ncap = 0;
  int64_t graph_launches = 0;
  hipStream_t graph_stream = nullptr;  // capture is not allowed on the legacy default stream
  hipEvent_t graph_dep = nullptr;
};

namespace tpc {

// Host-side checks of everything that can be checked without touching device
// memory.  Offsets and coordinates are checked on the device.
int validate(const tpc_event* ev, const tpc_geometry* geo, const tpc_params* p) {
  if (!ev || !geo || !p) return fail(TPC_ERR_INVALID_ARG, "null event, geometry or params");
  if (geo->n_rows < 3 || geo->n_rows > TPC_MAX_ROWS)
    return fail(TPC_ERR_INVALID_ARG, "n_rows %d outside [3, %d]", geo->n_rows, TPC_MAX_ROWS);
  if (!geo->row_x) return fail(TPC_ERR_INVALID_ARG, "row_x is null");
  for (int r = 0; r < geo->n_rows; ++r) {
    if (!std::isfinite(geo->row_x[r]) || geo->row_x[r] <= 0.f)
      return fail(TPC_ERR_INVALID_ARG, "row_x[%d] not finite and positive", r);
    if (r && !(geo->row_x[r] > geo->row_x[r - 1]))
      return fail(TPC_ERR_INVALID_ARG, "row_x not strictly increasing at %d", r);
  }
  if (!(geo->tan_half_angle > 0.f) || !std::isfinite(geo->tan_half_angle))
    return fail(TPC_ERR_INVALID_ARG, "tan_half_angle must be positive");
  if (!(geo->z_max > 0.f) || !std::isfinite(geo->z_max))
    return fail(TPC_ERR_INVALID_ARG, "z_max must be positive");
  if (ev->n_sectors < 1 || ev->n_sectors > 4096)
    return fail(TPC_ERR_INVALID_ARG, "n_sectors %d outside [1, 4096]", ev->n_sectors);
  if (ev->n_clusters < 0 || ev->n_clusters > 0x7fffffffLL)
    return fail(TPC_ERR_INVALID_ARG, "n_clusters %lld outside [0, 2^31-1]",
                (long long)ev->n_clusters);
  if ((int64_t)ev->n_sectors * geo->n_rows + ev->n_clusters + 1 > 0x7fffffffLL)
    return fail(TPC_ERR_INVALID_ARG, "event too large for int32 indexing");
  if (!ev->row_offsets || !ev->sector_id)
    return fail(TPC_ERR_INVALID_ARG, "row_offsets or sector_id is null");
  if (ev->n_clusters > 0 && (!ev->y || !ev->z)) return fail(TPC_ERR_INVALID_ARG, "y or z is null");
  auto pos = [](float v) { return std::isfinite(v) && v > 0.f; };
  if (!pos(p->sigma_y) || !pos(p->sigma_z)) return fail(TPC_ERR_INVALID_ARG, "sigma must be > 0");
  if (!pos(p->nf_win_y) || !pos(p->nf_win_z)) return fail(TPC_ERR_INVALID_ARG, "nf window must be > 0");
  if (!(p->nf_chi2_max >= 0.f)) return fail(TPC_ERR_INVALID_ARG, "nf_chi2_max must be >= 0");
  if (p->min_seed_len < 2 || p->min_seed_len > geo->n_rows)
    return fail(TPC_ERR_INVALID_ARG, "min_seed_len must be in [2, n_rows]");
  if (p->seed_window < 2) return fail(TPC_ERR_INVALID_ARG, "seed_window must be >= 2");
  if (!pos(p->chi2_gate)) return fail(TPC_ERR_INVALID_ARG, "chi2_gate must be > 0");
  if (p->max_miss < 0) return fail(TPC_ERR_INVALID_ARG, "max_miss must be >= 0");
  if (!(p->max_sinphi > 0.f && p->max_sinphi < 1.f))
    return fail(TPC_ERR_INVALID_ARG, "max_sinphi must be in (0, 1)");
  if (!std::isfinite(p->alpha) || !std::isfinite(p->beta) || p->beta == 0.f)
    return fail(TPC_ERR_INVALID_ARG, "alpha must be finite, beta finite and non-zero");
  if (p->min_clusters < 3) return fail(TPC_ERR_INVALID_ARG, "min_clusters must be >= 3");
  if (!pos(p->min_pt)) return fail(TPC_ERR_INVALID_ARG, "min_pt must be > 0");
  if (!pos(p->prior_sinphi) || !pos(p->prior_tanl) || !pos(p->prior_qpt))
    return fail(TPC_ERR_INVALID_ARG, "prior variances must be > 0");
  if (p->max_tracklets < 0) return fail(TPC_ERR_INVALID_ARG, "max_tracklets must be >= 0");
  return TPC_OK;
}

// Lanes per wave of the lane-schedule constructor.  Its time is the critical
// path of the longest tracklets; a wave with fewer lanes takes shorter steps
// (fewer scattered loads and phases per step) as long as the waves do not
// queue on the SIMDs.  Automatic (0): a multiple of four in [8, 64] that
// grows with the square root of the expected number of tracklets (one per
// 36 clusters).
static int32_t lanes_per_wave(int32_t requested, int64_t n_clusters) {
  if (requested > 0) return requested;
  // measured best: about one lane per 16k clusters up to 0.27 M (1 to 2 at
  // 17k to 33k, 4 at 67k, 8 at 0.13 M, 16 to 20 at 0.27 M: a small event's
  // tracklets never fill the chip, and the fewer lanes a wave has, the
  // shorter its steps), then the square-root rule: 24 to 32 at 0.53 M, 40
  // for a central event (1.3 M; 32 and 36 within 1.5%), 64 for 4.6 M
  const double waves = (double)(n_clusters / 36 + 1) / 2048.0;
  const int32_t a = 4 * (int32_t)std::lround(2.2 * std::sqrt(waves) + 0.5);
  const int64_t lin = n_clusters / 16384;
  return (int32_t)std::max<int64_t>(1, std::min<int64_t>(std::min(64, std::max(8, a)), lin));
}

// Clusters per chunk of the selection's LDS argmax: smaller chunks give more
// workgroups to a sector of a central event, larger ones read the
// tracklets' headers fewer times in a dense sector (measured: 2048 below 64k
// clusters per sector, else 4096).  Speed only.
static int32_t own_chunk(int64_t n_clusters, int64_t n_rowslots, int32_t n_rows) {
  const int64_t sectors = std::max<int64_t>(1, n_rowslots / std::max<int32_t>(1, n_rows));
  return n_clusters / sectors < 65536 ? 2048 : 4096;
}
// The selection's launch order (speed only): by sector when many dense
// sectors (more than four events' worth, 64k clusters or more each) make
// many rounds of workgroups, so that the workgroups of a sector run together
// and share its tracklets' headers and hit rows in the caches; otherwise
// every sector's first workgroups first, which puts the busy ones of sparse
// sectors (fewer chunks than workgroups) together.
static int32_t own_by_sector(int32_t order, int64_t n_rowslots, int32_t n_rows, int32_t chunk) {
  if (order != 0) return order == 2 ? 1 : 0;
  const int64_t sectors = n_rowslots / std::max<int32_t>(1, n_rows);
  return chunk == 4096 && sectors > 144 ? 1 : 0;
}

// Mean clusters per row slot of an event or batch (speed only: every form of
// the per-row kernels gives the same results).
static int64_t row_mean(int64_t n_clusters, int64_t n_rowslots) {
  return n_clusters / (n_rowslots > 0 ? n_rowslots : 1);
}
// Many sparse row slots (a batch of six or more events averaging fewer than
// 128 clusters per row): the per-row kernels are then bound by how many row
// slots the chip holds at once, and one wave per row slot holds more.  A
// single event keeps four waves per row slot: its rows are few, and a sparse
// mean can hide a few full sectors.
static bool sparse_rows(int64_t n_clusters, int64_t n_rowslots) {
  return n_rowslots >= 32768 && row_mean(n_clusters, n_rowslots) < 128;
}
// The neighbours finder's stage: the tuning's choice, or by density (larger
// rows and longer candidate lists above 320 clusters per row; on many sparse
// rows one wave per row slot, whose workgroups fit the CU three times as
// often, which the grid, evolution and seed kernels then take too).
static int32_t nf_stage_of(int32_t stage, int64_t n_clusters, int64_t n_rowslots) {
  if (stage != 0) return stage;
  if (row_mean(n_clusters, n_rowslots) > 320) return 2;
  return sparse_rows(n_clusters, n_rowslots) ? 3 : 1;
}

KParams make_kparams(const tpc_geometry* geo, float bz, const tpc_params* p) {
  KParams k;
  std::memset(&k, 0, sizeof(k));
  for (int r = 0; r < geo->n_rows; ++r) k.row_x[r] = geo->row_x[r];
  k.n_rows = geo->n_rows;
  k.tan_half = geo->tan_half_angle;
  k.z_max = geo->z_max;
  k.bz = bz;
  k.k_curv = 0.00299792458f * bz;
  k.sigma_y = p->sigma_y;
  k.sigma_z = p->sigma_z;
  k.sy2 = p->sigma_y * p->sigma_y;
  k.sz2 = p->sigma_z * p->sigma_z;
  k.nf_win_y = p->nf_win_y;
  k.nf_win_z = p->nf_win_z;
  k.nf_chi2_max = p->nf_chi2_max;
  k.min_seed_len = p->min_seed_len;
  k.seed_window = p->seed_window;
  k.chi2_gate = p->chi2_gate;
  k.max_miss = p->max_miss;
  k.max_sinphi = p->max_sinphi;
  k.alpha = p->alpha;
  k.beta = p->beta;
  k.min_clusters = p->min_clusters;
  k.max_qpt = 1.f / p->min_pt;
  k.prior_sinphi = p->prior_sinphi;
  k.prior_tanl = p->prior_tanl;
  k.prior_qpt = p->prior_qpt;
  k.bin_occupancy = 1.0f;
  k.construct_blocks = 0;
  k.construct_schedule = 0;
  k.nf_stage = 1;
  k.own_chunk = 4096;
  k.construct_lanes = 64;
  return k;
}

uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* p = (const unsigned char*)data;
  for (size_t i = 0; i < n; ++i) h = (h ^ p[i]) * 1099511628211ull;
  return h;
}

DevEvent make_devevent(const tpc_event* ev) {
  DevEvent d;
  d.y = ev->y;
  d.z = ev->z;
  d.ro = ev->row_offsets;
  d.sector_id = ev->sector_id;
  d.n_sectors = ev->n_sectors;
  d.n_clusters = (int32_t)ev->n_clusters;
  d.n_dev = nullptr;
  return d;
}

int64_t default_tracklets(const tpc_ctx* ctx, int64_t N, const tpc_params* p) {
  if (p->max_tracklets > 0) return p->max_tracklets;
  int64_t t = N / 24 + 256;  // one per 24 clusters (central events have one per 36)
  const int64_t l = (int64_t)std::ceil(ctx->learned_ratio * (double)N) + 256;
  return l > t ? l : t;
}

// Tracklets this call will probably find: as many per cluster as the last
// call found, else one per 36 clusters (a central event).  Sizes launches
// only; the reservation is default_tracklets.
int32_t expected_tracklets(const tpc_ctx* ctx, int64_t N) {
  const double r = ctx->seen_ratio > 0.0 ? ctx->seen_ratio : 1.0 / 36.0;
  const double t = std::ceil(r * (double)N) + 1.0;
  return t > 2e9 ? 2000000000 : (int32_t)t;
}

// After an overflow: the reservation for this call and the ratio learned from it.
int64_t grow_tracklets(tpc_ctx* ctx, int64_t need, int64_t N) {
  const int64_t T = need + need / 8 + 64;
  const double r = (double)T / (double)(N > 0 ? N : 1);
  if (r > ctx->learned_ratio) ctx->learned_ratio = r;
  return T;
}

int ensure_arena(tpc_ctx* ctx, int64_t N, int64_t R, int64_t T, hipStream_t st) {
  size_t need = scratch_bytes(N, R, T);
  if (need <= ctx->arena_bytes) return TPC_OK;
  size_t want = need + need / 4;
  if (ctx->budget && want > ctx->budget) want = need;
  if (ctx->budget && need > ctx->budget)
    return fail(TPC_ERR_OOM, "scratch of %zu bytes exceeds the context budget %zu", need,
                ctx->budget);
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (ctx->arena) {
    e = hipFree(ctx->arena);
    ctx->arena = nullptr;
    ctx->arena_bytes = 0;
    if (e != hipSuccess) return hip_fail(e, "hipFree");
  }
  e = hipMalloc(&ctx->arena, want);
  if (e != hipSuccess) {
    ctx->arena = nullptr;
    (void)hipGetLastError();
    return fail(TPC_ERR_OOM, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
  }
  ctx->arena_bytes = want;
  return TPC_OK;
}

// Global tracking scratch, followed by the merger's (with room for cap_rec
// list entries) when with_merge.
int ensure_glob(tpc_ctx* ctx, int64_t N, int64_t S, int64_t T, bool with_merge, int64_t cap_rec,
                hipStream_t st) {
  size_t need = global_bytes(N, T) + (with_merge ? merge_bytes(N, S, T, cap_rec) : 0);
  if (need <= ctx->glob_bytes) return TPC_OK;
  size_t want = need + need / 4;
  if (ctx->budget && ctx->arena_bytes + want > ctx->budget) want = need;
  if (ctx->budget && ctx->arena_bytes + need > ctx->budget)
    return fail(TPC_ERR_OOM, "global tracking scratch of %zu bytes exceeds the context budget",
                need);
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (ctx->glob_arena) {
    e = hipFree(ctx->glob_arena);
    ctx->glob_arena = nullptr;
    ctx->glob_bytes = 0;
    if (e != hipSuccess) return hip_fail(e, "hipFree");
  }
  e = hipMalloc(&ctx->glob_arena, want);
  if (e != hipSuccess) {
    ctx->glob_arena = nullptr;
    (void)hipGetLastError();
    return fail(TPC_ERR_OOM, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
  }
  ctx->glob_bytes = want;
  return TPC_OK;
}

// Runs the kernels up to `upto`, reads the counters back, maps device error
// bits to return codes.  With `po`, global tracking follows the whole path
// and its counters land in h_counters[C_COUNT ..].  On a tracklet overflow the reservation is raised and
// the event is run once more (results do not depend on the reservation).
//
// no_alloc: the scratch is the static per-device array (static_scratch), never
// the context's arena: nothing is allocated, and an event whose scratch does
// not fit the array fails with TPC_ERR_OOM.  The tracklet reservation is
// capped to what fits; an overflow is retried once with a larger one if it
// fits.
int run_event(tpc_ctx* ctx, const tpc_event* ev, const tpc_geometry* geo, float bz,
              const tpc_params* p, const Outputs& out, int upto, hipStream_t st,
              Scratch* sc_out, const ProOutputs* po = nullptr, const MergeOutputs* mo = nullptr,
              float merge_chi2 = 0.f, bool no_alloc = false) {
  int rc = validate(ev, geo, p);
  if (rc) return rc;
  if (!std::isfinite(bz)) return fail(TPC_ERR_INVALID_ARG, "bz must be finite");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  const int64_t N = ev->n_clusters, R = (int64_t)ev->n_sectors * geo->n_rows;
  KParams kp = make_kparams(geo, bz, p);
  kp.bin_occupancy = ctx->tuning.bin_occupancy;
  kp.construct_blocks = ctx->tuning.construct_blocks;
  kp.construct_schedule = ctx->tuning.construct_schedule;
  kp.construct_lanes = lanes_per_wave(ctx->tuning.construct_lanes, N);
  kp.n_cu = ctx->n_cu;
  kp.expect_tl = expected_tracklets(ctx, N);
  kp.nf_stage = nf_stage_of(ctx->tuning.nf_stage, N, R);
  kp.row_wave = kp.nf_stage == 3;
  kp.own_chunk = own_chunk(N, R, kp.n_rows);
  kp.own_by_sector = own_by_sector(ctx->tuning.own_order, R, kp.n_rows, kp.own_chunk);
  {  // neighbouring sectors' centre lines are one sector width, 2 atan(tan_half), apart
    const double w = 2.0 * std::atan((double)geo->tan_half_angle);
    kp.rot_c = (float)std::cos(w);
    kp.rot_s = (float)std::sin(w);
    for (int k = -9; k <= 8; ++k) {
      kp.rot_tab[k + 9][0] = (float)std::cos(k * w);
      kp.rot_tab[k + 9][1] = (float)std::sin(k * w);
    }
  }
  kp.merge_chi2 = merge_chi2;
  const DevEvent dev = make_devevent(ev);
  int64_t T = default_tracklets(ctx, N, p);
  void* fixed = nullptr;
  if (no_alloc) {
    fixed = static_scratch(ctx->device);
    if (!fixed) return fail(TPC_ERR_DEVICE, "static scratch of device %d not resolved", ctx->device);
    if (scratch_bytes(N, R, 256) > kStaticScratchBytes)
      return fail(TPC_ERR_OOM, "an event of %lld clusters needs more scratch than the static "
                               "%zu bytes", (long long)N, kStaticScratchBytes);
  }
  // the largest reservation up to T whose scratch fits the static array
  auto fit = [&](int64_t t) {
    while (t > 256 && scratch_bytes(N, R, t) > kStaticScratchBytes) t -= t / 16 + 1;
    return t < 256 ? 256 : t;
  };
  if (no_alloc) T = fit(T);
  for (int attempt = 0; attempt < 2; ++attempt) {
    if (!no_alloc) {
      rc = ensure_arena(ctx, N, R, T, st);
      if (rc) return rc;
    }
    Scratch sc;
    scratch_carve(no_alloc ? fixed : ctx->arena, N, R, T, &sc);
    GlobalScratch gs{};
    MergeScratch ms{};
    if (po || mo) {
      // the joined tracks' lists hold distinct clusters: at most N entries
      rc = ensure_glob(ctx, N, ev->n_sectors, T, mo != nullptr, N, st);
      if (rc) return rc;
      global_carve(ctx->glob_arena, N, T, &sc.ends, &gs);
      if (mo)
        merge_carve((char*)ctx->glob_arena + global_bytes(N, T), N, ev->n_sectors, T, N, &ms);
    }
    const bool timed = ctx->timer.mask != 0;
    e = enqueue_event(dev, kp, sc, out, upto, st, timed ? &ctx->timer : nullptr);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    const KernelTimer* tmr = timed ? &ctx->timer : nullptr;
    if (po && mo) {
      // end states; then the joins on the side stream while the
      // prolongations run on st; the lists wait for both
      if (!ctx->side) {
        e = hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "side stream");
      }
      e = enqueue_global(dev, kp, sc, out, gs, po, st, tmr, 0);
      if (e == hipSuccess) e = hipEventRecord(ctx->fork, st);
      if (e == hipSuccess) e = hipStreamWaitEvent(ctx->side, ctx->fork, 0);
      if (e == hipSuccess) e = enqueue_merge(dev, kp, sc, out, gs, po, ms, *mo, ctx->side, tmr, 0);
      if (e == hipSuccess) e = hipEventRecord(ctx->join, ctx->side);
      if (e == hipSuccess) e = enqueue_global(dev, kp, sc, out, gs, po, st, tmr, 1);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, ctx->join, 0);
      if (e != hipSuccess) return hip_fail(e, "kernel launch (global tracking)");
    } else if (po || mo) {
      e = enqueue_global(dev, kp, sc, out, gs, po, st, tmr);
      if (e != hipSuccess) return hip_fail(e, "kernel launch (global tracking)");
    }
    if (po || mo) {
      e = hipMemcpyAsync(ctx->h_counters + C_COUNT, gs.counters, sizeof(int32_t) * C_COUNT,
                         hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(counters)");
    }
    if (mo) {
      e = enqueue_merge(dev, kp, sc, out, gs, po, ms, *mo, st, tmr, po ? 1 : -1);
      if (e != hipSuccess) return hip_fail(e, "kernel launch (merger)");
      e = hipMemcpyAsync(ctx->h_counters + 2 * C_COUNT, ms.counters, sizeof(int32_t) * C_COUNT,
                         hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(counters)");
    }
    e = hipMemcpyAsync(ctx->h_counters, sc.counters, sizeof(int32_t) * C_COUNT,
                       hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(counters)");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    const int32_t* c = ctx->h_counters;
    if (c[C_ERR] & E_OFFSETS)
      return fail(TPC_ERR_INVALID_ARG, "row_offsets are not a valid non-decreasing partition "
                                       "of [0, n_clusters]");
    if (c[C_ERR] & E_NONFINITE)
      return fail(TPC_ERR_INVALID_ARG, "%d clusters have non-finite coordinates", c[C_NONFINITE]);
    if (upto >= STAGE_TRACKLETS && (c[C_ERR] & E_TL_OVERFLOW)) {
      const int64_t need = c[C_SEEDS];
      if (p->max_tracklets > 0 || attempt == 1)
        return fail(TPC_ERR_OVERFLOW, "%lld tracklets exceed the reservation of %lld",
                    (long long)need, (long long)T);
      T = grow_tracklets(ctx, need, N);
      if (no_alloc && scratch_bytes(N, R, T) > kStaticScratchBytes)
        return fail(TPC_ERR_OOM, "%lld tracklets need more scratch than the static %zu bytes",
                    (long long)need, kStaticScratchBytes);
      continue;
    }
    if (timed) {
      const int last = mo ? K_REFIT
                       : po ? K_PRO_OUTPUT
                       : upto >= STAGE_ALL ? K_OUTPUT
                       : upto >= STAGE_TRACKLETS ? K_CONSTRUCT
                       : upto >= STAGE_SEEDS ? K_SEED_WRITE : K_EVO;
      for (int k = 0; k <= last; ++k) {
        if (!(ctx->timer.mask >> k & 1u)) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ctx->timer.ev[k][0], ctx->timer.ev[k][1]) == hipSuccess) {
          ctx->kernel_ms[k] += ms;
          ctx->kernel_launches[k] += 1;
        }
      }
      (void)hipGetLastError();  // a kernel this call skipped has no recorded events
    }
    ctx->work[0] += 1;
    ctx->work[1] += c[C_SEEDS];
    if (N > 0 && upto >= STAGE_SEEDS) ctx->seen_ratio = (double)c[C_SEEDS] / (double)N;
    ctx->work[2] += (uint32_t)c[C_STEPS];
    ctx->work[3] += (uint32_t)c[C_UPDATES];
    ctx->work[4] += (uint32_t)c[C_CANDS];
    if (sc_out) *sc_out = sc;
    return TPC_OK;
  }
  return fail(TPC_ERR_OVERFLOW, "tracklet reservation retry failed");
}


int ensure_batch(tpc_ctx* ctx, int64_t N, int64_t S, int n_rows, int E, int64_t cap_tracks,
                 BatchBuffers* bb, BatchEventDesc** h_desc, int32_t** h_counts,
                 hipStream_t st) {
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t need = al(4 * (size_t)N) * 2 + al(4 * ((size_t)S * n_rows + 1)) + al(4 * (size_t)S) +
                      al(32 * (size_t)cap_tracks) + al(16 * (size_t)cap_tracks) +
                      al(4 * (size_t)N) * 2 + al(8 * (size_t)E) + al(sizeof(BatchEventDesc) * E) +
                      al(16);
  hipError_t e;
  if (need > ctx->batch_bytes) {
    if (ctx->budget && need + ctx->arena_bytes > ctx->budget)
      return fail(TPC_ERR_OOM, "batch buffers of %zu bytes exceed the context budget", need);
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (ctx->batch_arena) (void)hipFree(ctx->batch_arena);
    ctx->batch_arena = nullptr;
    ctx->batch_bytes = 0;
    e = hipMalloc(&ctx->batch_arena, need + need / 4);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(TPC_ERR_OOM, "hipMalloc(%zu) failed for the batch", need + need / 4);
    }
    ctx->batch_bytes = need + need / 4;
  }
  const size_t hneed = al(sizeof(BatchEventDesc) * E) + al(16) + 8 * (size_t)E + 64;
  if (hneed > ctx->h_batch_bytes) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (ctx->h_batch) (void)hipHostFree(ctx->h_batch);
    ctx->h_batch = nullptr;
    ctx->h_batch_bytes = 0;
    e = hipHostMalloc(&ctx->h_batch, 2 * hneed, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "hipHostMalloc(batch)");
    ctx->h_batch_bytes = 2 * hneed;
  }
  char* p = (char*)ctx->batch_arena;
  auto take = [&](size_t b) {
    void* q = p;
    p += al(b);
    return q;
  };
  bb->y = (float*)take(4 * (size_t)N);
  bb->z = (float*)take(4 * (size_t)N);
  bb->ro = (int32_t*)take(4 * ((size_t)S * n_rows + 1));
  bb->sector_id = (int32_t*)take(4 * (size_t)S);
  bb->par = (float*)take(32 * (size_t)cap_tracks);
  bb->meta = (int32_t*)take(16 * (size_t)cap_tracks);
  bb->tcl = (int32_t*)take(4 * (size_t)N);
  bb->ctr = (int32_t*)take(4 * (size_t)N);
  bb->ev_counts = (int32_t*)take(8 * (size_t)E);
  bb->desc = (BatchEventDesc*)take(sizeof(BatchEventDesc) * E);
  bb->hdr = (int32_t*)take(16);
  bb->cap_tracks = (int32_t)cap_tracks;
  *h_desc = (BatchEventDesc*)ctx->h_batch;
  *h_counts = (int32_t*)((char*)ctx->h_batch + al(sizeof(BatchEventDesc) * E) + al(16));
  return TPC_OK;
}

int check_outputs(const tpc_event* ev, const tpc_tracks* out) {
  if (!out || !out->n_tracks || !out->n_track_clusters)
    return fail(TPC_ERR_INVALID_ARG, "out or its size pointers are null");
  if (out->cap_tracks < 0 || out->cap_track_clusters < 0)
    return fail(TPC_ERR_INVALID_ARG, "negative capacity");
  if ((out->cap_tracks > 0 && (!out->track_par || !out->track_meta)) ||
      (out->cap_track_clusters > 0 && !out->track_cluster))
    return fail(TPC_ERR_INVALID_ARG, "output array is null");
  if (ev && ev->n_clusters > 0 && !out->cluster_track)
    return fail(TPC_ERR_INVALID_ARG, "cluster_track is null");
  return TPC_OK;
}

int run_batch(tpc_ctx* ctx, const tpc_event* evs, int E, const tpc_geometry* geo, float bz,
              const tpc_params* p, tpc_tracks* outs, hipStream_t st) {
  if (!evs || !outs || E < 1) return fail(TPC_ERR_INVALID_ARG, "need at least one event");
  int64_t N = 0, S = 0;
  for (int e = 0; e < E; ++e) {
    int rc = validate(&evs[e], geo, p);
    if (rc) return fail(rc, "event %d: %s", e, g_err.c_str());
    rc = check_outputs(&evs[e], &outs[e]);
    if (rc) return fail(rc, "event %d: %s", e, g_err.c_str());
    N += evs[e].n_clusters;
    S += evs[e].n_sectors;
  }
  if (!std::isfinite(bz)) return fail(TPC_ERR_INVALID_ARG, "bz must be finite");
  if (S * geo->n_rows + N + 1 > 0x7fffffffLL || S > 0x7fffffffLL / geo->n_rows)
    return fail(TPC_ERR_INVALID_ARG, "batch too large for int32 indexing");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  const int64_t R = S * geo->n_rows;
  const bool use_graph = ctx->tuning.use_graph != 0;
  if (use_graph) {
    // graph work runs on the context's own stream, after the caller's stream
    if (!ctx->graph_stream) {
      e = hipStreamCreateWithFlags(&ctx->graph_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
      e = hipEventCreateWithFlags(&ctx->graph_dep, hipEventDisableTiming);
      if (e != hipSuccess) return hip_fail(e, "hipEventCreateWithFlags");
    }
    e = hipEventRecord(ctx->graph_dep, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(ctx->graph_stream, ctx->graph_dep, 0);
    if (e != hipSuccess) return hip_fail(e, "stream ordering");
    st = ctx->graph_stream;
  }
  // With a graph, buffers are laid out for a capacity that later batches of
  // the same shape reuse; without, for this batch.
  int64_t ncap = N;
  if (use_graph) {
    ncap = ctx->graph_ncap > N ? ctx->graph_ncap : ((N + (1 << 20) - 1) >> 20) << 20;
    if (ncap < 1) ncap = 1;
  }
  const int64_t cap_tracks = ncap / p->min_clusters + 1;  // tracks own >= min_clusters clusters
  BatchBuffers bb;
  BatchEventDesc* hd;
  int32_t* hc;
  int rc = ensure_batch(ctx, ncap, S, geo->n_rows, E, cap_tracks, &bb, &hd, &hc, st);
  if (rc) return rc;
  int64_t cb = 0, sb = 0;
  for (int i = 0; i < E; ++i) {
    BatchEventDesc& d = hd[i];
    d.y = evs[i].y;
    d.z = evs[i].z;
    d.ro = evs[i].row_offsets;
    d.sector_id = evs[i].sector_id;
    d.n_clusters = (int32_t)evs[i].n_clusters;
    d.n_sectors = evs[i].n_sectors;
    d.cbase = (int32_t)cb;
    d.sbase = (int32_t)sb;
    d.track_par = outs[i].track_par;
    d.track_meta = outs[i].track_meta;
    d.track_cluster = outs[i].track_cluster;
    d.cluster_track = outs[i].cluster_track;
    d.cap_tracks = outs[i].cap_tracks;
    d.cap_track_clusters = outs[i].cap_track_clusters;
    cb += evs[i].n_clusters;
    sb += evs[i].n_sectors;
  }
  int32_t* hh = (int32_t*)(hd + E);
  hh = (int32_t*)(((uintptr_t)hh + 255) & ~(uintptr_t)255);
  hh[0] = (int32_t)N;
  e = hipMemcpyAsync(bb.desc, hd, sizeof(BatchEventDesc) * E, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(bb.hdr, hh, 16, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(batch descriptors)");
  tpc_event bev;
  bev.n_sectors = (int32_t)S;
  bev.sector_id = bb.sector_id;
  bev.n_clusters = N;
  bev.y = bb.y;
  bev.z = bb.z;
  bev.row_offsets = bb.ro;
  KParams kp = make_kparams(geo, bz, p);
  kp.bin_occupancy = ctx->tuning.bin_occupancy;
  kp.construct_blocks = ctx->tuning.construct_blocks;
  kp.construct_schedule = ctx->tuning.construct_schedule;
  kp.construct_lanes = lanes_per_wave(ctx->tuning.construct_lanes, N);
  kp.n_cu = ctx->n_cu;
  kp.expect_tl = expected_tracklets(ctx, N);
  kp.nf_stage = nf_stage_of(ctx->tuning.nf_stage, N, R);
  kp.row_wave = kp.nf_stage == 3;
  kp.own_chunk = own_chunk(N, R, kp.n_rows);
  kp.own_by_sector = own_by_sector(ctx->tuning.own_order, R, kp.n_rows, kp.own_chunk);
  DevEvent dev = make_devevent(&bev);
  if (use_graph) {
    dev.n_clusters = (int32_t)ncap;
    dev.n_dev = bb.hdr;
  }
  const Outputs o{(int32_t)cap_tracks, (int32_t)ncap, bb.par, bb.meta, bb.tcl, bb.ctr};
  int64_t T = default_tracklets(ctx, ncap, p);
  for (int attempt = 0; attempt < 2; ++attempt) {
    rc = ensure_arena(ctx, ncap, R, T, st);
    if (rc) return rc;
    Scratch sc;
    scratch_carve(ctx->arena, ncap, R, T, &sc);
    const bool graph_now = use_graph && attempt == 0;
    const bool timed = ctx->timer.mask != 0 && !graph_now;
    if (graph_now) {
      uint64_t key = fnv1a(&kp, sizeof(kp));
      const int64_t shape[6] = {E, S, ncap, T, (int64_t)(uintptr_t)ctx->arena,
                                (int64_t)(uintptr_t)ctx->batch_arena};
      key = fnv1a(shape, sizeof(shape), key);
      key = fnv1a(&st, sizeof(st), key);
      if (!ctx->graph_exec || key != ctx->graph_key) {
        if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
        if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
        ctx->graph_exec = nullptr;
        ctx->graph = nullptr;
        e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        hipError_t e1 = enqueue_batch_gather(bb, sc, E, geo->n_rows, (int)ncap, (int)S, st);
        hipError_t e2 = enqueue_event(dev, kp, sc, o, STAGE_ALL, st, nullptr, false);
        hipError_t e3 = enqueue_batch_scatter(bb, sc, E, st);
        e = hipStreamEndCapture(st, &ctx->graph);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e != hipSuccess) {
          (void)hipGetLastError();
          return hip_fail(e != hipSuccess ? e : hipErrorUnknown, "graph capture");
        }
        e = hipGraphInstantiate(&ctx->graph_exec, ctx->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        ctx->graph_key = key;
        ctx->graph_ncap = ncap;
      }
      e = hipGraphLaunch(ctx->graph_exec, st);
      if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
      ctx->graph_launches += 1;
    } else {
      e = enqueue_batch_gather(bb, sc, E, geo->n_rows, (int)ncap, (int)S, st);
      if (e == hipSuccess)
        e = enqueue_event(dev, kp, sc, o, STAGE_ALL, st, timed ? &ctx->timer : nullptr, false);
      if (e == hipSuccess) e = enqueue_batch_scatter(bb, sc, E, st);
      if (e != hipSuccess) return hip_fail(e, "kernel launch");
    }
    e = hipMemcpyAsync(ctx->h_counters, sc.counters, sizeof(int32_t) * C_COUNT,
                       hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hc, bb.ev_counts, 8 * (size_t)E, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(counts)");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    const int32_t* c = ctx->h_counters;
    if (c[C_ERR] & E_OFFSETS)
      return fail(TPC_ERR_INVALID_ARG, "row_offsets of an event are not a valid partition");
    if (graph_now && (c[C_ERR] & E_TL_OVERFLOW)) {
      // the replay's reservation was too small: drop the graph, re-run eagerly
      const int64_t need = c[C_SEEDS];
      T = grow_tracklets(ctx, need, ncap);
      if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
      if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
      ctx->graph_exec = nullptr;
      ctx->graph = nullptr;
      continue;
    }
    if (c[C_ERR] & E_NONFINITE)
      return fail(TPC_ERR_INVALID_ARG, "%d clusters have non-finite coordinates", c[C_NONFINITE]);
    if (c[C_ERR] & E_TL_OVERFLOW) {
      const int64_t need = c[C_SEEDS];
      if (p->max_tracklets > 0 || attempt == 1)
        return fail(TPC_ERR_OVERFLOW, "%lld tracklets exceed the reservation of %lld",
                    (long long)need, (long long)T);
      T = grow_tracklets(ctx, need, ncap);
      continue;
    }
    if (c[C_ERR] & E_CAPACITY) return fail(TPC_ERR_DEVICE, "internal batch output overflow");
    if (timed) {
      // only the kernels a batch launches: an elapsed-time query on an event
      // that was never recorded fails and would leave HIP's last error set
      for (int k = 0; k <= K_OUTPUT; ++k) {
        if (!(ctx->timer.mask >> k & 1u)) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ctx->timer.ev[k][0], ctx->timer.ev[k][1]) == hipSuccess) {
          ctx->kernel_ms[k] += ms;
          ctx->kernel_launches[k] += 1;
        }
      }
      (void)hipGetLastError();  // a kernel this call skipped has no recorded events
    }
    ctx->work[0] += E;
    ctx->work[1] += c[C_SEEDS];
    if (N > 0) ctx->seen_ratio = (double)c[C_SEEDS] / (double)N;
    ctx->work[2] += (uint32_t)c[C_STEPS];
    ctx->work[3] += (uint32_t)c[C_UPDATES];
    ctx->work[4] += (uint32_t)c[C_CANDS];
    int status = TPC_OK;
    for (int i = 0; i < E; ++i) {
      *outs[i].n_tracks = hc[2 * i];
      *outs[i].n_track_clusters = hc[2 * i + 1];
      if (hc[2 * i] > outs[i].cap_tracks || hc[2 * i + 1] > outs[i].cap_track_clusters)
        status = TPC_ERR_CAPACITY;
    }
    if (status) return fail(status, "outputs of at least one event are too small");
    return TPC_OK;
  }
  return fail(TPC_ERR_OVERFLOW, "tracklet reservation retry failed");
}

}  // namespace tpc

using namespace tpc;

extern "C" {

void tpc_params_default(tpc_params* p) {
  if (!p) return;
  p->sigma_y = 0.1f;
  p->sigma_z = 0.1f;
  p->nf_win_y = 4.0f;
  p->nf_win_z = 4.0f;
  p->nf_chi2_max = 25.0f;
  p->min_seed_len = 3;
  p->seed_window = 16;
  p->chi2_gate = 16.0f;
  p->max_miss = 10;
  p->max_sinphi = 0.95f;
  p->alpha = 6.0f;       // section 3.1
  p->beta = 1.0f;
  p->min_clusters = 30;  // section 5
  p->min_pt = 0.1f;
  p->prior_sinphi = 1.0f;
  p->prior_tanl = 1.0f;
  p->prior_qpt = 100.0f;
  p->max_tracklets = 0;
}

const char* tpc_last_error(void) { return g_err.c_str(); }

int tpc_validate(const tpc_event* ev, const tpc_geometry* geo, const tpc_params* params) {
  return validate(ev, geo, params);
}

int tpc_ctx_create(int device, size_t hbm_budget_bytes, tpc_ctx** out) {
  if (!out) return fail(TPC_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(TPC_ERR_INVALID_ARG, "device %d of %d", device, n);
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  tpc_ctx* c = new (std::nothrow) tpc_ctx();
  if (!c) return fail(TPC_ERR_OOM, "host allocation failed");
  c->device = device;
  c->budget = hbm_budget_bytes;
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) !=
      hipSuccess)
    c->n_cu = 0;
  tpc_tuning_default(&c->tuning);
  e = hipHostMalloc((void**)&c->h_counters, sizeof(int32_t) * 3 * C_COUNT, hipHostMallocDefault);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipHostMalloc");
  }
  // the allocation-free entry point's array on this device (once per device)
  e = static_scratch_init(device);
  if (e != hipSuccess) {
    (void)hipHostFree(c->h_counters);
    delete c;
    return hip_fail(e, "hipGetSymbolAddress(static scratch)");
  }
  *out = c;
  return TPC_OK;
}

int tpc_kernel_count(void) { return K_NUM; }

const char* tpc_kernel_name(int i) { return (i >= 0 && i < K_NUM) ? kKernelNames[i] : ""; }

void tpc_tuning_default(tpc_tuning* t) {
  if (!t) return;
  t->use_graph = 1;
  t->construct_blocks = 0;
  t->bin_occupancy = 1.0f;
  t->construct_schedule = 0;
  t->construct_lanes = 0;
  t->nf_stage = 0;
  t->own_order = 0;
}

int tpc_ctx_set_tuning(tpc_ctx* ctx, const tpc_tuning* t) {
  if (!ctx || !t) return fail(TPC_ERR_INVALID_ARG, "ctx or tuning is null");
  if (t->construct_blocks < 0 || t->construct_blocks > (1 << 20))
    return fail(TPC_ERR_INVALID_ARG, "construct_blocks outside [0, 2^20]");
  if (!(t->bin_occupancy >= 1.0f && t->bin_occupancy <= 64.f))
    return fail(TPC_ERR_INVALID_ARG, "bin_occupancy outside [1, 64]");
  if (t->construct_schedule != 0 && t->construct_schedule != 1)
    return fail(TPC_ERR_INVALID_ARG, "construct_schedule must be 0 or 1");
  if (t->construct_lanes < 0 || t->construct_lanes > 64)
    return fail(TPC_ERR_INVALID_ARG, "construct_lanes outside [0, 64]");
  if (t->nf_stage < 0 || t->nf_stage > 3)
    return fail(TPC_ERR_INVALID_ARG, "nf_stage must be 0, 1, 2 or 3");
  if (t->own_order < 0 || t->own_order > 2)
    return fail(TPC_ERR_INVALID_ARG, "own_order must be 0, 1 or 2");
  ctx->tuning = *t;
  return TPC_OK;
}

int tpc_ctx_graph_launches(tpc_ctx* ctx, int64_t* n) {
  if (!ctx || !n) return fail(TPC_ERR_INVALID_ARG, "ctx or n is null");
  *n = ctx->graph_launches;
  return TPC_OK;
}

int tpc_ctx_set_timing(tpc_ctx* ctx, uint32_t kernel_mask) {
  if (!ctx) return fail(TPC_ERR_INVALID_ARG, "ctx is null");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if (kernel_mask && !ctx->timer_ready) {
    for (int k = 0; k < K_NUM; ++k)
      for (int j = 0; j < 2; ++j) {
        e = hipEventCreate(&ctx->timer.ev[k][j]);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
      }
    ctx->timer_ready = true;
  }
  ctx->timer.mask = kernel_mask & ((1u << K_NUM) - 1u);
  return TPC_OK;
}

int tpc_ctx_get_stats(tpc_ctx* ctx, double* kernel_ms, int64_t* kernel_launches, int64_t* work) {
  if (!ctx) return fail(TPC_ERR_INVALID_ARG, "ctx is null");
  for (int k = 0; k < K_NUM; ++k) {
    if (kernel_ms) kernel_ms[k] = ctx->kernel_ms[k];
    if (kernel_launches) kernel_launches[k] = ctx->kernel_launches[k];
  }
  if (work)
    for (int i = 0; i < 5; ++i) work[i] = ctx->work[i];
  return TPC_OK;
}

int tpc_ctx_reset_stats(tpc_ctx* ctx) {
  if (!ctx) return fail(TPC_ERR_INVALID_ARG, "ctx is null");
  for (int k = 0; k < K_NUM; ++k) {
    ctx->kernel_ms[k] = 0.0;
    ctx->kernel_launches[k] = 0;
  }
  for (int i = 0; i < 5; ++i) ctx->work[i] = 0;
  return TPC_OK;
}

void tpc_ctx_destroy(tpc_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  if (ctx->graph_stream) (void)hipStreamDestroy(ctx->graph_stream);
  if (ctx->graph_dep) (void)hipEventDestroy(ctx->graph_dep);
  if (ctx->timer_ready)
    for (int k = 0; k < K_NUM; ++k)
      for (int j = 0; j < 2; ++j) (void)hipEventDestroy(ctx->timer.ev[k][j]);
  if (ctx->arena) (void)hipFree(ctx->arena);
  if (ctx->batch_arena) (void)hipFree(ctx->batch_arena);
  if (ctx->glob_arena) (void)hipFree(ctx->glob_arena);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  if (ctx->fork) (void)hipEventDestroy(ctx->fork);
  if (ctx->join) (void)hipEventDestroy(ctx->join);
  if (ctx->h_counters) (void)hipHostFree(ctx->h_counters);
  if (ctx->h_batch) (void)hipHostFree(ctx->h_batch);
  delete ctx;
}

int tpc_track_event(tpc_ctx* ctx, const tpc_event* ev, const tpc_geometry* geo, float bz_tesla,
                    const tpc_params* params, tpc_tracks* out, void* hip_stream) {
  if (!ctx) return fail(TPC_ERR_INVALID_ARG, "ctx is null");
  int rc0 = check_outputs(ev, out);
  if (rc0) return rc0;
  Outputs o{out->cap_tracks, out->cap_track_clusters, out->track_par, out->track_meta,
            out->track_cluster, out->cluster_track};
  hipStream_t st = (hipStream_t)hip_stream;
  int rc = run_event(ctx, ev, geo, bz_tesla, params, o, STAGE_ALL, st, nullptr);
  if (rc) return rc;
  const int32_t* c = ctx->h_counters;
  *out->n_tracks = c[C_TRACKS];
  *out->n_track_clusters = c[C_TRACK_CLUSTERS];
  if (c[C_ERR] & E_CAPACITY)
    return fail(TPC_ERR_CAPACITY, "need %d tracks / %d track clusters, have %d / %d",
                c[C_TRACKS], c[C_TRACK_CLUSTERS], out->cap_tracks, out->cap_track_clusters);
  return TPC_OK;
}

int tpc_track_event_noalloc(tpc_ctx* ctx, const tpc_event* ev, const tpc_geometry* geo,
                            float bz_tesla, const tpc_params* params, tpc_tracks* out,
                            void* hip_stream) {
  if (!ctx) return fail(TPC_ERR_INVALID_ARG, "ctx is null");
  int rc0 = check_outputs(ev, out);
  if (rc0) return rc0;
  Outputs o{out->cap_tracks, out->cap_track_clusters, out->track_par, out->track_meta,
            out->track_cluster, out->cluster_track};
  hipStream_t st = (hipStream_t)hip_stream;
  int rc = run_event(ctx, ev, geo, bz_tesla, params, o, STAGE_ALL, st, nullptr, nullptr, nullptr,
                     0.f, true);
  if (rc) return rc;
  const int32_t* c = ctx->h_counters;
  *out->n_tracks = c[C_TRACKS];
  *out->n_track_clusters = c[C_TRACK_CLUSTERS];
  if (c[C_ERR] & E_CAPACITY)
    return fail(TPC_ERR_CAPACITY, "need %d tracks / %d track clusters, have %d / %d",
                c[C_TRACKS], c[C_TRACK_CLUSTERS], out->cap_tracks, out->cap_track_clusters);
  return TPC_OK;
}

static int check_pro(const tpc_prolongations* pro) {
  if (!pro || !pro->n || !pro->n_clusters)
    return fail(TPC_ERR_INVALID_ARG, "pro or its size pointers are null");
  if (pro->cap < 0 || pro->cap_clusters < 0)
    return fail(TPC_ERR_INVALID_ARG, "negative prolongation capacity");
  if ((pro->cap > 0 && (!pro->par || !pro->meta)) || (pro->cap_clusters > 0 && !pro->cluster))
    return fail(TPC_ERR_INVALID_ARG, "prolongation output array is null");
  return TPC_OK;
}

// Sizes of the tracks and prolongations after global tracking.
static int global_sizes(tpc_ctx* ctx, tpc_tracks* out, tpc_prolongations* pro) {
  const int32_t* c = ctx->h_counters;
  const int32_t* g = ctx->h_counters + C_COUNT;
  *out->n_tracks = c[C_TRACKS];
  *out->n_track_clusters = c[C_TRACK_CLUSTERS];
  *pro->n = 0;
  *pro->n_clusters = 0;
  if (c[C_ERR] & E_CAPACITY)
    return fail(TPC_ERR_CAPACITY, "need %d tracks / %d track clusters, have %d / %d",
                c[C_TRACKS], c[C_TRACK_CLUSTERS], out->cap_tracks, out->cap_track_clusters);
  *pro->n = g[C_TRACKS];
  *pro->n_clusters = g[C_TRACK_CLUSTERS];
  if (g[C_ERR] & E_CAPACITY)
    return fail(TPC_ERR_CAPACITY, "need %d prolongations / %d clusters, have %d / %d",
                g[C_TRACKS], g[C_TRACK_CLUSTERS], pro->cap, pro->cap_clusters);
  return TPC_OK;
}

int tpc_track_event_global(tpc_ctx* ctx, const tpc_event* ev, const tpc_geometry* geo,
                           float bz_tesla, const tpc_params* params, tpc_tracks* out,
                           tpc_prolongations* pro, void* hip_stream) {
  if (!ctx) return fail(TPC_ERR_INVALID_ARG, "ctx is null");
  int rc0 = check_outputs(ev, out);
  if (rc0) return rc0;
  rc0 = check_pro(pro);
  if (rc0) return rc0;
  Outputs o{out->cap_tracks, out->cap_track_clusters, out->track_par, out->track_meta,
            out->track_cluster, out->cluster_track};
  ProOutputs po{pro->cap, pro->cap_clusters, pro->par, pro->meta, pro->cluster};
  hipStream_t st = (hipStream_t)hip_stream;
  int rc = run_event(ctx, ev, geo, bz_tesla, params, o, STAGE_ALL, st, nullptr, &po);
  if (rc) return rc;
  return global_sizes(ctx, out, pro);
}

int tpc_track_event_merged(tpc_ctx* ctx, const tpc_event* ev, const tpc_geometry* geo,
                           float bz_tesla, const tpc_params* params, float merge_chi2,
                           tpc_tracks* out, tpc_prolongations* pro, tpc_merged* mrg,
                           void* hip_stream) {
  if (!ctx) return fail(TPC_ERR_INVALID_ARG, "ctx is null");
  int rc0 = check_outputs(ev, out);
  if (rc0) return rc0;
  if (pro) {
    rc0 = check_pro(pro);
    if (rc0) return rc0;
  }
  if (!mrg || !mrg->n || !mrg->n_clusters)
    return fail(TPC_ERR_INVALID_ARG, "mrg or its size pointers are null");
  if (mrg->cap < 0 || mrg->cap_clusters < 0)
    return fail(TPC_ERR_INVALID_ARG, "negative merged-track capacity");
  if ((mrg->cap > 0 && (!mrg->par || !mrg->meta)) || (mrg->cap_clusters > 0 && !mrg->cluster) ||
      (out->cap_tracks > 0 && !mrg->track_merged))
    return fail(TPC_ERR_INVALID_ARG, "merged-track output array is null");
  if (!(merge_chi2 >= 0.f) || !std::isfinite(merge_chi2))
    return fail(TPC_ERR_INVALID_ARG, "merge_chi2 must be finite and >= 0");
  Outputs o{out->cap_tracks, out->cap_track_clusters, out->track_par, out->track_meta,
            out->track_cluster, out->cluster_track};
  ProOutputs po{pro ? pro->cap : 0, pro ? pro->cap_clusters : 0, pro ? pro->par : nullptr,
                pro ? pro->meta : nullptr, pro ? pro->cluster : nullptr};
  MergeOutputs mo{mrg->cap, mrg->cap_clusters, mrg->par, mrg->meta, mrg->cluster,
                  mrg->track_merged};
  hipStream_t st = (hipStream_t)hip_stream;
  int rc = run_event(ctx, ev, geo, bz_tesla, params, o, STAGE_ALL, st, nullptr,
                     pro ? &po : nullptr, &mo, merge_chi2);
  if (rc) return rc;
  *mrg->n = 0;
  *mrg->n_clusters = 0;
  if (pro) {
    rc = global_sizes(ctx, out, pro);
    if (rc) return rc;
  } else {
    const int32_t* c = ctx->h_counters;
    *out->n_tracks = c[C_TRACKS];
    *out->n_track_clusters = c[C_TRACK_CLUSTERS];
    if (c[C_ERR] & E_CAPACITY)
      return fail(TPC_ERR_CAPACITY, "need %d tracks / %d track clusters, have %d / %d",
                  c[C_TRACKS], c[C_TRACK_CLUSTERS], out->cap_tracks, out->cap_track_clusters);
  }
  const int32_t* m = ctx->h_counters + 2 * C_COUNT;
  *mrg->n = m[C_TRACKS];
  *mrg->n_clusters = m[C_TRACK_CLUSTERS];
  if (m[C_ERR] & E_CAPACITY)
    return fail(TPC_ERR_CAPACITY, "need %d merged tracks / %d clusters, have %d / %d",
                m[C_TRACKS], m[C_TRACK_CLUSTERS], mrg->cap, mrg->cap_clusters);
  return TPC_OK;
}

int tpc_refit(tpc_ctx* ctx, const tpc_event* ev, const tpc_geometry* geo, float bz_tesla,
              const tpc_params* params, int32_t n_lists, int32_t n_entries,
              const int32_t* offsets, const int32_t* clusters, float* par,
              int32_t* frame_sector, void* hip_stream) {
  if (!ctx) return fail(TPC_ERR_INVALID_ARG, "ctx is null");
  int rc = validate(ev, geo, params);
  if (rc) return rc;
  if (!std::isfinite(bz_tesla)) return fail(TPC_ERR_INVALID_ARG, "bz must be finite");
  if (n_lists < 0 || n_entries < 0) return fail(TPC_ERR_INVALID_ARG, "negative list sizes");
  if (n_lists > 0 && (!offsets || !par || (n_entries > 0 && !clusters)))
    return fail(TPC_ERR_INVALID_ARG, "offsets, clusters or par is null");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  const int64_t N = ev->n_clusters, R = (int64_t)ev->n_sectors * geo->n_rows, T = 1;
  hipStream_t st = (hipStream_t)hip_stream;
  rc = ensure_arena(ctx, N, R, T, st);
  if (rc) return rc;
  rc = ensure_glob(ctx, N, ev->n_sectors, T, true, n_entries, st);
  if (rc) return rc;
  KParams kp = make_kparams(geo, bz_tesla, params);
  kp.bin_occupancy = ctx->tuning.bin_occupancy;
  {
    const double w = 2.0 * std::atan((double)geo->tan_half_angle);
    for (int k = -9; k <= 8; ++k) {
      kp.rot_tab[k + 9][0] = (float)std::cos(k * w);
      kp.rot_tab[k + 9][1] = (float)std::sin(k * w);
    }
  }
  Scratch sc;
  scratch_carve(ctx->arena, N, R, T, &sc);
  GlobalScratch gs{};
  MergeScratch ms{};
  global_carve(ctx->glob_arena, N, T, &sc.ends, &gs);
  merge_carve((char*)ctx->glob_arena + global_bytes(N, T), N, ev->n_sectors, T, n_entries, &ms);
  const DevEvent dev = make_devevent(ev);
  Outputs o{0, 0, nullptr, nullptr, nullptr, nullptr};
  e = enqueue_event(dev, kp, sc, o, STAGE_GRID, st);
  if (e == hipSuccess)
    e = enqueue_refit(dev, kp, sc, ms, n_lists, n_entries, offsets, clusters, par, frame_sector,
                      st);
  if (e != hipSuccess) return hip_fail(e, "kernel launch (refit)");
  e = hipMemcpyAsync(ctx->h_counters, sc.counters, sizeof(int32_t) * C_COUNT,
                     hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(counters)");
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  const int32_t* c = ctx->h_counters;
  if (c[C_ERR] & E_OFFSETS)
    return fail(TPC_ERR_INVALID_ARG, "row_offsets are not a valid non-decreasing partition "
                                     "of [0, n_clusters]");
  if (c[C_ERR] & E_NONFINITE)
    return fail(TPC_ERR_INVALID_ARG, "%d clusters have non-finite coordinates", c[C_NONFINITE]);
  return TPC_OK;
}

int tpc_track_batch(tpc_ctx* ctx, const tpc_event* events, int n_events,
                    const tpc_geometry* geo, float bz_tesla, const tpc_params* params,
                    tpc_tracks* outs, void* hip_stream) {
  if (!ctx) return fail(TPC_ERR_INVALID_ARG, "ctx is null");
  return run_batch(ctx, events, n_events, geo, bz_tesla, params, outs, (hipStream_t)hip_stream);
}

int tpc_debug_links(tpc_ctx* ctx, const tpc_event* ev, const tpc_geometry* geo,
                    const tpc_params* params, int32_t* up, int32_t* dn, int32_t* up2,
                    int32_t* dn2, void* hip_stream) {
  if (!ctx) return fail(TPC_ERR_INVALID_ARG, "ctx is null");
  Outputs o{0, 0, nullptr, nullptr, nullptr, nullptr};
  hipStream_t st = (hipStream_t)hip_stream;
  Scratch sc;
  int rc = run_event(ctx, ev, geo, 0.f, params, o, STAGE_LINKS, st, &sc);
  if (rc) return rc;
  const size_t nb = sizeof(int32_t) * (size_t)ev->n_clusters;
  int32_t* dst[4] = {up, dn, up2, dn2};
  int32_t* src[4] = {sc.up, sc.dn, sc.up2, sc.dn2};
  for (int i = 0; i < 4; ++i) {
    if (!dst[i] || nb == 0) continue;
    hipError_t e = hipMemcpyAsync(dst[i], src[i], nb, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(links)");
  }
  hipError_t e = hipStreamSynchronize(st);
  return e == hipSuccess ? TPC_OK : hip_fail(e, "hipStreamSynchronize");
}

int tpc_debug_tracklets(tpc_ctx* ctx, const tpc_event* ev, const tpc_geometry* geo,
                        float bz_tesla, const tpc_params* params, int32_t cap,
                        int32_t* n_tracklets, int32_t* seeds, int32_t* hits, int32_t* row_lo,
                        int32_t* row_hi, int32_t* n, int32_t* ndf, float* chi2, float* par,
                        void* hip_stream) {
  if (!ctx || !n_tracklets || cap < 0) return fail(TPC_ERR_INVALID_ARG, "bad arguments");
  Outputs o{0, 0, nullptr, nullptr, nullptr, nullptr};
  hipStream_t st = (hipStream_t)hip_stream;
  Scratch sc;
  int rc = run_event(ctx, ev, geo, bz_tesla, params, o, STAGE_TRACKLETS, st, &sc);
  if (rc) return rc;
  const int32_t cnt = ctx->h_counters[C_SEEDS];
  *n_tracklets = cnt;
  if (cnt > cap) return fail(TPC_ERR_CAPACITY, "%d tracklets, capacity %d", cnt, cap);
  if (cnt > 0) {
    const size_t i4 = sizeof(int32_t) * (size_t)cnt;
    struct {
      void* d;
      const void* s;
      size_t b;
    } cp[] = {{seeds, sc.seeds, i4},   {row_lo, sc.row_lo, i4}, {row_hi, sc.row_hi, i4},
              {n, sc.n, i4},           {ndf, sc.ndf, i4},       {chi2, sc.chi2, i4},
              {par, sc.par, 6 * i4}};
    for (auto& x : cp) {
      if (!x.d) continue;
      hipError_t e = hipMemcpyAsync(x.d, x.s, x.b, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(tracklets)");
    }
    if (hits) {
      hipError_t e = hipMemcpy2DAsync(hits, sizeof(int32_t) * geo->n_rows, sc.hits,
                                      sizeof(int32_t) * kHitStride, sizeof(int32_t) * geo->n_rows,
                                      cnt, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return hip_fail(e, "hipMemcpy2DAsync(hits)");
    }
  }
  hipError_t e = hipStreamSynchronize(st);
  return e == hipSuccess ? TPC_OK : hip_fail(e, "hipStreamSynchronize");
}

}  // extern "C"
