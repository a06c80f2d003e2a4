// Serving loop of the tracker: events arrive one by one in host memory, are
// admitted while their device footprint fits a budget, are uploaded at once,
// and are tracked by worker threads as the GPU frees up: an event that finds
// a worker idle is tracked alone by the per-event path, events that queued
// behind busy workers are tracked together as one batch.  Several
// workers keep several batches in flight, so uploads, tracking and result
// downloads of different events overlap on the device.
//
// Each event's tracks are those it gets alone: batches never change results
// (tpc_track_batch), so an event's output does not depend on its neighbours.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/tpc_track.h"

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

thread_local std::string g_srv_err;

int srv_fail(int code, const std::string& msg) {
  g_srv_err = msg;
  return code;
}

// Caching allocator: buffers are kept per power-of-two size class.
class Pool {
 public:
  explicit Pool(bool host) : host_(host) {}
  ~Pool() {
    for (auto& kv : free_)
      for (void* p : kv.second) release(p);
  }
  void* get(size_t bytes) {
    size_t cls = 1 << 16;
    while (cls < bytes) cls <<= 1;
    std::lock_guard<std::mutex> g(m_);
    auto& v = free_[cls];
    if (!v.empty()) {
      void* p = v.back();
      v.pop_back();
      size_of_[p] = cls;
      return p;
    }
    void* p = nullptr;
    hipError_t e = host_ ? hipHostMalloc(&p, cls, hipHostMallocDefault) : hipMalloc(&p, cls);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    size_of_[p] = cls;
    return p;
  }
  void put(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(m_);
    free_[size_of_[p]].push_back(p);
  }

 private:
  void release(void* p) {
    if (host_)
      (void)hipHostFree(p);
    else
      (void)hipFree(p);
  }
  bool host_;
  std::mutex m_;
  std::map<size_t, std::vector<void*>> free_;
  std::unordered_map<void*, size_t> size_of_;
};

struct Job {
  uint64_t tag = 0;
  int32_t n_sectors = 0, n_rows = 0;
  int64_t n_clusters = 0;
  size_t footprint = 0;
  double t_submit = 0, t_done = 0;
  int status = 0;
  int32_t n_tracks = 0, n_track_clusters = 0;
  int32_t cap_tracks = 0;
  // device: inputs, outputs
  void* d_in = nullptr;   // y, z, row_offsets, sector_id
  void* d_out = nullptr;  // track_par, track_meta, track_cluster, cluster_track
  // pinned host: staged inputs, then results
  void* h_in = nullptr;
  void* h_out = nullptr;
  hipEvent_t uploaded = nullptr;
};

inline size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

struct tpc_server {
  tpc_server_config cfg;
  tpc_geometry geo;
  std::vector<float> row_x;
  float bz;
  tpc_params prm;
  Pool dpool{false}, hpool{true};
  hipStream_t copy_stream = nullptr;
  std::mutex m;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> ready;                  // uploaded, waiting for a worker
  std::deque<Job*> done;                   // finished, not yet polled
  std::unordered_map<uint64_t, Job*> kept; // polled, results not yet fetched
  size_t resident = 0;                     // device footprint of admitted events
  int64_t batches = 0, events_done = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::vector<tpc_ctx*> ctxs;
};

namespace {

size_t footprint_of(const tpc_server* s, int64_t n, int32_t n_sectors) {
  // inputs and outputs of the event plus its share of a worker's scratch
  // (grid, links, owner keys, tracklets): a conservative 160 B per cluster
  return (size_t)n * 160 + (size_t)n_sectors * s->geo.n_rows * 16 + (1 << 16);
}

void worker_main(tpc_server* s, int wi) {
  tpc_ctx* ctx = s->ctxs[wi];
  hipStream_t st = nullptr;
  (void)hipSetDevice(s->cfg.device);
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
  std::vector<Job*> jobs;
  std::vector<tpc_event> evs;
  std::vector<tpc_tracks> outs;
  std::vector<int32_t> nts, ncs;
  for (;;) {
    jobs.clear();
    {
      std::unique_lock<std::mutex> g(s->m);
      s->cv_work.wait(g, [&] { return s->stop || !s->ready.empty(); });
      if (s->stop && s->ready.empty()) break;
      while (!s->ready.empty() && (int)jobs.size() < s->cfg.max_batch) {
        jobs.push_back(s->ready.front());
        s->ready.pop_front();
      }
    }
    const int E = (int)jobs.size();
    evs.resize(E);
    outs.resize(E);
    nts.assign(E, 0);
    ncs.assign(E, 0);
    for (int i = 0; i < E; ++i) {
      Job* j = jobs[i];
      (void)hipStreamWaitEvent(st, j->uploaded, 0);
      char* in = (char*)j->d_in;
      const size_t n = (size_t)j->n_clusters, nro = (size_t)j->n_sectors * j->n_rows + 1;
      tpc_event& e = evs[i];
      e.n_sectors = j->n_sectors;
      e.n_clusters = j->n_clusters;
      e.y = (const float*)in;
      e.z = (const float*)(in + al(4 * n));
      e.row_offsets = (const int32_t*)(in + 2 * al(4 * n));
      e.sector_id = (const int32_t*)(in + 2 * al(4 * n) + al(4 * nro));
      char* out = (char*)j->d_out;
      tpc_tracks& o = outs[i];
      o.cap_tracks = j->cap_tracks;
      o.cap_track_clusters = (int32_t)n;
      o.n_tracks = &nts[i];
      o.n_track_clusters = &ncs[i];
      o.track_par = (float*)out;
      o.track_meta = (int32_t*)(out + al(32 * (size_t)j->cap_tracks));
      o.track_cluster = (int32_t*)(out + al(32 * (size_t)j->cap_tracks) + al(16 * (size_t)j->cap_tracks));
      o.cluster_track = (int32_t*)((char*)o.track_cluster + al(4 * n));
    }
    // a lone event (it arrived at an idle worker) takes the plain per-event
    // path at once; events that queued behind busy workers go as one batch
    const int rc = E == 1 ? tpc_track_event(ctx, &evs[0], &s->geo, s->bz, &s->prm, &outs[0], st)
                          : tpc_track_batch(ctx, evs.data(), E, &s->geo, s->bz, &s->prm,
                                            outs.data(), st);
    // results back to pinned host memory
    for (int i = 0; i < E && rc == TPC_OK; ++i) {
      Job* j = jobs[i];
      if (!s->cfg.keep_results) continue;
      char* h = (char*)j->h_out;
      const size_t n = (size_t)j->n_clusters;
      const size_t nt = (size_t)nts[i], nc = (size_t)ncs[i];
      (void)hipMemcpyAsync(h, outs[i].track_par, 32 * nt, hipMemcpyDeviceToHost, st);
      (void)hipMemcpyAsync(h + al(32 * (size_t)j->cap_tracks), outs[i].track_meta, 16 * nt,
                           hipMemcpyDeviceToHost, st);
      (void)hipMemcpyAsync(h + al(32 * (size_t)j->cap_tracks) + al(16 * (size_t)j->cap_tracks),
                           outs[i].track_cluster, 4 * nc, hipMemcpyDeviceToHost, st);
      (void)hipMemcpyAsync(h + al(32 * (size_t)j->cap_tracks) + al(16 * (size_t)j->cap_tracks) +
                               al(4 * n),
                           outs[i].cluster_track, 4 * n, hipMemcpyDeviceToHost, st);
    }
    (void)hipStreamSynchronize(st);
    const double t = now_s();
    {
      std::lock_guard<std::mutex> g(s->m);
      for (int i = 0; i < E; ++i) {
        Job* j = jobs[i];
        j->status = rc;
        j->n_tracks = nts[i];
        j->n_track_clusters = ncs[i];
        j->t_done = t;
        s->dpool.put(j->d_in);
        s->dpool.put(j->d_out);
        j->d_in = j->d_out = nullptr;
        s->resident -= j->footprint;
        s->done.push_back(j);
      }
      s->batches += 1;
      s->events_done += E;
    }
    s->cv_done.notify_all();
  }
  (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" {

void tpc_server_config_default(tpc_server_config* c) {
  if (!c) return;
  c->device = 0;
  c->hbm_budget_bytes = (size_t)32 << 30;
  c->max_batch = 64;
  c->n_workers = 2;
  c->use_graph = 1;
  c->keep_results = 1;
}

int tpc_server_create(const tpc_server_config* cfg, const tpc_geometry* geo, float bz_tesla,
                      const tpc_params* params, tpc_server** out) {
  if (!cfg || !geo || !params || !out) return srv_fail(TPC_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (cfg->max_batch < 1 || cfg->n_workers < 1 || cfg->n_workers > 16)
    return srv_fail(TPC_ERR_INVALID_ARG, "max_batch >= 1 and n_workers in [1, 16]");
  if (geo->n_rows < 3 || geo->n_rows > TPC_MAX_ROWS || !geo->row_x)
    return srv_fail(TPC_ERR_INVALID_ARG, "bad geometry");
  tpc_server* s = new (std::nothrow) tpc_server();
  if (!s) return srv_fail(TPC_ERR_OOM, "host allocation");
  s->cfg = *cfg;
  s->row_x.assign(geo->row_x, geo->row_x + geo->n_rows);
  s->geo = *geo;
  s->geo.row_x = s->row_x.data();
  s->bz = bz_tesla;
  s->prm = *params;
  if (hipSetDevice(cfg->device) != hipSuccess ||
      hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) != hipSuccess) {
    delete s;
    return srv_fail(TPC_ERR_DEVICE, "stream creation failed");
  }
  tpc_tuning tu;
  tpc_tuning_default(&tu);
  tu.use_graph = cfg->use_graph;
  for (int i = 0; i < cfg->n_workers; ++i) {
    tpc_ctx* c = nullptr;
    int rc = tpc_ctx_create(cfg->device, 0, &c);
    if (rc) {
      for (tpc_ctx* x : s->ctxs) tpc_ctx_destroy(x);
      (void)hipStreamDestroy(s->copy_stream);
      delete s;
      return srv_fail(rc, std::string("context: ") + tpc_last_error());
    }
    tpc_ctx_set_tuning(c, &tu);
    s->ctxs.push_back(c);
  }
  for (int i = 0; i < cfg->n_workers; ++i) s->workers.emplace_back(worker_main, s, i);
  *out = s;
  return TPC_OK;
}

int tpc_server_submit(tpc_server* s, const tpc_event* ev, uint64_t tag) {
  if (!s || !ev) return srv_fail(TPC_ERR_INVALID_ARG, "null argument");
  const double t0 = now_s();
  int rc = tpc_validate(ev, &s->geo, &s->prm);
  if (rc) return srv_fail(rc, tpc_last_error());
  const size_t n = (size_t)ev->n_clusters, nro = (size_t)ev->n_sectors * s->geo.n_rows + 1;
  const size_t fp = footprint_of(s, ev->n_clusters, ev->n_sectors);
  {
    std::lock_guard<std::mutex> g(s->m);
    if (s->stop) return srv_fail(TPC_ERR_INVALID_ARG, "server is stopping");
    if (s->resident + fp > s->cfg.hbm_budget_bytes) {
      if (fp > s->cfg.hbm_budget_bytes)
        return srv_fail(TPC_ERR_OOM, "event larger than the whole budget");
      return srv_fail(TPC_ERR_BUSY, "not admitted now: device budget in use");
    }
    s->resident += fp;
  }
  Job* j = new (std::nothrow) Job();
  if (!j) return srv_fail(TPC_ERR_OOM, "host allocation");
  j->tag = tag;
  j->n_sectors = ev->n_sectors;
  j->n_rows = s->geo.n_rows;
  j->n_clusters = ev->n_clusters;
  j->footprint = fp;
  j->t_submit = t0;
  j->cap_tracks = (int32_t)(n / (size_t)s->prm.min_clusters + 1);
  const size_t in_bytes = 2 * al(4 * n) + al(4 * nro) + al(4 * (size_t)ev->n_sectors);
  const size_t out_bytes = al(32 * (size_t)j->cap_tracks) + al(16 * (size_t)j->cap_tracks) +
                           2 * al(4 * n);
  (void)hipSetDevice(s->cfg.device);
  j->d_in = s->dpool.get(in_bytes);
  j->d_out = s->dpool.get(out_bytes);
  j->h_in = s->hpool.get(in_bytes);
  j->h_out = s->cfg.keep_results ? s->hpool.get(out_bytes) : nullptr;
  bool ok = j->d_in && j->d_out && j->h_in && (j->h_out || !s->cfg.keep_results);
  ok = ok && hipEventCreateWithFlags(&j->uploaded, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    s->dpool.put(j->d_in);
    s->dpool.put(j->d_out);
    s->hpool.put(j->h_in);
    s->hpool.put(j->h_out);
    std::lock_guard<std::mutex> g(s->m);
    s->resident -= fp;
    delete j;
    return srv_fail(TPC_ERR_OOM, "buffers for the event");
  }
  // stage in pinned memory, then one upload on the copy stream
  char* h = (char*)j->h_in;
  std::memcpy(h, ev->y, 4 * n);
  std::memcpy(h + al(4 * n), ev->z, 4 * n);
  std::memcpy(h + 2 * al(4 * n), ev->row_offsets, 4 * nro);
  std::memcpy(h + 2 * al(4 * n) + al(4 * nro), ev->sector_id, 4 * (size_t)ev->n_sectors);
  hipError_t e = hipMemcpyAsync(j->d_in, h, in_bytes, hipMemcpyHostToDevice, s->copy_stream);
  if (e == hipSuccess) e = hipEventRecord(j->uploaded, s->copy_stream);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(s->copy_stream);
    s->dpool.put(j->d_in);
    s->dpool.put(j->d_out);
    s->hpool.put(j->h_in);
    s->hpool.put(j->h_out);
    (void)hipEventDestroy(j->uploaded);
    delete j;
    std::lock_guard<std::mutex> g(s->m);
    s->resident -= fp;
    return srv_fail(TPC_ERR_DEVICE, hipGetErrorString(e));
  }
  {
    std::lock_guard<std::mutex> g(s->m);
    s->ready.push_back(j);
  }
  s->cv_work.notify_one();
  return TPC_OK;
}

int tpc_server_poll(tpc_server* s, tpc_server_done* out, int max, int* n_done, int timeout_ms) {
  if (!s || !out || !n_done || max < 1) return srv_fail(TPC_ERR_INVALID_ARG, "bad arguments");
  std::unique_lock<std::mutex> g(s->m);
  if (s->done.empty() && timeout_ms > 0)
    s->cv_done.wait_for(g, std::chrono::milliseconds(timeout_ms), [&] { return !s->done.empty(); });
  int k = 0;
  while (!s->done.empty() && k < max) {
    Job* j = s->done.front();
    s->done.pop_front();
    tpc_server_done& d = out[k++];
    d.tag = j->tag;
    d.status = j->status;
    d.n_tracks = j->n_tracks;
    d.n_track_clusters = j->n_track_clusters;
    d.t_submit = j->t_submit;
    d.t_done = j->t_done;
    if (s->cfg.keep_results && j->status == TPC_OK) {
      s->kept[j->tag] = j;
    } else {
      s->hpool.put(j->h_in);
      s->hpool.put(j->h_out);
      (void)hipEventDestroy(j->uploaded);
      delete j;
    }
  }
  *n_done = k;
  return TPC_OK;
}

int tpc_server_fetch(tpc_server* s, uint64_t tag, float* track_par, int32_t* track_meta,
                     int32_t* track_cluster, int32_t* cluster_track) {
  if (!s) return srv_fail(TPC_ERR_INVALID_ARG, "null server");
  Job* j;
  {
    std::lock_guard<std::mutex> g(s->m);
    auto it = s->kept.find(tag);
    if (it == s->kept.end()) return srv_fail(TPC_ERR_INVALID_ARG, "no kept result for this tag");
    j = it->second;
    s->kept.erase(it);
  }
  const char* h = (const char*)j->h_out;
  const size_t n = (size_t)j->n_clusters, nt = (size_t)j->n_tracks, nc = (size_t)j->n_track_clusters;
  const size_t o_meta = al(32 * (size_t)j->cap_tracks);
  const size_t o_tcl = o_meta + al(16 * (size_t)j->cap_tracks);
  const size_t o_ctr = o_tcl + al(4 * n);
  if (track_par) std::memcpy(track_par, h, 32 * nt);
  if (track_meta) std::memcpy(track_meta, h + o_meta, 16 * nt);
  if (track_cluster) std::memcpy(track_cluster, h + o_tcl, 4 * nc);
  if (cluster_track) std::memcpy(cluster_track, h + o_ctr, 4 * n);
  s->hpool.put(j->h_in);
  s->hpool.put(j->h_out);
  (void)hipEventDestroy(j->uploaded);
  delete j;
  return TPC_OK;
}

double tpc_server_now(void) { return now_s(); }

int tpc_server_stats(tpc_server* s, int64_t* batches, int64_t* events, size_t* resident) {
  if (!s) return srv_fail(TPC_ERR_INVALID_ARG, "null server");
  std::lock_guard<std::mutex> g(s->m);
  if (batches) *batches = s->batches;
  if (events) *events = s->events_done;
  if (resident) *resident = s->resident;
  return TPC_OK;
}

const char* tpc_server_last_error(void) { return g_srv_err.c_str(); }

void tpc_server_destroy(tpc_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->m);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  for (tpc_ctx* c : s->ctxs) tpc_ctx_destroy(c);
  (void)hipStreamSynchronize(s->copy_stream);
  for (Job* j : s->done) {
    s->hpool.put(j->h_in);
    s->hpool.put(j->h_out);
    (void)hipEventDestroy(j->uploaded);
    delete j;
  }
  for (auto& kv : s->kept) {
    s->hpool.put(kv.second->h_in);
    s->hpool.put(kv.second->h_out);
    (void)hipEventDestroy(kv.second->uploaded);
    delete kv.second;
  }
  (void)hipStreamDestroy(s->copy_stream);
  delete s;
}

}  // extern "C"
