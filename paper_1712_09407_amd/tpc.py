"""Python binding of libtpctrack.so (the C ABI in include/tpc_track.h).

Argument marshalling only: every step of the tracker runs in the library's
HIP kernels.  PyTorch provides device memory and the stream.  If the library
is not built, importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtpctrack.so")

TPC_OK, TPC_ERR_INVALID_ARG, TPC_ERR_CAPACITY, TPC_ERR_OOM, TPC_ERR_DEVICE, \
    TPC_ERR_OVERFLOW, TPC_ERR_BUSY = range(7)
TPC_MAX_ROWS = 160


class TpcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tpc error {code}: {msg}")
        self.code = code


class Geometry(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("row_x", C.POINTER(C.c_float)),
                ("tan_half_angle", C.c_float), ("z_max", C.c_float)]


class Event(C.Structure):
    _fields_ = [("n_sectors", C.c_int32), ("sector_id", C.c_void_p), ("n_clusters", C.c_int64),
                ("y", C.c_void_p), ("z", C.c_void_p), ("row_offsets", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("sigma_y", C.c_float), ("sigma_z", C.c_float), ("nf_win_y", C.c_float),
                ("nf_win_z", C.c_float), ("nf_chi2_max", C.c_float), ("min_seed_len", C.c_int32),
                ("seed_window", C.c_int32),
                ("chi2_gate", C.c_float), ("max_miss", C.c_int32), ("max_sinphi", C.c_float),
                ("alpha", C.c_float), ("beta", C.c_float), ("min_clusters", C.c_int32),
                ("min_pt", C.c_float), ("prior_sinphi", C.c_float), ("prior_tanl", C.c_float),
                ("prior_qpt", C.c_float), ("max_tracklets", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("use_graph", C.c_int32), ("construct_blocks", C.c_int32),
                ("bin_occupancy", C.c_float), ("construct_schedule", C.c_int32),
                ("construct_lanes", C.c_int32), ("nf_stage", C.c_int32),
                ("own_order", C.c_int32)]


class ServerConfig(C.Structure):
    _fields_ = [("device", C.c_int32), ("hbm_budget_bytes", C.c_size_t),
                ("max_batch", C.c_int32), ("n_workers", C.c_int32), ("use_graph", C.c_int32),
                ("keep_results", C.c_int32)]


class ServerDone(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("status", C.c_int32), ("n_tracks", C.c_int32),
                ("n_track_clusters", C.c_int32), ("t_submit", C.c_double),
                ("t_done", C.c_double)]


class Tracks(C.Structure):
    _fields_ = [("cap_tracks", C.c_int32), ("cap_track_clusters", C.c_int32),
                ("n_tracks", C.POINTER(C.c_int32)), ("n_track_clusters", C.POINTER(C.c_int32)),
                ("track_par", C.c_void_p), ("track_meta", C.c_void_p),
                ("track_cluster", C.c_void_p), ("cluster_track", C.c_void_p)]


class Prolongations(C.Structure):
    _fields_ = [("cap", C.c_int32), ("cap_clusters", C.c_int32), ("n", C.POINTER(C.c_int32)),
                ("n_clusters", C.POINTER(C.c_int32)), ("par", C.c_void_p), ("meta", C.c_void_p),
                ("cluster", C.c_void_p)]


class Merged(C.Structure):
    _fields_ = [("cap", C.c_int32), ("cap_clusters", C.c_int32), ("n", C.POINTER(C.c_int32)),
                ("n_clusters", C.POINTER(C.c_int32)), ("par", C.c_void_p), ("meta", C.c_void_p),
                ("cluster", C.c_void_p), ("track_merged", C.c_void_p)]


MERGE_CHI2 = 25.0   # joins: chi^2(5) <= 25, a 1e-4 tail for the same particle

EXPORTS = ["tpc_params_default", "tpc_validate", "tpc_ctx_create", "tpc_ctx_destroy",
           "tpc_track_event", "tpc_track_event_global", "tpc_track_event_merged", "tpc_refit",
           "tpc_track_batch", "tpc_debug_links", "tpc_debug_tracklets", "tpc_last_error",
           "tpc_kernel_count", "tpc_kernel_name", "tpc_ctx_set_timing", "tpc_ctx_get_stats",
           "tpc_ctx_reset_stats", "tpc_track_event_noalloc", "tpc_tuning_default",
           "tpc_ctx_set_tuning",
           "tpc_ctx_graph_launches", "tpc_server_config_default", "tpc_server_create",
           "tpc_server_submit", "tpc_server_poll", "tpc_server_fetch", "tpc_server_stats",
           "tpc_server_now", "tpc_server_last_error", "tpc_server_destroy"]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    L.tpc_params_default.argtypes = [P(Params)]
    L.tpc_params_default.restype = None
    L.tpc_validate.argtypes = [P(Event), P(Geometry), P(Params)]
    L.tpc_ctx_create.argtypes = [C.c_int, C.c_size_t, P(C.c_void_p)]
    L.tpc_ctx_destroy.argtypes = [C.c_void_p]
    L.tpc_ctx_destroy.restype = None
    L.tpc_track_event.argtypes = [C.c_void_p, P(Event), P(Geometry), C.c_float, P(Params),
                                  P(Tracks), C.c_void_p]
    L.tpc_track_event_noalloc.argtypes = [C.c_void_p, P(Event), P(Geometry), C.c_float,
                                          P(Params), P(Tracks), C.c_void_p]
    L.tpc_track_event_global.argtypes = [C.c_void_p, P(Event), P(Geometry), C.c_float,
                                         P(Params), P(Tracks), P(Prolongations), C.c_void_p]
    L.tpc_track_event_merged.argtypes = [C.c_void_p, P(Event), P(Geometry), C.c_float,
                                         P(Params), C.c_float, P(Tracks), P(Prolongations),
                                         P(Merged), C.c_void_p]
    L.tpc_refit.argtypes = [C.c_void_p, P(Event), P(Geometry), C.c_float, P(Params), C.c_int32,
                            C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                            C.c_void_p]
    L.tpc_track_batch.argtypes = [C.c_void_p, P(Event), C.c_int, P(Geometry), C.c_float,
                                  P(Params), P(Tracks), C.c_void_p]
    L.tpc_debug_links.argtypes = [C.c_void_p, P(Event), P(Geometry), P(Params), C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.tpc_debug_tracklets.argtypes = [C.c_void_p, P(Event), P(Geometry), C.c_float, P(Params),
                                      C.c_int32, P(C.c_int32)] + [C.c_void_p] * 9
    L.tpc_kernel_count.argtypes = []
    L.tpc_kernel_name.argtypes = [C.c_int]
    L.tpc_kernel_name.restype = C.c_char_p
    L.tpc_ctx_set_timing.argtypes = [C.c_void_p, C.c_uint32]
    L.tpc_ctx_get_stats.argtypes = [C.c_void_p, P(C.c_double), P(C.c_int64), P(C.c_int64)]
    L.tpc_ctx_reset_stats.argtypes = [C.c_void_p]
    L.tpc_tuning_default.argtypes = [P(Tuning)]
    L.tpc_tuning_default.restype = None
    L.tpc_ctx_set_tuning.argtypes = [C.c_void_p, P(Tuning)]
    L.tpc_ctx_graph_launches.argtypes = [C.c_void_p, P(C.c_int64)]
    L.tpc_server_config_default.argtypes = [P(ServerConfig)]
    L.tpc_server_config_default.restype = None
    L.tpc_server_create.argtypes = [P(ServerConfig), P(Geometry), C.c_float, P(Params),
                                    P(C.c_void_p)]
    L.tpc_server_submit.argtypes = [C.c_void_p, P(Event), C.c_uint64]
    L.tpc_server_poll.argtypes = [C.c_void_p, P(ServerDone), C.c_int, P(C.c_int), C.c_int]
    L.tpc_server_fetch.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p]
    L.tpc_server_stats.argtypes = [C.c_void_p, P(C.c_int64), P(C.c_int64), P(C.c_size_t)]
    L.tpc_server_now.argtypes = []
    L.tpc_server_now.restype = C.c_double
    L.tpc_server_last_error.argtypes = []
    L.tpc_server_last_error.restype = C.c_char_p
    L.tpc_server_destroy.argtypes = [C.c_void_p]
    L.tpc_server_destroy.restype = None
    L.tpc_last_error.argtypes = []
    L.tpc_last_error.restype = C.c_char_p
    return L


lib = _load()


def _check(rc):
    if rc != TPC_OK:
        raise TpcError(rc, lib.tpc_last_error().decode())


def default_params(**over) -> Params:
    p = Params()
    lib.tpc_params_default(C.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def validate(e: Event, geo: Geometry, params: Params = None) -> int:
    """Host-only argument checks; returns the TPC_* code."""
    return lib.tpc_validate(C.byref(e), C.byref(geo), C.byref(params or default_params()))


def last_error() -> str:
    return lib.tpc_last_error().decode()


def make_geometry(row_x, tan_half_angle, z_max):
    rx = np.ascontiguousarray(row_x, np.float32)
    g = Geometry(int(rx.shape[0]), rx.ctypes.data_as(C.POINTER(C.c_float)),
                 float(tan_half_angle), float(z_max))
    g._keep = rx
    return g


class DeviceEvent:
    """An event resident in device memory (torch tensors on the GPU)."""

    def __init__(self, y, z, row_offsets, sector_id):
        self.y, self.z, self.row_offsets, self.sector_id = y, z, row_offsets, sector_id

    @classmethod
    def from_host(cls, y, z, row_offsets, sector_id, device="cuda"):
        import torch
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dt)).to(device)
        return cls(t(y, np.float32), t(z, np.float32), t(row_offsets, np.int32),
                   t(sector_id, np.int32))

    @property
    def n_clusters(self):
        return int(self.y.shape[0])

    def cstruct(self) -> Event:
        for a in (self.y, self.z, self.row_offsets, self.sector_id):
            assert a.is_cuda and a.is_contiguous()
        return Event(int(self.sector_id.shape[0]), self.sector_id.data_ptr(),
                     self.n_clusters, self.y.data_ptr(), self.z.data_ptr(),
                     self.row_offsets.data_ptr())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Tracker:
    """One library context on one GPU."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = C.c_void_p()
        _check(lib.tpc_ctx_create(int(device), int(hbm_budget_bytes), C.byref(h)))
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            lib.tpc_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def track_event(self, ev: DeviceEvent, geo: Geometry, bz: float, params: Params = None,
                    cap_tracks: int = None, cap_track_clusters: int = None, stream=None,
                    out=None):
        """Run the whole path.  Returns a dict of device tensors trimmed to size.
        `out` may hold preallocated outputs (track_par, track_meta, track_cluster,
        cluster_track) to avoid allocation per call."""
        import torch
        n = ev.n_clusters
        dev = ev.y.device
        if out is None:
            ct = cap_tracks if cap_tracks is not None else max(16, n // 40)
            cc = cap_track_clusters if cap_track_clusters is not None else max(16, n)
            out = dict(track_par=torch.empty((ct, 8), dtype=torch.float32, device=dev),
                       track_meta=torch.empty((ct, 4), dtype=torch.int32, device=dev),
                       track_cluster=torch.empty(cc, dtype=torch.int32, device=dev),
                       cluster_track=torch.empty(max(n, 1), dtype=torch.int32, device=dev))
        nt, nc = C.c_int32(0), C.c_int32(0)
        tr = Tracks(int(out["track_par"].shape[0]), int(out["track_cluster"].shape[0]),
                    C.pointer(nt), C.pointer(nc), out["track_par"].data_ptr(),
                    out["track_meta"].data_ptr(), out["track_cluster"].data_ptr(),
                    out["cluster_track"].data_ptr())
        e = ev.cstruct()
        rc = lib.tpc_track_event(self._h, C.byref(e), C.byref(geo), float(bz),
                                 C.byref(params or default_params()), C.byref(tr),
                                 _stream_handle(stream))
        if rc == TPC_ERR_CAPACITY and (cap_tracks is None and cap_track_clusters is None):
            return self.track_event(ev, geo, bz, params, nt.value + 16, nc.value + 16, stream)
        _check(rc)
        return dict(n_tracks=nt.value, n_track_clusters=nc.value,
                    track_par=out["track_par"][:nt.value], track_meta=out["track_meta"][:nt.value],
                    track_cluster=out["track_cluster"][:nc.value],
                    cluster_track=out["cluster_track"][:n])

    def track_event_global(self, ev: DeviceEvent, geo: Geometry, bz: float,
                           params: Params = None, cap_tracks: int = None,
                           cap_track_clusters: int = None, cap_pro: int = None,
                           cap_pro_clusters: int = None, stream=None):
        """The whole path, then global tracking (section 5).  Returns the
        track dict of track_event and a dict of the prolongations (n,
        n_clusters, par [n][8], meta [n][5], cluster), device tensors."""
        import torch
        n = ev.n_clusters
        dev = ev.y.device
        auto = all(c is None for c in (cap_tracks, cap_track_clusters, cap_pro, cap_pro_clusters))
        ct = cap_tracks if cap_tracks is not None else max(16, n // 40)
        cc = cap_track_clusters if cap_track_clusters is not None else max(16, n)
        cp = cap_pro if cap_pro is not None else max(16, ct)
        cpc = cap_pro_clusters if cap_pro_clusters is not None else max(16, n // 8)
        f32 = dict(dtype=torch.float32, device=dev)
        i32 = dict(dtype=torch.int32, device=dev)
        out = dict(track_par=torch.empty((ct, 8), **f32), track_meta=torch.empty((ct, 4), **i32),
                   track_cluster=torch.empty(cc, **i32),
                   cluster_track=torch.empty(max(n, 1), **i32))
        po = dict(par=torch.empty((max(cp, 1), 8), **f32), meta=torch.empty((max(cp, 1), 5), **i32),
                  cluster=torch.empty(max(cpc, 1), **i32))
        nt, nc, npr, npc = C.c_int32(0), C.c_int32(0), C.c_int32(0), C.c_int32(0)
        tr = Tracks(ct, cc, C.pointer(nt), C.pointer(nc), out["track_par"].data_ptr(),
                    out["track_meta"].data_ptr(), out["track_cluster"].data_ptr(),
                    out["cluster_track"].data_ptr())
        pr = Prolongations(cp, cpc, C.pointer(npr), C.pointer(npc), po["par"].data_ptr(),
                           po["meta"].data_ptr(), po["cluster"].data_ptr())
        e = ev.cstruct()
        rc = lib.tpc_track_event_global(self._h, C.byref(e), C.byref(geo), float(bz),
                                        C.byref(params or default_params()), C.byref(tr),
                                        C.byref(pr), _stream_handle(stream))
        if rc == TPC_ERR_CAPACITY and auto:
            return self.track_event_global(ev, geo, bz, params, max(ct, nt.value + 16),
                                           max(cc, nc.value + 16), max(cp, npr.value + 16),
                                           max(cpc, npc.value + 16), stream)
        _check(rc)
        tracks = dict(n_tracks=nt.value, n_track_clusters=nc.value,
                      track_par=out["track_par"][:nt.value],
                      track_meta=out["track_meta"][:nt.value],
                      track_cluster=out["track_cluster"][:nc.value],
                      cluster_track=out["cluster_track"][:n])
        pro = dict(n=npr.value, n_clusters=npc.value, par=po["par"][:npr.value],
                   meta=po["meta"][:npr.value], cluster=po["cluster"][:npc.value])
        return tracks, pro

    def track_event_merged(self, ev: DeviceEvent, geo: Geometry, bz: float,
                           params: Params = None, merge_chi2: float = MERGE_CHI2,
                           use_global: bool = True, cap_merged: int = None,
                           cap_merged_clusters: int = None, stream=None):
        """The whole path (with global tracking if use_global), then the track
        merger with refit.  Returns (tracks, prolongations or None, merged):
        merged has n, n_clusters, par [n][8], meta [n][5], cluster and
        track_merged [n_tracks] (device tensors)."""
        import torch
        n = ev.n_clusters
        dev = ev.y.device
        ct, cc = max(16, n // 40), max(16, n)
        cp, cpc = max(16, ct), max(16, n // 8)
        cm = cap_merged if cap_merged is not None else ct
        cmc = cap_merged_clusters if cap_merged_clusters is not None else max(16, n + n // 8)
        auto = cap_merged is None and cap_merged_clusters is None
        for _ in range(3):
            f32 = dict(dtype=torch.float32, device=dev)
            i32 = dict(dtype=torch.int32, device=dev)
            out = dict(track_par=torch.empty((ct, 8), **f32),
                       track_meta=torch.empty((ct, 4), **i32),
                       track_cluster=torch.empty(cc, **i32),
                       cluster_track=torch.empty(max(n, 1), **i32))
            po = dict(par=torch.empty((cp, 8), **f32), meta=torch.empty((cp, 5), **i32),
                      cluster=torch.empty(cpc, **i32))
            mo = dict(par=torch.empty((max(cm, 1), 8), **f32),
                      meta=torch.empty((max(cm, 1), 5), **i32),
                      cluster=torch.empty(max(cmc, 1), **i32),
                      track_merged=torch.empty(ct, **i32))
            sz = [C.c_int32(0) for _ in range(6)]
            tr = Tracks(ct, cc, C.pointer(sz[0]), C.pointer(sz[1]), out["track_par"].data_ptr(),
                        out["track_meta"].data_ptr(), out["track_cluster"].data_ptr(),
                        out["cluster_track"].data_ptr())
            pr = Prolongations(cp, cpc, C.pointer(sz[2]), C.pointer(sz[3]), po["par"].data_ptr(),
                               po["meta"].data_ptr(), po["cluster"].data_ptr())
            mg = Merged(cm, cmc, C.pointer(sz[4]), C.pointer(sz[5]), mo["par"].data_ptr(),
                        mo["meta"].data_ptr(), mo["cluster"].data_ptr(),
                        mo["track_merged"].data_ptr())
            e = ev.cstruct()
            rc = lib.tpc_track_event_merged(self._h, C.byref(e), C.byref(geo), float(bz),
                                            C.byref(params or default_params()),
                                            float(merge_chi2), C.byref(tr),
                                            C.byref(pr) if use_global else None, C.byref(mg),
                                            _stream_handle(stream))
            if rc == TPC_ERR_CAPACITY and auto:
                v = [x.value for x in sz]
                ct, cc = max(ct, v[0] + 16), max(cc, v[1] + 16)
                cp, cpc = max(cp, v[2] + 16), max(cpc, v[3] + 16)
                cm, cmc = max(cm, v[4] + 16, ct), max(cmc, v[5] + 16)
                continue
            _check(rc)
            v = [x.value for x in sz]
            tracks = dict(n_tracks=v[0], n_track_clusters=v[1], track_par=out["track_par"][:v[0]],
                          track_meta=out["track_meta"][:v[0]],
                          track_cluster=out["track_cluster"][:v[1]],
                          cluster_track=out["cluster_track"][:n])
            pro = dict(n=v[2], n_clusters=v[3], par=po["par"][:v[2]], meta=po["meta"][:v[2]],
                       cluster=po["cluster"][:v[3]]) if use_global else None
            merged = dict(n=v[4], n_clusters=v[5], par=mo["par"][:v[4]], meta=mo["meta"][:v[4]],
                          cluster=mo["cluster"][:v[5]], track_merged=mo["track_merged"][:v[0]])
            return tracks, pro, merged
        raise TpcError(TPC_ERR_CAPACITY, "capacity retry failed")

    def refit(self, ev: DeviceEvent, geo: Geometry, bz: float, offsets, clusters,
              params: Params = None, stream=None):
        """The merger's refit of cluster lists (device int32 tensors: offsets
        [n + 1], clusters).  Returns (par [n][8], frame sector_id [n])."""
        import torch
        n = int(offsets.shape[0]) - 1
        dev = ev.y.device
        par = torch.empty((max(n, 1), 8), dtype=torch.float32, device=dev)
        fr = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        for a in (offsets, clusters):
            assert a.is_cuda and a.is_contiguous() and a.dtype == torch.int32
        e = ev.cstruct()
        _check(lib.tpc_refit(self._h, C.byref(e), C.byref(geo), float(bz),
                             C.byref(params or default_params()), n, int(clusters.shape[0]),
                             offsets.data_ptr(), clusters.data_ptr(), par.data_ptr(),
                             fr.data_ptr(), _stream_handle(stream)))
        return par[:n], fr[:n]

    def set_tuning(self, **kw):
        """Speed knobs (results never change): use_graph, construct_blocks,
        bin_occupancy, construct_schedule, construct_lanes, nf_stage, own_order.  Unnamed
        knobs keep their defaults."""
        tu = Tuning()
        lib.tpc_tuning_default(C.byref(tu))
        for k, v in kw.items():
            setattr(tu, k, v)
        _check(lib.tpc_ctx_set_tuning(self._h, C.byref(tu)))
        return {k: getattr(tu, k) for k, _ in Tuning._fields_}

    def graph_launches(self) -> int:
        n = C.c_int64(0)
        _check(lib.tpc_ctx_graph_launches(self._h, C.byref(n)))
        return n.value

    def set_timing(self, kernels=None):
        """Time the named kernels (None = all, [] = off) with HIP events."""
        names = kernel_names()
        mask = (1 << len(names)) - 1 if kernels is None else \
            sum(1 << names.index(k) for k in kernels)
        _check(lib.tpc_ctx_set_timing(self._h, mask))

    def stats(self):
        nk = lib.tpc_kernel_count()
        ms = (C.c_double * nk)()
        cnt = (C.c_int64 * nk)()
        work = (C.c_int64 * 5)()
        _check(lib.tpc_ctx_get_stats(self._h, ms, cnt, work))
        names = kernel_names()
        return dict(kernel_ms={names[i]: ms[i] for i in range(nk)},
                    kernel_launches={names[i]: cnt[i] for i in range(nk)},
                    events=work[0], tracklets=work[1], steps=work[2], updates=work[3],
                    candidates=work[4])

    def reset_stats(self):
        _check(lib.tpc_ctx_reset_stats(self._h))

    @staticmethod
    def batch_args(evs, outs=None):
        """The arguments of tpc_track_batch for the device events `evs`:
        (events, E, tracks, outs, sizes), with outputs allocated here unless
        `outs` holds them (one dict per event).  Built once, they serve
        repeated track_batch_raw calls; sizes[i] receives event i's counts."""
        import torch
        E = len(evs)
        if outs is None:
            outs = []
            for ev in evs:
                n = ev.n_clusters
                dev = ev.y.device
                ct = max(16, n // 30 + 1)
                outs.append(dict(
                    track_par=torch.empty((ct, 8), dtype=torch.float32, device=dev),
                    track_meta=torch.empty((ct, 4), dtype=torch.int32, device=dev),
                    track_cluster=torch.empty(max(16, n), dtype=torch.int32, device=dev),
                    cluster_track=torch.empty(max(n, 1), dtype=torch.int32, device=dev)))
        sizes = [(C.c_int32(0), C.c_int32(0)) for _ in range(E)]
        trs = (Tracks * E)(*[Tracks(int(o["track_par"].shape[0]), int(o["track_cluster"].shape[0]),
                                    C.pointer(a), C.pointer(b), o["track_par"].data_ptr(),
                                    o["track_meta"].data_ptr(), o["track_cluster"].data_ptr(),
                                    o["cluster_track"].data_ptr())
                             for o, (a, b) in zip(outs, sizes)])
        es = (Event * E)(*[ev.cstruct() for ev in evs])
        return es, E, trs, outs, sizes

    def track_batch(self, evs, geo: Geometry, bz: float, params: Params = None, outs=None,
                    stream=None):
        """Track several device events in one launch sequence.  Returns one
        dict per event, like track_event.  `outs` may hold preallocated
        outputs (one dict per event)."""
        es, E, trs, outs, sizes = self.batch_args(evs, outs)
        rc = lib.tpc_track_batch(self._h, es, E, C.byref(geo), float(bz),
                                 C.byref(params or default_params()), trs, _stream_handle(stream))
        _check(rc)
        res = []
        for ev, o, (a, b) in zip(evs, outs, sizes):
            res.append(dict(n_tracks=a.value, n_track_clusters=b.value,
                            track_par=o["track_par"][:a.value], track_meta=o["track_meta"][:a.value],
                            track_cluster=o["track_cluster"][:b.value],
                            cluster_track=o["cluster_track"][:ev.n_clusters]))
        return res

    def track_batch_raw(self, es, E, geo, bz, params, trs, stream_handle) -> int:
        """Direct call on prebuilt ctypes arrays (no allocation), for timing loops."""
        return lib.tpc_track_batch(self._h, es, E, C.byref(geo), float(bz), C.byref(params), trs,
                                   stream_handle)

    def track_event_raw(self, e: Event, geo: Geometry, bz: float, params: Params, tr: Tracks,
                        stream_handle) -> int:
        """Direct call on prebuilt structs (no allocation), for timing loops."""
        return lib.tpc_track_event(self._h, C.byref(e), C.byref(geo), float(bz),
                                   C.byref(params), C.byref(tr), stream_handle)

    def track_event_noalloc_raw(self, e: Event, geo: Geometry, bz: float, params: Params,
                                tr: Tracks, stream_handle) -> int:
        """tpc_track_event_noalloc on prebuilt structs: the caller's outputs,
        the library's static scratch; nothing is allocated."""
        return lib.tpc_track_event_noalloc(self._h, C.byref(e), C.byref(geo), float(bz),
                                           C.byref(params), C.byref(tr), stream_handle)

    def track_event_global_raw(self, e: Event, geo: Geometry, bz: float, params: Params,
                               tr: Tracks, pro: Prolongations, stream_handle) -> int:
        """tpc_track_event_global on prebuilt structs (no allocation)."""
        return lib.tpc_track_event_global(self._h, C.byref(e), C.byref(geo), float(bz),
                                          C.byref(params), C.byref(tr), C.byref(pro),
                                          stream_handle)

    def track_event_merged_raw(self, e: Event, geo: Geometry, bz: float, params: Params,
                               merge_chi2: float, tr: Tracks, pro, mg: Merged,
                               stream_handle) -> int:
        """tpc_track_event_merged on prebuilt structs (pro may be None)."""
        return lib.tpc_track_event_merged(self._h, C.byref(e), C.byref(geo), float(bz),
                                          C.byref(params), float(merge_chi2), C.byref(tr),
                                          C.byref(pro) if pro is not None else None,
                                          C.byref(mg), stream_handle)

    def links(self, ev: DeviceEvent, geo: Geometry, params: Params = None, stream=None):
        import torch
        n = max(ev.n_clusters, 1)
        bufs = [torch.empty(n, dtype=torch.int32, device=ev.y.device) for _ in range(4)]
        e = ev.cstruct()
        _check(lib.tpc_debug_links(self._h, C.byref(e), C.byref(geo),
                                   C.byref(params or default_params()),
                                   *[b.data_ptr() for b in bufs], _stream_handle(stream)))
        return [b[:ev.n_clusters] for b in bufs]

    def tracklets(self, ev: DeviceEvent, geo: Geometry, bz: float, params: Params = None,
                  cap: int = None, stream=None):
        import torch
        dev = ev.y.device
        cap = cap if cap is not None else max(64, ev.n_clusters // 8)
        nr = geo.n_rows
        i32 = dict(dtype=torch.int32, device=dev)
        b = dict(seeds=torch.empty(cap, **i32), hits=torch.empty((cap, nr), **i32),
                 row_lo=torch.empty(cap, **i32), row_hi=torch.empty(cap, **i32),
                 n=torch.empty(cap, **i32), ndf=torch.empty(cap, **i32),
                 chi2=torch.empty(cap, dtype=torch.float32, device=dev),
                 par=torch.empty((cap, 6), dtype=torch.float32, device=dev))
        cnt = C.c_int32(0)
        e = ev.cstruct()
        _check(lib.tpc_debug_tracklets(
            self._h, C.byref(e), C.byref(geo), float(bz), C.byref(params or default_params()),
            int(cap), C.byref(cnt),
            *[b[k].data_ptr() for k in ("seeds", "hits", "row_lo", "row_hi", "n", "ndf", "chi2",
                                        "par")], _stream_handle(stream)))
        k = cnt.value
        return {name: v[:k] for name, v in b.items()}


def kernel_names():
    return [lib.tpc_kernel_name(i).decode() for i in range(lib.tpc_kernel_count())]


def to_numpy(res: dict) -> dict:
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in res.items()}


class HostEvent:
    """An event in host memory (numpy), as a server takes it."""

    def __init__(self, y, z, row_offsets, sector_id):
        self.y = np.ascontiguousarray(y, np.float32)
        self.z = np.ascontiguousarray(z, np.float32)
        self.row_offsets = np.ascontiguousarray(row_offsets, np.int32)
        self.sector_id = np.ascontiguousarray(sector_id, np.int32)
        self.c = Event(int(self.sector_id.shape[0]), self.sector_id.ctypes.data,
                       int(self.y.shape[0]), self.y.ctypes.data, self.z.ctypes.data,
                       self.row_offsets.ctypes.data)

    @property
    def n_clusters(self):
        return int(self.y.shape[0])


class Server:
    """Continuous-batching server (tpc_server_*)."""

    def __init__(self, geo: Geometry, bz: float, params: Params = None, **cfg):
        c = ServerConfig()
        lib.tpc_server_config_default(C.byref(c))
        for k, v in cfg.items():
            setattr(c, k, v)
        h = C.c_void_p()
        rc = lib.tpc_server_create(C.byref(c), C.byref(geo), float(bz),
                                   C.byref(params or default_params()), C.byref(h))
        if rc:
            raise TpcError(rc, lib.tpc_server_last_error().decode())
        self._h, self.cfg, self._geo = h, c, geo
        self._buf = (ServerDone * 1024)()

    def submit(self, ev: HostEvent, tag: int) -> int:
        """TPC_OK, or TPC_ERR_BUSY when the event is not admitted now."""
        rc = lib.tpc_server_submit(self._h, C.byref(ev.c), int(tag))
        if rc not in (TPC_OK, TPC_ERR_BUSY):
            raise TpcError(rc, lib.tpc_server_last_error().decode())
        return rc

    def poll(self, timeout_ms: int = 0):
        n = C.c_int(0)
        _rc = lib.tpc_server_poll(self._h, self._buf, 1024, C.byref(n), int(timeout_ms))
        return [dict(tag=d.tag, status=d.status, n_tracks=d.n_tracks,
                     n_track_clusters=d.n_track_clusters, t_submit=d.t_submit, t_done=d.t_done)
                for d in self._buf[:n.value]]

    def fetch(self, done: dict, n_clusters: int):
        nt, nc = done["n_tracks"], done["n_track_clusters"]
        par = np.empty((nt, 8), np.float32)
        meta = np.empty((nt, 4), np.int32)
        tcl = np.empty(nc, np.int32)
        ctr = np.empty(max(n_clusters, 1), np.int32)
        rc = lib.tpc_server_fetch(self._h, int(done["tag"]), par.ctypes.data, meta.ctypes.data,
                                  tcl.ctypes.data, ctr.ctypes.data)
        if rc:
            raise TpcError(rc, lib.tpc_server_last_error().decode())
        return dict(n_tracks=nt, n_track_clusters=nc, track_par=par, track_meta=meta,
                    track_cluster=tcl, cluster_track=ctr[:n_clusters])

    def stats(self):
        b, e, r = C.c_int64(0), C.c_int64(0), C.c_size_t(0)
        _check(lib.tpc_server_stats(self._h, C.byref(b), C.byref(e), C.byref(r)))
        return dict(batches=b.value, events=e.value, resident_bytes=r.value)

    @staticmethod
    def now() -> float:
        return lib.tpc_server_now()

    def close(self):
        if getattr(self, "_h", None):
            lib.tpc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
