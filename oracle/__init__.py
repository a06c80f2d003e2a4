"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library: it loads its own
shared object, built from `tpc_oracle.c` with gcc, and takes plain numpy
arrays (host memory).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tpc_oracle.c")
LIB = os.path.join(HERE, "libtpcoracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no HIP) into oracle/libtpcoracle.so."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", "-o", tmp,
                               SRC, "-lm", "-lpthread"])
        os.replace(tmp, LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [("sigma_y", C.c_double), ("sigma_z", C.c_double),
                ("nf_win_y", C.c_double), ("nf_win_z", C.c_double),
                ("nf_chi2_max", C.c_double), ("min_seed_len", C.c_int32),
                ("seed_window", C.c_int32),
                ("chi2_gate", C.c_double), ("max_miss", C.c_int32),
                ("max_sinphi", C.c_double), ("alpha", C.c_double), ("beta", C.c_double),
                ("min_clusters", C.c_int32), ("min_pt", C.c_double),
                ("prior_sinphi", C.c_double), ("prior_tanl", C.c_double),
                ("prior_qpt", C.c_double)]


class Geometry(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("row_x", C.POINTER(C.c_float)),
                ("tan_half_angle", C.c_float), ("z_max", C.c_float)]


class EventS(C.Structure):
    _fields_ = [("n_sectors", C.c_int32), ("sector_id", C.POINTER(C.c_int32)),
                ("n_clusters", C.c_int64), ("y", C.POINTER(C.c_float)),
                ("z", C.POINTER(C.c_float)), ("row_offsets", C.POINTER(C.c_int32))]


class Tracks(C.Structure):
    _fields_ = [("cap_tracks", C.c_int32), ("cap_track_clusters", C.c_int32),
                ("n_tracks", C.c_int32), ("n_track_clusters", C.c_int32),
                ("track_par", C.POINTER(C.c_double)), ("track_meta", C.POINTER(C.c_int32)),
                ("track_cluster", C.POINTER(C.c_int32)), ("cluster_track", C.POINTER(C.c_int32))]


class Prolongations(C.Structure):
    _fields_ = [("cap", C.c_int32), ("cap_clusters", C.c_int32), ("n", C.c_int32),
                ("n_clusters", C.c_int32), ("par", C.POINTER(C.c_double)),
                ("meta", C.POINTER(C.c_int32)), ("cluster", C.POINTER(C.c_int32))]


class Merged(C.Structure):
    _fields_ = [("cap", C.c_int32), ("cap_clusters", C.c_int32), ("n", C.c_int32),
                ("n_clusters", C.c_int32), ("par", C.POINTER(C.c_double)),
                ("meta", C.POINTER(C.c_int32)), ("cluster", C.POINTER(C.c_int32)),
                ("track_merged", C.POINTER(C.c_int32))]


class Tracklets(C.Structure):
    _fields_ = [("hits", C.POINTER(C.c_int32)), ("row_lo", C.POINTER(C.c_int32)),
                ("row_hi", C.POINTER(C.c_int32)), ("n", C.POINTER(C.c_int32)),
                ("chi2", C.POINTER(C.c_double)), ("ndf", C.POINTER(C.c_int32)),
                ("par", C.POINTER(C.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.POINTER
        L.orc_params_default.argtypes = [P(Params)]
        L.orc_track_event.argtypes = [P(EventS), P(Geometry), C.c_double, P(Params), P(Tracks),
                                      C.c_int]
        L.orc_track_event_global.argtypes = [P(EventS), P(Geometry), C.c_double, P(Params),
                                             P(Tracks), P(Prolongations), C.c_int]
        L.orc_track_event_merged.argtypes = [P(EventS), P(Geometry), C.c_double, P(Params),
                                             C.c_double, P(Tracks), P(Prolongations), P(Merged),
                                             C.c_int]
        L.orc_refit.argtypes = [P(EventS), P(Geometry), C.c_double, P(Params), C.c_int32,
                                P(C.c_int32), P(C.c_int32), P(C.c_double), P(C.c_int32)]
        L.orc_rotate.argtypes = [C.c_double, P(C.c_double), P(C.c_double), C.c_double,
                                 C.c_double, P(C.c_double), P(C.c_double), P(C.c_double)]
        L.orc_neighbours.argtypes = [P(EventS), P(Geometry), P(Params), P(C.c_int32),
                                     P(C.c_int32)]
        L.orc_nf_chi2.argtypes = [P(EventS), P(Geometry), P(Params), C.c_int32, C.c_int32,
                                  C.c_int32]
        L.orc_nf_chi2.restype = C.c_double
        L.orc_evolve.argtypes = [C.c_int64, P(C.c_int32), P(C.c_int32), P(C.c_int32),
                                 P(C.c_int32)]
        L.orc_seeds.argtypes = [P(EventS), P(Geometry), P(Params), P(C.c_int32), P(C.c_int32),
                                P(C.c_int32), C.c_int64]
        L.orc_seeds.restype = C.c_int64
        L.orc_construct.argtypes = [P(EventS), P(Geometry), C.c_double, P(Params), P(C.c_int32),
                                    C.c_int64, P(C.c_int32), P(Tracklets)]
        L.orc_select.argtypes = [P(EventS), P(Geometry), C.c_double, P(Params), C.c_int64,
                                 P(C.c_int32), P(Tracklets), P(C.c_double), P(C.c_int32),
                                 P(C.c_int32)]
        L.orc_propagate.argtypes = [C.c_double, P(C.c_double), P(C.c_double), C.c_double,
                                    C.c_double, C.c_double, P(C.c_double)]
        L.orc_fit_hits.argtypes = [C.c_int32, P(C.c_double), P(C.c_double), P(C.c_double),
                                   C.c_double, P(Params), P(C.c_double), P(C.c_double),
                                   P(C.c_double), P(C.c_int32)]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def default_params(**over) -> Params:
    p = Params()
    lib().orc_params_default(C.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def params_dict(p: Params) -> dict:
    return {k: getattr(p, k) for k, _ in Params._fields_}


class _Ctx:
    """Keeps the numpy arrays behind the C structs alive."""

    def __init__(self, y, z, row_offsets, sector_id, row_x, tan_half, z_max):
        self.y = np.ascontiguousarray(y, np.float32)
        self.z = np.ascontiguousarray(z, np.float32)
        self.ro = np.ascontiguousarray(row_offsets, np.int32)
        self.sid = np.ascontiguousarray(sector_id, np.int32)
        self.rx = np.ascontiguousarray(row_x, np.float32)
        self.ev = EventS(int(self.sid.shape[0]), _p(self.sid, C.c_int32), int(self.y.shape[0]),
                         _p(self.y, C.c_float), _p(self.z, C.c_float), _p(self.ro, C.c_int32))
        self.geo = Geometry(int(self.rx.shape[0]), _p(self.rx, C.c_float), float(tan_half),
                            float(z_max))


def _ctx(ev, geo):
    row_x, tan_half, z_max = geo
    return _Ctx(ev["y"], ev["z"], ev["row_offsets"], ev["sector_id"], row_x, tan_half, z_max)


def track_event(ev: dict, geo, bz: float, params: Params | None = None, n_threads: int = 1):
    """Run the whole method.  ev: dict with y, z, row_offsets, sector_id;
    geo: (row_x float32[n_rows], tan_half_angle, z_max)."""
    cx = _ctx(ev, geo)
    prm = params or default_params()
    n = int(cx.y.shape[0])
    cap_t, cap_c = max(1, n // 8), max(1, n)
    for _ in range(2):
        par = np.zeros((cap_t, 8), np.float64)
        meta = np.zeros((cap_t, 4), np.int32)
        tcl = np.zeros(cap_c, np.int32)
        ctr = np.full(max(n, 1), -1, np.int32)
        out = Tracks(cap_t, cap_c, 0, 0, _p(par, C.c_double), _p(meta, C.c_int32),
                     _p(tcl, C.c_int32), _p(ctr, C.c_int32))
        rc = lib().orc_track_event(C.byref(cx.ev), C.byref(cx.geo), float(bz), C.byref(prm),
                                   C.byref(out), int(n_threads))
        if rc == 1:
            cap_t, cap_c = out.n_tracks, out.n_track_clusters
            continue
        if rc != 0:
            raise RuntimeError(f"orc_track_event failed: {rc}")
        nt, nc = out.n_tracks, out.n_track_clusters
        return dict(n_tracks=nt, n_track_clusters=nc, track_par=par[:nt].copy(),
                    track_meta=meta[:nt].copy(), track_cluster=tcl[:nc].copy(),
                    cluster_track=ctr[:n].copy())
    raise RuntimeError("capacity retry failed")


def neighbours(ev, geo, params=None):
    cx = _ctx(ev, geo)
    n = int(cx.y.shape[0])
    up = np.empty(max(n, 1), np.int32)
    dn = np.empty(max(n, 1), np.int32)
    rc = lib().orc_neighbours(C.byref(cx.ev), C.byref(cx.geo), C.byref(params or default_params()),
                              _p(up, C.c_int32), _p(dn, C.c_int32))
    if rc:
        raise RuntimeError("orc_neighbours failed")
    return up[:n], dn[:n]


def nf_chi2(ev, geo, d, c, u, params=None):
    cx = _ctx(ev, geo)
    return lib().orc_nf_chi2(C.byref(cx.ev), C.byref(cx.geo), C.byref(params or default_params()),
                             int(d), int(c), int(u))


def evolve(up, dn):
    up = np.ascontiguousarray(up, np.int32)
    dn = np.ascontiguousarray(dn, np.int32)
    n = up.shape[0]
    up2 = np.empty(max(n, 1), np.int32)
    dn2 = np.empty(max(n, 1), np.int32)
    if lib().orc_evolve(n, _p(up, C.c_int32), _p(dn, C.c_int32), _p(up2, C.c_int32),
                        _p(dn2, C.c_int32)):
        raise RuntimeError("orc_evolve failed")
    return up2[:n], dn2[:n]


def seeds(ev, geo, up2, dn2, params=None):
    cx = _ctx(ev, geo)
    up2 = np.ascontiguousarray(up2, np.int32)
    dn2 = np.ascontiguousarray(dn2, np.int32)
    prm = params or default_params()
    n = lib().orc_seeds(C.byref(cx.ev), C.byref(cx.geo), C.byref(prm), _p(up2, C.c_int32),
                        _p(dn2, C.c_int32), None, 0)
    if n < 0:
        raise RuntimeError("orc_seeds failed")
    out = np.empty(max(n, 1), np.int32)
    m = lib().orc_seeds(C.byref(cx.ev), C.byref(cx.geo), C.byref(prm), _p(up2, C.c_int32),
                        _p(dn2, C.c_int32), _p(out, C.c_int32), n)
    if m != n:
        raise RuntimeError("orc_seeds failed")
    return out[:n]


def _alloc_tracklets(n_tl, n_rows):
    a = dict(hits=np.full((max(n_tl, 1), n_rows), -1, np.int32),
             row_lo=np.zeros(max(n_tl, 1), np.int32), row_hi=np.zeros(max(n_tl, 1), np.int32),
             n=np.zeros(max(n_tl, 1), np.int32), chi2=np.zeros(max(n_tl, 1), np.float64),
             ndf=np.zeros(max(n_tl, 1), np.int32), par=np.zeros((max(n_tl, 1), 6), np.float64))
    s = Tracklets(_p(a["hits"], C.c_int32), _p(a["row_lo"], C.c_int32), _p(a["row_hi"], C.c_int32),
                  _p(a["n"], C.c_int32), _p(a["chi2"], C.c_double), _p(a["ndf"], C.c_int32),
                  _p(a["par"], C.c_double))
    return a, s


def construct(ev, geo, bz, up2, seeds_arr, params=None):
    cx = _ctx(ev, geo)
    up2 = np.ascontiguousarray(up2, np.int32)
    sd = np.ascontiguousarray(seeds_arr, np.int32)
    n_tl = int(sd.shape[0])
    a, s = _alloc_tracklets(n_tl, cx.geo.n_rows)
    rc = lib().orc_construct(C.byref(cx.ev), C.byref(cx.geo), float(bz),
                             C.byref(params or default_params()), _p(up2, C.c_int32), n_tl,
                             _p(sd, C.c_int32), C.byref(s))
    if rc:
        raise RuntimeError("orc_construct failed")
    return {k: v[:n_tl] for k, v in a.items()}


def track_event_global(ev: dict, geo, bz: float, params: Params | None = None,
                       n_threads: int = 1):
    """track_event, then the global-tracking prolongation of the tracks.
    Returns (tracks, prolongations): prolongations has n, par [n][8] (x, y,
    z, sinphi, tanl, qpt at the last collected cluster, chi2, ndf), meta
    [n][5] (track index, end, sector_id entered, n_clusters, first) and
    cluster."""
    cx = _ctx(ev, geo)
    prm = params or default_params()
    n = int(cx.y.shape[0])
    cap_t, cap_c = max(1, n // 8), max(1, n)
    cap_p, cap_pc = 2 * cap_t + 1, max(1, n)
    for _ in range(3):
        par = np.zeros((cap_t, 8), np.float64)
        meta = np.zeros((cap_t, 4), np.int32)
        tcl = np.zeros(cap_c, np.int32)
        ctr = np.full(max(n, 1), -1, np.int32)
        ppar = np.zeros((cap_p, 8), np.float64)
        pmeta = np.zeros((cap_p, 5), np.int32)
        pcl = np.zeros(cap_pc, np.int32)
        out = Tracks(cap_t, cap_c, 0, 0, _p(par, C.c_double), _p(meta, C.c_int32),
                     _p(tcl, C.c_int32), _p(ctr, C.c_int32))
        pro = Prolongations(cap_p, cap_pc, 0, 0, _p(ppar, C.c_double), _p(pmeta, C.c_int32),
                            _p(pcl, C.c_int32))
        rc = lib().orc_track_event_global(C.byref(cx.ev), C.byref(cx.geo), float(bz),
                                          C.byref(prm), C.byref(out), C.byref(pro),
                                          int(n_threads))
        if rc == 1:
            cap_t, cap_c = max(cap_t, out.n_tracks), max(cap_c, out.n_track_clusters)
            cap_p, cap_pc = max(cap_p, pro.n), max(cap_pc, pro.n_clusters)
            continue
        if rc != 0:
            raise RuntimeError(f"orc_track_event_global failed: {rc}")
        nt, nc, npr, npc = out.n_tracks, out.n_track_clusters, pro.n, pro.n_clusters
        tracks = dict(n_tracks=nt, n_track_clusters=nc, track_par=par[:nt].copy(),
                      track_meta=meta[:nt].copy(), track_cluster=tcl[:nc].copy(),
                      cluster_track=ctr[:n].copy())
        prol = dict(n=npr, n_clusters=npc, par=ppar[:npr].copy(), meta=pmeta[:npr].copy(),
                    cluster=pcl[:npc].copy())
        return tracks, prol
    raise RuntimeError("capacity retry failed")


MERGE_CHI2 = 25.0   # joins: chi^2(5) <= 25, a 1e-4 tail for the same particle


def track_event_merged(ev: dict, geo, bz: float, params: Params | None = None,
                       merge_chi2: float = MERGE_CHI2, use_global: bool = True,
                       n_threads: int = 1):
    """track_event (and, with use_global, the prolongations), then the track
    merger with refit.  Returns (tracks, prolongations or None, merged):
    merged has n, par [n][8] (x, y, z, sinphi, tanl, qpt at the innermost
    fitted cluster in the frame of sector meta[:, 0], chi2, ndf; ndf 0 =
    refit failed), meta [n][5] (frame sector_id, tracks joined, n_clusters,
    first, first track), cluster (path order), track_merged [n_tracks]."""
    cx = _ctx(ev, geo)
    prm = params or default_params()
    n = int(cx.y.shape[0])
    cap_t, cap_c = max(1, n // 8), max(1, n)
    cap_p, cap_pc = 2 * cap_t + 1, max(1, n)
    cap_m, cap_mc = cap_t, max(1, n)
    for _ in range(3):
        par = np.zeros((cap_t, 8), np.float64)
        meta = np.zeros((cap_t, 4), np.int32)
        tcl = np.zeros(cap_c, np.int32)
        ctr = np.full(max(n, 1), -1, np.int32)
        ppar = np.zeros((cap_p, 8), np.float64)
        pmeta = np.zeros((cap_p, 5), np.int32)
        pcl = np.zeros(cap_pc, np.int32)
        mpar = np.zeros((cap_m, 8), np.float64)
        mmeta = np.zeros((cap_m, 5), np.int32)
        mcl = np.zeros(cap_mc, np.int32)
        tm = np.full(cap_t, -1, np.int32)
        out = Tracks(cap_t, cap_c, 0, 0, _p(par, C.c_double), _p(meta, C.c_int32),
                     _p(tcl, C.c_int32), _p(ctr, C.c_int32))
        pro = Prolongations(cap_p, cap_pc, 0, 0, _p(ppar, C.c_double), _p(pmeta, C.c_int32),
                            _p(pcl, C.c_int32))
        mrg = Merged(cap_m, cap_mc, 0, 0, _p(mpar, C.c_double), _p(mmeta, C.c_int32),
                     _p(mcl, C.c_int32), _p(tm, C.c_int32))
        rc = lib().orc_track_event_merged(C.byref(cx.ev), C.byref(cx.geo), float(bz),
                                          C.byref(prm), float(merge_chi2), C.byref(out),
                                          C.byref(pro) if use_global else None, C.byref(mrg),
                                          int(n_threads))
        if rc == 1:
            cap_t, cap_c = max(cap_t, out.n_tracks), max(cap_c, out.n_track_clusters)
            cap_p, cap_pc = max(cap_p, pro.n), max(cap_pc, pro.n_clusters)
            cap_m, cap_mc = max(cap_m, mrg.n, out.n_tracks), max(cap_mc, mrg.n_clusters)
            continue
        if rc != 0:
            raise RuntimeError(f"orc_track_event_merged failed: {rc}")
        nt, nc = out.n_tracks, out.n_track_clusters
        tracks = dict(n_tracks=nt, n_track_clusters=nc, track_par=par[:nt].copy(),
                      track_meta=meta[:nt].copy(), track_cluster=tcl[:nc].copy(),
                      cluster_track=ctr[:n].copy())
        prol = dict(n=pro.n, n_clusters=pro.n_clusters, par=ppar[:pro.n].copy(),
                    meta=pmeta[:pro.n].copy(), cluster=pcl[:pro.n_clusters].copy()) \
            if use_global else None
        merged = dict(n=mrg.n, n_clusters=mrg.n_clusters, par=mpar[:mrg.n].copy(),
                      meta=mmeta[:mrg.n].copy(), cluster=mcl[:mrg.n_clusters].copy(),
                      track_merged=tm[:nt].copy())
        return tracks, prol, merged
    raise RuntimeError("capacity retry failed")


def refit(ev: dict, geo, bz: float, lists, params: Params | None = None):
    """The merger's refit of cluster lists (each in path order).  Returns
    (par [n][8], frame sector_id [n], -1 = failed)."""
    cx = _ctx(ev, geo)
    lens = [len(l) for l in lists]
    off = np.zeros(len(lists) + 1, np.int32)
    np.cumsum(lens, out=off[1:])
    cl = np.ascontiguousarray(np.concatenate([np.asarray(l, np.int32) for l in lists])
                              if lists else np.zeros(1, np.int32), np.int32)
    par = np.zeros((max(1, len(lists)), 8), np.float64)
    fr = np.zeros(max(1, len(lists)), np.int32)
    rc = lib().orc_refit(C.byref(cx.ev), C.byref(cx.geo), float(bz),
                         C.byref(params or default_params()), len(lists), _p(off, C.c_int32),
                         _p(cl, C.c_int32), _p(par, C.c_double), _p(fr, C.c_int32))
    if rc:
        raise RuntimeError("orc_refit failed")
    return par[:len(lists)], fr[:len(lists)]


def rotate(x: float, state, cov, d: float, bz: float):
    """Rotation of a state (5) and covariance (5x5) at x into a frame turned by
    d radians: returns (x', state', cov'), or None if the direction does not
    point along the new x axis."""
    st = np.ascontiguousarray(state, np.float64)
    cv = np.ascontiguousarray(cov if cov is not None else np.zeros((5, 5)), np.float64)
    xo = C.c_double(0.0)
    so = np.zeros(5, np.float64)
    co = np.zeros((5, 5), np.float64)
    rc = lib().orc_rotate(float(x), _p(st, C.c_double), _p(cv, C.c_double), float(d), float(bz),
                          C.byref(xo), _p(so, C.c_double), _p(co, C.c_double))
    if rc == 1:
        return None
    if rc:
        raise RuntimeError("orc_rotate failed")
    return xo.value, so, co


def select(ev, geo, bz, ids, tl: dict, params=None, weights=None):
    """tl: dict with hits, row_lo, row_hi, n, chi2, ndf, par (float64 [n,6]).
    weights: optional per-tracklet weights used instead of the computed ones."""
    cx = _ctx(ev, geo)
    ids = np.ascontiguousarray(ids, np.int32)
    n_tl = int(ids.shape[0])
    a = {k: np.ascontiguousarray(tl[k], dt) for k, dt in
         (("hits", np.int32), ("row_lo", np.int32), ("row_hi", np.int32), ("n", np.int32),
          ("chi2", np.float64), ("ndf", np.int32), ("par", np.float64))}
    s = Tracklets(_p(a["hits"], C.c_int32), _p(a["row_lo"], C.c_int32), _p(a["row_hi"], C.c_int32),
                  _p(a["n"], C.c_int32), _p(a["chi2"], C.c_double), _p(a["ndf"], C.c_int32),
                  _p(a["par"], C.c_double))
    n = int(cx.y.shape[0])
    owner = np.empty(max(n, 1), np.int32)
    keep = np.empty(max(n_tl, 1), np.int32)
    w = None if weights is None else np.ascontiguousarray(weights, np.float64)
    rc = lib().orc_select(C.byref(cx.ev), C.byref(cx.geo), float(bz),
                          C.byref(params or default_params()), n_tl, _p(ids, C.c_int32),
                          C.byref(s), None if w is None else _p(w, C.c_double),
                          _p(owner, C.c_int32), _p(keep, C.c_int32))
    if rc:
        raise RuntimeError("orc_select failed")
    return owner[:n], keep[:n_tl]


def propagate(x1, state, cov, x2, bz, max_sinphi=0.999):
    st = np.array(state, np.float64)
    cv = np.array(cov, np.float64).reshape(5, 5).copy()
    jac = np.zeros((5, 5), np.float64)
    rc = lib().orc_propagate(float(x1), _p(st, C.c_double), _p(cv, C.c_double), float(x2),
                             float(bz), float(max_sinphi), _p(jac, C.c_double))
    if rc:
        return None
    return st, cv, jac


def fit_hits(x, y, z, bz, params=None):
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    z = np.ascontiguousarray(z, np.float64)
    st = np.zeros(5)
    cov = np.zeros((5, 5))
    chi2 = C.c_double(0.0)
    ndf = C.c_int32(0)
    rc = lib().orc_fit_hits(int(x.shape[0]), _p(x, C.c_double), _p(y, C.c_double),
                            _p(z, C.c_double), float(bz), C.byref(params or default_params()),
                            _p(st, C.c_double), _p(cov, C.c_double), C.byref(chi2), C.byref(ndf))
    if rc:
        return None
    return st, cov, chi2.value, ndf.value
