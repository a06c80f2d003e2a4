#!/usr/bin/env python3
"""Throughput of the TPC sector tracker on one MI355X.

Workload: a central Pb-Pb-like event (36 sectors x 159 pad rows, 8000 primary
helix tracks, 5% noise clusters, about 1.33M clusters), tracked by the plain
per-event path (tpc_track_event).  One step = one whole event through every
stage: grid build, neighbours finder, evolution, seeds, tracklet
construction, assignment, selection, output.  Inputs are resident in HBM
before the timed region starts; outputs are preallocated.

Prints one JSON line.  Everything else goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "events/s & clusters/s at ≥99.99% track match; p50/p99 event latency"
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3

# Algorithmic FP32 operations of the constructor, counted from its arithmetic
# (a fused multiply-add counts as two): one exact helix step with the
# covariance transport, one Kalman update, one candidate tested against the
# chi^2 gate (plus the gate set-up, charged once per step).
FLOP_STEP = 174 + 20
FLOP_UPDATE = 129
FLOP_CAND = 11
# Algorithmic HBM bytes per cluster of the streaming kernels (each array read
# or written once per use): k_grid reads y, z twice and writes the 16-byte grid
# record, the bin start and cluster_track; k_nf reads the cluster's record, two
# neighbour rows (records and bins) and writes up, dn; k_evo reads the links
# and the partner's links and writes the reciprocal links and the start flag.
BYTES_PER_CLUSTER = {"k_grid": 16 + 16 + 4 + 4, "k_nf": 16 + 32 + 8 + 8, "k_evo": 8 + 8 + 8 + 1}


def path_bytes(N, tracklets, steps, cands, n_tracks, n_track_clusters):
    """Algorithmic HBM bytes of one event through the whole path (the staged
    accounting: every array touched once per use, row staging counted once per
    row and neighbour, hits of a tracklet row 12 B written and read back)."""
    b = sum(BYTES_PER_CLUSTER.values()) * N
    b += N + 8 * tracklets                              # seed flags, seeds
    b += 16 * cands + 12 * steps + 12 * steps           # candidates; hits written, read back
    b += 8 * N + 2 * 4 * steps                          # owner keys; hits read twice by k_own
    b += n_track_clusters * (4 + 8 + 8) + 48 * n_tracks  # output
    return b


# The method's algorithmic HBM bytes per cluster, staged (every stage reads
# its inputs and writes its outputs once): grid build 28, neighbours finder
# with evolution 16, seeds 8, tracklet construction 50-60, weights and
# assignment 16-32, selection and output 24.
STAGED_BYTES_PER_CLUSTER = (160, 190)


def staged_hbm(clusters_per_s):
    """The whole path against HBM under the staged algorithmic model."""
    lo, hi = STAGED_BYTES_PER_CLUSTER
    return dict(model="staged algorithmic bytes, 160-190 B per cluster (grid 28, links 16, "
                      "seeds 8, construction 50-60, assignment 16-32, selection and output 24)",
                bytes_per_cluster=[lo, hi], unit="GB/s", peak=PEAK_HBM_GBS,
                achieved=round(lo * clusters_per_s / 1e9, 2),
                achieved_high=round(hi * clusters_per_s / 1e9, 2),
                frac=round(lo * clusters_per_s / 1e9 / PEAK_HBM_GBS, 6),
                frac_high=round(hi * clusters_per_s / 1e9 / PEAK_HBM_GBS, 6))


def roofline_of(st, n_clusters_per_launch):
    """Roofline of the dominant kernel of a timed probe (stats with every
    kernel timed): the constructor against the FP32 vector peak (algorithmic
    FLOP from the device's work counters), a streaming kernel against HBM."""
    per = {k: st["kernel_ms"][k] / st["kernel_launches"][k] for k in st["kernel_ms"]
           if st["kernel_launches"][k] > 0}
    dominant = max(per, key=per.get)
    dom_ms = per[dominant]
    launches = max(1, st["kernel_launches"][dominant])
    if dominant == "k_construct":
        flops = (st["steps"] * FLOP_STEP + st["updates"] * FLOP_UPDATE +
                 st["candidates"] * FLOP_CAND) / launches
        achieved = flops / (dom_ms * 1e-3) / 1e12
        return dict(bound="alu", achieved=round(achieved, 4), peak=PEAK_FP32_TFLOPS,
                    unit="TFLOP/s", frac=round(achieved / PEAK_FP32_TFLOPS, 6),
                    kernel=dominant, kernel_ms=round(dom_ms, 5),
                    algorithmic_per_launch=f"{flops:.4g} FLOP"), per
    nbytes = BYTES_PER_CLUSTER.get(dominant, 16) * n_clusters_per_launch
    achieved = nbytes / (dom_ms * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(achieved, 2), peak=PEAK_HBM_GBS, unit="GB/s",
                frac=round(achieved / PEAK_HBM_GBS, 6), kernel=dominant,
                kernel_ms=round(dom_ms, 5), algorithmic_per_launch=f"{nbytes} B"), per


def timed_probe(tr, fn, reps=3):
    """Every kernel timed with HIP events over `reps` eager calls."""
    tr.set_timing(None)
    tr.reset_stats()
    for _ in range(reps):
        fn()
    st = tr.stats()
    tr.set_timing([])
    tr.reset_stats()
    return st


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_src_sha():
    """Hash of the device sources (kernels and track model): counter figures
    taken from other sources are not reported."""
    h = hashlib.sha256()
    for f in ("tpc_kernels.hip", "tpc_model.h"):
        h.update(open(os.path.join(ROOT, "paper_1712_09407_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def cpu_info():
    """The host CPU as /proc/cpuinfo describes it (first processor), with the
    logical CPU count and this process's affinity."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if not line.strip():
                break
            k, _, v = line.partition(":")
            info[k.strip()] = v.strip()
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return dict(cpu_model=info.get("model name", "unknown"),
                cpu_family=info.get("cpu family"), cpu_model_number=info.get("model"),
                stepping=info.get("stepping"), cpu_mhz=info.get("cpu MHz"),
                cache=info.get("cache size"), nproc=os.cpu_count(), affinity=aff)


def cpu_baseline(ev_host, geo_t, bz, gpu_res, n_clusters, seconds, params=None):
    """The FP64 oracle on this host's cores, on repeats of the same event."""
    import oracle
    from oracle import concordance
    try:
        cores = len(os.sched_getaffinity(0))      # every core this process may run on
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, cores)
    runs, t0 = 0, time.perf_counter()
    ref = None
    while True:
        ref = oracle.track_event(ev_host, geo_t, bz, params or oracle.default_params(),
                                 n_threads=cores)
        runs += 1
        el = time.perf_counter() - t0
        if el >= seconds or runs >= 200:
            break
    rep = concordance.compare(ref, gpu_res, n_clusters)
    t1 = time.perf_counter()
    oracle.track_event(ev_host, geo_t, bz, params or oracle.default_params(), n_threads=1)
    single = 1.0 / (time.perf_counter() - t1)
    base = dict(value=runs / el, unit="events/s", cores=cores, kind="oracle",
                sample=f"{runs} run(s) of the benchmark event ({n_clusters} clusters), "
                       f"{el:.1f} s wall, {cores} threads over sectors (every core of the "
                       f"process's affinity)",
                single_thread_value=round(single, 4), **cpu_info())
    conc = {k: rep[k] for k in ("cluster_concordance", "track_concordance", "cluster_concordance_ab",
                                "cluster_concordance_ba", "n_tracks_a", "n_tracks_b",
                                "par_compared", "par_fail", "par_max_rel", "par_other_seed")}
    conc["reference"] = "FP64 oracle"
    return base, conc


def _gen_event(args):
    from paper_1712_09407_amd import synth
    name, seed = args
    return synth.make_preset(name, seed)


def _gen_arrays(args):
    from paper_1712_09407_amd import synth
    name, seed = args
    e = synth.make_preset(name, seed) if name != "batch" else synth.batch_event(seed)
    return e.y, e.z, e.row_offsets, e.sector_id


def _pool_workers():
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


CENTRAL_SEEDS = list(range(2, 12))   # concordance over ten central events
ALPHA_SEEDS = [2, 3, 4]              # the alpha scan's central events
STRESS_SEEDS = [5000 + i for i in range(16)]


def raw_batch(tr, tpc, devs, geo, bz, prm):
    """A batch call on arguments marshalled once, with outputs allocated once
    (a caller that reuses its buffers, as the server does): the timed loops
    measure the library, not the Python binding's allocations.  Returns the
    call and the outputs."""
    import ctypes as C
    import torch
    es, E, trs, outs, sizes = tr.batch_args(devs)
    sh = C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def call():
        rc = tr.track_batch_raw(es, E, geo, bz, prm, trs, sh)
        if rc != 0:
            raise tpc.TpcError(rc, tpc.last_error())
    return call, outs, sizes


def pregenerate(args):
    """Every host event the benchmark needs, generated in worker processes
    before this process touches the GPU: a process that holds a GPU context
    must not fork.  Returns a dict of event lists."""
    import concurrent.futures as cf
    import multiprocessing as mp
    jobs = {"main": [("event", (args.event, args.seed))]}
    if args.extra:
        jobs["central"] = [("event", ("c2_central", s)) for s in CENTRAL_SEEDS]
        jobs["stress"] = [("arrays", ("c5_stress", s)) for s in STRESS_SEEDS]
    if args.batch_events > 0:
        jobs["batch"] = [("arrays", ("batch", 3000 + i)) for i in range(args.batch_events)]
    flat = [(k, i, kind, a) for k, v in jobs.items() for i, (kind, a) in enumerate(v)]
    # the main event is one of the central ones when it is a central seed
    reuse = args.extra and args.event == "c2_central" and args.seed in CENTRAL_SEEDS
    flat = [f for f in flat if not (reuse and f[0] == "main")]
    log(f"generating {len(flat)} host events with {_pool_workers()} processes")
    out = {k: [None] * len(v) for k, v in jobs.items()}
    with cf.ProcessPoolExecutor(_pool_workers(), mp_context=mp.get_context("fork")) as ex:
        futs = {ex.submit(_gen_event if kind == "event" else _gen_arrays, a): (k, i)
                for k, i, kind, a in flat}
        for f in cf.as_completed(futs):
            k, i = futs[f]
            out[k][i] = f.result()
    if reuse:
        out["main"] = [out["central"][CENTRAL_SEEDS.index(args.seed)]]
    return out


def oracle_params(tpc, gpu_params):
    """The oracle's constants: the GPU's FP32 values, widened."""
    import oracle
    vals = {}
    for k, t in oracle.Params._fields_:
        v = getattr(gpu_params, k)
        vals[k] = float(np.float32(v)) if isinstance(v, float) else v
    return oracle.default_params(**vals)


# Oracle work of the sections: each section stores what the oracle needs here
# and the cpu_baseline leg (the only code that runs the oracle) fills in the
# comparisons.
ORACLE_CHECKS = {}


def single_sector_section(tr, tpc, synth, geo, prm, steps, log_):
    """One sector, 200 tracks: the plain path on the smallest event (latency
    bound); the oracle's time and concordance come from the cpu_baseline leg."""
    import torch
    e = synth.make_preset("c1_sector", 1)
    dev = tpc.DeviceEvent.from_host(e.y, e.z, e.row_offsets, e.sector_id)
    for _ in range(5):
        res = tr.track_event(dev, geo, e.bz, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = tr.track_event(dev, geo, e.bz, prm)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res = tpc.to_numpy(res)
    ORACLE_CHECKS["single_sector"] = dict(
        ev=dict(y=e.y, z=e.z, row_offsets=e.row_offsets, sector_id=e.sector_id), bz=e.bz,
        res=res, n=e.n_clusters)
    return dict(workload=f"one sector, 200 helix tracks, 2% noise, seed 1, {e.n_clusters} clusters",
                events_per_s=round(steps / el, 1), clusters_per_s=round(e.n_clusters * steps / el, 1),
                ms_per_event=round(el / steps * 1e3, 4), n_tracks=int(res["n_tracks"]))


def central_concordance_section(tr, tpc, synth, geo, prm, events, log_):
    """The GPU's tracks of several central events (so that concordance with
    the oracle, computed by the cpu_baseline leg, resolves 99.99% on ~100k
    tracks)."""
    runs = []
    for e in events:
        dev = tpc.DeviceEvent.from_host(e.y, e.z, e.row_offsets, e.sector_id)
        runs.append((dict(y=e.y, z=e.z, row_offsets=e.row_offsets, sector_id=e.sector_id),
                     tpc.to_numpy(tr.track_event(dev, geo, e.bz, prm))))
    ORACLE_CHECKS["central_concordance"] = dict(runs=runs)
    return dict(workload=f"{len(events)} central events (seeds {CENTRAL_SEEDS[0]}-"
                         f"{CENTRAL_SEEDS[len(events) - 1]})",
                tracks=int(sum(r["n_tracks"] for _, r in runs)),
                clusters=int(sum(len(h["y"]) for h, _ in runs)))


def central_batched_section(tr, tpc, synth, geo, prm, events, steps, log_):
    """Central events tracked several at a time (one launch sequence per
    batch, graph replay): the constructor's tail, in which a single event's
    longest tracklets run on an otherwise idle chip, is shared by the batch.
    Throughput against the plain per-event path of the headline; the first
    event's tracks must be bitwise those of the event alone."""
    import torch
    devs = [tpc.DeviceEvent.from_host(e.y, e.z, e.row_offsets, e.sector_id) for e in events]
    n_cl = sum(d.n_clusters for d in devs)
    tr.set_tuning(use_graph=0)
    st = timed_probe(tr, lambda: tr.track_batch(devs, geo, events[0].bz, prm), reps=2)
    per = {k: v / 2 / len(devs) for k, v in st["kernel_ms"].items() if v > 0}
    tr.set_tuning()
    res = tr.track_batch(devs, geo, events[0].bz, prm)
    alone = tr.track_event(devs[0], geo, events[0].bz, prm)
    a, b = tpc.to_numpy(res[0]), tpc.to_numpy(alone)
    same = all(np.array_equal(np.asarray(a[k]).view(np.uint8), np.asarray(b[k]).view(np.uint8))
               for k in ("track_par", "track_meta", "track_cluster", "cluster_track"))
    call, _, _ = raw_batch(tr, tpc, devs, geo, events[0].bz, prm)
    call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return dict(workload=f"{len(devs)} central events per batch (seeds {CENTRAL_SEEDS[0]}-"
                         f"{CENTRAL_SEEDS[len(devs) - 1]}), {n_cl} clusters",
                events_per_s=round(len(devs) * steps / el, 1),
                clusters_per_s=round(n_cl * steps / el, 1),
                ms_per_batch=round(el / steps * 1e3, 3),
                ms_per_event=round(el / steps / len(devs) * 1e3, 4),
                path_hbm=staged_hbm(n_cl * steps / el),
                kernels_ms_per_event={k: round(v, 4) for k, v in per.items()},
                first_event_bitwise_as_alone=bool(same))


def stress_section(tr, tpc, synth, geo, host, steps, log_):
    """Stress events (20000 primaries + 6000 loopers, 10% noise, sigma 0.15)
    in batches of len(host): throughput, the dominant kernel's roofline and
    the path against HBM; concordance and parameter error against the oracle
    on the first event come from the cpu_baseline leg."""
    import torch
    n_events = len(host)
    prm = tpc.default_params(sigma_y=0.15, sigma_z=0.15)
    devs = [tpc.DeviceEvent.from_host(*h) for h in host]
    n_cl = sum(d.n_clusters for d in devs)
    tr.set_tuning(use_graph=0)
    st = timed_probe(tr, lambda: tr.track_batch(devs, geo, 0.5, prm), reps=2)
    roof, per = roofline_of(st, n_cl)
    tr.set_tuning()
    res = tr.track_batch(devs, geo, 0.5, prm)
    call, _, _ = raw_batch(tr, tpc, devs, geo, 0.5, prm)
    call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    y, z, ro, si = host[0]
    ORACLE_CHECKS["stress"] = dict(ev=dict(y=y, z=z, row_offsets=ro, sector_id=si), bz=0.5,
                                   res=tpc.to_numpy(res[0]), n=len(y), prm=prm)
    cps = n_cl * steps / el
    return dict(workload=f"{n_events} stress events per batch (20000 primaries + 6000 loopers, "
                         f"10% noise, sigma 0.15 cm; seeds {STRESS_SEEDS[0]}+), {n_cl} clusters",
                events_per_s=round(n_events * steps / el, 2),
                clusters_per_s=round(cps, 1),
                ms_per_batch=round(el / steps * 1e3, 3),
                roofline=roof, path_hbm=staged_hbm(cps),
                kernels_ms_per_batch={k: round(v, 4) for k, v in per.items()})


def global_section(tr, tpc, synth, geo, prm, e, dev_ev, steps, log_):
    """Global tracking (section 5) on the benchmark event: the whole path
    followed by the prolongation of the tracks into neighbouring sectors,
    against the plain path, and what it adds against MC truth; the oracle's
    prolongations (concordance) come from the cpu_baseline leg."""
    import torch
    from paper_1712_09407_amd import quality
    for _ in range(3):
        trk, pro = tr.track_event_global(dev_ev, geo, e.bz, prm)
        tr.track_event(dev_ev, geo, e.bz, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        tr.track_event(dev_ev, geo, e.bz, prm)
    torch.cuda.synchronize()
    plain = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        trk, pro = tr.track_event_global(dev_ev, geo, e.bz, prm)
    torch.cuda.synchronize()
    glob = (time.perf_counter() - t0) / steps
    tr.set_timing(None)  # per-kernel means over 10 calls
    tr.reset_stats()
    for _ in range(10):
        tr.track_event_global(dev_ev, geo, e.bz, prm)
    st = tr.stats()
    tr.set_timing([])
    trk, pro = tpc.to_numpy(trk), tpc.to_numpy(pro)
    q = quality.prolongation_report(e, trk, pro)
    ORACLE_CHECKS["global_tracking"] = dict(
        ev=dict(y=e.y, z=e.z, row_offsets=e.row_offsets, sector_id=e.sector_id), bz=e.bz,
        trk=trk, pro=pro)
    ks = ("k_construct", "k_pro_init", "k_prolong", "k_pro_own", "k_pro_reduce", "k_pro_scan",
          "k_pro_output")
    return dict(workload="benchmark central event, whole path + prolongation into "
                         "neighbouring sectors",
                events_per_s=round(1.0 / glob, 2), ms_per_event=round(glob * 1e3, 4),
                plain_ms_per_event=round(plain * 1e3, 4),
                overhead_ms=round((glob - plain) * 1e3, 4),
                kernels_ms={k: round(st["kernel_ms"][k] / max(1, st["kernel_launches"][k]), 5)
                            for k in ks},
                **q)


def merge_section(tr, tpc, synth, geo, prm, e, dev_ev, steps, log_):
    """The track merger with refit on the benchmark event: the whole path,
    global tracking, joins and refits, against the plain and global paths;
    quality of the joined tracks against MC truth with and without global
    tracking (section 5's claim) and of the sector tracks; the oracle's
    joined tracks (concordance) come from the cpu_baseline leg."""
    import torch
    from paper_1712_09407_amd import quality

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    plain = timed(lambda: tr.track_event(dev_ev, geo, e.bz, prm))
    glob = timed(lambda: tr.track_event_global(dev_ev, geo, e.bz, prm))
    merged = timed(lambda: tr.track_event_merged(dev_ev, geo, e.bz, prm))
    merged0 = timed(lambda: tr.track_event_merged(dev_ev, geo, e.bz, prm, use_global=False))
    tr.set_timing(None)  # per-kernel means over 10 calls
    tr.reset_stats()
    for _ in range(10):
        trk, pro, mg = tr.track_event_merged(dev_ev, geo, e.bz, prm)
    st = tr.stats()
    tr.set_timing([])
    trk, mg = tpc.to_numpy(trk), tpc.to_numpy(mg)
    _, _, mg0 = tr.track_event_merged(dev_ev, geo, e.bz, prm, use_global=False)
    mg0 = tpc.to_numpy(mg0)
    ORACLE_CHECKS["merger"] = dict(
        ev=dict(y=e.y, z=e.z, row_offsets=e.row_offsets, sector_id=e.sector_id), bz=e.bz,
        trk=trk, mg=mg)
    ks = ("k_ends", "k_mrg_init", "k_mrg_match", "k_mrg_link", "k_mrg_chain", "k_mrg_reduce",
          "k_mrg_scan", "k_mrg_write", "k_rowmap", "k_refit")

    def q(rep):
        out = {k: (round(v, 6) if isinstance(v, float) else v) for k, v in rep.items()
               if k != "resolution"}
        out["resolution"] = {k: round(v, 6) for k, v in rep.get("resolution", {}).items()}
        return out

    sec = quality.evaluate(e, trk)
    # the refit's algorithmic work: every list cluster is one helix step
    # (174 FLOP) and one Kalman update (129 FLOP) in each of the two passes
    # (FP32 vector ALU; the seed circle and rotations are negligible)
    refit_ms = st["kernel_ms"]["k_refit"] / max(1, st["kernel_launches"]["k_refit"])
    refit_flop = 2.0 * (174 + 129) * int(mg["n_clusters"])
    refit_tf = refit_flop / (refit_ms * 1e-3) / 1e12 if refit_ms > 0 else 0.0
    return dict(workload="benchmark central event: sector tracks joined across sector edges "
                         "and the membrane, refitted from their cluster lists",
                events_per_s=round(1.0 / merged, 2), ms_per_event=round(merged * 1e3, 4),
                ms_per_event_without_global=round(merged0 * 1e3, 4),
                global_ms_per_event=round(glob * 1e3, 4),
                plain_ms_per_event=round(plain * 1e3, 4),
                kernels_ms={k: round(st["kernel_ms"][k] / max(1, st["kernel_launches"][k]), 5)
                            for k in ks},
                roofline_refit=dict(bound="alu", achieved=round(refit_tf, 4),
                                    peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                                    frac=round(refit_tf / PEAK_FP32_TFLOPS, 6),
                                    kernel="k_refit", kernel_ms=round(refit_ms, 5),
                                    algorithmic_per_launch=f"{refit_flop:.4g} FLOP",
                                    note="latency-bound: the longest list is a chain of "
                                         "dependent Kalman steps"),
                tracks=int(trk["n_tracks"]), joined_tracks=int(mg["n"]),
                joins=int(trk["n_tracks"] - mg["n"]),
                quality_sector_tracks=dict(efficiency=round(sec["efficiency"], 6),
                                           resolution={k: round(v, 6) for k, v in
                                                       sec["resolution"].items()}),
                quality_joined=q(quality.merged_report(e, mg0)),
                quality_joined_with_global=q(quality.merged_report(e, mg)))


def cpu_baseline_leg(tpc, prm, main_args, log_):
    """The oracle, on this host's cores: the headline baseline, then the
    comparisons the sections asked for (ORACLE_CHECKS).  Returns the baseline,
    the headline concordance and, per section, fields to merge into it."""
    import oracle
    from oracle import concordance
    from paper_1712_09407_amd import synth
    geo_t = (synth.ROW_X, synth.TAN_HALF, synth.Z_MAX)
    op = oracle_params(tpc, prm)
    base, conc = cpu_baseline(*main_args, op)
    cores = max(1, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                else (os.cpu_count() or 1))
    extra = {}
    for name, chk in ORACLE_CHECKS.items():
        log_(f"oracle check: {name}")
        try:
            if name == "single_sector":
                t1 = time.perf_counter()
                ref = oracle.track_event(chk["ev"], geo_t, chk["bz"], op, n_threads=1)
                t_orc = time.perf_counter() - t1
                rep = concordance.compare(ref, chk["res"], chk["n"])
                extra[name] = dict(oracle_s_per_event=round(t_orc, 4), oracle_cores=1,
                                   cluster_concordance=rep["cluster_concordance"],
                                   track_concordance=rep["track_concordance"],
                                   par_fail=rep["par_fail"])
            elif name == "central_concordance":
                worst, miss_tr, par_fail, par_cmp, t_orc = 1.0, 0, 0, 0, 0.0
                for ev, res in chk["runs"]:
                    t1 = time.perf_counter()
                    ref = oracle.track_event(ev, geo_t, 0.5, op, n_threads=cores)
                    t_orc += time.perf_counter() - t1
                    rep = concordance.compare(ref, res, len(ev["y"]))
                    worst = min(worst, rep["cluster_concordance"], rep["track_concordance"])
                    miss_tr += round((1 - rep["track_concordance"]) * rep["n_tracks_a"])
                    par_fail += rep["par_fail"]
                    par_cmp += rep["par_compared"]
                extra[name] = dict(worst_concordance=worst, unmatched_tracks=miss_tr,
                                   par_compared=par_cmp, par_fail=par_fail,
                                   oracle_s_per_event=round(t_orc / len(chk["runs"]), 4),
                                   oracle_cores=cores)
            elif name == "stress":
                t1 = time.perf_counter()
                ref = oracle.track_event(chk["ev"], geo_t, chk["bz"],
                                         oracle_params(tpc, chk["prm"]), n_threads=cores)
                t_orc = time.perf_counter() - t1
                rep = concordance.compare(ref, chk["res"], chk["n"])
                extra[name] = dict(oracle_s_per_event=round(t_orc, 3), oracle_cores=cores,
                                   cluster_concordance=rep["cluster_concordance"],
                                   track_concordance=rep["track_concordance"],
                                   par_compared=rep["par_compared"], par_fail=rep["par_fail"],
                                   par_max_rel=rep["par_max_rel"],
                                   par_other_seed=rep["par_other_seed"])
            elif name == "merger":
                t1 = time.perf_counter()
                rtr, _, rmg = oracle.track_event_merged(chk["ev"], geo_t, chk["bz"], op,
                                                        merge_chi2=tpc.MERGE_CHI2,
                                                        n_threads=cores)
                t_orc = time.perf_counter() - t1
                rep = concordance.compare_merged(rtr, rmg, chk["trk"], chk["mg"],
                                                 len(chk["ev"]["y"]))
                extra[name] = dict(oracle_s_per_event=round(t_orc, 4), oracle_cores=cores,
                                   oracle_joined_tracks=int(rmg["n"]),
                                   **{k: (round(v, 7) if isinstance(v, float) else v)
                                      for k, v in rep.items()})
            elif name == "global_tracking":
                t1 = time.perf_counter()
                rtr, rpro = oracle.track_event_global(chk["ev"], geo_t, chk["bz"], op,
                                                      n_threads=cores)
                t_orc = time.perf_counter() - t1
                extra[name] = dict(oracle_s_per_event=round(t_orc, 4), oracle_cores=cores,
                                   oracle_prolongations=int(rpro["n"]),
                                   **concordance.compare_prolongations(
                                       rtr, rpro, chk["trk"], chk["pro"], len(chk["ev"]["y"])))
        except Exception as exc:  # the headline line must still be printed
            extra[name] = dict(oracle_error=f"{type(exc).__name__}: {exc}")
    return base, conc, extra


def alpha_scan_section(tr, tpc, synth, geo, evs, log_):
    """Track-finding quality against MC truth as a function of the weight's
    alpha (section 3.1; alpha = infinity is the longest-track rule), on
    central events."""
    from paper_1712_09407_amd import quality
    devs = [tpc.DeviceEvent.from_host(e.y, e.z, e.row_offsets, e.sector_id) for e in evs]
    rows = {}
    for a in quality.ALPHAS:
        prm = tpc.default_params(alpha=quality.alpha_value(a))
        reps = [quality.evaluate(e, tpc.to_numpy(tr.track_event(d, geo, e.bz, prm)))
                for e, d in zip(evs, devs)]
        m = quality.merge(reps)
        rows["inf" if a == float("inf") else f"{a:g}"] = dict(
            efficiency=round(m["efficiency"], 5), clone_rate=round(m["clone_rate"], 5),
            fake_rate=round(m["fake_rate"], 5), tracks=m["tracks"],
            **{f"res_{k}": round(v, 6) for k, v in m["resolution"].items() if k != "tracks"})
        log_(f"alpha {a}: {rows['inf' if a == float('inf') else f'{a:g}']}")
    return dict(workload=f"{len(evs)} central events (seeds {ALPHA_SEEDS[0]}-{ALPHA_SEEDS[-1]}), "
                         "quality against MC truth per alpha", alphas=rows)


def batched_section(tr, tpc, synth, geo, prm, host, steps, log_):
    """Many events of very different multiplicity in one launch sequence
    (graph replay, autotuned), against the plain per-event loop on the same
    events; the dominant kernel's roofline (eager probe, every kernel timed)
    and the path against HBM."""
    import ctypes as C
    import torch
    from paper_1712_09407_amd import tune
    n_events = len(host)
    devs = [tpc.DeviceEvent.from_host(*h) for h in host]
    n_cl = sum(d.n_clusters for d in devs)
    # plain per-event loop over the same events (each call on arguments and
    # outputs prepared once, like the batch's)
    tr.set_tuning(use_graph=0)
    singles = [tr.batch_args([d]) for d in devs]
    sh = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for d in devs[:4]:
        tr.track_event(d, geo, 0.5, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for es1, _, trs1, _, _ in singles:
        rc = tr.track_event_raw(es1[0], geo, 0.5, prm, trs1[0], sh)
        if rc != 0:
            raise tpc.TpcError(rc, tpc.last_error())
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    # autotune, then time graph replays of the whole batch
    name = torch.cuda.get_device_name(0)
    rec = tune.autotune(tr, devs, geo, 0.5, prm, reps=1, device_name=name, use_cache=False,
                        log=log_)
    tuned = tr.set_tuning(use_graph=0, **rec["best"])
    st = timed_probe(tr, lambda: tr.track_batch(devs, geo, 0.5, prm), reps=2)
    roof, per = roofline_of(st, n_cl)
    tr.set_tuning(use_graph=1, **rec["best"])
    res = tr.track_batch(devs, geo, 0.5, prm)
    call, _, _ = raw_batch(tr, tpc, devs, geo, 0.5, prm)
    call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tr.set_tuning()
    cps = n_cl * steps / el
    return dict(workload=f"{n_events} events, multiplicity log-uniform 100-8000 tracks "
                         f"(seeds 3000+), {n_cl} clusters", events=n_events, clusters=n_cl,
                events_per_s=round(n_events * steps / el, 2),
                clusters_per_s=round(cps, 1),
                ms_per_batch=round(el / steps * 1e3, 3),
                plain_loop_events_per_s=round(n_events / plain_s, 2),
                speedup_vs_plain=round((n_events * steps / el) / (n_events / plain_s), 3),
                tuned=rec["best"], graph=True,
                tracks=int(sum(r["n_tracks"] for r in res)),
                roofline=roof, path_hbm=staged_hbm(cps),
                kernels_ms_per_batch={k: round(v, 4) for k, v in per.items()})


def serving_section(tpc, synth, geo, prm, host, rates, n_events, log_):
    """Poisson arrivals of events with log-uniform multiplicity: the
    continuous-batching server against the one-at-a-time path, same GPU."""
    from paper_1712_09407_amd import serve
    pool = [tpc.HostEvent(*h) for h in host]
    out = dict(workload=f"Poisson arrivals, {len(pool)} distinct events of multiplicity "
                        f"log-uniform 100-8000 tracks, two runs of {n_events} events per "
                        f"rate and configuration",
               rates={})
    configs = (("continuous_batching", dict(max_batch=64, n_workers=2, use_graph=1)),
               ("one_at_a_time", dict(max_batch=1, n_workers=1, use_graph=0)))
    for rate in rates:
        # two arrival sequences per configuration, the configurations taking
        # turns; the percentiles are over both runs' events
        runs = {name: [] for name, _ in configs}
        for seed in (4, 5):
            for name, cfg in configs:
                srv = tpc.Server(geo, 0.5, prm, keep_results=0, **cfg)
                serve.run(srv, pool, rate_hz=rate, n_events=min(64, n_events), seed=99)  # warm
                res, _ = serve.run(srv, pool, rate_hz=rate, n_events=n_events, seed=seed)
                srv.close()
                runs[name].append(res)
        row = {}
        for name, rs in runs.items():
            lat = np.concatenate([r["lat_ms"] for r in rs])
            row[name] = dict(p50_ms=round(float(np.percentile(lat, 50)), 3),
                             p99_ms=round(float(np.percentile(lat, 99)), 3),
                             mean_ms=round(float(lat.mean()), 3),
                             sustained_events_per_s=round(
                                 float(np.mean([r["sustained_events_per_s"] for r in rs])), 1),
                             offered_events_per_s=round(
                                 float(np.mean([r["offered_events_per_s"] for r in rs])), 1),
                             events=int(lat.size),
                             batches=int(sum(r["stats"]["batches"] for r in rs)),
                             busy_retries=int(sum(r["busy_retries"] for r in rs)))
            log_(f"serve {rate} Hz {name}: {row[name]}")
        out["rates"][str(int(rate))] = row
    # admission under a small budget: a central-size event (1.33M clusters at
    # about 160 B each) nearly fills 256 MiB, so arrivals wait for completions
    rate = max(rates)
    try:
        srv = tpc.Server(geo, 0.5, prm, keep_results=0, max_batch=64, n_workers=2, use_graph=1,
                         hbm_budget_bytes=256 << 20)
        serve.run(srv, pool, rate_hz=rate, n_events=min(64, n_events), seed=99)
        res, _ = serve.run(srv, pool, rate_hz=rate, n_events=n_events, seed=4)
        srv.close()
        out["small_budget"] = dict(budget_bytes=256 << 20, rate_hz=rate,
                                   **{k: res[k] for k in ("p50_ms", "p99_ms", "mean_ms",
                                                          "sustained_events_per_s",
                                                          "offered_events_per_s",
                                                          "busy_retries")},
                                   batches=res["stats"]["batches"])
    except Exception as exc:  # the headline line must still be printed
        out["small_budget"] = dict(error=f"{type(exc).__name__}: {exc}")
    log_(f"serve {rate} Hz, 256 MiB budget: {out['small_budget']}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--event", choices=("c2_central", "c1_sector", "c5_stress"),
                    default="c2_central",
                    help="the timed event (the headline is the central event; the others "
                         "are for profiling)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="wall time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one plain 256 MiB device copy first (counter scale for rocprofv3)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--batch-events", type=int, default=64,
                    help="events in the batched-path measurement (0 = skip)")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--no-extra", dest="extra", action="store_false",
                    help="skip the single-sector, ten-event concordance and stress sections")
    ap.add_argument("--path", choices=("plain", "global", "merged"), default="plain",
                    help="the timed step: the sector tracker (default), plus global tracking, "
                         "plus the track merger with refit")
    ap.add_argument("--serve-events", type=int, default=2000,
                    help="events per arrival rate in the serving measurement (0 = skip)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the tracker runs on a single GPU; --gpus must be 1 "
              "(several GPUs would each track their own events, one process per GPU)", file=sys.stderr)
        sys.exit(2)

    # every host event first: nothing may fork once the GPU is initialised
    host = pregenerate(args)
    import torch
    from paper_1712_09407_amd import synth, tpc
    import ctypes as C

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    e = host["main"][0]
    log("benchmark event", args.event, "seed", args.seed, e.n_clusters, "clusters")
    N = e.n_clusters
    geo = tpc.make_geometry(synth.ROW_X, synth.TAN_HALF, synth.Z_MAX)
    dev_ev = tpc.DeviceEvent.from_host(e.y, e.z, e.row_offsets, e.sector_id, device=dev)
    prm = tpc.default_params(sigma_y=e.config.sigma, sigma_z=e.config.sigma)
    tr = tpc.Tracker(0)
    cap_t, cap_c = max(1024, N // 40), N
    out = dict(track_par=torch.empty((cap_t, 8), dtype=torch.float32, device=dev),
               track_meta=torch.empty((cap_t, 4), dtype=torch.int32, device=dev),
               track_cluster=torch.empty(cap_c, dtype=torch.int32, device=dev),
               cluster_track=torch.empty(N, dtype=torch.int32, device=dev))
    if args.copy_probe:
        a = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: 268435456 bytes read, 268435456 bytes written")
        del a, b
    stream = torch.cuda.current_stream()
    sh = C.c_void_p(stream.cuda_stream)
    nt, nc = C.c_int32(0), C.c_int32(0)
    tracks = tpc.Tracks(cap_t, cap_c, C.pointer(nt), C.pointer(nc), out["track_par"].data_ptr(),
                        out["track_meta"].data_ptr(), out["track_cluster"].data_ptr(),
                        out["cluster_track"].data_ptr())
    cev = dev_ev.cstruct()
    # outputs of the global and merged paths, allocated once
    i32 = dict(dtype=torch.int32, device=dev)
    f32 = dict(dtype=torch.float32, device=dev)
    pbuf = dict(par=torch.empty((cap_t, 8), **f32), meta=torch.empty((cap_t, 5), **i32),
                cluster=torch.empty(max(16, N // 8), **i32))
    mbuf = dict(par=torch.empty((cap_t, 8), **f32), meta=torch.empty((cap_t, 5), **i32),
                cluster=torch.empty(N, **i32), track_merged=torch.empty(cap_t, **i32))
    psz = [C.c_int32(0) for _ in range(4)]
    pro = tpc.Prolongations(cap_t, int(pbuf["cluster"].shape[0]), C.pointer(psz[0]),
                            C.pointer(psz[1]), pbuf["par"].data_ptr(), pbuf["meta"].data_ptr(),
                            pbuf["cluster"].data_ptr())
    mg = tpc.Merged(cap_t, N, C.pointer(psz[2]), C.pointer(psz[3]), mbuf["par"].data_ptr(),
                    mbuf["meta"].data_ptr(), mbuf["cluster"].data_ptr(),
                    mbuf["track_merged"].data_ptr())

    def step():
        if args.path == "plain":
            rc = tr.track_event_raw(cev, geo, e.bz, prm, tracks, sh)
        elif args.path == "global":
            rc = tr.track_event_global_raw(cev, geo, e.bz, prm, tracks, pro, sh)
        else:
            rc = tr.track_event_merged_raw(cev, geo, e.bz, prm, tpc.MERGE_CHI2, tracks, pro, mg,
                                           sh)
        if rc != 0:
            raise tpc.TpcError(rc, tpc.last_error())

    # warm-up, then one more step with every kernel timed: the dominant kernel
    for i in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    tr.set_timing(None)
    tr.reset_stats()
    step()
    st = tr.stats()
    per = {k: st["kernel_ms"][k] / max(1, st["kernel_launches"][k]) for k in st["kernel_ms"]}
    dominant = max(per, key=per.get)
    log("warm-up kernel ms:", {k: round(v, 4) for k, v in per.items()}, "dominant:", dominant)

    # timed region: only the dominant kernel carries an event pair
    tr.reset_stats()
    tr.set_timing([dominant])
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        step()
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = tr.stats()
    log(f"timed {args.steps} steps in {el:.4f} s")
    res = dict(n_tracks=nt.value, n_track_clusters=nc.value,
               track_par=out["track_par"][:nt.value].cpu().numpy(),
               track_meta=out["track_meta"][:nt.value].cpu().numpy(),
               track_cluster=out["track_cluster"][:nc.value].cpu().numpy(),
               cluster_track=out["cluster_track"][:N].cpu().numpy())

    dom_ms = st["kernel_ms"][dominant] / max(1, st["kernel_launches"][dominant])
    ev_n = max(1, st["events"])
    if dominant == "k_construct":
        flops = (st["steps"] * FLOP_STEP + st["updates"] * FLOP_UPDATE +
                 st["candidates"] * FLOP_CAND) / ev_n
        achieved = flops / (dom_ms * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=round(achieved, 4), peak=PEAK_FP32_TFLOPS,
                    unit="TFLOP/s", frac=round(achieved / PEAK_FP32_TFLOPS, 6),
                    kernel=dominant, kernel_ms=round(dom_ms, 5),
                    algorithmic_per_launch=f"{flops:.4g} FLOP")
        work_key = "flop_per_launch"
    else:
        nbytes = BYTES_PER_CLUSTER.get(dominant, 16) * N
        achieved = nbytes / (dom_ms * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=round(achieved, 2), peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=round(achieved / PEAK_HBM_GBS, 6), kernel=dominant,
                    kernel_ms=round(dom_ms, 5), algorithmic_per_launch=f"{nbytes} B")
    traffic = None
    if os.path.exists(args.traffic_json):
        tj = json.load(open(args.traffic_json))
        if tj.get("kernel") == dominant and tj.get("kernel_src_sha") == kernel_src_sha():
            traffic = tj.get("bytes_per_launch")
    roof["traffic"] = traffic

    # the whole path against HBM: the staged algorithmic model, the
    # implementation's own traffic model, and the counters
    eps = args.steps / el
    path_hbm = staged_hbm(N * eps)
    pb = path_bytes(N, st["tracklets"] / ev_n, st["steps"] / ev_n, st["candidates"] / ev_n,
                    nt.value, nc.value)
    path_hbm["implementation_model"] = dict(
        note="this implementation's traffic model: 16 B per candidate record, per-row hits "
             "written and read back, owner keys",
        bytes_per_event=int(pb), frac=round(pb * eps / 1e9 / PEAK_HBM_GBS, 6))
    path_hbm["measured_bytes_per_event"] = None
    if os.path.exists(args.traffic_json):
        tj = json.load(open(args.traffic_json))
        if tj.get("kernel_src_sha") == kernel_src_sha() and tj.get("path_bytes_per_event"):
            mb = tj["path_bytes_per_event"]
            path_hbm.update(measured_bytes_per_event=int(mb),
                            measured_frac=round(mb * eps / 1e9 / PEAK_HBM_GBS, 6))

    ms = el / args.steps * 1e3
    lat_ms = sorted(x * 1e3 for x in lat)
    p = lambda q: lat_ms[min(len(lat_ms) - 1, int(math.ceil(q * len(lat_ms))) - 1)]
    line = dict(metric=METRIC, value=round(args.steps / el, 3), unit="events/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=round(ms, 4),
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
                data="synthetic",
                config=dict(workload={
                                "c2_central": "central Pb-Pb-like event, ",
                                "c1_sector": "one sector, ",
                                "c5_stress": "stress event, "}[args.event] + {
                                "plain": "plain per-event path",
                                "global": "per-event path with global tracking",
                                "merged": "per-event path with global tracking and the track "
                                          "merger with refit"}[args.path] + {
                                "c2_central": ": 36 sectors x 159 rows, 8000 primary helix "
                                              "tracks, 5% noise clusters",
                                "c1_sector": ": 159 rows, 200 helix tracks, 2% noise clusters",
                                "c5_stress": ": 36 sectors x 159 rows, 20000 primaries + 6000 "
                                             "loopers, 10% noise, sigma 0.15 cm"}[args.event],
                            n_clusters=N, seed=args.seed, bz_tesla=e.bz),
                clusters_per_s=round(N * args.steps / el, 1),
                latency_ms=dict(p50=round(p(0.5), 4), p99=round(p(0.99), 4)),
                n_tracks=nt.value,
                kernels_ms={k: round(v, 5) for k, v in per.items()},
                work_per_event=dict(tracklets=st["tracklets"] / ev_n, steps=st["steps"] / ev_n,
                                    updates=st["updates"] / ev_n,
                                    candidates=st["candidates"] / ev_n),
                roofline=roof, path_hbm=path_hbm)
    if args.batch_events > 0:
        log("batched path ...")
        line["batched"] = batched_section(tr, tpc, synth, geo, prm, host["batch"],
                                          args.batch_steps, log)
        log("batched:", line["batched"])
    if args.serve_events > 0 and args.batch_events > 0:
        log("serving ...")
        line["serving"] = serving_section(tpc, synth, geo, prm, host["batch"],
                                          (200.0, 500.0, 1000.0), args.serve_events, log)
    if args.extra:
        alpha_evs = [host["central"][CENTRAL_SEEDS.index(s_)] for s_ in ALPHA_SEEDS]
        sections = (("single_sector", lambda: single_sector_section(tr, tpc, synth, geo, prm, 500, log)),
                    ("central_concordance", lambda: central_concordance_section(
                        tr, tpc, synth, geo, prm, host["central"], log)),
                    ("central_batched", lambda: central_batched_section(
                        tr, tpc, synth, geo, prm, host["central"][:8], 10, log)),
                    ("stress", lambda: stress_section(tr, tpc, synth, geo, host["stress"], 3, log)),
                    ("global_tracking", lambda: global_section(tr, tpc, synth, geo, prm, e,
                                                               dev_ev, 20, log)),
                    ("merger", lambda: merge_section(tr, tpc, synth, geo, prm, e, dev_ev, 20,
                                                     log)),
                    ("alpha_scan", lambda: alpha_scan_section(tr, tpc, synth, geo, alpha_evs, log)))
        for name, fn in sections:
            log(f"{name} ...")
            try:
                line[name] = fn()
            except Exception as exc:  # the headline line must still be printed
                line[name] = dict(error=f"{type(exc).__name__}: {exc}")
            log(f"{name}:", line[name])
    if not args.no_cpu_baseline:
        log("oracle baseline on the host cores ...")
        ev_host = dict(y=e.y, z=e.z, row_offsets=e.row_offsets, sector_id=e.sector_id)
        base, conc, extra = cpu_baseline_leg(
            tpc, prm, (ev_host, (synth.ROW_X, synth.TAN_HALF, synth.Z_MAX), e.bz, res, N,
                       args.cpu_seconds), log)
        line["cpu_baseline"] = base
        line["concordance"] = conc
        for name, fields in extra.items():
            if isinstance(line.get(name), dict):
                line[name].update(fields)
    else:
        line["cpu_baseline"] = None
    tr.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
