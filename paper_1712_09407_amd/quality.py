"""Track-finding quality against the Monte-Carlo truth of synthetic events.

The paper studies the weight of its cluster assignment (section 3.1): the
weight w = n (alpha - chi^2/beta) of a tracklet trades its length against its
fit quality, alpha -> infinity gives the longest-track rule, and the value
alpha = 6 was chosen from a scan of the tracking quality (the scan's figure is
lost).  This module measures that quality on the tracker's output.  The
definitions are the usual ones, stated here because the paper does not:

* a sector segment of a particle is its clusters in one sector slot; it is
  findable if it has at least `min_clusters` (section 5: 30) clusters;
* a track's label is the particle of most of its clusters; the track is fake
  if the label is noise or covers less than `purity` of its clusters;
* a findable segment is found if a non-fake track of its sector slot carries
  its label; further such tracks are clones;
* efficiency = found / findable, clone rate = clones / found,
  fake rate = fakes / tracks;
* resolution: for the first (non-clone) track of each found segment, the
  track parameters (at its innermost cluster) minus the truth of the
  particle at that cluster: y, z (cm), sin(phi), tan(lambda) and the relative
  q/pT error; each as the half-width of the central 68% (a robust sigma).

Only host-side numpy: it reads the tracker's output dict (either path) and
the event's truth.
"""
from __future__ import annotations

import math

import numpy as np

from . import synth


def _true_sinphi(e: synth.Event, c: np.ndarray, slot_of: np.ndarray) -> np.ndarray:
    """Local sin(phi) of the particle at cluster c: the direction of its circle
    (through the origin, centre on the side given by q B) at the true
    crossing, relative to the sector's centre line."""
    row = e.row_of()[c] % synth.N_ROWS
    x = synth.ROW_X[row].astype(np.float64)
    alpha = np.array([synth.sector_alpha(int(s)) for s in e.sector_id])[slot_of]
    X = x * np.cos(alpha) - e.y_true[c] * np.sin(alpha)
    Y = x * np.sin(alpha) + e.y_true[c] * np.cos(alpha)
    p = e.mc_track[c]
    R = e.track_pt[p] / (synth.C_LIGHT * abs(e.bz))
    h = np.sign(e.track_q[p] * e.bz)
    phi0 = e.track_phi0[p]
    cx, cy = R * h * np.sin(phi0), -R * h * np.cos(phi0)
    psi = np.arctan2(Y - cy, X - cx) - h * (math.pi / 2)  # velocity direction (phi0 at the origin)
    return np.sin(psi - alpha)


def _w68(v: np.ndarray) -> float:
    if v.size == 0:
        return float("nan")
    lo, hi = np.percentile(v, [16.0, 84.0])
    return float(0.5 * (hi - lo))


def evaluate(e: synth.Event, res: dict, min_clusters: int = 30, purity: float = 0.9) -> dict:
    """Efficiency, clone and fake rates and resolution of one event's tracks."""
    mc = np.asarray(e.mc_track)
    n_slots = int(e.sector_id.shape[0])
    slot = e.row_of() // synth.N_ROWS
    sig = mc >= 0
    seg_key = mc[sig].astype(np.int64) * n_slots + slot[sig]
    keys, cnt = np.unique(seg_key, return_counts=True)
    findable = set(keys[cnt >= min_clusters].tolist())

    meta = np.asarray(res["track_meta"])
    tcl = np.asarray(res["track_cluster"])
    par = np.asarray(res["track_par"], np.float64)
    found, first_of = set(), []
    fakes = clones = 0
    for t in range(int(res["n_tracks"])):
        cl = tcl[meta[t, 2]:meta[t, 2] + meta[t, 1]]
        lab, c = np.unique(mc[cl], return_counts=True)
        j = int(np.argmax(c))
        if lab[j] < 0 or c[j] < purity * cl.shape[0]:
            fakes += 1
            continue
        key = int(lab[j]) * n_slots + int(slot[cl[0]])
        if key in found:
            clones += 1
            continue
        found.add(key)
        inner = cl[mc[cl] == lab[j]][0]  # innermost cluster of the particle
        first_of.append((t, int(cl[0]), int(inner)))
    n_found = len(found & findable)
    out = dict(findable=len(findable), found=n_found,
               efficiency=n_found / max(1, len(findable)),
               clones=clones, clone_rate=clones / max(1, len(found)),
               fakes=fakes, fake_rate=fakes / max(1, int(res["n_tracks"])),
               tracks=int(res["n_tracks"]))
    # resolution at the track's innermost cluster, when it is the particle's
    sel = [(t, c0) for t, c0, inner in first_of if c0 == inner]
    if sel:
        t = np.array([a for a, _ in sel])
        c0 = np.array([b for _, b in sel])
        p = mc[c0]
        q_pt = e.track_q[p] / e.track_pt[p]
        out["resolution"] = dict(
            tracks=int(t.shape[0]),
            y_cm=_w68(par[t, 1] - e.y_true[c0]),
            z_cm=_w68(par[t, 2] - e.z_true[c0]),
            sinphi=_w68(par[t, 3] - _true_sinphi(e, c0, slot[c0])),
            tanl=_w68(par[t, 4] - e.track_tanl[p]),
            qpt_rel=_w68((par[t, 5] - q_pt) / q_pt),
            charge_wrong=float(np.mean(np.sign(par[t, 5]) != np.sign(q_pt))))
    return out


def merge(reports: list) -> dict:
    """Sum of counts and recomputed rates over several events' reports; the
    resolution entries are averaged weighted by their track counts."""
    tot = {k: sum(r[k] for r in reports) for k in ("findable", "found", "clones", "fakes", "tracks")}
    tot["efficiency"] = tot["found"] / max(1, tot["findable"])
    tot["clone_rate"] = tot["clones"] / max(1, tot["found"])
    tot["fake_rate"] = tot["fakes"] / max(1, tot["tracks"])
    rs = [r["resolution"] for r in reports if "resolution" in r]
    if rs:
        n = sum(r["tracks"] for r in rs)
        tot["resolution"] = {k: sum(r[k] * r["tracks"] for r in rs) / n
                             for k in rs[0] if k != "tracks"}
        tot["resolution"]["tracks"] = n
    return tot


ALPHAS = (1.0, 2.0, 4.0, 6.0, 10.0, math.inf)


def alpha_value(alpha: float) -> float:
    """The weight's alpha as the tracker takes it.  Infinity becomes 1e9: an
    FP32 value (exactly 15625000 * 2^6) so large that alpha - chi^2/(ndf beta)
    rounds to alpha itself whenever chi^2/ndf < 32, so w = n alpha orders by
    length alone and equal lengths tie, to be broken by the seed id: the
    longest-track rule of section 3.1."""
    return 1.0e9 if math.isinf(alpha) else float(alpha)


def prolongation_report(e: synth.Event, res: dict, pro: dict, min_clusters: int = 30,
                        purity: float = 0.9) -> dict:
    """What global tracking (section 5) adds to one event's tracks.

    A short piece is a particle's clusters in one sector slot when they are
    fewer than `min_clusters` (so no sector track can hold them) and the
    particle has a found (non-fake) sector track in another slot.  Reported:
    the clusters of short pieces, the fraction of them that a prolongation of
    one of the particle's tracks collected, and the purity of the prolongation
    clusters (the fraction that belong to the particle of their track).
    """
    mc = np.asarray(e.mc_track)
    slot = e.row_of() // synth.N_ROWS
    meta = np.asarray(res["track_meta"])
    tcl = np.asarray(res["track_cluster"])
    label = np.full(int(res["n_tracks"]), -1, np.int64)
    for t in range(int(res["n_tracks"])):
        cl = tcl[meta[t, 2]:meta[t, 2] + meta[t, 1]]
        lab, c = np.unique(mc[cl], return_counts=True)
        j = int(np.argmax(c))
        if lab[j] >= 0 and c[j] >= purity * cl.shape[0]:
            label[t] = lab[j]
    found = set(label[label >= 0].tolist())
    sig = mc >= 0
    key = mc[sig].astype(np.int64) * int(e.sector_id.shape[0]) + slot[sig]
    keys, cnt = np.unique(key, return_counts=True)
    short = {int(k) for k, n in zip(keys, cnt)
             if n < min_clusters and int(k) // int(e.sector_id.shape[0]) in found}
    in_short = np.zeros(mc.shape[0], bool)
    idx = np.nonzero(sig)[0]
    in_short[idx] = np.isin(key, np.fromiter(short, np.int64, len(short)))
    pm = np.asarray(pro["meta"])
    pcl = np.asarray(pro["cluster"])
    got = right = 0
    total_pro = int(pcl.shape[0])
    for k in range(int(pro["n"])):
        t, _, _, n, first = (int(v) for v in pm[k])
        cl = pcl[first:first + n]
        ok = mc[cl] == label[t]
        right += int(np.sum(ok & (label[t] >= 0)))
        got += int(np.sum(ok & in_short[cl] & (label[t] >= 0)))
    n_short = int(np.sum(in_short))
    return dict(prolongations=int(pro["n"]), prolongation_clusters=total_pro,
                short_piece_clusters=n_short,
                short_piece_recovered=got / max(1, n_short),
                prolongation_purity=right / max(1, total_pro))


def merged_report(e: synth.Event, merged: dict, min_clusters: int = 30,
                  purity: float = 0.9) -> dict:
    """Quality of joined (merged) tracks against the truth.

    A particle is findable if it has at least `min_clusters` clusters in the
    event; it is found if a joined track with at least `purity` of its list
    on the particle carries it; further such tracks are split tracks.
    Resolution: for the first joined track of each found particle whose
    refit succeeded and whose list starts on the particle, its parameters
    (at the innermost fitted cluster, the list's first, in that sector's
    frame) minus the truth there, as half-widths of the central 68%."""
    mc = np.asarray(e.mc_track)
    sig = mc >= 0
    lab_all, cnt_all = np.unique(mc[sig], return_counts=True)
    findable = set(lab_all[cnt_all >= min_clusters].tolist())
    meta = np.asarray(merged["meta"]).reshape(-1, 5)
    par = np.asarray(merged["par"], np.float64).reshape(-1, 8)
    cl_all = np.asarray(merged["cluster"])
    slot = e.row_of() // synth.N_ROWS
    rows = e.row_of() % synth.N_ROWS
    found, first = set(), []
    splits = fakes = 0
    for k in range(meta.shape[0]):
        cl = cl_all[meta[k, 3]:meta[k, 3] + meta[k, 2]]
        lab, c = np.unique(mc[cl], return_counts=True)
        j = int(np.argmax(c))
        if lab[j] < 0 or c[j] < purity * cl.shape[0]:
            fakes += 1
            continue
        if lab[j] in found:
            splits += 1
            continue
        found.add(int(lab[j]))
        c0 = int(cl[0])
        if par[k, 7] > 0 and mc[c0] == lab[j] and \
                par[k, 0] == np.float32(synth.ROW_X[rows[c0]]) and \
                meta[k, 0] == e.sector_id[slot[c0]]:
            first.append((k, c0))
    n_found = len(found & findable)
    out = dict(findable=len(findable), found=n_found,
               efficiency=n_found / max(1, len(findable)), split=splits,
               split_rate=splits / max(1, len(found)), fakes=fakes,
               fake_rate=fakes / max(1, meta.shape[0]), tracks=int(meta.shape[0]),
               mean_clusters=float(np.mean(meta[:, 2])) if meta.shape[0] else 0.0)
    if first:
        k = np.array([a for a, _ in first])
        c0 = np.array([b for _, b in first])
        p = mc[c0]
        q_pt = e.track_q[p] / e.track_pt[p]
        out["resolution"] = dict(
            tracks=int(k.shape[0]),
            y_cm=_w68(par[k, 1] - e.y_true[c0]),
            z_cm=_w68(par[k, 2] - e.z_true[c0]),
            sinphi=_w68(par[k, 3] - _true_sinphi(e, c0, slot[c0])),
            tanl=_w68(par[k, 4] - e.track_tanl[p]),
            qpt_rel=_w68((par[k, 5] - q_pt) / q_pt),
            charge_wrong=float(np.mean(np.sign(par[k, 5]) != np.sign(q_pt))))
    return out
