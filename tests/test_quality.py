"""The quality report (efficiency, clones, fakes, resolution against MC
truth) on hand-made outputs whose answers are known, and on the oracle."""
import numpy as np
import pytest

from conftest import event_dict
from paper_1712_09407_amd import quality, synth


def truth_tracks(e, min_clusters=30):
    """One perfect track per findable sector segment: the particle's clusters
    in row order and its true parameters at the innermost of them."""
    slot = e.row_of() // synth.N_ROWS
    par, meta, tcl = [], [], []
    for p in np.unique(e.mc_track[e.mc_track >= 0]):
        for s in np.unique(slot[e.mc_track == p]):
            cl = np.nonzero((e.mc_track == p) & (slot == s))[0]
            if cl.shape[0] < min_clusters:
                continue
            cl = cl[np.argsort(e.row_of()[cl], kind="stable")]
            c0 = cl[:1]
            sp = quality._true_sinphi(e, c0, slot[c0])[0]
            row = e.row_of()[c0[0]] % synth.N_ROWS
            par.append([synth.ROW_X[row], e.y_true[c0[0]], e.z_true[c0[0]], sp, e.track_tanl[p],
                        e.track_q[p] / e.track_pt[p], 0.0, 1.0])
            meta.append([int(e.sector_id[s]), cl.shape[0], len(tcl), 0])
            tcl.extend(cl.tolist())
    return dict(n_tracks=len(par), track_par=np.array(par), track_meta=np.array(meta, np.int32),
                track_cluster=np.array(tcl, np.int32))


@pytest.fixture(scope="module")
def event():
    return synth.make_event(synth.EventConfig(n_tracks=300), 21)


def test_perfect_tracks_score_perfectly(event):
    res = truth_tracks(event)
    q = quality.evaluate(event, res)
    assert q["findable"] == res["n_tracks"] > 100
    assert q["efficiency"] == 1.0 and q["clones"] == 0 and q["fakes"] == 0
    r = q["resolution"]
    for k in ("y_cm", "z_cm", "sinphi", "tanl", "qpt_rel"):
        assert abs(r[k]) < 1e-9, k
    assert r["charge_wrong"] == 0.0


def test_a_copy_is_a_clone_and_noise_is_a_fake(event):
    res = truth_tracks(event)
    n = res["n_tracks"]
    # append a copy of track 0 and a track made of noise clusters
    m0 = res["track_meta"][0]
    cl0 = res["track_cluster"][m0[2]:m0[2] + m0[1]]
    noise = np.nonzero(event.mc_track < 0)[0][:40]
    tcl = np.concatenate([res["track_cluster"], cl0, noise])
    meta = np.vstack([res["track_meta"], [m0[0], m0[1], len(res["track_cluster"]), 0],
                      [0, 40, len(res["track_cluster"]) + m0[1], 0]]).astype(np.int32)
    par = np.vstack([res["track_par"], res["track_par"][0], res["track_par"][0]])
    q = quality.evaluate(event, dict(n_tracks=n + 2, track_par=par, track_meta=meta,
                                     track_cluster=tcl))
    assert q["clones"] == 1 and q["fakes"] == 1 and q["efficiency"] == 1.0
    assert q["fake_rate"] == pytest.approx(1 / (n + 2))


def test_true_direction_matches_a_noiseless_fit(orc, geo):
    """The helix geometry of the truth (direction at a crossing) agrees with
    the oracle's fit of a noiseless track, which recovers it exactly."""
    cfg = synth.EventConfig(n_tracks=1, sectors=(0,), phi_range_deg=(0.0, 20.0),
                            ignore_membrane=True, sigma=0.0, noise_frac=0.0, pt_min=0.35,
                            pt_mean=0.2)
    checked, big = 0, 0
    for seed in range(50, 70):
        e = synth.make_event(cfg, seed)
        res = orc.track_event(event_dict(e), geo, e.bz)
        if res["n_tracks"] != 1:
            continue
        checked += 1
        q = quality.evaluate(e, res)
        r = q["resolution"]
        assert r["sinphi"] < 1e-6 and r["qpt_rel"] < 1e-6 and r["tanl"] < 1e-6
        assert r["charge_wrong"] == 0.0
        big += abs(res["track_par"][0, 3]) > 0.1   # directions well away from radial
    assert checked >= 5 and big >= 2


def test_oracle_quality_on_one_sector(orc, geo):
    e = synth.make_preset("c1_sector", 1)
    q = quality.evaluate(e, orc.track_event(event_dict(e), geo, e.bz))
    assert q["efficiency"] > 0.95 and q["fake_rate"] < 0.02 and q["clone_rate"] < 0.02
    r = q["resolution"]
    assert 0.02 < r["y_cm"] < 0.2 and r["charge_wrong"] < 0.01


def test_merge_sums_counts():
    a = dict(findable=10, found=9, clones=1, fakes=0, tracks=10,
             resolution=dict(tracks=9, y_cm=0.1, z_cm=0.1, sinphi=0.01, tanl=0.01, qpt_rel=0.02,
                             charge_wrong=0.0))
    b = dict(findable=30, found=27, clones=0, fakes=3, tracks=30,
             resolution=dict(tracks=27, y_cm=0.2, z_cm=0.1, sinphi=0.01, tanl=0.01, qpt_rel=0.02,
                             charge_wrong=0.0))
    m = quality.merge([a, b])
    assert m["efficiency"] == 36 / 40 and m["fake_rate"] == 3 / 40
    assert m["resolution"]["y_cm"] == pytest.approx((0.9 + 5.4) / 36)


def test_alpha_infinity_is_the_longest_track_rule():
    a = np.float32(quality.alpha_value(float("inf")))
    for n in (30, 100, 159):
        for chi in (0.5, 1.0, 5.0, 30.0):
            w = np.float32(n) * (a - np.float32(chi))
            assert w == np.float32(n) * a     # the fit quality no longer counts
    assert np.float32(31) * a > np.float32(30) * a


def test_prolongation_report_on_known_answers(event):
    """Perfect sector tracks plus prolongations that carry exactly the short
    pieces of their particles recover all of them at purity 1; no
    prolongations recover none; a prolongation of another particle's clusters
    has purity 0."""
    res = truth_tracks(event)
    slot = event.row_of() // synth.N_ROWS
    mc = event.mc_track
    lab = {int(mc[res["track_cluster"][m[2]]]): t for t, m in enumerate(res["track_meta"])}
    meta, cl = [], []
    for p, t in sorted(lab.items()):
        for s in np.unique(slot[mc == p]):
            c = np.nonzero((mc == p) & (slot == s))[0]
            if c.shape[0] < 30:
                meta.append([t, 1, int(event.sector_id[s]), c.shape[0], len(cl)])
                cl.extend(c.tolist())
    order = np.argsort([m[0] * 2 + m[1] for m in meta], kind="stable")
    pro = dict(n=len(meta), meta=np.array(meta, np.int32)[order], cluster=np.array(cl, np.int32))
    # re-base the offsets after sorting
    pro["meta"][:, 4] = np.concatenate([[0], np.cumsum(pro["meta"][:-1, 3])])
    pro["cluster"] = np.concatenate([np.array(cl, np.int32)[m[4]:m[4] + m[3]]
                                     for m in np.array(meta, np.int32)[order]])
    r = quality.prolongation_report(event, res, pro)
    assert r["short_piece_clusters"] == len(cl) > 20
    assert r["short_piece_recovered"] == 1.0 and r["prolongation_purity"] == 1.0
    none = dict(n=0, meta=np.zeros((0, 5), np.int32), cluster=np.zeros(0, np.int32))
    assert quality.prolongation_report(event, res, none)["short_piece_recovered"] == 0.0
    # attach track 0's prolongation to track 1 instead: wrong particle
    wrong = dict(pro)
    wrong["meta"] = pro["meta"].copy()
    wrong["meta"][:, 0] = (pro["meta"][:, 0] + 1) % res["n_tracks"]
    r = quality.prolongation_report(event, res, wrong)
    assert r["prolongation_purity"] == 0.0 and r["short_piece_recovered"] == 0.0


def test_merged_report_on_known_answers(event):
    """One perfect joined track per particle (its clusters in path order, the
    truth at the first one): efficiency 1, no splits or fakes, zero
    resolution; a copy of one is a split track, a list of noise a fake."""
    slot = event.row_of() // synth.N_ROWS
    rows = event.row_of() % synth.N_ROWS
    mc = event.mc_track
    par, meta, cl = [], [], []
    for p in np.unique(mc[mc >= 0]):
        c = np.nonzero(mc == p)[0]
        if c.shape[0] < 30:
            continue
        x = synth.ROW_X[rows[c]].astype(np.float64)
        c = c[np.argsort(np.hypot(x, event.y_true[c]), kind="stable")]
        c0 = c[:1]
        par.append([synth.ROW_X[rows[c0[0]]], event.y_true[c0[0]], event.z_true[c0[0]],
                    quality._true_sinphi(event, c0, slot[c0])[0], event.track_tanl[p],
                    event.track_q[p] / event.track_pt[p], 0.0, 2.0 * c.shape[0] - 5])
        meta.append([int(event.sector_id[slot[c0[0]]]), 1, c.shape[0], len(cl), 0])
        cl.extend(c.tolist())
    m = dict(par=np.array(par), meta=np.array(meta, np.int32), cluster=np.array(cl, np.int32))
    r = quality.merged_report(event, m)
    assert r["efficiency"] == 1.0 and r["split"] == 0 and r["fakes"] == 0
    assert r["resolution"]["tracks"] == len(par) > 100
    for k in ("y_cm", "z_cm", "sinphi", "tanl", "qpt_rel"):
        assert abs(r["resolution"][k]) < 1e-9, k
    noise = np.nonzero(mc < 0)[0][:40]
    m2 = dict(par=np.vstack([m["par"], m["par"][:1], m["par"][:1]]),
              meta=np.vstack([m["meta"], [m["meta"][0, 0], 1, m["meta"][0, 2], len(cl), 0],
                              [0, 1, 40, len(cl) + m["meta"][0, 2], 0]]).astype(np.int32),
              cluster=np.concatenate([m["cluster"], m["cluster"][:m["meta"][0, 2]], noise]))
    r = quality.merged_report(event, m2)
    assert r["split"] == 1 and r["fakes"] == 1 and r["efficiency"] == 1.0


def test_global_tracking_keeps_efficiency_and_improves_resolution(orc, geo):
    """Section 5: with global tracking the joined tracks are found as before
    (efficiency, splits and fakes within 1e-3: a short track that gains a few
    clusters of another particle can fall below the 90% purity of a found
    track) and, holding more clusters, are measured better (q/pT and
    sin(phi) resolution)."""
    e = synth.make_event(synth.EventConfig(n_tracks=3000), 31)
    ev = event_dict(e)
    _, _, with_g = orc.track_event_merged(ev, geo, e.bz, n_threads=4)
    _, _, without = orc.track_event_merged(ev, geo, e.bz, use_global=False, n_threads=4)
    a, b = quality.merged_report(e, without), quality.merged_report(e, with_g)
    assert a["efficiency"] > 0.99 and abs(b["efficiency"] - a["efficiency"]) <= 1e-3
    assert abs(b["split_rate"] - a["split_rate"]) <= 1e-3
    assert abs(b["fake_rate"] - a["fake_rate"]) <= 1e-3
    assert b["mean_clusters"] > a["mean_clusters"] + 2
    assert b["resolution"]["qpt_rel"] < a["resolution"]["qpt_rel"]
    assert b["resolution"]["sinphi"] < a["resolution"]["sinphi"]
