"""Pins of the oracle's track merger with refit: refits of cluster lists that
span several sectors against the helix truth and the chi^2 law, and joins of
the sector tracks of one particle (across a side edge and across the
membrane) against the Monte-Carlo truth."""
import math

import numpy as np
import pytest

from conftest import event_dict
from paper_1712_09407_amd import quality, synth


def path_order(e, cl):
    """A primary's clusters in path order: increasing radius from the beam."""
    row = e.row_of()[cl] % synth.N_ROWS
    x = synth.ROW_X[row].astype(np.float64)
    return cl[np.argsort(np.hypot(x, e.y_true[cl]), kind="stable")]


def truth_at(e, c):
    """(x, y, z, sinphi, tanl, q/pT) of the particle at cluster c."""
    slot = e.row_of()[[c]] // synth.N_ROWS
    p = e.mc_track[c]
    return np.array([synth.ROW_X[e.row_of()[c] % synth.N_ROWS], e.y_true[c], e.z_true[c],
                     quality._true_sinphi(e, np.array([c]), slot)[0], e.track_tanl[p],
                     e.track_q[p] / e.track_pt[p]])


def crossing(seed, phi_range, sigma=0.0, n=8, pt=1.9, **kw):
    cfg = synth.EventConfig(n_tracks=n, sectors=tuple(range(18)), phi_range_deg=phi_range,
                            sigma=sigma, noise_frac=0.0, pt_min=pt, pt_mean=1e-9, eta_max=0.5,
                            **kw)
    return synth.make_event(cfg, seed)


def test_refit_recovers_noiseless_helices_across_sectors(orc, geo):
    """Lists of a particle's clusters in one or two sectors (path order): the
    refit ends on the truth at the innermost cluster, in its sector's frame;
    a rotation with the wrong sign or a wrong Jacobian misses by far more."""
    n_multi = n_single = 0
    for seed in range(10, 16):
        e = crossing(seed, (16.0, 18.0))
        slot = e.row_of() // synth.N_ROWS
        lists, parts = [], []
        for p in np.unique(e.mc_track[e.mc_track >= 0]):
            cl = path_order(e, np.nonzero(e.mc_track == p)[0])
            if cl.shape[0] < 10:
                continue
            lists.append(cl)
            parts.append(cl)
        par, frame = orc.refit(event_dict(e), geo, e.bz, lists)
        for cl, P, f in zip(parts, par, frame):
            t = truth_at(e, cl[0])
            assert f == e.sector_id[slot[cl[0]]]
            assert np.allclose(P[:5], t[:5], rtol=0, atol=1e-6), (P, t)
            # FP32 cluster storage: y near 40 cm rounds by ~4e-6 cm against a
            # sagitta of ~3 cm, so q/pT is exact to ~1e-6 relative
            assert abs(P[5] / t[5] - 1) < 1e-5
            # clusters are stored in FP32: ~1e-6 cm residuals, chi2 ~1e-8
            assert P[6] < 1e-6 and P[7] == 2 * cl.shape[0] - 5
            multi = np.unique(slot[cl]).shape[0] > 1
            n_multi += multi
            n_single += not multi
    assert n_multi >= 10 and n_single >= 5


def test_refit_chi2_follows_its_ndf_across_sectors(orc, geo):
    """Smeared (sigma = 0.1 cm, the fit's resolution) lists over two sectors:
    chi^2 summed over all lists divided by the summed ndf is 1 within three
    standard deviations of that ratio (sqrt(2 / ndf))."""
    chi2 = ndf = 0.0
    pulls = []
    for seed in range(20, 32):
        e = crossing(seed, (16.0, 18.0), sigma=0.1, n=12)
        slot = e.row_of() // synth.N_ROWS
        lists = []
        for p in np.unique(e.mc_track[e.mc_track >= 0]):
            cl = path_order(e, np.nonzero(e.mc_track == p)[0])
            if cl.shape[0] >= 20 and np.unique(slot[cl]).shape[0] > 1:
                lists.append(cl)
        par, _ = orc.refit(event_dict(e), geo, e.bz, lists)
        for cl, P in zip(lists, par):
            chi2 += P[6]
            ndf += P[7]
            pulls.append((P[5] - truth_at(e, cl[0])[5]))
    assert ndf > 5000
    assert abs(chi2 / ndf - 1) < 3 * math.sqrt(2 / ndf), chi2 / ndf


def _label(e, tr, t):
    m = tr["track_meta"][t]
    v, c = np.unique(e.mc_track[tr["track_cluster"][m[2]:m[2] + m[1]]], return_counts=True)
    return v[np.argmax(c)]


@pytest.mark.parametrize("kind", ["side", "membrane"])
def test_sector_tracks_of_one_particle_are_joined(orc, geo, kind):
    """Noiseless particles with at least 30 clusters on both sides of a
    sector edge (side) or of the central membrane (membrane: tracks nearly
    parallel to it from a vertex close to it) give two sector tracks; the
    merger joins them into one track holding all the particle's clusters, in
    path order, whose refit ends on the truth."""
    joined = 0
    for seed in range(40, 48):
        if kind == "side":
            e = crossing(seed, (16.0, 18.0))
        else:
            cfg = synth.EventConfig(n_tracks=8, sectors=tuple(range(36)),
                                    phi_range_deg=(7.0, 13.0), sigma=0.0, noise_frac=0.0,
                                    pt_min=4.0, pt_mean=1e-9, eta_max=0.012,
                                    vertex_sigma_z=1.0)
            e = synth.make_event(cfg, seed)
        tr, _, mg = orc.track_event_merged(event_dict(e), geo, e.bz)
        slot = e.row_of() // synth.N_ROWS
        for k in range(mg["n"]):
            segs = np.nonzero(mg["track_merged"] == k)[0]
            assert mg["meta"][k, 1] == segs.shape[0]
            labs = {_label(e, tr, t) for t in segs}
            assert len(labs) == 1                                   # one particle
            if segs.shape[0] < 2:
                continue
            joined += 1
            p = labs.pop()
            m = mg["meta"][k]
            cl = mg["cluster"][m[3]:m[3] + m[2]]
            mine = np.nonzero(e.mc_track == p)[0]
            assert set(cl.tolist()) == set(mine.tolist())          # all of them
            assert np.array_equal(cl, path_order(e, cl))           # in path order
            sl = slot[cl]
            if kind == "side":
                assert set(e.sector_id[np.unique(sl)].tolist()) == {0, 1}
            else:
                assert set(e.sector_id[np.unique(sl)].tolist()) == {0, 18}
            t = truth_at(e, cl[0])
            P = mg["par"][k]
            assert np.allclose(P[:5], t[:5], rtol=0, atol=1e-6) and abs(P[5] / t[5] - 1) < 1e-5
    assert joined >= 3


def test_merged_output_partitions_the_tracks(orc, geo):
    e = synth.make_event(synth.EventConfig(n_tracks=1500), 8)
    tr, pr, mg = orc.track_event_merged(event_dict(e), geo, e.bz, n_threads=4)
    nt = tr["n_tracks"]
    tm = mg["track_merged"]
    assert np.all((tm >= 0) & (tm < mg["n"]))                      # every track, once
    assert np.array_equal(np.bincount(tm, minlength=mg["n"]), mg["meta"][:, 1])
    heads = mg["meta"][:, 4]
    assert np.all(np.diff(heads) > 0) and np.array_equal(tm[heads], np.arange(mg["n"]))
    assert np.array_equal(mg["meta"][:, 3], np.concatenate([[0], np.cumsum(mg["meta"][:-1, 2])]))
    # each list: the inner prolongation of its first track (reversed into path
    # order), the tracks' own clusters chain by chain, the outer prolongation
    # of its last track
    pro_of = {(int(t), int(end)): (int(f), int(n)) for t, end, _, n, f in pr["meta"]}
    ct = tr["cluster_track"]
    joined = 0
    for k in range(mg["n"]):
        m = mg["meta"][k]
        cl = mg["cluster"][m[3]:m[3] + m[2]]
        segs = np.nonzero(tm == k)[0]
        own_in_list = cl[np.isin(ct[cl], segs)]
        order = list(dict.fromkeys(ct[own_in_list].tolist()))       # chain order
        assert order[0] == m[4] and sorted(order) == sorted(segs.tolist())
        want = []
        if (order[0], 0) in pro_of:
            f, n = pro_of[(order[0], 0)]
            want += pr["cluster"][f:f + n][::-1].tolist()
        for t in order:
            a = tr["track_meta"][t]
            want += tr["track_cluster"][a[2]:a[2] + a[1]].tolist()
        if (order[-1], 1) in pro_of:
            f, n = pro_of[(order[-1], 1)]
            want += pr["cluster"][f:f + n].tolist()
        assert cl.tolist() == want
        joined += segs.shape[0] > 1
        assert len({_label(e, tr, t) for t in segs}) == 1
    assert joined > 50
    assert np.sum(mg["par"][:, 7] == 0) <= 2                        # refits that failed
    assert mg["n_clusters"] == mg["cluster"].shape[0] and nt == tm.shape[0]


def test_merged_comparison_detects_differences(orc, geo):
    from oracle import concordance
    e = synth.make_event(synth.EventConfig(n_tracks=1500), 8)
    tr, _, mg = orc.track_event_merged(event_dict(e), geo, e.bz, n_threads=4)
    rep = concordance.compare_merged(tr, mg, tr, mg, e.n_clusters)
    assert rep["joins_same_frac"] == 1.0 and rep["cluster_concordance_ab"] == 1.0
    assert rep["identical"] == mg["n"] and rep["par_fail"] == 0
    # B splits the first joined track of two and shifts the q/pT of another
    k = int(np.nonzero(mg["meta"][:, 1] == 2)[0][0])
    b = {key: (v.copy() if hasattr(v, "copy") else v) for key, v in mg.items()}
    segs = np.nonzero(mg["track_merged"] == k)[0]
    b["track_merged"][segs[1]] = mg["n"]                  # a joined track of its own
    m = b["meta"][k].copy()
    first_len = tr["track_meta"][segs[0], 1]
    b["meta"] = np.vstack([b["meta"], [m[0], 1, 0, 0, segs[1]]])
    b["par"] = np.vstack([b["par"], b["par"][k]])
    j = (k + 1) % mg["n"]
    b["par"][j, 5] *= 1.01
    rep = concordance.compare_merged(tr, mg, tr, b, e.n_clusters)
    assert rep["joins_same"] == mg["n"] - 1
    assert rep["par_fail"] == 1 and rep["identical"] == mg["n"]
    assert first_len > 0
