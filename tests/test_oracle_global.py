"""Pins of the oracle's global tracking (section 5): the frame rotation
against exact helix geometry, and prolongations of noiseless tracks that
cross a sector edge against the Monte-Carlo truth."""
import math

import numpy as np
import pytest

from conftest import event_dict
from paper_1712_09407_amd import quality, synth

BZ = 0.5
WIDTH = 2 * math.atan(float(synth.TAN_HALF))


def test_rotation_jacobian_matches_exact_helix_geometry(orc):
    """Perturb one state parameter, rotate, and carry the rotated state back to
    the unperturbed rotated reference plane with the exact helix step: the
    change per unit perturbation is the Jacobian's column.  The oracle's
    rotation of a covariance with unit variance in parameter i alone must be
    the outer product of that column with itself."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        x = rng.uniform(90, 240)
        st = np.array([rng.uniform(-0.15, 0.15) * x, rng.uniform(-100, 100),
                       rng.uniform(-0.6, 0.6), rng.uniform(-1, 1), rng.uniform(-4, 4)])
        d = rng.choice([-1.0, 1.0]) * WIDTH
        x1, s1, _ = orc.rotate(x, st, None, d, BZ)
        eps = 1e-6
        for i in range(5):
            sp = st.copy()
            sp[i] += eps
            x2, s2, _ = orc.rotate(x, sp, None, d, BZ)
            cov = np.zeros((5, 5))
            s3, _, _ = orc.propagate(x2, s2, cov, x1, BZ, max_sinphi=0.9999)
            col = (s3 - s1) / eps
            e = np.zeros((5, 5))
            e[i, i] = 1.0
            _, _, ce = orc.rotate(x, st, e, d, BZ)
            assert np.allclose(ce, np.outer(col, col), rtol=1e-5, atol=1e-6), (i, ce, col)


def test_rotation_round_trip_is_the_identity(orc):
    rng = np.random.default_rng(5)
    for _ in range(50):
        x = rng.uniform(90, 240)
        st = np.array([rng.uniform(-0.15, 0.15) * x, rng.uniform(-100, 100),
                       rng.uniform(-0.5, 0.5), rng.uniform(-1, 1), rng.uniform(-4, 4)])
        d = rng.uniform(-0.4, 0.4)
        x1, s1, _ = orc.rotate(x, st, None, d, BZ)
        x2, s2, _ = orc.rotate(x1, s1, None, -d, BZ)
        assert abs(x2 - x) < 1e-9 and np.allclose(s2, st, rtol=0, atol=1e-12)


def _crossing_event(seed, phi_range, n=8, sigma=0.0):
    """Noiseless tracks of pT 1.9 GeV in sector 0 whose negative ones bend
    towards the 20-degree boundary: from 14.5-15.5 degrees they cross it near
    the outer rows (a short outer piece in sector 1), from 17.2-18.2 degrees
    near the inner rows (a short inner piece in sector 0)."""
    cfg = synth.EventConfig(n_tracks=n, sectors=tuple(range(18)), phi_range_deg=phi_range,
                            sigma=sigma, noise_frac=0.0, pt_min=1.9, pt_mean=1e-9,
                            eta_max=0.5)
    return synth.make_event(cfg, seed)


@pytest.mark.parametrize("phi_range,end", [((14.5, 15.5), 1), ((17.2, 18.2), 0)])
def test_prolongations_collect_the_particles_free_clusters(orc, geo, phi_range, end):
    n_prol = 0
    for seed in range(8):
        e = _crossing_event(100 + seed, phi_range)
        slot = e.row_of() // synth.N_ROWS
        tr, pr = orc.track_event_global(event_dict(e), geo, e.bz)
        plain = orc.track_event(event_dict(e), geo, e.bz)
        for k in ("track_par", "track_meta", "track_cluster", "cluster_track"):
            assert np.array_equal(tr[k], plain[k])            # sector tracks unchanged
        mc = e.mc_track
        for k in range(pr["n"]):
            t, e_k, sec, n, first = pr["meta"][k]
            assert e_k == end
            m = tr["track_meta"][t]
            lab = np.bincount(mc[tr["track_cluster"][m[2]:m[2] + m[1]]]).argmax()
            cl = pr["cluster"][first:first + n]
            nslot = int(np.nonzero(e.sector_id == sec)[0][0])
            # the neighbour the particles bend into: same half, index +1 from
            # the outer end (sector 0 -> 1), -1 from the inner end (1 -> 0)
            assert sec == (m[0] // 18) * 18 + (m[0] % 18 + (1 if end else 17)) % 18
            assert np.all(mc[cl] == lab)                       # only its particle
            assert np.all(slot[cl] == nslot)                   # in the sector entered
            free = np.nonzero((mc == lab) & (slot == nslot) & (tr["cluster_track"] < 0))[0]
            assert set(cl.tolist()) == set(free.tolist())      # all of them
            rows = e.row_of()[cl]
            assert np.all(np.diff(rows) == (1 if end else -1))  # in order, away from the track
            # the fit ends on the truth at its last cluster (noiseless clusters)
            c = cl[-1:]
            p = mc[c[0]]
            P = pr["par"][k]
            assert P[0] == pytest.approx(float(synth.ROW_X[rows[-1] % synth.N_ROWS]), abs=1e-9)
            assert abs(P[1] - e.y_true[c[0]]) < 1e-4 and abs(P[2] - e.z_true[c[0]]) < 1e-4
            assert abs(P[3] - quality._true_sinphi(e, c, slot[c])[0]) < 1e-4
            assert abs(P[4] - e.track_tanl[p]) < 1e-4
            assert abs(P[5] * e.track_pt[p] / e.track_q[p] - 1) < 1e-3
            assert P[7] == 2 * n and P[6] < 1e-6
            n_prol += 1
    assert n_prol >= 6


def test_no_prolongation_without_a_neighbour(orc, geo):
    e = synth.make_preset("c1_sector", 1)   # one sector slot only
    tr, pr = orc.track_event_global(event_dict(e), geo, e.bz)
    assert tr["n_tracks"] > 50 and pr["n"] == 0


def test_prolonged_clusters_are_free_and_unique(orc, geo):
    e = synth.make_event(synth.EventConfig(n_tracks=1500), 8)
    tr, pr = orc.track_event_global(event_dict(e), geo, e.bz, n_threads=4)
    assert pr["n"] > 20
    cl = pr["cluster"]
    assert np.unique(cl).shape[0] == cl.shape[0]             # each cluster once
    assert np.all(tr["cluster_track"][cl] < 0)               # never a sector track's
    meta = pr["meta"]
    order = meta[:, 0] * 2 + meta[:, 1]
    assert np.all(np.diff(order) > 0)                        # (track, end) order
    assert np.array_equal(meta[:, 4], np.concatenate([[0], np.cumsum(meta[:-1, 3])]))
    def label(cl):
        v, c = np.unique(e.mc_track[cl], return_counts=True)
        return v[np.argmax(c)]

    tm, tc = tr["track_meta"], tr["track_cluster"]
    purity = np.mean([np.all(e.mc_track[cl[f:f + n]] == label(tc[tm[t, 2]:tm[t, 2] + tm[t, 1]]))
                      for t, _, _, n, f in meta])
    assert purity > 0.9


def test_prolongation_comparison_detects_differences(orc, geo):
    from oracle import concordance
    e = synth.make_event(synth.EventConfig(n_tracks=1500), 8)
    tr, pr = orc.track_event_global(event_dict(e), geo, e.bz, n_threads=4)
    rep = concordance.compare_prolongations(tr, pr, tr, pr, e.n_clusters)
    assert rep["cluster_concordance_ab"] == rep["cluster_concordance_ba"] == 1.0
    assert rep["identical"] == rep["n_a"] == pr["n"] == rep["par_compared"]
    assert rep["par_fail"] == 0 and rep["other_seed"] == 0
    # B loses the last cluster of its first prolongation and shifts another's q/pT
    b = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in pr.items()}
    m = b["meta"]
    keep = np.ones(b["cluster"].shape[0], bool)
    keep[m[0, 4] + m[0, 3] - 1] = False
    b["cluster"] = b["cluster"][keep]
    m[0, 3] -= 1
    m[1:, 4] -= 1
    b["n_clusters"] -= 1
    b["par"][1, 5] *= 1.01
    rep = concordance.compare_prolongations(tr, pr, tr, b, e.n_clusters)
    assert rep["cluster_concordance_ab"] == pytest.approx(1 - 1 / pr["n_clusters"])
    assert rep["cluster_concordance_ba"] == 1.0
    assert rep["identical"] == pr["n"] - 1 and rep["par_fail"] == 1
