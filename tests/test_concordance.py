"""The concordance comparator (section 3.3 metric) on hand-made outputs."""
import numpy as np
import pytest

from oracle import concordance


def make(tracks, n_clusters, seeds=None):
    par, meta, tcl = [], [], []
    ctr = np.full(n_clusters, -1, np.int32)
    for i, cl in enumerate(tracks):
        meta.append([0, len(cl), len(tcl), seeds[i] if seeds else cl[0]])
        par.append([85.0, 1.0, 2.0, 0.1, 0.2, 0.5, 60.0, 55.0])
        for c in cl:
            ctr[c] = i
        tcl.extend(cl)
    return dict(track_par=np.array(par, np.float64).reshape(-1, 8),
                track_meta=np.array(meta, np.int32).reshape(-1, 4),
                track_cluster=np.array(tcl, np.int32), cluster_track=ctr)


T = [list(range(0, 40)), list(range(40, 75)), list(range(75, 110))]
N = 120


def test_identical_outputs_are_fully_concordant():
    r = concordance.compare(make(T, N), make(T, N), N)
    assert r["cluster_concordance"] == 1.0 and r["track_concordance"] == 1.0
    assert r["par_compared"] == 3 and r["par_fail"] == 0


def test_one_missing_cluster():
    b = [T[0][:-1], T[1], T[2]]
    r = concordance.compare(make(T, N), make(b, N), N)
    tot = sum(len(t) for t in T)
    assert r["cluster_concordance_ab"] == pytest.approx((tot - 1) / tot)
    assert r["par_compared"] == 2


def test_track_order_does_not_matter():
    a = make(T, N)
    b = make(T[::-1], N, seeds=[t[0] for t in T[::-1]])
    r = concordance.compare(a, b, N)
    assert r["cluster_concordance"] == 1.0 and r["matched"] == 3


def test_missing_track_counts_all_its_clusters():
    r = concordance.compare(make(T, N), make(T[:2], N), N)
    tot = sum(len(t) for t in T)
    assert r["cluster_concordance_ab"] == pytest.approx((tot - len(T[2])) / tot)
    assert r["cluster_concordance_ba"] == 1.0
    assert r["track_concordance_ab"] == pytest.approx(2 / 3)


def test_extra_track_counts_in_reverse_direction():
    extra = T + [list(range(110, 120))]
    r = concordance.compare(make(T, N), make(extra, N), N)
    assert r["cluster_concordance_ab"] == 1.0
    assert r["cluster_concordance_ba"] == pytest.approx(110 / 120)


def test_split_track_matches_the_larger_half_only():
    b = [T[0][:25], T[0][25:], T[1], T[2]]
    r = concordance.compare(make(T, N), make(b, N), N)
    assert r["matched"] == 3
    tot = sum(len(t) for t in T)
    assert r["cluster_concordance_ab"] == pytest.approx((tot - 15) / tot)


def test_parameter_tolerance():
    a, b = make(T, N), make(T, N)
    b["track_par"][1, 5] *= 1 + 5e-3
    r = concordance.compare(a, b, N)
    assert r["par_fail"] == 1 and r["par_max_rel"] == pytest.approx(5e-3, rel=1e-6)
