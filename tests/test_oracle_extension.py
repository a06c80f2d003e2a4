"""Known-answer pins of the oracle's extension rule (section 1: clusters
that meet a chi^2 condition are collected row by row, repeated until no
more are found; the readings: the chi^2 gate on S = H C H^T + V, a stop
after more than max_miss consecutive rows without a cluster, a prediction
outside the trapezoid counted as a miss and not a stop, the smallest
(chi^2, index) among the candidates).

Each case is one tracklet built by the oracle's construction from a chain
given explicitly (the links up2 and the seed), on clusters placed exactly on
a particle's trajectory (tests/helix.py, independent of the tracker), so
that the expected clusters are known row by row.  A one-line mistake in the
rule (max_miss off by one, a gate without V, an outside prediction treated
as a stop, the larger of two equal candidates) fails one of them.
"""
import math

import numpy as np
import pytest

from helix import at_x

SECTOR_ROWS = 159


def geometry():
    from paper_1712_09407_amd import synth
    return synth.ROW_X, synth.TAN_HALF, synth.Z_MAX


def one_sector_event(rows_yz):
    """rows_yz: {row: [(y, z), ...]} -> event dict (one sector slot, clusters
    in row order, FP32) and the cluster index of each (row, k)."""
    ys, zs, ro, index = [], [], [0], {}
    for r in range(SECTOR_ROWS):
        for k, (y, z) in enumerate(rows_yz.get(r, [])):
            index[(r, k)] = len(ys)
            ys.append(y)
            zs.append(z)
        ro.append(len(ys))
    ev = dict(y=np.array(ys, np.float32), z=np.array(zs, np.float32),
              row_offsets=np.array(ro, np.int32), sector_id=np.array([0], np.int32))
    return ev, index


def build(orc, ev, chain, bz, params=None):
    """The oracle's tracklet of the chain (list of cluster indices, one per
    consecutive row, linked outward)."""
    n = ev["y"].shape[0]
    up2 = np.full(n, -1, np.int32)
    for a, b in zip(chain[:-1], chain[1:]):
        up2[a] = b
    tl = orc.construct(ev, geometry(), bz, up2, np.array([chain[0]], np.int32),
                       params or orc.default_params())
    return {k: v[0] for k, v in tl.items()}


def collected_rows(tl):
    h = tl["hits"]
    return [r for r in range(tl["row_lo"], tl["row_hi"] + 1) if h[r] >= 0]


def helix_rows(st, rows, bz=0.5, x0_row=10):
    X = geometry()[0].astype(np.float64)
    out = {}
    for r in rows:
        s = at_x(X[x0_row], st, X[r], bz)
        out[r] = [(s[0], s[1])]
    return out


# a particle of pT 2 GeV: every crossing well inside the sector
ST = (2.0, 30.0, 0.05, 0.3, 0.5)


@pytest.mark.parametrize("gap,bridged", [(10, True), (11, False)])
def test_gap_of_max_miss_rows_is_bridged_and_one_more_stops(orc, gap, bridged):
    """Rows 10-19 are the chain, rows 20-59 and 60+gap-140 hold the
    particle's clusters: a gap of max_miss (10) empty rows is bridged, one
    of 11 ends the extension."""
    assert orc.default_params().max_miss == 10
    rows = [r for r in range(10, 141) if not 60 <= r < 60 + gap]
    ev, idx = one_sector_event(helix_rows(ST, rows))
    chain = [idx[(r, 0)] for r in range(10, 20)]
    got = collected_rows(build(orc, ev, chain, 0.5))
    want = rows if bridged else [r for r in rows if r < 60]
    assert got == want


def test_chain_cut_short_is_completed_by_the_gated_extension(orc):
    """Only rows 10-12 are linked (a chain of three): the extension, not the
    chain, collects rows 13-140, and the fit is the particle's."""
    rows = list(range(10, 141))
    ev, idx = one_sector_event(helix_rows(ST, rows))
    tl = build(orc, ev, [idx[(r, 0)] for r in (10, 11, 12)], 0.5)
    assert collected_rows(tl) == rows
    assert tl["n"] == len(rows) and tl["ndf"] == 2 * len(rows) - 5
    X = geometry()[0].astype(np.float64)
    truth = at_x(X[10], ST, X[10], 0.5)
    assert np.allclose(tl["par"][1:], truth, rtol=1e-5, atol=2e-5)


def s00_of_straight_fit(x_rows, x_pred, sigma2, prior_sinphi):
    """Predicted variance of y at x_pred (plus the measurement's) for a
    straight track with sin phi = 0 in a field-free sector: the filter is
    then exactly linear in (y, sin phi), y(x) = y_pred + s (x - x_pred), with
    the first cluster as the initial y (variance sigma^2), a prior of
    variance prior_sinphi on s, and each later cluster a measurement of
    variance sigma^2.  Closed form: the inverse of the information matrix."""
    info = np.zeros((2, 2))
    for x in x_rows:
        h = np.array([1.0, x - x_pred])
        info += np.outer(h, h) / sigma2
    info[1, 1] += 1.0 / prior_sinphi
    return np.linalg.inv(info)[0, 0] + sigma2


@pytest.mark.parametrize("side", [-1, +1])
def test_chi2_gate_on_both_sides_of_its_edge(orc, side):
    """A straight track at y = 0, z = 50 (B = 0) on rows 10-59, and on row 60
    one candidate at y = d with d^2 / S00 = gate (1 -/+ 1e-5), S = H C H^T + V
    in closed form: collected below the gate, not above it."""
    prm = orc.default_params()
    X = geometry()[0].astype(np.float64)
    rows = list(range(10, 60))
    s00 = s00_of_straight_fit(X[rows], X[60], prm.sigma_y ** 2, prm.prior_sinphi)
    d = np.float32(math.sqrt(prm.chi2_gate * s00 * (1.0 + side * 1e-5)))
    chi2 = float(d) ** 2 / s00
    assert (chi2 < prm.chi2_gate) == (side < 0)
    rows_yz = {r: [(0.0, 50.0)] for r in rows}
    rows_yz[60] = [(d, 50.0)]
    ev, idx = one_sector_event(rows_yz)
    tl = build(orc, ev, [idx[(r, 0)] for r in range(10, 20)], 0.0)
    want = rows + [60] if side < 0 else rows
    assert collected_rows(tl) == want


def test_equal_chi2_candidates_take_the_smaller_index(orc):
    """Two candidates at y = +d and y = -d around a straight track at y = 0
    have the same chi^2: the one with the smaller cluster index is taken,
    whichever side it is on."""
    rows = list(range(10, 60))
    for first in (+1, -1):
        rows_yz = {r: [(0.0, 50.0)] for r in rows}
        rows_yz[60] = [(first * 0.05, 50.0), (-first * 0.05, 50.0)]
        ev, idx = one_sector_event(rows_yz)
        tl = build(orc, ev, [idx[(r, 0)] for r in range(10, 20)], 0.0)
        assert tl["hits"][60] == idx[(60, 0)]


def test_prediction_outside_the_sector_is_a_miss_not_a_stop(orc):
    """A low-pT particle near the sector edge: inside on rows 10-20, outside
    (|y| > x tan(10 deg)) on rows 21-28, inside again from row 29.  The eight
    rows outside are misses (fewer than max_miss), so the extension goes on
    and collects the clusters after the particle comes back."""
    X, tan_half, _ = geometry()
    X = X.astype(np.float64)
    x0 = X[10]
    st = (x0 * float(tan_half) - 0.4, 10.0, math.sin(math.radians(13.25)), 0.2, 2.5)
    inside, margin = {}, np.inf
    for r in range(10, 80):
        s = at_x(x0, st, X[r], 0.5)
        edge = X[r] * float(tan_half)
        inside[r] = abs(s[0]) <= edge
        margin = min(margin, abs(abs(s[0]) - edge))
    assert margin > 1e-3                      # no decision within rounding of the edge
    outside = [r for r in inside if not inside[r]]
    assert outside == list(range(21, 29))
    rows = [r for r in range(10, 80) if inside[r]]
    ev, idx = one_sector_event(helix_rows(st, rows))
    tl = build(orc, ev, [idx[(r, 0)] for r in range(10, 16)], 0.5)
    assert collected_rows(tl) == rows
