"""Generator pins: reproducibility, geometry, closed-form helix crossings."""
import math

import numpy as np
import pytest

from paper_1712_09407_amd import synth


def test_seed_reproducible_bitwise():
    a = synth.make_preset("c1_sector", 7)
    b = synth.make_preset("c1_sector", 7)
    c = synth.make_preset("c1_sector", 8)
    for k in ("y", "z", "row_offsets", "mc_track"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    assert not np.array_equal(a.y[:100], c.y[:100])


def test_layout_and_ranges():
    e = synth.make_event(synth.EventConfig(n_tracks=300), 3)
    ro = e.row_offsets
    assert ro.dtype == np.int32 and ro[0] == 0 and ro[-1] == e.n_clusters
    assert np.all(np.diff(ro) >= 0)
    assert ro.shape[0] == 36 * 159 + 1
    row = e.row_of()
    r = row % 159
    s = e.sector_id[row // 159]
    x = synth.ROW_X[r].astype(np.float64)
    assert np.all(np.abs(e.y.astype(np.float64)) <= x * float(synth.TAN_HALF))
    assert np.all(np.abs(e.z) <= 250.0)
    assert np.all(e.z[s < 18] >= 0) and np.all(e.z[s >= 18] < 0)


def test_row_geometry():
    # rows evenly spaced from 85 to 247 cm (reading of the lost geometry figure)
    assert synth.ROW_X.shape == (159,)
    assert abs(float(synth.ROW_X[0]) - 85.0) < 1e-5 and abs(float(synth.ROW_X[-1]) - 247.0) < 1e-4
    assert np.allclose(np.diff(synth.ROW_X.astype(np.float64)), 162.0 / 158.0, atol=1e-5)


def test_noiseless_crossings_lie_on_helix():
    cfg = synth.EventConfig(n_tracks=40, sigma=0.0, noise_frac=0.0, ignore_membrane=True)
    e = synth.make_event(cfg, 11)
    row = e.row_of()
    x = synth.ROW_X[row % 159].astype(np.float64)
    alpha = np.array([synth.sector_alpha(int(s)) for s in e.sector_id])[row // 159]
    X = x * np.cos(alpha) - e.y_true * np.sin(alpha)
    Y = x * np.sin(alpha) + e.y_true * np.cos(alpha)
    t = e.mc_track
    R = e.track_pt[t] / (synth.C_LIGHT * 0.5)
    h = np.sign(e.track_q[t] * 0.5)
    phi0 = e.track_phi0[t]
    cx, cy = R * h * np.sin(phi0), -R * h * np.cos(phi0)
    # circle through the origin with the right centre
    assert np.max(np.abs(np.hypot(X - cx, Y - cy) - R) / R) < 1e-12
    # z linear in the transverse arc: arc = R * turning angle
    ang0 = np.arctan2(-cy, -cx)
    ang = np.arctan2(Y - cy, X - cx)
    turn = np.mod(h * (ang0 - ang), 2 * math.pi)
    z = e.track_z0[t] + e.track_tanl[t] * R * turn
    assert np.max(np.abs(z - e.z_true)) < 1e-9
    # the FP32 clusters are the rounded truth when sigma = 0
    assert np.max(np.abs(e.y.astype(np.float64) - e.y_true)) < 1e-4


def test_central_event_size():
    e = synth.make_preset("c2_central", 2)
    n = e.n_clusters
    assert 1.2e6 < n < 1.45e6
    noise = (e.mc_track < 0).sum()
    assert abs(noise / (n - noise) - 0.05) < 0.002


def test_batch_multiplicity_log_uniform():
    m = np.array([synth.batch_multiplicity(3000 + i) for i in range(64)])
    assert m.min() >= 100 and m.max() <= 8000
    assert 100 < np.median(m) < 4000
