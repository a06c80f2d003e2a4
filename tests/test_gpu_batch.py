"""Batched path: every event of a batch gets exactly the tracks it gets alone."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1712_09407_amd import synth, tpc  # noqa: E402

KEYS = ("track_par", "track_meta", "track_cluster", "cluster_track")


def say(*a):
    print("[gpu-batch]", *a, flush=True)


@pytest.fixture(scope="module")
def tracker():
    t = tpc.Tracker(0)
    yield t
    t.close()


@pytest.fixture(scope="module")
def geo():
    return tpc.make_geometry(synth.ROW_X, synth.TAN_HALF, synth.Z_MAX)


@pytest.fixture(scope="module")
def events():
    evs = []
    for i, n in enumerate([300, 2500, 100, 6000, 900]):
        evs.append(synth.make_event(synth.EventConfig(n_tracks=n), 3000 + i))
    evs.append(synth.make_preset("c1_sector", 7))                       # one sector slot
    evs.append(synth.make_event(synth.EventConfig(n_tracks=0, noise_frac=0.0), 9))  # empty
    say("clusters", [e.n_clusters for e in evs])
    return evs


def dev(e):
    return tpc.DeviceEvent.from_host(e.y, e.z, e.row_offsets, e.sector_id)


def test_batch_equals_events_alone(tracker, geo, events):
    devs = [dev(e) for e in events]
    batch = [tpc.to_numpy(r) for r in tracker.track_batch(devs, geo, 0.5)]
    for e, d, b in zip(events, devs, batch):
        alone = tpc.to_numpy(tracker.track_event(d, geo, 0.5))
        assert b["n_tracks"] == alone["n_tracks"]
        for k in KEYS:
            assert np.array_equal(b[k], alone[k]), k
    assert sum(b["n_tracks"] for b in batch) > 1000


def test_batch_order_does_not_matter(tracker, geo, events):
    devs = [dev(e) for e in events]
    fwd = [tpc.to_numpy(r) for r in tracker.track_batch(devs, geo, 0.5)]
    rev = [tpc.to_numpy(r) for r in tracker.track_batch(devs[::-1], geo, 0.5)][::-1]
    for a, b in zip(fwd, rev):
        for k in KEYS:
            assert np.array_equal(a[k], b[k]), k


def test_batch_rejects_one_bad_event(tracker, geo, events):
    e = events[1]
    ro = e.row_offsets.copy()
    ro[5] = ro[6] + 1
    bad = tpc.DeviceEvent.from_host(e.y, e.z, ro, e.sector_id)
    with pytest.raises(tpc.TpcError) as ex:
        tracker.track_batch([dev(events[0]), bad], geo, 0.5)
    assert ex.value.code == tpc.TPC_ERR_INVALID_ARG
    # the context keeps working
    assert tracker.track_batch([dev(events[0])], geo, 0.5)[0]["n_tracks"] > 0


def test_batch_capacity_is_per_event(tracker, geo, events):
    devs = [dev(events[0]), dev(events[1])]
    full = tracker.track_batch(devs, geo, 0.5)
    outs = []
    for i, d in enumerate(devs):
        n = d.n_clusters
        ct = 2 if i == 1 else max(16, n // 30 + 1)
        outs.append(dict(track_par=torch.empty((ct, 8), device="cuda"),
                         track_meta=torch.empty((ct, 4), dtype=torch.int32, device="cuda"),
                         track_cluster=torch.empty(n, dtype=torch.int32, device="cuda"),
                         cluster_track=torch.empty(n, dtype=torch.int32, device="cuda")))
    with pytest.raises(tpc.TpcError) as ex:
        tracker.track_batch(devs, geo, 0.5, outs=outs)
    assert ex.value.code == tpc.TPC_ERR_CAPACITY
    assert full[1]["n_tracks"] > 2


def test_graph_replays_match_eager(tracker, geo, events):
    devs = [dev(e) for e in events[:5]]
    tracker.set_tuning(use_graph=0)
    eager = [tpc.to_numpy(r) for r in tracker.track_batch(devs, geo, 0.5)]
    tracker.set_tuning(use_graph=1)
    n0 = tracker.graph_launches()
    for rep in range(4):
        got = [tpc.to_numpy(r) for r in tracker.track_batch(devs, geo, 0.5)]
        for a, b in zip(eager, got):
            for k in KEYS:
                assert np.array_equal(a[k], b[k]), (rep, k)
        # eager work and a synchronisation between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        tracker.track_event(devs[0], geo, 0.5)
    assert tracker.graph_launches() >= n0 + 4
    # a different batch of the same shape replays the same graph
    other = [dev(synth.make_event(synth.EventConfig(n_tracks=n), 4000 + i))
             for i, n in enumerate([500, 200, 3000, 150, 700])]
    g = [tpc.to_numpy(r) for r in tracker.track_batch(other, geo, 0.5)]
    tracker.set_tuning(use_graph=0)
    e2 = [tpc.to_numpy(r) for r in tracker.track_batch(other, geo, 0.5)]
    for a, b in zip(g, e2):
        for k in KEYS:
            assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("blocks,occ,sched,lanes,nf,own", [
    (0, 1.0, 0, 64, 0, 0), (0, 1.0, 1, 64, 0, 0), (64, 1.0, 0, 64, 0, 0), (64, 1.0, 1, 64, 0, 0),
    (7, 1.0, 0, 64, 0, 0), (512, 2.0, 1, 64, 0, 0), (0, 1.5, 0, 64, 0, 0), (2048, 4.0, 0, 64, 0, 0),
    (2048, 4.0, 1, 64, 0, 0), (0, 1.0, 0, 16, 0, 0), (0, 1.0, 0, 1, 0, 0), (40, 1.0, 0, 8, 0, 0),
    (0, 1.0, 0, 0, 1, 0), (0, 1.0, 0, 0, 2, 0), (0, 2.0, 1, 64, 2, 0), (0, 1.0, 0, 0, 3, 0),
    (0, 2.0, 1, 64, 3, 0), (0, 1.0, 0, 0, 0, 1), (0, 1.0, 0, 0, 0, 2), (0, 2.0, 1, 64, 2, 2)])
def test_tuning_never_changes_results(tracker, geo, events, blocks, occ, sched, lanes, nf, own):
    devs = [dev(e) for e in events[:4]]
    tracker.set_tuning(use_graph=0, construct_schedule=0)
    ref = [tpc.to_numpy(r) for r in tracker.track_batch(devs, geo, 0.5)]
    tracker.set_tuning(use_graph=1, construct_blocks=blocks, bin_occupancy=occ,
                       construct_schedule=sched, construct_lanes=lanes, nf_stage=nf,
                       own_order=own)
    got = [tpc.to_numpy(r) for r in tracker.track_batch(devs, geo, 0.5)]
    tracker.set_tuning()
    for a, b in zip(ref, got):
        for k in KEYS:
            assert np.array_equal(a[k], b[k]), k


def test_autotuner_picks_a_candidate(tracker, geo, events, tmp_path, monkeypatch):
    from paper_1712_09407_amd import tune
    monkeypatch.setenv("TPC_TUNE_CACHE", str(tmp_path / "tune.json"))
    devs = [dev(e) for e in events[:4]]
    rec = tune.autotune(tracker, devs, geo, 0.5, reps=1,
                        candidates=[dict(construct_blocks=0, bin_occupancy=1.0),
                                    dict(construct_blocks=256, bin_occupancy=2.0)])
    assert rec["best"] in [c["setting"] for c in rec["tried"]]
    assert tune.load("gpu", devs)["best"] == rec["best"]
    tracker.set_tuning()


def test_tuning_rejects_out_of_range_settings(tracker):
    with pytest.raises(tpc.TpcError):
        tracker.set_tuning(bin_occupancy=0.5)
    with pytest.raises(tpc.TpcError):
        tracker.set_tuning(construct_schedule=2)
    with pytest.raises(tpc.TpcError):
        tracker.set_tuning(construct_lanes=65)
    with pytest.raises(tpc.TpcError):
        tracker.set_tuning(nf_stage=4)
    with pytest.raises(tpc.TpcError):
        tracker.set_tuning(own_order=3)
    tracker.set_tuning()
