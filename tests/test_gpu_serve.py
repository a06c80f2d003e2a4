"""Serving loop: continuous batching, admission by footprint; every event's
tracks are the same alone and in the mix."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1712_09407_amd import serve, synth, tpc  # noqa: E402

KEYS = ("track_par", "track_meta", "track_cluster", "cluster_track")


def say(*a):
    print("[gpu-serve]", *a, flush=True)


@pytest.fixture(scope="module")
def geo():
    return tpc.make_geometry(synth.ROW_X, synth.TAN_HALF, synth.Z_MAX)


@pytest.fixture(scope="module")
def pool():
    evs = [synth.make_event(synth.EventConfig(n_tracks=n), 4000 + i)
           for i, n in enumerate([150, 1200, 400, 3000, 100, 800, 2000, 250])]
    return [tpc.HostEvent(e.y, e.z, e.row_offsets, e.sector_id) for e in evs]


@pytest.fixture(scope="module")
def alone(geo, pool):
    tr = tpc.Tracker(0)
    out = []
    for h in pool:
        d = tpc.DeviceEvent.from_host(h.y, h.z, h.row_offsets, h.sector_id)
        out.append(tpc.to_numpy(tr.track_event(d, geo, 0.5)))
    tr.close()
    return out


def _check_same(fetched, pool, alone):
    for k, r in fetched.items():
        ref = alone[k % len(pool)]
        assert r["n_tracks"] == ref["n_tracks"]
        for key in KEYS:
            assert np.array_equal(r[key], ref[key]), (k, key)


def test_mix_equals_alone(geo, pool, alone):
    srv = tpc.Server(geo, 0.5, max_batch=8, n_workers=2)
    res, fetched = serve.run(srv, pool, rate_hz=2000.0, n_events=40, keep=set(range(40)))
    say(res)
    assert res["stats"]["batches"] < 40          # events were batched together
    _check_same(fetched, pool, alone)
    srv.close()


def _footprint(h):
    # the server's admission footprint of an event (160 B per cluster, plus
    # 16 B per row slot and 64 KiB)
    return 160 * h.n_clusters + 16 * 36 * 159 + (1 << 16)


def test_admission_by_footprint_defers_not_fails(geo, pool, alone):
    """A budget that holds one copy of the largest event: a second copy
    submitted right after the first is deferred (BUSY), not failed, and is
    admitted once the first has finished; both give the tracks of the event
    alone, and nothing stays resident."""
    big = max(range(len(pool)), key=lambda i: pool[i].n_clusters)
    fp = _footprint(pool[big])
    srv = tpc.Server(geo, 0.5, max_batch=4, n_workers=2, hbm_budget_bytes=fp + fp // 2)
    assert srv.submit(pool[big], 0) == tpc.TPC_OK
    busy, done = 0, {}
    rc = srv.submit(pool[big], 1)
    while rc == tpc.TPC_ERR_BUSY:
        busy += 1
        for d in srv.poll(timeout_ms=2):
            done[int(d["tag"])] = d
        rc = srv.submit(pool[big], 1)
    assert rc == tpc.TPC_OK
    assert busy > 0                      # the second copy had to wait for the first
    while len(done) < 2:
        for d in srv.poll(timeout_ms=100):
            done[int(d["tag"])] = d
    fetched = {}
    for k, d in done.items():
        assert d["status"] == tpc.TPC_OK
        fetched[k] = srv.fetch(d, pool[big].n_clusters)
    say("busy retries", busy)
    for r in fetched.values():
        assert r["n_tracks"] == alone[big]["n_tracks"]
        for key in KEYS:
            assert np.array_equal(r[key], alone[big][key]), key
    assert srv.stats()["resident_bytes"] == 0
    srv.close()


def test_event_larger_than_budget_is_refused(geo, pool):
    srv = tpc.Server(geo, 0.5, hbm_budget_bytes=1 << 20)
    with pytest.raises(tpc.TpcError) as ex:
        srv.submit(pool[3], 0)
    assert ex.value.code == tpc.TPC_ERR_OOM
    srv.close()


def test_one_at_a_time_path(geo, pool, alone):
    srv = tpc.Server(geo, 0.5, max_batch=1, n_workers=1, use_graph=0)
    res, fetched = serve.run(srv, pool, rate_hz=500.0, n_events=16, keep=set(range(16)))
    say(res)
    assert res["stats"]["batches"] == 16
    _check_same(fetched, pool, alone)
    srv.close()
