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


def test_admission_by_footprint_defers_not_fails(geo, pool, alone):
    # room for about two of the larger events at a time
    budget = 2 * 160 * max(h.n_clusters for h in pool) + (1 << 20)
    srv = tpc.Server(geo, 0.5, max_batch=4, n_workers=2, hbm_budget_bytes=budget)
    res, fetched = serve.run(srv, pool, rate_hz=5000.0, n_events=24, keep=set(range(24)))
    say(res)
    assert res["busy_retries"] > 0
    assert res["stats"]["resident_bytes"] == 0
    _check_same(fetched, pool, alone)
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
