"""GPU path (through the C ABI) against the FP64 oracle.

Integer work that has a unique answer given the same inputs (evolution,
chain starts, output ordering) must be bit-exact.  Decisions taken on FP32
values (neighbour pair, chi^2 gate, weight comparison) may differ from the
FP64 oracle only at verified near-ties; the whole-event agreement is the
paper's cluster-by-cluster concordance, required >= 99.99% both ways, with
matched tracks' parameters within 1e-3 relative.
"""
import os

import types

import numpy as np
import pytest

from conftest import event_dict, f32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import concordance  # noqa: E402
from paper_1712_09407_amd import synth, tpc  # noqa: E402

THREADS = min(16, os.cpu_count() or 1)
GEO_T = (synth.ROW_X, synth.TAN_HALF, synth.Z_MAX)


def say(*a):
    print("[gpu-test]", *a, flush=True)


@pytest.fixture(scope="module")
def tracker():
    t = tpc.Tracker(0)
    yield t
    t.close()


@pytest.fixture(scope="module")
def geo():
    return tpc.make_geometry(*GEO_T)


def params_pair(orc, sigma=0.1, **kw):
    """The same constants for both sides (FP32 values, widened for the oracle)."""
    g = tpc.default_params(sigma_y=sigma, sigma_z=sigma, **kw)
    o = orc.default_params(**{k: f32(getattr(g, k)) if isinstance(getattr(g, k), float)
                              else getattr(g, k) for k, _ in orc.Params._fields_})
    return g, o


_events = {}


def get_event(name, seed):
    key = (name, seed)
    if key not in _events:
        say("generate", name, seed)
        _events[key] = synth.make_preset(name, seed)
    return _events[key]


def dev_event(e):
    return tpc.DeviceEvent.from_host(e.y, e.z, e.row_offsets, e.sector_id, device="cuda:0")


# ------------------------------------------------------------- links
def check_links(orc, e, prm_o, up_g, dn_g, up_o, dn_o):
    ev = event_dict(e)
    mism = np.nonzero((up_g != up_o) | (dn_g != dn_o))[0]
    for c in mism:
        co = orc.nf_chi2(ev, GEO_T, dn_o[c], c, up_o[c], prm_o) if up_o[c] >= 0 else None
        cg = orc.nf_chi2(ev, GEO_T, dn_g[c], c, up_g[c], prm_o) if up_g[c] >= 0 else None
        cut = prm_o.nf_chi2_max
        if co is not None and cg is not None:
            assert abs(cg - co) <= 1e-4 * max(1.0, co), (c, co, cg)   # near-tie of two pairs
        else:
            v = co if co is not None else cg
            assert abs(v - cut) <= 1e-4 * max(1.0, cut), (c, v)       # at the cut
    return mism.size


@pytest.mark.parametrize("name,seed", [("c1_sector", 1), ("c2_central", 2)])
def test_links_match_oracle(orc, tracker, geo, name, seed):
    e = get_event(name, seed)
    say("links", name, seed, e.n_clusters)
    pg, po = params_pair(orc, e.config.sigma)
    up, dn, up2, dn2 = (x.cpu().numpy() for x in tracker.links(dev_event(e), geo, pg))
    uo, do_ = orc.neighbours(event_dict(e), GEO_T, po)
    n_bad = check_links(orc, e, po, up, dn, uo, do_)
    assert n_bad <= max(2, 1e-5 * e.n_clusters), n_bad
    # evolution is integer work: bit-exact on the GPU's own links
    eu, ed = orc.evolve(up, dn)
    assert np.array_equal(eu, up2) and np.array_equal(ed, dn2)
    assert (up2 >= 0).sum() > 0.5 * e.n_clusters


# ------------------------------------------------------------- tracklets
@pytest.mark.parametrize("name,seed", [("c1_sector", 1), ("c2_central", 2), ("c5_stress", 5000)])
def test_seeds_and_tracklets_match_oracle(orc, tracker, geo, name, seed):
    e = get_event(name, seed)
    say("tracklets", name, seed)
    pg, po = params_pair(orc, e.config.sigma)
    dev = dev_event(e)
    _, _, up2, dn2 = (x.cpu().numpy() for x in tracker.links(dev, geo, pg))
    tl = tpc.to_numpy(tracker.tracklets(dev, geo, e.bz, pg))
    # chain starts: bit-exact given the same links
    seeds_o = orc.seeds(event_dict(e), GEO_T, up2, dn2, po)
    assert np.array_equal(tl["seeds"], seeds_o)
    # construction from the same seeds along the same links
    ref = orc.construct(event_dict(e), GEO_T, e.bz, up2, tl["seeds"], po)
    n_tl = seeds_o.shape[0]
    same = np.zeros(n_tl, bool)
    for t in range(n_tl):
        lo, hi = tl["row_lo"][t], tl["row_hi"][t]
        if tl["n"][t] != ref["n"][t]:
            continue
        if tl["n"][t] == 0:
            same[t] = True
            continue
        same[t] = (lo == ref["row_lo"][t] and hi == ref["row_hi"][t] and
                   np.array_equal(tl["hits"][t, lo:hi + 1], ref["hits"][t, lo:hi + 1]))
    frac = same.mean()
    say("identical tracklets", frac, n_tl, "differing", int((~same).sum()))
    assert frac >= 0.9999
    ok = same & (ref["n"] > 0)
    assert np.array_equal(tl["par"][ok, 0].astype(np.float64), ref["par"][ok, 0])
    # parameters: the 1e-3 relative tolerance is for tracklets long enough to
    # become tracks; shorter ones are weakly constrained and only their
    # clusters must agree
    ok &= ref["n"] >= po.min_clusters
    P, R = tl["par"][ok].astype(np.float64), ref["par"][ok]
    floors = np.array([1.0, 1.0, 0.1, 0.1, 0.1])
    rel = np.abs(P[:, 1:] - R[:, 1:]) / np.maximum(np.abs(R[:, 1:]), floors)
    worst = int(np.argmax(rel.max(axis=1)))
    say("worst parameter difference", rel.max(axis=1)[worst], "n", ref["n"][ok][worst],
        "gpu", P[worst], "oracle", R[worst])
    assert rel.max() <= 1e-3, rel.max(axis=0)
    c = tl["chi2"][ok].astype(np.float64)
    cdev = np.abs(c - ref["chi2"][ok]) / np.maximum(ref["chi2"][ok], 1.0)
    say("chi2 deviation: max", cdev.max(), "above 1e-3", np.mean(cdev > 1e-3))
    assert np.mean(cdev > 1e-3) <= 1e-3
    assert np.array_equal(tl["ndf"][ok], ref["ndf"][ok])


def test_selection_matches_oracle_on_gpu_tracklets(orc, tracker, geo):
    """Assignment and selection are integer work once the weights are known.
    The weight decides an argmax, so both sides take it in the kernel's
    precision: the oracle is given the FP32 weights (same formula and
    operation order as the kernel) and must then agree exactly."""
    e = get_event("c2_central", 2)
    say("selection")
    pg, po = params_pair(orc, e.config.sigma)
    dev = dev_event(e)
    tl = tpc.to_numpy(tracker.tracklets(dev, geo, e.bz, pg))
    res = tpc.to_numpy(tracker.track_event(dev, geo, e.bz, pg))
    n32 = tl["n"].astype(np.float32)
    ndf32 = np.maximum(tl["ndf"], 1).astype(np.float32)
    w32 = n32 * (np.float32(pg.alpha) - (tl["chi2"] / ndf32) / np.float32(pg.beta))
    w32 = w32 + np.float32(0.0)
    tlo = dict(hits=tl["hits"], row_lo=tl["row_lo"], row_hi=tl["row_hi"], n=tl["n"],
               chi2=tl["chi2"].astype(np.float64), ndf=tl["ndf"],
               par=tl["par"].astype(np.float64))
    owner, keep = orc.select(event_dict(e), GEO_T, e.bz, tl["seeds"], tlo, po,
                             weights=w32.astype(np.float64))
    kept = np.nonzero(keep)[0]
    want = {int(tl["seeds"][t]): sorted(int(c) for c in tl["hits"][t, tl["row_lo"][t]:tl["row_hi"][t] + 1]
                                        if c >= 0 and owner[c] == t) for t in kept}
    got = {}
    m = res["track_meta"]
    for i in range(res["n_tracks"]):
        got[int(m[i, 3])] = sorted(res["track_cluster"][m[i, 2]:m[i, 2] + m[i, 1]].tolist())
    diff = [k for k in set(want) | set(got) if want.get(k) != got.get(k)]
    say("selection differences", len(diff), "of", len(want))
    assert not diff


# ------------------------------------------------------------- end to end
def check_other_seed_fits(orc, tracker, e, pg, po, res, pairs):
    """Matched tracks with identical clusters whose seeds differ (the chains
    of the two runs start at different clusters, e.g. after a neighbour-pair
    near-tie) are not the same fit: each ran its own outward filter, and the
    inward fit starts from that filter's state.  The oracle's construction
    from the GPU's seed, along the GPU's links, must reproduce the GPU's
    parameters: then the difference is the seed, not the arithmetic."""
    say("identical clusters from another seed", len(pairs))
    if not len(pairs):
        return
    _, _, up2, _ = (x.cpu().numpy() for x in tracker.links(dev_event(e), geo_of(), pg))
    ib = pairs[:, 1]
    seeds = res["track_meta"][ib, 3].astype(np.int32)
    tlo = orc.construct(event_dict(e), GEO_T, e.bz, up2, seeds, po)
    assert np.array_equal(tlo["ndf"], res["track_par"][ib, 7].astype(np.int32))
    dev = concordance.rel_dev(tlo["par"][:, 1:6], res["track_par"][ib, 1:6])
    say("  oracle from the GPU's seeds: max deviation", dev.max())
    assert dev.max() <= 1e-3


def geo_of():
    return tpc.make_geometry(*GEO_T)


@pytest.mark.parametrize("name,seed", [("c1_sector", 1), ("c2_central", 2), ("c2_central", 3),
                                       ("c5_stress", 5000)])
def test_end_to_end_concordance(orc, tracker, geo, name, seed):
    e = get_event(name, seed)
    say("end-to-end", name, seed, e.n_clusters)
    pg, po = params_pair(orc, e.config.sigma)
    res = tpc.to_numpy(tracker.track_event(dev_event(e), geo, e.bz, pg))
    ref = orc.track_event(event_dict(e), GEO_T, e.bz, po, n_threads=THREADS)
    rep = concordance.compare(ref, res, e.n_clusters)
    say(name, seed, {k: rep[k] for k in ("n_tracks_a", "n_tracks_b", "cluster_concordance",
                                         "track_concordance", "par_compared", "par_max_rel",
                                         "par_fail")})
    assert rep["cluster_concordance"] >= 0.9999
    assert rep["track_concordance"] >= 0.9999
    # identical clusters grown from the same seed: the same fit (section 3.3)
    assert rep["par_fail"] == 0, rep["par_max_rel"]
    check_other_seed_fits(orc, tracker, e, pg, po, res, rep["other_seed_pairs"])
    # output invariants
    m = res["track_meta"]
    assert np.all(m[:, 1] >= 30)
    assert np.all(np.diff(m[:, 3]) > 0)                           # sorted by seed id
    assert np.sum(res["cluster_track"] >= 0) == res["n_track_clusters"]


@pytest.mark.parametrize("alpha_gpu,alpha_orc", [(1.0, 1.0), (1e9, 1e30)])
def test_other_alphas_match_the_oracle(orc, tracker, geo, alpha_gpu, alpha_orc):
    """Section 3.1's weight w = n (alpha - chi^2/beta) at a small alpha and at
    alpha = infinity, the longest-track rule: on the GPU alpha = 1e9, where
    FP32 rounds alpha - chi^2/ndf to alpha, so w orders by length alone, as
    the oracle's 1e30 does in FP64.  The same concordance bar as at alpha = 6."""
    e = get_event("c2_central", 2)
    say("alpha", alpha_gpu, alpha_orc)
    pg, po = params_pair(orc, e.config.sigma, alpha=alpha_gpu)
    po.alpha = alpha_orc
    res = tpc.to_numpy(tracker.track_event(dev_event(e), geo, e.bz, pg))
    ref = orc.track_event(event_dict(e), GEO_T, e.bz, po, n_threads=THREADS)
    rep = concordance.compare(ref, res, e.n_clusters)
    say({k: rep[k] for k in ("n_tracks_a", "n_tracks_b", "cluster_concordance_ab",
                             "cluster_concordance_ba", "track_concordance", "par_compared",
                             "par_max_rel", "par_fail")})
    assert rep["cluster_concordance"] >= 0.9999
    assert rep["track_concordance"] >= 0.9999
    assert rep["par_fail"] == 0, rep["par_max_rel"]
    check_other_seed_fits(orc, tracker, e, pg, po, res, rep["other_seed_pairs"])


def test_deterministic(orc, tracker, geo):
    e = get_event("c2_central", 2)
    dev = dev_event(e)
    a = tpc.to_numpy(tracker.track_event(dev, geo, e.bz))
    b = tpc.to_numpy(tracker.track_event(dev, geo, e.bz))
    for k in ("track_par", "track_meta", "track_cluster", "cluster_track"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("name,seed", [("c1_sector", 1), ("c2_central", 2), ("c5_stress", 5),
                                       ("dense", 31), ("sparse", 77)])
def test_constructor_schedules_agree_bitwise(tracker, geo, name, seed):
    """The row-synchronous and the lane-per-tracklet constructor run the same
    lane steps: every output bit must agree (dense rows exercise the
    global-memory search of the row-synchronous schedule).  The lane
    constructor runs with its default lanes per wave and with 64; it keeps its
    hit rows in LDS when its whole grid stays resident with them (the central
    and smaller events here) and in the hits array otherwise (the stress
    event), so both storages are compared with the row-synchronous one."""
    if name == "dense":
        e = synth.make_event(synth.EventConfig(n_tracks=150, sectors=(0,), phi_range_deg=(0, 20),
                                               ignore_membrane=True, noise_frac=20.0), seed)
        assert np.diff(e.row_offsets).max() > 1024
    elif name == "sparse":
        e = synth.make_event(synth.EventConfig(n_tracks=3), seed)
    else:
        e = get_event(name, seed)
    say("schedules", name, seed, e.n_clusters)
    dev = dev_event(e)
    out = []
    for tuning in (dict(construct_schedule=0), dict(construct_schedule=1),
                   dict(construct_schedule=0, construct_lanes=64)):
        tracker.set_tuning(**tuning)
        tl = tracker.tracklets(dev, geo, e.bz)
        res = tpc.to_numpy(tracker.track_event(dev, geo, e.bz))
        out.append((tpc.to_numpy(tl), res))
    tracker.set_tuning()
    tla, ra = out[0]
    for tlb, rb in out[1:]:
        for k in tla:
            if k != "hits":
                assert np.array_equal(tla[k].view(np.uint8), tlb[k].view(np.uint8)), k
        for t in range(len(tla["seeds"])):  # hits are defined on [row_lo, row_hi]
            lo, hi = tla["row_lo"][t], tla["row_hi"][t]
            assert np.array_equal(tla["hits"][t, lo:hi + 1], tlb["hits"][t, lo:hi + 1]), t
        for k in ("track_par", "track_meta", "track_cluster", "cluster_track"):
            assert np.array_equal(ra[k].view(np.uint8), rb[k].view(np.uint8)), k


@pytest.mark.parametrize("name", ["c1_sector", "c2_central", "crowded", "dense"])
def test_neighbour_forms_agree_bitwise(tracker, geo, name):
    """The neighbours finder's three forms (512-cluster stage with four waves,
    1024-cluster stage with 8-bit lists, 256-cluster stage with one wave per
    row slot, which also runs the grid, evolution and seed kernels with one
    wave per row slot) give the same links and tracks bit for bit: on the
    central event the one-wave form takes its rows of more than 256 clusters
    through the global-memory search, on the crowded one its wave-wide
    search, on the dense one every form takes some rows through the
    global-memory search, and the one-wave grid kernel counts its rows of more
    than 1024 bins in global memory."""
    if name == "crowded":
        e = crowded_event(41, 3.0, 140)
    elif name == "dense":
        e = synth.make_event(synth.EventConfig(n_tracks=150, sectors=(0,), phi_range_deg=(0, 20),
                                               ignore_membrane=True, noise_frac=20.0), 31)
    else:
        e = get_event(name, {"c1_sector": 1, "c2_central": 2}[name])
    say("neighbour forms", name, e.n_clusters)
    dev = dev_event(e)
    links, res = [], []
    for form in (1, 2, 3):
        tracker.set_tuning(nf_stage=form)
        links.append([x.cpu().numpy() for x in tracker.links(dev, geo)])
        res.append(tpc.to_numpy(tracker.track_event(dev, geo, e.bz)))
    tracker.set_tuning()
    if name == "c2_central":
        assert np.diff(e.row_offsets).max() > 256
    if name == "dense":
        assert np.diff(e.row_offsets).max() > 1024
    for other in links[1:]:
        for a, b in zip(links[0], other):
            assert np.array_equal(a, b)
    for other in res[1:]:
        for k in ("track_par", "track_meta", "track_cluster", "cluster_track"):
            assert np.array_equal(res[0][k].view(np.uint8), other[k].view(np.uint8)), k


# ------------------------------------------------------------- edge cases
def test_empty_and_sparse_events(orc, tracker, geo):
    ro = np.zeros(36 * 159 + 1, np.int32)
    dev = tpc.DeviceEvent.from_host(np.zeros(0), np.zeros(0), ro, np.arange(36))
    res = tracker.track_event(dev, geo, 0.5)
    assert res["n_tracks"] == 0
    e = synth.make_event(synth.EventConfig(n_tracks=3), 77)     # mostly empty rows
    pg, po = params_pair(orc)
    res = tpc.to_numpy(tracker.track_event(dev_event(e), geo, e.bz, pg))
    ref = orc.track_event(event_dict(e), GEO_T, e.bz, po)
    assert concordance.compare(ref, res, e.n_clusters)["cluster_concordance"] == 1.0


def test_dense_rows_use_the_global_memory_path(orc, tracker, geo):
    """Rows with more clusters than the LDS stage holds (noise flood, as in the
    paper's section 6 incident) must give the same links."""
    cfg = synth.EventConfig(n_tracks=150, sectors=(0,), phi_range_deg=(0, 20),
                            ignore_membrane=True, noise_frac=20.0)
    e = synth.make_event(cfg, 31)
    assert np.diff(e.row_offsets).max() > 1024
    pg, po = params_pair(orc)
    up, dn, _, _ = (x.cpu().numpy() for x in tracker.links(dev_event(e), geo, pg))
    uo, do_ = orc.neighbours(event_dict(e), GEO_T, po)
    assert check_links(orc, e, po, up, dn, uo, do_) <= max(2, 1e-5 * e.n_clusters)
    res = tpc.to_numpy(tracker.track_event(dev_event(e), geo, e.bz, pg))
    ref = orc.track_event(event_dict(e), GEO_T, e.bz, po)
    rep = concordance.compare(ref, res, e.n_clusters)
    say("noise flood", {k: rep[k] for k in ("cluster_concordance", "track_concordance",
                                            "par_fail")})
    assert rep["cluster_concordance"] >= 0.9999 and rep["track_concordance"] >= 0.9999


def crowded_event(seed, noise_frac, n_hot):
    """One sector with a hot spot of n_hot clusters in a 6 x 6 cm box on every
    row: each of them sees about n_hot window candidates in both neighbour
    rows, more than a lane's candidate list holds."""
    cfg = synth.EventConfig(n_tracks=100, sectors=(0,), phi_range_deg=(0, 20),
                            ignore_membrane=True, noise_frac=noise_frac)
    e = synth.make_event(cfg, seed)
    rng = np.random.default_rng(seed)
    ys, zs, ro = [], [], [0]
    for r in range(e.row_offsets.shape[0] - 1):
        a, b = e.row_offsets[r], e.row_offsets[r + 1]
        ys += [e.y[a:b], rng.uniform(-3.0, 3.0, n_hot).astype(np.float32)]
        zs += [e.z[a:b], rng.uniform(97.0, 103.0, n_hot).astype(np.float32)]
        ro.append(ro[-1] + (b - a) + n_hot)
    return types.SimpleNamespace(y=np.concatenate(ys), z=np.concatenate(zs),
                                 row_offsets=np.array(ro, np.int32), sector_id=e.sector_id,
                                 bz=e.bz, n_clusters=int(ro[-1]))


@pytest.mark.parametrize("noise_frac,n_hot", [(0.0, 30), (3.0, 140)])
def test_crowded_windows_match_the_oracle(orc, tracker, geo, noise_frac, n_hot):
    """Clusters with more window candidates than a lane's list (12 on sparse
    rows, 32 on dense ones, about 300 clusters per row and more) are searched
    by the whole wave: the links are the oracle's (up to near-ties)."""
    e = crowded_event(41, noise_frac, n_hot)
    say("crowded", noise_frac, n_hot, e.n_clusters)
    dense = e.n_clusters > 320 * (e.row_offsets.shape[0] - 1)
    assert dense == (n_hot > 32)
    pg, po = params_pair(orc)
    up, dn, _, _ = (x.cpu().numpy() for x in tracker.links(dev_event(e), geo, pg))
    uo, do_ = orc.neighbours(event_dict(e), GEO_T, po)
    assert check_links(orc, e, po, up, dn, uo, do_) <= max(2, 1e-5 * e.n_clusters)
    hot = np.concatenate([np.arange(e.row_offsets[r + 1] - n_hot, e.row_offsets[r + 1])
                          for r in range(1, e.row_offsets.shape[0] - 2)])
    assert (up[hot] >= 0).mean() > 0.9                    # the hot spot links up


def test_wide_thin_rows_match_the_oracle(orc, tracker, geo):
    """Dense rows (one sector, 0.44 clusters per cm^2, z in a 20 cm slab) on
    which a window's candidates lie in several bin rows of the row's grid,
    each as wide as the sector: on the outer rows about one in ten clusters
    has at most 32 candidates in a neighbour row that lie more than 255
    positions apart in grid order, beyond what an 8-bit list entry holds,
    and about as many have more than 32.  Both go to the wave-wide search:
    the links are the oracle's (up to near-ties)."""
    rng = np.random.default_rng(43)
    xr = synth.ROW_X.astype(np.float64)
    ys, zs, ro = [], [], [0]
    for r in range(synth.N_ROWS):
        hw = xr[r] * float(synth.TAN_HALF)
        n = int(0.44 * 2.0 * hw * 20.0)
        ys.append(rng.uniform(-hw, hw, n).astype(np.float32))
        zs.append(rng.uniform(0.0, 20.0, n).astype(np.float32))
        ro.append(ro[-1] + n)
    e = types.SimpleNamespace(y=np.concatenate(ys), z=np.concatenate(zs),
                              row_offsets=np.array(ro, np.int32),
                              sector_id=np.array([0], np.int32), bz=0.5, n_clusters=int(ro[-1]))
    say("wide thin rows", e.n_clusters)
    assert e.n_clusters > 320 * synth.N_ROWS                  # the dense configuration
    pg, po = params_pair(orc)
    up, dn, _, _ = (x.cpu().numpy() for x in tracker.links(dev_event(e), geo, pg))
    uo, do_ = orc.neighbours(event_dict(e), GEO_T, po)
    assert check_links(orc, e, po, up, dn, uo, do_) <= max(2, 1e-5 * e.n_clusters)
    assert (up >= 0).mean() > 0.9


def test_invalid_offsets_and_nonfinite(tracker, geo):
    e = get_event("c1_sector", 1)
    ro = e.row_offsets.copy()
    ro[10], ro[11] = ro[11], ro[10] - 1                            # decreasing
    dev = tpc.DeviceEvent.from_host(e.y, e.z, ro, e.sector_id)
    with pytest.raises(tpc.TpcError) as ex:
        tracker.track_event(dev, geo, e.bz)
    assert ex.value.code == tpc.TPC_ERR_INVALID_ARG
    ro = e.row_offsets.copy()
    ro[-1] -= 1                                                    # last != n_clusters
    with pytest.raises(tpc.TpcError):
        tracker.track_event(tpc.DeviceEvent.from_host(e.y, e.z, ro, e.sector_id), geo, e.bz)
    y = e.y.copy()
    y[100] = np.nan
    with pytest.raises(tpc.TpcError) as ex:
        tracker.track_event(tpc.DeviceEvent.from_host(y, e.z, e.row_offsets, e.sector_id), geo,
                            e.bz)
    assert "non-finite" in str(ex.value)
    # the context still works afterwards
    assert tracker.track_event(dev_event(e), geo, e.bz)["n_tracks"] > 0


def test_capacity_error_reports_sizes(tracker, geo):
    e = get_event("c1_sector", 1)
    dev = dev_event(e)
    full = tracker.track_event(dev, geo, e.bz)
    with pytest.raises(tpc.TpcError) as ex:
        tracker.track_event(dev, geo, e.bz, cap_tracks=3, cap_track_clusters=100)
    assert ex.value.code == tpc.TPC_ERR_CAPACITY
    assert str(full["n_tracks"]) in str(ex.value)


def test_tracklet_reservation_overflow_and_retry(orc, tracker, geo):
    # many short straight tracks: far more tracklets per cluster than a central event
    rng = np.random.default_rng(4)
    rows = []
    for r in range(159):
        rows.append([])
    ys, zs, rs = [], [], []
    for k in range(600):
        r0 = int(rng.integers(1, 140))
        y0, z0 = rng.uniform(-10, 10), rng.uniform(5, 240)
        for r in range(r0, r0 + 12):
            ys.append(y0 + 0.01 * (r - r0))
            zs.append(z0 + 0.02 * (r - r0))
            rs.append(r)
    rs = np.array(rs)
    order = np.argsort(rs, kind="stable")
    y = np.array(ys, np.float32)[order]
    z = np.array(zs, np.float32)[order]
    ro = np.zeros(160, np.int32)
    np.cumsum(np.bincount(rs, minlength=159), out=ro[1:])
    dev = tpc.DeviceEvent.from_host(y, z, ro, np.array([0]))
    p_small = tpc.default_params(min_clusters=10, max_tracklets=16)
    with pytest.raises(tpc.TpcError) as ex:
        tracker.track_event(dev, geo, 0.5, p_small)
    assert ex.value.code == tpc.TPC_ERR_OVERFLOW
    fresh = tpc.Tracker(0)
    auto = tpc.to_numpy(fresh.track_event(dev, geo, 0.5, tpc.default_params(min_clusters=10)))
    big = tpc.to_numpy(tracker.track_event(dev, geo, 0.5,
                                           tpc.default_params(min_clusters=10,
                                                              max_tracklets=100000)))
    fresh.close()
    assert auto["n_tracks"] > 100
    for k in ("track_par", "track_meta", "track_cluster"):
        assert np.array_equal(auto[k], big[k])
