"""Track-by-track and cluster-by-cluster concordance of two tracker outputs.

Test infrastructure.  This is the comparison of section 3.3 of the paper:
the tracks of two runs are put in one-to-one correspondence, then for every
pair each row is checked for an identical cluster; a track without a
counterpart counts as entirely different.

Readings used where the paper gives no detail:
  * tracks a (run A) and b (run B) correspond when each is the other's best
    partner by shared clusters (ties: the smaller seed id) and they share more
    than half of the shorter one;
  * per pair the rows of both tracks are checked, so a row where only one of
    them has a cluster counts as a disagreement;
  * the figure is reported in both directions, A->B counting A's unmatched
    tracks and B->A counting B's.

Both outputs use the tracker's output layout: track_par [n, 8] (x, y, z,
sinphi, tanl, qpt, chi2, ndf), track_meta [n, 4] (sector, n_clusters, first,
seed_id), track_cluster (cluster indices), cluster_track [n_clusters].
"""
from __future__ import annotations

import numpy as np

PAR_FLOORS = np.array([1.0, 1.0, 0.1, 0.1, 0.1])   # y, z cm; sinphi; tanl; q/pT 1/GeV


def rel_dev(ref, got, with_x=False):
    """Largest relative deviation of each row of parameters from the
    reference: |got - ref| / max(|ref|, floor), floors 1 cm for x, y, z,
    0.1 for sin phi and tan lambda, 0.1 GeV^-1 for q/pT (relative above
    the floor, absolute below it)."""
    fl = np.concatenate([[1.0], PAR_FLOORS]) if with_x else PAR_FLOORS
    ref = np.asarray(ref, np.float64)
    got = np.asarray(got, np.float64)
    return (np.abs(got - ref) / np.maximum(np.abs(ref), fl)).max(axis=-1)


def _track_of_clusters(res):
    meta = np.asarray(res["track_meta"]).reshape(-1, 4)
    n = meta[:, 1].astype(np.int64)
    owner = np.repeat(np.arange(meta.shape[0], dtype=np.int64), n)
    first = meta[:, 2].astype(np.int64)
    idx = np.concatenate([np.arange(f, f + k) for f, k in zip(first, n)]) if len(n) else \
        np.zeros(0, np.int64)
    cl = np.asarray(res["track_cluster"])[idx].astype(np.int64)
    return cl, owner, n, meta[:, 3].astype(np.int64)


def _best_partner(cl_a, own_a, n_a, ct_b, seed_b):
    """For each track of A: (best track of B or -1, shared clusters)."""
    lab = np.asarray(ct_b)[cl_a].astype(np.int64)
    ok = lab >= 0
    a, b = own_a[ok], lab[ok]
    best = np.full(n_a.shape[0], -1, np.int64)
    shared = np.zeros(n_a.shape[0], np.int64)
    if a.size == 0:
        return best, shared
    nb = int(b.max()) + 1
    keys, cnt = np.unique(a * nb + b, return_counts=True)
    ka, kb = keys // nb, keys % nb
    # order: by a, then count descending, then seed id ascending -> first per a wins
    order = np.lexsort((seed_b[kb], -cnt, ka))
    ka, kb, cnt = ka[order], kb[order], cnt[order]
    firsts = np.ones(ka.shape[0], bool)
    firsts[1:] = ka[1:] != ka[:-1]
    best[ka[firsts]] = kb[firsts]
    shared[ka[firsts]] = cnt[firsts]
    return best, shared


def _match(res_a, res_b, n_clusters: int):
    cl_a, own_a, n_a, seed_a = _track_of_clusters(res_a)
    cl_b, own_b, n_b, seed_b = _track_of_clusters(res_b)
    ct_a = np.asarray(res_a["cluster_track"])[:n_clusters]
    ct_b = np.asarray(res_b["cluster_track"])[:n_clusters]
    best_ab, sh_ab = _best_partner(cl_a, own_a, n_a, ct_b, seed_b)
    best_ba, sh_ba = _best_partner(cl_b, own_b, n_b, ct_a, seed_a)
    ia = np.arange(n_a.shape[0])
    mutual = best_ab >= 0
    mutual[mutual] &= best_ba[best_ab[mutual]] == ia[mutual]
    mutual &= 2 * sh_ab > np.minimum(n_a, n_b[np.maximum(best_ab, 0)] if n_b.size else 0)
    match_a = np.where(mutual, best_ab, -1)
    match_b = np.full(n_b.shape[0], -1, np.int64)
    match_b[match_a[mutual]] = ia[mutual]
    return n_a, n_b, sh_ab, mutual, match_a, match_b


def match_tracks(res_a, res_b, n_clusters: int):
    """The one-to-one correspondence of the two runs' tracks: for each track
    of A its partner in B or -1, and for each track of B its partner in A."""
    _, _, _, _, match_a, match_b = _match(res_a, res_b, n_clusters)
    return match_a, match_b


def compare(res_a, res_b, n_clusters: int, rel_tol: float = 1e-3) -> dict:
    """Concordance of run B against run A (A = reference, e.g. the oracle)."""
    n_a, n_b, sh_ab, mutual, match_a, match_b = _match(res_a, res_b, n_clusters)
    ia = np.arange(n_a.shape[0])
    # per matched pair: identical clusters (same cluster => same row) and the union of rows
    agree = np.where(mutual, sh_ab, 0)
    union = np.where(mutual, n_a + n_b[np.maximum(match_a, 0)] - sh_ab if n_b.size else n_a, n_a)
    tot_ab = union.sum()
    tot_ba = np.where(match_b >= 0, 0, n_b).sum() + union[mutual].sum()
    agree_sum = agree.sum()
    out = dict(
        n_tracks_a=int(n_a.shape[0]), n_tracks_b=int(n_b.shape[0]),
        matched=int(mutual.sum()),
        track_concordance_ab=float(mutual.sum() / max(1, n_a.shape[0])),
        track_concordance_ba=float(mutual.sum() / max(1, n_b.shape[0])),
        cluster_concordance_ab=float(agree_sum / max(1, tot_ab)),
        cluster_concordance_ba=float(agree_sum / max(1, tot_ba)),
        clusters_a=int(n_a.sum()), clusters_b=int(n_b.sum()),
    )
    # parameters of matched pairs with identical cluster sets, the same
    # reference x and the same seed: the same fit, so rounding alone may
    # separate them.  A pair grown from different seeds (two chains of the
    # same clusters, e.g. after a link near-tie) ran another outward filter,
    # whose end state is the inward fit's linearisation point: such pairs
    # are listed in other_seed_pairs, not compared here.
    same = mutual & (agree == n_a) & (n_a == n_b[np.maximum(match_a, 0)] if n_b.size else False)
    pa = np.asarray(res_a["track_par"]).reshape(-1, 8)
    pb = np.asarray(res_b["track_par"]).reshape(-1, 8)
    ma = np.asarray(res_a["track_meta"]).reshape(-1, 4)
    mb = np.asarray(res_b["track_meta"]).reshape(-1, 4)
    ia_s = ia[same]
    ib_s = match_a[same]
    if ia_s.size:
        samex = pa[ia_s, 0] == pb[ib_s, 0]
        ia_s, ib_s = ia_s[samex], ib_s[samex]
    other = np.zeros(0, np.int64)
    if ia_s.size:
        same_seed = ma[ia_s, 3] == mb[ib_s, 3]
        other = np.stack([ia_s[~same_seed], ib_s[~same_seed]], axis=1)
        ia_s, ib_s = ia_s[same_seed], ib_s[same_seed]
    out["other_seed_pairs"] = other.reshape(-1, 2)
    out["par_other_seed"] = int(other.shape[0])
    if ia_s.size:
        worst = rel_dev(pa[ia_s, 1:6], pb[ib_s, 1:6])
        out.update(par_compared=int(ia_s.size), par_max_rel=float(worst.max()),
                   par_fail=int((worst > rel_tol).sum()),
                   par_fail_frac=float((worst > rel_tol).mean()))
    else:
        out.update(par_compared=0, par_max_rel=0.0, par_fail=0, par_fail_frac=0.0)
    out["cluster_concordance"] = min(out["cluster_concordance_ab"], out["cluster_concordance_ba"])
    out["track_concordance"] = min(out["track_concordance_ab"], out["track_concordance_ba"])
    return out


def _prolongations_by_key(pro, track_key=None):
    """(key of the prolonged track, end) -> (sector id entered, clusters,
    par); the key is the track index, mapped through track_key if given
    (tracks without a key get a key of their own, -1 - index)."""
    out = {}
    meta = np.asarray(pro["meta"]).reshape(-1, 5)
    for k in range(int(pro["n"])):
        t, end, sec, n, first = (int(v) for v in meta[k])
        key = t if track_key is None else int(track_key[t])
        if key < 0:
            key = -1 - t
        out[(key, end)] = (sec, np.asarray(pro["cluster"][first:first + n]),
                           np.asarray(pro["par"][k], np.float64))
    return out


def compare_prolongations(tracks_a, pro_a, tracks_b, pro_b, n_clusters: int,
                          rel_tol: float = 1e-3, chi2_tol: float = 1e-2) -> dict:
    """Agreement of two runs' global-tracking prolongations.  Their tracks are
    put in correspondence first (as in compare: a track is the same track in
    both runs even when FP32 and FP64 chose different seeds among tracklets
    with the same clusters); prolongations are then matched by (track, end).
    cluster_concordance_ab: the fraction of A's prolongation clusters that
    B's prolongation of the same (track, end) also holds; _ba the other way.
    For pairs with identical clusters whose tracks grew from the same seed in
    both runs, the parameters x..q/pT must agree within rel_tol relative
    (rel_dev's floors), ndf exactly and chi2 within chi2_tol relative
    (absolute below 1).  The chi2 of an update is r^2/S with a residual r of
    about sigma: an FP32 rounding of 1e-5 in sin(phi) of the filtered state,
    over the 10-20 cm lever arm to the next cluster, moves r by ~2e-4 cm, i.e.
    chi2 by several 1e-3 relative, while the parameters agree far within
    rel_tol; chi2_tol = 1e-2 covers that."""
    match_a, match_b = match_tracks(tracks_a, tracks_b, n_clusters)
    seed_a = np.asarray(tracks_a["track_meta"]).reshape(-1, 4)[:, 3]
    seed_b = np.asarray(tracks_b["track_meta"]).reshape(-1, 4)[:, 3]
    a = _prolongations_by_key(pro_a)
    b = _prolongations_by_key(pro_b, match_b)   # unmatched tracks: negative keys
    same = sum(np.intersect1d(v[1], b[k][1]).size for k, v in a.items() if k in b)
    tot_a = sum(v[1].size for v in a.values())
    tot_b = sum(v[1].size for v in b.values())
    identical = compared = fail = other_seed = 0
    for k, v in a.items():
        if not (k in b and b[k][0] == v[0] and np.array_equal(b[k][1], v[1])):
            continue
        identical += 1
        if seed_a[k[0]] != seed_b[match_a[k[0]]]:
            # the same track built from another seed: its end states come from
            # another outward filter, so its parameters are not compared
            other_seed += 1
            continue
        compared += 1
        pa, pb = v[2], b[k][2]
        ok = rel_dev(pa[:6], pb[:6], with_x=True) <= rel_tol
        ok = ok and pb[7] == pa[7] and abs(pb[6] - pa[6]) <= chi2_tol * max(1.0, abs(pa[6]))
        fail += 0 if ok else 1
    return dict(n_a=len(a), n_b=len(b), clusters_a=tot_a, clusters_b=tot_b,
                cluster_concordance_ab=same / max(1, tot_a),
                cluster_concordance_ba=same / max(1, tot_b),
                identical=identical, other_seed=other_seed, par_compared=compared,
                par_fail=fail)


def compare_merged(tracks_a, merged_a, tracks_b, merged_b, n_clusters: int,
                   rel_tol: float = 1e-3, chi2_tol: float = 1e-2, min_fit: int = 30) -> dict:
    """Agreement of two runs' joined (merged) tracks.  A joined track of B
    corresponds to the joined track of A that holds the partner of B's first
    sector track (the tracks' one-to-one correspondence, as in compare).
    joins_same: A's joined tracks whose sector tracks map one-to-one onto one
    joined track of B; cluster_concordance_ab / _ba: the fraction of A's (B's)
    list clusters that the corresponding list of the other run holds; for
    identical lists, the refit parameters must agree within rel_tol relative
    (rel_dev's floors), ndf exactly and chi2 within chi2_tol (the refit is a
    function of the list alone, so only FP32/FP64 rounding separates them),
    for refits that fitted at least min_fit clusters on both sides (ndf >=
    2 min_fit - 5).  Shorter fits are counted, not compared: they are lists
    (of loopers) whose steps pass the |sin phi| limit near a turning point, and
    which steps fail there is decided in FP32 and FP64 near the limit, so the
    fitted subsets, hence the fits, differ.  par_max_rel: the largest relative
    parameter deviation among the compared fits."""
    match_a, match_b = match_tracks(tracks_a, tracks_b, n_clusters)
    ma, mb = np.asarray(merged_a["meta"]).reshape(-1, 5), np.asarray(merged_b["meta"]).reshape(-1, 5)
    tma, tmb = np.asarray(merged_a["track_merged"]), np.asarray(merged_b["track_merged"])
    la = [np.asarray(merged_a["cluster"][m[3]:m[3] + m[2]]) for m in ma]
    lb = [np.asarray(merged_b["cluster"][m[3]:m[3] + m[2]]) for m in mb]
    # joined track of B for each joined track of A, through A's first track
    corr = np.full(len(la), -1, np.int64)
    for k, m in enumerate(ma):
        tb = match_a[m[4]]
        if tb >= 0:
            corr[k] = tmb[tb]
    same_join = 0
    for k in range(len(la)):
        if corr[k] < 0:
            continue
        segs_a = np.nonzero(tma == k)[0]
        segs_b = np.nonzero(tmb == corr[k])[0]
        mapped = match_a[segs_a]
        same_join += int(np.all(mapped >= 0) and np.array_equal(np.sort(mapped), segs_b))
    shared = sum(np.intersect1d(la[k], lb[corr[k]]).size for k in range(len(la)) if corr[k] >= 0)
    tot_a = sum(x.size for x in la)
    tot_b = sum(x.size for x in lb)
    pa_all = np.asarray(merged_a["par"], np.float64).reshape(-1, 8)
    pb_all = np.asarray(merged_b["par"], np.float64).reshape(-1, 8)
    identical = compared = fail = short = 0
    max_rel = 0.0
    for k in range(len(la)):
        if corr[k] < 0 or not np.array_equal(la[k], lb[corr[k]]):
            continue
        identical += 1
        pa, pb = pa_all[k], pb_all[corr[k]]
        if pa[7] < 2 * min_fit - 5 or pb[7] < 2 * min_fit - 5:
            short += 1
            continue
        compared += 1
        rel = rel_dev(pa[:6], pb[:6], with_x=True)
        max_rel = max(max_rel, float(rel))
        ok = rel <= rel_tol
        ok = ok and pb[7] == pa[7] and abs(pb[6] - pa[6]) <= chi2_tol * max(1.0, abs(pa[6]))
        fail += 0 if ok else 1
    return dict(n_a=len(la), n_b=len(lb), joins_same=same_join,
                joins_same_frac=same_join / max(1, len(la)),
                clusters_a=tot_a, clusters_b=tot_b,
                cluster_concordance_ab=shared / max(1, tot_a),
                cluster_concordance_ba=shared / max(1, tot_b),
                identical=identical, short_fits=short, par_compared=compared, par_fail=fail,
                par_max_rel=max_rel)
