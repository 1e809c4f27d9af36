"""Pins of the oracle's re-rank references (CPU): the bounded walk against
Observation 1 (the minimal re-rank set lies inside what the walk visits;
when every bound holds the walk visits at most the objects whose lower
bound is at most the k-th upper bound and stops early with the exact
top-k), the minimal set on the worked re-rank example, the early re-rank
accounting of the improved IVF+PQ search (Algorithm 4) on a hand-computed
example, and the collector's definition against a replay of the paper's
Push / Update / Collect workflow."""
import numpy as np
import pytest

import oracle
import synth


# --------------------------------------------------------------------------
# Observation 1: minimal re-rank set
# --------------------------------------------------------------------------

def test_min_rerank_worked_example():
    """Top-2 of four objects laid out as in the re-rank example of the
    overview figure: objects 6 and 45 are the top 2 with 45 the boundary
    object, the intervals of 45 and 12 contain Dist_k, and object 8's lower
    bound exceeds object 6's upper bound.  The minimal set is {45, 12}; a
    path that returns exact distances also needs object 6's."""
    ids = np.array([6, 45, 12, 8], np.int64)
    lb = np.array([1.0, 2.5, 2.8, 4.5], np.float32)
    ub = np.array([2.0, 4.0, 5.0, 7.0], np.float32)
    ex = np.array([1.5, 3.0, 4.0, 6.0], np.float32)
    n_min, n_min_out, dk = oracle.min_rerank(lb, ub, ex, ids, 2)
    assert dk == np.float32(3.0)
    assert n_min == 2 and n_min_out == 3
    # fewer objects than k: no boundary object
    assert oracle.min_rerank(lb[:1], ub[:1], ex[:1], ids[:1], 2)[:2] == (0, 0)
    # Dist_k on an interval's edge belongs to it (closed interval)
    n_min, _, _ = oracle.min_rerank(np.array([1.0, 3.0], np.float32), np.array([3.0, 9.0], np.float32),
                                    np.array([2.0, 3.0], np.float32), np.array([0, 1], np.int64), 2)
    assert n_min == 2


def _walk_fixture(eps0, k, nprobe, seed_index=3):
    d, n, nlist, nq = 64, 1500, 4, 5
    w = synth.small_workload("ivfrabitq_1m_d960", n=n, nlist=nlist, nq=nq, d=d, seed_index=seed_index)
    x, q = synth.base_vectors(w), synth.query_vectors(w)
    tr, ip = synth.kmeans_draws(n, nlist, 64 * nlist, 0)
    P = synth.rotation_orthogonal(d, 320 + seed_index)
    ix = oracle.build_ivf_rabitq(x, nlist, tr, ip, P)
    r = oracle.search_rabitq(ix, q, k, nprobe, eps0=eps0, debug=True)
    per_q = []
    for i in range(nq):
        lists = r["probe_lists"][r["probe_off"][i]:r["probe_off"][i + 1]]
        slots = np.concatenate([np.arange(ix["list_off"][j], ix["list_off"][j + 1]) for j in lists])
        ids = ix["list_ids"][slots]
        es = slice(r["est_off"][i], r["est_off"][i + 1])
        ex = oracle.canon_l2_batch(q[i], x[ids])
        per_q.append(dict(ids=ids, lb=r["est_lb"][es], ub=r["est_ub"][es], ex=ex,
                          visited=int(r["n_visited"][i]), out=r["ids"][r["off"][i]:r["off"][i + 1]],
                          dists=r["dists"][r["off"][i]:r["off"][i + 1]]))
    return per_q


@pytest.mark.parametrize("eps0", [0.0, 0.3, 1.9])
def test_walk_visits_the_minimal_set(eps0):
    """Whatever the bounds, the walk visits every object whose lower bound is
    at most Dist_k (its running k-th exact key never drops below Dist_k), so
    Observation 1's minimal set is inside the visited prefix and the visited
    count is at least the minimal set's size."""
    k = 40
    for o in _walk_fixture(eps0, k, 2):
        order = np.lexsort((o["ids"], o["lb"]))
        visited = set(o["ids"][order[:o["visited"]]].tolist())
        dk_pos = np.lexsort((o["ids"], o["ex"]))[k - 1]
        dk = o["ex"][dk_pos]
        must = set(o["ids"][o["lb"] <= dk].tolist())
        assert must <= visited
        n_min, _, got_dk = oracle.min_rerank(o["lb"], o["ub"], o["ex"], o["ids"], k)
        assert got_dk == dk
        minimal = set(o["ids"][(o["lb"] <= dk) & (dk <= o["ub"])].tolist())
        assert len(minimal) == n_min and minimal <= visited


def test_walk_with_holding_bounds_stops_early_and_is_exact():
    """A confidence wide enough that every bound of the fixture holds (checked
    first): the walk then stops before the end of the scan, visits only
    objects whose lower bound is at most U (the k-th smallest upper bound),
    and still returns the exact top-k over every scanned object."""
    k = 30
    for o in _walk_fixture(4.0, k, 4, seed_index=4):
        assert np.all((o["lb"] <= o["ex"]) & (o["ex"] <= o["ub"])), "fixture: a bound fails"
        n = len(o["ids"])
        assert o["visited"] < n, "fixture: the walk did not stop early"
        U = np.sort(o["ub"])[k - 1]
        assert o["visited"] <= int((o["lb"] <= U).sum())
        top = np.lexsort((o["ids"], o["ex"]))[:k]
        np.testing.assert_array_equal(o["out"], o["ids"][top])
        np.testing.assert_array_equal(o["dists"], o["ex"][top])


# --------------------------------------------------------------------------
# Algorithm 4: early re-rank accounting
# --------------------------------------------------------------------------

def test_early_rerank_hand_example():
    """Two lists, nearest first: [1, 2, 3, 4] (ids 0-3) then [0.5, 1.0, 2.5,
    10] (ids 4-7), kc = 4, m = 4, one sample list (it holds 4 >= 1 * kc
    keys).  Codebook: d_min 1, d_max 4, delta 3/256, sample cells 0, 85,
    170, 255, so cells 1-85 map to bucket 1, 86-170 to 2, 171-255 to 3.
    j = ceil(4 * 4 / 8) = 2: the sample's 2nd key is 2.0, in cell 85,
    bucket 1 = tau_pred.  In the second list 0.5 and 1.0 fall in cell 0
    (bucket 0 < 1): early; 2.5 and 10 do not.  Candidates (4 smallest by key,
    id): ids 4, 0, 5, 1, so both early objects are candidates and two
    candidates (ids 0 and 1, from the sample) are re-ranked afterwards."""
    keys = np.array([1, 2, 3, 4, 0.5, 1.0, 2.5, 10], np.float32)
    ids = np.arange(8, dtype=np.int64)
    off = np.array([0, 4, 8], np.int64)
    r = oracle.early_rerank(keys, ids, off, 4, 4, nsample=1, sample_factor=1)
    assert r == dict(tau_pred=1, n_early=2, n_early_cand=2, n_late=2)
    # one bucket: nothing lies below the predicted bucket
    assert oracle.early_rerank(keys, ids, off, 4, 1, nsample=1, sample_factor=1)["n_early"] == 0
    # the sample covers every list: nothing is scanned after it
    r = oracle.early_rerank(keys, ids, off, 4, 4, nsample=2, sample_factor=1)
    assert r["n_early"] == 0 and r["n_late"] == 4


def test_early_rerank_invariants():
    """Early objects lie after the sample and below tau_pred; the useful
    ones plus the late ones are exactly the candidates; a larger candidate
    count never lowers tau_pred."""
    rng = np.random.default_rng(41)
    sizes = rng.integers(20, 200, 12)
    off = np.zeros(13, np.int64)
    off[1:] = np.cumsum(sizes)
    n = int(off[-1])
    # nearest lists first: keys grow with the list rank
    keys = np.concatenate([rng.standard_normal(s) ** 2 + 0.3 * j for j, s in enumerate(sizes)]).astype(np.float32)
    ids = rng.permutation(n).astype(np.int64)
    prev = -1
    for kc in (10, 100, 300, 700):
        r = oracle.early_rerank(keys, ids, off, kc, 64, nsample=2, sample_factor=2)
        assert r["n_early_cand"] <= r["n_early"]
        assert r["n_early_cand"] + r["n_late"] == kc
        assert r["tau_pred"] >= prev
        prev = r["tau_pred"]
        col = oracle.collect_bbc(keys, ids, off, kc, 64, 2, 2)
        ns = 2
        while ns < 12 and off[ns] < 2 * kc:
            ns += 1
        b = np.array([oracle.bucket_of(x, col["dmin"], col["delta"], col["map"]) for x in keys])
        early = np.zeros(n, bool)
        early[off[ns]:] = b[off[ns]:] < r["tau_pred"]
        assert int(early.sum()) == r["n_early"]
        assert int(np.isin(ids[early], col["cand_ids"]).sum()) == r["n_early_cand"]


# --------------------------------------------------------------------------
# the collector's definition against the paper's workflow
# --------------------------------------------------------------------------

def _replay_result_buffer(keys, ids, off, kc, col, m):
    """Algorithm 1 as the paper runs it: Push appends an object whose bucket
    is at most tau, Update refreshes tau after each list (first bucket whose
    running count reaches kc), Collect returns the buckets below tau plus
    the best s of bucket tau."""
    bufs = [[] for _ in range(m)]
    tau = m
    for g in range(len(off) - 1):
        for i in range(off[g], off[g + 1]):
            a = oracle.bucket_of(keys[i], col["dmin"], col["delta"], col["map"])
            if a <= tau:
                bufs[a].append((float(keys[i]), int(ids[i])))
        run = 0
        tau = m
        for b in range(m):
            run += len(bufs[b])
            if run >= kc:
                tau = b
                break
    out = [x for b in range(min(tau, m)) for x in bufs[b]]
    s = kc - len(out)
    if tau < m:
        out += sorted(bufs[tau])[:s]
    return tau, s, sorted(i for _, i in out)


@pytest.mark.parametrize("m", [1, 3, 16, 256])
def test_collect_definition_matches_paper_workflow(m):
    """The threshold bucket refreshed once per list (the paper) ends where
    the single cut over the whole histogram puts it (the oracle and the
    GPU): tau only moves down as keys arrive, and keys dropped by an earlier
    tau lie above the final one.  The collected sets are equal."""
    rng = np.random.default_rng(50 + m)
    for trial in range(5):
        sizes = rng.integers(0, 60, 9)
        off = np.zeros(10, np.int64)
        off[1:] = np.cumsum(sizes)
        n = int(off[-1])
        keys = (rng.integers(0, 30, n) * 0.25).astype(np.float32)  # ties
        ids = rng.permutation(n).astype(np.int64)
        for kc in (1, max(1, n // 4), n):
            col = oracle.collect_bbc(keys, ids, off, kc, m, 2, 2)
            tau, s, cand = _replay_result_buffer(keys, ids, off, min(kc, n), col, m)
            assert (tau, s) == (col["tau"], col["s"])
            np.testing.assert_array_equal(cand, np.sort(col["cand_ids"]))


@pytest.mark.parametrize("metric", [0, 1])
def test_rerank_counts_relations(metric):
    """The re-rank size report (minimal set <= minimal set with the top-k,
    minimal set <= visited <= S, and the visited prefix inside |C| when the
    walk's k-th exact key is at most U) on a small index, L2 and IP."""
    d, n, nlist, nq, k = 64, 2000, 4, 6, 50
    w = synth.small_workload("ivfrabitq_1m_d960", n=n, nlist=nlist, nq=nq, d=d, seed_index=4)
    x, q = synth.base_vectors(w), synth.query_vectors(w)
    if metric:
        q = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)
    tr, ip = synth.kmeans_draws(n, nlist, 64 * nlist, 0)
    ix = oracle.build_ivf_rabitq(x, nlist, tr, ip, synth.rotation_orthogonal(d, 331), metric=metric)
    c = oracle.rerank_counts(ix, q, k, 3)
    assert np.all(c["min"] <= c["min_out"])
    assert np.all(c["min"] <= c["visited"]) and np.all(c["visited"] <= c["S"])
    assert np.all(c["C"] <= c["S"]) and np.all(c["min"] >= 1)
    assert np.mean(c["visited"] <= c["C"]) >= 0.8
