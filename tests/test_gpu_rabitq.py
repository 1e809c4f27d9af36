"""GPU parity of the RaBitQ path against the oracle through the C ABI: the
index build (rotation, codes, factors), every object's estimated key and
bounds, and the bounded re-rank's final ids and distances (L2 and IP,
float32 and float16 rows, uneven k / nprobe, and the item-by-item walk
taken when the bin walk's checks fail)."""
import functools

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bbc():
    import paper_2604_01960_amd as b
    b.load()
    return b


@functools.lru_cache(maxsize=8)
def _data(d, n, nq, nlist, metric, fp16=False, seed_index=2):
    w = synth.small_workload("ivfrabitq_1m_d960", n=n, nlist=nlist, nq=nq, d=d, seed_index=seed_index)
    x = synth.base_vectors(w)
    q = synth.query_vectors(w)
    if metric == 1:
        x = (x / np.linalg.norm(x, axis=1, keepdims=True)).astype(np.float32)
        q = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)
    if fp16:
        x = x.astype(np.float16)
    tr, ip = synth.kmeans_draws(n, nlist, 64 * nlist, 0)
    P = synth.rotation_orthogonal(d, 300 + seed_index)
    ix = oracle.build_ivf_rabitq(x, nlist, tr, ip, P, metric=metric)
    return x, q, tr, ip, P, ix


FORMS = {"per_query": "1", "wide": "2", "tiles": "3"}


def _gpu_index(bbc, x, ix, eps0=0.0, form="per_query"):
    """The re-rank form (one block per query, or the exact keys of all
    candidates first, by a device-wide grid or tile-major from rows staged
    once per group of queries) is fixed when the index is made."""
    import os
    old = os.environ.get("BBC_WALK_FORM")
    os.environ["BBC_WALK_FORM"] = FORMS[form]
    try:
        return bbc.Index.create_rabitq(ix["centroids"], ix["list_off"], ix["list_ids"], ix["P"], ix["codes"],
                                       ix["factors"], x, metric=ix["metric"], eps0=eps0)
    finally:
        if old is None:
            del os.environ["BBC_WALK_FORM"]
        else:
            os.environ["BBC_WALK_FORM"] = old


def _check_search(g, ix, q, k, nprobe, eps0=oracle.RABITQ_EPS0):
    tr = g.search_traced(q, k, nprobe)
    ref = oracle.search_rabitq(ix, q, k, nprobe, eps0=eps0, debug=True)
    np.testing.assert_array_equal(tr["probe_lists"], ref["probe_lists"])
    np.testing.assert_array_equal(tr["probe_keys"], ref["probe_keys"])
    np.testing.assert_array_equal(tr["n_scanned"], ref["n_scanned"])
    np.testing.assert_array_equal(tr["est_keys"], ref["est_key"])
    np.testing.assert_array_equal(tr["est_lb"], ref["est_lb"])
    np.testing.assert_array_equal(tr["est_ub"], ref["est_ub"])
    np.testing.assert_array_equal(tr["counts"], ref["counts"])
    np.testing.assert_array_equal(tr["ids"], ref["ids"])
    np.testing.assert_array_equal(tr["dists"], ref["dists"])
    # the bin walk re-ranks whole bins: at least what the item walk visits
    assert np.all(tr["n_visited"] >= np.minimum(ref["n_visited"], tr["n_scanned"]) - 0)
    return tr, ref


@pytest.mark.parametrize("run_list", ["1", "0"])
def test_tile_runs_listed_or_searched(bbc, run_list):
    """Tile-major exact keys with half-precision rows of 64 dimensions (512
    rows per tile, so a pair holds up to 8 runs of 64 candidates in a tile):
    300 queries over 6 lists of about 2000 rows with large k put more than
    1024 runs in most tiles.  The waves claim runs from the tile's list when
    they fit it and otherwise find each run's pair by binary search;
    BBC_RERANK_RUN_LIST=0 takes the search for every tile.  Results equal
    the oracle's either way."""
    import os
    x, q, tr, ip, P, ix = _data(64, 12000, 300, 6, 0, True)
    print(f"[case] rabitq tile runs d=64 fp16 nq=300 run_list={run_list}", flush=True)
    old = os.environ.get("BBC_RERANK_RUN_LIST")
    os.environ["BBC_RERANK_RUN_LIST"] = run_list
    try:
        g = _gpu_index(bbc, x, ix, form="tiles")
    finally:
        if old is None:
            os.environ.pop("BBC_RERANK_RUN_LIST")
        else:
            os.environ["BBC_RERANK_RUN_LIST"] = old
    rng = np.random.default_rng(5)
    k = rng.integers(2000, 6000, 300).astype(np.int32)
    _check_search(g, ix, q, k, 6)


@pytest.mark.parametrize("d", [128, 960])
def test_gpu_build_matches_oracle(bbc, d):
    n = 6000 if d == 128 else 2500
    x, q, tr, ip, P, ix = _data(d, n, 4, 12, 0)
    print(f"[case] rabitq build d={d} n={n}", flush=True)
    g = bbc.Index.build_rabitq(x, 12, tr, ip, P)
    np.testing.assert_array_equal(g.get(bbc.FIELD_CENTROIDS), ix["centroids"])
    np.testing.assert_array_equal(g.get(bbc.FIELD_LIST_IDS), ix["list_ids"])
    np.testing.assert_array_equal(g.get(bbc.FIELD_RABITQ_CODES), ix["codes"])
    np.testing.assert_array_equal(g.get(bbc.FIELD_RABITQ_FACTORS), ix["factors"])
    np.testing.assert_array_equal(g.get(bbc.FIELD_ROT_CENTROIDS), ix["rot_centroids"])


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("cfg", [
    # (d, n, nq, nlist, metric, fp16, k, nprobe)
    (128, 6000, 8, 12, 0, False, 200, 4),
    (960, 2500, 5, 8, 0, False, 300, 3),
    (256, 5000, 6, 10, 1, True, 250, 3),
])
def test_bounds_and_results_match_oracle(bbc, cfg, form):
    d, n, nq, nlist, metric, fp16, k, nprobe = cfg
    x, q, tr, ip, P, ix = _data(d, n, nq, nlist, metric, fp16)
    print(f"[case] rabitq search d={d} metric={metric} fp16={fp16} k={k} nprobe={nprobe} form={form}", flush=True)
    g = _gpu_index(bbc, x, ix, form=form)
    _check_search(g, ix, q, k, nprobe)


@pytest.mark.parametrize("form", list(FORMS))
def test_uneven_and_edge_cases(bbc, form):
    x, q, tr, ip, P, ix = _data(128, 6000, 8, 12, 0)
    g = _gpu_index(bbc, x, ix, form=form)
    k = np.array([1, 7, 64, 500, 6000, 40, 2000, 9000], np.int32)
    npb = np.array([1, 12, 2, 5, 12, 1, 3, 4], np.int32)
    print("[case] rabitq uneven", flush=True)
    tr, ref = _check_search(g, ix, q, k, npb)
    assert np.all(tr["ids"][tr["off"][-2] + tr["counts"][-1]:] == -1)  # k > S pads


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("eps0", [0.05, 0.4])
def test_narrow_bounds_take_the_exact_walk(bbc, eps0, form):
    """With narrow bounds many fail, so the bin walk's checks fail and the
    item-by-item walk must still return the oracle's result."""
    x, q, tr, ip, P, ix = _data(128, 6000, 8, 12, 0)
    g = _gpu_index(bbc, x, ix, eps0=eps0, form=form)
    print(f"[case] rabitq eps0={eps0} form={form}", flush=True)
    _check_search(g, ix, q, 150, 4, eps0=eps0)


def test_device_io_and_repeat(bbc):
    import torch
    x, q, tr, ip, P, ix = _data(256, 5000, 6, 10, 1, True)
    g = _gpu_index(bbc, x, ix)
    a = g.search(q, 250, 3)
    b = g.search(q, 250, 3)
    for u, v in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(u, v)
    ids, dists, counts, off = g.search(torch.from_numpy(q).cuda(), 250, 3)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ids.cpu().numpy(), a[0])
    np.testing.assert_array_equal(dists.cpu().numpy(), a[1])


@pytest.mark.parametrize("sort", ["walk", "cand_sort", "cand_sort_ranges"])
def test_tile_keys_many_queries(bbc, sort):
    """Tile-major exact keys with more queries per list than one group of
    pairs holds (several groups per list), one wave per candidate row.  The
    candidates reach tile order from the walk's bin pass (slot order), or
    from the candidate sort, with all bins counted at once or, with the bin
    counters cut to one list's tiles, each query's ranks in ranges."""
    import os
    x, q, tr, ip, P, ix = _data(256, 5000, 200, 10, 1, True)
    env = {"walk": {}, "cand_sort": {"BBC_WALK_PRESORT": "0"},
           "cand_sort_ranges": {"BBC_WALK_PRESORT": "0", "BBC_RERANK_SORT_BINS": "1"}}[sort]
    os.environ.update(env)
    try:
        g = _gpu_index(bbc, x, ix, form="tiles")
    finally:
        for v in env:
            os.environ.pop(v, None)
    print(f"[case] rabitq tile keys, 200 queries, sort={sort}", flush=True)
    _check_search(g, ix, q, 120, 8)


@pytest.mark.parametrize("alpha", ["0", "0.8", "1"])
@pytest.mark.parametrize("form", ["wide", "tiles"])
@pytest.mark.parametrize("d,metric", [(128, 0), (256, 1)])
def test_wide_form_two_rounds(bbc, alpha, form, d, metric):
    """The wide form's exact keys in two rounds: the first round computes C's
    lower-bound bins up to alpha of the way from the k-th lb to U, the walk
    settles the queries whose stop point lies inside them, and the others get
    the rest of C and a second walk.  Results equal the oracle's for every
    alpha (0: the first round holds only the bins up to the k-th lb, so most
    queries take the second round; 1: one round over all of C), and the keys
    computed never exceed |C| (fewer than |C| for most queries at 0.8: on
    this data the stop point lies 0.45 to 0.76 of the way, in bins)."""
    import os
    x, q, tr, ip, P, ix = _data(d, 12000, 16, 16, metric)
    print(f"[case] two rounds d={d} metric={metric} form={form} alpha={alpha}", flush=True)
    old = os.environ.get("BBC_WALK_ALPHA")
    os.environ["BBC_WALK_ALPHA"] = alpha
    try:
        g = _gpu_index(bbc, x, ix, eps0=oracle.RABITQ_EPS0, form=form)
    finally:
        if old is None:
            del os.environ["BBC_WALK_ALPHA"]
        else:
            os.environ["BBC_WALK_ALPHA"] = old
    rng = np.random.default_rng(int(float(alpha) * 10) + d)
    k = rng.integers(1, 3000, q.shape[0]).astype(np.int32)
    npb = rng.integers(1, 17, q.shape[0]).astype(np.int32)
    tr_ = g.search_traced(q, k, npb)
    ref = oracle.search_rabitq(ix, q, k, npb, debug=True)
    np.testing.assert_array_equal(tr_["counts"], ref["counts"])
    np.testing.assert_array_equal(tr_["ids"], ref["ids"])
    np.testing.assert_array_equal(tr_["dists"], ref["dists"])
    # keys computed against |C| = objects with lb <= the k-th smallest ub
    nC = np.zeros(q.shape[0], np.int64)
    for i in range(q.shape[0]):
        sl = slice(ref["est_off"][i], ref["est_off"][i + 1])
        lb, ub = ref["est_lb"][sl], ref["est_ub"][sl]
        nC[i] = len(lb) if len(lb) <= k[i] else int(np.sum(lb <= np.partition(ub, k[i] - 1)[k[i] - 1]))
    assert np.all(tr_["n_visited"] <= nC)
    if alpha == "1":
        np.testing.assert_array_equal(tr_["n_visited"], nC)
    if alpha == "0.8":
        assert np.mean(tr_["n_visited"] < nC) >= 0.5
    g.free()
