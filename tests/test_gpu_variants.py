"""GPU parity, through the C ABI, of the kernel variants that the large
workloads run, at sizes where they are really taken (not only at small
test sizes): the collector codebook with 48 sample slots per thread and
with the sample read from memory, the final top-k with 24 and 32 candidates
per thread and its memory form, on 8-bit and 4-bit PQ; the RaBitQ walk
resolving its exact stop point outside LDS and the RaBitQ scan on a 1-D
grid (forced by test knobs); and the BF16 probe on adversarial centroids
(duplicates, near-equidistant to a few ulps, norms from 2^-10 to 2^10),
whose probe set must equal the oracle's float32 probe."""
import os

import numpy as np
import pytest

import oracle
import synth
from helpers import check_trace, expected_steps, make_gpu_index, oracle_pq_index

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bbc():
    import paper_2604_01960_amd as b
    b.load()
    return b


@pytest.mark.parametrize("cfg", [
    # (base, n, nlist, M, bits, nq, k, nprobe, ratio, codebook slots, final-top-k items per thread)
    ("ivfpq_100k_d128", 100_000, 64, 16, 8, 6, 8000, 48, 2.5, 48, 24),
    ("ivfpq_100k_d128", 100_000, 64, 16, 8, 6, 12000, 64, 2.5, 0, 32),
    ("ivfpq_100k_d128", 100_000, 64, 16, 8, 5, 16000, 64, 2.5, 0, 0),
    ("ivfpq4_10m_d96", 60_000, 32, 48, 4, 5, 15000, 32, 2.5, 0, 0),
])
def test_large_k_variants_match_oracle(bbc, cfg):
    base, n, nlist, M, bits, nq, k, nprobe, ratio, cb_form, fin_form = cfg
    w, ix, q = oracle_pq_index(base, n, nlist, M, bits, nq)
    print(f"[case] {base} n={n} k={k} nprobe={nprobe} r={ratio} forms=({cb_form},{fin_form})", flush=True)
    g = make_gpu_index(bbc, ix)
    tr = g.search_traced(q, k, nprobe, ratio=ratio, buckets=256, nsample=8)
    assert tr["kernel_forms"][0] == cb_form and tr["kernel_forms"][1] == fin_form, tr["kernel_forms"]
    # the samples and candidate sets really are in the variant's range
    ns = int(tr["n_sample_keys"].max())
    if cb_form == 48:
        assert 32 * 1024 < ns <= 48 * 1024, ns
    elif cb_form == 0:
        assert ns > 48 * 1024, ns
    kc = int(tr["n_cand"].max())
    lo, hi = {24: (16 * 1024, 24 * 1024), 32: (24 * 1024, 32 * 1024), 0: (32 * 1024, 1 << 40)}[fin_form]
    assert lo < kc <= hi, kc
    exp = expected_steps(ix, q, k, nprobe, ratio, 256, 8)
    check_trace(tr, exp, 256)
    g.free()


@pytest.mark.parametrize("lds_cap", ["", "1024"])
def test_final_topk_groups_match_oracle(bbc, lds_cap):
    """A batch above the size from which the final top-k runs one launch per
    kernel form (256 queries, one per CU): per-query k spread so that the
    queries' candidate sets select every form (8, 16, 24 and 32 items per
    thread and the memory form); ids and distances equal the oracle's.  With
    the LDS buffer cut to 1024 results, every result set above it groups its
    winners by bin in the scratch buffer."""
    nq = 300
    w, ix, q = oracle_pq_index("ivfpq_100k_d128", 100_000, 64, 16, 8, nq)
    ks = np.array([500, 3000, 6000, 8000, 12000, 16000], np.int32)
    k = ks[np.arange(nq) % len(ks)]
    print(f"[case] final top-k groups nq={nq} lds_cap={lds_cap or 'default'}", flush=True)
    old = os.environ.get("BBC_FINAL_LDS_CAP")
    if lds_cap:
        os.environ["BBC_FINAL_LDS_CAP"] = lds_cap
    try:
        g = make_gpu_index(bbc, ix)
    finally:
        if old is None:
            os.environ.pop("BBC_FINAL_LDS_CAP", None)
        else:
            os.environ["BBC_FINAL_LDS_CAP"] = old
    got = g.search(q, k, 48, ratio=2.5)
    ref = oracle.search_pq(ix, q, k.astype(np.int64), np.full(nq, 48, np.int64), 2.5)
    np.testing.assert_array_equal(got[3], ref["off"])
    np.testing.assert_array_equal(got[0], ref["ids"])
    np.testing.assert_array_equal(got[1], ref["dists"])
    np.testing.assert_array_equal(got[2], ref["counts"])
    g.free()


@pytest.mark.parametrize("fraction", ["0.6", "0.3", "0.02"])
def test_tighter_filter_matches_oracle(bbc, fraction):
    """The lists after the sample filtered at the upper edge of the cell by
    which the sample's running count reaches fraction * K_c: a query left
    short of K_c keys at or below that bound is scanned again at d_max (at
    0.02 nearly every query is).  Estimated keys, codebook, threshold
    bucket, candidates and results equal the oracle's, for equal and for
    per-query k and nprobe."""
    nq = 24
    w, ix, q = oracle_pq_index("ivfpq_100k_d128", 40_000, 64, 32, 8, nq)
    print(f"[case] tighter filter fraction={fraction} nq={nq}", flush=True)
    old = os.environ.get("BBC_FILTER_FRACTION")
    os.environ["BBC_FILTER_FRACTION"] = fraction
    try:
        g = make_gpu_index(bbc, ix)
    finally:
        if old is None:
            os.environ.pop("BBC_FILTER_FRACTION")
        else:
            os.environ["BBC_FILTER_FRACTION"] = old
    rng = np.random.default_rng(11)
    kk = rng.integers(50, 3000, nq).astype(np.int32)
    npb = rng.integers(4, 33, nq).astype(np.int32)
    for k, nprobe in ((1500, 24), (kk, npb)):
        tr = g.search_traced(q, k, nprobe, ratio=2.0, buckets=256, nsample=3)
        exp = expected_steps(ix, q, k, nprobe, 2.0, 256, 3)
        check_trace(tr, exp, 256)
        got = g.search(q, k, nprobe, ratio=2.0)
        ref = oracle.search_pq(ix, q, np.broadcast_to(np.asarray(k, np.int64), (nq,)),
                               np.broadcast_to(np.asarray(nprobe, np.int64), (nq,)), 2.0)
        np.testing.assert_array_equal(got[0], ref["ids"])
        np.testing.assert_array_equal(got[1], ref["dists"])
    g.free()


@pytest.mark.parametrize("sort", ["1", "0"])
def test_pair_sort_forms_match_oracle(bbc, sort):
    """The (query, rank) pairs sorted by list with per-block LDS histograms
    (1, the default) or device-wide atomics (0): a ragged batch of 70
    queries (blocks of 32 queries, the last one partial) with per-query k
    and nprobe, PQ (the scan's sort by (phase, list) and the re-rank's by
    list) and RaBitQ with tile-major keys (the scan's and re-rank's sort by
    list); ids and distances equal the oracle's."""
    nq = 70
    w, ix, q = oracle_pq_index("ivfpq_100k_d128", 20_000, 64, 16, 8, nq)
    rng = np.random.default_rng(17)
    k = rng.integers(1, 1500, nq).astype(np.int32)
    npb = rng.integers(1, 33, nq).astype(np.int32)
    print(f"[case] pair sort form {sort}: pq nq={nq}", flush=True)
    old = os.environ.get("BBC_PAIR_SORT")
    os.environ["BBC_PAIR_SORT"] = sort
    try:
        g = make_gpu_index(bbc, ix)
    finally:
        if old is None:
            os.environ.pop("BBC_PAIR_SORT")
        else:
            os.environ["BBC_PAIR_SORT"] = old
    got = g.search(q, k, npb, ratio=2.0)
    ref = oracle.search_pq(ix, q, k.astype(np.int64), npb.astype(np.int64), 2.0)
    np.testing.assert_array_equal(got[3], ref["off"])
    np.testing.assert_array_equal(got[0], ref["ids"])
    np.testing.assert_array_equal(got[1], ref["dists"])
    g.free()
    x, q, ix = _rabitq_data(128, 12000, nq, 24)
    print(f"[case] pair sort form {sort}: rabitq tile keys nq={nq}", flush=True)
    g = _rabitq_index(bbc, x, ix, {"BBC_PAIR_SORT": sort, "BBC_WALK_FORM": "3"})
    k = rng.integers(1, 800, nq).astype(np.int32)
    npb = rng.integers(1, 25, nq).astype(np.int32)
    tr = g.search_traced(q, k, npb)
    _check_rabitq(tr, ix, q, k, npb)
    g.free()


def _rabitq_data(d, n, nq, nlist):
    w = synth.small_workload("ivfrabitq_1m_d960", n=n, nlist=nlist, nq=nq, d=d, seed_index=2)
    x, q = synth.base_vectors(w), synth.query_vectors(w)
    tr, ip = synth.kmeans_draws(n, nlist, 64 * nlist, 0)
    P = synth.rotation_orthogonal(d, 302)
    return x, q, oracle.build_ivf_rabitq(x, nlist, tr, ip, P)


def _rabitq_index(bbc, x, ix, env):
    old = {v: os.environ.get(v) for v in env}
    os.environ.update(env)
    try:
        return bbc.Index.create_rabitq(ix["centroids"], ix["list_off"], ix["list_ids"], ix["P"], ix["codes"],
                                       ix["factors"], x, metric=ix["metric"])
    finally:
        for v, o in old.items():
            if o is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = o


def _check_rabitq(tr, ix, q, k, nprobe):
    ref = oracle.search_rabitq(ix, q, k, nprobe, debug=True)
    np.testing.assert_array_equal(tr["probe_lists"], ref["probe_lists"])
    np.testing.assert_array_equal(tr["est_lb"], ref["est_lb"])
    np.testing.assert_array_equal(tr["est_ub"], ref["est_ub"])
    np.testing.assert_array_equal(tr["counts"], ref["counts"])
    np.testing.assert_array_equal(tr["ids"], ref["ids"])
    np.testing.assert_array_equal(tr["dists"], ref["dists"])


@pytest.mark.parametrize("form", ["1", "2"])
def test_rabitq_walk_stop_point_outside_lds(bbc, form):
    """With the walk's LDS capacity for the objects above the k-th exact key
    cut to 2, queries with more of them resolve the exact stop point with
    radix selects in global memory; results equal the oracle's, and the
    default capacity resolves the same queries in LDS.  (The wide form's
    processed prefix is the shortest one, so few of its objects lie above
    the k-th key: the capacity is cut below that count.)"""
    x, q, ix = _rabitq_data(128, 20000, 24, 16)
    k, nprobe = 2500, 16
    print(f"[case] rabitq walk qcap=2 form={form}", flush=True)
    g = _rabitq_index(bbc, x, ix, {"BBC_WALK_QCAP": "2", "BBC_WALK_FORM": form})
    tr = g.search_traced(q, k, nprobe)
    assert np.any(tr["walk_path"] == 2), tr["walk_path"]
    _check_rabitq(tr, ix, q, k, nprobe)
    g.free()
    g = _rabitq_index(bbc, x, ix, {"BBC_WALK_FORM": form})
    tr2 = g.search_traced(q, k, nprobe)
    assert np.all(tr2["walk_path"][tr["walk_path"] == 2] == 1)
    np.testing.assert_array_equal(tr2["ids"], tr["ids"])
    g.free()


def test_rabitq_scan_one_dimensional_grid(bbc):
    """The scan's 1-D grid of (query, rank) pairs (taken for batches beyond
    65535 queries), forced at a small batch: bounds and results unchanged."""
    x, q, ix = _rabitq_data(128, 6000, 9, 12)
    print("[case] rabitq scan 1-D grid", flush=True)
    g = _rabitq_index(bbc, x, ix, {"BBC_RQ_SCAN_1D": "1", "BBC_WALK_FORM": "1"})
    k = np.array([10, 300, 2000, 50, 700, 6000, 1, 90, 400], np.int32)
    npb = np.array([12, 3, 7, 1, 12, 12, 2, 5, 9], np.int32)
    tr = g.search_traced(q, k, npb)
    assert tr["kernel_forms"][2] == 1
    _check_rabitq(tr, ix, q, k, npb)
    g.free()


# --------------------------------------------------------------------------
# BF16 probe on adversarial centroids
# --------------------------------------------------------------------------

def _adversarial_centroids(rng, d, q0):
    """Centroids that attack the BF16 pre-filter's error bound: near-
    equidistant from q0 (sign flips and permutations of one offset, so the
    exact distances agree and float32 keys differ by a few ulps), exact
    duplicates (keys tie, broken by list id), and offsets whose norms span
    2^-10 to 2^10."""
    v = rng.standard_normal(d).astype(np.float32)
    near = []
    for _ in range(40):
        near.append(q0 + rng.permutation(v) * rng.choice([-1.0, 1.0], d).astype(np.float32))
    dup_src = q0 + 1.5 * rng.standard_normal(d).astype(np.float32)
    dups = [dup_src.copy() for _ in range(12)]
    scaled = []
    for e in range(-10, 11):
        u = rng.standard_normal(d).astype(np.float32)
        scaled.append(q0 + np.float32(2.0 ** e) * u / np.linalg.norm(u))
    far = [np.float32(2.0 ** 10) * rng.standard_normal(d).astype(np.float32) for _ in range(8)]
    cent = np.array(near + dups + scaled + far, np.float32)
    return cent[rng.permutation(len(cent))]


def _index_from_centroids(rng, cent, rows_per_list=6):
    nlist, d = cent.shape
    x = (np.repeat(cent, rows_per_list, 0) + 0.01 * rng.standard_normal((nlist * rows_per_list, d))).astype(np.float32)
    a = oracle.kmeans_assign(x, cent)
    order = np.argsort(a, kind="stable").astype(np.int64)
    off = np.zeros(nlist + 1, np.int64)
    off[1:] = np.cumsum(np.bincount(a, minlength=nlist))
    return x, a, order, off


def test_bf16_probe_adversarial_centroids(bbc):
    rng = np.random.default_rng(77)
    d = 64
    q0 = rng.standard_normal(d).astype(np.float32)
    cent = _adversarial_centroids(rng, d, q0)
    x, a, order, off = _index_from_centroids(rng, cent)
    M = 8
    cb = rng.standard_normal((M, 16, d // M)).astype(np.float32)
    codes = oracle.pq_encode(oracle.residuals(x, order, cent, a), cb)
    g = bbc.Index.create_pq(cent, off, order, cb, codes, x)
    qs = np.array([q0, q0 * np.float32(1.0 + 2.0 ** -20), cent[3], cent[10] + np.float32(1e-3),
                   np.float32(2.0 ** 9) * q0, np.float32(2.0 ** -9) * q0], np.float32)
    nlist = cent.shape[0]
    for nprobe in (1, 5, 12, 30, 41, 52, nlist):
        print(f"[case] bf16 probe adversarial nprobe={nprobe}", flush=True)
        tr = g.search_traced(qs, 5, nprobe, ratio=1.0)
        lists, keys, poff = oracle.probe(qs, cent, nprobe)
        np.testing.assert_array_equal(tr["probe_lists"], lists, err_msg=f"nprobe {nprobe}")
        np.testing.assert_array_equal(tr["probe_keys"], keys)
        assert np.all(tr["n_recheck"] >= nprobe)
    g.free()


def test_bf16_probe_adversarial_inner_product(bbc):
    """The same attack under the inner-product metric (RaBitQ index)."""
    rng = np.random.default_rng(78)
    d = 64
    q0 = rng.standard_normal(d).astype(np.float32)
    cent = _adversarial_centroids(rng, d, q0)
    x, a, order, off = _index_from_centroids(rng, cent)
    P = synth.rotation_orthogonal(d, 330)
    codes, fac = oracle.rabitq_encode(x, order, off, cent, P)
    g = bbc.Index.create_rabitq(cent, off, order, P, codes, fac, x, metric=1)
    qs = np.array([q0, -q0, cent[7], np.float32(2.0 ** 8) * q0, np.float32(2.0 ** -8) * cent[20]], np.float32)
    nlist = cent.shape[0]
    for nprobe in (1, 7, 25, 40, nlist):
        print(f"[case] bf16 probe adversarial IP nprobe={nprobe}", flush=True)
        tr = g.search_traced(qs, 5, nprobe)
        lists, keys, poff = oracle.probe(qs, cent, nprobe, metric=1)
        np.testing.assert_array_equal(tr["probe_lists"], lists, err_msg=f"nprobe {nprobe}")
        np.testing.assert_array_equal(tr["probe_keys"], keys)
    g.free()
