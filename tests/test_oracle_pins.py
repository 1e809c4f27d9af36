"""Pins of the oracle against facts fixed outside the oracle itself: the
paper's worked example, exact integer arithmetic, brute force on tiny
inputs, library sorts and closed-form special cases (CPU only)."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def lex_order(keys, ids):
    """Reference total order: numeric key, then smaller id (numpy lexsort)."""
    return np.lexsort((np.asarray(ids), np.asarray(keys)))


# --------------------------------------------------------------------------
# Update / threshold bucket: the paper's worked example (Overview section)
# --------------------------------------------------------------------------

def test_update_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "worked_example_update.json")))
    edges = np.array(g["codebook"])
    m = len(edges) - 1

    def bucket(x):  # B[i] = [c_i, c_{i+1})
        return int(np.searchsorted(edges, x, side="right") - 1)

    counts = np.zeros(m, np.int64)
    for x in g["distances_before"]:
        counts[bucket(x)] += 1
    tau = oracle.update(counts, g["k"])
    assert tau + 1 == g["expected_threshold_bucket_before_1based"]
    assert edges[tau + 1] == g["expected_relaxed_threshold_before"]
    b9 = bucket(g["inserted_distance"])
    assert b9 + 1 == g["expected_bucket_of_inserted_1based"]
    counts[b9] += 1
    tau = oracle.update(counts, g["k"])
    assert tau + 1 == g["expected_threshold_bucket_after_1based"]
    assert edges[tau + 1] == g["expected_relaxed_threshold_after"]


def test_update_below_k_is_infinite():
    assert oracle.update([1, 2, 3], 7) == 3  # m stands for "accept everything"
    assert oracle.update([0, 0, 5], 5) == 2
    assert oracle.update([5, 0, 0], 1) == 0


# --------------------------------------------------------------------------
# canonical arithmetic against exact integer results and float64 bounds
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d", [4, 8, 96, 128, 132, 768, 960, 1024])
def test_canon_l2_ip_exact_on_integers(d):
    rng = np.random.default_rng(d)
    for _ in range(20):
        a = rng.integers(-8, 9, d)
        b = rng.integers(-8, 9, d)
        assert float(oracle.canon_l2(a, b)) == float(((a - b) ** 2).sum())
        assert float(oracle.canon_ip(a, b)) == float((a * b).sum())


@pytest.mark.parametrize("d", [96, 128, 960])
def test_canon_l2_within_rounding_bound(d):
    rng = np.random.default_rng(7)
    for _ in range(50):
        a = rng.standard_normal(d).astype(np.float32)
        b = rng.standard_normal(d).astype(np.float32)
        ex = float(((a.astype(np.float64) - b) ** 2).sum())
        got = float(oracle.canon_l2(a, b))
        # sum of d non-negative terms, each rounded twice, depth <= d/4+6
        assert abs(got - ex) <= (d + 16) * 2.0 ** -23 * ex


# --------------------------------------------------------------------------
# collector: the definition (first kc of (key, id)) and the result buffer
# --------------------------------------------------------------------------

def test_topk_sort_matches_lexsort():
    rng = np.random.default_rng(1)
    keys = rng.integers(0, 20, 500).astype(np.float32)  # heavy ties
    ids = rng.permutation(500).astype(np.int64)
    order = lex_order(keys, ids)
    for kc in (1, 37, 499, 500, 600):
        k_, i_ = oracle.topk_sort(keys, ids, kc)
        np.testing.assert_array_equal(i_, ids[order][:kc])
        np.testing.assert_array_equal(k_, keys[order][:kc])


def _grouped_keys(rng, ngrp, heavy_ties):
    sizes = rng.integers(0, 120, ngrp)
    sizes[rng.integers(0, ngrp)] = 0
    n = int(sizes.sum())
    if heavy_ties:
        keys = rng.integers(0, 9, n).astype(np.float32) * np.float32(0.5)
    else:
        keys = (rng.standard_normal(n) ** 2 * 3 + 10).astype(np.float32)
    ids = rng.permutation(n).astype(np.int64) * 3 + 1
    off = np.zeros(ngrp + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    return keys, ids, off


@pytest.mark.parametrize("m", [1, 2, 8, 80, 256])
@pytest.mark.parametrize("ties", [False, True])
def test_collect_equals_definition(m, ties):
    rng = np.random.default_rng(100 * m + ties)
    for trial in range(6):
        keys, ids, off = _grouped_keys(rng, 12, ties)
        n = int(off[-1])
        for kc in {1, max(1, n // 3), n - 1, n, n + 5}:
            if kc < 1:
                continue
            for ns in (1, 3, 100):
                r = oracle.collect_bbc(keys, ids, off, kc, m, ns)
                want_k, want_i = oracle.topk_sort(keys, ids, kc)
                got = np.sort(r["cand_ids"])
                np.testing.assert_array_equal(got, np.sort(want_i))
                # the superset (buckets <= tau) contains the exact top-kc
                b = np.array([oracle.bucket_of(x, r["dmin"], r["delta"], r["map"]) for x in keys])
                sup = set(ids[b <= r["tau"]].tolist())
                assert set(want_i.tolist()) <= sup
                # counts histogram all keys; tau is the first bucket reaching kc
                np.testing.assert_array_equal(r["counts"], np.bincount(b, minlength=m))
                kk = min(kc, n)
                assert oracle.update(r["counts"], kk) == r["tau"]
                assert r["s"] == kk - int(r["counts"][:r["tau"]].sum())


def test_collect_invariant_under_codebook():
    """Any monotone bucket map yields the same candidates (the codebook only
    affects speed): vary the sample size and the number of buckets."""
    rng = np.random.default_rng(5)
    keys, ids, off = _grouped_keys(rng, 20, False)
    kc = int(off[-1]) // 4
    ref = None
    for m in (1, 3, 17, 256):
        for ns in (1, 2, 7, 20):
            for sf in (1, 2, 3):
                got = np.sort(oracle.collect_bbc(keys, ids, off, kc, m, ns, sf)["cand_ids"])
                if ref is None:
                    ref = got
                np.testing.assert_array_equal(got, ref)


def test_codebook_equal_depth():
    rng = np.random.default_rng(9)
    keys = (rng.standard_normal(5000) ** 2 + 4).astype(np.float32)
    ids = np.arange(5000, dtype=np.int64)
    for m in (4, 32, 100, 256):
        for kc in (100, 1000, 5000):
            dmin, delta, mp = oracle.codebook(keys, ids, kc, m)
            top_k, _ = oracle.topk_sort(keys, ids, kc)
            assert dmin == top_k[0]
            assert np.all(np.diff(mp.astype(int)) >= 0) and mp[0] == 0 and mp.max() < m
            cells = np.array([oracle.cell_of(x, dmin, delta) for x in top_k])
            assert cells.max() == 255 or top_k[-1] == top_k[0]
            per_cell = np.bincount(cells, minlength=256)
            per_bucket = np.bincount(mp[cells], minlength=m)
            assert per_bucket.max() <= np.ceil(kc / m) + per_cell.max()


# --------------------------------------------------------------------------
# probe, PQ tables and keys on exactly representable data
# --------------------------------------------------------------------------

def test_probe_integer_exact():
    rng = np.random.default_rng(3)
    c = rng.integers(-3, 4, (40, 12)).astype(np.float32)
    q = rng.integers(-3, 4, (9, 12)).astype(np.float32)
    for npb in (1, 5, 40):
        lists, keys, off = oracle.probe(q, c, npb)
        for i in range(len(q)):
            exact = ((q[i].astype(np.int64) - c.astype(np.int64)) ** 2).sum(1)
            want = lex_order(exact, np.arange(40))[:npb]
            np.testing.assert_array_equal(lists[off[i]:off[i + 1]], want)
            np.testing.assert_array_equal(keys[off[i]:off[i + 1]], exact[want])


@pytest.mark.parametrize("M,bits", [(4, 8), (8, 4), (16, 8)])
def test_pq_table_and_key_integer_exact(M, bits):
    d, ksub = 32, 1 << bits
    rng = np.random.default_rng(M + bits)
    q = rng.integers(-4, 5, d).astype(np.float32)
    cen = rng.integers(-4, 5, d).astype(np.float32)
    cb = rng.integers(-4, 5, (M, ksub, d // M)).astype(np.float32)
    lut = oracle.pq_lut(q, cen, cb, M, ksub)
    r = (q - cen).astype(np.int64).reshape(M, 1, d // M)
    want = ((r - cb.astype(np.int64)) ** 2).sum(-1)
    np.testing.assert_array_equal(lut, want.astype(np.float32))
    codes = rng.integers(0, ksub, (50, M)).astype(np.uint8)
    keys = oracle.pq_keys(lut, codes)
    recon = cb[np.arange(M)[None, :], codes].reshape(50, d).astype(np.int64)  # reconstructed residuals
    want_k = ((q.astype(np.int64) - cen - recon) ** 2).sum(1)
    np.testing.assert_array_equal(keys, want_k.astype(np.float32))


def test_pq_adc_identity_single_subspace():
    """M = 1, centroid 0 and a query equal to codeword b*: the residual is the
    codeword, its table entry is exactly 0 and every other entry is the
    squared distance between the two codewords."""
    rng = np.random.default_rng(11)
    d = 8
    cb = rng.standard_normal((1, 16, d)).astype(np.float32)
    cen = np.zeros(d, np.float32)
    b_star = 5
    q = cb[0, b_star].copy()
    lut = oracle.pq_lut(q, cen, cb, 1, 16)
    assert lut[0, b_star] == 0.0
    ex = ((q.astype(np.float64) - cb[0].astype(np.float64)) ** 2).sum(1)
    np.testing.assert_allclose(lut[0], ex, rtol=1e-6)
    assert np.all(np.delete(lut[0], b_star) > 0)


# --------------------------------------------------------------------------
# index build steps
# --------------------------------------------------------------------------

def test_kmeans_assign_integer_bruteforce():
    rng = np.random.default_rng(2)
    x = rng.integers(-5, 6, (300, 16)).astype(np.float32)
    c = rng.integers(-5, 6, (17, 16)).astype(np.float32)
    got = oracle.kmeans_assign(x, c)
    dist = ((x[:, None, :].astype(np.int64) - c[None].astype(np.int64)) ** 2).sum(-1)
    np.testing.assert_array_equal(got, dist.argmin(1))  # argmin: first (smallest id) on ties


def test_kmeans_converges_to_exact_means():
    """Separated dyadic clusters: sums are exact in float64, so the trained
    centroids must be exactly the float32-rounded cluster means."""
    rng = np.random.default_rng(4)
    centers = np.array([[0, 0], [100, 0], [0, 100], [100, 100]], np.float64)
    lab = rng.integers(0, 4, 400)
    x = (centers[lab] + rng.integers(-16, 17, (400, 2)) / 8.0).astype(np.float32)
    x = np.pad(x, ((0, 0), (0, 2)))
    init = np.array([np.flatnonzero(lab == j)[0] for j in range(4)])
    cent = oracle.kmeans_train(x, np.arange(400), init, 4, 5)
    for j in range(4):
        want = x[lab == j].astype(np.float64).mean(0).astype(np.float32)
        np.testing.assert_array_equal(cent[j], want)


def test_kmeans_refills_empty_clusters():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((500, 8)).astype(np.float32)
    # two identical seeds: one of them is empty after the first assignment
    x[1] = x[0]
    cent = oracle.kmeans_train(x, np.arange(500), np.array([0, 1, 2, 3, 4]), 5, 4)
    a = oracle.kmeans_assign(x, cent)
    assert len(np.unique(a)) == 5


def test_pq_encode_bruteforce():
    rng = np.random.default_rng(8)
    r = rng.integers(-4, 5, (200, 24)).astype(np.float32)
    cb = rng.integers(-4, 5, (6, 16, 4)).astype(np.float32)
    got = oracle.pq_encode(r, cb)
    sub = r.reshape(200, 6, 1, 4).astype(np.int64)
    dist = ((sub - cb[None].astype(np.int64)) ** 2).sum(-1)
    np.testing.assert_array_equal(got, dist.argmin(-1))


# --------------------------------------------------------------------------
# end to end
# --------------------------------------------------------------------------

def _manual_integer_index(rng, n=600, d=16, nlist=6, M=4, bits=4):
    x = rng.integers(0, 4, (n, d)).astype(np.float32)
    cent = rng.integers(0, 4, (nlist, d)).astype(np.float32)
    assign = oracle.kmeans_assign(x, cent)
    order = np.argsort(assign, kind="stable").astype(np.int64)
    off = np.zeros(nlist + 1, np.int64)
    off[1:] = np.cumsum(np.bincount(assign, minlength=nlist))
    ksub = 1 << bits
    cb = rng.integers(-2, 3, (M, ksub, d // M)).astype(np.float32)
    codes = oracle.pq_encode(oracle.residuals(x, order, cent, assign), cb)
    return dict(kind="pq", n=n, d=d, nlist=nlist, M=M, ksub=ksub, bits=bits, metric=0, centroids=cent,
                assign=assign, list_off=off, list_ids=order, codes=codes, codebook=cb, base=x)


def test_search_full_probe_equals_exhaustive_integer():
    """nprobe = nlist and r*k >= n: the path re-ranks every object, so its
    output must be the exhaustive exact kNN, ties by id, bit for bit."""
    rng = np.random.default_rng(12)
    ix = _manual_integer_index(rng)
    q = rng.integers(0, 4, (7, 16)).astype(np.float32)
    n = ix["n"]
    for k in (1, 50, n, n + 10):
        res = oracle.search_pq(ix, q, k, ix["nlist"], float(n) + 1.0)
        for i in range(len(q)):
            dist = ((ix["base"].astype(np.int64) - q[i].astype(np.int64)) ** 2).sum(1)
            order = lex_order(dist, np.arange(n))
            cnt = min(k, n)
            s = slice(res["off"][i], res["off"][i + 1])
            assert res["counts"][i] == cnt
            np.testing.assert_array_equal(res["ids"][s][:cnt], order[:cnt])
            np.testing.assert_array_equal(res["dists"][s][:cnt], dist[order[:cnt]].astype(np.float32))
            assert np.all(res["ids"][s][cnt:] == -1) and np.all(np.isinf(res["dists"][s][cnt:]))


def test_search_candidates_are_topk_of_estimates():
    rng = np.random.default_rng(13)
    ix = _manual_integer_index(rng, n=800, d=16, nlist=8)
    q = rng.integers(0, 4, (5, 16)).astype(np.float32)
    res = oracle.search_pq(ix, q, 40, 3, 2.5, debug=True)
    for i in range(len(q)):
        lists = res["probe_lists"][res["probe_off"][i]:res["probe_off"][i + 1]]
        keys, ids = [], []
        for j in lists:
            lut = oracle.pq_lut(q[i], ix["centroids"][j], ix["codebook"], ix["M"], ix["ksub"])
            sl = slice(ix["list_off"][j], ix["list_off"][j + 1])
            keys.append(oracle.pq_keys(lut, ix["codes"][sl]))
            ids.append(ix["list_ids"][sl])
        keys, ids = np.concatenate(keys), np.concatenate(ids)
        kc = int(res["n_cand"][i])
        assert res["n_scanned"][i] == len(keys) and kc == min(len(keys), 100)
        order = lex_order(keys, ids)[:kc]
        c = slice(res["cand_off"][i], res["cand_off"][i] + kc)
        np.testing.assert_array_equal(res["cand_ids"][c], ids[order])


def test_exact_knn64_bruteforce():
    rng = np.random.default_rng(14)
    x = rng.standard_normal((400, 12)).astype(np.float32)
    q = rng.standard_normal((3, 12)).astype(np.float32)
    ids, dists = oracle.exact_knn64(x, q, 25)
    for i in range(3):
        dd = ((x.astype(np.float64) - q[i].astype(np.float64)) ** 2).sum(1)
        order = lex_order(dd, np.arange(400))[:25]
        np.testing.assert_array_equal(ids[i], order)
        np.testing.assert_allclose(dists[i], dd[order], rtol=1e-12)


def test_float_pipeline_against_fp64_ground_truth():
    """Continuous data, full probe and full re-rank: float32 results agree with
    the float64 ground truth up to near-ties (distances within 1e-5)."""
    w = synth.small_workload("ivfpq_100k_d128", n=3000, nlist=8, nq=4)
    x = synth.base_vectors(w)
    q = synth.query_vectors(w)
    tr, ip = synth.kmeans_draws(w.n, w.nlist, 64 * w.nlist, 0)
    pr, pi = synth.pq_draws(w.n, 16, 256, 2000, 0)
    ix = oracle.build_ivf_pq(x, w.nlist, 16, 8, tr, ip, pr, pi, 4)
    res = oracle.search_pq(ix, q, 200, w.nlist, 3000.0)
    gi, gd = oracle.exact_knn64(x, q, 200)
    for i in range(len(q)):
        s = slice(res["off"][i], res["off"][i + 1])
        np.testing.assert_allclose(res["dists"][s], gd[i], rtol=1e-5)
        assert len(np.intersect1d(res["ids"][s], gi[i])) >= 198
