"""Pins of O_64, the oracle's float64 shadow of the query paths (used to
report distance error and recall against float64, never for parity):
exact agreement with the float32 oracle where every value is an integer,
and with float64 exhaustive kNN where the path degenerates to it (CPU)."""
import numpy as np
import pytest

import oracle
import synth


def _integer_pq_index(rng, n=700, d=16, nlist=7, M=4, bits=4):
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


def test_pq64_equals_fp32_oracle_on_integers():
    """Integer data and codebooks: every table entry, key and distance is an
    integer below 2^24, exact in both precisions, so the two paths must give
    the same ids (ties by id) and the same distances, with partial probes and
    partial candidate sets."""
    rng = np.random.default_rng(31)
    ix = _integer_pq_index(rng)
    q = rng.integers(0, 4, (9, 16)).astype(np.float32)
    for k, npb, r in ((20, 2, 1.5), (150, 4, 2.0), (900, 7, 1.0)):
        a = oracle.search_pq(ix, q, k, npb, r)
        b = oracle.search_pq64(ix, q, k, npb, r)
        np.testing.assert_array_equal(a["counts"], b["counts"])
        np.testing.assert_array_equal(a["ids"], b["ids"])
        np.testing.assert_array_equal(a["dists"].astype(np.float64), b["dists"])


def test_pq64_full_probe_is_exhaustive_knn():
    """nprobe = nlist and r*k >= n re-rank every object: O_64 is then the
    float64 exhaustive kNN, ids and distances."""
    w = synth.small_workload("ivfpq_100k_d128", n=2500, nlist=6, nq=4)
    x, q = synth.base_vectors(w), synth.query_vectors(w)
    tr, ip = synth.kmeans_draws(w.n, w.nlist, 64 * w.nlist, 0)
    pr, pi = synth.pq_draws(w.n, 16, 256, 2000, 0)
    ix = oracle.build_ivf_pq(x, w.nlist, 16, 8, tr, ip, pr, pi, 3)
    res = oracle.search_pq64(ix, q, 300, w.nlist, 2500.0)
    gi, gd = oracle.exact_knn64(x, q, 300)
    for i in range(len(q)):
        s = slice(res["off"][i], res["off"][i + 1])
        np.testing.assert_array_equal(res["ids"][s], gi[i])
        np.testing.assert_allclose(res["dists"][s], gd[i], rtol=1e-13)


def test_pq64_and_fp32_agree_up_to_rounding():
    """Continuous data at a partial probe: the float32 path differs from O_64
    only where float32 rounding reorders near-ties, and its distances are
    within float32 rounding of O_64's."""
    w = synth.small_workload("ivfpq_100k_d128", n=6000, nlist=16, nq=6)
    x, q = synth.base_vectors(w), synth.query_vectors(w)
    tr, ip = synth.kmeans_draws(w.n, w.nlist, 64 * w.nlist, 0)
    pr, pi = synth.pq_draws(w.n, 16, 256, 4000, 0)
    ix = oracle.build_ivf_pq(x, w.nlist, 16, 8, tr, ip, pr, pi, 4)
    a = oracle.search_pq(ix, q, 400, 5, 2.0)
    b = oracle.search_pq64(ix, q, 400, 5, 2.0)
    same = np.mean(a["ids"] == b["ids"])
    assert same > 0.97, same
    inter = np.mean([len(np.intersect1d(a["ids"][a["off"][i]:a["off"][i + 1]], b["ids"][b["off"][i]:b["off"][i + 1]]))
                     for i in range(len(q))]) / 400
    assert inter > 0.995, inter
    np.testing.assert_allclose(np.sort(a["dists"].astype(np.float64)), np.sort(b["dists"]), rtol=2e-6)


def _rabitq(d, n, nq, nlist, metric=0):
    w = synth.small_workload("ivfrabitq_1m_d960", n=n, nlist=nlist, nq=nq, d=d, seed_index=2)
    x, q = synth.base_vectors(w), synth.query_vectors(w)
    if metric == 1:
        x = (x / np.linalg.norm(x, axis=1, keepdims=True)).astype(np.float32)
        q = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)
    tr, ip = synth.kmeans_draws(n, nlist, 64 * nlist, 0)
    P = synth.rotation_orthogonal(d, 310)
    return x, q, oracle.build_ivf_rabitq(x, nlist, tr, ip, P, metric=metric)


@pytest.mark.parametrize("metric", [0, 1])
def test_rabitq64_wide_bounds_is_exhaustive_knn(metric):
    """Bounds wide enough to visit everything over all lists: O_64 returns
    the float64 exhaustive kNN (L2) / maximum inner products (IP)."""
    x, q, ix = _rabitq(64, 900, 3, 4, metric)
    r = oracle.search_rabitq64(ix, q, 120, 4, eps0=1e6)
    gi, gd = oracle.exact_knn64(x, q, 120, metric)
    for i in range(len(q)):
        s = slice(r["off"][i], r["off"][i + 1])
        np.testing.assert_array_equal(r["ids"][s], gi[i])
        np.testing.assert_allclose(r["dists"][s], gd[i], rtol=1e-13)
    assert np.all(r["n_visited"] == 900)


def test_rabitq64_close_to_fp32_oracle():
    """At the default confidence the float64 walk and the float32 walk
    return nearly the same ids (they differ only where rounding moves a bound
    or reorders a near-tie), with distances within float32 rounding."""
    x, q, ix = _rabitq(128, 4000, 6, 8)
    a = oracle.search_rabitq(ix, q, 200, 3)
    b = oracle.search_rabitq64(ix, q, 200, 3)
    inter = np.mean([len(np.intersect1d(a["ids"][a["off"][i]:a["off"][i + 1]], b["ids"][b["off"][i]:b["off"][i + 1]]))
                     for i in range(len(q))]) / 200
    assert inter > 0.995, inter
    common = a["ids"] == b["ids"]
    np.testing.assert_allclose(a["dists"][common].astype(np.float64), b["dists"][common], rtol=2e-6)
