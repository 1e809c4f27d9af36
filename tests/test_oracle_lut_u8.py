"""Pins of the oracle's one-byte PQ tables with integer sums (row f2): the
quantizer is pinned on tables that lie on an exact grid (every step exact,
so the one-byte key must equal the float32 key bit for bit), by its error
bound on random tables, by monotonicity, by the degenerate constant table,
and end to end by the exhaustive special case (all lists probed and every
object a candidate gives the exact k nearest)."""
import numpy as np
import pytest

import oracle
import synth


def _grid_table(rng, M, ksub, step):
    """lut[m][b] = lo_m + k[m][b] * step with integer k in [0, 255] (sub-space 0
    spans the whole range), lo_m and step dyadic: every float32 operation of
    the quantizer and of both key sums is exact."""
    k = rng.integers(0, 256, (M, ksub))
    k[0, 0], k[0, 1] = 0, 255
    for m in range(1, M):
        k[m, rng.integers(ksub)] = 0          # each sub-space reaches its low end
    lo = rng.integers(-64, 64, M) * 0.0625
    lut = (lo[:, None] + k * step).astype(np.float32)
    return lut, k


@pytest.mark.parametrize("M,ksub,step", [(16, 256, 0.25), (48, 16, 0.5), (4, 16, 2.0 ** -6), (32, 256, 1.0)])
def test_grid_table_quantizes_exactly(M, ksub, step):
    rng = np.random.default_rng(M * 131 + ksub)
    lut, k = _grid_table(rng, M, ksub, step)
    u, base, delta = oracle.pq_lut_u8(lut)
    assert delta == np.float32(step)
    np.testing.assert_array_equal(u, k.astype(np.uint8))
    lo = lut.min(1).astype(np.float64)
    assert base == np.float32(lo.sum())
    codes = rng.integers(0, ksub, (300, M)).astype(np.uint8)
    ku8 = oracle.pq_keys_u8(u, base, delta, codes)
    kf = oracle.pq_keys(lut, codes)
    np.testing.assert_array_equal(ku8, kf)


def test_error_bound_on_random_tables():
    rng = np.random.default_rng(11)
    for M, ksub in ((32, 256), (48, 16), (16, 256)):
        lut = (rng.gamma(2.0, 3.0, (M, ksub)) * rng.uniform(0.2, 5.0, (M, 1))).astype(np.float32)
        u, base, delta = oracle.pq_lut_u8(lut)
        lo = lut.min(1)
        span = float((lut.max(1) - lo).max())
        assert abs(float(delta) - span / 255.0) <= 1e-6 * span
        # per entry: within half a step (plus float32 rounding of the steps)
        rec = lo[:, None].astype(np.float64) + u.astype(np.float64) * float(delta)
        err = np.abs(rec - lut.astype(np.float64))
        assert err.max() <= 0.5 * float(delta) + 4e-6 * float(np.abs(lut).max())
        # the widest sub-space uses the full code range, every sub-space's minimum is 0
        assert u.min(1).max() == 0 and u.max() == 255
        codes = rng.integers(0, ksub, (500, M)).astype(np.uint8)
        ku8 = oracle.pq_keys_u8(u, base, delta, codes).astype(np.float64)
        kf = oracle.pq_keys(lut, codes).astype(np.float64)
        assert np.abs(ku8 - kf).max() <= M * (0.5 * float(delta)) + 1e-5 * np.abs(kf).max()
        # the integer part of the key is the plain sum of the looked-up codes
        K = u[np.arange(M)[None, :], codes.astype(np.int64)].sum(1)
        np.testing.assert_array_equal(
            ku8.astype(np.float32), (np.float32(base) + (K.astype(np.float32) * np.float32(delta))).astype(np.float32))


def test_monotone_within_each_subspace():
    rng = np.random.default_rng(12)
    lut = rng.standard_normal((24, 256)).astype(np.float32) ** 2
    u, _, _ = oracle.pq_lut_u8(lut)
    for m in range(lut.shape[0]):
        o = np.argsort(lut[m], kind="stable")
        assert np.all(np.diff(u[m][o].astype(np.int64)) >= 0)


def test_constant_table():
    lut = np.full((8, 16), 3.5, np.float32)
    u, base, delta = oracle.pq_lut_u8(lut)
    assert delta == 1.0 and base == np.float32(28.0)
    assert not u.any()
    codes = np.random.default_rng(1).integers(0, 16, (10, 8)).astype(np.uint8)
    np.testing.assert_array_equal(oracle.pq_keys_u8(u, base, delta, codes), np.full(10, 28.0, np.float32))


def test_u8_search_exhaustive_equals_exact_knn():
    """All lists probed and K_c = S: the one-byte estimate only orders the
    candidates, and the exact re-rank returns the exact k nearest."""
    w = synth.small_workload("ivfpq_100k_d128", n=3000, nlist=8, nq=6)
    x, q = synth.base_vectors(w), synth.query_vectors(w)
    tr, ip = synth.kmeans_draws(w.n, w.nlist, 512, 0)
    pr, pi = synth.pq_draws(w.n, 16, 256, 2000, 0)
    ix = oracle.build_ivf_pq(x, w.nlist, 16, 8, tr, ip, pr, pi, 4)
    k = 50
    res = oracle.search_pq(ix, q, k, w.nlist, float(w.n) / k + 1.0, lut_u8=True)
    for i in range(q.shape[0]):
        ex = oracle.canon_l2_batch(q[i], x)
        order = np.lexsort((np.arange(w.n), ex))[:k]
        np.testing.assert_array_equal(res["ids"][i * k:(i + 1) * k], order)
        np.testing.assert_array_equal(res["dists"][i * k:(i + 1) * k], ex[order])


def test_u8_candidates_follow_the_u8_keys():
    """The one-byte path's candidates are the K_c smallest one-byte keys
    (keys formed per probed list from that list's table), ties by id."""
    w = synth.small_workload("ivfpq4_10m_d96", n=4000, nlist=16, nq=4, pq_m=48, pq_bits=4)
    x, q = synth.base_vectors(w), synth.query_vectors(w)
    tr, ip = synth.kmeans_draws(w.n, w.nlist, 1024, 0)
    pr, pi = synth.pq_draws(w.n, 48, 16, 3000, 0)
    ix = oracle.build_ivf_pq(x, w.nlist, 48, 4, tr, ip, pr, pi, 4)
    k, nprobe, r = 120, 6, 2.5
    res = oracle.search_pq(ix, q, k, nprobe, r, debug=True, lut_u8=True)
    for i in range(q.shape[0]):
        lists = res["probe_lists"][res["probe_off"][i]:res["probe_off"][i + 1]]
        keys, ids = [], []
        for j in lists:
            u, base, delta = oracle.pq_lut_u8(oracle.pq_lut(q[i], ix["centroids"][j], ix["codebook"], 48, 16))
            sl = slice(ix["list_off"][j], ix["list_off"][j + 1])
            keys.append(oracle.pq_keys_u8(u, base, delta, ix["codes"][sl]))
            ids.append(ix["list_ids"][sl])
        keys, ids = np.concatenate(keys), np.concatenate(ids)
        kc = int(res["n_cand"][i])
        o = np.lexsort((ids, keys))[:kc]
        c0 = res["cand_off"][i]
        np.testing.assert_array_equal(res["cand_ids"][c0:c0 + kc], ids[o])
        np.testing.assert_array_equal(res["cand_keys"][c0:c0 + kc], keys[o])
