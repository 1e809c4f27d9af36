"""Pins of the oracle's RaBitQ steps (the bounded quantizer of the
background and Algorithm 3): rotation, codes and factors, the bit-plane
estimator, bound coverage, and the bounded re-rank's stop rule."""
import numpy as np
import pytest

import oracle
import synth


def _mixture(d, n, nq, nlist, seed_index=2, metric="l2"):
    w = synth.small_workload("ivfrabitq_1m_d960", n=n, nlist=nlist, nq=nq, d=d, seed_index=seed_index)
    x = synth.base_vectors(w)
    q = synth.query_vectors(w)
    if metric == "ip":
        x = (x / np.linalg.norm(x, axis=1, keepdims=True)).astype(np.float32)
        q = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)
    tr, ip = synth.kmeans_draws(n, nlist, 64 * nlist, 0)
    return w, x, q, tr, ip


def test_rotation_is_orthogonal_and_transposed():
    P = synth.rotation_orthogonal(128, 300)
    assert np.abs(P.astype(np.float64).T @ P - np.eye(128)).max() < 1e-5
    # integer operands: every partial sum is exact, so the result must equal
    # P^T v computed in integers (pins the index order)
    rng = np.random.default_rng(0)
    Pi = rng.integers(-3, 4, (64, 64)).astype(np.float32)
    v = rng.integers(-5, 6, (7, 64)).astype(np.float32)
    got = oracle.rotate(Pi, v)
    want = (v.astype(np.int64) @ Pi.astype(np.int64)).astype(np.float32)
    np.testing.assert_array_equal(got, want)


def test_codes_and_factors_against_float64():
    d, n, nlist = 128, 2000, 4
    w, x, q, tr, ip = _mixture(d, n, 1, nlist)
    P = synth.rotation_orthogonal(d, 301)
    ix = oracle.build_ivf_rabitq(x, nlist, tr, ip, P)
    cent = ix["centroids"].astype(np.float64)
    for p in range(0, n, 37):
        j = int(np.searchsorted(ix["list_off"], p, side="right") - 1)
        xv = x[ix["list_ids"][p]].astype(np.float64)
        r = xv - cent[j]
        y = P.astype(np.float64).T @ r
        bits = np.unpackbits(ix["codes"][p].view(np.uint8), bitorder="little")[:d].astype(bool)
        clear = np.abs(y) > 1e-4 * np.abs(y).max()
        np.testing.assert_array_equal(bits[clear], (y > 0)[clear])
        nr = np.linalg.norm(r)
        ipoo = np.abs(y).sum() / (nr * np.sqrt(d))
        f, g = 1.0 / ipoo, np.sqrt(1.0 - ipoo * ipoo) / ipoo
        fac = ix["factors"][p].astype(np.float64)
        np.testing.assert_allclose(fac[:3], [nr, f, g], rtol=1e-4)
        assert fac[3] == bits.sum()


def test_zero_residual_object():
    d = 64
    P = synth.rotation_orthogonal(d, 302)
    c = np.ones((1, d), np.float32)
    x = np.vstack([c, c + 0.5]).astype(np.float32)
    codes, fac = oracle.rabitq_encode(x, np.array([0, 1]), np.array([0, 2]), c, P)
    assert np.all(codes[0] == 0)
    np.testing.assert_array_equal(fac[0], [0.0, 1.0, 0.0, 0.0])
    assert fac[1][0] == np.float32(np.sqrt(np.float32(d * 0.25)))


def test_bit_planes_estimator_closed_form():
    """With f = 1, nr = 1, IP metric and a = 0, key = -<x_bar, y_bar>, and
    <x_bar, y_bar> = sum_i s_i (vl + delta u_i) / sqrt(D) with s_i = +-1 by the
    code bit and u the 4-bit quantized query (D = 64 and 128)."""
    rng = np.random.default_rng(5)
    for D in (64, 128):
        for trial in range(20):
            y = rng.standard_normal(D).astype(np.float32) * 3
            planes, scal = oracle.rabitq_prep(y)
            vl, delta = np.float32(y.min()), np.float32((y.max() - y.min()) * np.float32(1.0 / 15.0))
            assert scal[0] == vl and scal[1] == delta
            u = np.clip(np.floor((y - vl) / delta + np.float32(0.5)), 0, 15).astype(np.int64)
            # the planes hold u bit by bit
            pb = np.stack([np.unpackbits(planes[b].view(np.uint8), bitorder="little")[:D] for b in range(4)])
            np.testing.assert_array_equal((pb * (1 << np.arange(4))[:, None]).sum(0), u)
            code_bits = rng.integers(0, 2, D)
            code = np.packbits(code_bits.astype(np.uint8), bitorder="little").view(np.uint32)[None, :]
            fac = np.array([[1.0, 1.0, 0.0, code_bits.sum()]], np.float32)
            key, lb, ub = oracle.rabitq_bounds(code, fac, planes, scal, metric=1, a=0.0, qn=1.0)
            s = 2.0 * code_bits - 1.0
            want = (s * (float(vl) + float(delta) * u)).sum() / np.sqrt(D)
            assert abs(-float(key[0]) - want) <= 1e-5 * (np.abs(y).sum() / np.sqrt(D) + 1.0), (D, trial)
            assert lb[0] == key[0] and ub[0] == key[0]  # g = 0: no error term


@pytest.mark.parametrize("d,metric", [(128, "l2"), (960, "l2"), (256, "ip")])
def test_bounds_cover_true_distance(d, metric):
    """The bound is eps0 standard errors of the estimator wide: with the
    estimation error close to normal, it holds for about P(|Z| <= 1.9) = 94%
    of (query, object) pairs (a bound twice too wide or too narrow would give
    99.98% or 66%), and the estimate is unbiased."""
    n, nlist, nq = 3000 if d < 960 else 1500, 4, 6
    w, x, q, tr, ip = _mixture(d, n, nq, nlist, metric=metric)
    P = synth.rotation_orthogonal(d, 303)
    m = 0 if metric == "l2" else 1
    ix = oracle.build_ivf_rabitq(x, nlist, tr, ip, P, metric=m)
    r = oracle.search_rabitq(ix, q, 10, nlist, debug=True)
    inside, total, err = 0, 0, []
    for i in range(nq):
        lists = r["probe_lists"][r["probe_off"][i]:r["probe_off"][i + 1]]
        slots = np.concatenate([np.arange(ix["list_off"][j], ix["list_off"][j + 1]) for j in lists])
        ids = ix["list_ids"][slots]
        xs = x[ids].astype(np.float64)
        qq = q[i].astype(np.float64)
        true = ((xs - qq) ** 2).sum(1) if m == 0 else -(xs @ qq)
        es = slice(r["est_off"][i], r["est_off"][i + 1])
        lb, ub, key = r["est_lb"][es], r["est_ub"][es], r["est_key"][es]
        inside += int(((lb <= true) & (true <= ub)).sum())
        total += len(true)
        err.append(key - true)
    err = np.concatenate(err)
    assert 0.92 <= inside / total <= 0.97, inside / total
    assert abs(err.mean()) < 0.1 * err.std() + 1e-6


def _exact_topk(ix, q, k, metric):
    ids = np.arange(ix["n"])
    if metric == 0:
        keys = np.array([oracle.canon_l2(q, ix["base"][i]) for i in ids], np.float32)
    else:
        keys = np.array([-oracle.canon_ip(q, ix["base"][i]) for i in ids], np.float32)
    o = np.lexsort((ids, keys))[:k]
    return ids[o], keys[o]


@pytest.mark.parametrize("metric", [0, 1])
def test_wide_bounds_give_the_exact_top_k(metric):
    """With eps0 so large that every bound holds, scanning every list returns
    the exact top-k by (canonical key, id), padded when k exceeds n."""
    d, n, nlist, nq = 64, 800, 4, 3
    w, x, q, tr, ip = _mixture(d, n, nq, nlist, metric="l2" if metric == 0 else "ip")
    P = synth.rotation_orthogonal(d, 304)
    ix = oracle.build_ivf_rabitq(x, nlist, tr, ip, P, metric=metric)
    for k in (1, 37, 300, 1000):
        r = oracle.search_rabitq(ix, q, k, nlist, eps0=1e6)
        for i in range(nq):
            ei, ek = _exact_topk(ix, q[i], min(k, n), metric)
            got = slice(r["off"][i], r["off"][i + 1])
            assert r["counts"][i] == min(k, n)
            np.testing.assert_array_equal(r["ids"][got][:len(ei)], ei)
            np.testing.assert_array_equal(r["dists"][got][:len(ei)], ek if metric == 0 else -ek)
            assert np.all(r["ids"][got][len(ei):] == -1)


def test_stop_rule_brute_force_small():
    """eps0 = 0.3 (bounds often fail): the output is the best k of the walked
    prefix in (lb, id) order, and the prefix ends exactly where the rule says,
    checked by re-walking with a plain sorted list."""
    d, n, nlist, nq, k = 64, 600, 3, 4, 25
    w, x, q, tr, ip = _mixture(d, n, nq, nlist)
    P = synth.rotation_orthogonal(d, 305)
    ix = oracle.build_ivf_rabitq(x, nlist, tr, ip, P)
    for eps in (0.0, 0.3, 1.9):
        r = oracle.search_rabitq(ix, q, k, 2, eps0=eps, debug=True)
        for i in range(nq):
            lists = r["probe_lists"][r["probe_off"][i]:r["probe_off"][i + 1]]
            slots = np.concatenate([np.arange(ix["list_off"][j], ix["list_off"][j + 1]) for j in lists])
            ids = ix["list_ids"][slots]
            lb = r["est_lb"][r["est_off"][i]:r["est_off"][i + 1]]
            order = np.lexsort((ids, lb))
            best = []  # sorted (key, id)
            t = 0
            for t in range(len(order) + 1):
                if t == len(order):
                    break
                o = order[t]
                if len(best) == k and lb[o] > best[-1][0]:
                    break
                ex = np.float32(oracle.canon_l2(q[i], x[ids[o]]))
                best = sorted(best + [(ex, int(ids[o]))])[:k]
            assert r["n_visited"][i] == t
            got = slice(r["off"][i], r["off"][i] + len(best))
            np.testing.assert_array_equal(r["ids"][got], [b[1] for b in best])
            np.testing.assert_array_equal(r["dists"][got], [b[0] for b in best])


def test_visited_grows_with_eps0():
    d, n, nlist, nq, k = 128, 2000, 4, 4, 50
    w, x, q, tr, ip = _mixture(d, n, nq, nlist)
    P = synth.rotation_orthogonal(d, 306)
    ix = oracle.build_ivf_rabitq(x, nlist, tr, ip, P)
    prev = None
    for eps in (0.0, 0.5, 1.0, 1.9, 4.0):
        r = oracle.search_rabitq(ix, q, k, nlist, eps0=eps, debug=True)
        if prev is not None:
            assert np.all(r["n_visited"] >= prev)
        prev = r["n_visited"]


def test_fp16_base_is_converted_exactly():
    d, n, nlist = 64, 500, 2
    w, x, q, tr, ip = _mixture(d, n, 2, nlist, metric="ip")
    x16 = x.astype(np.float16)
    P = synth.rotation_orthogonal(d, 307)
    a = oracle.build_ivf_rabitq(x16, nlist, tr, ip, P, metric=1)
    b = oracle.build_ivf_rabitq(x16.astype(np.float32), nlist, tr, ip, P, metric=1)
    assert a["fp16"] and not b["fp16"]
    for key in ("centroids", "codes", "factors", "list_ids"):
        np.testing.assert_array_equal(a[key], b[key])
