"""GPU parity of the early re-rank (Algorithm 4, the improved IVF+PQ search)
through the C ABI: the scan computes the exact distance of every object
after the codebook sample whose bucket lies below the predicted threshold
bucket, and the candidates among them are not re-ranked again.  Every step
and the results equal the oracle's plain path; the predicted threshold and
the number of early exact distances equal the oracle's accounting of
Algorithm 4; the early keys reused are the early candidates (all of them
whenever the prediction does not exceed the threshold bucket)."""
import os

import numpy as np
import pytest

from helpers import check_trace, expected_steps, make_gpu_index, oracle_pq_index

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bbc():
    import paper_2604_01960_amd as b
    b.load()
    return b


def _index(bbc, ix, env):
    old = {v: os.environ.get(v) for v in env}
    os.environ.update(env)
    try:
        return make_gpu_index(bbc, ix)
    finally:
        for v, o in old.items():
            if o is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = o


def _check_early(tr, exp):
    n_exact_pred = 0
    for i, e in enumerate(exp):
        er = e["early"]
        if er is None or e["n_cand"] == 0:
            continue
        assert tr["tau_pred"][i] == er["tau_pred"], f"tau_pred q{i}"
        assert tr["n_early"][i] == er["n_early"], f"n_early q{i}"
        assert tr["n_early_used"][i] <= er["n_early_cand"], f"n_early_used q{i}"
        if er["tau_pred"] <= tr["tau"][i]:
            assert tr["n_early_used"][i] == er["n_early_cand"], f"n_early_used q{i}"
            n_exact_pred += 1
    return n_exact_pred


@pytest.mark.parametrize("form", ["tile", "per_query"])
@pytest.mark.parametrize("variant", ["0", "1", "2"])
@pytest.mark.parametrize("cfg", [
    # (base workload, n, nlist, M, bits, nq, k, nprobe, ratio, m, nsample)
    ("ivfpq_100k_d128", 20000, 64, 16, 8, 12, 300, 16, 2.0, 64, 8),
    ("ivfpq_1m_d128", 24000, 60, 32, 8, 10, 700, 24, 1.5, 256, 3),
    ("ivfpq4_10m_d96", 20000, 50, 48, 4, 10, 400, 20, 2.5, 80, 8),
])
def test_early_rerank_matches_oracle(bbc, cfg, variant, form):
    base, n, nlist, M, bits, nq, k, nprobe, ratio, m, ns = cfg
    w, ix, q = oracle_pq_index(base, n, nlist, M, bits, nq)
    print(f"[case] early re-rank {base} n={n} M={M} bits={bits} k={k} nprobe={nprobe} variant={variant} "
          f"form={form}", flush=True)
    env = {"BBC_SCAN_VARIANT": variant}
    if form == "per_query":
        env["BBC_RERANK_FORM"] = "1"
    g = _index(bbc, ix, env)
    rng = np.random.default_rng(int(variant) * 7 + 1)
    kk = rng.integers(1, 2 * k, nq).astype(np.int32)
    npb = rng.integers(1, nprobe + 1, nq).astype(np.int32)
    for kq, nq_probe in ((k, nprobe), (kk, npb)):
        tr = g.search_traced(q, kq, nq_probe, ratio=ratio, buckets=m, nsample=ns, early_rerank=True)
        exp = expected_steps(ix, q, kq, nq_probe, ratio, m, ns)
        check_trace(tr, exp, m)
        _check_early(tr, exp)
    assert np.sum(tr["n_early"]) > 0  # the case really re-ranks early
    import torch
    qd = torch.from_numpy(q).to("cuda:0")
    a = g.search(qd, kk, npb, ratio=ratio, buckets=m, nsample=ns, early_rerank=True)
    b = g.search(qd, kk, npb, ratio=ratio, buckets=m, nsample=ns)
    torch.cuda.synchronize()
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())
    g.free()


def test_early_rerank_large_k(bbc):
    """Large K_c (codebook sample in memory, final top-k memory form): the
    same results as the plain search and the oracle's accounting."""
    w, ix, q = oracle_pq_index("ivfpq_100k_d128", 100_000, 64, 16, 8, 5)
    print("[case] early re-rank large k", flush=True)
    g = make_gpu_index(bbc, ix)
    tr = g.search_traced(q, 16000, 64, ratio=2.5, buckets=256, nsample=8, early_rerank=True)
    exp = expected_steps(ix, q, 16000, 64, 2.5, 256, 8)
    check_trace(tr, exp, 256)
    _check_early(tr, exp)
    g.free()


def test_early_rerank_refusals(bbc):
    w, ix, q = oracle_pq_index("ivfpq_100k_d128", 4000, 8, 16, 8, 3)
    g = make_gpu_index(bbc, ix)
    with pytest.raises(bbc.BBCError) as e:
        g.search(q, 10, 2, early_rerank=True, collector="sort")
    assert e.value.code == bbc.EINVAL
    with pytest.raises(bbc.BBCError) as e:
        g.search(q, 10, 2, early_rerank=True, lut_u8=True)
    assert e.value.code == bbc.EUNSUPPORTED
    g.free()
