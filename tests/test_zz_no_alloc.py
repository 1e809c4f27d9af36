"""The allocation-free search (bbc_search_noalloc) through the C ABI: its
results equal bbc_search's (device I/O, the index's own workspace) bit for
bit, on two calls in a row on the shared per-GPU array, the second with a
smaller batch (the array keeps the first call's contents); for PQ and for
RaBitQ, with per-query k and nprobe.  A batch that needs more than the
array is refused before anything runs, and host I/O is refused."""
import numpy as np
import pytest

import oracle
import synth
from helpers import make_gpu_index, oracle_pq_index

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bbc():
    import paper_2604_01960_amd as b
    b.load()
    return b


def _run_both(bbc, g, q, k, npb, ratio=2.0):
    import torch
    qt = torch.from_numpy(q).to("cuda:0")
    nq = q.shape[0]
    tot = int(np.sum(k))
    ref = g.search(qt, k, npb, ratio=ratio)
    out = (torch.full((tot,), -7, dtype=torch.int64, device="cuda:0"),
           torch.full((tot,), 7.0, dtype=torch.float32, device="cuda:0"),
           torch.full((nq,), -7, dtype=torch.int32, device="cuda:0"))
    got = g.search_noalloc(qt, k, npb, out, ratio=ratio)
    torch.cuda.synchronize()
    for a, b in zip(got[:3], ref[:3]):
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    return ref


def test_noalloc_pq_two_calls_match_search(bbc):
    w, ix, q = oracle_pq_index("ivfpq_100k_d128", 20000, 32, 16, 8, 24)
    print("[case] noalloc PQ 20000x128, 24 then 7 queries", flush=True)
    g = make_gpu_index(bbc, ix)
    rng = np.random.default_rng(5)
    k = rng.integers(1, 1500, 24).astype(np.int32)
    npb = rng.integers(1, 33, 24).astype(np.int32)
    ref = _run_both(bbc, g, q, k, npb, ratio=2.5)
    # the first call against the oracle too
    o = oracle.search_pq(ix, q, k.astype(np.int64), npb.astype(np.int64), 2.5)
    np.testing.assert_array_equal(ref[0].cpu().numpy(), o["ids"])
    np.testing.assert_array_equal(ref[1].cpu().numpy(), o["dists"])
    # second call: a smaller batch on the array the first one filled
    _run_both(bbc, g, q[5:12].copy(), k[5:12].copy(), npb[5:12].copy(), ratio=2.5)
    g.free()


def test_noalloc_rabitq_two_calls_match_search(bbc):
    d, n, nq, nlist = 128, 8000, 10, 16
    w = synth.small_workload("ivfrabitq_1m_d960", n=n, nlist=nlist, nq=nq, d=d, seed_index=2)
    x, q = synth.base_vectors(w), synth.query_vectors(w)
    tr, ip = synth.kmeans_draws(n, nlist, 64 * nlist, 0)
    P = synth.rotation_orthogonal(d, 302)
    ix = oracle.build_ivf_rabitq(x, nlist, tr, ip, P)
    print("[case] noalloc RaBitQ 8000x128, 10 then 3 queries", flush=True)
    g = bbc.Index.create_rabitq(ix["centroids"], ix["list_off"], ix["list_ids"], ix["P"], ix["codes"],
                                ix["factors"], x, metric=ix["metric"])
    k = np.array([10, 300, 2000, 50, 700, 1500, 1, 90, 400, 1200], np.int32)
    npb = np.array([12, 3, 7, 1, 16, 12, 2, 5, 9, 16], np.int32)
    ref = _run_both(bbc, g, q, k, npb)
    o = oracle.search_rabitq(ix, q, k, npb)
    np.testing.assert_array_equal(ref[0].cpu().numpy(), o["ids"])
    np.testing.assert_array_equal(ref[1].cpu().numpy(), o["dists"])
    _run_both(bbc, g, q[2:5].copy(), k[2:5].copy(), npb[2:5].copy())
    g.free()


def test_noalloc_refuses_oversized_batch_and_host_io(bbc):
    import ctypes as C

    import torch
    w, ix, q = oracle_pq_index("ivfpq_100k_d128", 20000, 32, 16, 8, 24)
    g = make_gpu_index(bbc, ix)
    per_query = g.query_bytes(20000, 32, ratio=1.0)
    cap = 128 << 20
    nq = 2 * cap // per_query + 2
    print(f"[case] noalloc refusal: {nq} queries of {per_query} bytes", flush=True)
    qt = torch.zeros((nq, q.shape[1]), dtype=torch.float32, device="cuda:0")
    qt[:] = torch.from_numpy(q[0]).to("cuda:0")
    out = (torch.empty(nq * 20000, dtype=torch.int64, device="cuda:0"),
           torch.empty(nq * 20000, dtype=torch.float32, device="cuda:0"),
           torch.empty(nq, dtype=torch.int32, device="cuda:0"))
    with pytest.raises(bbc.BBCError) as e:
        g.search_noalloc(qt, 20000, 32, out, ratio=1.0)
    assert e.value.code == bbc.ENOMEM
    assert "allocation-free maximum" in str(e.value)
    # host I/O is refused (device pointers only)
    lib = bbc.load()
    kk = np.full(1, 5, np.int32)
    npb = np.full(1, 4, np.int32)
    off = np.array([0, 5], np.int64)
    ids = np.empty(5, np.int64)
    dist = np.empty(5, np.float32)
    cnt = np.empty(1, np.int32)
    p = bbc.SearchParams(2.0, 0, 0, 0, 0, 0, None)
    rc = lib.bbc_search_noalloc(g._h, q[:1].ctypes.data, 1, kk.ctypes.data, npb.ctypes.data, C.byref(p),
                                off.ctypes.data, ids.ctypes.data, dist.ctypes.data, cnt.ctypes.data)
    assert rc == bbc.EINVAL
    g.free()
