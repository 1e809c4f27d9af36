"""Serving form through the C ABI: requests submitted one by one and answered
from overlapping device batches return the oracle's ids and distances, the
same alone and in the mix; admission by memory and slots bounds what is in
flight; the ticket protocol (busy, collected once, unknown) and argument
errors hold."""
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


def _collect(srv, tickets, timeout_ms=120000):
    out = []
    for t in tickets:
        r = srv.wait(t, timeout_ms)
        assert r is not None, f"ticket {t} not answered in {timeout_ms} ms"
        out.append(r)
    return out


@pytest.mark.parametrize("lanes", [1, 3])
def test_pq_server_matches_oracle_alone_and_in_the_mix(bbc, lanes):
    nq = 40
    w, ix, q = oracle_pq_index("ivfpq4_10m_d96", 20000, 50, 48, 4, nq)
    g = make_gpu_index(bbc, ix)
    k, npb = synth.uneven_k_nprobe(nq, (20, 3000), (1, 50), seed=31)
    ref = oracle.search_pq(ix, q, k.astype(np.int64), npb.astype(np.int64), 2.0)
    print(f"[case] pq server lanes={lanes}", flush=True)
    srv = g.server(mem_budget=1 << 32, max_slots=8, lanes=lanes, ratio=2.0)
    tickets = [srv.submit(q[i], int(k[i]), int(npb[i])) for i in range(nq)]
    res = _collect(srv, tickets)
    st = srv.stats()
    srv.free()
    assert st["requests"] == nq and st["pending"] == 0
    assert 1 <= st["max_batch"] <= 8 and st["max_inflight"] <= 8
    sizes = g.search_sizes(q, k, npb, ratio=2.0)
    for i, (ids, dists, info) in enumerate(res):
        s = slice(ref["off"][i], ref["off"][i + 1])
        np.testing.assert_array_equal(ids, ref["ids"][s], err_msg=f"request {i}")
        np.testing.assert_array_equal(dists, ref["dists"][s], err_msg=f"request {i}")
        assert info["count"] == ref["counts"][i] and info["latency_ns"] > 0 and info["status"] == 0
        assert info["n_scanned"] == sizes["n_scanned"][i] and info["n_reranked"] == sizes["n_cand"][i]
        assert 1 <= info["batch_size"] <= 8
        if i % 8 == 0:  # the same request searched alone
            a = g.search(q[i:i + 1], int(k[i]), int(npb[i]), ratio=2.0)
            np.testing.assert_array_equal(ids, a[0])
            np.testing.assert_array_equal(dists, a[1])


def test_admission_bounds_what_is_in_flight(bbc):
    nq = 24
    w, ix, q = oracle_pq_index("ivfpq4_10m_d96", 20000, 50, 48, 4, nq)
    g = make_gpu_index(bbc, ix)
    k, npb = 700, 12
    one = g.query_bytes(k, npb, ratio=2.0)
    assert one > 0
    direct = g.search(q, k, npb, ratio=2.0)
    for budget, slots, cap in [(one, 64, 1), (3 * one, 64, 3), (1 << 32, 2, 2)]:
        print(f"[case] admission budget={budget} slots={slots}", flush=True)
        srv = g.server(mem_budget=budget, max_slots=slots, lanes=4, ratio=2.0)
        tickets = [srv.submit(q[i], k, npb) for i in range(nq)]
        res = _collect(srv, tickets)
        st = srv.stats()
        # a request bigger than the whole budget is refused at submission
        # (the budget of one request: any larger one; the others: when the
        # largest request this index allows is bigger still)
        big = g.query_bytes(20 * k, 50, ratio=2.0)
        if budget == one:
            assert big > budget
        if big > budget:
            with pytest.raises(bbc.BBCError) as e:
                srv.submit(q[0], 20 * k, 50)
            assert e.value.code == bbc.ENOMEM
        srv.free()
        assert st["max_inflight"] <= cap and st["max_batch"] <= cap and st["requests"] == nq
        for i, (ids, dists, info) in enumerate(res):
            s = slice(direct[3][i], direct[3][i + 1])
            np.testing.assert_array_equal(ids, direct[0][s])
            np.testing.assert_array_equal(dists, direct[1][s])


def test_ticket_protocol_and_errors(bbc):
    w, ix, q = oracle_pq_index("ivfpq4_10m_d96", 20000, 50, 48, 4, 8)
    g = make_gpu_index(bbc, ix)
    L = bbc.load()
    print("[case] server tickets", flush=True)
    srv = g.server(mem_budget=1 << 30, max_slots=16)
    t = srv.submit(q[0], 500, 10)
    # ready or busy, never an error, until collected once
    got = None
    for _ in range(200000):
        got = srv.poll(t)
        if got is not None:
            break
    if got is None:
        got = srv.wait(t, 60000)
    assert got is not None and got[2]["count"] == 500
    assert L.bbc_server_poll(srv._h, t, None, None, None) == bbc.EINVAL   # collected
    assert L.bbc_server_poll(srv._h, 10 ** 9, None, None, None) == bbc.EINVAL  # never issued
    assert L.bbc_server_wait(srv._h, t, 10, None, None, None) == bbc.EINVAL
    for args in [(q[0], 0, 10), (q[0], 10, 0), (q[0], 10, 51)]:
        with pytest.raises(bbc.BBCError) as e:
            srv.submit(*args)
        assert e.value.code == bbc.EINVAL
    bad = q[0].copy()
    bad[3] = np.nan
    with pytest.raises(bbc.BBCError):
        srv.submit(bad, 10, 5)
    # requests still queued when the server is destroyed are answered first
    for i in range(8):
        srv.submit(q[i], 300, 20)
    srv.free()


def test_rabitq_server_matches_oracle(bbc):
    d, n, nlist, nq = 256, 5000, 10, 12
    wl = synth.small_workload("ivfrabitq_1m_d960", n=n, nlist=nlist, nq=nq, d=d, seed_index=2)
    x = synth.base_vectors(wl)
    q = synth.query_vectors(wl)
    x = (x / np.linalg.norm(x, axis=1, keepdims=True)).astype(np.float32)
    q = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)
    x16 = x.astype(np.float16)
    tr, ip = synth.kmeans_draws(n, nlist, 64 * nlist, 0)
    P = synth.rotation_orthogonal(d, 302)
    ix = oracle.build_ivf_rabitq(x16, nlist, tr, ip, P, metric=1)
    g = bbc.Index.create_rabitq(ix["centroids"], ix["list_off"], ix["list_ids"], ix["P"], ix["codes"],
                                ix["factors"], x16, metric=1, eps0=oracle.RABITQ_EPS0)
    rng = np.random.default_rng(17)
    k = rng.integers(10, 1500, nq).astype(np.int32)
    npb = rng.integers(1, nlist + 1, nq).astype(np.int32)
    ref = oracle.search_rabitq(ix, q, k, npb)
    print("[case] rabitq server", flush=True)
    srv = g.server(mem_budget=1 << 30, max_slots=4, lanes=2)
    res = _collect(srv, [srv.submit(q[i], int(k[i]), int(npb[i])) for i in range(nq)])
    srv.free()
    sizes = g.search_sizes(q, k, npb)
    for i, (ids, dists, info) in enumerate(res):
        s = slice(ref["off"][i], ref["off"][i + 1])
        np.testing.assert_array_equal(ids, ref["ids"][s], err_msg=f"request {i}")
        np.testing.assert_array_equal(dists, ref["dists"][s])
        assert info["count"] == ref["counts"][i]
        assert info["n_scanned"] == sizes["n_scanned"][i] and info["n_reranked"] == sizes["n_visited"][i]
