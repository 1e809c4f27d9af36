"""The comparator collectors (heap, sort) return the same candidates and the
same final ids and distances as the bucket collector and the oracle, on the
same scan output (result-collector background; Algorithm 1)."""
import numpy as np
import pytest

from helpers import check_trace, expected_steps, make_gpu_index, oracle_pq_index

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bbc():
    import paper_2604_01960_amd as b
    b.load()
    return b


@pytest.mark.parametrize("collector", ["heap", "sort", "heap_lds"])
@pytest.mark.parametrize("cfg", [
    # (base workload, n, nlist, M, bits, nq, k, nprobe, ratio)
    ("ivfpq_100k_d128", 20000, 64, 16, 8, 10, 300, 12, 2.0),
    ("ivfpq4_10m_d96", 20000, 50, 48, 4, 8, 900, 10, 2.5),
])
def test_comparators_match_oracle(bbc, collector, cfg):
    base, n, nlist, M, bits, nq, k, nprobe, ratio = cfg
    w, ix, q = oracle_pq_index(base, n, nlist, M, bits, nq)
    print(f"[case] {collector} {base} n={n} k={k} nprobe={nprobe} r={ratio}", flush=True)
    g = make_gpu_index(bbc, ix)
    tr = g.search_traced(q, k, nprobe, ratio=ratio, collector=collector)
    exp = expected_steps(ix, q, k, nprobe, ratio, 256, 8)
    check_trace(tr, exp, 256, bucket=False)


def test_comparators_uneven_and_ties(bbc):
    """Per-query k and nprobe (K_c = S, K_c < S, one list), and integer data
    where estimated keys tie massively (the heap and the selection must cut
    ties by id)."""
    import oracle
    w, ix, q = oracle_pq_index("ivfpq_100k_d128", 12000, 40, 16, 8, 10)
    g = make_gpu_index(bbc, ix)
    k = np.array([1, 5, 300, 2000, 12000, 50, 7, 999, 64, 3], np.int32)
    npb = np.array([1, 40, 3, 7, 40, 2, 1, 11, 5, 39], np.int32)
    for collector in ("heap", "sort", "heap_lds"):
        print(f"[case] uneven {collector}", flush=True)
        tr = g.search_traced(q, k, npb, ratio=1.7, collector=collector)
        check_trace(tr, expected_steps(ix, q, k, npb, 1.7, 256, 8), 256, bucket=False)

    rng = np.random.default_rng(21)
    n, d, nlist, M = 5000, 16, 10, 4
    x = rng.integers(0, 3, (n, d)).astype(np.float32)
    cent = rng.integers(0, 3, (nlist, d)).astype(np.float32)
    a = oracle.kmeans_assign(x, cent)
    order = np.argsort(a, kind="stable").astype(np.int64)
    off = np.zeros(nlist + 1, np.int64)
    off[1:] = np.cumsum(np.bincount(a, minlength=nlist))
    cb = rng.integers(-1, 2, (M, 16, d // M)).astype(np.float32)
    codes = oracle.pq_encode(oracle.residuals(x, order, cent, a), cb)
    tix = dict(kind="pq", n=n, d=d, nlist=nlist, M=M, ksub=16, bits=4, metric=0, centroids=cent, assign=a,
               list_off=off, list_ids=order, codes=codes, codebook=cb, base=x)
    tq = rng.integers(0, 3, (6, d)).astype(np.float32)
    tg = make_gpu_index(bbc, tix)
    exp = expected_steps(tix, tq, 700, 4, 2.0, 16, 2)
    for collector in ("heap", "sort", "heap_lds"):
        print(f"[case] integer ties {collector}", flush=True)
        tr = tg.search_traced(tq, 700, 4, ratio=2.0, collector=collector)
        check_trace(tr, exp, 16, bucket=False)


def test_collectors_agree_at_scale(bbc):
    """The 100k x 128 workload at k = 5000: the three collectors return
    identical ids and distances."""
    w, ix, q = oracle_pq_index("ivfpq_100k_d128", 100_000, 256, 16, 8, 100)
    print("[case] collectors at 100k, k=5000", flush=True)
    g = make_gpu_index(bbc, ix)
    ref = g.search(q, 5000, 32, ratio=2.0, collector="bucket")
    for collector in ("heap", "sort"):
        got = g.search(q, 5000, 32, ratio=2.0, collector=collector)
        for x, y in zip(got[:3], ref[:3]):
            np.testing.assert_array_equal(x, y)


def test_heap_in_global_memory_and_keep_all_keys(bbc):
    """K_c above the LDS heap's capacity (19,456) takes the global-memory
    heap; the bucket collector with every key kept (no relaxed-threshold
    filter: all S keys reach it, as for heap and sort) returns the same, and
    every step of it equals the oracle."""
    w, ix, q = oracle_pq_index("ivfpq_100k_d128", 100_000, 64, 16, 8, 4)
    print("[case] global heap, K_c = 24000", flush=True)
    g = make_gpu_index(bbc, ix)
    ref = g.search(q, 16000, 48, ratio=1.5, collector="bucket")
    for kw in (dict(collector="heap"), dict(collector="heap_lds"), dict(collector="bucket", keep_all_keys=True)):
        got = g.search(q, 16000, 48, ratio=1.5, **kw)
        for x, y in zip(got[:3], ref[:3]):
            np.testing.assert_array_equal(x, y)
    tr = g.search_traced(q, 3000, 20, ratio=2.0, keep_all_keys=True)
    check_trace(tr, expected_steps(ix, q, 3000, 20, 2.0, 256, 8), 256)
    np.testing.assert_array_equal(tr["n_survivors"], tr["n_scanned"])
