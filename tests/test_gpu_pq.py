"""GPU parity of the PQ query path against the oracle, step by step, through
the C ABI (probe, estimated keys, codebook, histogram and threshold bucket,
candidate set, exact keys, final ids and distances)."""
import numpy as np
import pytest

from helpers import check_trace, expected_steps, make_gpu_index, oracle_pq_index

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bbc():
    import paper_2604_01960_amd as b
    b.load()
    return b


@pytest.mark.parametrize("cfg", [
    # (base workload, n, nlist, M, bits, d, nq, k, nprobe, ratio, m, nsample)
    ("ivfpq_100k_d128", 20000, 64, 16, 8, 0, 12, 300, 12, 2.0, 64, 8),
    ("ivfpq_1m_d128", 24000, 60, 32, 8, 0, 10, 700, 9, 1.5, 256, 3),
    ("ivfpq4_10m_d96", 20000, 50, 48, 4, 0, 10, 400, 10, 2.5, 80, 8),
])
def test_every_step_matches_oracle(bbc, cfg):
    base, n, nlist, M, bits, d, nq, k, nprobe, ratio, m, ns = cfg
    w, ix, q = oracle_pq_index(base, n, nlist, M, bits, nq, d)
    print(f"[case] {base} n={n} nlist={nlist} M={M} bits={bits} k={k} nprobe={nprobe} r={ratio} m={m}", flush=True)
    g = make_gpu_index(bbc, ix)
    tr = g.search_traced(q, k, nprobe, ratio=ratio, buckets=m, nsample=ns)
    exp = expected_steps(ix, q, k, nprobe, ratio, m, ns)
    check_trace(tr, exp, m)


def test_uneven_and_edge_cases(bbc):
    w, ix, q = oracle_pq_index("ivfpq_100k_d128", 12000, 40, 16, 8, 14)
    print("[case] uneven/edge n=12000 nlist=40", flush=True)
    g = make_gpu_index(bbc, ix)
    sizes = np.diff(ix["list_off"])
    k = np.array([1, 5, 300, 2000, 12000, 50, 7, 999, 20000, 64, 3, 1000, 250, 4000], np.int32)
    npb = np.array([1, 40, 3, 7, 40, 2, 1, 11, 40, 5, 39, 1, 13, 4], np.int32)
    for ratio in (1.0, 1.7):
        for m in (1, 2, 256):
            tr = g.search_traced(q, k, npb, ratio=ratio, buckets=m, nsample=2)
            exp = expected_steps(ix, q, k, npb, ratio, m, 2)
            check_trace(tr, exp, m)
    # k larger than everything scanned pads with -1 / +inf
    ids, dists, counts, off = g.search(q[:1], 5000, 1, ratio=1.0)
    s = int(sizes[tr["probe_lists"][0]]) if False else int(counts[0])
    assert np.all(ids[s:] == -1) and np.all(np.isinf(dists[s:]))


def test_ties_on_integer_data(bbc):
    """Integer vectors: exact keys tie massively; ids must still match."""
    import oracle
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
    ix = dict(kind="pq", n=n, d=d, nlist=nlist, M=M, ksub=16, bits=4, metric=0, centroids=cent, assign=a,
              list_off=off, list_ids=order, codes=codes, codebook=cb, base=x)
    q = rng.integers(0, 3, (6, d)).astype(np.float32)
    print("[case] integer ties", flush=True)
    g = make_gpu_index(bbc, ix)
    tr = g.search_traced(q, 700, 4, ratio=2.0, buckets=16, nsample=2)
    exp = expected_steps(ix, q, 700, 4, 2.0, 16, 2)
    check_trace(tr, exp, 16)


def test_full_100k_config_bit_exact(bbc):
    """The 100k x 128 / IVF256 / PQ16x8 workload: all 100 queries, k=5000, nprobe=32."""
    import oracle
    w, ix, q = oracle_pq_index("ivfpq_100k_d128", 100_000, 256, 16, 8, 100)
    print("[case] full 100k config", flush=True)
    g = make_gpu_index(bbc, ix)
    ids, dists, counts, off = g.search(q, 5000, 32, ratio=2.0)
    ref = oracle.search_pq(ix, q, 5000, 32, 2.0)
    np.testing.assert_array_equal(counts, ref["counts"])
    np.testing.assert_array_equal(ids, ref["ids"])
    np.testing.assert_array_equal(dists, ref["dists"])


def test_repeat_and_device_io(bbc):
    import torch
    w, ix, q = oracle_pq_index("ivfpq_100k_d128", 20000, 64, 16, 8, 12)
    g = make_gpu_index(bbc, ix)
    a = g.search(q, 300, 12, ratio=2.0)
    b = g.search(q, 300, 12, ratio=2.0)
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)
    qt = torch.from_numpy(q).cuda()
    ids, dists, counts, off = g.search(qt, 300, 12, ratio=2.0)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ids.cpu().numpy(), a[0])
    np.testing.assert_array_equal(dists.cpu().numpy(), a[1])
    np.testing.assert_array_equal(counts.cpu().numpy(), a[2])


@pytest.mark.parametrize("bcap", [64, 4096])
def test_large_threshold_buckets(bbc, bcap):
    """Threshold buckets larger than the LDS sort capacity: their members are
    selected from global scratch (or, beyond K_c members, by passes over the
    survivors); both give the oracle's candidates (few buckets, large k)."""
    import os
    w, ix, q = oracle_pq_index("ivfpq_100k_d128", 20000, 64, 16, 8, 10)
    os.environ["BBC_COLLECT_BCAP"] = str(bcap)
    try:
        g = make_gpu_index(bbc, ix)
    finally:
        del os.environ["BBC_COLLECT_BCAP"]
    k = np.array([300, 900, 2500, 4000, 1200, 700, 3000, 150, 5000, 2000], np.int32)
    npb = np.array([6, 12, 20, 30, 9, 64, 25, 3, 40, 15], np.int32)
    for m in (4, 16, 64):
        print(f"[case] large threshold buckets bcap={bcap} m={m}", flush=True)
        tr = g.search_traced(q, k, npb, ratio=2.0, buckets=m, nsample=8)
        exp = expected_steps(ix, q, k, npb, 2.0, m, 8)
        check_trace(tr, exp, m)
        if bcap == 64:
            assert np.any(tr["n_boundary"] > 64)


@pytest.mark.parametrize("form", ["tile", "tile_ranges", "per_query"])
@pytest.mark.parametrize("shape", ["long_lists", "many_queries"])
def test_rerank_forms(bbc, form, shape):
    """Both re-rank forms against the oracle: the tile-major one (a list's
    rows staged in LDS once per group of queries) and one block per query.
    Long lists span many tiles (one bin each); many queries per list fill
    several groups of pairs for one list.  With the bin counters cut to one
    list's tiles, the candidate sort takes each query's ranks in ranges."""
    import os
    if shape == "long_lists":
        w, ix, q = oracle_pq_index("ivfpq4_10m_d96", 20000, 6, 48, 4, 10)
        k = np.array([50, 900, 2500, 4000, 1200, 700, 3000, 150, 5000, 2000], np.int32)
        npb = np.array([1, 2, 3, 6, 4, 2, 5, 1, 6, 3], np.int32)
    else:
        w, ix, q = oracle_pq_index("ivfpq_100k_d128", 20000, 32, 16, 8, 150)
        k = np.full(150, 200, np.int32)
        npb = np.full(150, 20, np.int32)
        npb[::7] = 32
    os.environ["BBC_RERANK_FORM"] = {"tile": "0", "tile_ranges": "0", "per_query": "1"}[form]
    if form == "tile_ranges":
        os.environ["BBC_RERANK_SORT_BINS"] = "1"
    try:
        g = make_gpu_index(bbc, ix)
    finally:
        del os.environ["BBC_RERANK_FORM"]
        os.environ.pop("BBC_RERANK_SORT_BINS", None)
    print(f"[case] rerank form={form} shape={shape}", flush=True)
    tr = g.search_traced(q, k, npb, ratio=2.0, buckets=64, nsample=2)
    exp = expected_steps(ix, q, k, npb, 2.0, 64, 2)
    check_trace(tr, exp, 64)


@pytest.mark.parametrize("variant", ["0", "1", "2", "3", "4"])
@pytest.mark.parametrize("cfg", [
    # (base workload, n, nlist, M, bits, nq, k, nprobe, ratio, m, nsample)
    ("ivfpq_100k_d128", 20000, 64, 16, 8, 12, 300, 12, 2.0, 64, 8),
    ("ivfpq_1m_d128", 24000, 60, 32, 8, 10, 700, 9, 1.5, 256, 3),
    ("ivfpq4_10m_d96", 20000, 50, 48, 4, 10, 400, 10, 2.5, 80, 8),
])
def test_one_byte_tables_match_oracle(bbc, cfg, variant):
    """One-byte tables with integer sums: estimated keys (base + K * delta),
    codebook, threshold bucket, candidates and results equal the oracle's
    one-byte path, in each scan block shape."""
    import os
    base, n, nlist, M, bits, nq, k, nprobe, ratio, m, ns = cfg
    w, ix, q = oracle_pq_index(base, n, nlist, M, bits, nq)
    print(f"[case] u8 tables {base} n={n} M={M} bits={bits} k={k} nprobe={nprobe} variant={variant}", flush=True)
    old = os.environ.get("BBC_SCAN_VARIANT")
    os.environ["BBC_SCAN_VARIANT"] = variant
    try:
        g = make_gpu_index(bbc, ix)
    finally:
        if old is None:
            os.environ.pop("BBC_SCAN_VARIANT")
        else:
            os.environ["BBC_SCAN_VARIANT"] = old
    rng = np.random.default_rng(int(variant) + 3)
    kk = rng.integers(1, 2 * k, nq).astype(np.int32)
    npb = rng.integers(1, nprobe + 1, nq).astype(np.int32)
    for kq, nq_probe in ((k, nprobe), (kk, npb)):
        tr = g.search_traced(q, kq, nq_probe, ratio=ratio, buckets=m, nsample=ns, lut_u8=True)
        exp = expected_steps(ix, q, kq, nq_probe, ratio, m, ns, lut_u8=True)
        check_trace(tr, exp, m)
    # the device-I/O search returns the same as the traced one
    import torch
    ids, dists, counts, off = g.search(torch.from_numpy(q).to("cuda:0"), kk, npb, ratio=ratio, buckets=m,
                                       nsample=ns, lut_u8=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ids.cpu().numpy(), tr["ids"])
    np.testing.assert_array_equal(dists.cpu().numpy(), tr["dists"])
    g.free()


@pytest.mark.parametrize("variant", ["0", "1", "2", "3", "4"])
def test_scan_block_shapes_match_oracle(bbc, variant):
    """Every block shape of the float-table scan of 8-bit codes, among them
    the sliced tables (variants 0 and 4: two 16-sub-space slices, two blocks
    per CU).  Lists of about 3000 codes take the sliced scan through more than
    one chunk of passes (the slices rebuilt per chunk), short lists through
    one; per-query k and nprobe."""
    import os
    w, ix, q = oracle_pq_index("ivfpq_1m_d128", 24000, 8, 32, 8, 8)
    sizes = np.diff(ix["list_off"])
    assert sizes.max() > 2048 and sizes.min() < 2048
    print(f"[case] scan shape variant={variant} lists {sizes.min()}..{sizes.max()}", flush=True)
    old = os.environ.get("BBC_SCAN_VARIANT")
    os.environ["BBC_SCAN_VARIANT"] = variant
    try:
        g = make_gpu_index(bbc, ix)
    finally:
        if old is None:
            os.environ.pop("BBC_SCAN_VARIANT")
        else:
            os.environ["BBC_SCAN_VARIANT"] = old
    rng = np.random.default_rng(int(variant) + 11)
    kk = rng.integers(1, 3000, q.shape[0]).astype(np.int32)
    npb = rng.integers(1, 9, q.shape[0]).astype(np.int32)
    for kq, nq_probe, ns in ((900, 5, 2), (kk, npb, 3)):
        tr = g.search_traced(q, kq, nq_probe, ratio=1.5, buckets=256, nsample=ns)
        check_trace(tr, expected_steps(ix, q, kq, nq_probe, 1.5, 256, ns), 256)
    g.free()


def test_one_byte_tables_refused_where_unsupported(bbc):
    """A scan shape without the grouped kernel refuses one-byte tables
    (BBC_EUNSUPPORTED); so does a RaBitQ index (BBC_EINVAL)."""
    import oracle
    import synth
    w, ix, q = oracle_pq_index("ivfpq_100k_d128", 4000, 8, 8, 8, 3)
    g = make_gpu_index(bbc, ix)
    with pytest.raises(bbc.BBCError) as e:
        g.search(q, 10, 2, lut_u8=True)
    assert e.value.code == bbc.EUNSUPPORTED
    g.free()
    d, n, nlist = 64, 2000, 4
    w = synth.small_workload("ivfrabitq_1m_d960", n=n, nlist=nlist, nq=2, d=d, seed_index=2)
    x = synth.base_vectors(w)
    tr, ip = synth.kmeans_draws(n, nlist, 64 * nlist, 0)
    rix = oracle.build_ivf_rabitq(x, nlist, tr, ip, synth.rotation_orthogonal(d, 302))
    g = bbc.Index.create_rabitq(rix["centroids"], rix["list_off"], rix["list_ids"], rix["P"], rix["codes"],
                                rix["factors"], x, metric=rix["metric"])
    with pytest.raises(bbc.BBCError) as e:
        g.search(synth.query_vectors(w), 10, 2, lut_u8=True)
    assert e.value.code == bbc.EINVAL
    g.free()
