"""Index files on the GPU: the file written for an oracle-built index holds
the oracle's arrays in the documented layout, and the index loaded back
searches exactly like the original and the oracle (PQ and RaBitQ with
float16 rows); an index built on the GPU survives the round trip."""
import numpy as np
import pytest

import oracle
import synth
from helpers import make_gpu_index, oracle_pq_index, read_index_file

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bbc():
    import paper_2604_01960_amd as b
    b.load()
    return b


def _same_search(a, b, q, k, npb):
    ra, rb = a.search(q, k, npb), b.search(q, k, npb)
    for x, y in zip(ra[:3], rb[:3]):
        np.testing.assert_array_equal(x, y)
    return ra


def test_pq_file_round_trip(bbc, tmp_path):
    w, ix, q = oracle_pq_index("ivfpq_100k_d128", 20000, 64, 16, 8, 12)
    g = make_gpu_index(bbc, ix)
    path = str(tmp_path / "pq.bbc")
    print("[case] pq file round trip", flush=True)
    g.save(path)
    f = read_index_file(path)
    assert (f["quant"], f["n"], f["d"], f["nlist"]) == (0, ix["n"], ix["d"], ix["nlist"])
    for key in ("centroids", "list_off", "list_ids", "codebook", "codes", "base"):
        np.testing.assert_array_equal(f[key], ix[key], err_msg=key)
    h = bbc.Index.load(path)
    ref = oracle.search_pq(ix, q, 700, 9, 2.0)
    got = _same_search(g, h, q, 700, 9)
    np.testing.assert_array_equal(got[0], ref["ids"])
    np.testing.assert_array_equal(got[1], ref["dists"])


def test_rabitq_fp16_file_round_trip(bbc, tmp_path):
    d, n, nlist, nq = 256, 5000, 10, 6
    wl = synth.small_workload("ivfrabitq_ip_10m_d768", n=n, nlist=nlist, nq=nq, d=d)
    x = synth.base_vectors(wl)
    q = synth.query_vectors(wl)
    q = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)
    tr, ip = synth.kmeans_draws(n, nlist, 64 * nlist, 0)
    P = synth.rotation_orthogonal(d, 310)
    ix = oracle.build_ivf_rabitq(x, nlist, tr, ip, P, metric=1)
    g = bbc.Index.create_rabitq(ix["centroids"], ix["list_off"], ix["list_ids"], ix["P"], ix["codes"],
                                ix["factors"], x, metric=1, eps0=oracle.RABITQ_EPS0)
    path = str(tmp_path / "rq.bbc")
    print("[case] rabitq fp16 file round trip", flush=True)
    g.save(path)
    f = read_index_file(path)
    assert (f["quant"], f["metric"], f["storage"]) == (1, 1, 1)
    assert np.float32(f["eps0"]) == np.float32(oracle.RABITQ_EPS0)
    for key in ("centroids", "list_off", "list_ids", "P", "codes", "factors"):
        np.testing.assert_array_equal(f[key], ix[key], err_msg=key)
    np.testing.assert_array_equal(f["base"].view(np.uint16), x.view(np.uint16))
    h = bbc.Index.load(path)
    np.testing.assert_array_equal(h.get(bbc.FIELD_ROT_CENTROIDS), ix["rot_centroids"])
    ref = oracle.search_rabitq(ix, q, 400, 4)
    got = _same_search(g, h, q, 400, 4)
    np.testing.assert_array_equal(got[0], ref["ids"])
    np.testing.assert_array_equal(got[1], ref["dists"])


def test_altered_file_is_refused(bbc, tmp_path):
    """One flipped bit anywhere in a saved file's arrays fails the load with
    BBC_EINVAL (checksum mismatch); the untouched file still loads."""
    w, ix, q = oracle_pq_index("ivfpq_100k_d128", 4000, 8, 16, 8, 2)
    g = make_gpu_index(bbc, ix)
    path = str(tmp_path / "flip.bbc")
    print("[case] altered index file", flush=True)
    g.save(path)
    raw = np.fromfile(path, np.uint8)
    for pos in (56, raw.size // 2, raw.size - 9):
        bad = raw.copy()
        bad[pos] ^= 0x10
        bp = str(tmp_path / f"flip_{pos}.bbc")
        bad.tofile(bp)
        with pytest.raises(bbc.BBCError) as e:
            bbc.Index.load(bp)
        assert e.value.code == bbc.EINVAL and "checksum" in str(e.value)
    h = bbc.Index.load(path)
    _same_search(g, h, q, 50, 3)


def test_gpu_built_index_round_trip(bbc, tmp_path):
    w = synth.small_workload("ivfpq4_10m_d96", n=30000, nlist=40, nq=8, pq_m=48, pq_bits=4)
    x = synth.base_vectors(w)
    q = synth.query_vectors(w)
    tr, ip = synth.kmeans_draws(w.n, w.nlist, 64 * w.nlist, 0)
    pr, pi = synth.pq_draws(w.n, 48, 16, w.pq_train, 0)
    g = bbc.Index.build_pq(x, w.nlist, 48, 4, tr, ip, pr, pi)
    path = str(tmp_path / "built.bbc")
    print("[case] gpu-built pq file round trip", flush=True)
    g.save(path)
    h = bbc.Index.load(path)
    for fld in (bbc.FIELD_CENTROIDS, bbc.FIELD_LIST_IDS, bbc.FIELD_CODES, bbc.FIELD_CODEBOOK, bbc.FIELD_BASE):
        np.testing.assert_array_equal(g.get(fld), h.get(fld))
    np.testing.assert_array_equal(h.get(bbc.FIELD_BASE), x)
    _same_search(g, h, q, 2000, 11)
