"""GPU index build (k-means + residual PQ) against the oracle's build: the
same draws must give bit-identical centroids, lists, codebooks and codes."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bbc():
    import paper_2604_01960_amd as b
    b.load()
    return b


@pytest.mark.parametrize("base,n,nlist,M,bits,iters", [
    ("ivfpq_100k_d128", 20000, 64, 16, 8, 6),
    ("ivfpq4_10m_d96", 15000, 48, 48, 4, 5),
    ("ivfpq_100k_d128", 100_000, 256, 16, 8, 10),
])
def test_build_matches_oracle(bbc, base, n, nlist, M, bits, iters):
    w = synth.small_workload(base, n=n, nlist=nlist, nq=1, pq_m=M, pq_bits=bits) if n != synth.workload(base).n \
        else synth.workload(base)
    print(f"[case] build {base} n={n} nlist={nlist} M={M} bits={bits}", flush=True)
    x = synth.base_vectors(w)
    tr, ip = synth.kmeans_draws(w.n, nlist, w.train_per_list * nlist, 0)
    pr, pi = synth.pq_draws(w.n, M, 1 << bits, min(w.pq_train, n // 2), 0)
    ref = oracle.build_ivf_pq(x, nlist, M, bits, tr, ip, pr, pi, iters)
    g = bbc.Index.build_pq(x, nlist, M, bits, tr, ip, pr, pi, iters)
    np.testing.assert_array_equal(g.get(bbc.FIELD_CENTROIDS), ref["centroids"])
    np.testing.assert_array_equal(g.get(bbc.FIELD_LIST_OFF), ref["list_off"])
    np.testing.assert_array_equal(g.get(bbc.FIELD_LIST_IDS), ref["list_ids"])
    np.testing.assert_array_equal(g.get(bbc.FIELD_CODEBOOK), ref["codebook"])
    np.testing.assert_array_equal(g.get(bbc.FIELD_CODES), ref["codes"])
