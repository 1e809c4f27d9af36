"""Pins of the oracle's PQ codebook training (per-sub-space k-means on
residual sub-vectors, 10 Lloyd rounds in the build), against closed forms
(CPU): separated dyadic clusters make every float64 sum exact, so each
trained codeword must be the float32-rounded mean of its cluster in its own
sub-space; a codeword that never receives a member keeps its seed."""
import numpy as np

import oracle


def _subspace_clusters(rng, n, M, dsub, ksub, used):
    """Rows whose sub-vector m belongs to cluster lab[:, m] (independent
    labels per sub-space), cluster centres distinct per sub-space, dyadic
    noise (multiples of 1/8)."""
    lab = rng.integers(0, used, (n, M))
    centres = np.zeros((M, ksub, dsub))
    for m in range(M):
        for b in range(ksub):
            centres[m, b] = [100.0 * b + 7.0 * m + 5.0 * e * (m + 1) for e in range(dsub)]
    x = np.zeros((n, M * dsub))
    for m in range(M):
        x[:, m * dsub:(m + 1) * dsub] = centres[m][lab[:, m]] + rng.integers(-16, 17, (n, dsub)) / 8.0
    return x.astype(np.float32), lab


def test_pq_train_gives_exact_subspace_means():
    rng = np.random.default_rng(61)
    n, M, dsub, ksub = 600, 4, 3, 4
    x, lab = _subspace_clusters(rng, n, M, dsub, ksub, ksub)
    init = np.array([[np.flatnonzero(lab[:, m] == b)[0] for b in range(ksub)] for m in range(M)], np.int64)
    cb = oracle.pq_train(x, M, ksub, init, 4)
    assert cb.shape == (M, ksub, dsub)
    for m in range(M):
        sub = x[:, m * dsub:(m + 1) * dsub].astype(np.float64)
        for b in range(ksub):
            want = sub[lab[:, m] == b].mean(0).astype(np.float32)
            np.testing.assert_array_equal(cb[m, b], want, err_msg=f"sub-space {m} codeword {b}")
    # the trained codebook encodes every sub-vector to its own cluster
    np.testing.assert_array_equal(oracle.pq_encode(x, cb), lab)


def test_pq_train_empty_codeword_keeps_its_seed():
    """Sub-space data with 3 clusters for 4 codewords, codeword 3 seeded on
    the same row as codeword 0: in the first round every tie goes to the
    smaller codeword, so codeword 3 has no member and keeps the seed
    sub-vector, while 0..2 become their clusters' means.  (In later rounds
    codeword 0 moves to its mean and the seed row's neighbours may join
    codeword 3, so one round is the case with a closed form.)"""
    rng = np.random.default_rng(62)
    n, M, dsub, ksub = 400, 2, 4, 4
    x, lab = _subspace_clusters(rng, n, M, dsub, ksub, 3)
    init = np.zeros((M, ksub), np.int64)
    for m in range(M):
        for b in range(3):
            init[m, b] = np.flatnonzero(lab[:, m] == b)[0]
        init[m, 3] = init[m, 0]
    cb = oracle.pq_train(x, M, ksub, init, 1)
    for m in range(M):
        sub = x[:, m * dsub:(m + 1) * dsub]
        np.testing.assert_array_equal(cb[m, 3], sub[init[m, 3]])
        for b in range(3):
            want = sub[lab[:, m] == b].astype(np.float64).mean(0).astype(np.float32)
            np.testing.assert_array_equal(cb[m, b], want)


def test_pq_train_zero_iterations_keeps_seeds():
    rng = np.random.default_rng(63)
    x = rng.standard_normal((50, 8)).astype(np.float32)
    init = rng.permutation(50)[:8].reshape(2, 4).astype(np.int64)
    cb = oracle.pq_train(x, 2, 4, init, 0)
    for m in range(2):
        for b in range(4):
            np.testing.assert_array_equal(cb[m, b], x[init[m, b], m * 4:(m + 1) * 4])
