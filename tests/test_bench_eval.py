"""The benchmark's evaluation helpers (float64 recall and distance error),
checked on the CPU against values fixed by construction."""
import numpy as np
import torch

import bench


def _data(seed=0, n=300, d=8, nq=5):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, d)).astype(np.float32)
    q = rng.standard_normal((nq, d)).astype(np.float32)
    return x, q


def test_ground_truth_and_recall():
    x, q = _data()
    x64 = torch.from_numpy(x).double()
    ids, keys = bench.ground_truth(torch, x64, q, 20, keep_on_device=True)
    d = ((x.astype(np.float64)[None] - q.astype(np.float64)[:, None]) ** 2).sum(-1)
    for i in range(len(q)):
        o = np.argsort(d[i], kind="stable")[:20]
        np.testing.assert_array_equal(np.sort(ids[i].numpy()), np.sort(o))
        np.testing.assert_allclose(keys[i].numpy(), d[i][o], rtol=1e-9)
    # exact results: recall 1; half replaced by non-neighbours: 0.5; pads never count
    got = ids[:, :10].clone()
    assert bench.recall_device(torch, got.reshape(-1), ids, 10) == 1.0
    far = torch.from_numpy(np.argsort(d, axis=1)[:, -5:].copy())
    half = torch.cat([got[:, :5], far], 1)
    assert bench.recall_device(torch, half.reshape(-1), ids, 10) == 0.5
    pad = got.clone()
    pad[:, 7:] = -1
    assert abs(bench.recall_device(torch, pad.reshape(-1), ids, 10) - 0.7) < 1e-12


def test_distance_errors():
    x, q = _data(1)
    x64 = torch.from_numpy(x).double()
    k = 12
    ids, keys = bench.ground_truth(torch, x64, q, k, keep_on_device=True)
    # the exact neighbours with float32-rounded distances: the paper's
    # relative error is 0 and the float32 error is at most one rounding
    d32 = keys.float()
    e = bench.distance_errors(torch, x64, q, ids.reshape(-1), d32.reshape(-1), k, keys)
    assert e["rel_err_mean"] < 1e-12 and e["rel_err_max_query"] < 1e-12  # GT keys use the expanded form
    assert 0 < e["fp32_vs_fp64_max"] <= 2.0 ** -24 * 1.0001 + 1e-12
    # returning the 2nd..(k+1)-th neighbours: error = mean of |D_{i+1} - D_i| / D_i
    ids2, keys2 = bench.ground_truth(torch, x64, q, k + 1, keep_on_device=True)
    shifted = ids2[:, 1:]
    e2 = bench.distance_errors(torch, x64, q, shifted.reshape(-1), keys2[:, 1:].float().reshape(-1), k, keys2)
    a, b = keys2[:, 1:].sqrt(), keys2[:, :k].sqrt()
    want = ((a - b) / b).mean(1)
    assert abs(e2["rel_err_mean"] - float(want.mean())) < 1e-12
    assert abs(e2["rel_err_max_query"] - float(want.max())) < 1e-12
