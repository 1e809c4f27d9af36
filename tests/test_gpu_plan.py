"""Captured plans (the batched uneven form): a HIP graph replay of a batch
with per-query k and nprobe gives the oracle's results (ids and distances
bit for bit) and the eager search's, on every replay, with eager work and
synchronisation between replays; autotuning changes nothing in the
results."""
import numpy as np
import pytest

from helpers import make_gpu_index, oracle_pq_index

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bbc():
    import paper_2604_01960_amd as b
    b.load()
    return b


def _bufs(torch, k):
    tot = int(np.sum(k))
    return (torch.empty(tot, dtype=torch.int64, device="cuda"), torch.empty(tot, dtype=torch.float32, device="cuda"),
            torch.empty(len(k), dtype=torch.int32, device="cuda"))


@pytest.mark.parametrize("autotune", [False, True])
def test_pq_plan_replays_match_eager(bbc, autotune):
    import torch
    import synth
    w, ix, q = oracle_pq_index("ivfpq4_10m_d96", 20000, 50, 48, 4, 64)
    g = make_gpu_index(bbc, ix)
    k, npb = synth.uneven_k_nprobe(64, (100, 5000), (4, 50), seed=7)
    import oracle
    qd = torch.from_numpy(q).cuda()
    orc = oracle.search_pq(ix, q, k, npb, 2.0)
    ref = g.search(q, k, npb, ratio=2.0)
    np.testing.assert_array_equal(ref[0], orc["ids"])
    np.testing.assert_array_equal(ref[1], orc["dists"])
    out = _bufs(torch, k)
    print(f"[case] pq plan autotune={autotune}", flush=True)
    plan = g.plan(qd, k, npb, out, ratio=2.0, autotune=autotune)
    info = plan.info()
    assert info["workspace_bytes"] > 0 and info["scan_variant"] in (0, 1, 2, 3, 4)
    if autotune:
        assert info["buckets"] in (64, 128, 256) and info["sample_factor"] in (2, 3, 4)
        assert info["bcap"] in (1024, 4096)
    for rep in range(4):
        for t in out:
            t.fill_(-7)
        plan.execute()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out[0].cpu().numpy(), orc["ids"], err_msg=f"replay {rep}")
        np.testing.assert_array_equal(out[1].cpu().numpy(), orc["dists"])
        np.testing.assert_array_equal(out[2].cpu().numpy(), orc["counts"])
        # eager work on the same index between replays
        again = g.search(q[:5], 300, 7, ratio=2.0)
        assert again[2].shape == (5,)
    # new query contents in the same buffer are searched by the next replay
    q2 = np.ascontiguousarray(q[::-1])
    qd.copy_(torch.from_numpy(q2))
    plan.execute()
    torch.cuda.synchronize()
    orc2 = oracle.search_pq(ix, q2, k, npb, 2.0)
    np.testing.assert_array_equal(out[0].cpu().numpy(), orc2["ids"])
    np.testing.assert_array_equal(out[1].cpu().numpy(), orc2["dists"])
    plan.free()


def test_rabitq_plan_replays_match_eager(bbc):
    import torch
    import oracle
    import synth
    w = synth.small_workload("ivfrabitq_1m_d960", n=6000, nlist=12, nq=16, d=128, seed_index=2)
    x, q = synth.base_vectors(w), synth.query_vectors(w)
    tr, ip = synth.kmeans_draws(6000, 12, 64 * 12, 0)
    P = synth.rotation_orthogonal(128, 302)
    ix = oracle.build_ivf_rabitq(x, 12, tr, ip, P)
    g = bbc.Index.create_rabitq(ix["centroids"], ix["list_off"], ix["list_ids"], ix["P"], ix["codes"],
                                ix["factors"], x)
    k, npb = synth.uneven_k_nprobe(16, (50, 2000), (2, 12), seed=8)
    ref = oracle.search_rabitq(ix, q, k, npb)
    qd = torch.from_numpy(q).cuda()
    out = _bufs(torch, k)
    print("[case] rabitq plan", flush=True)
    plan = g.plan(qd, k, npb, out)
    for rep in range(3):
        plan.execute()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out[0].cpu().numpy(), ref["ids"], err_msg=f"replay {rep}")
        np.testing.assert_array_equal(out[1].cpu().numpy(), ref["dists"])
        g.search(q[:3], 100, 3)
    plan.free()
