"""Shared test helpers: seeded oracle-built indexes and per-step expected
values computed by the oracle only."""
from __future__ import annotations

import functools

import numpy as np

import oracle
import synth


@functools.lru_cache(maxsize=8)
def oracle_pq_index(base_name: str, n: int, nlist: int, M: int, bits: int, nq: int, d: int = 0,
                    iters: int = 10):
    """Index built by the oracle from a scaled-down seeded workload."""
    w = synth.workload(base_name)
    kw = dict(pq_m=M, pq_bits=bits)
    if d:
        kw["d"] = d
    if n == w.n and nlist == w.nlist and nq == w.nq:
        w = synth.workload(base_name, **kw)
    else:
        w = synth.small_workload(base_name, n=n, nlist=nlist, nq=nq, **kw)
    x = synth.base_vectors(w)
    q = synth.query_vectors(w)
    tr, ip = synth.kmeans_draws(w.n, w.nlist, w.train_per_list * w.nlist, 0)
    pr, pi = synth.pq_draws(w.n, M, 1 << bits, w.pq_train, 0)
    ix = oracle.build_ivf_pq(x, w.nlist, M, bits, tr, ip, pr, pi, iters)
    return w, ix, q


def make_gpu_index(bbc, ix):
    return bbc.Index.create_pq(ix["centroids"], ix["list_off"], ix["list_ids"], ix["codebook"], ix["codes"],
                               ix["base"])


def expected_steps(ix, q, k, nprobe, ratio, m, nsample, sample_factor=2, lut_u8=False):
    """Per query, everything the GPU trace reports, from the oracle alone
    (lut_u8: one-byte tables with integer sums)."""
    nq = q.shape[0]
    kk = np.broadcast_to(np.asarray(k), (nq,)).astype(np.int64)
    npb = np.broadcast_to(np.asarray(nprobe), (nq,)).astype(np.int64)
    res = oracle.search_pq(ix, q, kk, npb, ratio, debug=True, lut_u8=lut_u8)
    out = []
    for i in range(nq):
        lists = res["probe_lists"][res["probe_off"][i]:res["probe_off"][i + 1]]
        keys, ids, sizes = [], [], []
        for j in lists:
            lut = oracle.pq_lut(q[i], ix["centroids"][j], ix["codebook"], ix["M"], ix["ksub"])
            sl = slice(ix["list_off"][j], ix["list_off"][j + 1])
            if lut_u8:
                keys.append(oracle.pq_keys_u8(*oracle.pq_lut_u8(lut), ix["codes"][sl]))
            else:
                keys.append(oracle.pq_keys(lut, ix["codes"][sl]))
            ids.append(ix["list_ids"][sl])
            sizes.append(sl.stop - sl.start)
        keys = np.concatenate(keys) if keys else np.zeros(0, np.float32)
        ids = np.concatenate(ids) if ids else np.zeros(0, np.int64)
        goff = np.zeros(len(lists) + 1, np.int64)
        goff[1:] = np.cumsum(sizes)
        kc_t = int(np.ceil(ratio * float(kk[i])))
        col = oracle.collect_bbc(keys, ids, goff, kc_t, m, nsample, sample_factor) if len(keys) else None
        early = oracle.early_rerank(keys, ids, goff, kc_t, m, nsample, sample_factor) if len(keys) else None
        kc = int(res["n_cand"][i])
        cand = res["cand_ids"][res["cand_off"][i]:res["cand_off"][i] + kc]
        exact = np.array([oracle.canon_l2(q[i], ix["base"][c]) for c in cand], np.float32)
        s = slice(res["off"][i], res["off"][i + 1])
        out.append(dict(probe_lists=lists, probe_keys=res["probe_keys"][res["probe_off"][i]:res["probe_off"][i + 1]],
                        est_keys=keys, est_ids=ids, n_scanned=int(res["n_scanned"][i]), n_cand=kc,
                        collect=col, early=early, cand_ids=cand, cand_exact=exact, ids=res["ids"][s],
                        dists=res["dists"][s],
                        count=int(res["counts"][i])))
    return out


def sort_pairs(ids, keys):
    o = np.lexsort((ids, keys))
    return ids[o], keys[o]


def check_trace(tr, exp, m, bucket=True):
    """Every step of a traced GPU search against the oracle's expectation
    (the bucket collector's codebook, counts and threshold only when
    `bucket`)."""
    nq = len(exp)
    for i in range(nq):
        e = exp[i]
        ps = slice(int(np.sum([len(x["probe_lists"]) for x in exp[:i]])),
                   int(np.sum([len(x["probe_lists"]) for x in exp[:i + 1]])))
        np.testing.assert_array_equal(tr["probe_lists"][ps], e["probe_lists"], err_msg=f"probe q{i}")
        np.testing.assert_array_equal(tr["probe_keys"][ps], e["probe_keys"], err_msg=f"probe keys q{i}")
        assert tr["n_scanned"][i] == e["n_scanned"]
        es = slice(tr["est_off"][i], tr["est_off"][i + 1])
        np.testing.assert_array_equal(tr["est_keys"][es], e["est_keys"], err_msg=f"estimated keys q{i}")
        assert tr["n_cand"][i] == e["n_cand"]
        col = e["collect"]
        if bucket and col is not None and e["n_cand"] > 0:
            assert tr["dmin"][i] == col["dmin"] and tr["delta"][i] == col["delta"], f"codebook q{i}"
            np.testing.assert_array_equal(tr["map"][i], col["map"], err_msg=f"map q{i}")
            # buckets below the threshold bucket exactly; from it on only in
            # sum: a key the scan rejects (above its filter bound) is counted
            # in the last bucket, and with the tighter filter of the lists
            # after the sample that bound lies below d_max
            t = int(col["tau"])
            np.testing.assert_array_equal(tr["bucket_counts"][i][:t], col["counts"][:t], err_msg=f"counts q{i}")
            assert int(np.sum(tr["bucket_counts"][i][t:m])) == int(np.sum(col["counts"][t:])), f"counts q{i}"
            assert tr["tau"][i] == col["tau"] and tr["s"][i] == col["s"], f"tau/s q{i}"
        cs = slice(tr["cand_off"][i], tr["cand_off"][i + 1])
        gi, gk = sort_pairs(tr["cand_ids"][cs], tr["cand_exact"][cs])
        ei, ek = sort_pairs(e["cand_ids"], e["cand_exact"])
        np.testing.assert_array_equal(gi, ei, err_msg=f"candidates q{i}")
        np.testing.assert_array_equal(gk, ek, err_msg=f"exact keys q{i}")
        os_ = slice(tr["off"][i], tr["off"][i + 1])
        assert tr["counts"][i] == e["count"]
        np.testing.assert_array_equal(tr["ids"][os_], e["ids"], err_msg=f"ids q{i}")
        np.testing.assert_array_equal(tr["dists"][os_], e["dists"], err_msg=f"dists q{i}")


def word_fnv64(body: bytes) -> int:
    """The index file checksum as documented: FNV-1a over little-endian
    64-bit words of `body` (the last zero-padded)."""
    pad = (-len(body)) % 8
    words = np.frombuffer(body + b"\0" * pad, "<u8")
    h, mask = 0xcbf29ce484222325, (1 << 64) - 1
    for w in words.tolist():
        h = ((h ^ w) * 0x100000001b3) & mask
    return h


def read_index_file(path):
    """Arrays of an index file, parsed from its documented layout (a 56-byte
    header of int32 quant, metric, storage, d, nlist, pq_m, pq_bits, 0, int64
    n, float32 eps0, then the packed arrays and a 64-bit checksum); checks
    that the sizes add up to the file size and the checksum."""
    raw = np.fromfile(path, np.uint8)
    assert raw[:8].tobytes() == b"BBCIDX2\0"
    quant, metric, storage, d, nlist, pq_m, pq_bits, _ = (int(v) for v in raw[8:40].view(np.int32))
    n = int(raw[40:48].view(np.int64)[0])
    eps0 = float(raw[48:52].view(np.float32)[0])
    off = 56

    def take(dtype, shape):
        nonlocal off
        nb = int(np.prod(shape)) * np.dtype(dtype).itemsize
        a = raw[off:off + nb].view(dtype).reshape(shape).copy()
        off += nb
        return a

    f = dict(quant=quant, metric=metric, storage=storage, d=d, nlist=nlist, n=n, eps0=eps0)
    f["centroids"] = take(np.float32, (nlist, d))
    f["list_off"] = take(np.int64, (nlist + 1,))
    f["list_ids"] = take(np.int64, (n,))
    if quant == 0:
        f["codebook"] = take(np.float32, (pq_m, 1 << pq_bits, d // pq_m))
        f["codes"] = take(np.uint8, (n, pq_m))
    else:
        f["P"] = take(np.float32, (d, d))
        f["codes"] = take(np.uint32, (n, d // 32))
        f["factors"] = take(np.float32, (n, 4))
    f["base"] = take(np.float16 if storage == 1 else np.float32, (n, d))
    assert off + 8 == raw.size
    assert int(raw[off:].view("<u8")[0]) == word_fnv64(raw[56:off].tobytes())
    return f
