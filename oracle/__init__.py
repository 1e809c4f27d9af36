"""Oracle for the BBC large-k IVF query path (arxiv 2604.01960).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg use this package.  It shares no code with the GPU library
(``paper_2604_01960_amd``) and never imports it.

The arithmetic lives in ``oracle.c`` (plain C, canonical float32 order, see
its header) and ``oracle64.c`` (O_64, the same query paths in float64, for
distance-error reporting only); this module only marshals numpy arrays
through ctypes and composes the index build from the C steps.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRC64 = os.path.join(_HERE, "oracle64.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=c11", "-Wall", "-Wno-unknown-pragmas"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, canonical float flags)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, _SRC64, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            # ORACLE_LIB: another build of the same sources (the sanitizer
            # test loads an instrumented one)
            path = os.environ.get("ORACLE_LIB")
            if not path:
                path = _LIB_PATH
                if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(
                        os.path.getmtime(_SRC), os.path.getmtime(_SRC64)):
                    build()
            L = C.CDLL(path)
            vp, i32, i64, f32, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_double
            L.orc_canon_l2.restype = f32
            L.orc_canon_l2.argtypes = [vp, vp, i32]
            L.orc_canon_ip.restype = f32
            L.orc_canon_ip.argtypes = [vp, vp, i32]
            L.orc_canon_l2_batch.argtypes = [vp, vp, i64, i32, vp]
            L.orc_canon_ip_batch.argtypes = [vp, vp, i64, i32, vp]
            L.orc_topk_sort.argtypes = [vp, vp, i64, i64, vp, vp]
            L.orc_update.restype = i32
            L.orc_update.argtypes = [vp, i32, i64]
            L.orc_cell_of.restype = i32
            L.orc_cell_of.argtypes = [f32, f32, f32]
            L.orc_codebook.argtypes = [vp, vp, i64, i64, i32, vp, vp, vp]
            L.orc_bucket_of.restype = i32
            L.orc_bucket_of.argtypes = [f32, f32, f32, vp]
            L.orc_collect_bbc.argtypes = [vp, vp, vp, i32, i64, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp]
            L.orc_probe.argtypes = [vp, i64, i32, vp, i32, i32, vp, vp, vp, vp]
            L.orc_pq_lut.argtypes = [vp, vp, i32, i32, i32, vp, vp]
            L.orc_pq_key.restype = f32
            L.orc_pq_key.argtypes = [vp, vp, i32, i32]
            L.orc_pq_keys.argtypes = [vp, vp, i64, i32, i32, vp]
            L.orc_pq_lut_u8.argtypes = [vp, i32, i32, vp, vp, vp]
            L.orc_pq_key_u8.restype = f32
            L.orc_pq_key_u8.argtypes = [vp, vp, i32, i32, f32, f32]
            L.orc_pq_keys_u8.argtypes = [vp, vp, i64, i32, i32, f32, f32, vp]
            L.orc_kmeans_assign.argtypes = [vp, vp, i64, i32, vp, i32, vp]
            L.orc_kmeans_update.argtypes = [vp, vp, i64, i32, vp, i32, vp]
            L.orc_kmeans_train.argtypes = [vp, i32, vp, i64, vp, i32, i32, vp]
            L.orc_pq_train.argtypes = [vp, i64, i32, i32, i32, vp, i32, vp]
            L.orc_pq_encode.argtypes = [vp, i64, i32, i32, i32, vp, vp]
            L.orc_residuals.argtypes = [vp, vp, i64, i32, vp, vp, vp]
            L.orc_search_pq.argtypes = [i64, i32, i32, vp, vp, vp, vp, i32, i32, vp, vp, i32,
                                        vp, i64, vp, vp, f64, i32, vp, vp, vp, vp,
                                        vp, vp, vp, vp, vp, vp, vp, vp]
            L.orc_exact_knn64.argtypes = [vp, i64, i32, vp, i64, i32, i32, vp, vp]
            L.orc_rotate.argtypes = [vp, i32, vp, i64, vp]
            L.orc_rabitq_encode.argtypes = [vp, vp, vp, i32, vp, i32, vp, vp, vp]
            L.orc_rabitq_prep.argtypes = [vp, i32, vp, vp]
            L.orc_rabitq_bounds.argtypes = [vp, vp, i64, i32, vp, vp, i32, f32, f32, f32, vp, vp, vp]
            L.orc_search_rabitq.argtypes = [i64, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, i32, f32,
                                            vp, i64, vp, vp, vp, vp, vp, vp,
                                            vp, vp, vp, vp, vp, vp, vp, vp, vp]
            L.orc_early_rerank.argtypes = [vp, vp, vp, i32, i64, i32, i32, i32, vp, vp, vp, vp]
            L.orc_min_rerank.argtypes = [vp, vp, vp, vp, i64, i64, vp, vp, vp]
            L.o64_search_pq.argtypes = [i64, i32, i32, vp, vp, vp, vp, i32, i32, vp, vp,
                                        vp, i64, vp, vp, f64, vp, vp, vp, vp]
            L.o64_search_rabitq.argtypes = [i64, i32, i32, vp, vp, vp, vp, vp, vp, vp, i32, f64,
                                            vp, i64, vp, vp, vp, vp, vp, vp, vp]
            L.orc_num_threads.restype = C.c_int
            L.orc_set_threads.argtypes = [i32]
            _lib = L
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's loops over queries (n < 1: all host cores)."""
    lib().orc_set_threads(int(n))


# --------------------------------------------------------------------------
# canonical arithmetic
# --------------------------------------------------------------------------

def canon_l2(a, b) -> np.float32:
    a, b = _f32(a), _f32(b)
    return np.float32(lib().orc_canon_l2(_p(a), _p(b), a.shape[0]))


def canon_ip(a, b) -> np.float32:
    a, b = _f32(a), _f32(b)
    return np.float32(lib().orc_canon_ip(_p(a), _p(b), a.shape[0]))


def canon_l2_batch(q, x) -> np.ndarray:
    q, x = _f32(q), _f32(x)
    out = np.empty(x.shape[0], dtype=np.float32)
    lib().orc_canon_l2_batch(_p(q), _p(x), x.shape[0], x.shape[1], _p(out))
    return out


def canon_ip_batch(q, x) -> np.ndarray:
    q, x = _f32(q), _f32(x)
    out = np.empty(x.shape[0], dtype=np.float32)
    lib().orc_canon_ip_batch(_p(q), _p(x), x.shape[0], x.shape[1], _p(out))
    return out


# --------------------------------------------------------------------------
# collector
# --------------------------------------------------------------------------

def topk_sort(keys, ids, kc):
    """First kc of (key, id) ascending."""
    keys, ids = _f32(keys), _i64(ids)
    kc = min(int(kc), keys.shape[0])
    ok = np.empty(kc, np.float32)
    oi = np.empty(kc, np.int64)
    _check(lib().orc_topk_sort(_p(keys), _p(ids), keys.shape[0], kc, _p(ok), _p(oi)), "topk_sort")
    return ok, oi


def update(counts, k) -> int:
    """Threshold bucket: first bucket where the running count reaches k (m if never)."""
    c = _i64(counts)
    return int(lib().orc_update(_p(c), c.shape[0], int(k)))


def cell_of(key, dmin, delta) -> int:
    return int(lib().orc_cell_of(float(np.float32(key)), float(np.float32(dmin)), float(np.float32(delta))))


def bucket_of(key, dmin, delta, mp) -> int:
    mp = np.ascontiguousarray(mp, dtype=np.uint8)
    return int(lib().orc_bucket_of(float(np.float32(key)), float(np.float32(dmin)), float(np.float32(delta)),
                                   _p(mp)))


def codebook(sample_keys, sample_ids, kc, m):
    sk, si = _f32(sample_keys), _i64(sample_ids)
    dmin = np.zeros(1, np.float32)
    delta = np.zeros(1, np.float32)
    mp = np.zeros(256, np.uint8)
    _check(lib().orc_codebook(_p(sk), _p(si), sk.shape[0], int(kc), int(m), _p(dmin), _p(delta), _p(mp)),
           "codebook")
    return dmin[0], delta[0], mp


def collect_bbc(keys, ids, grp_off, kc, m, nsample=8, sample_factor=2) -> Dict[str, object]:
    """Result-buffer workflow over objects grouped by probed list (nearest first)."""
    keys, ids, grp_off = _f32(keys), _i64(ids), _i64(grp_off)
    ngrp = grp_off.shape[0] - 1
    kc = min(int(kc), int(grp_off[-1]))
    dmin = np.zeros(1, np.float32)
    delta = np.zeros(1, np.float32)
    mp = np.zeros(256, np.uint8)
    tau = np.zeros(1, np.int32)
    s = np.zeros(1, np.int64)
    ck = np.empty(max(kc, 1), np.float32)
    ci = np.empty(max(kc, 1), np.int64)
    counts = np.zeros(m, np.int64)
    _check(lib().orc_collect_bbc(_p(keys), _p(ids), _p(grp_off), ngrp, kc, int(m), int(nsample), int(sample_factor),
                                 _p(dmin), _p(delta), _p(mp), _p(tau), _p(s), _p(ck), _p(ci), _p(counts)),
           "collect_bbc")
    return dict(dmin=dmin[0], delta=delta[0], map=mp, tau=int(tau[0]), s=int(s[0]),
                cand_keys=ck[:kc], cand_ids=ci[:kc], counts=counts, kc=kc)


def early_rerank(keys, ids, grp_off, kc, m, nsample=8, sample_factor=2) -> Dict[str, int]:
    """Early re-rank accounting of the improved IVF+PQ search (Algorithm 4):
    predicted threshold bucket, early set size, early objects that are
    candidates, candidates re-ranked afterwards (see oracle.c)."""
    keys, ids, grp_off = _f32(keys), _i64(ids), _i64(grp_off)
    ngrp = grp_off.shape[0] - 1
    tp = np.zeros(1, np.int32)
    out = np.zeros(3, np.int64)
    _check(lib().orc_early_rerank(_p(keys), _p(ids), _p(grp_off), ngrp, int(kc), int(m), int(nsample),
                                  int(sample_factor), _p(tp), _p(out[0:]), _p(out[1:]), _p(out[2:])),
           "early_rerank")
    return dict(tau_pred=int(tp[0]), n_early=int(out[0]), n_early_cand=int(out[1]), n_late=int(out[2]))


def min_rerank(lb, ub, exact, ids, k):
    """Observation 1's minimal re-rank set: (|set|, |set united with the exact
    top-k|, Dist_k)."""
    lb, ub, ex, ids = _f32(lb), _f32(ub), _f32(exact), _i64(ids)
    a = np.zeros(2, np.int64)
    dk = np.zeros(1, np.float32)
    _check(lib().orc_min_rerank(_p(lb), _p(ub), _p(ex), _p(ids), lb.shape[0], int(k), _p(a[0:]), _p(a[1:]),
                                _p(dk)), "min_rerank")
    return int(a[0]), int(a[1]), dk[0]


# --------------------------------------------------------------------------
# probe / PQ
# --------------------------------------------------------------------------

def probe(queries, centroids, nprobe, metric=0):
    q, c = _f32(queries), _f32(centroids)
    nq = q.shape[0]
    npb = _i32(np.broadcast_to(np.asarray(nprobe), (nq,)))
    off = np.zeros(nq + 1, np.int64)
    off[1:] = np.cumsum(npb)
    lists = np.empty(off[-1], np.int32)
    keys = np.empty(off[-1], np.float32)
    _check(lib().orc_probe(_p(q), nq, q.shape[1], _p(c), c.shape[0], int(metric), _p(npb), _p(off),
                           _p(lists), _p(keys)), "probe")
    return lists, keys, off


def pq_lut(q, centroid, codebook_arr, M, ksub):
    q, c, cb = _f32(q), _f32(centroid), _f32(codebook_arr)
    lut = np.empty((M, ksub), np.float32)
    lib().orc_pq_lut(_p(q), _p(c), q.shape[0], M, ksub, _p(cb), _p(lut))
    return lut


def pq_lut_u8(lut):
    """One-byte table of a float32 table [M, ksub]: (u8 [M, ksub], base, delta)."""
    lut = _f32(lut)
    M, ksub = lut.shape
    u = np.empty((M, ksub), np.uint8)
    b = np.zeros(1, np.float32)
    dl = np.zeros(1, np.float32)
    lib().orc_pq_lut_u8(_p(lut), M, ksub, _p(u), _p(b), _p(dl))
    return u, b[0], dl[0]


def pq_keys_u8(u, base, delta, codes):
    """Estimated keys of the rows of codes [n, M] against one one-byte table."""
    u = np.ascontiguousarray(u, dtype=np.uint8)
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    M, ksub = u.shape
    out = np.empty(codes.shape[0], np.float32)
    lib().orc_pq_keys_u8(_p(u), _p(codes), codes.shape[0], M, ksub, float(base), float(delta), _p(out))
    return out


def pq_keys(lut, codes):
    """Estimated keys of the rows of codes [n, M] against one table."""
    lut = _f32(lut)
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    M, ksub = lut.shape
    out = np.empty(codes.shape[0], np.float32)
    lib().orc_pq_keys(_p(lut), _p(codes), codes.shape[0], M, ksub, _p(out))
    return out


# --------------------------------------------------------------------------
# index build
# --------------------------------------------------------------------------

def kmeans_assign(x, c, rows=None):
    x, c = _f32(x), _f32(c)
    rows_a = None if rows is None else _i64(rows)
    n = x.shape[0] if rows is None else rows_a.shape[0]
    out = np.empty(n, np.int32)
    lib().orc_kmeans_assign(_p(x), _p(rows_a), n, x.shape[1], _p(c), c.shape[0], _p(out))
    return out


def kmeans_train(x, train_rows, init_pos, nc, iters):
    x = _f32(x)
    tr, ip = _i64(train_rows), _i64(init_pos)
    c = np.empty((nc, x.shape[1]), np.float32)
    _check(lib().orc_kmeans_train(_p(x), x.shape[1], _p(tr), tr.shape[0], _p(ip), nc, iters, _p(c)),
           "kmeans_train")
    return c


def residuals(x, rows, c, assign_all):
    x, c, a = _f32(x), _f32(c), _i32(assign_all)
    rows_a = None if rows is None else _i64(rows)
    n = x.shape[0] if rows is None else rows_a.shape[0]
    out = np.empty((n, x.shape[1]), np.float32)
    lib().orc_residuals(_p(x), _p(rows_a), n, x.shape[1], _p(c), _p(a), _p(out))
    return out


def pq_train(resid, M, ksub, init_pos, iters):
    r = _f32(resid)
    ip = _i64(init_pos)
    cb = np.empty((M, ksub, r.shape[1] // M), np.float32)
    _check(lib().orc_pq_train(_p(r), r.shape[0], r.shape[1], M, ksub, _p(ip), iters, _p(cb)), "pq_train")
    return cb


def pq_encode(resid, codebook_arr):
    r, cb = _f32(resid), _f32(codebook_arr)
    M, ksub, _ = cb.shape
    codes = np.empty((r.shape[0], M), np.uint8)
    lib().orc_pq_encode(_p(r), r.shape[0], r.shape[1], M, ksub, _p(cb), _p(codes))
    return codes


def build_ivf_pq(x, nlist, M, bits, train_rows, init_pos, pq_rows, pq_init, iters=10):
    """IVF k-means + residual PQ.  Random draws (training rows, seeds) are inputs.

    Returns the index as numpy arrays: lists hold their rows in ascending row
    order; codes are list-ordered, one code per byte."""
    x = _f32(x)
    n, d = x.shape
    if d % M:
        raise ValueError("d must be a multiple of M")
    ksub = 1 << bits
    cent = kmeans_train(x, train_rows, init_pos, nlist, iters)
    assign = kmeans_assign(x, cent)
    order = np.argsort(assign, kind="stable").astype(np.int64)
    counts = np.bincount(assign, minlength=nlist)
    list_off = np.zeros(nlist + 1, np.int64)
    list_off[1:] = np.cumsum(counts)
    pr = _i64(pq_rows)
    cb = pq_train(residuals(x, pr, cent, assign), M, ksub, pq_init, iters)
    codes = pq_encode(residuals(x, order, cent, assign), cb)
    return dict(kind="pq", n=n, d=d, nlist=nlist, M=M, ksub=ksub, bits=bits, metric=0,
                centroids=cent, assign=assign, list_off=list_off, list_ids=order,
                codes=codes, codebook=cb, base=x)


# --------------------------------------------------------------------------
# RaBitQ (rotation, codes, query quantization, bounds)
# --------------------------------------------------------------------------

RABITQ_EPS0 = 1.9   # the cited method's default confidence parameter


def rotate(P, v):
    """y = P^T v for each row v (sequential float32 sums, see oracle.c)."""
    P = _f32(P)
    v = _f32(np.atleast_2d(v))
    D = P.shape[0]
    y = np.empty_like(v)
    lib().orc_rotate(_p(P), D, _p(v), v.shape[0], _p(y))
    return y


def rabitq_encode(x, list_ids, list_off, centroids, P):
    """Codes [n][D/32] uint32 and factors [n][4] (nr, f, g, popcount) of the
    objects in list-slot order."""
    x = _f32(x)
    n, D = x.shape
    nlist = len(list_off) - 1
    codes = np.empty((n, D // 32), np.uint32)
    fac = np.empty((n, 4), np.float32)
    _check(lib().orc_rabitq_encode(_p(x), _p(_i64(list_ids)), _p(_i64(list_off)), nlist, _p(_f32(centroids)),
                                   D, _p(_f32(P)), _p(codes), _p(fac)), "rabitq_encode")
    return codes, fac


def rabitq_prep(y):
    """Quantized query side of one rotated vector: planes [4][D/32] and
    scal = (vl, delta, c1, c2, c3, c4)."""
    y = _f32(y)
    D = y.shape[0]
    planes = np.empty((4, D // 32), np.uint32)
    scal = np.empty(6, np.float32)
    lib().orc_rabitq_prep(_p(y), D, _p(planes), _p(scal))
    return planes, scal


def rabitq_bounds(codes, factors, planes, scal, metric, a, qn=0.0, eps0=RABITQ_EPS0):
    """(key, lb, ub) of the objects for one prepared query side."""
    codes = np.ascontiguousarray(codes, np.uint32)
    factors = _f32(factors)
    n = codes.shape[0]
    D = codes.shape[1] * 32
    key = np.empty(n, np.float32)
    lb = np.empty(n, np.float32)
    ub = np.empty(n, np.float32)
    lib().orc_rabitq_bounds(_p(codes), _p(factors), n, D, _p(np.ascontiguousarray(planes, np.uint32)),
                            _p(_f32(scal)), int(metric), float(a), float(qn), float(eps0), _p(key), _p(lb), _p(ub))
    return key, lb, ub


def build_ivf_rabitq(x, nlist, train_rows, init_pos, P, iters=10, metric=0):
    """IVF k-means + RaBitQ codes of the residuals.  The rotation P and the
    k-means draws are inputs.  Base rows may be float16 (converted exactly)."""
    xf = _f32(x)
    n, d = xf.shape
    if d % 64:
        raise ValueError("RaBitQ needs d to be a multiple of 64")
    cent = kmeans_train(xf, train_rows, init_pos, nlist, iters)
    assign = kmeans_assign(xf, cent)
    order = np.argsort(assign, kind="stable").astype(np.int64)
    counts = np.bincount(assign, minlength=nlist)
    list_off = np.zeros(nlist + 1, np.int64)
    list_off[1:] = np.cumsum(counts)
    codes, fac = rabitq_encode(xf, order, list_off, cent, P)
    return dict(kind="rabitq", n=n, d=d, nlist=nlist, metric=int(metric), centroids=cent,
                rot_centroids=rotate(P, cent), P=_f32(P), assign=assign, list_off=list_off, list_ids=order,
                codes=codes, factors=fac, base=xf, fp16=(np.asarray(x).dtype == np.float16))


def search_rabitq(index, queries, k, nprobe, eps0=RABITQ_EPS0, debug=False):
    """Full RaBitQ query path with the bounded re-rank.  Returns dict(ids,
    dists, counts, off[, probe_*, n_scanned, est_key / est_lb / est_ub (by
    scanned slot, probe order), est_off, n_visited])."""
    q = _f32(queries)
    nq = q.shape[0]
    kk = _i32(np.broadcast_to(np.asarray(k), (nq,)))
    npb = _i32(np.broadcast_to(np.asarray(nprobe), (nq,)))
    off = np.zeros(nq + 1, np.int64)
    off[1:] = np.cumsum(kk)
    res = dict(ids=np.empty(off[-1], np.int64), dists=np.empty(off[-1], np.float32),
               counts=np.empty(nq, np.int32), off=off)
    ix = index
    dbg = [None] * 9
    if debug:
        poff = np.zeros(nq + 1, np.int64)
        poff[1:] = np.cumsum(npb)
        pl = np.empty(poff[-1], np.int32)
        pk = np.empty(poff[-1], np.float32)
        # scanned sizes first (probe only), then the per-object arrays
        sizes = np.diff(ix["list_off"])
        _check(lib().orc_probe(_p(q), nq, ix["d"], _p(_f32(ix["centroids"])), ix["nlist"], ix["metric"],
                               _p(npb), _p(poff), _p(pl), _p(pk)), "probe")
        ns = np.array([sizes[pl[poff[i]:poff[i + 1]]].sum() for i in range(nq)], np.int64)
        eoff = np.zeros(nq + 1, np.int64)
        eoff[1:] = np.cumsum(ns)
        ek = np.empty(eoff[-1], np.float32)
        el = np.empty(eoff[-1], np.float32)
        eu = np.empty(eoff[-1], np.float32)
        nv = np.empty(nq, np.int64)
        nsc = np.empty(nq, np.int64)
        dbg = [pl, pk, poff, nsc, ek, el, eu, eoff, nv]
        res.update(probe_lists=pl, probe_keys=pk, probe_off=poff, n_scanned=nsc, est_key=ek, est_lb=el,
                   est_ub=eu, est_off=eoff, n_visited=nv)
    _check(lib().orc_search_rabitq(
        ix["n"], ix["d"], ix["nlist"], _p(_f32(ix["centroids"])), _p(_f32(ix["rot_centroids"])),
        _p(_f32(ix["P"])), _p(_i64(ix["list_off"])), _p(_i64(ix["list_ids"])),
        _p(np.ascontiguousarray(ix["codes"], np.uint32)), _p(_f32(ix["factors"])), _p(_f32(ix["base"])),
        ix["metric"], float(eps0), _p(q), nq, _p(kk), _p(npb), _p(off), _p(res["ids"]), _p(res["dists"]),
        _p(res["counts"]), *[_p(a) for a in dbg]), "search_rabitq")
    return res


# --------------------------------------------------------------------------
# search
# --------------------------------------------------------------------------

def search_pq(index, queries, k, nprobe, ratio, debug=False, lut_u8=False):
    """Full PQ query path (lut_u8: one-byte tables with integer sums).
    Returns dict(ids, dists, counts, off[, debug...])."""
    q = _f32(queries)
    nq = q.shape[0]
    kk = _i32(np.broadcast_to(np.asarray(k), (nq,)))
    npb = _i32(np.broadcast_to(np.asarray(nprobe), (nq,)))
    off = np.zeros(nq + 1, np.int64)
    off[1:] = np.cumsum(kk)
    ids = np.empty(off[-1], np.int64)
    dists = np.empty(off[-1], np.float32)
    counts = np.empty(nq, np.int32)
    res = dict(ids=ids, dists=dists, counts=counts, off=off)
    pl = pk = poff = ns = nc = ck = ci = coff = None
    if debug:
        poff = np.zeros(nq + 1, np.int64)
        poff[1:] = np.cumsum(npb)
        pl = np.empty(poff[-1], np.int32)
        pk = np.empty(poff[-1], np.float32)
        ns = np.empty(nq, np.int64)
        nc = np.empty(nq, np.int64)
        kcmax = np.ceil(float(ratio) * kk.astype(np.float64)).astype(np.int64)
        coff = np.zeros(nq + 1, np.int64)
        coff[1:] = np.cumsum(kcmax)
        ck = np.empty(coff[-1], np.float32)
        ci = np.empty(coff[-1], np.int64)
        res.update(probe_lists=pl, probe_keys=pk, probe_off=poff, n_scanned=ns, n_cand=nc,
                   cand_keys=ck, cand_ids=ci, cand_off=coff)
    ix = index
    _check(lib().orc_search_pq(
        ix["n"], ix["d"], ix["nlist"], _p(_f32(ix["centroids"])), _p(_i64(ix["list_off"])),
        _p(_i64(ix["list_ids"])), _p(np.ascontiguousarray(ix["codes"], np.uint8)), ix["M"], ix["ksub"],
        _p(_f32(ix["codebook"])), _p(_f32(ix["base"])), ix["metric"],
        _p(q), nq, _p(kk), _p(npb), float(ratio), int(bool(lut_u8)), _p(off), _p(ids), _p(dists), _p(counts),
        _p(pl), _p(pk), _p(poff), _p(ns), _p(nc), _p(ck), _p(ci), _p(coff)), "search_pq")
    return res


def search_pq64(index, queries, k, nprobe, ratio):
    """O_64: the PQ query path in float64 (same steps as search_pq).
    Returns dict(ids, dists (float64), counts, off)."""
    q = _f32(queries)
    nq = q.shape[0]
    kk = _i32(np.broadcast_to(np.asarray(k), (nq,)))
    npb = _i32(np.broadcast_to(np.asarray(nprobe), (nq,)))
    off = np.zeros(nq + 1, np.int64)
    off[1:] = np.cumsum(kk)
    res = dict(ids=np.empty(off[-1], np.int64), dists=np.empty(off[-1], np.float64),
               counts=np.empty(nq, np.int32), off=off)
    ix = index
    _check(lib().o64_search_pq(
        ix["n"], ix["d"], ix["nlist"], _p(_f32(ix["centroids"])), _p(_i64(ix["list_off"])),
        _p(_i64(ix["list_ids"])), _p(np.ascontiguousarray(ix["codes"], np.uint8)), ix["M"], ix["ksub"],
        _p(_f32(ix["codebook"])), _p(_f32(ix["base"])), _p(q), nq, _p(kk), _p(npb), float(ratio), _p(off),
        _p(res["ids"]), _p(res["dists"]), _p(res["counts"])), "search_pq64")
    return res


def search_rabitq64(index, queries, k, nprobe, eps0=RABITQ_EPS0):
    """O_64: the RaBitQ query path with the bounded walk in float64.
    Returns dict(ids, dists (float64), counts, off, n_visited)."""
    q = _f32(queries)
    nq = q.shape[0]
    kk = _i32(np.broadcast_to(np.asarray(k), (nq,)))
    npb = _i32(np.broadcast_to(np.asarray(nprobe), (nq,)))
    off = np.zeros(nq + 1, np.int64)
    off[1:] = np.cumsum(kk)
    res = dict(ids=np.empty(off[-1], np.int64), dists=np.empty(off[-1], np.float64),
               counts=np.empty(nq, np.int32), off=off, n_visited=np.empty(nq, np.int64))
    ix = index
    _check(lib().o64_search_rabitq(
        ix["n"], ix["d"], ix["nlist"], _p(_f32(ix["centroids"])), _p(_f32(ix["P"])), _p(_i64(ix["list_off"])),
        _p(_i64(ix["list_ids"])), _p(np.ascontiguousarray(ix["codes"], np.uint32)), _p(_f32(ix["factors"])),
        _p(_f32(ix["base"])), ix["metric"], float(eps0), _p(q), nq, _p(kk), _p(npb), _p(off), _p(res["ids"]),
        _p(res["dists"]), _p(res["counts"]), _p(res["n_visited"])), "search_rabitq64")
    return res


def exact_knn64(base, queries, k, metric=0):
    """Exact k nearest over all rows in float64, ties by smaller row id."""
    b, q = _f32(base), _f32(queries)
    nq = q.shape[0]
    ids = np.empty((nq, k), np.int64)
    dists = np.empty((nq, k), np.float64)
    _check(lib().orc_exact_knn64(_p(b), b.shape[0], b.shape[1], _p(q), nq, int(k), int(metric),
                                 _p(ids), _p(dists)), "exact_knn64")
    return ids, dists


def rerank_counts(index, queries, k, nprobe, eps0=RABITQ_EPS0):
    """Re-rank sizes of the RaBitQ path per query (row f4): S (objects
    scanned), the bounded walk's visited objects, |C| = objects whose lower
    bound is at most the k-th smallest upper bound, and Observation 1's
    minimal set (objects whose bound interval holds the k-th exact key) and
    that set united with the exact top-k.  Exact keys of every scanned object
    by the canonical float32 order (negated inner product for IP)."""
    q = _f32(queries)
    nq = q.shape[0]
    kk = np.broadcast_to(np.asarray(k), (nq,)).astype(np.int64)
    npb = np.broadcast_to(np.asarray(nprobe), (nq,)).astype(np.int64)
    res = search_rabitq(index, q, kk, npb, eps0=eps0, debug=True)
    out = {f: np.zeros(nq, np.int64) for f in ("S", "visited", "C", "min", "min_out")}
    base = index["base"]
    for i in range(nq):
        lists = res["probe_lists"][res["probe_off"][i]:res["probe_off"][i + 1]]
        ids = np.concatenate([index["list_ids"][index["list_off"][j]:index["list_off"][j + 1]] for j in lists])
        sl = slice(res["est_off"][i], res["est_off"][i + 1])
        lb, ub = res["est_lb"][sl], res["est_ub"][sl]
        rows = np.asarray(base[ids], np.float32)
        ex = canon_l2_batch(q[i], rows) if index["metric"] == 0 else -canon_ip_batch(q[i], rows)
        S = len(ids)
        out["S"][i] = S
        out["visited"][i] = res["n_visited"][i]
        if S > kk[i]:
            U = np.partition(ub, kk[i] - 1)[kk[i] - 1]
            out["C"][i] = int(np.sum(lb <= U))
        else:
            out["C"][i] = S
        a, b, _ = min_rerank(lb, ub, ex, ids, int(kk[i]))
        out["min"][i], out["min_out"][i] = a, b
    return out
