"""MI355X query path for large-k ANN search with a bucket-based result collector.

Thin ctypes binding over the C ABI in ``include/bbc.h`` (``libbbc.so``, built
from ``csrc/`` for gfx950).  This module only marshals arguments; every step
of the search runs in the library's HIP kernels.  There is no fallback: if
the library is missing, importing the binding's entry points raises.

Host numpy arrays use the blocking host-I/O mode; torch tensors on a GPU use
the device-I/O mode on the current torch stream (torch supplies device
memory and streams only).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbbc.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "bbc.h")

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, EBUSY = 0, -1, -2, -3, -4, -6
METRIC_L2, METRIC_IP = 0, 1
QUANT_PQ, QUANT_RABITQ = 0, 1
COLLECT = {"bucket": 0, "heap": 1, "sort": 2, "heap_lds": 3}
FIELD_CENTROIDS, FIELD_LIST_OFF, FIELD_LIST_IDS, FIELD_CODES, FIELD_CODEBOOK = 0, 1, 2, 3, 4
FIELD_RABITQ_CODES, FIELD_RABITQ_FACTORS, FIELD_ROT_CENTROIDS, FIELD_ROTATION, FIELD_BASE = 5, 6, 7, 8, 9
STORAGE_FP32, STORAGE_FP16 = 0, 1
STAGES = {0: "probe", 1: "sample_scan", 2: "scan", 3: "collect", 4: "rerank", 5: "final_topk", 6: "codebook"}


class BBCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bbc error {code}: {msg}")
        self.code = code


class SearchParams(C.Structure):
    _fields_ = [("ncand_ratio", C.c_double), ("collector", C.c_int32), ("buckets", C.c_int32),
                ("nsample", C.c_int32), ("sample_factor", C.c_int32), ("device_io", C.c_int32),
                ("stream", C.c_void_p), ("lut_u8", C.c_int32), ("early_rerank", C.c_int32),
                ("keep_all_keys", C.c_int32)]


class BuildParams(C.Structure):
    _fields_ = [("nlist", C.c_int32), ("kmeans_iters", C.c_int32), ("metric", C.c_int32), ("quant", C.c_int32),
                ("pq_m", C.c_int32), ("pq_bits", C.c_int32),
                ("train_rows", C.c_void_p), ("n_train", C.c_int64), ("init_pos", C.c_void_p),
                ("pq_rows", C.c_void_p), ("n_pq", C.c_int64), ("pq_init", C.c_void_p),
                ("rotation", C.c_void_p), ("rabitq_eps0", C.c_float), ("storage", C.c_int32)]


class RequestInfo(C.Structure):
    _fields_ = [("count", C.c_int32), ("status", C.c_int32), ("latency_ns", C.c_int64), ("n_scanned", C.c_int64),
                ("n_reranked", C.c_int64), ("batch_size", C.c_int64)]


class SearchTrace(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in (
        "probe_lists", "probe_keys", "n_scanned", "n_cand", "n_recheck", "dmin", "delta", "map", "tau", "s",
        "bucket_counts", "n_boundary", "est_keys", "est_off", "cand_ids", "cand_exact", "cand_off",
        "n_sample_lists", "n_survivors", "n_sample_keys", "est_lb", "est_ub", "n_visited", "kernel_forms",
        "walk_path", "tau_pred", "n_early", "n_early_used")]


_lib = None


def load(path: Optional[str] = None):
    """Load libbbc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    # One HIP runtime per process: when torch is present its bundled runtime
    # must be the one loaded first, so that libbbc.so binds to it (same
    # SONAME) instead of bringing up a second runtime next to it.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with paper_2604_01960_amd.build_lib.build()")
    L = C.CDLL(p)
    vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.bbc_index_create_pq.restype = i32
    L.bbc_index_create_pq.argtypes = [i32, i64, i32, i32, i32, vp, vp, vp, i32, i32, vp, vp, vp, C.POINTER(vp)]
    L.bbc_index_create_rabitq.restype = i32
    L.bbc_index_create_rabitq.argtypes = [i32, i64, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, i32, C.c_float,
                                          C.POINTER(vp)]
    L.bbc_build_index.restype = i32
    L.bbc_build_index.argtypes = [i32, vp, i64, i32, C.POINTER(BuildParams), C.POINTER(vp)]
    L.bbc_search.restype = i32
    L.bbc_search.argtypes = [vp, vp, i64, vp, vp, C.POINTER(SearchParams), vp, vp, vp, vp]
    L.bbc_search_traced.restype = i32
    L.bbc_search_noalloc.restype = i32
    L.bbc_search_noalloc.argtypes = [vp, vp, i64, vp, vp, C.POINTER(SearchParams), vp, vp, vp, vp]
    L.bbc_search_traced.argtypes = [vp, vp, i64, vp, vp, C.POINTER(SearchParams), vp, vp, vp, vp,
                                    C.POINTER(SearchTrace)]
    L.bbc_query_bytes.restype = i64
    L.bbc_query_bytes.argtypes = [vp, i32, i32, C.POINTER(SearchParams)]
    L.bbc_index_info.restype = i32
    L.bbc_index_info.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.bbc_index_get.restype = i32
    L.bbc_index_get.argtypes = [vp, i32, vp, i64]
    L.bbc_index_free.restype = None
    L.bbc_index_free.argtypes = [vp]
    L.bbc_stage_timing.restype = i32
    L.bbc_stage_timing.argtypes = [i32]
    L.bbc_stage_times.restype = i32
    L.bbc_stage_times.argtypes = [vp, vp, i32, i32]
    L.bbc_plan_create.restype = i32
    L.bbc_plan_create.argtypes = [vp, i64, vp, vp, C.POINTER(SearchParams), vp, vp, vp, vp, vp, i32, C.POINTER(vp)]
    L.bbc_plan_execute.restype = i32
    L.bbc_plan_execute.argtypes = [vp, vp]
    L.bbc_plan_info.restype = i32
    L.bbc_plan_info.argtypes = [vp, vp, vp, vp, vp, vp]
    L.bbc_plan_free.restype = None
    L.bbc_plan_free.argtypes = [vp]
    L.bbc_server_create.restype = i32
    L.bbc_server_create.argtypes = [vp, C.POINTER(SearchParams), i64, i32, i32, C.POINTER(vp)]
    L.bbc_server_submit.restype = i32
    L.bbc_server_submit.argtypes = [vp, vp, i32, i32, C.POINTER(C.c_uint64)]
    L.bbc_server_poll.restype = i32
    L.bbc_server_poll.argtypes = [vp, C.c_uint64, vp, vp, C.POINTER(RequestInfo)]
    L.bbc_server_wait.restype = i32
    L.bbc_server_wait.argtypes = [vp, C.c_uint64, i32, vp, vp, C.POINTER(RequestInfo)]
    L.bbc_server_stats.restype = i32
    L.bbc_server_stats.argtypes = [vp, vp, vp, vp, vp, vp]
    L.bbc_server_destroy.restype = None
    L.bbc_server_destroy.argtypes = [vp]
    L.bbc_index_save.restype = i32
    L.bbc_index_save.argtypes = [vp, C.c_char_p]
    L.bbc_index_load.restype = i32
    L.bbc_index_load.argtypes = [i32, C.c_char_p, C.POINTER(vp)]
    L.bbc_last_error.restype = C.c_char_p
    L.bbc_last_error.argtypes = []
    _lib = L
    return L


def _check(rc: int):
    if rc != OK:
        raise BBCError(rc, load().bbc_last_error().decode(errors="replace"))


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return int(a.data_ptr())  # torch tensor


def _is_torch_gpu(x) -> bool:
    return hasattr(x, "is_cuda") and bool(x.is_cuda)


def _per_query(v, nq, name) -> np.ndarray:
    a = np.asarray(v)
    if a.ndim == 0:
        a = np.full(nq, int(a), dtype=np.int32)
    if a.shape != (nq,):
        raise ValueError(f"{name} must be a scalar or have shape ({nq},)")
    return np.ascontiguousarray(a, dtype=np.int32)


class Index:
    """A device-resident IVF index (owns its device memory)."""

    def __init__(self, handle: int, device: int = 0):
        self._h = C.c_void_p(handle)
        self.device = device
        n, d, nlist, metric, quant, m, bits, st = (C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32(),
                                                   C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32())
        _check(load().bbc_index_info(self._h, C.byref(n), C.byref(d), C.byref(nlist), C.byref(metric),
                                     C.byref(quant), C.byref(m), C.byref(bits), C.byref(st)))
        self.n, self.d, self.nlist = n.value, d.value, nlist.value
        self.metric, self.quant, self.pq_m, self.pq_bits = metric.value, quant.value, m.value, bits.value
        self.storage = st.value

    # -- construction ------------------------------------------------------
    @classmethod
    def create_pq(cls, centroids, list_off, list_ids, codebook, codes, base, metric=METRIC_L2, device=0):
        cent = _np(centroids, np.float32)
        lo = _np(list_off, np.int64)
        li = _np(list_ids, np.int64)
        cb = _np(codebook, np.float32)
        cd = _np(codes, np.uint8)
        b = _np(base, np.float32)
        nlist, d = cent.shape
        M = cb.shape[0]
        bits = int(round(np.log2(cb.shape[1])))
        h = C.c_void_p()
        _check(load().bbc_index_create_pq(device, b.shape[0], d, nlist, metric, _ptr(cent), _ptr(lo), _ptr(li),
                                          M, bits, _ptr(cb), _ptr(cd), _ptr(b), C.byref(h)))
        return cls(h.value, device)

    @classmethod
    def build_pq(cls, base, nlist, pq_m, pq_bits, train_rows, init_pos, pq_rows, pq_init, iters=10, device=0):
        """Build an IVF-PQ index on the GPU from base vectors and the random draws."""
        b = _np(base, np.float32)
        tr, ip = _np(train_rows, np.int64), _np(init_pos, np.int64)
        pr, pi = _np(pq_rows, np.int64), _np(pq_init, np.int64)
        p = BuildParams(int(nlist), int(iters), METRIC_L2, QUANT_PQ, int(pq_m), int(pq_bits),
                        _ptr(tr), tr.shape[0], _ptr(ip), _ptr(pr), pr.shape[0], _ptr(pi), None, 0.0, STORAGE_FP32)
        h = C.c_void_p()
        _check(load().bbc_build_index(device, _ptr(b), b.shape[0], b.shape[1], C.byref(p), C.byref(h)))
        return cls(h.value, device)

    @classmethod
    def create_rabitq(cls, centroids, list_off, list_ids, rotation, codes, factors, base, metric=METRIC_L2,
                      eps0: float = 0.0, device=0):
        """RaBitQ index from host arrays (codes [n][d/32] uint32 and factors
        [n][4] in list-slot order; base float32 or float16 in row order)."""
        cent = _np(centroids, np.float32)
        lo = _np(list_off, np.int64)
        li = _np(list_ids, np.int64)
        P = _np(rotation, np.float32)
        cd = _np(codes, np.uint32)
        fac = _np(factors, np.float32)
        fp16 = np.asarray(base).dtype == np.float16
        b = _np(base, np.float16 if fp16 else np.float32)
        nlist, d = cent.shape
        h = C.c_void_p()
        _check(load().bbc_index_create_rabitq(device, b.shape[0], d, nlist, int(metric), _ptr(cent), _ptr(lo),
                                              _ptr(li), _ptr(P), _ptr(cd), _ptr(fac), _ptr(b),
                                              STORAGE_FP16 if fp16 else STORAGE_FP32, float(eps0), C.byref(h)))
        return cls(h.value, device)

    @classmethod
    def build_rabitq(cls, base, nlist, train_rows, init_pos, rotation, metric=METRIC_L2, iters=10,
                     eps0: float = 0.0, device=0):
        """Build an IVF-RaBitQ index on the GPU (base float32 or float16)."""
        fp16 = np.asarray(base).dtype == np.float16
        b = _np(base, np.float16 if fp16 else np.float32)
        tr, ip = _np(train_rows, np.int64), _np(init_pos, np.int64)
        P = _np(rotation, np.float32)
        p = BuildParams(int(nlist), int(iters), int(metric), QUANT_RABITQ, 0, 0, _ptr(tr), tr.shape[0], _ptr(ip),
                        None, 0, None, _ptr(P), float(eps0), STORAGE_FP16 if fp16 else STORAGE_FP32)
        h = C.c_void_p()
        _check(load().bbc_build_index(device, _ptr(b), b.shape[0], b.shape[1], C.byref(p), C.byref(h)))
        return cls(h.value, device)

    def free(self):
        if self._h and self._h.value:
            load().bbc_index_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    # -- files -------------------------------------------------------------
    def save(self, path: str):
        """Write the index file (layout in include/bbc.h)."""
        _check(load().bbc_index_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, path: str, device: int = 0) -> "Index":
        h = C.c_void_p()
        _check(load().bbc_index_load(int(device), os.fsencode(path), C.byref(h)))
        return cls(h.value, device)

    # -- introspection -----------------------------------------------------
    def get(self, field: int) -> np.ndarray:
        shapes = {
            FIELD_CENTROIDS: ((self.nlist, self.d), np.float32),
            FIELD_LIST_OFF: ((self.nlist + 1,), np.int64),
            FIELD_LIST_IDS: ((self.n,), np.int64),
            FIELD_CODES: ((self.n, self.pq_m), np.uint8),
            FIELD_CODEBOOK: ((self.pq_m, 1 << self.pq_bits, self.d // max(self.pq_m, 1)), np.float32),
            FIELD_RABITQ_CODES: ((self.n, self.d // 32), np.uint32),
            FIELD_RABITQ_FACTORS: ((self.n, 4), np.float32),
            FIELD_ROT_CENTROIDS: ((self.nlist, self.d), np.float32),
            FIELD_ROTATION: ((self.d, self.d), np.float32),
            FIELD_BASE: ((self.n, self.d), np.float16 if self.storage == STORAGE_FP16 else np.float32),
        }
        shape, dt = shapes[field]
        out = np.empty(shape, dt)
        _check(load().bbc_index_get(self._h, field, _ptr(out), out.nbytes))
        return out

    def query_bytes(self, k: int, nprobe: int, ratio: float = 2.0) -> int:
        p = SearchParams(float(ratio), 0, 0, 0, 0, 0, None)
        v = load().bbc_query_bytes(self._h, int(k), int(nprobe), C.byref(p))
        if v < 0:
            _check(int(v))
        return int(v)

    # -- search --------------------------------------------------------------
    def _params(self, ratio, collector, buckets, nsample, device_io, stream, sample_factor=0, lut_u8=False,
                early_rerank=False, keep_all_keys=False):
        return SearchParams(float(ratio), COLLECT[collector] if isinstance(collector, str) else int(collector),
                            int(buckets), int(nsample), int(sample_factor), int(device_io), stream,
                            int(bool(lut_u8)), int(bool(early_rerank)), int(bool(keep_all_keys)))

    def search(self, queries, k, nprobe, ratio: float = 2.0, collector="bucket", buckets: int = 0,
               nsample: int = 0, out=None, stream=None, lut_u8: bool = False, early_rerank: bool = False, keep_all_keys: bool = False, sample_factor: int = 0):
        """Search a batch.  numpy queries: blocking, returns (ids, dists, counts, offsets)
        as numpy.  torch GPU queries: enqueued on `stream` (default: torch's current
        stream); `out` may hold preallocated (ids, dists, counts) torch tensors."""
        nq = int(queries.shape[0])
        kk = _per_query(k, nq, "k")
        npb = _per_query(nprobe, nq, "nprobe")
        off = np.zeros(nq + 1, np.int64)
        off[1:] = np.cumsum(kk)
        if _is_torch_gpu(queries):
            import torch
            if queries.dtype != torch.float32 or not queries.is_contiguous():
                raise ValueError("queries must be a contiguous float32 tensor")
            if stream is None:
                stream = torch.cuda.current_stream(queries.device).cuda_stream
            if out is None:
                out = (torch.empty(int(off[-1]), dtype=torch.int64, device=queries.device),
                       torch.empty(int(off[-1]), dtype=torch.float32, device=queries.device),
                       torch.empty(nq, dtype=torch.int32, device=queries.device))
            ids, dists, counts = out
            p = self._params(ratio, collector, buckets, nsample, 1, stream, sample_factor=sample_factor, lut_u8=lut_u8, early_rerank=early_rerank, keep_all_keys=keep_all_keys)
            _check(load().bbc_search(self._h, _ptr(queries), nq, _ptr(kk), _ptr(npb), C.byref(p), _ptr(off),
                                     _ptr(ids), _ptr(dists), _ptr(counts)))
            return ids, dists, counts, off
        q = _np(queries, np.float32)
        ids = np.empty(int(off[-1]), np.int64)
        dists = np.empty(int(off[-1]), np.float32)
        counts = np.empty(nq, np.int32)
        p = self._params(ratio, collector, buckets, nsample, 0, stream, sample_factor=sample_factor, lut_u8=lut_u8, early_rerank=early_rerank, keep_all_keys=keep_all_keys)
        _check(load().bbc_search(self._h, _ptr(q), nq, _ptr(kk), _ptr(npb), C.byref(p), _ptr(off),
                                 _ptr(ids), _ptr(dists), _ptr(counts)))
        return ids, dists, counts, off

    def search_noalloc(self, queries, k, nprobe, out, ratio: float = 2.0, collector="bucket", buckets: int = 0,
                       nsample: int = 0, stream=None, lut_u8: bool = False, early_rerank: bool = False, keep_all_keys: bool = False, sample_factor: int = 0):
        """bbc_search_noalloc: torch GPU queries and preallocated (ids, dists, counts)
        torch tensors; enqueued on `stream` (default: torch's current stream).  The
        workspace is the library's fixed per-GPU array (BBC_NOALLOC_MAX_BYTES)."""
        import torch
        nq = int(queries.shape[0])
        kk = _per_query(k, nq, "k")
        npb = _per_query(nprobe, nq, "nprobe")
        off = np.zeros(nq + 1, np.int64)
        off[1:] = np.cumsum(kk)
        if not _is_torch_gpu(queries) or queries.dtype != torch.float32 or not queries.is_contiguous():
            raise ValueError("queries must be a contiguous float32 GPU tensor")
        if stream is None:
            stream = torch.cuda.current_stream(queries.device).cuda_stream
        ids, dists, counts = out
        if ids.numel() < int(off[-1]) or dists.numel() < int(off[-1]) or counts.numel() < nq:
            raise ValueError("output tensors are too small")
        p = self._params(ratio, collector, buckets, nsample, 1, stream, sample_factor=sample_factor, lut_u8=lut_u8, early_rerank=early_rerank, keep_all_keys=keep_all_keys)
        _check(load().bbc_search_noalloc(self._h, _ptr(queries), nq, _ptr(kk), _ptr(npb), C.byref(p), _ptr(off),
                                         _ptr(ids), _ptr(dists), _ptr(counts)))
        return ids, dists, counts, off

    def search_counts(self, queries, k, nprobe, ratio: float = 2.0, buckets: int = 0, nsample: int = 0,
                      lut_u8: bool = False, early_rerank: bool = False, keep_all_keys: bool = False, sample_factor: int = 0):
        """Host search returning only per-query sizes: S, K_c, rechecked lists,
        threshold-bucket size."""
        q = _np(queries, np.float32)
        nq = q.shape[0]
        kk = _per_query(k, nq, "k")
        npb = _per_query(nprobe, nq, "nprobe")
        off = np.zeros(nq + 1, np.int64)
        off[1:] = np.cumsum(kk)
        r = dict(n_scanned=np.empty(nq, np.int64), n_cand=np.empty(nq, np.int64), n_recheck=np.empty(nq, np.int32),
                 n_boundary=np.empty(nq, np.int64), n_sample_lists=np.empty(nq, np.int32),
                 n_survivors=np.empty(nq, np.int64), n_sample_keys=np.empty(nq, np.int64))
        if early_rerank:
            r.update(tau_pred=np.empty(nq, np.int32), n_early=np.empty(nq, np.int64),
                     n_early_used=np.empty(nq, np.int64))
        ids = np.empty(int(off[-1]), np.int64)
        dists = np.empty(int(off[-1]), np.float32)
        counts = np.empty(nq, np.int32)
        tr = SearchTrace(**{f: _ptr(v) for f, v in r.items()})
        p = self._params(ratio, "bucket", buckets, nsample, 0, None, sample_factor=sample_factor, lut_u8=lut_u8, early_rerank=early_rerank, keep_all_keys=keep_all_keys)
        _check(load().bbc_search_traced(self._h, _ptr(q), nq, _ptr(kk), _ptr(npb), C.byref(p), _ptr(off),
                                        _ptr(ids), _ptr(dists), _ptr(counts), C.byref(tr)))
        return r

    def plan(self, queries, k, nprobe, out, ratio: float = 2.0, collector="bucket", buckets: int = 0,
             nsample: int = 0, autotune: bool = False, lut_u8: bool = False, early_rerank: bool = False, keep_all_keys: bool = False, sample_factor: int = 0) -> Plan:
        """Capture the search of a fixed device batch (torch queries and
        `out` = (ids, dists, counts) torch buffers) into a replayable plan."""
        import torch
        nq = int(queries.shape[0])
        kk = _per_query(k, nq, "k")
        npb = _per_query(nprobe, nq, "nprobe")
        off = np.zeros(nq + 1, np.int64)
        off[1:] = np.cumsum(kk)
        ids, dists, counts = out
        assert ids.numel() == off[-1] and dists.numel() == off[-1] and counts.numel() == nq
        p = self._params(ratio, collector, buckets, nsample, 1, None, sample_factor=sample_factor, lut_u8=lut_u8, early_rerank=early_rerank, keep_all_keys=keep_all_keys)
        h = C.c_void_p()
        torch.cuda.synchronize()
        _check(load().bbc_plan_create(self._h, nq, _ptr(kk), _ptr(npb), C.byref(p), _ptr(queries), _ptr(off),
                                      _ptr(ids), _ptr(dists), _ptr(counts), 1 if autotune else 0, C.byref(h)))
        return Plan(h.value, self, (queries, ids, dists, counts))

    def server(self, mem_budget: int, max_slots: int = 1024, lanes: int = 2, ratio: float = 2.0,
               collector="bucket", buckets: int = 0, nsample: int = 0, lut_u8: bool = False, early_rerank: bool = False, keep_all_keys: bool = False, sample_factor: int = 0) -> "Server":
        """A continuous-batching server over this index (bbc_server_*)."""
        p = self._params(ratio, collector, buckets, nsample, 1, None, sample_factor=sample_factor, lut_u8=lut_u8, early_rerank=early_rerank, keep_all_keys=keep_all_keys)
        h = C.c_void_p()
        _check(load().bbc_server_create(self._h, C.byref(p), int(mem_budget), int(max_slots), int(lanes),
                                        C.byref(h)))
        return Server(h.value, self)

    def search_sizes(self, queries, k, nprobe, ratio: float = 2.0, lut_u8: bool = False, early_rerank: bool = False, keep_all_keys: bool = False, sample_factor: int = 0) -> Dict[str, np.ndarray]:
        """Host search returning per-query sizes only: S (n_scanned), the
        candidates re-ranked (n_cand: K_c for PQ, the objects re-ranked for
        RaBitQ) and, for RaBitQ, n_visited."""
        q = _np(queries, np.float32)
        nq = q.shape[0]
        kk = _per_query(k, nq, "k")
        npb = _per_query(nprobe, nq, "nprobe")
        off = np.zeros(nq + 1, np.int64)
        off[1:] = np.cumsum(kk)
        r = dict(n_scanned=np.empty(nq, np.int64), n_cand=np.empty(nq, np.int64))
        fields = ["n_scanned", "n_cand"]
        if self.quant == QUANT_RABITQ:
            r["n_visited"] = np.empty(nq, np.int64)
            fields.append("n_visited")
        tr = SearchTrace(**{f: _ptr(r[f]) for f in fields})
        p = self._params(ratio, "bucket", 0, 0, 0, None, sample_factor=sample_factor, lut_u8=lut_u8, early_rerank=early_rerank, keep_all_keys=keep_all_keys)
        ids = np.empty(int(off[-1]), np.int64)
        dists = np.empty(int(off[-1]), np.float32)
        counts = np.empty(nq, np.int32)
        _check(load().bbc_search_traced(self._h, _ptr(q), nq, _ptr(kk), _ptr(npb), C.byref(p), _ptr(off),
                                        _ptr(ids), _ptr(dists), _ptr(counts), C.byref(tr)))
        return r

    def search_traced(self, queries, k, nprobe, ratio: float = 2.0, collector="bucket", buckets: int = 0,
                      nsample: int = 0, lut_u8: bool = False, early_rerank: bool = False, keep_all_keys: bool = False, sample_factor: int = 0) -> Dict[str, np.ndarray]:
        """Host search that also returns every intermediate of the path."""
        q = _np(queries, np.float32)
        nq = q.shape[0]
        kk = _per_query(k, nq, "k")
        npb = _per_query(nprobe, nq, "nprobe")
        m = buckets if buckets else 256
        off = np.zeros(nq + 1, np.int64)
        off[1:] = np.cumsum(kk)
        L = load()
        p = self._params(ratio, collector, buckets, nsample, 0, None, sample_factor=sample_factor, lut_u8=lut_u8, early_rerank=early_rerank, keep_all_keys=keep_all_keys)
        r = dict(
            ids=np.empty(int(off[-1]), np.int64), dists=np.empty(int(off[-1]), np.float32),
            counts=np.empty(nq, np.int32), off=off,
            probe_lists=np.empty(int(npb.sum()), np.int32), probe_keys=np.empty(int(npb.sum()), np.float32),
            n_scanned=np.empty(nq, np.int64), n_cand=np.empty(nq, np.int64), n_recheck=np.empty(nq, np.int32),
            dmin=np.empty(nq, np.float32), delta=np.empty(nq, np.float32), map=np.empty((nq, 256), np.uint8),
            tau=np.empty(nq, np.int32), s=np.empty(nq, np.int64), bucket_counts=np.empty((nq, m), np.int32),
            n_boundary=np.empty(nq, np.int64), est_off=np.zeros(nq + 1, np.int64),
            cand_off=np.zeros(nq + 1, np.int64), n_sample_keys=np.zeros(nq, np.int64),
            n_survivors=np.zeros(nq, np.int64), kernel_forms=np.full(4, -9, np.int32))
        rabitq = self.quant == QUANT_RABITQ
        if rabitq:
            r["n_visited"] = np.empty(nq, np.int64)
            r["walk_path"] = np.full(nq, -1, np.int32)
        if early_rerank:
            r["tau_pred"] = np.full(nq, -1, np.int32)
            r["n_early"] = np.full(nq, -1, np.int64)
            r["n_early_used"] = np.full(nq, -1, np.int64)
        tr = SearchTrace(**{f: _ptr(r[f]) for f in (
            "probe_lists", "probe_keys", "n_scanned", "n_cand", "n_recheck", "dmin", "delta", "map", "tau", "s",
            "bucket_counts", "n_boundary", "est_off", "cand_off", "n_sample_keys", "n_survivors", "kernel_forms")
            + (("n_visited", "walk_path") if rabitq else ())
            + (("tau_pred", "n_early", "n_early_used") if early_rerank else ())})
        _check(L.bbc_search_traced(self._h, _ptr(q), nq, _ptr(kk), _ptr(npb), C.byref(p), _ptr(off),
                                   _ptr(r["ids"]), _ptr(r["dists"]), _ptr(r["counts"]), C.byref(tr)))
        # second pass for the ragged arrays, now that their sizes are known
        r["est_keys"] = np.empty(int(r["est_off"][-1]), np.float32)
        tr.est_keys = _ptr(r["est_keys"])
        if rabitq:
            r["est_lb"] = np.empty(int(r["est_off"][-1]), np.float32)
            r["est_ub"] = np.empty(int(r["est_off"][-1]), np.float32)
            tr.est_lb = _ptr(r["est_lb"])
            tr.est_ub = _ptr(r["est_ub"])
        else:
            r["cand_ids"] = np.empty(int(r["cand_off"][-1]), np.int64)
            r["cand_exact"] = np.empty(int(r["cand_off"][-1]), np.float32)
            tr.cand_ids = _ptr(r["cand_ids"])
            tr.cand_exact = _ptr(r["cand_exact"])
        _check(L.bbc_search_traced(self._h, _ptr(q), nq, _ptr(kk), _ptr(npb), C.byref(p), _ptr(off),
                                   _ptr(r["ids"]), _ptr(r["dists"]), _ptr(r["counts"]), C.byref(tr)))
        return r


class Plan:
    """A captured batch (bbc_plan_*): fixed queries / outputs on the device,
    replayed as one HIP graph launch by execute()."""

    def __init__(self, handle: int, index: "Index", keep):
        self._h = C.c_void_p(handle)
        self._index = index   # the index must outlive the plan
        self._keep = keep     # buffers the graph reads and writes

    def execute(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(load().bbc_plan_execute(self._h, C.c_void_p(int(s.cuda_stream))))

    def info(self) -> Dict[str, int]:
        v, b, f, c, w = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
        _check(load().bbc_plan_info(self._h, C.byref(v), C.byref(b), C.byref(f), C.byref(c), C.byref(w)))
        return dict(scan_variant=v.value, buckets=b.value, sample_factor=f.value, bcap=c.value,
                    workspace_bytes=w.value)

    def free(self):
        if self._h and self._h.value:
            load().bbc_plan_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """Single requests in, device batches inside (bbc_server_*).  submit()
    returns a ticket; poll() returns None while the result is not ready, else
    (ids, dists, info) with info a dict of bbc_request_info; wait() blocks up
    to a timeout."""

    def __init__(self, handle: int, index: "Index"):
        self._h = C.c_void_p(handle)
        self._index = index   # the index must outlive the server
        self._k: Dict[int, int] = {}
        self._d = int(index.d)

    def submit(self, query, k: int, nprobe: int) -> int:
        q = _np(query, np.float32).reshape(-1)
        if q.shape[0] != self._d:
            raise ValueError(f"query must have {self._d} values")
        t = C.c_uint64()
        _check(load().bbc_server_submit(self._h, _ptr(q), int(k), int(nprobe), C.byref(t)))
        self._k[t.value] = int(k)
        return t.value

    def _take(self, ticket: int, timeout_ms: Optional[int]):
        k = self._k.get(int(ticket))
        if k is None:
            raise BBCError(EINVAL, "unknown ticket")
        ids = np.empty(k, np.int64)
        dists = np.empty(k, np.float32)
        info = RequestInfo()
        if timeout_ms is None:
            rc = load().bbc_server_poll(self._h, int(ticket), _ptr(ids), _ptr(dists), C.byref(info))
        else:
            rc = load().bbc_server_wait(self._h, int(ticket), int(timeout_ms), _ptr(ids), _ptr(dists),
                                        C.byref(info))
        if rc == EBUSY:
            return None
        del self._k[int(ticket)]
        _check(rc)
        return ids, dists, {f: getattr(info, f) for f, _ in RequestInfo._fields_}

    def poll(self, ticket: int):
        return self._take(ticket, None)

    def wait(self, ticket: int, timeout_ms: int = 60000):
        return self._take(ticket, timeout_ms)

    def stats(self) -> Dict[str, int]:
        v = [C.c_int64() for _ in range(5)]
        _check(load().bbc_server_stats(self._h, *[C.byref(x) for x in v]))
        return dict(batches=v[0].value, requests=v[1].value, max_batch=v[2].value, max_inflight=v[3].value,
                    pending=v[4].value)

    def free(self):
        if self._h and self._h.value:
            load().bbc_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def stage_timing(enable: bool = True):
    _check(load().bbc_stage_timing(1 if enable else 0))


def stage_times(reset: bool = False) -> Dict[str, Dict[str, float]]:
    ms = np.zeros(8, np.float64)
    n = np.zeros(8, np.int64)
    _check(load().bbc_stage_times(_ptr(ms), _ptr(n), 8, 1 if reset else 0))
    return {name: dict(ms=float(ms[i]), launches=int(n[i])) for i, name in STAGES.items()}


def declared_symbols() -> Sequence[str]:
    """Names of the functions declared in include/bbc.h."""
    import re
    text = open(HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bbc_[a-z_0-9]+)\s*\(", text)))
