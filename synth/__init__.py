"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws random numbers and nothing else: it holds none of the
search method's arithmetic (no distances, no tables, no selection).  Every
random quantity the index build or the search consumes is drawn here and
passed in as an input, so the oracle and the GPU library see identical draws.

The datasets of the paper (Wiki, C4, MSMARCO, Deep100M; dataset table in the
experiments section) are not available; the workloads below are Gaussian
mixtures shaped like them: isotropic components around N(0, I) centres, so
that query-to-object distances concentrate as described for the C4 data in
the result-buffer section.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "workload", "mixture_centers", "base_vectors",
    "query_vectors", "kmeans_draws", "pq_draws", "rotation_orthogonal",
    "uneven_k_nprobe", "poisson_arrivals", "small_workload",
]

CHUNK_ROWS = 1 << 20
BLOCK_ROWS = 1 << 15  # rows drawn per block inside a chunk (bounds the float64 temporaries)


@dataclass(frozen=True)
class Workload:
    """Shape of one synthetic workload (data, index and query parameters)."""
    name: str
    n: int                      # number of base vectors
    d: int                      # dimensionality
    ncomp: int                  # Gaussian mixture components
    nlist: int                  # IVF lists
    quant: str                  # "pq" or "rabitq"
    nq: int                     # queries per batch
    k: Tuple[int, ...]          # k values used (uneven workloads draw per query)
    nprobe: int                 # probes (uneven workloads draw per query)
    metric: str = "l2"          # "l2" or "ip"
    sigma: float = 0.3          # isotropic noise std
    var_range: Optional[Tuple[float, float]] = None  # per-dim noise variance ~U(a,b)
    pq_m: int = 0
    pq_bits: int = 8
    fp16: bool = False          # base stored as unit-norm fp16
    seed_index: int = 0         # data seed 100+i, queries 200+i, rotation 300+i, arrivals 400+i
    kmeans_iters: int = 10
    train_per_list: int = 64    # k-means training sample: min(n, train_per_list * nlist)
    pq_train: int = 65536       # PQ training sample size (rows)
    uneven: bool = False
    arrival_qps: float = 0.0    # served from a Poisson stream at this rate (0: batch workload)
    serve_seconds: float = 0.0  # length of the arrival stream

    @property
    def seed_data(self) -> int:
        return 100 + self.seed_index

    @property
    def seed_queries(self) -> int:
        return 200 + self.seed_index

    @property
    def seed_rotation(self) -> int:
        return 300 + self.seed_index

    @property
    def seed_arrivals(self) -> int:
        return 400 + self.seed_index


WORKLOADS = {
    # 100k x 128, 256 components, IVF256 + PQ16x8, 100 queries, k=5000, nprobe=32
    "ivfpq_100k_d128": Workload("ivfpq_100k_d128", 100_000, 128, 256, 256, "pq", 100,
                                (5000,), 32, pq_m=16, pq_bits=8, seed_index=0),
    # 1M x 128, 1024 components, IVF1024 + PQ32x8, 10k queries, k in {5000, 10000}, nprobe=64
    "ivfpq_1m_d128": Workload("ivfpq_1m_d128", 1_000_000, 128, 1024, 1024, "pq", 10_000,
                              (5000, 10000), 64, pq_m=32, pq_bits=8, seed_index=1),
    # 1M x 960, per-dim variance U(0.5,2), IVF1024 + 1-bit RaBitQ, 1000 queries, k=10000, nprobe=128
    "ivfrabitq_1m_d960": Workload("ivfrabitq_1m_d960", 1_000_000, 960, 1024, 1024, "rabitq",
                                  1000, (10000,), 128, var_range=(0.5, 2.0), seed_index=2),
    # 10M x 96, IVF4096 + PQ48x4, 4096 queries with uneven k and nprobe
    "ivfpq4_10m_d96": Workload("ivfpq4_10m_d96", 10_000_000, 96, 4096, 4096, "pq", 4096,
                               (100, 50000), 0, pq_m=48, pq_bits=4, seed_index=3, uneven=True),
    # 10M x 768 unit fp16, inner product, IVF8192 + RaBitQ, served from a Poisson stream
    "ivfrabitq_ip_10m_d768": Workload("ivfrabitq_ip_10m_d768", 10_000_000, 768, 8192, 8192,
                                      "rabitq", 8192, (1000, 20000), 128, metric="ip",
                                      fp16=True, seed_index=4, arrival_qps=2000.0, serve_seconds=30.0),
}


def workload(name: str, **overrides) -> Workload:
    w = WORKLOADS[name]
    return replace(w, **overrides) if overrides else w


def small_workload(base: str, n: int, nlist: int, nq: int, **overrides) -> Workload:
    """A scaled-down copy of a workload (same shape rules, fewer rows)."""
    w = WORKLOADS[base]
    ncomp = max(1, min(w.ncomp, n // 400))
    return replace(w, name=f"{base}_n{n}", n=n, nlist=nlist, nq=nq, ncomp=ncomp, **overrides)


def _noise_scale(w: Workload, ss: np.random.SeedSequence) -> np.ndarray:
    if w.var_range is None:
        return np.full(w.d, w.sigma, dtype=np.float64)
    rng = np.random.default_rng(ss)
    lo, hi = w.var_range
    return np.sqrt(rng.uniform(lo, hi, size=w.d))


def mixture_centers(w: Workload) -> Tuple[np.ndarray, np.ndarray]:
    """Component centres ~ N(0, I_d) and the per-dimension noise std."""
    ss = np.random.SeedSequence(w.seed_data)
    c_ss, v_ss = ss.spawn(2)
    centers = np.random.default_rng(c_ss).standard_normal((w.ncomp, w.d))
    return centers, _noise_scale(w, v_ss)


def _draw_points(w: Workload, n: int, seed: int, out_dtype) -> np.ndarray:
    """Rows in chunks of CHUNK_ROWS, each from its own child seed (labels
    first, then the noise row by row), so chunks are drawn in parallel
    threads and in row blocks without changing a value."""
    centers, scale = mixture_centers(w)
    nchunks = max(1, math.ceil(n / CHUNK_ROWS))
    children = np.random.SeedSequence(seed).spawn(nchunks)
    out = np.empty((n, w.d), dtype=out_dtype)

    def chunk(ci):
        lo = ci * CHUNK_ROWS
        hi = min(n, lo + CHUNK_ROWS)
        rng = np.random.default_rng(children[ci])
        labels = rng.integers(0, w.ncomp, size=hi - lo)
        for b in range(lo, hi, BLOCK_ROWS):
            e = min(hi, b + BLOCK_ROWS)
            pts = centers[labels[b - lo:e - lo]] + rng.standard_normal((e - b, w.d)) * scale
            if w.fp16:
                pts /= np.linalg.norm(pts, axis=1, keepdims=True)
            out[b:e] = pts.astype(out_dtype)

    workers = min(nchunks, os.cpu_count() or 1, 16)
    if workers > 1:
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(chunk, range(nchunks)))
    else:
        for ci in range(nchunks):
            chunk(ci)
    return out


def base_vectors(w: Workload) -> np.ndarray:
    """Base vectors [n, d]: float32, or float16 rows of unit norm when w.fp16."""
    return _draw_points(w, w.n, w.seed_data + 1_000_000, np.float16 if w.fp16 else np.float32)


def query_vectors(w: Workload, nq: Optional[int] = None) -> np.ndarray:
    """Queries [nq, d] float32 from the same mixture, fresh labels and noise.

    For unit-norm workloads the query rows are drawn in float64 and cast;
    their normalisation is done by the caller in float32 (it is part of
    query preparation, not of the draw)."""
    nq = w.nq if nq is None else nq
    wq = replace(w, fp16=False)
    return _draw_points(wq, nq, w.seed_queries, np.float32)


def kmeans_draws(n: int, nlist: int, train_size: int, seed: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Training sample rows (ascending) and the positions in that sample that
    seed the centroids (nlist distinct positions, in draw order)."""
    rng = np.random.default_rng(seed)
    train_size = min(n, train_size)
    if train_size < n:
        train = np.sort(rng.choice(n, size=train_size, replace=False)).astype(np.int64)
    else:
        train = np.arange(n, dtype=np.int64)
    if nlist > train_size:
        raise ValueError("nlist exceeds the training sample")
    init = rng.choice(train_size, size=nlist, replace=False).astype(np.int64)
    return train, init


def pq_draws(n: int, m: int, ksub: int, train_size: int, seed: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """PQ training rows (ascending) and, per sub-space, the ksub distinct
    sample positions that seed its codebook: [m, ksub]."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(2)[1])
    train_size = min(n, train_size)
    if train_size < n:
        train = np.sort(rng.choice(n, size=train_size, replace=False)).astype(np.int64)
    else:
        train = np.arange(n, dtype=np.int64)
    if ksub > train_size:
        raise ValueError("codebook size exceeds the PQ training sample")
    init = np.stack([rng.choice(train_size, size=ksub, replace=False) for _ in range(m)]).astype(np.int64)
    return train, init


def rotation_orthogonal(dim: int, seed: int) -> np.ndarray:
    """A random orthogonal [dim, dim] matrix (Haar distributed: QR of a
    standard normal draw, columns signed by R's diagonal), as float32.  It is
    the random rotation of the RaBitQ codes, drawn here and passed to the
    index build and to the oracle alike."""
    g = np.random.default_rng(seed).standard_normal((dim, dim))
    qm, rm = np.linalg.qr(g)
    qm = qm * np.where(np.diag(rm) < 0, -1.0, 1.0)[None, :]
    return np.ascontiguousarray(qm.astype(np.float32))


def uneven_k_nprobe(nq: int, k_range: Tuple[int, int], nprobe_range: Tuple[int, int],
                    seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """Per-query k log-uniform in k_range and nprobe uniform in nprobe_range (inclusive)."""
    rng = np.random.default_rng(seed)
    lo, hi = k_range
    k = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi + 1), size=nq))).astype(np.int64)
    k = np.clip(k, lo, hi)
    npb = rng.integers(nprobe_range[0], nprobe_range[1] + 1, size=nq).astype(np.int64)
    return k.astype(np.int32), npb.astype(np.int32)


def poisson_arrivals(rate: float, duration_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds, ascending) of a Poisson process."""
    rng = np.random.default_rng(seed)
    n_est = int(rate * duration_s * 1.2 + 100)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_est))
    while t[-1] < duration_s:
        t = np.concatenate([t, t[-1] + np.cumsum(rng.exponential(1.0 / rate, size=n_est))])
    return t[t < duration_s]


def request_stream(w: Workload, pool: int, rate: Optional[float] = None,
                   duration_s: Optional[float] = None) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """A serving workload's requests: Poisson arrival times (seconds), the
    query of each (an index into a pool of `pool` queries, uniform) and its k
    (log-uniform over the workload's k range)."""
    rate = w.arrival_qps if rate is None else rate
    duration_s = w.serve_seconds if duration_s is None else duration_s
    t = poisson_arrivals(rate, duration_s, w.seed_arrivals)
    rng = np.random.default_rng(w.seed_arrivals + 1)
    qi = rng.integers(0, pool, size=t.shape[0]).astype(np.int64)
    k, _ = uneven_k_nprobe(t.shape[0], w.k, (1, 1), w.seed_arrivals + 2)
    return t, qi, k


def integer_vectors(n: int, d: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Small-integer-valued float32 vectors: every distance among them is an
    exactly representable integer, so results are independent of rounding."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(n, d)).astype(np.float32)
