#!/usr/bin/env python3
"""Benchmark of the large-k IVF-PQ query path on one MI355X.

Workload: 1,000,000 x 128 float32 vectors from a 1024-component Gaussian
mixture (sigma 0.3), IVF with 1024 lists, PQ 32 x 8 bits, batches of 10,000
queries at k = 5000 and k = 10000 (synthetic data; the paper's datasets are
not available).  The index is built on the GPU by the library.

Metric: queries per second at recall@k >= 0.95.  The operating point
(nprobe, candidate ratio r) is the cheapest one whose mean recall on a
query sample reaches 0.95, against exact float64 ground truth.  One step
is one pass of the whole path over the 10,000-query batch for each k, with
queries and results resident in device memory.  Per-stage device time is
measured with HIP events on the search stream during the timed steps; the
dominant stage gives the roofline entry.  The oracle (plain C on the host
cores) is timed on a bounded query sample as the CPU baseline.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector issue peak (non-packed): 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz, one operation (an add, a multiply or a fused multiply-add) per
# lane per clock
VALU_PEAK_TOPS = 39.3


# LDS read peak: 256 CUs x 128 bytes per clock (32 banks of 4 bytes) x 2.4 GHz
LDS_PEAK_GBS = 256 * 128 * 2.4
# last-level (Infinity) cache: a code array that fits is served from it once warm
CACHE_BYTES = 256 << 20


def scan_entry(kernel, avg_ms, code_bytes_pl, lds_bytes_pl, traffic, codes_total_bytes):
    """Roofline entry of a PQ code scan.  Two algorithmic byte counts per
    launch: the code bytes read (one code row per (query, object)) and the
    table bytes gathered from LDS (4 bytes per (query, sub-space, object)).
    When the index's code array fits in the last-level cache the codes are
    cache-served and the scan is held against the LDS roof; otherwise the
    bound is the roof of which the scan reaches the larger fraction.  The
    HBM bytes the counters measured (`traffic`) are reported beside it."""
    sec = avg_ms * 1e-3
    code_rate = code_bytes_pl / sec / 1e9
    lds_rate = lds_bytes_pl / sec / 1e9
    cache_served = codes_total_bytes <= CACHE_BYTES
    hbm_frac, lds_frac = code_rate / HBM_PEAK_GBS, lds_rate / LDS_PEAK_GBS
    if cache_served or lds_frac >= hbm_frac:
        bound, achieved, peak, alg = "lds", lds_rate, LDS_PEAK_GBS, lds_bytes_pl
    else:
        bound, achieved, peak, alg = "hbm", code_rate, HBM_PEAK_GBS, code_bytes_pl
    e = {"kernel": kernel, "bound": bound, "achieved": round(achieved, 1), "peak": round(peak, 1), "unit": "GB/s",
         "frac": round(achieved / peak, 4), "traffic": traffic, "avg_launch_ms": round(avg_ms, 4),
         "algorithmic_bytes_per_launch": int(alg),
         "code_bytes_per_launch": int(code_bytes_pl), "code_bytes_rate_gbs": round(code_rate, 1),
         "lds_table_bytes_per_launch": int(lds_bytes_pl), "lds_frac": round(lds_frac, 4),
         "codes_cache_served": cache_served}
    if traffic:
        e["hbm_traffic_rate_gbs"] = round(traffic / sec / 1e9, 1)
        e["hbm_traffic_frac"] = round(traffic / sec / 1e9 / HBM_PEAK_GBS, 4)
    return e


def rerank_tile_form(d: int) -> bool:
    """Whether the PQ re-rank runs tile-major (rows of at most 32 chunks)."""
    return d % 4 == 0 and d <= 128 and os.environ.get("BBC_RERANK_FORM", "0") == "0"


def rerank_entry(ms_per_launch: float, kc_per_launch: float, d: int) -> dict:
    """Roofline entry of the tile-major PQ re-rank stage: each candidate row is
    staged once per group of queries, so the stage is bound by the 2 d vector
    operations (a subtract and a fused multiply-add per element) of each
    candidate."""
    tops = kc_per_launch * 2 * d / (ms_per_launch * 1e-3) / 1e12
    return {"kernel": "rt_rerank_tile (tile-major re-rank stage, with its pair and candidate sorts)",
            "bound": "alu", "achieved": round(tops, 2), "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": round(tops / VALU_PEAK_TOPS, 4), "traffic": None, "avg_launch_ms": round(ms_per_launch, 4),
            "algorithmic_ops_per_launch": int(kc_per_launch * 2 * d)}
CSRC = os.path.join(ROOT, "paper_2604_01960_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SCAN = "pq_scan_grouped<1, ...> (scan through the relaxed threshold)"
KERNEL_SAMPLE = "pq_scan_grouped<0, ...> (scan of the codebook sample lists)"
METRIC = "QPS at recall@k=0.95, k=5000-10000, bucket vs heap collector; p99 ms"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def measured_traffic(workload, stage, sources):
    """HBM bytes per launch from the committed counter record of this kernel
    and workload, or None when there is none or the kernel's sources have
    changed since the counters were taken."""
    from paper_2604_01960_amd import profiling
    path = os.path.join(PROFILES, f"hbm_traffic_{stage}_{workload}.md")
    if not os.path.exists(path):
        return None
    try:
        rec = profiling.read_traffic(path)
    except ValueError:
        return None
    if rec.get("sources_sha256") != profiling.sources_sha256(sources):
        return None
    return int(rec["traffic_bytes"])


def oracle_sample(run, n_total, seconds, per_call):
    """Calls run(lo, hi) on consecutive query ranges of per_call queries until
    `seconds` of CPU work are spent or n_total queries are done; returns
    (queries done, seconds)."""
    done, t = 0, 0.0
    while done < n_total and t < seconds:
        hi = min(n_total, done + per_call)
        t0 = time.perf_counter()
        run(done, hi)
        t += time.perf_counter() - t0
        done = hi
    return done, t


def recall_at_k(ids, off, gt, k):
    r = []
    for i in range(gt.shape[0]):
        got = ids[off[i]:off[i] + k]
        r.append(len(set(got.tolist()) & set(gt[i, :k].tolist())) / k)
    return float(sum(r) / len(r))


def ground_truth(torch, x_gpu64, q, kmax, metric=0, keep_on_device=False):
    """Exact float64 k nearest (evaluation only): squared L2, or the largest
    inner products for metric 1.  Returns the ids [nq, kmax] (numpy), or,
    with keep_on_device, (ids, keys) as device tensors (keys: squared L2, or
    -<q, x>)."""
    ids, keys = [], []
    xn = (x_gpu64 * x_gpu64).sum(1)
    for s in range(0, q.shape[0], 50):
        qq = torch.from_numpy(q[s:s + 50]).to(x_gpu64.device, torch.float64)
        if metric == 0:
            d = xn[None, :] - 2.0 * (qq @ x_gpu64.T) + (qq * qq).sum(1)[:, None]
        else:
            d = -(qq @ x_gpu64.T)
        t = torch.topk(d, kmax, dim=1, largest=False, sorted=True)
        if keep_on_device:
            ids.append(t.indices)
            keys.append(t.values)
        else:
            ids.append(t.indices.cpu().numpy())
    if keep_on_device:
        return torch.cat(ids), torch.cat(keys)
    import numpy as np
    return np.concatenate(ids)


def recall_device(torch, ids, gt_ids, k):
    """Mean recall@k of result ids [nq * k] (device, -1 pads never match)
    against ground-truth ids [nq, >= k] (device)."""
    nq = gt_ids.shape[0]
    got = ids.view(nq, k)
    hits = 0
    for s in range(0, nq, 256):
        g = torch.sort(gt_ids[s:s + 256, :k], dim=1).values
        r = got[s:s + 256]
        pos = torch.searchsorted(g, r).clamp_(max=k - 1)
        hits += int((torch.gather(g, 1, pos) == r).sum())
    return hits / (nq * k)


def distance_errors(torch, x64, q, ids, dists, k, gt_keys, metric=0):
    """Distance error of the returned results against float64 (evaluation):
     - fp32: |d32 - d64| / |d64| over the returned (id, distance) pairs, with
       d64 the float64 distance of the same id (the float32 path's rounding);
     - rel_err: the relative-error measure of the paper's experiments, the
       mean over queries of (1/k) sum_i |D_i - D*_i| / D*_i with D_i the
       float64 distance of the i-th returned object and D*_i that of the i-th
       true neighbour, on non-squared L2 distances (|<q, x>| for IP).
    ids/dists: [nq * k] device tensors; gt_keys: [nq, >= k] float64 keys."""
    nq = gt_keys.shape[0]
    ids = ids.view(nq, k)
    dists = dists.view(nq, k)
    fmax, fsum, fn, rel_q = 0.0, 0.0, 0, []
    dev = x64.device
    for s in range(0, nq, 16):
        qq = torch.from_numpy(q[s:s + 16]).to(dev, torch.float64)
        i = ids[s:s + 16]
        valid = i >= 0
        rows = x64[i.clamp(min=0)]
        if metric == 0:
            d64 = ((rows - qq[:, None, :]) ** 2).sum(-1)
        else:
            d64 = (rows * qq[:, None, :]).sum(-1)
        d32 = dists[s:s + 16].to(torch.float64)
        den = d64.abs().clamp_min(1e-300)
        fe = ((d32 - d64).abs() / den)[valid]
        if fe.numel():
            fmax = max(fmax, float(fe.max()))
            fsum += float(fe.sum())
            fn += int(fe.numel())
        g = gt_keys[s:s + 16, :k]
        if metric == 0:
            a, b = d64.clamp_min(0).sqrt(), g.clamp_min(0).sqrt()
        else:
            a, b = d64.abs(), g.abs()
        r = ((a - b).abs() / b.clamp_min(1e-300))
        r = torch.where(valid, r, torch.zeros_like(r))
        rel_q.append(r.sum(1) / valid.sum(1).clamp_min(1))
    rel = torch.cat(rel_q)
    return {"fp32_vs_fp64_max": fmax, "fp32_vs_fp64_mean": fsum / max(1, fn), "rel_err_mean": float(rel.mean()),
            "rel_err_max_query": float(rel.max())}


def host_cpu():
    """Host CPU model name and logical core count."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ivfpq_1m_d128")
    ap.add_argument("--nq", type=int, default=0, help="queries per batch (default: the workload's)")
    ap.add_argument("--n", type=int, default=0,
                    help="a scaled-down copy of the workload with this many rows (about 1221 per list)")
    ap.add_argument("--recall-queries", type=int, default=200)
    ap.add_argument("--target-recall", type=float, default=0.95)
    ap.add_argument("--nprobe", type=str, default="", help="fixed nprobe per k, e.g. 128,128 (skips the sweep)")
    ap.add_argument("--ratio", type=str, default="", help="fixed r per k, e.g. 2,2 (skips the sweep)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-queries", type=int, default=3000)
    ap.add_argument("--cpu-queries-1t", type=int, default=200, help="oracle queries timed on one thread")
    ap.add_argument("--o64-queries", type=int, default=100, help="queries searched by the float64 oracle O_64")
    ap.add_argument("--f4-queries", type=int, default=8,
                    help="RaBitQ: queries whose re-rank sizes are set against the minimal re-rank set")
    ap.add_argument("--no-compare", action="store_true", help="skip the heap / sort collector comparison")
    ap.add_argument("--graph", action="store_true",
                    help="batch workloads: also time the steps as captured plans (serial and concurrent)")
    ap.add_argument("--small-k", type=str, default="100,1000",
                    help="small k values (nprobe 64, r 2) at which the collectors are also compared")
    ap.add_argument("--sample-factor", type=int, default=0,
                    help="PQ: the codebook sample holds at least this many times K_c keys (0 = the library's 2)")
    ap.add_argument("--early-rerank", action="store_true",
                    help="PQ: early re-rank during the scan (Algorithm 4)")
    ap.add_argument("--lut-u8", action="store_true",
                    help="PQ: one-byte distance tables with integer sums (fast-scan table accounting)")
    ap.add_argument("--tables", choices=["f32", "u8"], default=None,
                    help="PQ distance tables (default: u8 for the 4-bit fast-scan workload, f32 otherwise)")
    ap.add_argument("--serve-qps", type=float, default=0.0, help="serving: arrival rate (default: the workload's)")
    ap.add_argument("--serve-seconds", type=float, default=None, help="serving: stream length (default: the workload's)")
    ap.add_argument("--serve-budget", type=int, default=16 << 30, help="serving: workspace bytes in flight")
    ap.add_argument("--serve-slots", type=int, default=512, help="serving: requests in flight")
    ap.add_argument("--serve-lanes", type=int, default=2, help="serving: batches in flight")
    ap.add_argument("--serve-warmup", type=int, default=256, help="serving: closed-loop warmup requests")
    ap.add_argument("--capacity-requests", type=int, default=4096,
                    help="serving: closed-loop requests for the capacity figure (0 skips it)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="oracle sample length (seconds of CPU work; the RaBitQ, uneven and serving runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (3 times) for counter calibration")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); multi-GPU runs are not supported",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        # an elementwise kernel that reads and writes BYTES bytes once each
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 4 * n, "kernel": "elementwise mul"}), flush=True)
        return

    import paper_2604_01960_amd as bbc
    import synth

    assert torch.cuda.is_available(), "a GPU is required"
    dev = torch.device("cuda:0")
    bbc.load()
    w = synth.workload(args.workload)
    if args.tables:
        args.lut_u8 = args.tables == "u8"
    elif not args.lut_u8:
        args.lut_u8 = w.quant == "pq" and w.pq_bits == 4  # fast-scan codes: one-byte tables
    if args.n:
        w = synth.small_workload(args.workload, n=args.n, nlist=max(16, args.n // 1221), nq=w.nq)
    if w.arrival_qps:
        return run_serving(args, w, np, torch, bbc, synth, dev)
    if w.quant == "rabitq":
        return run_rabitq(args, w, np, torch, bbc, synth, dev)
    if w.uneven:
        return run_uneven(args, w, np, torch, bbc, synth, dev)
    nq = args.nq or w.nq
    ks = list(w.k)
    t0 = time.time()
    x = synth.base_vectors(w)
    q = synth.query_vectors(w, nq)
    tr, ip = synth.kmeans_draws(w.n, w.nlist, w.train_per_list * w.nlist, 0)
    pr, pi = synth.pq_draws(w.n, w.pq_m, 1 << w.pq_bits, w.pq_train, 0)
    log(f"data {x.shape} queries {q.shape} in {time.time() - t0:.1f}s")
    t0 = time.time()
    index = bbc.Index.build_pq(x, w.nlist, w.pq_m, w.pq_bits, tr, ip, pr, pi, w.kmeans_iters)
    build_s = time.time() - t0
    log(f"GPU index build {build_s:.1f}s")

    # ---- recall operating point ---------------------------------------------
    rq = q[: args.recall_queries]
    gt = None
    x64 = torch.from_numpy(x).to(dev, torch.float64)
    t0 = time.time()
    # float64 exact kNN of the whole batch (evaluation: recall and distance
    # error are computed over every query)
    gt_full_ids, gt_full_keys = ground_truth(torch, x64, q, max(ks), keep_on_device=True)
    log(f"float64 ground truth of {nq} queries in {time.time() - t0:.1f}s")
    if args.recall_queries > 0:
        gt = gt_full_ids[: args.recall_queries].cpu().numpy()
    elif not (args.nprobe and args.ratio):
        raise SystemExit("--recall-queries 0 needs a fixed operating point (--nprobe and --ratio)")
    nprobe_grid = [64, 96, 128, 160, 192, 256]
    ratio_grid = [1.25, 1.5, 1.75, 2.0, 2.5, 3.0, 4.0]
    qd = torch.from_numpy(q).to(dev)
    fixed_np = [int(v) for v in args.nprobe.split(",")] if args.nprobe else []
    fixed_r = [float(v) for v in args.ratio.split(",")] if args.ratio else []
    op = {}
    for ki, k in enumerate(ks):
        if fixed_np and fixed_r:
            rec = None
            if gt is not None:
                ids, _, _, off = index.search(rq, k, fixed_np[ki], ratio=fixed_r[ki], lut_u8=args.lut_u8, early_rerank=args.early_rerank, sample_factor=args.sample_factor)
                rec = recall_at_k(ids, off, gt, k)
            op[k] = dict(nprobe=fixed_np[ki], ratio=fixed_r[ki], recall=rec, sample_factor=args.sample_factor or 2)
            continue
        cands = []
        for npb in nprobe_grid:
            for r in ratio_grid:
                ids, _, _, off = index.search(rq, k, npb, ratio=r, lut_u8=args.lut_u8, early_rerank=args.early_rerank, sample_factor=args.sample_factor)
                rec = recall_at_k(ids, off, gt, k)
                if rec >= args.target_recall:
                    cands.append(dict(nprobe=npb, ratio=r, recall=rec))
                    break
        if not cands:
            raise SystemExit(f"recall {args.target_recall} not reached for k={k}")
        for c in cands:  # one timed full batch per candidate
            index.search(qd, k, c["nprobe"], ratio=c["ratio"], lut_u8=args.lut_u8, early_rerank=args.early_rerank, sample_factor=args.sample_factor)
            torch.cuda.synchronize()
            t = time.perf_counter()
            index.search(qd, k, c["nprobe"], ratio=c["ratio"], lut_u8=args.lut_u8, early_rerank=args.early_rerank, sample_factor=args.sample_factor)
            torch.cuda.synchronize()
            c["probe_ms"] = (time.perf_counter() - t) * 1e3
        # the fastest candidate whose recall over the whole batch reaches the
        # target (the sweep's sample only shortlists)
        best = None
        for c in sorted(cands, key=lambda c: c["probe_ms"]):
            o = index.search(qd, k, c["nprobe"], ratio=c["ratio"], lut_u8=args.lut_u8, early_rerank=args.early_rerank, sample_factor=args.sample_factor)
            torch.cuda.synchronize()
            c["recall_batch"] = recall_device(torch, o[0], gt_full_ids, k)
            if c["recall_batch"] >= args.target_recall:
                best = c
                break
        if best is None:
            best = max(cands, key=lambda c: c["recall_batch"])
        op[k] = best
        # the codebook sample's size (a tighter relaxed threshold against a
        # costlier codebook; results are identical): the fastest of 2, 3, 4
        # times K_c on the whole batch, unless given
        if args.sample_factor:
            best["sample_factor"] = args.sample_factor
        else:
            sf_ms = {}
            for f in (2, 3, 4):
                index.search(qd, k, best["nprobe"], ratio=best["ratio"], lut_u8=args.lut_u8,
                             early_rerank=args.early_rerank, sample_factor=f)
                torch.cuda.synchronize()
                t = time.perf_counter()
                index.search(qd, k, best["nprobe"], ratio=best["ratio"], lut_u8=args.lut_u8,
                             early_rerank=args.early_rerank, sample_factor=f)
                torch.cuda.synchronize()
                sf_ms[f] = (time.perf_counter() - t) * 1e3
            best["sample_factor"] = min(sf_ms, key=sf_ms.get)
            log(f"k={k}: sample factor times {sf_ms}")
        log(f"k={k}: candidates {cands} -> {best}")

    # ---- timed steps ------------------------------------------------------------
    outs = {}
    for k in ks:
        outs[k] = (torch.empty(nq * k, dtype=torch.int64, device=dev), torch.empty(nq * k, dtype=torch.float32, device=dev),
                   torch.empty(nq, dtype=torch.int32, device=dev))

    def step(per_k_events=None):
        for k in ks:
            if per_k_events is not None:
                per_k_events[k][0].record()
            index.search(qd, k, op[k]["nprobe"], ratio=op[k]["ratio"], out=outs[k], lut_u8=args.lut_u8, early_rerank=args.early_rerank, sample_factor=op[k]["sample_factor"])
            if per_k_events is not None:
                per_k_events[k][1].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    bbc.stage_times(reset=True)
    bbc.stage_timing(True)
    lat = {k: [] for k in ks}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev_all = []
    for _ in range(args.steps):
        ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for k in ks}
        step(ev)
        ev_all.append(ev)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    bbc.stage_timing(False)
    stages = bbc.stage_times(reset=True)
    for ev in ev_all:
        for k in ks:
            lat[k].append(ev[k][0].elapsed_time(ev[k][1]))
    total_q = nq * len(ks) * args.steps
    value = total_q / elapsed
    per_k = {}
    for k in ks:
        arr = np.array(lat[k])
        # recall and distance error of the last timed step's results, every query
        rec = recall_device(torch, outs[k][0], gt_full_ids, k)
        derr = distance_errors(torch, x64, q, outs[k][0], outs[k][1], k, gt_full_keys)
        per_k[str(k)] = dict(nprobe=op[k]["nprobe"], ratio=op[k]["ratio"], sample_factor=op[k]["sample_factor"],
                             recall=round(rec, 4),
                             recall_queries=nq, recall_target_reached=rec >= args.target_recall,
                             dist_err={n: float(f"{v:.3e}") for n, v in derr.items()},
                             qps=round(nq / (arr.mean() / 1e3), 1), batch_ms_p50=round(float(np.percentile(arr, 50)), 3),
                             batch_ms_p99=round(float(np.percentile(arr, 99)), 3))
        log(f"k={k}: recall over {nq} queries {rec:.4f}, distance error {derr}")

    # ---- the same steps replayed as captured plans (one per k, the operating
    # point above): in turn on one stream, and the k batches on streams of
    # their own at once (each plan has its own workspace); results equal the
    # eager step's --------------------------------------------------------------
    graph = None
    if args.graph:
        outs_g = {k: tuple(torch.empty_like(t) for t in outs[k]) for k in ks}
        plans = {k: index.plan(qd, k, op[k]["nprobe"], outs_g[k], ratio=op[k]["ratio"], lut_u8=args.lut_u8,
                               early_rerank=args.early_rerank, sample_factor=op[k]["sample_factor"]) for k in ks}
        streams = {k: torch.cuda.Stream() for k in ks}

        def gstep_serial():
            for k in ks:
                plans[k].execute()

        def gstep_concurrent():
            cur = torch.cuda.current_stream()
            for k in ks:
                streams[k].wait_stream(cur)
                plans[k].execute(streams[k])
            for k in ks:
                cur.wait_stream(streams[k])

        graph = {}
        for name, fn in (("serial", gstep_serial), ("concurrent", gstep_concurrent)):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                fn()
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            same = all(bool(torch.equal(outs_g[k][0], outs[k][0])) and bool(torch.equal(outs_g[k][1], outs[k][1]))
                       for k in ks)
            graph[name] = dict(qps=round(total_q / el, 1), ms_per_step=round(el / args.steps * 1e3, 3),
                               identical_to_eager=same)
            log(f"graph {name}: {graph[name]}")
        for pl in plans.values():
            pl.free()
        del plans

    # ---- collector comparison: same batch, same operating point ---------------
    collectors = {}
    if not args.no_compare:
        for k in ks:
            res_k = {}
            ref = None
            # "bucket": the production path (the scan keeps only keys at or
            # below the relaxed threshold d_max); "bucket_all_keys": every
            # scanned key reaches the collector, as for heap and sort
            for name in ("bucket", "bucket_all_keys", "heap", "heap_lds", "sort"):
                col = "bucket" if name.startswith("bucket") else name
                kw = dict(collector=col, lut_u8=args.lut_u8, early_rerank=args.early_rerank and col == "bucket",
                          sample_factor=op[k]["sample_factor"],
                          keep_all_keys=name == "bucket_all_keys")
                o = (torch.empty_like(outs[k][0]), torch.empty_like(outs[k][1]), torch.empty_like(outs[k][2]))
                index.search(qd, k, op[k]["nprobe"], ratio=op[k]["ratio"], out=o, **kw)
                torch.cuda.synchronize()
                bbc.stage_times(reset=True)
                bbc.stage_timing(True)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                index.search(qd, k, op[k]["nprobe"], ratio=op[k]["ratio"], out=o, **kw)
                e1.record()
                torch.cuda.synchronize()
                bbc.stage_timing(False)
                st = bbc.stage_times(reset=True)
                if ref is None:
                    ref = o
                same = bool(torch.equal(o[0], ref[0]) and torch.equal(o[1], ref[1]) and torch.equal(o[2], ref[2]))
                scan_ms = st["sample_scan"]["ms"] + st["scan"]["ms"]
                res_k[name] = dict(batch_ms=round(e0.elapsed_time(e1), 3), collector_ms=round(st["collect"]["ms"], 3),
                                   scan_ms=round(scan_ms, 3), qps=round(nq / (e0.elapsed_time(e1) / 1e3), 1),
                                   identical_to_bucket=same)
                log(f"k={k} collector {name}: {res_k[name]}")
            collectors[str(k)] = res_k

    # ---- small k: the bucket collector must not slow it down -------------------
    small_k = {}
    if not args.no_compare and args.small_k:
        for k in [int(v) for v in args.small_k.split(",")]:
            res_k, ref = {}, None
            o = (torch.empty(nq * k, dtype=torch.int64, device=dev), torch.empty(nq * k, dtype=torch.float32, device=dev),
                 torch.empty(nq, dtype=torch.int32, device=dev))
            for col in ("bucket", "heap", "sort"):
                index.search(qd, k, 64, ratio=2.0, collector=col, out=o)
                torch.cuda.synchronize()
                ms = []
                for _ in range(3):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    index.search(qd, k, 64, ratio=2.0, collector=col, out=o)
                    e1.record()
                    torch.cuda.synchronize()
                    ms.append(e0.elapsed_time(e1))
                cur = [t.clone() for t in o]
                if ref is None:
                    ref = cur
                same = all(bool(torch.equal(a_, b_)) for a_, b_ in zip(cur, ref))
                res_k[col] = dict(batch_ms=round(float(np.median(ms)), 3), qps=round(nq / (np.median(ms) / 1e3), 1),
                                  identical_to_bucket=same)
            small_k[str(k)] = res_k
            log(f"small k={k}: {res_k}")

    # ---- sizes for the algorithmic byte counts ---------------------------------
    sizes = {}
    for k in ks:
        c = index.search_counts(q, k, op[k]["nprobe"], ratio=op[k]["ratio"], lut_u8=args.lut_u8, early_rerank=args.early_rerank, sample_factor=op[k]["sample_factor"])
        sizes[k] = dict(S=int(c["n_scanned"].sum()), Kc=int(c["n_cand"].sum()),
                        sample_keys=int(c["n_sample_keys"].sum()),
                        recheck_mean=float(c["n_recheck"].mean()), boundary_mean=float(c["n_boundary"].mean()),
                        sample_lists_mean=float(c["n_sample_lists"].mean()),
                        survivors_mean=float(c["n_survivors"].mean()))
        if args.early_rerank:
            sizes[k].update(early_mean=float(c["n_early"].mean()), early_used_mean=float(c["n_early_used"].mean()))
    d = w.d
    code_bytes = w.pq_m if w.pq_bits == 8 else (w.pq_m + 1) // 2
    # algorithmic bytes per step of the kernels that dominate their stage
    algo = {
        # scan of the non-sample lists: one code row per scanned object
        "scan": sum(sizes[k]["S"] - sizes[k]["sample_keys"] for k in ks) * code_bytes,
        # scan of the codebook sample lists
        "sample_scan": sum(sizes[k]["sample_keys"] for k in ks) * code_bytes,
        # re-rank: a d*4-byte row plus its 4-byte slot per candidate
        "rerank": sum(sizes[k]["Kc"] for k in ks) * (4 * d + 4),
        # bucket collection: each survivor's (key, slot) read once, each
        # candidate's slot written once
        "collect": sum(int(round(sizes[k]["survivors_mean"] * nq)) * 8 + sizes[k]["Kc"] * 4 for k in ks),
    }
    kernels = {"scan": (KERNEL_SCAN, [os.path.join(CSRC, f) for f in ("pq_scan.hip", "common.h", "kernels.h")]),
               "rerank": ("rerank_half_kernel", [os.path.join(CSRC, f) for f in ("rerank.hip", "common.h", "kernels.h")]),
               "sample_scan": (KERNEL_SAMPLE, [os.path.join(CSRC, f) for f in ("pq_scan.hip", "common.h", "kernels.h")]),
               "collect": ("collect_bucket_kernel", [os.path.join(CSRC, f) for f in ("collect.hip", "common.h",
                                                                                     "kernels.h")])}
    entries = {}
    for name in algo:
        st = stages[name]
        if st["launches"] == 0:
            continue
        avg_ms = st["ms"] / st["launches"]
        bytes_total = algo[name] * args.steps
        bytes_per_launch = bytes_total / st["launches"]
        gbs = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        if name == "rerank" and rerank_tile_form(d):
            kc_pl = sum(sizes[k]["Kc"] for k in ks) * args.steps / st["launches"]
            entries[name] = rerank_entry(avg_ms, kc_pl, d)
            continue
        if name in ("scan", "sample_scan"):
            entries[name] = scan_entry(kernels[name][0], avg_ms, bytes_per_launch,
                                       bytes_per_launch / code_bytes * w.pq_m * (1 if args.lut_u8 else 4),
                                       measured_traffic(w.name, name, kernels[name][1]), w.n * code_bytes)
            continue
        entries[name] = {"kernel": kernels[name][0], "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "traffic": measured_traffic(w.name, name, kernels[name][1]),
                         "avg_launch_ms": round(avg_ms, 4), "algorithmic_bytes_per_launch": int(bytes_per_launch)}
    dominant = max(entries, key=lambda s: stages[s]["ms"])
    roof = entries[dominant]
    others = {n: e for n, e in entries.items() if n != dominant}
    stage_ms = {s: round(v["ms"] / max(1, args.steps), 4) for s, v in stages.items()}

    # ---- oracle CPU baseline, and the oracle's verdict on the GPU results ------
    cpu = None
    oracle_match = None
    fp64_oracle = None
    if not args.no_cpu:
        import oracle
        t0 = time.time()
        oix = oracle.build_ivf_pq(x, w.nlist, w.pq_m, w.pq_bits, tr, ip, pr, pi, w.kmeans_iters)
        log(f"oracle index build {time.time() - t0:.1f}s")
        # the oracle searches its own build; the GPU searched the GPU build:
        # the comparison below needs them to be the same index
        build_same = bool(np.array_equal(index.get(bbc.FIELD_CENTROIDS), oix["centroids"])
                          and np.array_equal(index.get(bbc.FIELD_LIST_IDS), oix["list_ids"])
                          and np.array_equal(index.get(bbc.FIELD_CODEBOOK), oix["codebook"])
                          and np.array_equal(index.get(bbc.FIELD_CODES), oix["codes"]))
        nqc = min(args.cpu_queries, nq)
        oracle.set_threads(0)
        t_cpu = 0.0
        mism_ids = mism_d = 0
        for k in ks:
            t0 = time.perf_counter()
            ref = oracle.search_pq(oix, q[:nqc], k, op[k]["nprobe"], op[k]["ratio"], lut_u8=args.lut_u8)
            t_cpu += time.perf_counter() - t0
            gi = outs[k][0][: nqc * k].cpu().numpy().reshape(nqc, k)
            gd = outs[k][1][: nqc * k].cpu().numpy().reshape(nqc, k)
            gc = outs[k][2][:nqc].cpu().numpy()
            ri, rd = ref["ids"].reshape(nqc, k), ref["dists"].reshape(nqc, k)
            mism_ids += int(np.sum(np.any(ri != gi, axis=1) | (ref["counts"] != gc)))
            mism_d += int(np.sum(np.any(rd.view(np.uint32) != gd.view(np.uint32), axis=1)))
        threads = oracle.num_threads()
        # one thread, on a shorter sample
        n1 = max(1, min(nqc, args.cpu_queries_1t))
        oracle.set_threads(1)
        t1 = 0.0
        for k in ks:
            t0 = time.perf_counter()
            oracle.search_pq(oix, q[:n1], k, op[k]["nprobe"], op[k]["ratio"], lut_u8=args.lut_u8)
            t1 += time.perf_counter() - t0
        oracle.set_threads(0)
        model, ncpu = host_cpu()
        cpu = {"value": round(nqc * len(ks) / t_cpu, 2), "unit": "queries/s", "cores": threads,
               "kind": "oracle", "value_1_thread": round(n1 * len(ks) / t1, 2), "cpu_model": model,
               "host_logical_cpus": ncpu,
               "sample": f"first {nqc} queries of the batch at each k in {ks} on {threads} threads ({t_cpu:.1f}s), "
                         f"first {n1} on 1 thread ({t1:.1f}s); same nprobe/r operating point, oracle-built index"}
        oracle_match = {"queries": nqc * len(ks), "index_build_identical": build_same,
                        "queries_with_different_ids": mism_ids, "queries_with_different_dists": mism_d,
                        "match": build_same and mism_ids == 0 and mism_d == 0,
                        "what": "ids, counts and float32 distance bits of the GPU's timed-step results against "
                                "the oracle on the same queries"}
        log(f"oracle match {oracle_match}")
        # O_64, the float64 shadow of the path, on a few queries
        n64 = min(args.o64_queries, nq)
        if n64 > 0:
            agree = []
            for k in ks:
                r64 = oracle.search_pq64(oix, q[:n64], k, op[k]["nprobe"], op[k]["ratio"])
                gi = outs[k][0][: n64 * k].cpu().numpy().reshape(n64, k)
                i64 = r64["ids"].reshape(n64, k)
                agree.append(float(np.mean([len(np.intersect1d(gi[j], i64[j])) / k for j in range(n64)])))
            fp64_oracle = {"queries": n64 * len(ks), "id_overlap_per_k": dict(zip(map(str, ks), agree)),
                           "what": "mean |GPU ids & O_64 ids| / k: the same path run in float64"}
            log(f"O_64 {fp64_oracle}")

    res = {
        "metric": METRIC, "value": round(value, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "nlist": w.nlist, "pq": f"{w.pq_m}x{w.pq_bits}",
                   "nq": nq, "k": ks, "collector": "bucket", "buckets": 256, "nsample": 8,
                   "tables": "u8" if args.lut_u8 else "f32", "early_rerank": bool(args.early_rerank)},
        "per_k": per_k,
        "latency_ms": {"p50": round(float(np.percentile(sum(lat.values(), []), 50)), 3),
                       "p99": round(float(np.percentile(sum(lat.values(), []), 99)), 3),
                       "what": "device time of one 10,000-query batch"},
        "stage_ms_per_step": stage_ms,
        "graph": graph,
        "collectors": collectors,
        "collectors_small_k": small_k,
        "sizes": sizes,
        "roofline": roof,
        "roofline_other_kernels": others,
        "cpu_baseline": cpu,
        "oracle_match": oracle_match,
        "fp64_oracle": fp64_oracle,
        "build_s": round(build_s, 2),
    }
    print(json.dumps(res), flush=True)


def run_uneven(args, w, np, torch, bbc, synth, dev):
    """Batched uneven PQ workload: per-query k (log-uniform) and nprobe
    (uniform), one batch per step, timed eagerly and as a captured plan (one
    graph launch, autotuned scan geometry and bucket count)."""
    nq = args.nq or w.nq
    k, npb = synth.uneven_k_nprobe(nq, (100, 50000), (16, 256), seed=w.seed_queries)
    t0 = time.time()
    x = synth.base_vectors(w)
    q = synth.query_vectors(w, nq)
    tr, ip = synth.kmeans_draws(w.n, w.nlist, w.train_per_list * w.nlist, 0)
    pr, pi = synth.pq_draws(w.n, w.pq_m, 1 << w.pq_bits, w.pq_train, 0)
    log(f"data {x.shape} queries {q.shape} in {time.time() - t0:.1f}s")
    t0 = time.time()
    index = bbc.Index.build_pq(x, w.nlist, w.pq_m, w.pq_bits, tr, ip, pr, pi, w.kmeans_iters)
    build_s = time.time() - t0
    log(f"GPU index build {build_s:.1f}s")
    ns = min(args.recall_queries, nq)
    rsel = np.linspace(0, nq - 1, ns).astype(np.int64)  # a spread sample of the batch (k varies)
    gt = None
    if ns:
        x64 = torch.from_numpy(x).to(dev, torch.float64)
        gt = ground_truth(torch, x64, q[rsel], int(k[rsel].max()))
        del x64
        torch.cuda.empty_cache()
    elif not args.ratio:
        raise SystemExit("--recall-queries 0 needs a fixed --ratio")

    def mean_recall(ids, off):
        r = [len(set(ids[off[j]:off[j + 1]].tolist()) & set(gt[j, :k[i]].tolist())) / k[i] for j, i in enumerate(rsel)]
        return float(np.mean(r))

    if args.ratio:
        ratio = float(args.ratio.split(",")[0])
        rec = None
        if gt is not None:
            ids, _, _, off = index.search(q[rsel], k[rsel], npb[rsel], ratio=ratio, lut_u8=args.lut_u8, early_rerank=args.early_rerank, sample_factor=args.sample_factor)
            rec = mean_recall(ids, off)
    else:
        # nprobe is fixed per query by the workload, so a query with few
        # probes and a large k may not reach the target at any r: take the
        # first r that reaches it, else the knee of the saturated curve (the
        # smallest r within 0.005 of the best recall)
        ratio, rec, curve = None, None, []
        for r in (1.5, 2.0, 3.0, 4.0, 6.0, 8.0):
            ids, _, _, off = index.search(q[rsel], k[rsel], npb[rsel], ratio=r, lut_u8=args.lut_u8, early_rerank=args.early_rerank, sample_factor=args.sample_factor)
            rr = mean_recall(ids, off)
            log(f"ratio {r}: mean recall {rr:.4f}")
            curve.append((r, rr))
            if rr >= args.target_recall:
                ratio, rec = r, rr
                break
        if ratio is None:
            top = max(rr for _, rr in curve)
            ratio, rec = next((r, rr) for r, rr in curve if rr >= top - 0.005)
            log(f"recall {args.target_recall} not reachable with these nprobe (best {top:.4f}); r = {ratio} "
                f"(recall {rec:.4f})")
    qd = torch.from_numpy(q).to(dev)
    tot = int(k.sum())
    out = (torch.empty(tot, dtype=torch.int64, device=dev), torch.empty(tot, dtype=torch.float32, device=dev),
           torch.empty(nq, dtype=torch.int32, device=dev))

    def timed(fn, stage_timing=False):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        if stage_timing:  # the timed steps only
            bbc.stage_times(reset=True)
            bbc.stage_timing(True)
        ev = []
        t_s = time.perf_counter()
        for _ in range(args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            ev.append((e0, e1))
        torch.cuda.synchronize()
        el = time.perf_counter() - t_s
        if stage_timing:
            bbc.stage_timing(False)
        return el, np.array([a.elapsed_time(b) for a, b in ev])

    eager_s, eager_ms = timed(lambda: index.search(qd, k, npb, ratio=ratio, out=out, lut_u8=args.lut_u8, early_rerank=args.early_rerank, sample_factor=args.sample_factor), stage_timing=True)
    stages = bbc.stage_times(reset=True)
    t0 = time.time()
    plan = index.plan(qd, k, npb, out, ratio=ratio, autotune=True, lut_u8=args.lut_u8, early_rerank=args.early_rerank, sample_factor=args.sample_factor)
    plan_s = time.time() - t0
    info = plan.info()
    graph_s, graph_ms = timed(lambda: plan.execute())
    ids_g = out[0].cpu().numpy()
    ref = index.search(q, k, npb, ratio=ratio, buckets=info["buckets"], lut_u8=args.lut_u8,
                       early_rerank=args.early_rerank, sample_factor=info["sample_factor"])
    same = bool(np.array_equal(ids_g, ref[0]))
    value = nq * args.steps / graph_s
    sz = index.search_counts(q, k, npb, ratio=ratio, lut_u8=args.lut_u8, early_rerank=args.early_rerank, sample_factor=args.sample_factor)
    S, Kc, nsurv = int(sz["n_scanned"].sum()), int(sz["n_cand"].sum()), int(sz["n_survivors"].sum())
    nsk = int(sz["n_sample_keys"].sum())
    code_bytes = w.pq_m if w.pq_bits == 8 else (w.pq_m + 1) // 2
    algo = {"scan": (S - nsk) * code_bytes, "rerank": Kc * (4 * w.d + 4), "collect": nsurv * 8 + Kc * 4}
    names = {"scan": KERNEL_SCAN, "rerank": "rerank_half_kernel", "collect": "collect_bucket_kernel"}
    entries = {}
    for name in algo:
        st = stages[name]
        if st["launches"] == 0:
            continue
        avg_ms = st["ms"] / st["launches"]
        bpl = algo[name] * args.steps / st["launches"]
        gbs = bpl / (avg_ms * 1e-3) / 1e9
        if name == "rerank" and rerank_tile_form(w.d):
            entries[name] = rerank_entry(avg_ms, Kc * args.steps / st["launches"], w.d)
            continue
        if name == "scan":
            src = [os.path.join(CSRC, f) for f in ("pq_scan.hip", "common.h", "kernels.h")]
            entries[name] = scan_entry(names[name], avg_ms, bpl, bpl / code_bytes * w.pq_m * (1 if args.lut_u8 else 4),
                                       measured_traffic(w.name, name, src), w.n * code_bytes)
            continue
        entries[name] = {"kernel": names[name], "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                         "avg_launch_ms": round(avg_ms, 4), "algorithmic_bytes_per_launch": int(bpl)}
    dominant = max(entries, key=lambda s: stages[s]["ms"])
    cpu = None
    if not args.no_cpu:
        import oracle
        oix = dict(kind="pq", n=w.n, d=w.d, nlist=w.nlist, M=w.pq_m, ksub=1 << w.pq_bits, bits=w.pq_bits, metric=0,
                   centroids=index.get(bbc.FIELD_CENTROIDS), list_off=index.get(bbc.FIELD_LIST_OFF),
                   list_ids=index.get(bbc.FIELD_LIST_IDS), codes=index.get(bbc.FIELD_CODES),
                   codebook=index.get(bbc.FIELD_CODEBOOK), base=x)
        per_call = max(8, oracle.num_threads())
        nqc, t_cpu = oracle_sample(lambda lo, hi: oracle.search_pq(oix, q[lo:hi], k[lo:hi], npb[lo:hi], ratio, lut_u8=args.lut_u8),
                                   min(args.cpu_queries, nq), args.cpu_seconds, per_call)
        cpu = {"value": round(nqc / t_cpu, 2), "unit": "queries/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"first {nqc} queries of the batch (their own k and nprobe), same r, {per_call} per "
                         f"oracle call; oracle search over the index arrays of the GPU build (bit-identical to the "
                         f"oracle's own build); {t_cpu:.1f}s of CPU work"}
    res = {
        "metric": f"QPS at mean recall@k={args.target_recall}, k log-uniform in [100, 50000], nprobe uniform in "
                  f"[16, 256] (batched uneven form)",
        "value": round(value, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(graph_s / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "nlist": w.nlist, "pq": f"{w.pq_m}x{w.pq_bits}",
                   "nq": nq, "k_mean": float(k.mean()), "nprobe_mean": float(npb.mean()), "ratio": ratio,
                   "tables": "u8" if args.lut_u8 else "f32", "early_rerank": bool(args.early_rerank)},
        "recall": None if rec is None else round(rec, 4),
        "recall_target_reached": rec is not None and rec >= args.target_recall,
        "graph": {"qps": round(value, 1), "batch_ms_p50": round(float(np.percentile(graph_ms, 50)), 3),
                  "plan_create_s": round(plan_s, 2), "autotuned": info, "identical_to_eager": same},
        "eager": {"qps": round(nq * args.steps / eager_s, 1),
                  "batch_ms_p50": round(float(np.percentile(eager_ms, 50)), 3)},
        "stage_ms_per_step": {s: round(v["ms"] / max(1, args.steps), 4) for s, v in stages.items()},
        "sizes": {"S_mean": S / nq, "Kc_mean": Kc / nq, "survivors_mean": nsurv / nq, "sample_keys_mean": nsk / nq},
        "roofline": entries[dominant],
        "roofline_other_kernels": {n: e for n, e in entries.items() if n != dominant},
        "cpu_baseline": cpu,
        "build_s": round(build_s, 2),
    }
    print(json.dumps(res), flush=True)


def run_rabitq(args, w, np, torch, bbc, synth, dev):
    """RaBitQ workload: one batch of queries at one k per step, nprobe swept
    to the smallest value whose mean recall@k reaches the target."""
    nq = args.nq or w.nq
    k = int(w.k[0])
    metric = bbc.METRIC_IP if w.metric == "ip" else bbc.METRIC_L2
    t0 = time.time()
    x = synth.base_vectors(w)
    q = synth.query_vectors(w, nq)
    if metric == bbc.METRIC_IP:  # unit queries, normalised in float32
        q = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32)
    tr, ip = synth.kmeans_draws(w.n, w.nlist, w.train_per_list * w.nlist, 0)
    P = synth.rotation_orthogonal(w.d, w.seed_rotation)
    log(f"data {x.shape} {x.dtype} queries {q.shape} in {time.time() - t0:.1f}s")
    t0 = time.time()
    index = bbc.Index.build_rabitq(x, w.nlist, tr, ip, P, metric=metric, iters=w.kmeans_iters)
    build_s = time.time() - t0
    log(f"GPU index build {build_s:.1f}s")
    rq = q[: args.recall_queries]
    gt = None
    if len(rq):
        x64 = torch.from_numpy(x).to(dev).to(torch.float64)
        gt = ground_truth(torch, x64, rq, k, metric)
        del x64
        torch.cuda.empty_cache()
    elif not args.nprobe:
        raise SystemExit("--recall-queries 0 needs a fixed --nprobe")
    if args.nprobe:
        npb = int(args.nprobe.split(",")[0])
        rec = None
        if gt is not None:
            ids, _, _, off = index.search(rq, k, npb)
            rec = recall_at_k(ids, off, gt, k)
    else:
        npb, rec = None, None
        for cand in [32, 64, 96, 128, 192, 256, 384, 512, 768, 1024]:
            if cand > w.nlist:
                break
            ids, _, _, off = index.search(rq, k, cand)
            r = recall_at_k(ids, off, gt, k)
            log(f"nprobe {cand}: recall {r:.4f}")
            if r >= args.target_recall:
                npb, rec = cand, r
                break
        if npb is None:
            raise SystemExit(f"recall {args.target_recall} not reached")
    qd = torch.from_numpy(q).to(dev)
    out = (torch.empty(nq * k, dtype=torch.int64, device=dev), torch.empty(nq * k, dtype=torch.float32, device=dev),
           torch.empty(nq, dtype=torch.int32, device=dev))
    for _ in range(args.warmup):
        index.search(qd, k, npb, out=out)
    torch.cuda.synchronize()
    bbc.stage_times(reset=True)
    bbc.stage_timing(True)
    lat = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        index.search(qd, k, npb, out=out)
        e1.record()
        lat.append((e0, e1))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    bbc.stage_timing(False)
    stages = bbc.stage_times(reset=True)
    lat_ms = np.array([a.elapsed_time(b) for a, b in lat])
    value = nq * args.steps / elapsed
    sz = index.search_sizes(q, k, npb)
    S, nv = int(sz["n_scanned"].sum()), int(sz["n_visited"].sum())
    row_bytes = (2 if x.dtype == np.float16 else 4) * w.d
    algo = {"scan": S * (w.d // 8 + 16), "rerank": nv * (row_bytes + 4)}
    names = {"scan": "rabitq_scan_kernel (bounds of every scanned object)",
             "rerank": "rabitq_walk_kernel (bounded re-rank)"}
    # batches larger than the compute-unit count take the wide form with
    # tile-major exact keys (rows from LDS): priced by arithmetic instead
    tile_keys = nq > 256 and os.environ.get("BBC_WALK_FORM", "0") in ("0", "3")
    entries = {}
    for name in algo:
        st = stages[name]
        if st["launches"] == 0:
            continue
        avg_ms = st["ms"] / st["launches"]
        if name == "rerank" and tile_keys:
            e = rerank_entry(avg_ms, nv * args.steps / st["launches"], w.d)
            e["kernel"] = ("rt_rerank_tile_wide + rabitq_walk_kernel (exact keys of the candidate set C, "
                           "tile-major, then the walk over them)")
            entries[name] = e
            continue
        bpl = algo[name] * args.steps / st["launches"]
        gbs = bpl / (avg_ms * 1e-3) / 1e9
        entries[name] = {"kernel": names[name], "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                         "avg_launch_ms": round(avg_ms, 4), "algorithmic_bytes_per_launch": int(bpl)}
    dominant = max(entries, key=lambda s: stages[s]["ms"])
    cpu = None
    f4 = None
    oix = dict(kind="rabitq", n=w.n, d=w.d, nlist=w.nlist, metric=metric,
               centroids=index.get(bbc.FIELD_CENTROIDS), rot_centroids=index.get(bbc.FIELD_ROT_CENTROIDS),
               P=P, list_off=index.get(bbc.FIELD_LIST_OFF), list_ids=index.get(bbc.FIELD_LIST_IDS),
               codes=index.get(bbc.FIELD_RABITQ_CODES), factors=index.get(bbc.FIELD_RABITQ_FACTORS),
               base=x)
    if args.f4_queries > 0:
        nf = min(args.f4_queries, nq)
        f4 = rerank_report(oix, q[:nf], k, npb, sz["n_visited"][:nf])
        log(f"re-rank sizes {f4}")
    if not args.no_cpu:
        import oracle
        oix["base"] = np.ascontiguousarray(x, dtype=np.float32)
        per_call = max(8, oracle.num_threads())
        nqc, t_cpu = oracle_sample(lambda lo, hi: oracle.search_rabitq(oix, q[lo:hi], k, npb),
                                   min(args.cpu_queries, nq), args.cpu_seconds, per_call)
        cpu = {"value": round(nqc / t_cpu, 2), "unit": "queries/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"first {nqc} queries of the batch, same nprobe, {per_call} per oracle call; oracle "
                         f"search over the index arrays of the GPU build (bit-identical to the oracle's own build); "
                         f"{t_cpu:.1f}s of CPU work"}
    res = {
        "metric": f"QPS at recall@k={args.target_recall}, k={k}, RaBitQ with the bounded re-rank",
        "value": round(value, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "nlist": w.nlist, "quant": "rabitq",
                   "metric": w.metric, "storage": str(x.dtype), "nq": nq, "k": k, "nprobe": npb},
        "recall": None if rec is None else round(rec, 4),
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 3),
                       "p99": round(float(np.percentile(lat_ms, 99)), 3),
                       "what": f"device time of one {nq}-query batch"},
        "stage_ms_per_step": {s: round(v["ms"] / max(1, args.steps), 4) for s, v in stages.items()},
        "sizes": {"S_mean": S / nq, "reranked_mean": nv / nq},
        "rerank_vs_minimal": f4,
        "roofline": entries[dominant],
        "roofline_other_kernels": {n: e for n, e in entries.items() if n != dominant},
        "cpu_baseline": cpu,
        "build_s": round(build_s, 2),
    }
    print(json.dumps(res), flush=True)


def rerank_report(oix, qs, ks, npbs, gpu_exact):
    """Row f4: re-rank sizes on a sample of queries, against Observation 1's
    minimum (oracle.rerank_counts), beside the exact distances the GPU
    computed for the same queries."""
    import numpy as np
    import oracle
    c = oracle.rerank_counts(oix, qs, ks, npbs)
    mn = np.maximum(c["min"], 1)
    g = np.asarray(gpu_exact, np.float64)
    return {"queries": int(len(qs)), "S_mean": float(c["S"].mean()),
            "gpu_exact_mean": float(g.mean()), "walk_visited_mean": float(c["visited"].mean()),
            "C_mean": float(c["C"].mean()), "minimal_mean": float(c["min"].mean()),
            "minimal_with_topk_mean": float(c["min_out"].mean()),
            "gpu_over_minimal": float(np.mean(g / mn)), "walk_over_minimal": float(np.mean(c["visited"] / mn)),
            "what": "per query: S scanned; exact distances the GPU computed (all of C = {lb <= k-th ub} in the "
                    "wide form); the oracle's bounded walk; |C|; Observation 1's minimal set (bound interval holds "
                    "the k-th exact key) and that set with the exact top-k"}


def recall_each(ids, off, gt, ks):
    """recall@k_i of each request against its exact top-k_i."""
    out = []
    for i, k in enumerate(ks):
        k = int(k)
        got = ids[off[i]:off[i] + k]
        out.append(len(set(got.tolist()) & set(gt[i, :k].tolist())) / k)
    import numpy as np
    return np.array(out)


def run_serving(args, w, np, torch, bbc, synth, dev):
    """Serving form: single requests from the workload's seeded Poisson stream
    (k log-uniform over its range, each query drawn from a pool) through the
    continuous-batching server.  nprobe is set per k band (four log-spaced
    bands) to the smallest value whose mean recall@k on a sample of the
    stream's requests reaches the target.  Reports the served rate, per
    request latency (submission to completion), the closed-loop capacity,
    and the roofline of the dominant kernel over the open-loop phase."""
    import queue
    import threading
    assert w.quant == "rabitq", "the serving workload is a RaBitQ index"
    metric = bbc.METRIC_IP if w.metric == "ip" else bbc.METRIC_L2
    pool_n = args.nq or w.nq
    rate = args.serve_qps or w.arrival_qps
    seconds = w.serve_seconds if args.serve_seconds is None else args.serve_seconds
    t0 = time.time()
    x = synth.base_vectors(w)
    pool = synth.query_vectors(w, pool_n)
    if metric == bbc.METRIC_IP:  # unit queries, normalised in float32
        pool = (pool / np.linalg.norm(pool, axis=1, keepdims=True)).astype(np.float32)
    tr, ip = synth.kmeans_draws(w.n, w.nlist, w.train_per_list * w.nlist, 0)
    P = synth.rotation_orthogonal(w.d, w.seed_rotation)
    log(f"data {x.shape} {x.dtype} pool {pool.shape} in {time.time() - t0:.1f}s")
    t0 = time.time()
    index = bbc.Index.build_rabitq(x, w.nlist, tr, ip, P, metric=metric, iters=w.kmeans_iters)
    build_s = time.time() - t0
    log(f"GPU index build {build_s:.1f}s")

    # ---- operating point: nprobe per k band -----------------------------------
    kmin, kmax = w.k
    edges = np.geomspace(kmin, kmax + 1, 5)
    band_of = lambda kk: np.clip(np.searchsorted(edges, kk, side="right") - 1, 0, 3)
    grid = [8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048]
    grid = [g for g in grid if g <= w.nlist]
    fixed = [int(v) for v in args.nprobe.split(",")] if args.nprobe else []
    st_t, st_q, st_k = synth.request_stream(w, pool_n, rate, max(seconds, 1.0))
    R = min(args.recall_queries, len(st_t))
    band_np, band_rec = [0] * 4, [None] * 4
    if R > 0:
        sq, sk = pool[st_q[:R]], st_k[:R].astype(np.int32)
        x64 = torch.from_numpy(x).to(dev).to(torch.float64)
        gt = ground_truth(torch, x64, sq, int(sk.max()), metric)
        del x64
        torch.cuda.empty_cache()
        sb = band_of(sk)
        for b in range(4):
            m = np.nonzero(sb == b)[0]
            cands = [fixed[b]] if fixed else grid
            for npb in cands:
                if len(m) == 0:
                    band_np[b] = npb
                    break
                ids, _, _, off = index.search(sq[m], sk[m], npb)
                rec = float(recall_each(ids, off, gt[m], sk[m]).mean())
                log(f"band {b} ({len(m)} requests, k {int(edges[b])}-{int(edges[b + 1]) - 1}) nprobe {npb}: "
                    f"recall {rec:.4f}")
                band_np[b], band_rec[b] = npb, rec
                if rec >= args.target_recall:
                    break
        counts = np.bincount(sb, minlength=4)
        rec_all = float(sum(band_rec[b] * counts[b] for b in range(4) if band_rec[b] is not None) / max(1, R))
    elif len(fixed) == 4:
        band_np, rec_all = fixed, None
    else:
        raise SystemExit("--recall-queries 0 needs --nprobe with four values (one per k band)")
    log(f"nprobe per band {band_np}")

    t_arr, qi, ks = st_t, st_q, st_k.astype(np.int32)
    if seconds < 1.0:
        keep = t_arr < seconds
        t_arr, qi, ks = t_arr[keep], qi[keep], ks[keep]
    npr = np.array(band_np, np.int32)[band_of(ks)]
    n = len(t_arr)
    srv = index.server(mem_budget=args.serve_budget, max_slots=args.serve_slots, lanes=args.serve_lanes)

    def closed_loop(count):
        j = np.arange(count) % n
        t = time.perf_counter()
        tk = [srv.submit(pool[qi[i]], int(ks[i]), int(npr[i])) for i in j]
        for tt in tk:
            assert srv.wait(tt, 600000) is not None
        return time.perf_counter() - t

    closed_loop(min(args.serve_warmup, n))
    capacity = None
    if args.capacity_requests:
        el = closed_loop(args.capacity_requests)
        st = srv.stats()
        capacity = {"qps": round(args.capacity_requests / el, 1), "requests": args.capacity_requests,
                    "what": "all requests submitted at once, closed loop"}
        log(f"capacity {capacity['qps']} QPS")
    base_stats = srv.stats()

    # ---- open loop: Poisson arrivals ------------------------------------------
    q_tk = queue.Queue()
    t_sub = np.zeros(n)
    lag = np.zeros(n)

    def producer():
        # sleeps (never spins holding the interpreter lock) until each arrival
        base = time.perf_counter()
        q_tk.put(base)
        for i in range(n):
            target = base + t_arr[i]
            dt = target - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            t_sub[i] = time.perf_counter()
            q_tk.put(srv.submit(pool[qi[i]], int(ks[i]), int(npr[i])))
            lag[i] = t_sub[i] - target

    switch = sys.getswitchinterval()
    sys.setswitchinterval(1e-4)
    bbc.stage_times(reset=True)
    bbc.stage_timing(True)
    th = threading.Thread(target=producer)
    th.start()
    base = q_tk.get()
    infos = []
    for i in range(n):
        r = srv.wait(q_tk.get(), 600000)
        assert r is not None
        infos.append(r[2])
        if (i + 1) % 10000 == 0:
            log(f"served {i + 1}/{n}")
    th.join()
    sys.setswitchinterval(switch)
    bbc.stage_timing(False)
    stages = bbc.stage_times(reset=True)
    st = srv.stats()
    srv.free()
    srv_ms = np.array([f["latency_ns"] for f in infos]) / 1e6
    lat_ms = lag * 1e3 + srv_ms  # from the scheduled arrival
    done = t_sub + srv_ms / 1e3
    wall = float(done.max() - base)
    served = n / wall
    S = int(sum(f["n_scanned"] for f in infos))
    nv = int(sum(f["n_reranked"] for f in infos))
    bsz = np.array([f["batch_size"] for f in infos])
    row_bytes = (2 if x.dtype == np.float16 else 4) * w.d
    algo = {"scan": S * (w.d // 8 + 16), "rerank": nv * (row_bytes + 4)}
    names = {"scan": "rabitq_scan_kernel (bounds of every scanned object)",
             "rerank": "rabitq_exact_kernel + rabitq_walk_kernel (re-rank stage, wide form: exact keys of all "
                       "candidates, then the bounded walk)"}
    entries = {}
    for name in algo:
        sg = stages[name]
        if sg["launches"] == 0:
            continue
        avg_ms = sg["ms"] / sg["launches"]
        bpl = algo[name] / sg["launches"]
        gbs = bpl / (avg_ms * 1e-3) / 1e9
        entries[name] = {"kernel": names[name], "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                         "avg_launch_ms": round(avg_ms, 4), "algorithmic_bytes_per_launch": int(bpl),
                         "launches": sg["launches"]}
    dominant = max(entries, key=lambda s_: stages[s_]["ms"])

    cpu = None
    f4 = None
    if args.f4_queries > 0 or not args.no_cpu:
        oix = dict(kind="rabitq", n=w.n, d=w.d, nlist=w.nlist, metric=metric,
                   centroids=index.get(bbc.FIELD_CENTROIDS), rot_centroids=index.get(bbc.FIELD_ROT_CENTROIDS),
                   P=P, list_off=index.get(bbc.FIELD_LIST_OFF), list_ids=index.get(bbc.FIELD_LIST_IDS),
                   codes=index.get(bbc.FIELD_RABITQ_CODES), factors=index.get(bbc.FIELD_RABITQ_FACTORS),
                   base=np.ascontiguousarray(x, dtype=np.float32))
    if args.f4_queries > 0:
        nf = min(args.f4_queries, n)
        f4 = rerank_report(oix, pool[qi[:nf]], ks[:nf], npr[:nf], [f["n_reranked"] for f in infos[:nf]])
        log(f"re-rank sizes {f4}")
    if not args.no_cpu:
        import oracle
        per_call = max(8, oracle.num_threads())
        done_n, t_cpu = oracle_sample(
            lambda lo, hi: oracle.search_rabitq(oix, pool[qi[lo:hi]], ks[lo:hi], npr[lo:hi]), n, args.cpu_seconds,
            per_call)
        cpu = {"value": round(done_n / t_cpu, 2), "unit": "queries/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"the first {done_n} requests of the stream (their k and nprobe), {per_call} per oracle call, "
                         f"over the index arrays of the GPU build; {t_cpu:.1f}s of CPU work"}
    res = {
        "metric": f"served QPS at recall@k>={args.target_recall} under Poisson arrivals at {rate:g}/s, "
                  f"k log-uniform in [{kmin}, {kmax}]; p50/p99 latency",
        "value": round(served, 1), "unit": "queries/s", "n_gpus": 1, "steps": n,
        "warmup": min(args.serve_warmup, n), "ms_per_step": round(wall / n * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "nlist": w.nlist, "quant": "rabitq",
                   "metric": w.metric, "storage": str(x.dtype), "pool": pool_n, "arrival_qps": rate,
                   "seconds": seconds, "k_range": [kmin, kmax], "nprobe_by_k_band": band_np,
                   "k_band_edges": [int(e) for e in edges]},
        "recall": None if rec_all is None else round(rec_all, 4),
        "recall_by_band": [None if r is None else round(r, 4) for r in band_rec],
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 3),
                       "p90": round(float(np.percentile(lat_ms, 90)), 3),
                       "p99": round(float(np.percentile(lat_ms, 99)), 3),
                       "max": round(float(lat_ms.max()), 3), "mean": round(float(lat_ms.mean()), 3),
                       "what": "per request, scheduled arrival to completion (submission lag, queueing, "
                               "batch, query upload and result download included)"},
        "server_latency_ms": {"p50": round(float(np.percentile(srv_ms, 50)), 3),
                              "p99": round(float(np.percentile(srv_ms, 99)), 3),
                              "what": "submission to completion, as seen by the server"},
        "offered_qps": rate,
        "capacity": capacity,
        "submit_lag_ms": {"p99": round(float(np.percentile(lag, 99)) * 1e3, 3),
                          "max": round(float(lag.max()) * 1e3, 3)},
        "server": {"budget_bytes": args.serve_budget, "max_slots": args.serve_slots, "lanes": args.serve_lanes,
                   "batches": st["batches"] - base_stats["batches"], "mean_batch": round(float(bsz.mean()), 2),
                   "max_batch": int(bsz.max()), "max_inflight": st["max_inflight"]},
        "stage_ms_per_request": {s_: round(v["ms"] / n, 5) for s_, v in stages.items()},
        "sizes": {"S_mean": S / n, "reranked_mean": nv / n},
        "roofline": entries[dominant],
        "roofline_other_kernels": {k_: e for k_, e in entries.items() if k_ != dominant},
        "rerank_vs_minimal": f4,
        "cpu_baseline": cpu,
        "build_s": round(build_s, 2),
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
