"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host only): an instrumented build of oracle.c and oracle64.c runs a
small PQ and RaBitQ query path end to end (index build, search with its
debug outputs, collector, early re-rank, minimal re-rank, float64 shadow,
exact kNN) in a child process, which must finish with no sanitizer report
and with the same results as the plain build."""
import os
import subprocess
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

SCRIPT = r'''
import sys, numpy as np
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[2])
import oracle, synth
from helpers import oracle_pq_index
w, ix, q = oracle_pq_index("ivfpq_100k_d128", 3000, 8, 16, 8, 4, iters=3)
k = np.array([5, 40, 200, 3000], np.int64)
r = oracle.search_pq(ix, q, k, np.array([1, 3, 8, 8], np.int64), 1.5, debug=True)
r64 = oracle.search_pq64(ix, q, k, np.array([1, 3, 8, 8], np.int64), 1.5)
keys = np.sort(np.random.default_rng(1).random(5000).astype(np.float32))
ids = np.arange(5000, dtype=np.int64)
goff = np.array([0, 700, 2100, 5000], np.int64)
col = oracle.collect_bbc(keys, ids, goff, 900, 64, 1, 2)
er = oracle.early_rerank(keys, ids, goff, 900, 64, 1, 2)
d, n, nlist = 64, 1500, 4
wl = synth.small_workload("ivfrabitq_1m_d960", n=n, nlist=nlist, nq=3, d=d, seed_index=2)
x = synth.base_vectors(wl)
tr, ip = synth.kmeans_draws(n, nlist, 64 * nlist, 0)
rix = oracle.build_ivf_rabitq(x, nlist, tr, ip, synth.rotation_orthogonal(d, 302), iters=3)
rr = oracle.search_rabitq(rix, synth.query_vectors(wl), 30, 2, debug=True)
gt = oracle.exact_knn64(x, synth.query_vectors(wl), 10)
out = [r["ids"], r["dists"], r64["dists"], col["cand_ids"], np.array([er["tau_pred"]]), rr["ids"], rr["dists"],
       gt[0] if isinstance(gt, tuple) else gt]
np.savez(sys.argv[3], *out)
print("done")
'''


def _build(tmp_path, sanitize):
    import oracle
    so = str(tmp_path / ("liboracle_san.so" if sanitize else "liboracle_plain.so"))
    flags = list(oracle.CFLAGS)
    if sanitize:
        flags += ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    subprocess.check_call(["gcc", *flags, "-o", so, os.path.join(ROOT, "oracle", "oracle.c"),
                           os.path.join(ROOT, "oracle", "oracle64.c"), "-lm"])
    return so


def _run(tmp_path, so, preload, name):
    out = str(tmp_path / f"{name}.npz")
    env = dict(os.environ, ORACLE_LIB=so, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    if preload:
        env["LD_PRELOAD"] = preload
    p = subprocess.run([sys.executable, "-c", SCRIPT, ROOT, HERE, out], env=env, capture_output=True, text=True,
                       timeout=600)
    return p, out


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    san = _build(tmp_path, True)
    plain = _build(tmp_path, False)
    p, out_san = _run(tmp_path, san, asan, "san")
    report = p.stdout + p.stderr
    assert p.returncode == 0, report[-4000:]
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert "done" in p.stdout
    q, out_plain = _run(tmp_path, plain, None, "plain")
    assert q.returncode == 0, (q.stdout + q.stderr)[-2000:]
    a, b = np.load(out_san), np.load(out_plain)
    for key in a.files:
        np.testing.assert_array_equal(a[key], b[key], err_msg=key)
