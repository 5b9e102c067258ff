"""Oracle errors of the full-size batched workload on a 16 384-row sample.

TEST INFRASTRUCTURE (not collected by pytest; run by hand).  The FP64 oracle
forms every sampled row of A explicitly, O(n (d + b)) work per row, which at
n = 2^22, d = 128 takes about a second per row and thread: far too long for
a GPU run.  So the work is split in two:

  1. ``oracle``: compute the oracle's values on the sampled rows on the CPU and
     keep them in a cache directory, keyed by (workload, metric, seed, rows).
     Resumable: rows are done in chunks and each chunk is saved as it ends.
  2. ``errors``: read the GPU's results on the same rows (written by
     ``bench.py --dump-rows FILE``) and print the error figures of the three
     forms (batched l1, single-column l1, batched l2 squared) as text, for
     ``profiles/``.

The sample follows the subsample reading of the design notes: 16 384 rows
uniformly without replacement (seed_sub of the workload), plus the points at
rank 0 and rank n-1 of coordinates 0 and d-1 (the scan boundaries) and 16
rows of the longest run of tied values of coordinate 0.

Usage:
  python tests/full_sample.py oracle --metric l1 --cache DIR [--threads T]
  python tests/full_sample.py oracle --metric l2sq --cache DIR
  python tests/full_sample.py errors --gpu FILE.npz --cache DIR [--out FILE]
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

M_ROWS = 16384
N, D, B = 1 << 22, 128, 64


def workload():
    return synth.workload3(N, D, B)


def sample_rows(X):
    from oracle import sampling
    return sampling.workload3_rows(X, M_ROWS)


def rows_key(rows):
    return hashlib.sha256(np.ascontiguousarray(rows, dtype=np.int64).tobytes()).hexdigest()[:16]


def cache_file(cache, metric, rows):
    return os.path.join(cache, "w3_n%d_d%d_b%d_%s_seed%d_%s.npz" % (N, D, B, metric, synth.seeds(3)["sub"],
                                                                      rows_key(rows)))


def cmd_oracle(a):
    import oracle
    if a.threads:
        os.environ["OMP_NUM_THREADS"] = str(a.threads)
    oracle.build(force=False)
    met = {"l1": oracle.L1, "l2sq": oracle.L2SQ}[a.metric]
    X, Z = workload()
    rows, extra, tie_len = sample_rows(X)
    os.makedirs(a.cache, exist_ok=True)
    path = cache_file(a.cache, a.metric, rows)
    m = rows.size
    if os.path.exists(path):
        c = dict(np.load(path))
        done = int(c["done"])
        o, rn, ad = c["o"], c["rn"], c["ad"]
    else:
        done = 0
        o = np.zeros((m, B)); rn = np.zeros(m); ad = np.zeros((m, B))
    X64 = X.astype(np.float64)
    Z64 = Z.astype(np.float64)
    print("rows %d (tie run %d), done %d, threads %d" % (m, tie_len, done, oracle.num_threads()), flush=True)
    while done < m:
        hi = min(m, done + a.chunk)
        t0 = time.perf_counter()
        o[done:hi], rn[done:hi], ad[done:hi] = oracle.matvec(X64, Z64, met, rows[done:hi])
        done = hi
        np.savez(path + ".tmp.npz", rows=rows, o=o, rn=rn, ad=ad, done=done)
        os.replace(path + ".tmp.npz", path)
        print("%s: %d / %d rows (%.1f s per chunk)" % (a.metric, done, m, time.perf_counter() - t0), flush=True)


SRCS = ("l1_pass.h", "l1_common.h", "k_l1.hip", "k_prep.hip", "k_sort.hip", "k_l2_mfma.hip", "k_l2.hip")


def sources_hash():
    """The kernel code the sampled results come from (comments ignored; the
    benchmark reports these figures only while the code is unchanged)."""
    from paper_2210_15114_amd.build import code_hash
    return code_hash([os.path.join(ROOT, "paper_2210_15114_amd", "csrc", f) for f in SRCS])


def fmt(e):
    return "spec %.3e  per_row %.3e  componentwise %.3e  max_abs %.3e" % (
        e["spec"], e["per_row"], e["componentwise"], e["max_abs"])


def cmd_errors(a):
    from oracle import metrics
    X, Z = workload()
    rows, extra, tie_len = sample_rows(X)
    g = np.load(a.gpu)
    if not np.array_equal(g["rows"], rows):
        raise SystemExit("the GPU file holds other rows than this sample")
    Z64 = Z.astype(np.float64)
    lines = ["# Errors against the FP64 oracle on %d sampled rows of the batched workload" % rows.size,
             "# (n = %d, d = %d, U[0,1) FP32 points; Z n x %d N(0,1) FP32; seeds X %d, Z %d, sample %d)"
             % (N, D, B, synth.seeds(3)["X"], synth.seeds(3)["Z"], synth.seeds(3)["sub"]),
             "# rows: %d uniform without replacement + %d boundary/tie rows (longest tie run of coordinate 0: %d)"
             % (M_ROWS, len(set(extra)), tie_len),
             "# GPU rows: %s" % os.path.basename(a.gpu),
             "# sources_sha256_16: %s" % sources_hash(),
             "# GPU rows written by: python bench.py --dump-rows %s" % os.path.basename(a.gpu),
             "# oracle rows computed by: python tests/full_sample.py oracle --metric l1 --cache <dir>"
             " (and --metric l2sq), on the host",
             "# command: python tests/full_sample.py errors --gpu %s --cache <dir>" % os.path.basename(a.gpu)]
    for metric, keys in (("l1", ("l1", "single")), ("l2sq", ("l2sq",))):
        path = cache_file(a.cache, metric, rows)
        if not os.path.exists(path):
            lines.append("%s: oracle cache missing" % metric)
            continue
        c = np.load(path)
        if int(c["done"]) < rows.size:
            lines.append("%s: oracle cache incomplete (%d rows)" % (metric, int(c["done"])))
            continue
        o, rn, ad = c["o"], c["rn"], c["ad"]
        if metric == "l2sq":
            frob = metrics.frob_l2sq(X)
        else:
            frob = metrics.frob_from_rows(rn, N)
        for k in keys:
            if k not in g.files:
                continue
            e = metrics.errors(g[k], o, rn, ad, Z64, frob)
            lines.append("%-7s %s" % (k + ":", fmt(e)))
    text = "\n".join(lines) + "\n"
    sys.stdout.write(text)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)


def main():
    p = argparse.ArgumentParser()
    sub = p.add_subparsers(dest="cmd", required=True)
    po = sub.add_parser("oracle")
    po.add_argument("--metric", choices=("l1", "l2sq"), required=True)
    po.add_argument("--cache", required=True)
    po.add_argument("--threads", type=int, default=0)
    po.add_argument("--chunk", type=int, default=256)
    pe = sub.add_parser("errors")
    pe.add_argument("--gpu", required=True)
    pe.add_argument("--cache", required=True)
    pe.add_argument("--out", default="")
    pr = sub.add_parser("rows")
    a = p.parse_args()
    if a.cmd == "oracle":
        cmd_oracle(a)
    elif a.cmd == "errors":
        cmd_errors(a)
    else:
        X, _ = workload()
        rows, extra, tie_len = sample_rows(X)
        print(rows.size, rows_key(rows), extra, tie_len)


if __name__ == "__main__":
    main()
