#!/usr/bin/env python3
"""Benchmark of the l1 distance-matrix matvec on one MI355X.

Workload: n = 2^22 points, d = 128 coordinates uniform on [0, 1) in FP32,
Z = n x 64 right-hand sides N(0, 1) in FP32 (seeded, synthetic).

* value: batched columns/s = 64 / (time of one b = 64 query), the query being
  the totals kernel plus one chained-scan pass per coordinate (Algorithm 2);
  the per-coordinate sort (Algorithm 1) is one-time preparation, timed once
  and reported as prep_ms.
* single-vector form: 64 sequential b = 1 queries on the 64 columns.
* l2 squared: one b = 64 query of the low-rank form (Algorithm 3), with its
  own roofline: algorithmic bytes of the query, 8nd + 8nb + 16n, over the
  query's time, and the counter traffic of its kernels when the committed
  counter runs match the kernel source.
* tuned_variants: the pass tile variant the library's tuner chose for b = 64
  and b = 1 on this data, with the timed pass of every variant.
* multi: 512 datasets of uneven n and d (float and integer), b = 8, one
  captured-graph launch per query, with oracle spot checks.
* lowrank: rank-32 block-Krylov approximation at n = 2^21, d = 32 (block 40,
  8 iterations, 9 queries).
* approx_l2: approximate Euclidean products through the l1 path on Gaussian
  embeddings of the mixture points (k = 256): timings and the sampled error.
* single_vector_mixture: the plain single-vector method at n = 2^20, d = 64
  (32-component Gaussian mixture): 100 timed queries, median / p10 / p90, for
  l1 and l2 squared, with errors against the oracle.
* precision_stress: points 10^4 + U[0,1) (n = 2^20, d = 16) with z ~ N(0,1)
  and z = 1 + 10^-3 N(0,1): l1, p = 3 and l2 squared errors against the oracle
  on sampled and scan-boundary rows.
* roofline: algorithmic bytes of one coordinate pass, 12 n b + 8 n (perm and
  sorted values read once, the Z rows gathered once, the Out rows read and
  written once), over the pass kernel's mean device time from HIP events on
  the query stream, against the 8 TB/s HBM peak; beside it the rates of a
  plain copy and of the pass's random row accesses alone (dm_gather_probe).
* cpu_baseline: the FP64 CPU oracle (explicit rows of A, O(n^2 d)) on a
  bounded sample of rows of the same workload, extrapolated to whole columns.

Prints exactly one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "l1_pass_n4194304_d128_b64_traffic.txt")
PASS_SRCS = [os.path.join(ROOT, "paper_2210_15114_amd", "csrc", f) for f in ("l1_pass.h", "l1_common.h")]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def src_hash(paths):
    """Hash of the kernel code (comments and whitespace runs ignored) that the
    stored counter and error figures were taken with."""
    from paper_2210_15114_amd.build import code_hash
    return code_hash(paths)


def read_traffic(variant):
    """HBM bytes per pass from committed counter runs, if they still describe
    the kernel (same sources, same tile variant)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256_16") != src_hash(PASS_SRCS) or kv.get("variant") != str(variant):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


L2_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "l2sq_n4194304_d128_b64_traffic.txt")
L2_SRCS = [os.path.join(ROOT, "paper_2210_15114_amd", "csrc", "k_l2_mfma.hip")]


def read_l2_traffic():
    """HBM bytes per l2-squared query (all its kernels) from the committed
    counter runs, if the kernel source is unchanged since."""
    if not os.path.exists(L2_TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(L2_TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256_16") != src_hash(L2_SRCS):
        return None
    try:
        return float(kv["traffic_bytes_per_query"])
    except (KeyError, ValueError):
        return None


SAMPLE_FILE = os.path.join(ROOT, "profiles", "errors_n4194304_d128_b64_16k_rows.txt")
SAMPLE_SRCS = [os.path.join(ROOT, "paper_2210_15114_amd", "csrc", f) for f in
               ("l1_pass.h", "l1_common.h", "k_l1.hip", "k_prep.hip", "k_sort.hip", "k_l2_mfma.hip", "k_l2.hip")]


def read_sample_errors():
    """Error figures on the 16 384-row sample from the committed offline oracle
    comparison, if they were taken with these kernel sources."""
    if not os.path.exists(SAMPLE_FILE):
        return None
    out, kv = {}, {}
    for line in open(SAMPLE_FILE):
        if line.startswith("# sources_sha256_16:"):
            kv["sha"] = line.split(":", 1)[1].strip()
        elif ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            f = v.split()
            try:
                out[k.strip()] = {f[i]: float(f[i + 1]) for i in range(0, len(f) - 1, 2)}
            except ValueError:
                pass
    if kv.get("sha") != src_hash(SAMPLE_SRCS):
        return None
    return out


def run_lowrank(args, dm, synth, np, torch, dev):
    """Rank-32 block-Krylov approximation of the l1 matrix at n = 2^21, d = 32
    (50-component Gaussian mixture), block 40, 8 iterations: wall time of one
    call (after one warm-up call), orthonormality of U, and the residual of
    the top Ritz pair through one more query."""
    n, d, k, block, iters = 1 << 21, 32, 32, 40, 8
    X = synth.workload5(n, d)
    om = synth.rhs_normal(n, block, synth.seeds(5)["Z"], np.float64)
    Xd = torch.from_numpy(X).to(dev)
    omd = torch.from_numpy(om).to(dev)
    h = dm.prepare(Xd, dm.L1)
    v, _ = h.tune(block, reps=3)
    h.lowrank(k, omd, iters)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U, lam, sweeps = h.lowrank(k, omd, iters)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    # orthonormality of U on the host (outside the timed call)
    Uh = U.cpu()
    orth = float((Uh.t() @ Uh - torch.eye(k, dtype=torch.float64)).abs().max())
    del Uh
    u1 = U[:, 0].float().contiguous()
    y1 = h.matvec(u1)
    h.sync()
    l1 = float(lam[0])
    resid = float(torch.linalg.vector_norm(y1.double() - l1 * u1.double()) / abs(l1))
    h.free()
    log("lowrank: %.1f ms (n=%d, rank %d, block %d, %d iterations), sweeps %d, orth %.2e, top residual %.2e" %
        (ms, n, k, block, iters, sweeps, orth, resid))
    return {"n": n, "d": d, "rank": k, "block": block, "iters": iters, "ms": round(ms, 1), "queries": iters + 1,
            "jacobi_sweeps": sweeps, "orthonormality": orth, "top_ritz_residual": resid, "lam_top": l1,
            "pass_variant": v}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def pct(sorted_vals, q):
    """The q-quantile of sorted values (nearest rank)."""
    i = min(len(sorted_vals) - 1, max(0, int(round(q * (len(sorted_vals) - 1)))))
    return sorted_vals[i]


def run_single_mixture(args, dm, synth, np, torch, dev, stream):
    """The plain single-vector method on the mixture workload: n = 2^20,
    d = 64, 32 Gaussians; 100 distinct z on the device; preparation timed
    once; 10 warm-up and 100 timed single-vector queries (median, p10, p90)
    for l1 and l2 squared; errors against the oracle on sampled rows."""
    import oracle
    from oracle import metrics
    n, d, nq = 1 << 20, 64, 100
    X, Z = synth.workload2(n, d, nq)
    Xd = torch.from_numpy(X).to(dev)
    Zc = torch.from_numpy(np.ascontiguousarray(Z.T)).to(dev)      # nq x n: row q is query q
    res = {"n": n, "d": d, "queries": nq}
    rows = synth.subsample_rows(n, 8, synth.seeds(2)["sub"])
    for name, metric in (("l1", dm.L1), ("l2sq", dm.L2SQ)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = dm.prepare(Xd, metric)
        prep_ms = (time.perf_counter() - t0) * 1e3
        if metric == dm.L1:
            h.tune(1, reps=4)
        out = torch.empty(n, dtype=torch.float32, device=dev)
        for i in range(10):
            h.matvec(Zc[i % nq], out=out)
        h.sync()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * nq)]
        for q in range(nq):
            evs[2 * q].record(stream)
            h.matvec(Zc[q], out=out)
            evs[2 * q + 1].record(stream)
        torch.cuda.synchronize()
        h.sync()
        t = sorted(evs[2 * q].elapsed_time(evs[2 * q + 1]) for q in range(nq))
        y = out.cpu().numpy().astype(np.float64)      # the result of the last query
        z = Z[:, nq - 1].astype(np.float64)[:, None]
        o, rn, ad = oracle.matvec(X.astype(np.float64), z, oracle.L1 if metric == dm.L1 else oracle.L2SQ, rows)
        frob = metrics.frob_from_rows(rn, n) if metric == dm.L1 else metrics.frob_l2sq(X.astype(np.float64))
        err = metrics.errors(y[rows][:, None], o, rn, ad, z, frob)
        res[name] = {"prep_ms": round(prep_ms, 1), "median_ms": round(pct(t, 0.5), 4), "p10_ms": round(pct(t, 0.1), 4),
                     "p90_ms": round(pct(t, 0.9), 4), "columns_per_s": round(1e3 / pct(t, 0.5), 1),
                     "error_spec": err["spec"], "error_per_row": err["per_row"],
                     "form": ("sorted passes, one per coordinate (Algorithm 2)" if metric == dm.L1 else
                              "plain FP64 single-vector form of Algorithm 3 (b < 16 takes no matrix cores)")}
        log("mixture single-vector %s: median %.3f ms (p10 %.3f, p90 %.3f), prep %.1f ms, error %.2e" %
            (name, pct(t, 0.5), pct(t, 0.1), pct(t, 0.9), prep_ms, err["spec"]))
        h.free()
    return res


def run_precision_stress(args, dm, synth, np, torch, dev, stream):
    """Points far from the origin: n = 2^20, d = 16, X = 10^4 + U[0,1) FP32,
    and right-hand sides N(0, 1) or the Perron-like 1 + 10^-3 N(0, 1); one
    query each of l1 (b = 64 and b = 1), odd p = 3 and l2 squared (b = 64),
    errors against the FP64 oracle on 48 sampled rows plus the scan
    boundaries (ranks 0 and n - 1 of the first and last coordinate)."""
    import oracle
    from oracle import metrics
    n, d = 1 << 20, 16
    X = (1.0e4 + synth.rng(4242).random((n, d))).astype(np.float32)
    X64 = X.astype(np.float64)
    extra = []
    for k in (0, d - 1):
        o = np.argsort(X[:, k], kind="stable")
        extra += [int(o[0]), int(o[-1])]
    rows = synth.subsample_rows(n, 48, 4243, extra=extra)
    Xd = torch.from_numpy(X).to(dev)
    res = {"workload": "n=2^20, d=16, X = 1e4 + U[0,1) FP32", "rows": int(rows.size)}
    cases = (("l1", dm.L1, oracle.L1, (("positive", 64), ("normal", 64), ("positive", 1))),
             ("l3", dm.L3, oracle.L3, (("positive", 64),)),
             ("l2sq", dm.L2SQ, oracle.L2SQ, (("positive", 64), ("normal", 64))))
    for name, metric, ometric, zs in cases:
        h = dm.prepare(Xd, metric)
        for zk, b in zs:
            Z = synth.rhs_positive(n, b, 4244 + b) if zk == "positive" else synth.rhs_normal(n, b, 4245 + b)
            Zd = torch.from_numpy(Z if b > 1 else Z[:, 0].copy()).to(dev)
            y = h.matvec(Zd)
            h.sync()
            Y = y.cpu().numpy().astype(np.float64).reshape(n, b)
            Z64 = Z.astype(np.float64)
            o, rn, ad = oracle.matvec(X64, Z64, ometric, rows)
            frob = metrics.frob_l2sq(X64) if name == "l2sq" else metrics.frob_from_rows(rn, n)
            e = metrics.errors(Y[rows], o, rn, ad, Z64, frob)
            key = "%s_b%d_z_%s" % (name, b, zk)
            res[key] = {"spec": e["spec"], "per_row": e["per_row"]}
            log("precision stress %s: spec %.2e per-row %.2e" % (key, e["spec"], e["per_row"]))
        h.free()
    return res


def run_approx_l2(args, dm, synth, np, torch, dev, stream):
    """Approximate l2 products at n = 2^20, d = 64 (32-component mixture), k =
    256 embedding rows: embedding, preparation of the embedded points, one
    b = 64 query, and the relative Frobenius error of B against the exact
    Euclidean matrix estimated from sampled rows."""
    import oracle
    from oracle import approx_l2
    n, d, k, b = 1 << 20, 64, 256, 64
    X, _ = synth.workload2(n, d, 1)
    g = synth.rng(synth.seeds(2)["Z"] + 7)
    G = g.standard_normal((k, d))
    Z = synth.rhs_normal(n, b, synth.seeds(2)["Z"] + 8, np.float32)
    Xd, Gd, Zd = torch.from_numpy(X).to(dev), torch.from_numpy(G).to(dev), torch.from_numpy(Z).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Xe = dm.embed_l2(Xd, Gd)
    torch.cuda.synchronize()
    t_embed = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    h = dm.prepare(Xe, dm.L1)
    t_prep = (time.perf_counter() - t0) * 1e3
    h.tune(b, reps=3)
    out = torch.empty((n, b), dtype=torch.float32, device=dev)
    h.matvec(Zd, out=out)
    h.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    reps = 3
    for _ in range(reps):
        h.matvec(Zd, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    h.sync()
    ms = e0.elapsed_time(e1) / reps
    h.free()
    rows = synth.subsample_rows(n, 8, synth.seeds(2)["sub"] + 1)
    A = approx_l2.explicit_l2(X, rows)
    B = oracle.explicit(Xe.cpu().numpy(), oracle.L1, rows)
    rel = float(np.linalg.norm(A - B) / np.linalg.norm(A))
    log("approx l2: embed %.1f ms, prep %.1f ms, b=%d query %.2f ms, relative error %.4f (expected spread %.4f)" %
        (t_embed, t_prep, b, ms, rel, np.sqrt(np.pi / 2 - 1) / np.sqrt(k)))
    return {"n": n, "d": d, "k": k, "b": b, "embed_ms": round(t_embed, 2), "prep_ms": round(t_prep, 1),
            "ms_per_query": round(ms, 3), "columns_per_s": round(b / (ms * 1e-3), 1),
            "relative_frobenius_sampled_rows": rel, "expected_spread": float(np.sqrt(np.pi / 2 - 1) / np.sqrt(k))}


def run_sortfree(args, dm, synth, np, torch, dev, stream):
    """The sort-free family (Appendix A) on n = 2^20 points, d = 64: l_4^4 and
    l_6^6 on the 32-component mixture, KL divergence and cross entropy on
    Dirichlet(1) probability vectors, the squared Mahalanobis distance and the
    bilinear form with a seeded SPD matrix.  Single vector (b = 1) and blocks
    of b = 16 and b = 64; 3 warm-up and 10 timed queries each (median).  Reported per
    query: time, the algorithmic HBM bytes (moments read X, or its FP64
    logarithms for KL and cross entropy, plus Z; the point pass reads X and
    writes Out; the totals read Z) and their rate, and the FP64 operation
    rate; errors against the oracle on 4 sampled rows for l_4^4 and KL."""
    import oracle
    from oracle import metrics
    n, d = 1 << 20, 64
    Xm, _ = synth.workload2(n, d, 1)
    P = synth.simplex_points(n, d, synth.seeds(2)["X"] + 11)
    M = synth.square_matrix(d, synth.seeds(2)["X"] + 12, "spd")
    rows = synth.subsample_rows(n, 4, synth.seeds(2)["sub"] + 3)
    cases = (("l4", dm.L4, Xm, None, 4), ("l6", dm.L6, Xm, None, 6), ("kl", dm.KL, P, None, 1),
             ("ce", dm.CE, P, None, 1), ("maha2", dm.MAHA2, Xm, M, 1), ("bilinear", dm.BILINEAR, Xm, M, 1))
    res = {"n": n, "d": d}
    for b in (1, 16, 64):
        Z = synth.rhs_normal(n, b, synth.seeds(2)["Z"] + 20 + b, np.float32)
        Zd = torch.from_numpy(Z).to(dev)
        out = torch.empty((n, b), dtype=torch.float32, device=dev)
        for name, metric, X, Mm, nt in cases:
            Xd = torch.from_numpy(X).to(dev)
            h = dm.prepare(Xd, metric, M=Mm)
            for _ in range(3):
                h.matvec(Zd, out=out)
            h.sync()
            evs = [torch.cuda.Event(enable_timing=True) for _ in range(20)]
            for q in range(10):
                evs[2 * q].record(stream)
                h.matvec(Zd, out=out)
                evs[2 * q + 1].record(stream)
            torch.cuda.synchronize()
            h.sync()
            ms = pct(sorted(evs[2 * q].elapsed_time(evs[2 * q + 1]) for q in range(10)), 0.5)
            xb = n * d * (8 if metric in (dm.KL, dm.CE) else 4)
            nbytes = xb + n * d * 4 + 3 * n * b * 4
            # FP64 operations per (point, coordinate, column): even p takes NT
            # FMAs and NT - 1 products for the moments and a Horner step of NT
            # FMAs plus an add per point; the linear forms one FMA in each stage
            flops = float(n) * d * b * (5 * nt if nt > 1 else 4)
            ent = {"ms": round(ms, 4), "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1),
                   "fp64_TFLOPs": round(flops / (ms * 1e-3) / 1e12, 2)}
            if name in ("l4", "kl") and b == 1:
                y = out.cpu().numpy().astype(np.float64)
                o, rn, ad = oracle.matvec(X.astype(np.float64), Z.astype(np.float64),
                                          oracle.L4 if name == "l4" else oracle.KL, rows)
                ent["error_spec"] = metrics.errors(y[rows], o, rn, ad, Z.astype(np.float64),
                                                   metrics.frob_from_rows(rn, n))["spec"]
            res["%s_b%d" % (name, b)] = ent
            log("sort-free %s b=%d: %.3f ms/query, %.0f GB/s, %.2f FP64 TFLOP/s" %
                (name, b, ms, ent["GBps"], ent["fp64_TFLOPs"]))
            h.free()
            del Xd
        del Zd, out
    return res


def run_oddp_tv(args, dm, torch, dev, stream, Xd, Zd):
    """Odd p (l_3^3 and l_5^5, the p+1 chained prefix sums of each coordinate
    pass) and total variation (the l1 query halved) on the batched workload's
    points and right-hand sides.  Per metric: preparation once, one warm-up
    and 3 timed queries (mean), then one query with the library's events
    around every coordinate pass for its average device time.  The pass of
    odd p moves the bytes of the l1 pass (perm and sorted values, Z rows read,
    Out rows read and written: 12nb + 8n - 4nb/d per pass averaged over the d
    passes), so its rate is given against the same HBM peak."""
    n, d = Xd.shape
    b = Zd.shape[1]
    Out = torch.empty((n, b), dtype=torch.float32, device=dev)
    bytes_pass = 12.0 * n * b + 8.0 * n - 4.0 * n * b / d
    res = {"n": n, "d": d, "b": b, "bytes_per_pass": bytes_pass}
    for name, metric in (("l3", dm.L3), ("l5", dm.L5), ("tv", dm.TV)):
        h = dm.prepare(Xd, metric)
        h.reserve(b)
        h.matvec(Zd, out=Out)
        h.sync()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3
        e0.record(stream)
        for _ in range(reps):
            h.matvec(Zd, out=Out)
        e1.record(stream)
        torch.cuda.synchronize()
        h.sync()
        ms = e0.elapsed_time(e1) / reps
        h.profile(True)
        h.matvec(Zd, out=Out)
        h.sync()
        pass_ms, pass_n = h.profile_read(dm.K_L1_PASS)
        h.profile(False)
        h.free()
        avg = pass_ms / max(pass_n, 1)
        ach = bytes_pass / (avg * 1e-3) / 1e9
        res[name] = {"ms_per_query": round(ms, 3), "columns_per_s": round(b / (ms * 1e-3), 1),
                     "avg_pass_ms": round(avg, 4), "pass_GBps": round(ach, 1),
                     "pass_frac_of_hbm_peak": round(ach / HBM_PEAK_GBPS, 4)}
        log("%s: %.2f ms/query, pass %.4f ms (%.0f GB/s)" % (name, ms, avg, ach))
    del Out
    return res


def pass_kernel_name(variant, b):
    """Kernel of a float l1 pass variant: 0/1 the keep kernel, 2/3 the
    re-gathering kernel; odd variants halve the ranks per slot."""
    bp = 1
    while bp < b:
        bp *= 2
    r = 16 if (bp >= 32 or bp < 4) else 8
    if variant & 1:
        r //= 2
    fam = "l1_pass_keep_kernel" if variant < 2 else "l1_pass_kernel"
    return "%s<FloatPath,%d,R=%d>" % (fam, bp, r)


def run_multi(args, dm, synth, np, torch, dev, stream):
    """512 datasets of uneven n and d (float and integer), b = 8, one graph launch per query."""
    import oracle
    b = 8
    specs = synth.workload4_specs(args.multi_count)
    log("multi: generating %d datasets" % len(specs))
    Xs, Zs = [], []
    for sp in specs:
        X, Z = synth.workload4_dataset(sp, b)
        Xs.append(X)
        Zs.append(Z)
    Xd = [torch.from_numpy(X).to(dev) for X in Xs]
    Zd = [torch.from_numpy(Z).to(dev) for Z in Zs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = dm.prepare_multi(Xd)
    prep_ms = (time.perf_counter() - t0) * 1e3
    # tile variant of the coordinate-round launches, chosen by the library's
    # tuner on these datasets (the winner's plan stays captured)
    tv, tms, outs = h.tune(Zd, reps=3)
    log("multi: tuned variant %d, ms per query %s" % (tv, ["%.2f" % t for t in tms]))
    for _ in range(max(1, args.warmup)):
        outs = h.matvec(Zd, outs)
    h.sync()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        h.matvec(Zd, outs)
    e1.record(stream)
    torch.cuda.synchronize()
    h.sync()
    ms = e0.elapsed_time(e1) / args.steps
    pc = sum(sp.n * sp.d for sp in specs)
    model = sum(sp.n * sp.d * (168 if sp.is_int else 104) for sp in specs)
    # spot check: integer datasets bit-exact, float ones within the normalised bound, 16 rows each
    checked, worst = 0, 0.0
    g = synth.rng(4242)
    for i in list(range(len(specs)))[:: max(1, len(specs) // 8)]:
        rows = np.sort(g.choice(specs[i].n, size=min(16, specs[i].n), replace=False))
        Y = outs[i].cpu().numpy()[rows]
        if specs[i].is_int:
            o, ov = oracle.matvec_int(Xs[i], Zs[i], oracle.L1, rows)
            assert ov == 0 and np.array_equal(Y, o), "multi-dataset integer result differs from the oracle"
        else:
            o, rn, ad = oracle.matvec(Xs[i].astype(np.float64), Zs[i].astype(np.float64), oracle.L1, rows)
            worst = max(worst, float((np.abs(Y - o) / ad).max()))
        checked += 1
    log("multi: %d datasets, %.3f ms/query, prep %.0f ms" % (len(specs), ms, prep_ms))
    res = {"datasets": len(specs), "b": b, "ms_per_query": round(ms, 3), "prep_ms": round(prep_ms, 1),
           "point_coords": pc, "point_coord_columns_per_s": pc * b / (ms * 1e-3),
           "model_GBps_effective": round(model / (ms * 1e-3) / 1e9, 1),
           "spot_checked_datasets": checked, "float_componentwise_max": worst,
           "tuned_variant": tv, "ms_per_query_by_variant": [round(t, 3) for t in tms]}
    h.free()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 22)
    ap.add_argument("--d", type=int, default=128)
    ap.add_argument("--b", type=int, default=64)
    ap.add_argument("--cpu-rows", type=int, default=96, help="oracle sample size for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-single", action="store_true", help="skip the single-vector leg")
    ap.add_argument("--no-l2", action="store_true", help="skip the l2-squared leg")
    ap.add_argument("--no-multi", action="store_true", help="skip the multi-dataset leg")
    ap.add_argument("--no-lowrank", action="store_true", help="skip the block-Krylov low-rank leg")
    ap.add_argument("--no-mixture", action="store_true", help="skip the single-vector mixture leg")
    ap.add_argument("--no-approx-l2", action="store_true", help="skip the approximate l2 leg")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision-stress leg")
    ap.add_argument("--no-sortfree", action="store_true", help="skip the sort-free family leg")
    ap.add_argument("--no-oddp", action="store_true", help="skip the odd-p and total-variation leg")
    ap.add_argument("--multi-count", type=int, default=512)
    ap.add_argument("--dump-rows", default="", help="write the results on the 16 384-row sample to this .npz")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the method is measured on one GPU's share "
              "(multi-GPU sharding is described in the design notes, not run)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2210_15114_amd as dm
    import synth

    n, d, b = args.n, args.d, args.b
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    log("generating inputs n=%d d=%d b=%d" % (n, d, b))
    X, Z = synth.workload3(n, d, b)
    Xd = torch.from_numpy(X).to(dev)
    Zd = torch.from_numpy(Z).to(dev)
    torch.cuda.synchronize()

    # ---- achievable HBM bandwidth (plain copy of X) ----
    buf = torch.empty_like(Xd)
    for _ in range(2):
        dm.copy_probe(buf, Xd)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 5
    for _ in range(reps):
        dm.copy_probe(buf, Xd)
    e1.record()
    torch.cuda.synchronize()
    copy_gbps = 2.0 * Xd.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del buf
    log("copy probe %.0f GB/s" % copy_gbps)

    # ---- achievable rate of the pass's random row accesses: Out[p] += Z[p]
    # over a random permutation p (the gather and read-modify-write of one
    # pass without its scan), 4n + 12nb bytes per probe ----
    gather_gbps = None
    if b in (4, 8, 16, 32, 64):
        gen = torch.Generator(device=dev)
        gen.manual_seed(2210)
        permd = torch.randperm(n, device=dev, generator=gen).to(torch.int32)
        Ob = torch.zeros_like(Zd)
        for _ in range(2):
            dm.gather_probe(permd, Zd, Ob)
        e0.record()
        for _ in range(reps):
            dm.gather_probe(permd, Zd, Ob)
        e1.record()
        torch.cuda.synchronize()
        gather_gbps = (4.0 * n + 12.0 * n * b) * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del permd, Ob
        log("random-row probe %.0f GB/s" % gather_gbps)

    # ---- preparation (Algorithm 1), timed once ----
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = dm.prepare(Xd, dm.L1)
    prep_ms = (time.perf_counter() - t0) * 1e3
    log("prep %.1f ms" % prep_ms)
    # tile variant of the pass, chosen by the library's tuner on this data
    tuned = {}
    vb, tms = h.tune(b, reps=4)
    tuned["b%d" % b] = {"variant": vb, "ms_per_pass": [round(t, 4) for t in tms]}
    log("tuned b=%d: variant %d, ms per pass %s" % (b, vb, ["%.3f" % t for t in tms]))
    h.reserve(b)
    Out = torch.empty((n, b), dtype=torch.float32, device=dev)

    # ---- batched queries ----
    for _ in range(args.warmup):
        h.matvec(Zd, out=Out)
    h.sync()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(args.steps):
        h.matvec(Zd, out=Out)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    h.sync()
    ms_step = evs[0].elapsed_time(evs[-1]) / args.steps
    step_ms = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps))
    median_ms = step_ms[len(step_ms) // 2] if len(step_ms) % 2 else 0.5 * (step_ms[len(step_ms) // 2 - 1] + step_ms[len(step_ms) // 2])
    cols_s = b / (ms_step * 1e-3)
    # per-launch device time of the pass kernel: HIP events around every
    # launch on the query stream, in steps of their own (the events add a few
    # microseconds per launch, so the timed steps above run without them)
    prof_steps = max(1, min(5, args.steps))
    h.profile(True)
    Out2 = torch.empty_like(Out)
    for _ in range(prof_steps):
        h.matvec(Zd, out=Out2)
    h.sync()
    pass_ms, pass_n = h.profile_read(dm.K_L1_PASS)
    tot_ms, tot_n = h.profile_read(dm.K_TOTALS)
    h.profile(False)
    avg_pass_ms = pass_ms / max(pass_n, 1)
    # run-to-run agreement of two identical queries (the chained scan adds a
    # timing-dependent set of predecessor records: not guaranteed bitwise)
    # ulps are counted where |y| >= 2^-10 max|y| (near zero an ulp is
    # meaningless); the largest difference is also given relative to max|y|
    big = Out.abs() >= Out.abs().max() * 2.0 ** -10
    ulp = torch.abs(torch.nextafter(Out, torch.full_like(Out, float("inf"))) - Out)
    dif = (Out - Out2).abs()
    repro = {"identical_fraction": float((Out == Out2).float().mean().item()),
             "max_ulps_large": float((dif / ulp)[big].max().item()),
             "max_diff_over_max_abs": float((dif.max() / Out.abs().max()).item())}
    del big, ulp, dif, Out2
    log("batched: %.2f ms/step (wall %.2f ms), %.1f columns/s, pass %.3f ms x %d; run-to-run %s" %
        (ms_step, wall * 1e3 / args.steps, cols_s, avg_pass_ms, pass_n // prof_steps, repro))

    # per launch, averaged over the d passes of a query: each pass reads perm
    # and xs (8n), the Z rows (4nb) and the Out rows (4nb) and writes Out (4nb);
    # the first pass reads no Out
    bytes_pass = 12.0 * n * b + 8.0 * n - 4.0 * n * b / d
    achieved = bytes_pass / (avg_pass_ms * 1e-3) / 1e9
    traffic = read_traffic(vb)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "achievable_GBps": round(copy_gbps, 1), "frac_of_achievable": round(achieved / copy_gbps, 4),
                "random_row_probe_GBps": round(gather_gbps, 1) if gather_gbps else None,
                "frac_of_random_row_probe": round(achieved / gather_gbps, 4) if gather_gbps else None,
                "measured_GBps": round(traffic / (avg_pass_ms * 1e-3) / 1e9, 1) if traffic else None,
                "kernel": pass_kernel_name(vb, b), "variant": vb, "bytes_per_launch": bytes_pass,
                "avg_launch_ms": round(avg_pass_ms, 4), "launches": pass_n}

    # ---- single-vector form on the same 64 columns ----
    single = None
    single_out = None
    if not args.no_single:
        v1, tms1 = h.tune(1, reps=8)
        tuned["b1"] = {"variant": v1, "ms_per_pass": [round(t, 4) for t in tms1]}
        log("tuned b=1: variant %d, ms per pass %s" % (v1, ["%.3f" % t for t in tms1]))
        Zc = Zd.t().contiguous()                     # 64 x n: row c is column c of Z
        Oc = torch.empty_like(Zc)
        h.matvec(Zc[0], out=Oc[0])                   # warm-up (scratch for b = 1)
        h.sync()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for c in range(b):
            h.matvec(Zc[c], out=Oc[c])
        e1.record(stream)
        torch.cuda.synchronize()
        h.sync()
        t_single = e0.elapsed_time(e1) * 1e-3
        single_cols = b / t_single
        dif = (Oc.t() - Out).abs().max().item()
        scale = Out.abs().max().item()
        single = {"columns_per_s": round(single_cols, 2), "ms_per_column": round(t_single * 1e3 / b, 3),
                  "max_abs_diff_vs_batched": dif, "max_abs_out": scale}
        log("single-z: %.2f columns/s; batched/single = %.2f" % (single_cols, cols_s / single_cols))
        single_out = Oc.t().contiguous()              # n x b, column c from the c-th single query
        del Zc, Oc

    # ---- l2 squared ----
    l2 = None
    if not args.no_l2:
        h2 = dm.prepare(Xd, dm.L2SQ)
        O2 = torch.empty((n, b), dtype=torch.float32, device=dev)
        for _ in range(max(1, args.warmup)):
            h2.matvec(Zd, out=O2)
        h2.sync()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            h2.matvec(Zd, out=O2)
        e1.record(stream)
        torch.cuda.synchronize()
        h2.sync()
        ms2 = e0.elapsed_time(e1) / args.steps
        # algorithmic bytes of a query: X read by both contractions (2 x 4nd),
        # Z read once (4nb, the totals come with X^T Z), Out written once
        # (4nb), ||x||^2 read by both (2 x 8n)
        bytes2 = 2.0 * n * d * 4 + 2.0 * n * b * 4 + 2.0 * n * 8
        ach2 = bytes2 / (ms2 * 1e-3) / 1e9
        tr2 = read_l2_traffic() if (n, d, b) == (1 << 22, 128, 64) else None
        l2 = {"columns_per_s": round(b / (ms2 * 1e-3), 1), "ms_per_query": round(ms2, 3),
              "achieved_GBps": round(ach2, 1),
              "roofline": {"bound": "hbm", "achieved": round(ach2, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                           "frac": round(ach2 / HBM_PEAK_GBPS, 4), "traffic": tr2,
                           "scope": "whole query (X^T Z with totals, reduction, apply) on the query stream",
                           "bytes_per_query": bytes2, "achievable_GBps": round(copy_gbps, 1),
                           "frac_of_achievable": round(ach2 / copy_gbps, 4)}}
        log("l2sq: %.3f ms/query" % ms2)
        O2h = O2.cpu().numpy()
        h2.free()
        del O2
        l2["form"] = "BF16 hi+lo matrix cores for X^T Z and X V, FP64 rank-one terms"

    # ---- many datasets in one captured graph ----
    multi = None
    if not args.no_multi:
        multi = run_multi(args, dm, synth, np, torch, dev, stream)

    # ---- plain single-vector method on the mixture workload ----
    mixture = None
    if not args.no_mixture:
        mixture = run_single_mixture(args, dm, synth, np, torch, dev, stream)
    precision = None
    if not args.no_precision:
        precision = run_precision_stress(args, dm, synth, np, torch, dev, stream)

    # ---- approximate l2 through the l1 path ----
    approx = None
    if not args.no_approx_l2:
        approx = run_approx_l2(args, dm, synth, np, torch, dev, stream)

    # ---- odd p and total variation on the batched workload ----
    oddp = None
    if not args.no_oddp:
        oddp = run_oddp_tv(args, dm, torch, dev, stream, Xd, Zd)

    # ---- the sort-free family ----
    sortfree = None
    if not args.no_sortfree:
        sortfree = run_sortfree(args, dm, synth, np, torch, dev, stream)

    # ---- block-Krylov low rank ----
    lowrank = None
    if not args.no_lowrank:
        lowrank = run_lowrank(args, dm, synth, np, torch, dev)

    # ---- CPU oracle on a bounded sample (and the accuracy of the GPU result there) ----
    cpu = None
    errors = None
    Outh = Out.cpu().numpy()
    if not args.no_cpu_baseline:
        import oracle
        from oracle import metrics
        perm, _, _ = h.sorted()
        p0 = perm[0].cpu().numpy()
        pl = perm[d - 1].cpu().numpy()
        extra = [p0[0], p0[-1], pl[0], pl[-1]]
        s = synth.seeds(3)
        rows = synth.subsample_rows(n, args.cpu_rows, s["sub"], extra)
        X64 = X.astype(np.float64)
        Z64 = Z.astype(np.float64)
        threads = oracle.num_threads()
        t0 = time.perf_counter()
        o, rn, ad = oracle.matvec(X64, Z64, oracle.L1, rows)
        t_or = time.perf_counter() - t0
        cols_cpu = b / (t_or * n / rows.size)
        cpu = {"value": cols_cpu, "unit": "columns/s", "cores": threads, "kind": "oracle", "cpu": cpu_model(),
               "sample": "%d of %d rows (uniform seeded sample plus the scan-boundary points), all %d columns, "
                         "%.1f s; extrapolated by n/rows" % (rows.size, n, b, t_or)}
        frob = metrics.frob_from_rows(rn, n)
        errors = {"rows": int(rows.size), "l1": metrics.errors(Outh[rows], o, rn, ad, Z64, frob)}
        if single_out is not None:
            ys = single_out.index_select(0, torch.from_numpy(rows).to(dev)).cpu().numpy()
            errors["single_z"] = metrics.errors(ys, o, rn, ad, Z64, frob)
        if l2 is not None:
            o2, rn2, ad2 = oracle.matvec(X64, Z64, oracle.L2SQ, rows[:16])
            frob2 = float(np.sqrt(max(rn2.mean() * n, 0.0)))
            errors["l2sq_16rows"] = metrics.errors(O2h[rows[:16]], o2, rn2, ad2, Z64, frob2)
        log("cpu oracle: %.3g columns/s on %d threads; errors %s" % (cols_cpu, threads, errors))

    # ---- the GPU's results on the 16 384-row sample, for the offline oracle
    # comparison (tests/full_sample.py), and the committed figures of that
    # comparison when they describe these kernels ----
    if args.dump_rows:
        from oracle import sampling
        srows, _, _ = sampling.workload3_rows(X)
        ri = torch.from_numpy(srows).to(dev)
        dump = {"rows": srows, "l1": Out.index_select(0, ri).cpu().numpy()}
        if single_out is not None:
            dump["single"] = single_out.index_select(0, ri).cpu().numpy()
        if l2 is not None:
            dump["l2sq"] = O2h[srows]
        np.savez(args.dump_rows, **dump)
        log("wrote %d sampled rows to %s" % (srows.size, args.dump_rows))
    errors_16k = read_sample_errors()

    result = {
        "metric": "l1 dist-matvec columns/s (n=4M,d=128,b=64) batched vs single-z; % HBM peak",
        "value": round(cols_s, 2),
        "unit": "columns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "median_ms_per_step": round(median_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "l1 batched matvec, n=%d points, d=%d coordinates U[0,1) FP32, "
                               "Z %dx%d N(0,1) FP32" % (n, d, n, b), "n": n, "d": d, "b": b},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "single_z": single,
        "tuned_variants": tuned,
        "batched_vs_single": round(cols_s / single["columns_per_s"], 2) if single else None,
        "hbm_frac": roofline["frac"],
        "copy_probe_GBps": round(copy_gbps, 1),
        "random_row_probe_GBps": round(gather_gbps, 1) if gather_gbps else None,
        "prep_ms": round(prep_ms, 1),
        "totals_ms_per_step": round(tot_ms / prof_steps, 4),
        "run_to_run": repro,
        "l2sq": l2,
        "multi": multi,
        "lowrank": lowrank,
        "single_vector_mixture": mixture,
        "precision_stress": precision,
        "approx_l2": approx,
        "oddp_tv": oddp,
        "sortfree": sortfree,
        "errors": errors,
        "errors_16k_rows": errors_16k,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
