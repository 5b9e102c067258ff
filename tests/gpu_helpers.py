"""Shared helpers for the GPU parity tests (marshal numpy <-> device, oracle
comparisons).  Imports the oracle (test infrastructure) and the binding."""
from __future__ import annotations

import numpy as np

import oracle
from oracle import metrics

U32 = 2.0 ** -24


def torch_mod():
    import torch
    return torch


def dev(a):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run(X, Z, metric, b_as_vector=False):
    """Prepare X on the GPU, run one query, return (numpy Out, handle)."""
    import paper_2210_15114_amd as dm
    h = dm.prepare(dev(X), metric)
    Zd = dev(Z)
    Y = h.matvec(Zd)
    h.sync()
    return Y.cpu().numpy(), h


def float_errors(Xf32, Zf32, Y, metric, rows=None):
    """Errors of a float result against the FP64 oracle on the FP32 inputs."""
    X64 = Xf32.astype(np.float64)
    Z64 = Zf32.astype(np.float64)
    if Z64.ndim == 1:
        Z64 = Z64[:, None]
    n = X64.shape[0]
    r = np.arange(n) if rows is None else np.asarray(rows)
    o, rn, ad = oracle.matvec(X64, Z64, metric, r)
    if metric == oracle.L2SQ:
        frob = metrics.frob_l2sq(X64)
    else:
        frob = metrics.frob_from_rows(rn, n)
    Yr = np.asarray(Y, dtype=np.float64).reshape(n, -1)[r]
    return metrics.errors(Yr, o, rn, ad, Z64, frob), o


def bound_ratio(err, bound):
    """max(err / bound) over all entries, where a zero error against a zero
    bound counts as 0 and a nonzero error against a zero bound as infinity
    (a single point, or a constant coordinate, has an exact zero result)."""
    err = np.abs(np.asarray(err, dtype=np.float64))
    bound = np.broadcast_to(np.asarray(bound, dtype=np.float64), err.shape)
    pos = bound > 0
    r = np.where(pos, err / np.where(pos, bound, 1.0), np.where(err == 0, 0.0, np.inf))
    return float(r.max()) if r.size else 0.0


def centres(Xf32):
    """The per-coordinate shift the library applies to float points before the
    sorted and l2-squared queries form anything from them (its documented
    rule): the FP32 midpoint m of [min, max] when every value x of the
    coordinate has m/2 <= x <= 2m (or the mirror image for negative values),
    so that x - m is exact in FP32 (Sterbenz), else 0."""
    X = np.asarray(Xf32, dtype=np.float32)
    lo, hi = X.min(axis=0), X.max(axis=0)
    half = np.float32(0.5)
    m = half * lo + half * hi
    two = np.float32(2.0)
    ok = ((lo > 0) & (m <= two * lo) & (hi <= two * m)) | ((hi < 0) & (m >= two * hi) & (lo >= two * m))
    return np.where(ok, m, np.float32(0.0)).astype(np.float32)


def centred(Xf32):
    """X - c (exact in FP32 by the choice of c)."""
    X = np.asarray(Xf32, dtype=np.float32)
    return X - centres(X)[None, :]


def method_scale_l1(Xf32, Zf32, rows):
    """sum_k (|x~_ik| sum_j |z_j| + sum_j |x~_jk z_j|): size of the terms the l1
    method forms for row i (used to state its FP32 error bound), with x~ the
    centred coordinates the method works on."""
    X = np.abs(centred(Xf32).astype(np.float64))
    Z = np.abs(Zf32.astype(np.float64))
    if Z.ndim == 1:
        Z = Z[:, None]
    zl1 = Z.sum(axis=0)                      # b
    t1 = X.T @ Z                             # d x b
    return X[rows].sum(axis=1)[:, None] * zl1[None, :] + t1.sum(axis=0)[None, :]
