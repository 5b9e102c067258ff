"""Rows on which the oracle is evaluated for the full-size batched workload.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The FP64 oracle forms
each sampled row of A explicitly, so a full-size error figure is taken on a
sample: 16 384 rows uniformly without replacement (the workload's seed_sub),
plus the points at rank 0 and rank n-1 of coordinates 0 and d-1 (where the
sorted scan starts and ends) and 16 rows of the longest run of tied values of
coordinate 0 (stable order, ties by ascending point index).
"""
from __future__ import annotations

import numpy as np

import synth

M_ROWS = 16384


def boundary_and_tie_rows(X):
    """Scan-boundary points of coordinates 0 and d-1, and 16 rows of the longest
    tie run of coordinate 0; returns (rows, length of that run)."""
    X = np.asarray(X)
    extra = []
    for k in (0, X.shape[1] - 1):
        o = np.argsort(X[:, k], kind="stable")
        extra += [int(o[0]), int(o[-1])]
    o = np.argsort(X[:, 0], kind="stable")
    v = X[o, 0]
    starts = np.flatnonzero(np.concatenate([[True], v[1:] != v[:-1]]))
    lens = np.diff(np.concatenate([starts, [v.size]]))
    i = int(np.argmax(lens))
    extra += [int(r) for r in o[starts[i]:starts[i] + lens[i]][:16]]
    return extra, int(lens[i])


def workload3_rows(X, m: int = M_ROWS):
    """The sample of the batched workload: (rows, extra rows, tie-run length)."""
    extra, tie_len = boundary_and_tie_rows(X)
    rows = synth.subsample_rows(X.shape[0], m, synth.seeds(3)["sub"], extra)
    return rows, extra, tie_len
