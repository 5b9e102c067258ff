"""GPU parity at the full workload sizes, in the launch configurations the
benchmark times, on sampled rows that the FP64 oracle computes one by one.

* single vector, n = 2^20 points, d = 64, 32-component Gaussian mixture, one
  z ~ N(0,1): l1 and l2-squared;
* block of b = 64 columns, n = 2^22 points, d = 128, uniform [0,1) FP32:
  l1 (the benchmarked pass) and l2-squared (matrix-core path; 256 rows
  including the 16 points of largest norm);
* 512 datasets of uneven n and d, float and integer, b = 8, one graph
  launch: every dataset checked (4 rows; all rows of the 16 smallest),
  integer datasets bit-exact, float datasets within the bounds.

The sampled rows include the points at the ends of every tile size the pass
kernels use in coordinate 0, where the chained scan hands its carry from
one tile to the next.  Bounds are those of the small-size tests: normalised
error <= 1e-6 and the per-row arithmetic bounds of each path.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import L1, L2SQ

from gpu_helpers import U32, bound_ratio, centred, dev, float_errors, method_scale_l1

pytestmark = pytest.mark.gpu
dm = pytest.importorskip("paper_2210_15114_amd")


def _rows(X, m, seed):
    """m seeded rows plus the points at tile edges of coordinate 0's sorted order."""
    n = X.shape[0]
    order = np.argsort(X[:, 0], kind="stable")
    edges = []
    for t in (128, 256, 512, 1024, 2048, 4096, 8192, 16384):
        for r in (t - 1, t):
            if r < n:
                edges.append(order[r])
    edges += [order[0], order[n - 1]]
    return synth.subsample_rows(n, m, seed, extra=edges)


def _l2_scale(X32, Z32, rows):
    """M_i of the l2-squared bound, for the given rows only (on the centred
    coordinates the method works with)."""
    X = centred(X32).astype(np.float64)
    Z = np.abs(Z32.astype(np.float64)).reshape(X.shape[0], -1)
    nrm = np.einsum("ij,ij->i", X, X)
    t = np.abs(X).T @ Z
    Xr = X[rows]
    return (nrm[rows][:, None] * Z.sum(axis=0)[None, :] + (nrm @ Z)[None, :] + 2 * np.abs(Xr) @ t)


def _check_l1(X32, Z32, Y, rows):
    e, o = float_errors(X32, Z32, Y, L1, rows)
    d = X32.shape[1]
    S = method_scale_l1(X32, Z32, rows)
    err = np.abs(Y.reshape(X32.shape[0], -1)[rows].astype(np.float64) - o)
    ratio = bound_ratio(err, ((8 + 3 * d) * U32 * S))
    print("l1 errors", e, "bound-ratio", ratio)
    assert e["spec"] <= 1e-6 and e["per_row"] <= 1e-6
    assert ratio <= 1.0


def _check_l2(X32, Z32, Y, rows, tol):
    e, o = float_errors(X32, Z32, Y, L2SQ, rows)
    M = _l2_scale(X32, Z32, rows)
    err = np.abs(Y.reshape(X32.shape[0], -1)[rows].astype(np.float64) - o)
    ratio = bound_ratio(err, (tol * M))
    print("l2sq errors", e, "bound-ratio", ratio)
    assert e["spec"] <= 1e-6
    assert ratio <= 1.0


def test_mixture_single_vector_l1_and_l2sq():
    X, Z = synth.workload2()                     # n = 2^20, d = 64, one column
    z = Z[:, 0].copy()
    s = synth.seeds(2)
    rows = _rows(X, 48, s["sub"])
    Xd, zd = dev(X), dev(z)
    h = dm.prepare(Xd, L1)
    y = h.matvec(zd)
    h.sync()
    _check_l1(X, z, y.cpu().numpy(), rows)
    h.free()
    h2 = dm.prepare(Xd, L2SQ)
    y2 = h2.matvec(zd)
    h2.sync()
    _check_l2(X, z, y2.cpu().numpy(), rows, 4 * U32)
    h2.free()


def test_uniform_block_of_64_l1_and_l2sq():
    X, Z = synth.workload3()                     # n = 2^22, d = 128, b = 64
    s = synth.seeds(3)
    rows = _rows(X, 16, s["sub"])
    Xd, Zd = dev(X), dev(Z)
    h = dm.prepare(Xd, L1)
    Y = h.matvec(Zd)
    h.sync()
    Yl1 = Y.cpu().numpy()
    h.free()
    del Y
    h2 = dm.prepare(Xd, L2SQ)
    Y2 = h2.matvec(Zd)
    h2.sync()
    Yl2 = Y2.cpu().numpy()
    h2.free()
    del Xd, Zd, Y2
    _check_l1(X, Z, Yl1, rows)
    # l2 squared: 240 seeded rows and the 16 points of largest norm (the
    # largest terms of the expansion)
    nrm = np.einsum("ij,ij->i", X.astype(np.float64), X.astype(np.float64))
    far = np.argsort(nrm, kind="stable")[-16:]
    rows2 = synth.subsample_rows(X.shape[0], 240, s["sub"] + 1, extra=far)
    _check_l2(X, Z, Yl2, rows2, 2.0 ** -13)


def test_uneven_512_datasets_one_graph():
    b = 8
    specs = synth.workload4_specs(512)
    Xs, Zs = [], []
    for sp in specs:
        X, Z = synth.workload4_dataset(sp, b)
        Xs.append(X)
        Zs.append(Z)
    h = dm.prepare_multi([dev(X) for X in Xs])
    outs = h.matvec([dev(Z) for Z in Zs])
    h.sync()
    # every dataset on 4 seeded rows, and every row of the 16 smallest ones
    g = synth.rng(synth.seeds(4)["sub"])
    smallest = set(np.argsort([sp.n for sp in specs], kind="stable")[:16].tolist())
    for i, sp in enumerate(specs):
        rows = np.arange(sp.n) if i in smallest else np.sort(g.choice(sp.n, size=min(4, sp.n), replace=False))
        Y = outs[i].cpu().numpy()
        if sp.is_int:
            o, ov = oracle.matvec_int(Xs[i], Zs[i], L1, rows)
            assert ov == 0
            assert np.array_equal(Y[rows], o), "dataset %d (n=%d, d=%d)" % (i, sp.n, sp.d)
        else:
            _check_l1(Xs[i], Zs[i], Y, rows)
    h.free()
