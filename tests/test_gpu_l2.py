"""GPU parity of the l2-squared path (Algorithm 3) against the CPU oracle.

Integer inputs: bit-exact against the exact oracle (wrapping int64 is exact
modulo 2^64 and the guard keeps results below 2^63).  Float inputs: against
the FP64 oracle on the FP32-rounded inputs, normalised error <= 1e-6, and the
componentwise bound below, derived from the arithmetic of each path:
  * vector path (b < 16): FP64 accumulation, one FP32 rounding of the result;
  * matrix-core path (b >= 16): products of BF16 hi/lo splits, each operand
    kept to about 2^-16 relative, so |y_i - o_i| <= 2^-13 * M_i with
    M_i = ||x_i||^2 ||z||_1 + sum_j ||x_j||^2 |z_j| + 2 sum_k |x_ik| sum_j |x_jk z_j|.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import L2SQ

from gpu_helpers import U32, bound_ratio, centred, dev, float_errors, run

pytestmark = pytest.mark.gpu
dm = pytest.importorskip("paper_2210_15114_amd")


def _mscale(X32, Z32):
    X = (centred(X32) if X32.dtype.kind == "f" else X32).astype(np.float64)
    Z = np.abs(Z32.astype(np.float64))
    nrm = (X * X).sum(axis=1)
    zl1 = Z.sum(axis=0)
    t = np.abs(X).T @ Z
    return nrm[:, None] * zl1[None, :] + (nrm @ Z)[None, :] + 2 * np.abs(X) @ t


# matrix-core shapes: d <= 32 (4 waves split the points), 33..64 (2), 65..96
# (one wave idle), 97..128; b up to 32 (one column tile) and beyond; d = 128,
# b = 64 with n a multiple of 4096 takes the kernel that also forms the totals
@pytest.mark.parametrize("n,d,b", [(1, 3, 1), (2048, 16, 1), (3001, 7, 4), (5000, 64, 16), (4099, 128, 64),
                                   (3000, 20, 24), (257, 33, 17), (4500, 96, 40), (9001, 128, 33),
                                   (4096, 128, 64), (8192, 128, 64)])
def test_float(n, d, b):
    g = synth.rng(700 + n + b)
    X = g.standard_normal((n, d), dtype=np.float32)
    Z = g.standard_normal((n, b), dtype=np.float32)
    Y, _ = run(X, Z, L2SQ)
    e, o = float_errors(X, Z, Y, L2SQ)
    M = _mscale(X, Z)
    err = np.abs(Y.astype(np.float64) - o)
    tol = 2.0 ** -13 if b >= 16 else 4 * U32
    ratio = bound_ratio(err, (tol * M))
    print("errors", e, "bound-ratio", ratio)
    assert e["spec"] <= 1e-6
    assert ratio <= 1.0


@pytest.mark.parametrize("b", [1, 5, 64])
def test_integer_bit_exact(b):
    g = synth.rng(800 + b)
    n, d = 3333, 16
    X = g.integers(-2 ** 15, 2 ** 15, size=(n, d)).astype(np.int32)
    Z = np.rint(4096 * g.standard_normal((n, b))).astype(np.int32)
    Y, _ = run(X, Z, L2SQ)
    o, ov = oracle.matvec_int(X, Z, L2SQ)
    assert ov == 0
    assert np.array_equal(Y, o)


def test_identical_points_give_zero():
    X = np.tile(np.array([[1.0, 2.0, -3.0]], np.float32), (500, 1))
    Z = synth.rng(9).standard_normal((500, 2)).astype(np.float32)
    Y, _ = run(X, Z, L2SQ)
    assert np.abs(Y).max() <= 1e-3 * np.abs(Z).sum()


@pytest.mark.parametrize("b", [1, 16, 64])
def test_nonfinite_rhs_flagged(b):
    g = synth.rng(850 + b)
    X = g.standard_normal((700, 8)).astype(np.float32)
    Z = g.standard_normal((700, b)).astype(np.float32)
    Z[333, b - 1] = np.inf
    h = dm.prepare(dev(X), L2SQ)
    h.matvec(dev(Z))
    with pytest.raises(dm.DMError) as ei:
        h.sync()
    assert ei.value.status == dm.ERR_NONFINITE
    Z[333, b - 1] = 0.0
    h.matvec(dev(Z))
    h.sync()


@pytest.mark.parametrize("case", ["inf", "nan", "both_infs"])
def test_nonfinite_rhs_flagged_fused_totals(case):
    # d = 128, b = 64, n = 4096: the totals come from the X^T Z kernel, and a
    # non-finite z shows as a non-finite column sum (+inf and -inf give NaN)
    g = synth.rng(860)
    n, d, b = 4096, 128, 64
    X = g.standard_normal((n, d)).astype(np.float32)
    Z = g.standard_normal((n, b)).astype(np.float32)
    Z0 = Z.copy()
    if case == "inf":
        Z[4000, 7] = np.inf
    elif case == "nan":
        Z[17, 63] = np.nan
    else:
        Z[5, 30] = np.inf
        Z[4095, 30] = -np.inf
    h = dm.prepare(dev(X), L2SQ)
    h.matvec(dev(Z))
    with pytest.raises(dm.DMError) as ei:
        h.sync()
    assert ei.value.status == dm.ERR_NONFINITE
    Y = h.matvec(dev(Z0))
    h.sync()
    e, _ = float_errors(X, Z0, Y.cpu().numpy(), L2SQ)
    assert e["spec"] <= 1e-6


@pytest.mark.parametrize("n,d,b", [(8192, 128, 64), (4099, 96, 40), (3001, 7, 4)])
def test_float_query_is_bitwise_reproducible(n, d, b):
    # every sum of the l2-squared query has a fixed order (no look-back chain)
    g = synth.rng(870 + n)
    X = g.standard_normal((n, d), dtype=np.float32)
    Z = g.standard_normal((n, b), dtype=np.float32)
    h = dm.prepare(dev(X), L2SQ)
    Zd = dev(Z)
    Y1 = h.matvec(Zd).cpu().numpy()
    Y2 = h.matvec(Zd).cpu().numpy()
    h.sync()
    assert np.array_equal(Y1, Y2)
