"""l_p^p products for odd p (the odd-p theorem of Appendix A.1): the sort of
Algorithm 1, prefix sums of z x^t for t = 0..p chained across tiles, and the
binomial combination.  Integer data bit-exact against the exact oracle;
float data against the FP64 oracle within the normalised bound and the
per-row bound (4p + 8 + 3d) u32 S_i, where
    S_i = sum_k sum_t C(p, t) |x_ik|^(p-t) sum_j |z_j| |x_jk|^t
bounds every term the combination forms (D_t, the Horner steps and the d
additions into Out each round once on terms of that size)."""
from math import comb

import numpy as np
import pytest

import oracle
import synth

from gpu_helpers import U32, bound_ratio, centred, dev, float_errors

pytestmark = pytest.mark.gpu
dm = pytest.importorskip("paper_2210_15114_amd")

METRIC = {3: 4, 5: 5}


def _scale(X, Z, p):
    """Size of the terms the odd-p method forms, on the centred coordinates
    it works with (integer data is not shifted)."""
    X = np.abs((centred(X) if X.dtype.kind == "f" else X).astype(np.float64))
    Z = np.abs(Z.astype(np.float64)).reshape(X.shape[0], -1)
    S = np.zeros((X.shape[0], Z.shape[1]))
    for k in range(X.shape[1]):
        xk = X[:, k]
        for t in range(p + 1):
            W = (xk ** t) @ Z                       # sum_j |z_j| |x_jk|^t, per column
            S += comb(p, t) * (xk ** (p - t))[:, None] * W[None, :]
    return S


@pytest.mark.parametrize("p,b", [(3, 1), (3, 5), (3, 64), (5, 1), (5, 8), (5, 33)])
def test_integer_bit_exact(p, b):
    g = synth.rng(8000 + 10 * p + b)
    n, d = 3001, 3
    lim = 1000 if p == 3 else 100
    X = g.integers(-lim, lim + 1, size=(n, d)).astype(np.int32)
    Z = np.rint((4096 if p == 3 else 256) * g.standard_normal((n, b))).astype(np.int32)
    o, ov = oracle.matvec_int(X, Z, METRIC[p])
    assert ov == 0
    h = dm.prepare(dev(X), METRIC[p])
    Y = h.matvec(dev(Z))
    h.sync()
    assert np.array_equal(Y.cpu().numpy(), o)
    Y64 = h.matvec(dev(Z.astype(np.int64)))
    h.sync()
    assert np.array_equal(Y64.cpu().numpy(), o)
    h.free()


@pytest.mark.parametrize("p,b,dist", [(3, 1, "normal"), (3, 16, "normal"), (3, 64, "uniform"),
                                      (5, 1, "uniform"), (5, 8, "normal"), (5, 64, "uniform")])
def test_float_within_bounds(p, b, dist):
    g = synth.rng(8100 + 10 * p + b)
    n, d = 4099 if b > 1 else 20001, 5
    X = (g.standard_normal((n, d)) if dist == "normal" else g.random((n, d))).astype(np.float32)
    Z = g.standard_normal((n, b)).astype(np.float32)
    h = dm.prepare(dev(X), METRIC[p])
    Y = h.matvec(dev(Z)).cpu().numpy()
    h.sync()
    h.free()
    e, o = float_errors(X, Z, Y, METRIC[p])
    S = _scale(X, Z, p)
    ratio = bound_ratio(np.abs(Y.reshape(n, -1).astype(np.float64) - o), ((4 * p + 8 + 3 * d) * U32 * S))
    print("p", p, "errors", e, "bound-ratio", ratio)
    assert e["spec"] <= 1e-6
    assert ratio <= 1.0


def test_integer_overflow_guard_trips():
    X = np.array([[0], [2 ** 20]], dtype=np.int32)
    Z = np.array([[2 ** 20], [1]], dtype=np.int32)       # ||z||_1 range^3 >= 2^80
    h = dm.prepare(dev(X), METRIC[3])
    h.matvec(dev(Z))
    with pytest.raises(dm.DMError) as ex:
        h.sync()
    assert ex.value.status == dm.ERR_OVERFLOW
    h.free()
