"""Approximate l2 products through the l1 path (Appendix A.4).

* The Gaussian embedding X' = X G^T / (beta k) on the GPU matches the FP64
  oracle to one FP32 rounding (FP64 accumulation), for float and integer
  points and ragged sizes.
* The l1 query on X' is the unchanged l1 path: it matches the oracle's l1
  product over the same embedded points within the l1 bounds.
* The approximation itself: B (the l1 matrix of X') is within the embedding
  theorem's error of the exact Euclidean distance matrix A: ||A - B||_F /
  ||A||_F against the expected relative spread sqrt(pi/2 - 1) / sqrt(k) of
  one entry (the theorem bounds the Frobenius norm; the error of one product
  A z is reported with a loose sanity bound, since clustered points make the
  entry errors correlated).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import L1
from oracle import approx_l2

from gpu_helpers import U32, bound_ratio, dev, float_errors, method_scale_l1

pytestmark = pytest.mark.gpu
dm = pytest.importorskip("paper_2210_15114_amd")


@pytest.mark.parametrize("dtype", [np.float32, np.float64, np.int32])
def test_embedding_matches_oracle(dtype):
    g = synth.rng(4040)
    n, d, k = 5001, 37, 131            # ragged against the 64 x 64 output tiles and 32-coordinate steps
    if dtype == np.int32:
        X = g.integers(-1000, 1000, size=(n, d)).astype(np.int32)
    else:
        X = g.standard_normal((n, d)).astype(dtype)
    G = g.standard_normal((k, d))
    Y = dm.embed_l2(dev(X), dev(G)).cpu().numpy().astype(np.float64)
    o = approx_l2.embed(X, G)
    scale = np.abs(X.astype(np.float64)) @ np.abs(G).T / (approx_l2.BETA * k)
    err = np.abs(Y - o)
    # one FP32 rounding of the FP64 result, plus the FP64 sum's own error
    assert np.all(err <= U32 * np.abs(o) + 1e-13 * scale)


def test_approximate_l2_query():
    g = synth.rng(4141)
    n, d, k, b = 4096, 16, 512, 4
    X = synth.gaussian_mixture(n, d, 8, 4242, 5.0, np.float32)
    G = g.standard_normal((k, d))
    Z = g.standard_normal((n, b)).astype(np.float32)
    Xe = dm.embed_l2(dev(X), dev(G))
    h = dm.prepare(Xe, L1)
    Y = h.matvec(dev(Z)).cpu().numpy()
    h.sync()
    h.free()
    Xe = Xe.cpu().numpy()
    # (1) the query is the l1 path on the embedded points
    e, o = float_errors(Xe, Z, Y, L1)
    S = method_scale_l1(Xe, Z, np.arange(n))
    ratio = bound_ratio(np.abs(Y.astype(np.float64) - o), ((8 + 3 * k) * U32 * S))
    print("l1 errors on X'", e, "bound-ratio", ratio)
    assert e["spec"] <= 1e-6 and ratio <= 1.0
    # (2) B approximates the Euclidean distance matrix A
    A = approx_l2.explicit_l2(X)
    B = oracle.explicit(Xe, L1)
    expect = np.sqrt(np.pi / 2 - 1) / np.sqrt(k)
    frob = np.linalg.norm(A - B) / np.linalg.norm(A)
    Az = A @ Z.astype(np.float64)
    qrel = np.linalg.norm(Az - Y) / np.linalg.norm(Az)
    print("frobenius", frob, "query", qrel, "expected spread", expect)
    assert frob <= 1.5 * expect          # the theorem's guarantee (Frobenius)
    assert qrel <= 4 * expect            # a product with one z: a sanity bound only
