"""Block-Krylov low-rank approximation on the GPU (Appendix C.1, Table 2).

Checked at n = 8192 points (d = 32, a 50-component Gaussian mixture, the
recipe of the low-rank workload) against
  * the FP64 oracle's block Krylov iteration from the same start block
    (same Krylov space, products formed from the explicit A): Ritz values
    agree to the accuracy of the FP32 products;
  * Eckart-Young: ||A - A_k||_F from the eigenvalues of the explicit A is a
    lower bound, and the GPU approximation comes within a small factor of it;
  * orthonormality of the returned U.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import L1, L2SQ
from oracle import lowrank as olr

from gpu_helpers import dev

pytestmark = pytest.mark.gpu
dm = pytest.importorskip("paper_2210_15114_amd")


def _mixture(n, d):
    return synth.gaussian_mixture(n, d, 50, synth.seeds(5)["X"], 5.0, np.float32)


def test_rank32_against_eckart_young_and_oracle():
    n, d, k, block, iters = 8192, 32, 32, 40, 8
    X = _mixture(n, d)
    omega = synth.rhs_normal(n, block, synth.seeds(5)["Z"], np.float64)
    h = dm.prepare(dev(X), L1)
    U, lam, sweeps = h.lowrank(k, dev(omega), iters)
    U, lam = U.cpu().numpy(), lam.cpu().numpy()
    h.free()
    A = oracle.explicit(X, L1)
    Uo, lo = olr.block_krylov(lambda W: A @ W, n, k, block, iters, omega)
    opt = olr.optimal_error(A, k)
    err = olr.approx_error(A, U, lam)
    err_o = olr.approx_error(A, Uo, lo)
    orth = float(np.abs(U.T @ U - np.eye(k)).max())
    dlam = float(np.abs(lam - lo).max() / abs(lo[0]))
    print("sweeps", sweeps, "orth", orth, "dlam/|lam1|", dlam, "err", err, "oracle err", err_o, "optimal", opt,
          "eps", err / opt - 1)
    assert orth <= 1e-10
    assert np.all(np.abs(lam[:-1]) >= np.abs(lam[1:]))
    assert dlam <= 1e-5
    assert abs(err - err_o) <= 1e-4 * err_o
    assert err >= opt * (1 - 1e-9)
    assert err <= 1.01 * opt


def test_exact_low_rank_matrix_is_recovered():
    # l2 squared on d = 3 coordinates: A has rank <= d + 2 = 5, so a basis of
    # 2 blocks of 8 columns spans it and the rank-5 approximation is A itself
    g = synth.rng(5151)
    n, d = 3000, 3
    X = g.standard_normal((n, d)).astype(np.float32)
    omega = g.standard_normal((n, 8))
    h = dm.prepare(dev(X), L2SQ)
    U, lam, _ = h.lowrank(5, dev(omega), 2)
    U, lam = U.cpu().numpy(), lam.cpu().numpy()
    h.free()
    A = oracle.explicit(X, L2SQ)
    rel = olr.approx_error(A, U, lam) / np.linalg.norm(A)
    print("relative error", rel, "lam", lam)
    assert rel <= 1e-5


@pytest.mark.parametrize("block", [33, 36, 48, 64])
def test_blocks_that_split_into_two_queries(block):
    # a block above 32 columns that is not a multiple of 32 runs each product
    # as a query of its first 32 columns and one of the rest (33: 32 + 1,
    # 36: 32 + 4, 48: 32 + 16; 64 is one query); the rank-5 matrix of l2
    # squared on d = 3 coordinates must come back exactly whatever the split
    g = synth.rng(5353 + block)
    n, d = 3000, 3
    X = g.standard_normal((n, d)).astype(np.float32)
    omega = g.standard_normal((n, block))
    h = dm.prepare(dev(X), L2SQ)
    U, lam, _ = h.lowrank(5, dev(omega), 1)
    U, lam = U.cpu().numpy(), lam.cpu().numpy()
    h.free()
    A = oracle.explicit(X, L2SQ)
    rel = olr.approx_error(A, U, lam) / np.linalg.norm(A)
    orth = float(np.abs(U.T @ U - np.eye(5)).max())
    print("block", block, "relative error", rel, "orth", orth)
    assert rel <= 1e-5
    assert orth <= 1e-10


def test_lowrank_rejects_bad_arguments():
    X = synth.rng(1).standard_normal((500, 2)).astype(np.float32)
    h = dm.prepare(dev(X), L1)
    import torch
    om = torch.zeros((500, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(dm.DMError):
        h.lowrank(9, om[:, :4].contiguous(), 2)     # rank above block * iters = 8
    with pytest.raises(dm.DMError):
        h.lowrank(4, torch.zeros((500, 65), dtype=torch.float64, device="cuda"), 1)   # block above 64
    h.free()
    Xi = synth.rng(2).integers(-5, 5, size=(300, 2)).astype(np.int32)
    hi = dm.prepare(dev(Xi), L1)
    with pytest.raises(dm.DMError):
        hi.lowrank(2, torch.zeros((300, 4), dtype=torch.float64, device="cuda"), 2)
    hi.free()


@pytest.mark.parametrize("metric,d,rank", [(oracle.MAHA2, 3, 5), (oracle.L4, 1, 5), (oracle.BILINEAR, 4, 4)])
def test_exact_low_rank_of_the_sort_free_metrics(metric, d, rank):
    # the expansions have rank at most d + 2 (Mahalanobis), p + 1 per coordinate
    # (even p; d = 1 here) and d (the bilinear form), so the rank-r
    # approximation from a large enough Krylov basis is A itself
    g = synth.rng(5252 + metric)
    n = 2500
    X = g.standard_normal((n, d)).astype(np.float32)
    M = synth.square_matrix(d, 5253, "spd") if metric in oracle.MATRIX_METRICS else None
    omega = g.standard_normal((n, 8))
    h = dm.prepare(dev(X), metric, M=M)
    U, lam, _ = h.lowrank(rank, dev(omega), 2)
    U, lam = U.cpu().numpy(), lam.cpu().numpy()
    h.free()
    A = oracle.explicit(X, metric, M=M)
    rel = olr.approx_error(A, U, lam) / np.linalg.norm(A)
    print("metric", metric, "relative error", rel)
    assert rel <= 1e-5


def test_lowrank_refuses_a_non_symmetric_bilinear_form():
    import torch
    X = synth.rng(5254).standard_normal((300, 3)).astype(np.float32)
    h = dm.prepare(dev(X), oracle.BILINEAR, M=synth.square_matrix(3, 5255, "general"))
    om = torch.zeros((300, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(dm.DMError) as ex:
        h.lowrank(2, om, 1)
    assert ex.value.status == dm.ERR_STATE
    h.free()
