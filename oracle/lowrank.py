"""FP64 references for the low-rank application of the matvec (Appendix C).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``optimal_error`` - ||A - A_k||_F of the best rank-k approximation of a
  symmetric A, from its eigenvalues (Eckart-Young: the singular values of a
  symmetric matrix are the absolute eigenvalues).
* ``approx_error``  - ||A - U diag(lam) U^T||_F for a returned factorisation.
* ``block_krylov``  - block Krylov iteration driven only by products with A
  (the matrix-vector query model of Section 1 and the top-k singular value
  result cited in Appendix C.1); the FP64 counterpart of the GPU routine.
"""
from __future__ import annotations

import numpy as np


def optimal_error(A, k: int) -> float:
    A = np.asarray(A, dtype=np.float64)
    w = np.linalg.eigvalsh(0.5 * (A + A.T))
    s = np.sort(np.abs(w))[::-1]
    return float(np.sqrt(np.sum(s[k:] ** 2)))


def approx_error(A, U, lam) -> float:
    A = np.asarray(A, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    B = (U * lam[None, :]) @ U.T
    return float(np.linalg.norm(A - B))


def block_krylov(apply_A, n: int, k: int, block: int, iters: int, omega) -> tuple:
    """Rank-k approximation U diag(lam) U^T from products with A only.

    Basis K = [A W, A^2 W, ..., A^iters W] with W = omega (n x block), each
    block orthonormalised against itself before the next product to keep the
    powers well conditioned; then an orthonormal basis Q of K, T = Q^T A Q, its
    eigen-decomposition, and the k eigenpairs of largest |lambda|.
    """
    W = np.asarray(omega, dtype=np.float64)
    blocks = []
    cur = W
    for _ in range(iters):
        cur = apply_A(cur)
        q, _ = np.linalg.qr(cur)
        blocks.append(q)
        cur = q
    K = np.concatenate(blocks, axis=1)
    Q, _ = np.linalg.qr(K)
    T = Q.T @ apply_A(Q)
    T = 0.5 * (T + T.T)
    w, V = np.linalg.eigh(T)
    idx = np.argsort(-np.abs(w))[:k]
    return Q @ V[:, idx], w[idx]
