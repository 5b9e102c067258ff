"""FP64 references for the approximate l2 query (Appendix A.4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``BETA``        - sqrt(2/pi), the mean of |g| for a standard Gaussian g,
  the constant of the embedding theorem.
* ``embed``       - the map T of the embedding theorem applied to every point:
  T(x)_i = (1 / (beta k)) sum_j G_ij x_j, i.e. X' = X G^T / (beta k).
* ``explicit_l2`` - rows of the exact Euclidean distance matrix,
  A_ij = ||x_i - x_j||_2, from the l2-squared oracle.
"""
from __future__ import annotations

import math

import numpy as np

BETA = math.sqrt(2.0 / math.pi)


def embed(X, G) -> np.ndarray:
    X = np.asarray(X, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    k = G.shape[0]
    return (X @ G.T) / (BETA * k)


def explicit_l2(X, rows=None) -> np.ndarray:
    from . import explicit, L2SQ
    return np.sqrt(np.maximum(explicit(X, L2SQ, rows), 0.0))
