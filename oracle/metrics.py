"""Error metrics and matrix norms used to assess a computed ``A z``.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The acceptance metric for floating-point results is, per right-hand side c,

    max_i |y_ic - o_ic| / (||A||_F * ||z_c||_2)

where o is the FP64 oracle.  Two stricter figures are reported beside it:

    per-row        max_i |y_ic - o_ic| / (||A_i||_2 * ||z_c||_2)   (>= the above)
    componentwise  max_i |y_ic - o_ic| / sum_j |A_ij| |z_jc|

||A||_F needs all n^2 entries.  For l2 squared it has an exact closed form in
O(n d^2) (``frob_l2sq``); for l1 it is estimated from sampled rows.
"""
from __future__ import annotations

import numpy as np


def frob_l2sq(X) -> float:
    """Exact ||A||_F for A_ij = ||x_i - x_j||^2, from O(n d^2) sums.

    With a_i = ||x_i||^2 and G = X X^T, A = a 1^T + 1 a^T - 2G, so
    ||A||_F^2 = 2n sum a_i^2 + 2 (sum a_i)^2 + 4 ||X^T X||_F^2 - 8 a^T X (X^T 1).
    (The decomposition is the one of Section 1.2.)  A is unchanged by a
    translation of the points, so the sums are formed on X minus its column
    means: their cancellation then scales with the spread of the points, not
    with their distance from the origin.
    """
    X = np.asarray(X, dtype=np.float64)
    X = X - X.mean(axis=0)[None, :]
    n = X.shape[0]
    a = np.einsum("ij,ij->i", X, X)
    g = X.T @ X
    s = X.sum(axis=0)
    f2 = 2.0 * n * np.dot(a, a) + 2.0 * a.sum() ** 2 + 4.0 * np.sum(g * g) - 8.0 * np.dot(a, X @ s)
    return float(np.sqrt(max(f2, 0.0)))


def frob_from_rows(rownorm2, n: int) -> float:
    """||A||_F, exact when rownorm2 holds every row, else the sampling estimate
    (n / m) * sum over the m sampled rows of ||A_i||^2."""
    rn = np.asarray(rownorm2, dtype=np.float64)
    m = rn.size
    if m == 0:
        return 0.0
    return float(np.sqrt(rn.sum() * (n / m)))


def errors(y, o, rownorm2, absdot, Z, frob: float) -> dict:
    """All three error figures, maximised over the sampled rows and the columns.

    y, o: m x b (result and oracle on the same sampled rows), rownorm2: m,
    absdot: m x b, Z: n x b (the right-hand sides), frob: ||A||_F.
    """
    y = np.asarray(y, dtype=np.float64).reshape(np.shape(o))
    o = np.asarray(o, dtype=np.float64)
    if o.ndim == 1:
        o = o[:, None]
        y = y.reshape(o.shape)
    Z = np.asarray(Z, dtype=np.float64)
    if Z.ndim == 1:
        Z = Z[:, None]
    err = np.abs(y - o)
    zn = np.sqrt(np.sum(Z * Z, axis=0))  # b
    tiny = np.finfo(np.float64).tiny
    spec = err / np.maximum(frob * zn[None, :], tiny)
    rown = np.sqrt(np.asarray(rownorm2, dtype=np.float64))[:, None]
    per_row = err / np.maximum(rown * zn[None, :], tiny)
    comp = err / np.maximum(np.asarray(absdot, dtype=np.float64), tiny)
    rel = err / np.maximum(np.abs(o), tiny)
    return {
        "spec": float(spec.max()) if spec.size else 0.0,
        "per_row": float(per_row.max()) if per_row.size else 0.0,
        "componentwise": float(comp.max()) if comp.size else 0.0,
        "max_abs": float(err.max()) if err.size else 0.0,
        "max_rel": float(rel.max()) if rel.size else 0.0,
    }
