"""CPU oracle for the distance-matrix matrix-vector product ``A z``.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library (``paper_2210_15114_amd``) and never imports it.

Contents
--------
* ``matvec``        - the plain definition (A z)_i = sum_j z_j f(x_i, x_j), rows
                      of A formed explicitly, FP64 (``dm_oracle.c``); exact int64
                      variant with __int128 accumulation.
* ``explicit``      - the whole n x n matrix A (small n).
* ``exact_matvec``  - exact rational arithmetic (``fractions.Fraction``) for tiny n.
* ``sort_coords``   - Algorithm 1 (preprocessing): per coordinate the stable
                      sorted order, its inverse and the sorted values.
* ``totals``        - the full sums that Algorithm 2 reads at position n
                      (sum_j z_j and sum_j x_j(i) z_j), plus sum_j s_j z_j.
* ``alg2_query``    - Algorithm 2 in exact integer arithmetic, step by step in
                      the paper's order (prefix arrays B_i, C_i, then the
                      per-point lookups), for tiny inputs.
* ``alg3_query``    - Algorithm 3 (l2 squared) in exact arithmetic, in the
                      reading that uses sum_j y_j and sum_j y_j ||x_j||^2.
* ``odd_p_query``   - l_p^p for odd p (Appendix A.1) in exact arithmetic.
* ``even_p_query``  - Algorithm 5 (even p) in exact arithmetic, with the
                      binomial coefficients and weights restored.
* ``kl_query``      - Algorithm 4 (KL divergence), FP64, in the paper's order.
* ``mahalanobis_query`` - Algorithms 8 and 9 (the bilinear form x^T M y), FP64.
* ``metrics``       - error metrics and norms used to assess a result.
* ``lowrank``       - FP64 references for the low-rank application (Appendix C).
* ``approx_l2``     - FP64 references for the approximate l2 query (Appendix A.4).

Readings of the paper that the oracle fixes (the paper is silent or garbled
there) are listed in the repository's design notes; each function cites the
passage it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

L1 = 1
L2SQ = 2
TV = 3
L3 = 4
L5 = 5
L4 = 6
L6 = 7
KL = 8
CE = 9
MAHA2 = 10
BILINEAR = 11
MATRIX_METRICS = (MAHA2, BILINEAR)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile dm_oracle.c with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-std=c11", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, c_int = ctypes.c_int64, ctypes.c_int32, ctypes.c_int
        lib.oracle_rows_f64.argtypes = [P, i64, i32, c_int, P, P, i64, P]
        lib.oracle_rows_f64.restype = None
        lib.oracle_matvec_f64.argtypes = [P, i64, i32, c_int, P, P, i32, P, i64, P, P, P]
        lib.oracle_matvec_f64.restype = None
        lib.oracle_matvec_i64.argtypes = [P, i64, i32, c_int, P, i32, P, i64, P]
        lib.oracle_matvec_i64.restype = i64
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _rows_arg(n, rows):
    if rows is None:
        return np.arange(n, dtype=np.int64)
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    if r.size and (r.min() < 0 or r.max() >= n):
        raise ValueError("row index out of range")
    return r


# ----------------------------------------------------------------------------
# the plain definition
# ----------------------------------------------------------------------------
def _matrix_arg(metric, M, d):
    if metric not in MATRIX_METRICS:
        return None
    if M is None:
        raise ValueError("this metric needs the d x d matrix M")
    M = np.ascontiguousarray(np.asarray(M, dtype=np.float64))
    if M.shape != (d, d):
        raise ValueError("M must be d x d")
    return M


def matvec(X, Z, metric: int, rows=None, M=None):
    """FP64 (A z) for the given rows, with the row norms and |A||z| sums.

    Follows the definition of the query in Section 1 and the expansion at the
    start of the proof of the p = 1 theorem in Section 2 (sum over j of
    z_j times the distance), forming every entry explicitly.  M (d x d) is
    the matrix of MAHA2 and BILINEAR.

    Returns (Y, rownorm2, absdot): Y is m x b, rownorm2 = ||A_i||_2^2 (m),
    absdot = sum_j |A_ij| |z_jc| (m x b).
    """
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    Z = np.asarray(Z, dtype=np.float64)
    if Z.ndim == 1:
        Z = Z[:, None]
    Z = np.ascontiguousarray(Z)
    n, d = X.shape
    if Z.shape[0] != n:
        raise ValueError("Z rows != n")
    b = Z.shape[1]
    r = _rows_arg(n, rows)
    Mm = _matrix_arg(metric, M, d)
    m = r.size
    Y = np.zeros((m, b), dtype=np.float64)
    rn = np.zeros(m, dtype=np.float64)
    ad = np.zeros((m, b), dtype=np.float64)
    if m:
        _load().oracle_matvec_f64(_ptr(X), n, d, metric, None if Mm is None else _ptr(Mm), _ptr(Z), b,
                                  _ptr(r), m, _ptr(Y), _ptr(rn), _ptr(ad))
    return Y, rn, ad


def matvec_int(X, Z, metric: int, rows=None):
    """Exact integer (A z) for the given rows; returns (Y int64, n_overflow).

    Entries and products are formed in __int128, so Y is exact whenever
    n_overflow == 0 (otherwise the offending outputs hold the low 64 bits).
    """
    X = np.ascontiguousarray(np.asarray(X, dtype=np.int64))
    Z = np.asarray(Z, dtype=np.int64)
    if Z.ndim == 1:
        Z = Z[:, None]
    Z = np.ascontiguousarray(Z)
    n, d = X.shape
    b = Z.shape[1]
    r = _rows_arg(n, rows)
    m = r.size
    Y = np.zeros((m, b), dtype=np.int64)
    ov = 0
    if m:
        ov = int(_load().oracle_matvec_i64(_ptr(X), n, d, metric, _ptr(Z), b, _ptr(r), m, _ptr(Y)))
    return Y, ov


def explicit(X, metric: int, rows=None, M=None) -> np.ndarray:
    """Rows of the explicit distance matrix A (FP64), m x n."""
    X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    n, d = X.shape
    r = _rows_arg(n, rows)
    Mm = _matrix_arg(metric, M, d)
    A = np.zeros((r.size, n), dtype=np.float64)
    if r.size:
        _load().oracle_rows_f64(_ptr(X), n, d, metric, None if Mm is None else _ptr(Mm), _ptr(r), r.size,
                                _ptr(A))
    return A


def exact_matvec(X, Z, metric: int):
    """Exact rational (A z), tiny n only: list (n) of lists (b) of Fractions.

    Every float input is converted exactly (Fraction(float) is exact).  The
    loop order is the coordinate-outer one of the proof of the p = 1 theorem
    (Section 2), which sums over coordinates i then points j.
    """
    X = np.asarray(X)
    Z = np.asarray(Z)
    if Z.ndim == 1:
        Z = Z[:, None]
    n, d = X.shape
    b = Z.shape[1]
    Xf = [[Fraction(X[i, k].item()) for k in range(d)] for i in range(n)]
    Zf = [[Fraction(Z[j, c].item()) for c in range(b)] for j in range(n)]
    out = []
    for i in range(n):
        row = []
        for c in range(b):
            acc = Fraction(0)
            for k in range(d):
                for j in range(n):
                    diff = Xf[i][k] - Xf[j][k]
                    f = abs(diff) if metric == L1 else diff * diff
                    acc += Zf[j][c] * f
            row.append(acc)
        out.append(row)
    return out


# ----------------------------------------------------------------------------
# Algorithm 1: preprocessing
# ----------------------------------------------------------------------------
def sort_coords(X):
    """Algorithm 1 (Section 2): for each coordinate, the sorted order of the points.

    Returns (perm, rank, xs), each d x n:
      perm[k][r] = index of the point at position r of the sorted k-th coordinates,
      rank[k][i] = position of point i in that order (the lookup "position of
                   x_k(i) in T_i" of Algorithm 2),
      xs[k][r]   = X[perm[k][r], k] (the array T_k itself).
    Ties are broken by ascending point index (a stable sort); -0.0 and +0.0
    compare equal, so they tie as well.
    """
    X = np.asarray(X)
    n, d = X.shape
    perm = np.empty((d, n), dtype=np.int64)
    rank = np.empty((d, n), dtype=np.int64)
    xs = np.empty((d, n), dtype=X.dtype)
    for k in range(d):
        p = np.argsort(X[:, k], kind="stable")
        perm[k] = p
        rank[k, p] = np.arange(n)
        xs[k] = X[p, k]
    return perm, rank, xs


# ----------------------------------------------------------------------------
# totals read by Algorithm 2 at position n
# ----------------------------------------------------------------------------
def totals(X, Z):
    """FP64 T0[c] = sum_j z_jc, T1[k, c] = sum_j x_jk z_jc and U[c] = sum_j s_j z_jc.

    T0 and T1 are the entries C_i[n] and B_i[n] of Algorithm 2 (Section 2);
    s_j = sum_k x_jk, so U = sum_k T1[k, :].
    """
    X = np.asarray(X, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    if Z.ndim == 1:
        Z = Z[:, None]
    T0 = Z.sum(axis=0)
    T1 = X.T @ Z
    s = X.sum(axis=1)
    U = s @ Z
    return T0, T1, U


# ----------------------------------------------------------------------------
# Algorithm 2 step by step (exact, tiny inputs)
# ----------------------------------------------------------------------------
def odd_p_query(X, y, p: int):
    """The l_p^p query for odd p in exact arithmetic, by the sort of
    Algorithm 1 and prefix sums of powers (the odd-p theorem of Appendix A.1,
    whose proof the paper omits).

    Reading of the combination: for odd p, |a - b|^p = sign(a - b)(a - b)^p,
    and the binomial expansion of (a - b)^p splits the sum over the points
    before a point's position (sign +) and after it (sign -):
        sum_j y_j |x_k(i) - x_j(i)|^p
          = sum_t C(p, t) (-1)^t x_k(i)^(p-t) (2 P_t - T_t),
    with P_t the inclusive partial sum of y_j x_j(i)^t up to the point's
    position in the stable sorted order and T_t the full sum.  Ties contribute
    zero to either side.  For p = 1 this is Algorithm 2.
    """
    from math import comb
    X = [[Fraction(v) if not isinstance(v, Fraction) else v for v in row] for row in np.asarray(X, dtype=object).tolist()]
    y = [Fraction(v) if not isinstance(v, Fraction) else v for v in np.asarray(y, dtype=object).ravel().tolist()]
    n = len(X)
    d = len(X[0]) if n else 0
    z = [Fraction(0)] * n
    for i in range(d):
        order = sorted(range(n), key=lambda j: (X[j][i], j))
        P = [[Fraction(0)] * (p + 1) for _ in range(n)]
        acc = [Fraction(0)] * (p + 1)
        for q, j in enumerate(order):
            for t in range(p + 1):
                acc[t] += y[j] * X[j][i] ** t
            P[q] = list(acc)
        T = acc
        for q, k in enumerate(order):
            x = X[k][i]
            z[k] += sum(comb(p, t) * (-1) ** t * x ** (p - t) * (2 * P[q][t] - T[t]) for t in range(p + 1))
    return z


def alg2_query(X, y):
    """Algorithm 2 (Section 2) in exact arithmetic for integer or rational inputs.

    The order of the steps is the paper's: per coordinate, the partial sums
    B_i (of y_j x_j(i)) and C_i (of y_j) in the sorted order of T_i; then per
    point k and coordinate i the position q of x_k(i), the four sums S1..S4 and
    the update z(k) += x_k(i) (S3 - S4) + S2 - S1.

    Reading of the positions: B_i[q] and C_i[q] are inclusive partial sums up to
    and including position q, with q the point's own position in the stable
    order (ties by ascending index).  In exact arithmetic any position inside a
    run of equal values gives the same result because every tied term is zero.
    """
    X = [[Fraction(v) if not isinstance(v, Fraction) else v for v in row] for row in np.asarray(X, dtype=object).tolist()]
    y = [Fraction(v) if not isinstance(v, Fraction) else v for v in np.asarray(y, dtype=object).ravel().tolist()]
    n = len(X)
    d = len(X[0]) if n else 0
    B, C, pos = [], [], []
    for i in range(d):
        order = sorted(range(n), key=lambda j: (X[j][i], j))
        bi, ci, acc_b, acc_c = [], [], Fraction(0), Fraction(0)
        for j in order:
            acc_b += y[j] * X[j][i]
            acc_c += y[j]
            bi.append(acc_b)
            ci.append(acc_c)
        p = [0] * n
        for q, j in enumerate(order):
            p[j] = q
        B.append(bi)
        C.append(ci)
        pos.append(p)
    z = [Fraction(0)] * n
    for k in range(n):
        for i in range(d):
            q = pos[i][k]
            s1 = B[i][q]
            s2 = B[i][n - 1] - B[i][q]
            s3 = C[i][q]
            s4 = C[i][n - 1] - C[i][q]
            z[k] += X[k][i] * (s3 - s4) + s2 - s1
    return z


def alg3_query(X, y):
    """Algorithm 3 (Appendix A, p = 2) in exact arithmetic.

    z(k) = ||x_k||^2 * S1 + S2 - 2 <x_k, v>, with v = sum_j y_j x_j,
    S1 = sum_j y_j and S2 = sum_j y_j ||x_j||^2 (the algorithm's listing squares
    y_j in S1 and S2; the identity ||x-y||^2 = ||x||^2 + ||y||^2 - 2<x,y> of
    Section 1.2 gives the first power, which is the reading used here).
    """
    X = [[Fraction(v) for v in row] for row in np.asarray(X, dtype=object).tolist()]
    y = [Fraction(v) for v in np.asarray(y, dtype=object).ravel().tolist()]
    n = len(X)
    d = len(X[0]) if n else 0
    nrm = [sum(v * v for v in row) for row in X]
    v = [sum(y[j] * X[j][i] for j in range(n)) for i in range(d)]
    s1 = sum(y)
    s2 = sum(y[j] * nrm[j] for j in range(n))
    return [nrm[k] * s1 + s2 - 2 * sum(X[k][i] * v[i] for i in range(d)) for k in range(n)]


def even_p_query(X, y, p: int):
    """The l_p^p query for even p in exact arithmetic, by the moment expansion
    of Algorithm 5 (Appendix A.1), step by step in the algorithm's order.

    Reading: the printed moments S_(i,t) lack the binomial coefficients and the
    weights y_j, and the printed sum starts at t = 1.  The binomial theorem
    gives (x_k(i) - x_j(i))^p = sum_(t=0..p) C(p, t) x_k(i)^t (-x_j(i))^(p-t),
    so the moments are
        S_(i,t) = C(p, t) sum_j y_j (-x_j(i))^(p-t),   t = 0 .. p,
    and z(k) = sum_i sum_(t=0..p) x_k(i)^t S_(i,t).
    """
    from math import comb
    X = [[Fraction(v) if not isinstance(v, Fraction) else v for v in row] for row in np.asarray(X, dtype=object).tolist()]
    y = [Fraction(v) if not isinstance(v, Fraction) else v for v in np.asarray(y, dtype=object).ravel().tolist()]
    n = len(X)
    d = len(X[0]) if n else 0
    S = [[comb(p, t) * sum(y[j] * (-X[j][i]) ** (p - t) for j in range(n)) for t in range(p + 1)]
         for i in range(d)]
    return [sum(X[k][i] ** t * S[i][t] for i in range(d) for t in range(p + 1)) for k in range(n)]


def kl_query(X, y):
    """Algorithm 4 (the KL query of Appendix A) in FP64, in the algorithm's
    order: S_i = sum_j y_j log x_j(i) per coordinate, the entropies
    H_k = -sum_i x_k(i) log x_k(i) per point (0 log 0 = 0), Y = sum_j y_j, and
    z(k) = -H_k Y - sum_i x_k(i) S_i.  X must be positive wherever a
    logarithm of it is taken.
    """
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    S = np.log(X).T @ y
    H = -np.where(X > 0, X * np.log(np.where(X > 0, X, 1.0)), 0.0).sum(axis=1)
    Y = y.sum(axis=0)
    return -np.multiply.outer(H, Y) - X @ S


def mahalanobis_query(X, y, M):
    """Algorithms 8 and 9 (Appendix A.2) in FP64: the preprocessing forms
    S = M X^T (column j is M x_j); a query takes v = S y and returns
    z(k) = <x_k, v>.  This is the query of the bilinear form x^T M y that the
    paragraph writes as its f.
    """
    X = np.asarray(X, dtype=np.float64)
    S = np.asarray(M, dtype=np.float64) @ X.T
    v = S @ np.asarray(y, dtype=np.float64)
    return X @ v


from . import metrics  # noqa: E402  (re-export)
from . import lowrank  # noqa: E402
from . import approx_l2  # noqa: E402
