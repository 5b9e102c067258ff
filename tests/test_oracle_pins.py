"""Pins for the CPU oracle: checks against what the paper and the mathematics fix.

None of these re-types the oracle's formula: each compares it with an
independent route (exact rational arithmetic, exact integers, closed forms,
special cases the paper discusses, invariances of the distance matrix).
"""
from fractions import Fraction

import numpy as np
import pytest

import synth
import oracle
from oracle import L1, L2SQ, metrics


def _rand(n, d, seed, kind="normal"):
    g = synth.rng(seed)
    if kind == "normal":
        return g.standard_normal((n, d))
    if kind == "int":
        return g.integers(-50, 50, size=(n, d), endpoint=True).astype(np.int64)
    raise ValueError(kind)


# ---------------------------------------------------------------------------
# exact rational brute force (Theorem for p = 1, Section 2; Algorithm 3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("metric", [L1, L2SQ])
def test_fp64_oracle_vs_exact_rational(oracle_mod, metric):
    X = _rand(23, 5, 11 + metric)
    Z = _rand(23, 3, 12 + metric)
    exact = oracle.exact_matvec(X, Z, metric)
    Y, rn, ad = oracle.matvec(X, Z, metric)
    u = 2.0 ** -53
    n, d = X.shape
    for i in range(n):
        for c in range(Z.shape[1]):
            err = abs(Fraction(Y[i, c]) - exact[i][c])
            # error of the FP64 loops: (d + n) roundings of terms bounded by |A_ij||z_j|
            bound = Fraction((n + d + 2) * u * ad[i, c])
            assert err <= bound, (i, c, float(err), float(bound))


def test_alg2_equals_definition_exactly():
    """Theorem for p = 1 (Section 2): Algorithm 2 computes A y exactly."""
    X = _rand(17, 4, 3, "int")
    X[5] = X[2]          # duplicate point
    X[:, 1] = 7          # an all-equal coordinate (one tie run)
    y = _rand(17, 1, 4, "int")[:, 0]
    z = oracle.alg2_query(X, y)
    ex = oracle.exact_matvec(X, y[:, None], L1)
    assert [row[0] for row in ex] == z


def test_alg3_reading_first_power_of_y():
    """Algorithm 3 with sum_j y_j and sum_j y_j ||x_j||^2 equals the definition;
    the squared-y form printed in the listing does not (it is not even linear)."""
    X = _rand(9, 3, 5, "int")
    y = _rand(9, 1, 6, "int")[:, 0]
    z = oracle.alg3_query(X, y)
    ex = [row[0] for row in oracle.exact_matvec(X, y[:, None], L2SQ)]
    assert z == ex
    # the listing as printed: S1 = sum y_j^2, S2 = sum y_j^2 ||x_j||^2
    Xf = [[Fraction(int(v)) for v in row] for row in X]
    yf = [Fraction(int(v)) for v in y]
    nrm = [sum(v * v for v in r) for r in Xf]
    v = [sum(yf[j] * Xf[j][i] for j in range(9)) for i in range(3)]
    s1 = sum(t * t for t in yf)
    s2 = sum(yf[j] ** 2 * nrm[j] for j in range(9))
    literal = [nrm[k] * s1 + s2 - 2 * sum(Xf[k][i] * v[i] for i in range(3)) for k in range(9)]
    assert literal != ex


# ---------------------------------------------------------------------------
# integers: exact oracle and FP64 oracle agree bit for bit below 2^53
# ---------------------------------------------------------------------------
def test_int_oracle_vs_python_bigint(oracle_mod):
    X = _rand(31, 6, 21, "int")
    Z = _rand(31, 2, 22, "int")
    for metric in (L1, L2SQ):
        Y, ov = oracle.matvec_int(X, Z, metric)
        assert ov == 0
        ex = oracle.exact_matvec(X, Z, metric)
        assert [[int(v) for v in row] for row in ex] == Y.tolist()


def test_int_oracle_reports_overflow(oracle_mod):
    X = np.array([[-(2 ** 31)], [2 ** 31 - 1]], dtype=np.int64)
    Z = np.array([[2 ** 32], [2 ** 32]], dtype=np.int64)
    Y, ov = oracle.matvec_int(X, Z, L1)       # (2^32 - 1) * 2^32 > 2^63
    assert ov == 2
    Y, ov = oracle.matvec_int(X, Z // 4, L1)
    assert ov == 0 and Y[0, 0] == (2 ** 32 - 1) * 2 ** 30


def test_int_and_fp64_bit_equal_workload1_integer(oracle_mod):
    X, z = synth.workload1("int")
    rows = np.arange(0, X.shape[0], 7)
    Yi, ov = oracle.matvec_int(X, z, L1, rows)
    assert ov == 0
    Yf, _, _ = oracle.matvec(X.astype(np.float64), z.astype(np.float64), L1, rows)
    # every partial sum is an integer below 2^53 in magnitude, so FP64 is exact
    assert np.abs(Yi).max() < 2 ** 53
    assert np.array_equal(Yf.astype(np.int64), Yi)
    assert np.array_equal(Yf, Yi.astype(np.float64))


# ---------------------------------------------------------------------------
# structure of the explicit matrix
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("metric", [L1, L2SQ])
def test_explicit_symmetric_zero_diag_nonneg(oracle_mod, metric):
    X = _rand(200, 7, 31)
    A = oracle.explicit(X, metric)
    assert np.array_equal(A, A.T)
    assert np.all(np.diag(A) == 0)
    assert np.all(A >= 0)
    # one entry recomputed by hand
    i, j = 3, 150
    if metric == L1:
        assert A[i, j] == pytest.approx(np.abs(X[i] - X[j]).sum(), rel=1e-15)
    else:
        assert A[i, j] == pytest.approx(((X[i] - X[j]) ** 2).sum(), rel=1e-15)


@pytest.mark.parametrize("metric", [L1, L2SQ])
def test_row_sums(oracle_mod, metric):
    X = _rand(300, 5, 41, "int").astype(np.float64)
    A = oracle.explicit(X, metric)
    Y, _, _ = oracle.matvec(X, np.ones((300, 1)), metric)
    assert np.array_equal(Y[:, 0], A.sum(axis=1))     # integers: exact either way


def test_l1_lattice_closed_form(oracle_mod):
    n, d = 257, 3
    i = np.arange(1, n + 1, dtype=np.int64)
    X = np.stack([i + 5 * k for k in range(d)], axis=1)      # shifted copies
    expect = d * (i * (i - 1) // 2 + (n - i) * (n - i + 1) // 2)
    Y, ov = oracle.matvec_int(X, np.ones((n, 1), np.int64), L1)
    assert ov == 0 and np.array_equal(Y[:, 0], expect)
    Yf, _, _ = oracle.matvec(X.astype(float), np.ones((n, 1)), L1)
    assert np.array_equal(Yf[:, 0], expect.astype(float))


def test_l2sq_lattice_closed_form(oracle_mod):
    # x_i = i in one dimension: sum_j (i - j)^2 over j = 1..n
    n = 101
    i = np.arange(1, n + 1, dtype=np.int64)
    s1 = n * (n + 1) // 2
    s2 = n * (n + 1) * (2 * n + 1) // 6
    expect = n * i * i - 2 * i * s1 + s2
    Y, ov = oracle.matvec_int(i[:, None], np.ones((n, 1), np.int64), L2SQ)
    assert np.array_equal(Y[:, 0], expect)


# ---------------------------------------------------------------------------
# the special cases of the lower bound for the query (Appendix A.5)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("metric", [L1, L2SQ])
def test_identical_points_give_zero(oracle_mod, metric):
    X = np.tile(np.array([[1.5, -2.0, 3.25]]), (64, 1))
    Z = _rand(64, 2, 51)
    Y, _, _ = oracle.matvec(X, Z, metric)
    assert np.all(Y == 0)


def test_outlier_case_golden(oracle_mod):
    """Fixture in tests/golden: n-1 identical points and one at distance 1."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "outlier_lower_bound.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    kv = {r[0]: r[1:] for r in rows}
    n, d = int(kv["n"][0]), int(kv["d"][0])
    X = np.array([float(v) for v in kv["X"]]).reshape(n, d)
    expect = np.array([float(v) for v in kv["A1"]])
    total = float(kv["sum"][0])
    for metric in (L1, L2SQ):   # distance 1 in one coordinate: l1 and l2^2 agree
        Y, _, _ = oracle.matvec(X, np.ones((n, 1)), metric)
        assert np.array_equal(Y[:, 0], expect)
        assert Y.sum() == total == 2 * (n - 1)


# ---------------------------------------------------------------------------
# invariances
# ---------------------------------------------------------------------------
def test_separability_over_coordinates(oracle_mod):
    """The proof of the p = 1 theorem swaps the sums: A = sum_k A^(k)."""
    X = _rand(150, 6, 61, "int")
    Z = _rand(150, 2, 62, "int")
    for metric in (L1, L2SQ):
        full, _ = oracle.matvec_int(X, Z, metric)
        parts = sum(oracle.matvec_int(X[:, k:k + 1], Z, metric)[0] for k in range(6))
        assert np.array_equal(full, parts)


def test_translation_scaling_permutation_linearity(oracle_mod):
    X = _rand(120, 4, 71, "int")
    Z = _rand(120, 2, 72, "int")
    W = _rand(120, 2, 73, "int")
    for metric in (L1, L2SQ):
        base, _ = oracle.matvec_int(X, Z, metric)
        shifted, _ = oracle.matvec_int(X + np.array([3, -7, 11, 0]), Z, metric)
        assert np.array_equal(base, shifted)
        scaled, _ = oracle.matvec_int(4 * X, Z, metric)
        assert np.array_equal(scaled, (4 if metric == L1 else 16) * base)
        p = synth.rng(74).permutation(120)
        permuted, _ = oracle.matvec_int(X[p], Z[p], metric)
        assert np.array_equal(permuted, base[p])
        lin, _ = oracle.matvec_int(X, 3 * Z - 2 * W, metric)
        other, _ = oracle.matvec_int(X, W, metric)
        assert np.array_equal(lin, 3 * base - 2 * other)


def test_block_identity_of_a_union(oracle_mod):
    """Section 3's reduction: for the union of two point sets, A_union [1;0]
    holds A_a 1 on the first block and the cross block's row sums below."""
    Xa = _rand(40, 3, 81, "int")
    Xb = _rand(30, 3, 82, "int")
    U = np.concatenate([Xa, Xb])
    e = np.concatenate([np.ones(40, np.int64), np.zeros(30, np.int64)])[:, None]
    Yu, _ = oracle.matvec_int(U, e, L1)
    Ya, _ = oracle.matvec_int(Xa, np.ones((40, 1), np.int64), L1)
    assert np.array_equal(Yu[:40], Ya)
    cross = np.abs(Xb[:, None, :] - Xa[None, :, :]).sum(axis=2).sum(axis=1)
    assert np.array_equal(Yu[40:, 0], cross)


# ---------------------------------------------------------------------------
# l2 squared structure (Section 1.2) and the Frobenius closed form
# ---------------------------------------------------------------------------
def test_l2sq_rank_and_frobenius(oracle_mod):
    X = _rand(300, 4, 91)
    A = oracle.explicit(X, L2SQ)
    s = np.linalg.svd(A, compute_uv=False)
    assert s[4 + 2] < 1e-9 * s[0]          # numerical rank <= d + 2
    assert s[4 + 1] > 1e-6 * s[0]
    assert metrics.frob_l2sq(X) == pytest.approx(np.linalg.norm(A), rel=1e-12)
    A1 = oracle.explicit(X, L1)
    assert np.linalg.svd(A1, compute_uv=False)[20] > 1e-6 * np.linalg.norm(A1)   # l1 is not low rank


def test_frob_l2sq_far_from_origin(oracle_mod):
    """The closed form on points 10^4 + U[0,1): the explicit A's norm, which
    is the same as that of the points moved back to the origin."""
    X = 1.0e4 + synth.rng(93).random((300, 4))
    A = oracle.explicit(X, L2SQ)
    assert metrics.frob_l2sq(X) == pytest.approx(np.linalg.norm(A), rel=1e-9)
    assert metrics.frob_l2sq(X) == pytest.approx(metrics.frob_l2sq(X - 1.0e4), rel=1e-9)


def test_frob_from_rows(oracle_mod):
    X = _rand(200, 3, 92)
    Y, rn, ad = oracle.matvec(X, np.ones((200, 1)), L1)
    A = oracle.explicit(X, L1)
    assert metrics.frob_from_rows(rn, 200) == pytest.approx(np.linalg.norm(A), rel=1e-12)


# ---------------------------------------------------------------------------
# Algorithm 1: the sort, its inverse and ties
# ---------------------------------------------------------------------------
def test_sort_coords_definition():
    X = _rand(500, 3, 101, "int").astype(np.float32)
    X[10:20, 0] = 0.0
    X[20:25, 0] = -0.0          # -0 and +0 tie
    perm, rank, xs = oracle.sort_coords(X)
    for k in range(3):
        ref = sorted(range(500), key=lambda j: (float(X[j, k]), j))
        assert perm[k].tolist() == ref
        assert np.array_equal(rank[k][perm[k]], np.arange(500))
        assert np.all(np.diff(xs[k].astype(np.float64)) >= 0)


def test_totals_definition():
    X = _rand(50, 3, 111, "int")
    Z = _rand(50, 2, 112, "int")
    T0, T1, U = oracle.totals(X, Z)
    for c in range(2):
        assert T0[c] == sum(int(Z[j, c]) for j in range(50))
        for k in range(3):
            assert T1[k, c] == sum(int(X[j, k]) * int(Z[j, c]) for j in range(50))
        assert U[c] == sum(int(X[j].sum()) * int(Z[j, c]) for j in range(50))


# ---------------------------------------------------------------------------
# the metrics themselves
# ---------------------------------------------------------------------------
def test_error_metrics_order(oracle_mod):
    X = _rand(100, 3, 121)
    Z = _rand(100, 2, 122)
    Y, rn, ad = oracle.matvec(X, Z, L1)
    A = oracle.explicit(X, L1)
    frob = np.linalg.norm(A)
    pert = Y + 1e-3
    e = metrics.errors(pert, Y, rn, ad, Z, frob)
    assert e["per_row"] >= e["spec"]
    assert e["max_abs"] == pytest.approx(1e-3, rel=1e-6)
    assert e["spec"] == pytest.approx(1e-3 / (frob * np.linalg.norm(Z, axis=0).min()), rel=1e-6)


# ---------------------------------------------------------------------------
# low-rank references (Appendix C): Eckart-Young and block Krylov
# ---------------------------------------------------------------------------
def _known_spectrum(seed=31):
    g = np.random.default_rng(seed)
    V, _ = np.linalg.qr(g.standard_normal((6, 6)))
    w = np.array([5.0, -4.0, 3.0, 0.5, -0.25, 0.1])
    return V, w, (V * w) @ V.T


def test_optimal_error_is_the_eigenvalue_tail():
    from oracle import lowrank
    V, w, A = _known_spectrum()
    # singular values of a symmetric matrix are |eigenvalues|: 5, 4, 3, 0.5, 0.25, 0.1
    assert abs(lowrank.optimal_error(A, 3) - np.sqrt(0.5 ** 2 + 0.25 ** 2 + 0.1 ** 2)) < 1e-12
    assert abs(lowrank.optimal_error(A, 0) - np.linalg.norm(A)) < 1e-12
    # the exact top eigenpairs attain it
    assert abs(lowrank.approx_error(A, V[:, :3], w[:3]) - lowrank.optimal_error(A, 3)) < 1e-12


def test_block_krylov_full_basis_gives_exact_eigenpairs():
    from oracle import lowrank
    V, w, A = _known_spectrum()
    g = np.random.default_rng(7)
    U, lam = lowrank.block_krylov(lambda W: A @ W, 6, 3, 3, 2, g.standard_normal((6, 3)))
    assert np.allclose(lam, [5.0, -4.0, 3.0], atol=1e-12)
    assert abs(lowrank.approx_error(A, U, lam) - lowrank.optimal_error(A, 3)) < 1e-12


def test_block_krylov_recovers_l2sq_matrix_of_rank_d_plus_2(oracle_mod):
    from oracle import lowrank
    g = np.random.default_rng(11)
    X = g.standard_normal((200, 2))
    A = oracle_mod.explicit(X, oracle_mod.L2SQ)
    assert np.linalg.matrix_rank(A) == 4
    U, lam = lowrank.block_krylov(lambda W: A @ W, 200, 4, 4, 2, g.standard_normal((200, 4)))
    assert lowrank.approx_error(A, U, lam) <= 1e-10 * np.linalg.norm(A)


# ---------------------------------------------------------------------------
# approximate l2 (Appendix A.4): the embedding constant and its concentration
# ---------------------------------------------------------------------------
def test_beta_is_the_mean_absolute_gaussian():
    from scipy import integrate
    from oracle import approx_l2
    val, _ = integrate.quad(lambda x: abs(x) * np.exp(-0.5 * x * x) / np.sqrt(2 * np.pi), -np.inf, np.inf)
    assert abs(approx_l2.BETA - val) < 1e-12


def test_embedding_preserves_l2_norms_in_l1():
    from oracle import approx_l2
    g = np.random.default_rng(101)
    X = g.standard_normal((5, 12)) * np.array([[1.0], [3.0], [0.01], [100.0], [7.0]])
    G = g.standard_normal((40000, 12))
    Y = approx_l2.embed(X, G)
    ratio = np.abs(Y).sum(axis=1) / np.linalg.norm(X, axis=1)
    # relative spread of one |g.x| / (beta ||x||) is sqrt(pi/2 - 1) = 0.755; over
    # k = 40000 samples its mean is within 4 standard errors of 1 w.h.p.
    assert np.all(np.abs(ratio - 1.0) < 4 * 0.755 / np.sqrt(40000))


def test_embedded_l1_matrix_approximates_l2_matrix(oracle_mod):
    from oracle import approx_l2
    g = np.random.default_rng(202)
    X = g.standard_normal((300, 10))
    A = approx_l2.explicit_l2(X)
    assert np.allclose(A, np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)), rtol=1e-12, atol=1e-12)
    k = 2000
    B = oracle_mod.explicit(approx_l2.embed(X, g.standard_normal((k, 10))), oracle_mod.L1)
    rel = np.linalg.norm(A - B) / np.linalg.norm(A)
    expect = np.sqrt(np.pi / 2 - 1) / np.sqrt(k)        # about 0.017
    assert 0.5 * expect < rel < 1.5 * expect


# ---------------------------------------------------------------------------
# total variation (Appendix A.3): the largest difference of event probabilities
# ---------------------------------------------------------------------------
def test_tv_is_the_largest_event_difference(oracle_mod):
    import itertools
    g = np.random.default_rng(303)
    d = 7
    X = g.dirichlet(np.ones(d), size=6)
    A = oracle_mod.explicit(X, oracle_mod.TV)
    for i in range(6):
        for j in range(6):
            best = 0.0
            for r in range(d + 1):
                for S in itertools.combinations(range(d), r):
                    idx = list(S)
                    best = max(best, abs(X[i, idx].sum() - X[j, idx].sum()))
            assert abs(A[i, j] - best) < 1e-14
    assert np.all(A <= 1.0 + 1e-15) and np.all(A >= 0.0)


# ---------------------------------------------------------------------------
# odd p (Appendix A.1): the moment-prefix combination and the oracle
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("p", [1, 3, 5])
def test_odd_p_combination_equals_definition_exactly(p):
    from fractions import Fraction
    import oracle
    g = np.random.default_rng(600 + p)
    X = g.integers(-6, 7, size=(9, 3))
    X[3] = X[5]                                   # ties
    y = g.integers(-5, 6, size=9)
    z = oracle.odd_p_query(X, y, p)
    for k in range(9):
        ref = sum(Fraction(int(y[j])) * sum(abs(int(X[k][i]) - int(X[j][i])) ** p for i in range(3)) for j in range(9))
        assert z[k] == ref


@pytest.mark.parametrize("metric,p", [(4, 3), (5, 5)])
def test_odd_p_oracle_against_exact(oracle_mod, metric, p):
    g = np.random.default_rng(700 + p)
    X = g.integers(-50, 51, size=(40, 4)).astype(np.int64)
    Z = g.integers(-9, 10, size=(40, 2)).astype(np.int64)
    o, ov = oracle_mod.matvec_int(X, Z, metric)
    assert ov == 0
    for c in range(2):
        ref = [sum(int(Z[j, c]) * sum(abs(int(X[k, i]) - int(X[j, i])) ** p for i in range(4)) for j in range(40))
               for k in range(40)]
        assert [int(v) for v in o[:, c]] == ref
    of, _, _ = oracle_mod.matvec(X.astype(np.float64), Z.astype(np.float64), metric)
    assert np.array_equal(of, o.astype(np.float64))     # below 2^53 the FP64 oracle is exact too


def test_l3_lattice_sum_of_cubes(oracle_mod):
    # x_i = i on a line: sum_j |i - j|^3 = (i(i-1)/2)^2 + ((n-i)(n-i+1)/2)^2
    n = 300
    X = np.arange(1, n + 1, dtype=np.float64)[:, None]
    o, _, _ = oracle_mod.matvec(X, np.ones((n, 1)), oracle_mod.L3)
    i = np.arange(1, n + 1, dtype=np.float64)
    ref = (i * (i - 1) / 2) ** 2 + ((n - i) * (n - i + 1) / 2) ** 2
    assert np.array_equal(o[:, 0], ref)


# ---------------------------------------------------------------------------
# the sort-free family (Appendix A): even p, KL, cross entropy, Mahalanobis
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("p", [2, 4, 6])
def test_even_p_expansion_equals_definition_exactly(p):
    # Algorithm 5 with the binomial coefficients and weights restored
    g = np.random.default_rng(800 + p)
    X = g.integers(-6, 7, size=(9, 3))
    y = g.integers(-5, 6, size=9)
    z = oracle.even_p_query(X, y, p)
    for k in range(9):
        ref = sum(int(y[j]) * sum((int(X[k][i]) - int(X[j][i])) ** p for i in range(3)) for j in range(9))
        assert z[k] == ref


def test_even_p_two_is_algorithm_3():
    g = np.random.default_rng(810)
    X = [[Fraction(int(v), 7) for v in row] for row in g.integers(-20, 21, size=(8, 3))]
    y = [Fraction(int(v), 3) for v in g.integers(-9, 10, size=8)]
    assert oracle.even_p_query(X, y, 2) == oracle.alg3_query(X, y)


@pytest.mark.parametrize("metric,p", [(oracle.L4, 4), (oracle.L6, 6)])
def test_even_p_oracle_against_moment_expansion(oracle_mod, metric, p):
    g = np.random.default_rng(820 + p)
    X = g.integers(-40, 41, size=(30, 3)).astype(np.int64)
    Z = g.integers(-9, 10, size=(30, 2)).astype(np.int64)
    o, ov = oracle_mod.matvec_int(X, Z, metric)
    assert ov == 0
    for c in range(2):
        assert [int(v) for v in o[:, c]] == [int(v) for v in oracle.even_p_query(X, Z[:, c], p)]
    of, _, _ = oracle_mod.matvec(X.astype(np.float64), Z.astype(np.float64), metric)
    assert np.array_equal(of, o.astype(np.float64))     # below 2^53 the FP64 oracle is exact too


@pytest.mark.parametrize("p", [4, 6])
def test_even_p_lattice_faulhaber(oracle_mod, p):
    # x_i = i on a line: sum_j (i - j)^p = F(i - 1) + F(n - i), F(N) = sum_(m<=N) m^p
    def F(N):
        if p == 4:
            return N * (N + 1) * (2 * N + 1) * (3 * N * N + 3 * N - 1) // 30
        return N * (N + 1) * (2 * N + 1) * (3 * N ** 4 + 6 * N ** 3 - 3 * N + 1) // 42
    n = 150
    X = np.arange(1, n + 1, dtype=np.int64)[:, None]
    o, ov = oracle_mod.matvec_int(X, np.ones((n, 1), np.int64), oracle.L4 if p == 4 else oracle.L6)
    assert ov == 0
    assert [int(v) for v in o[:, 0]] == [F(i - 1) + F(n - i) for i in range(1, n + 1)]


def _simplex(n, d, seed):
    g = np.random.default_rng(seed)
    P = g.random((n, d)) + 0.05
    return P / P.sum(axis=1, keepdims=True)


def test_kl_matches_scipy_relative_entropy(oracle_mod):
    from scipy.stats import entropy
    X = _simplex(12, 5, 830)
    A = oracle_mod.explicit(X, oracle.KL)
    ref = np.array([[entropy(X[i], X[j]) for j in range(12)] for i in range(12)])
    assert np.allclose(A, ref, rtol=1e-12, atol=1e-15)
    assert np.all(np.diag(A) == 0.0)                     # log(x / x) = 0
    off = ~np.eye(12, dtype=bool)
    assert np.all(A[off] > 0)                            # Gibbs' inequality
    assert not np.allclose(A, A.T)                       # not symmetric


def test_cross_entropy_is_entropy_plus_kl(oracle_mod):
    from scipy.stats import entropy
    X = _simplex(10, 4, 831)
    A = oracle_mod.explicit(X, oracle.CE)
    ref = np.array([[entropy(X[i]) + entropy(X[i], X[j]) for j in range(10)] for i in range(10)])
    assert np.allclose(A, ref, rtol=1e-12, atol=1e-15)


def test_kl_algorithm_4_equals_definition(oracle_mod):
    g = np.random.default_rng(832)
    X = g.random((40, 6)) * 3 + 0.01                     # positive, not normalised
    Z = g.standard_normal((40, 3))
    Y, _, _ = oracle_mod.matvec(X, Z, oracle.KL)
    Yq = oracle.kl_query(X, Z)
    L = np.abs(np.log(X))
    S = (np.abs(X) * L).sum(axis=1)[:, None] * np.abs(Z).sum(axis=0) + np.abs(X) @ (L.T @ np.abs(Z))
    assert np.all(np.abs(Y - Yq) <= 16 * (6 + 2) * 2.0 ** -53 * S)
    # a sign slip in either would move the result by about S
    assert np.max(np.abs(Y - Yq) / S) < 1e-12


def test_mahalanobis_identity_is_l2sq(oracle_mod):
    X = _rand(30, 4, 840)
    Z = _rand(30, 2, 841)
    Y, _, _ = oracle_mod.matvec(X, Z, oracle.MAHA2, M=np.eye(4))
    Y2, _, _ = oracle_mod.matvec(X, Z, L2SQ)
    assert np.array_equal(Y, Y2)


def test_mahalanobis_matches_scipy(oracle_mod):
    from scipy.spatial.distance import cdist
    g = np.random.default_rng(842)
    X = g.standard_normal((25, 5))
    B = g.standard_normal((5, 5))
    M = B @ B.T + 0.5 * np.eye(5)
    A = oracle_mod.explicit(X, oracle.MAHA2, M=M)
    ref = cdist(X, X, "mahalanobis", VI=M) ** 2
    assert np.allclose(A, ref, rtol=1e-10, atol=1e-12)


def test_mahalanobis_sees_only_the_symmetric_part(oracle_mod):
    g = np.random.default_rng(843)
    X = g.standard_normal((20, 4))
    M = g.standard_normal((4, 4))
    A = oracle_mod.explicit(X, oracle.MAHA2, M=M)
    As = oracle_mod.explicit(X, oracle.MAHA2, M=(M + M.T) / 2)
    assert np.allclose(A, As, rtol=1e-12, atol=1e-12)
    assert np.allclose(A, A.T, rtol=1e-12, atol=1e-12) and np.all(np.diag(A) == 0.0)


def test_bilinear_algorithms_8_and_9_equal_definition(oracle_mod):
    g = np.random.default_rng(844)
    X = g.standard_normal((30, 5))
    Z = g.standard_normal((30, 2))
    M = g.standard_normal((5, 5))                        # not symmetric
    Y, _, _ = oracle_mod.matvec(X, Z, oracle.BILINEAR, M=M)
    Yq = oracle.mahalanobis_query(X, Z, M)
    S = np.abs(X) @ np.abs(M) @ np.abs(X).T @ np.abs(Z)
    assert np.all(np.abs(Y - Yq) <= 64 * 2.0 ** -53 * S)
    A = oracle_mod.explicit(X, oracle.BILINEAR, M=M)
    assert np.allclose(A.T, oracle_mod.explicit(X, oracle.BILINEAR, M=M.T), rtol=1e-12, atol=1e-12)
    assert np.allclose(oracle_mod.explicit(X, oracle.BILINEAR, M=np.eye(5)), X @ X.T, rtol=1e-12, atol=1e-12)
