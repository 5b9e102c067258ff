"""Planted mistakes in the oracle must be caught by its pins.

Each case copies ``oracle/dm_oracle.c``, plants one plausible mistake (a dropped
term, a wrong sign or index, a transposed operand), compiles the copy on the
CPU, swaps it in for the real library and runs a battery of pins.  The test
passes when at least one pin fails for every mutant, and when every pin passes
for the unmodified source.
"""
import ctypes
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import L1, L2SQ

MUTANTS = {
    "l1_dropped_abs": ("a += fabs(diff);", "a += diff;"),
    "l2_wrong_square": ("a += diff * diff;", "a += diff * fabs(diff);"),
    "wrong_coordinate_index": ("double diff = xi[k] - xj[k];", "double diff = xi[k] - xj[(k + 1) % d];"),
    "transposed_rhs": ("y[c] += a * zj[c];", "y[c] += a * Z[c * (int64_t)b + (j % b)];"),
    "wrong_sign": ("y[c] += a * zj[c];", "y[c] -= a * zj[c];"),
    "dropped_first_point": ("        for (int64_t j = 0; j < n; ++j) {\n            double a = entry_f64",
                            "        for (int64_t j = 1; j < n; ++j) {\n            double a = entry_f64"),
    "row_index_ignored": ("        const double* xi = X + rows[t] * (int64_t)d;\n        double* y",
                          "        const double* xi = X + t * (int64_t)d;\n        double* y"),
    "int_dropped_abs": ("__int128 ad = diff < 0 ? -diff : diff;", "__int128 ad = diff;"),
    "int_wrong_column": ("acc[c] += a * (__int128)zj[c];", "acc[c] += a * (__int128)zj[0];"),
    "int_overflow_unchecked": ("if (acc[c] > (__int128)INT64_MAX || acc[c] < (__int128)INT64_MIN) overflow += 1;", ""),
    "even_p_wrong_power": ("(metric == DM_ORACLE_L4 ? 4 : 6); ++e) pw *= diff;",
                           "(metric == DM_ORACLE_L4 ? 3 : 6); ++e) pw *= diff;"),
    "int_even_p_odd_power": ("for (int e = 1; e < (metric == DM_ORACLE_L4 ? 4 : 6); ++e) pw *= diff;\n            a += pw;\n        } else {\n            a += diff * diff;\n        }\n    }\n    return a;",
                             "for (int e = 1; e < (metric == DM_ORACLE_L4 ? 4 : 5); ++e) pw *= diff;\n            a += pw;\n        } else {\n            a += diff * diff;\n        }\n    }\n    return a;"),
    "kl_swapped_arguments": ("a += xi[k] * log(xi[k] / xj[k]);", "a += xj[k] * log(xj[k] / xi[k]);"),
    "kl_dropped_entropy": ("a += xi[k] * log(xi[k] / xj[k]);", "a -= xi[k] * log(xj[k]);"),
    "ce_wrong_sign": ("if (xi[k] != 0.0) a -= xi[k] * log(xj[k]);", "if (xi[k] != 0.0) a += xi[k] * log(xj[k]);"),
    "maha_one_sided": ("a += (xi[k] - xj[k]) * M[(int64_t)k * d + l] * (xi[l] - xj[l]);",
                       "a += xi[k] * M[(int64_t)k * d + l] * (xi[l] - xj[l]);"),
    "bilinear_transposed": ("a += xi[k] * M[(int64_t)k * d + l] * xj[l];",
                            "a += xi[k] * M[(int64_t)l * d + k] * xj[l];"),
}


def _pins():
    """Quick pins; returns the names of those that fail."""
    failed = []

    def check(name, fn):
        try:
            ok = fn()
        except Exception:
            ok = False
        if not ok:
            failed.append(name)

    g = synth.rng(5)
    Xr = g.standard_normal((11, 3))
    Zr = g.standard_normal((11, 2))

    def exact_rational():
        for metric in (L1, L2SQ):
            ex = oracle.exact_matvec(Xr, Zr, metric)
            Y, _, ad = oracle.matvec(Xr, Zr, metric)
            for i in range(11):
                for c in range(2):
                    if abs(Fraction(Y[i, c]) - ex[i][c]) > Fraction(20 * 2.0 ** -53 * ad[i, c]):
                        return False
        return True

    def structure():
        for metric in (L1, L2SQ):
            A = oracle.explicit(Xr, metric)
            if not (np.array_equal(A, A.T) and np.all(np.diag(A) == 0) and np.all(A >= 0)):
                return False
        return True

    def lattice():
        n = 33
        i = np.arange(1, n + 1, dtype=np.int64)
        X = np.stack([i, i + 4], axis=1)
        e1 = 2 * (i * (i - 1) // 2 + (n - i) * (n - i + 1) // 2)
        rows = np.array([0, 7, 32])
        ok = True
        Yf, _, _ = oracle.matvec(X.astype(float), np.ones((n, 1)), L1, rows)
        ok &= np.array_equal(Yf[:, 0], e1[rows].astype(float))
        Yi, ov = oracle.matvec_int(X, np.ones((n, 1), np.int64), L1, rows)
        ok &= ov == 0 and np.array_equal(Yi[:, 0], e1[rows])
        s1, s2 = n * (n + 1) // 2, n * (n + 1) * (2 * n + 1) // 6
        e2 = 2 * (n * i * i - 2 * i * s1 + s2)
        Y2, _, _ = oracle.matvec(X.astype(float), np.ones((n, 1)), L2SQ, rows)
        ok &= np.array_equal(Y2[:, 0], e2[rows].astype(float))
        return bool(ok)

    def rhs_columns():
        Xi = g.integers(-9, 9, size=(20, 2)).astype(np.int64)
        Zi = g.integers(-9, 9, size=(20, 3)).astype(np.int64)
        for metric in (L1, L2SQ):
            ex = oracle.exact_matvec(Xi, Zi, metric)
            Y, ov = oracle.matvec_int(Xi, Zi, metric)
            if ov or [[int(v) for v in r] for r in ex] != Y.tolist():
                return False
        return True

    def overflow_flag():
        X = np.array([[-(2 ** 31)], [2 ** 31 - 1]], dtype=np.int64)
        Z = np.array([[2 ** 32], [2 ** 32]], dtype=np.int64)
        return oracle.matvec_int(X, Z, L1)[1] == 2

    def even_p():
        Xi = g.integers(-7, 8, size=(12, 2)).astype(np.int64)
        zi = g.integers(-5, 6, size=12).astype(np.int64)
        for metric, p in ((oracle.L4, 4), (oracle.L6, 6)):
            Y, ov = oracle.matvec_int(Xi, zi[:, None], metric)
            Yf, _, _ = oracle.matvec(Xi.astype(float), zi[:, None].astype(float), metric)
            ex = [int(v) for v in oracle.even_p_query(Xi, zi, p)]
            if ov or Y[:, 0].tolist() != ex or Yf[:, 0].tolist() != [float(v) for v in ex]:
                return False
        return True

    def divergences():
        from scipy.stats import entropy
        P = g.random((6, 3)) + 0.1
        P /= P.sum(axis=1, keepdims=True)
        A = oracle.explicit(P, oracle.KL)
        C = oracle.explicit(P, oracle.CE)
        kl = np.array([[entropy(P[i], P[j]) for j in range(6)] for i in range(6)])
        ce = np.array([[entropy(P[i]) + kl[i, j] for j in range(6)] for i in range(6)])
        return bool(np.allclose(A, kl, rtol=1e-12, atol=1e-15) and np.allclose(C, ce, rtol=1e-12, atol=1e-15))

    def quadratic_forms():
        from scipy.spatial.distance import cdist
        Xq = g.standard_normal((9, 3))
        B = g.standard_normal((3, 3))
        M = B @ B.T + 0.5 * np.eye(3)
        ok = np.allclose(oracle.explicit(Xq, oracle.MAHA2, M=M), cdist(Xq, Xq, "mahalanobis", VI=M) ** 2,
                         rtol=1e-10, atol=1e-12)
        Zq = g.standard_normal((9, 2))
        ok &= np.allclose(oracle.matvec(Xq, Zq, oracle.BILINEAR, M=B)[0], oracle.mahalanobis_query(Xq, Zq, B),
                          rtol=1e-12, atol=1e-12)
        return bool(ok)

    check("exact_rational", exact_rational)
    check("even_p", even_p)
    check("divergences", divergences)
    check("quadratic_forms", quadratic_forms)
    check("structure", structure)
    check("lattice", lattice)
    check("rhs_columns", rhs_columns)
    check("overflow_flag", overflow_flag)
    return failed


def _build_variant(tmp_path, src_text, tag):
    c = tmp_path / ("m_%s.c" % tag)
    so = tmp_path / ("m_%s.so" % tag)
    c.write_text(src_text)
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-std=c11", "-o", str(so), str(c), "-lm"])
    return str(so)


def _with_lib(path):
    saved = oracle._lib
    oracle._lib = None
    real = oracle._LIB
    oracle._LIB = path
    try:
        oracle._load()
        return _pins()
    finally:
        oracle._lib = saved
        oracle._LIB = real


def test_pins_pass_on_real_oracle(oracle_mod):
    assert _pins() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(oracle_mod, tmp_path, name):
    src = open(oracle._SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, "mutation anchor vanished: " + name
    mutated = src.replace(old, new, 1)
    failed = _with_lib(_build_variant(tmp_path, mutated, name))
    assert failed, "no pin caught mutant " + name
