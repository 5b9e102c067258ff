"""The sort-free family of Appendix A on the GPU: l_p^p for even p (Algorithm
5 with the binomial coefficients restored), the KL divergence (Algorithm 4),
cross entropy, the squared Mahalanobis distance and the bilinear form of
Algorithms 8 and 9.

Integer data (even p) is bit-exact against the exact oracle.  Float data is
checked against the FP64 oracle on the same FP32 inputs: normalised error
<= 1e-6, and per output

    |y - o| <= 2 u32 |o| + (n + d + 4p + 16) u64 S,

where the first term is the one rounding of the FP64 result to FP32 and S
bounds the magnitude of every term the FP64 moments and the per-point sums
form (for even p: sum_k sum_t C(p, t) |x~_ik|^(p-t) sum_j |z_j| |x~_jk|^t
with x~ = x - c, c the midpoint of each coordinate's range).
"""
from math import comb

import numpy as np
import pytest

import oracle
import synth
from oracle import metrics

from gpu_helpers import U32, bound_ratio, dev

pytestmark = pytest.mark.gpu
dm = pytest.importorskip("paper_2210_15114_amd")

U64 = 2.0 ** -53
EVEN = {4: oracle.L4, 6: oracle.L6}


def _centre(X):
    X = X.astype(np.float64)
    return 0.5 * (X.min(axis=0) + X.max(axis=0))


# Each scale function returns S on the given rows (m x b).
def _scale_even(p):
    def f(X, Z, r):
        Xc = np.abs(X.astype(np.float64) - _centre(X))
        Z = np.abs(Z.astype(np.float64)).reshape(X.shape[0], -1)
        S = np.zeros((r.size, Z.shape[1]))
        for k in range(X.shape[1]):
            xk = Xc[:, k]
            for t in range(p + 1):
                S += comb(p, t) * (xk[r] ** (p - t))[:, None] * ((xk ** t) @ Z)[None, :]
        return S
    return f


def _scale_log(entropy):
    def f(X, Z, r):
        X = X.astype(np.float64)
        Z = np.abs(Z.astype(np.float64)).reshape(X.shape[0], -1)
        L = np.abs(np.log(X))
        S = X[r] @ (L.T @ Z)
        if entropy:
            S += (X[r] * L[r]).sum(axis=1)[:, None] * Z.sum(axis=0)[None, :]
        return S
    return f


def _scale_quad(M, centred):
    def f(X, Z, r):
        X = X.astype(np.float64)
        if centred:
            X = X - _centre(X)
        A = np.abs(X)
        Z = np.abs(Z.astype(np.float64)).reshape(X.shape[0], -1)
        Ma = np.abs(M)
        S = A[r] @ ((Ma + Ma.T) @ (A.T @ Z))
        if centred:
            q = np.einsum("ik,kl,il->i", A, Ma, A)
            S += q[r][:, None] * Z.sum(axis=0)[None, :] + (q @ Z)[None, :]
        return S
    return f


def _sample_rows(n):
    """Every row of a small problem; else 200 seeded rows plus the first and
    last point of every apply workgroup size (32 .. 256 points) near the ends."""
    if n <= 2100:
        return np.arange(n)
    edges = [0, n - 1]
    for t in (32, 64, 128, 256):
        edges += [t - 1, t, n - 1 - (n % t)]
    return synth.subsample_rows(n, 200, 9999 + n, extra=edges)


def _check_float(X, Z, Y, metric, scale, M=None, rows=None, p=0):
    n, d = X.shape
    Z64 = Z.astype(np.float64).reshape(n, -1)
    r = _sample_rows(n) if rows is None else np.asarray(rows)
    o, rn, ad = oracle.matvec(X.astype(np.float64), Z64, metric, r, M=M)
    Yr = np.asarray(Y, dtype=np.float64).reshape(n, -1)[r]
    e = metrics.errors(Yr, o, rn, ad, Z64, metrics.frob_from_rows(rn, n))
    err = np.abs(Yr - o)
    bound = 2 * U32 * np.abs(o) + (n + d + 4 * p + 16) * U64 * scale(X, Z, r)
    ratio = bound_ratio(err, bound)
    print("metric", metric, "errors", e, "bound-ratio", ratio)
    assert e["spec"] <= 1e-6
    assert ratio <= 1.0


def _query(X, Z, metric, M=None):
    h = dm.prepare(dev(X), metric, M=M)
    Y = h.matvec(dev(Z))
    h.sync()
    out = Y.cpu().numpy()
    h.free()
    return out


# ---------------------------------------------------------------------------
# even p
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("p,b,n,d", [(4, 1, 3001, 3), (4, 5, 3001, 37), (4, 64, 2049, 3), (6, 1, 4097, 2),
                                     (6, 8, 3001, 25), (6, 33, 1000, 3)])
def test_even_p_integer_bit_exact(p, b, n, d):
    g = synth.rng(9000 + 10 * p + b)
    lim = 100 if p == 4 else 30
    X = g.integers(-lim, lim + 1, size=(n, d)).astype(np.int32)
    Z = np.rint((256 if p == 4 else 16) * g.standard_normal((n, b))).astype(np.int32)
    o, ov = oracle.matvec_int(X, Z, EVEN[p])
    assert ov == 0
    h = dm.prepare(dev(X), EVEN[p])
    Y = h.matvec(dev(Z))
    h.sync()
    assert np.array_equal(Y.cpu().numpy(), o)
    Y64 = h.matvec(dev(Z.astype(np.int64)))
    h.sync()
    assert np.array_equal(Y64.cpu().numpy(), o)
    h.free()


def test_even_p_integer_offset_data_is_exact():
    # large coordinates with a small spread: the moments of x - c stay small
    g = synth.rng(9100)
    n, d, b = 2500, 4, 3
    X = (10 ** 9 + g.integers(0, 50, size=(n, d))).astype(np.int64)
    Z = g.integers(-500, 501, size=(n, b)).astype(np.int64)
    o, ov = oracle.matvec_int(X, Z, oracle.L6)
    assert ov == 0
    Y = _query(X, Z, oracle.L6)
    assert np.array_equal(Y, o)


def test_even_p_integer_overflow_guard_trips():
    X = np.array([[0], [2 ** 16]], dtype=np.int32)
    Z = np.array([[2 ** 20], [1]], dtype=np.int32)       # ||z||_1 range^4 >= 2^84
    h = dm.prepare(dev(X), oracle.L4)
    h.matvec(dev(Z))
    with pytest.raises(dm.DMError) as ex:
        h.sync()
    assert ex.value.status == dm.ERR_OVERFLOW
    h.free()


@pytest.mark.parametrize("p,b,n,d,dist", [(4, 1, 20001, 5, "normal"), (4, 16, 4099, 37, "uniform"),
                                          (4, 64, 4099, 3, "normal"), (6, 1, 20001, 3, "uniform"),
                                          (6, 8, 4099, 17, "normal"), (6, 64, 2053, 5, "offset")])
def test_even_p_float_within_bounds(p, b, n, d, dist):
    g = synth.rng(9200 + 10 * p + b)
    if dist == "normal":
        X = g.standard_normal((n, d)).astype(np.float32)
    elif dist == "uniform":
        X = g.random((n, d)).astype(np.float32)
    else:                                                 # far from the origin
        X = (100.0 + g.random((n, d))).astype(np.float32)
    Z = g.standard_normal((n, b)).astype(np.float32)
    Y = _query(X, Z, EVEN[p])
    _check_float(X, Z, Y, EVEN[p], _scale_even(p), p=p)


def test_even_p_float64_input_is_rounded_once():
    g = synth.rng(9300)
    X64 = g.standard_normal((3000, 4))
    Z = g.standard_normal((3000, 2)).astype(np.float32)
    Y = _query(X64, Z, oracle.L4)
    X32 = X64.astype(np.float32)
    _check_float(X32, Z, Y, oracle.L4, _scale_even(4), p=4)


def test_single_point_and_single_coordinate():
    for metric in (oracle.L4, oracle.L6):
        Y = _query(np.array([[3.5]], dtype=np.float32), np.array([[2.0]], dtype=np.float32), metric)
        assert Y.shape == (1, 1) and Y[0, 0] == 0.0
        Yi = _query(np.array([[7]], dtype=np.int32), np.array([[5]], dtype=np.int32), metric)
        assert Yi[0, 0] == 0


# ---------------------------------------------------------------------------
# KL divergence and cross entropy
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("metric", [oracle.KL, oracle.CE])
@pytest.mark.parametrize("b,n,d,alpha", [(1, 20001, 8, 1.0), (3, 4099, 70, 0.5), (64, 2049, 16, 2.0)])
def test_divergences_within_bounds(metric, b, n, d, alpha):
    X = synth.simplex_points(n, d, 9400 + b + d, alpha=alpha)
    Z = synth.rhs_normal(n, b, 9500 + b)
    Y = _query(X, Z, metric)
    _check_float(X, Z, Y, metric, _scale_log(metric == oracle.KL))


def test_kl_of_unnormalised_positive_points():
    g = synth.rng(9600)
    X = (0.01 + 3 * g.random((5000, 6))).astype(np.float32)
    Z = g.standard_normal((5000, 2)).astype(np.float32)
    Y = _query(X, Z, oracle.KL)
    _check_float(X, Z, Y, oracle.KL, _scale_log(True))


@pytest.mark.parametrize("metric", [oracle.KL, oracle.CE])
def test_divergence_domain_is_checked(metric):
    X = synth.simplex_points(100, 4, 9700)
    X[17, 2] = 0.0
    with pytest.raises(dm.DMError) as ex:
        dm.prepare(dev(X), metric)
    assert ex.value.status == dm.ERR_ARG
    X[17, 2] = -0.25
    with pytest.raises(dm.DMError):
        dm.prepare(dev(X), metric)


def test_kl_handle_refuses_lowrank():
    import torch
    X = synth.simplex_points(500, 4, 9710)
    h = dm.prepare(dev(X), oracle.KL)
    om = torch.zeros((500, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(dm.DMError) as ex:
        h.lowrank(4, om, iters=2)
    assert ex.value.status == dm.ERR_STATE
    h.free()


# ---------------------------------------------------------------------------
# squared Mahalanobis distance and the bilinear form
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("b,n,d,kind", [(1, 20001, 8, "spd"), (5, 4099, 37, "general"), (64, 2049, 70, "spd")])
def test_mahalanobis_within_bounds(b, n, d, kind):
    g = synth.rng(9800 + b)
    X = (g.standard_normal((n, d)) + 3.0).astype(np.float32)
    Z = g.standard_normal((n, b)).astype(np.float32)
    M = synth.square_matrix(d, 9810 + d, kind)
    Y = _query(X, Z, oracle.MAHA2, M=M)
    _check_float(X, Z, Y, oracle.MAHA2, _scale_quad(M, True), M=M)


def test_mahalanobis_identity_matches_l2sq_oracle():
    g = synth.rng(9820)
    X = g.standard_normal((3000, 6)).astype(np.float32)
    Z = g.standard_normal((3000, 2)).astype(np.float32)
    Y = _query(X, Z, oracle.MAHA2, M=np.eye(6))
    _check_float(X, Z, Y, oracle.L2SQ, _scale_quad(np.eye(6), True))


@pytest.mark.parametrize("b,n,d", [(1, 20001, 8), (7, 4099, 37), (64, 2049, 70)])
def test_bilinear_within_bounds(b, n, d):
    g = synth.rng(9900 + b)
    X = g.standard_normal((n, d)).astype(np.float32)
    Z = g.standard_normal((n, b)).astype(np.float32)
    M = synth.square_matrix(d, 9910 + d, "general")
    Y = _query(X, Z, oracle.BILINEAR, M=M)
    _check_float(X, Z, Y, oracle.BILINEAR, _scale_quad(M, False), M=M)


def test_matrix_metric_needs_its_matrix():
    X = np.zeros((10, 3), dtype=np.float32)
    with pytest.raises(dm.DMError):
        dm.prepare(dev(X), oracle.MAHA2)
    with pytest.raises(dm.DMError) as ex:
        dm.prepare(dev(X), oracle.BILINEAR, M=np.full((3, 3), np.nan))
    assert ex.value.status == dm.ERR_NONFINITE


# ---------------------------------------------------------------------------
# full size: n = 2^20 points, d = 64, sampled rows
# ---------------------------------------------------------------------------
def test_full_size_sampled_rows():
    n, d = 1 << 20, 64
    X = synth.uniform_points(n, d, 9950)
    Z = synth.rhs_normal(n, 64, 9951)
    rows = synth.subsample_rows(n, 6, 9952, extra=[0, n - 1])
    Xd, Zd = dev(X), dev(Z)
    h = dm.prepare(Xd, oracle.L4)
    Y = h.matvec(Zd)
    h.sync()
    _check_float(X, Z, Y.cpu().numpy(), oracle.L4, _scale_even(4), rows=rows, p=4)
    h.free()
    del Y
    P = synth.simplex_points(n, d, 9953)
    z1 = Z[:, :1].copy()
    h = dm.prepare(dev(P), oracle.KL)
    y = h.matvec(dev(z1))
    h.sync()
    _check_float(P, z1, y.cpu().numpy(), oracle.KL, _scale_log(True), rows=rows)
    h.free()


# ---------------------------------------------------------------------------
# more coordinates than one workgroup spans (256 in the narrow moments)
# ---------------------------------------------------------------------------
def test_many_coordinates():
    g = synth.rng(9960)
    n = 3001
    X = g.integers(-20, 21, size=(n, 260)).astype(np.int32)
    Z = g.integers(-9, 10, size=(n, 4)).astype(np.int32)
    o, ov = oracle.matvec_int(X, Z, oracle.L4)
    assert ov == 0
    assert np.array_equal(_query(X, Z, oracle.L4), o)
    P = synth.simplex_points(n, 300, 9961)
    Zf = synth.rhs_normal(n, 2, 9962)
    _check_float(P, Zf, _query(P, Zf, oracle.KL), oracle.KL, _scale_log(True))
    Xf = g.standard_normal((n, 300)).astype(np.float32)
    Zw = synth.rhs_normal(n, 16, 9963)
    _check_float(Xf, Zw, _query(Xf, Zw, oracle.L4), oracle.L4, _scale_even(4), p=4)


# ---------------------------------------------------------------------------
# the matrix-core kernels of the single-moment forms: moments at d % 4 == 0
# with one column per lane for 4 <= b <= 16, two for even b <= 32 and four for
# b % 4 == 0 (others take the vector moments); the point pass at b >= 4
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("metric,b,n,d", [(oracle.KL, 20, 3001, 12), (oracle.MAHA2, 33, 2501, 37),
                                          (oracle.BILINEAR, 48, 4099, 64), (oracle.CE, 64, 2049, 70),
                                          (oracle.MAHA2, 64, 4099, 132), (oracle.KL, 40, 2053, 8),
                                          (oracle.KL, 16, 3001, 64), (oracle.MAHA2, 4, 2501, 36),
                                          (oracle.BILINEAR, 13, 4099, 20), (oracle.CE, 30, 2049, 68),
                                          (oracle.MAHA2, 32, 4099, 132), (oracle.BILINEAR, 9, 1031, 8),
                                          (oracle.KL, 25, 2053, 16)])
def test_matrix_core_shapes(metric, b, n, d):
    g = synth.rng(9970 + b + d)
    M = None
    if metric in (oracle.KL, oracle.CE):
        X = synth.simplex_points(n, d, 9971 + d)
        scale = _scale_log(metric == oracle.KL)
    else:
        X = (g.standard_normal((n, d)) + 2.0).astype(np.float32)
        M = synth.square_matrix(d, 9972 + d, "spd" if metric == oracle.MAHA2 else "general")
        scale = _scale_quad(M, metric == oracle.MAHA2)
    Z = g.standard_normal((n, b)).astype(np.float32)
    Y = _query(X, Z, metric, M=M)
    _check_float(X, Z, Y, metric, scale, M=M)


@pytest.mark.parametrize("b", [64, 30, 16])
def test_matrix_core_moments_with_unaligned_z(b):
    """Z 4 bytes past a 16-byte boundary: b = 64 (four columns per lane) and
    b = 30 (two) need 16- and 8-byte rows and take the vector moments, b = 16
    (one column per lane) stays on matrix cores."""
    import torch
    n, d = 3001, 16
    X = synth.simplex_points(n, d, 9980)
    Z = synth.rhs_normal(n, b, 9981)
    flat = torch.empty(n * b + 1, dtype=torch.float32, device="cuda")
    Zd = flat[1:].view(n, b)                     # 4 bytes past a 16-byte boundary
    Zd.copy_(torch.from_numpy(Z))
    assert Zd.data_ptr() % 16 != 0 and Zd.data_ptr() % 8 != 0
    h = dm.prepare(dev(X), oracle.KL)
    Y = h.matvec(Zd)
    h.sync()
    _check_float(X, Z, Y.cpu().numpy(), oracle.KL, _scale_log(True))
    h.free()


@pytest.mark.parametrize("p,b,n,d,aligned", [(4, 40, 3001, 70, True), (6, 48, 2053, 9, True),
                                              (4, 64, 3001, 33, False), (6, 20, 4099, 64, True),
                                              (4, 16, 2501, 40, False), (6, 30, 3001, 12, False),
                                              (4, 6, 3001, 70, True), (6, 13, 2049, 66, True)])
def test_even_p_matrix_core_shapes(p, b, n, d, aligned):
    import torch
    g = synth.rng(9990 + p + b + d)
    X = (g.standard_normal((n, d)) + 5.0).astype(np.float32)
    Z = g.standard_normal((n, b)).astype(np.float32)
    if aligned:
        Zd = dev(Z)
    else:
        flat = torch.empty(n * b + 1, dtype=torch.float32, device="cuda")
        Zd = flat[1:].view(n, b)
        Zd.copy_(torch.from_numpy(Z))
        assert Zd.data_ptr() % 16 != 0
    h = dm.prepare(dev(X), EVEN[p])
    Y = h.matvec(Zd)
    h.sync()
    _check_float(X, Z, Y.cpu().numpy(), EVEN[p], _scale_even(p), p=p)
    h.free()


@pytest.mark.parametrize("n", [1, 5, 17, 130])
@pytest.mark.parametrize("metric", [oracle.L4, oracle.L6, oracle.KL, oracle.MAHA2])
def test_matrix_core_paths_at_tiny_n(metric, n):
    # fewer points than one 4-row step, one 16-point tile or one 128-point workgroup
    g = synth.rng(9995 + n + metric)
    d, b = 8, 64
    M = None
    if metric == oracle.KL:
        X = synth.simplex_points(n, d, 9996 + n)
        scale = _scale_log(True)
    else:
        X = (g.standard_normal((n, d)) + 1.0).astype(np.float32)
        if metric == oracle.MAHA2:
            M = synth.square_matrix(d, 9997, "spd")
            scale = _scale_quad(M, True)
        else:
            scale = _scale_even(4 if metric == oracle.L4 else 6)
    Z = g.standard_normal((n, b)).astype(np.float32)
    Y = _query(X, Z, metric, M=M)
    p = {oracle.L4: 4, oracle.L6: 6}.get(metric, 0)
    if n == 1 and metric == oracle.KL:
        # D(x || x) = 0, reached through -H(x) sum z - sum_k x(k) log x(k) z: FP64 cancellation only
        r = np.arange(1)
        assert np.all(np.abs(Y) <= (d + 16) * U64 * scale(X, Z, r))
    elif n == 1:
        assert np.all(Y == 0.0)                     # the centred coordinates are exactly 0
    else:
        _check_float(X, Z, Y, metric, scale, M=M, p=p)


def test_full_size_wide_blocks_sampled_rows():
    # the benchmark's sort-free shapes at b = 64: n = 2^20 points, d = 64
    n, d, b = 1 << 20, 64, 64
    Xm, _ = synth.workload2(n, d, 1)
    P = synth.simplex_points(n, d, synth.seeds(2)["X"] + 11)
    M = synth.square_matrix(d, synth.seeds(2)["X"] + 12, "spd")
    Z = synth.rhs_normal(n, b, synth.seeds(2)["Z"] + 20 + b)
    rows = synth.subsample_rows(n, 3, 9998, extra=[0, n - 1])
    Zd = dev(Z)
    for metric, X, Mm, scale, p in ((oracle.L6, Xm, None, _scale_even(6), 6),
                                    (oracle.KL, P, None, _scale_log(True), 0),
                                    (oracle.MAHA2, Xm, M, _scale_quad(M, True), 0)):
        h = dm.prepare(dev(X), metric, M=Mm)
        Y = h.matvec(Zd)
        h.sync()
        _check_float(X, Z, Y.cpu().numpy(), metric, scale, M=Mm, rows=rows, p=p)
        h.free()
        del Y


# ---------------------------------------------------------------------------
# a non-finite right-hand side raises DM_ERR_NONFINITE on every path: the
# totals kernel, and the single-moment forms on matrix cores, which sum z
# inside their moments kernel and check the column sums
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("metric,b,d", [(oracle.KL, 64, 8), (oracle.MAHA2, 64, 12), (oracle.BILINEAR, 48, 16),
                                        (oracle.CE, 64, 4), (oracle.L4, 64, 5), (oracle.KL, 1, 8),
                                        (oracle.KL, 16, 8), (oracle.MAHA2, 6, 12), (oracle.CE, 26, 4),
                                        (oracle.L6, 8, 5), (oracle.L4, 20, 7)])
@pytest.mark.parametrize("case", ["inf", "nan", "both_infs"])
def test_nonfinite_rhs_flagged(metric, b, d, case):
    g = synth.rng(9990 + b + d)
    n = 3001
    M = None
    if metric in (oracle.KL, oracle.CE):
        X = synth.simplex_points(n, d, 9991 + d)
    else:
        X = (g.standard_normal((n, d)) + 2.0).astype(np.float32)
        if metric in (oracle.MAHA2, oracle.BILINEAR):
            M = synth.square_matrix(d, 9992 + d, "spd" if metric == oracle.MAHA2 else "general")
    Z = g.standard_normal((n, b)).astype(np.float32)
    Zbad = Z.copy()
    if case == "inf":
        Zbad[1234, b - 1] = np.inf
    elif case == "nan":
        Zbad[0, 0] = np.nan
    else:
        Zbad[7, b // 2] = np.inf
        Zbad[n - 1, b // 2] = -np.inf
    h = dm.prepare(dev(X), metric, M=M)
    h.matvec(dev(Zbad if b > 1 else Zbad[:, 0].copy()))
    with pytest.raises(dm.DMError) as ei:
        h.sync()
    assert ei.value.status == dm.ERR_NONFINITE
    Y = h.matvec(dev(Z if b > 1 else Z[:, 0].copy()))
    h.sync()
    Y = Y.cpu().numpy()
    h.free()
    assert np.all(np.isfinite(Y))
    Yref = _query(X, Z if b > 1 else Z[:, 0].copy(), metric, M=M)
    assert np.array_equal(Y, Yref)
