"""dm_matvec_static: the query with its scratch in the library's static device
array instead of the workspace.  Two calls in a row, the second on a smaller
input (so that whatever the first call left in the array must not leak into
the second), each checked against dm_matvec on the same handle and inputs:
bit-exact on integer data, and on float data within the l1 method's FP32
bound of each other and of the FP64 oracle.  Shapes beyond the array are
refused with DM_ERR_ARG."""
import numpy as np
import pytest

import oracle
import synth
from oracle import L1, L2SQ

from gpu_helpers import U32, bound_ratio, dev, float_errors, method_scale_l1

pytestmark = pytest.mark.gpu
dm = pytest.importorskip("paper_2210_15114_amd")


def _both(h, Z):
    import torch
    Zd = dev(Z)
    Zm = Zd if Zd.dim() == 2 else Zd.unsqueeze(1)
    odt = torch.int64 if h.is_int else torch.float32
    o1 = torch.empty((h.n, Zm.shape[1]), dtype=odt, device="cuda")
    o2 = torch.full_like(o1, 7)       # garbage the static call must overwrite
    h.matvec(Zm, out=o1)
    h.matvec_static(Zm, out=o2)
    h.sync()
    return o1.cpu().numpy(), o2.cpu().numpy()


def test_static_integer_two_calls_bit_exact():
    g = synth.rng(9301)
    for n, d, b in ((300001, 6, 64), (70001, 4, 8)):
        X = g.integers(-5000, 5000, size=(n, d)).astype(np.int32)
        Z = g.integers(-3000, 3000, size=(n, b)).astype(np.int32)
        h = dm.prepare(dev(X), L1)
        y1, y2 = _both(h, Z)
        h.free()
        assert np.array_equal(y1, y2), (n, d, b)
        rows = synth.subsample_rows(n, 24, 9302 + n)
        o, ov = oracle.matvec_int(X, Z, L1, rows)
        assert ov == 0 and np.array_equal(y2[rows], o)


def test_static_float_two_calls_within_bounds():
    g = synth.rng(9311)
    for n, d, b in (((1 << 20) + 5, 5, 64), (100003, 7, 1)):
        X = g.standard_normal((n, d)).astype(np.float32)
        Z = g.standard_normal((n, b)).astype(np.float32)
        if b == 1:
            Z = Z[:, 0].copy()
        h = dm.prepare(dev(X), L1)
        y1, y2 = _both(h, Z)
        h.free()
        rows = synth.subsample_rows(n, 32, 9312 + n)
        S = method_scale_l1(X, Z, rows)
        bound = (8 + 3 * d) * U32 * S
        assert bound_ratio(y1.reshape(n, -1)[rows] - y2.reshape(n, -1)[rows], 2 * bound) <= 1.0
        e, o = float_errors(X, Z, y2, L1, rows)
        assert e["spec"] <= 1e-6 and e["per_row"] <= 1e-6, e
        assert bound_ratio(y2.reshape(n, -1)[rows] - o, bound) <= 1.0


def test_static_l2sq_and_odd_p():
    g = synth.rng(9321)
    X = g.standard_normal((50001, 12)).astype(np.float32)
    Z = g.standard_normal((50001, 32)).astype(np.float32)
    for metric in (L2SQ, dm.L3):
        h = dm.prepare(dev(X), metric)
        y1, y2 = _both(h, Z)
        h.free()
        rows = synth.subsample_rows(X.shape[0], 16, 9322)
        e1, _ = float_errors(X, Z, y1, metric, rows)
        e2, _ = float_errors(X, Z, y2, metric, rows)
        assert e1["spec"] <= 1e-6 and e2["spec"] <= 1e-6, (e1, e2)


def test_static_fixed_order_paths_are_bitwise_equal():
    """Queries whose every sum has a fixed order give the same bits through
    either entry point: l2 squared at d = 128, b = 64 (the X^T Z kernel that
    also forms the totals), and the KL divergence on matrix cores (totals
    summed inside the moments kernel); the second call of each is smaller."""
    for metric, shapes in ((L2SQ, ((8192, 128, 64), (4096, 128, 64))),
                           (oracle.KL, ((3001, 8, 64), (1000, 8, 48)))):
        for n, d, b in shapes:
            g = synth.rng(9400 + n + b)
            if metric == oracle.KL:
                X = synth.simplex_points(n, d, 9401 + n)
            else:
                X = g.standard_normal((n, d)).astype(np.float32)
            Z = g.standard_normal((n, b)).astype(np.float32)
            h = dm.prepare(dev(X), metric)
            y1, y2 = _both(h, Z)
            h.free()
            assert np.array_equal(y1, y2), (metric, n, d, b)


def test_static_refuses_shapes_beyond_the_array():
    """n = 2^23 points at b = 64: the pass's look-back records alone (two
    records of 64 double-float pairs per 512-rank tile) exceed 32 MiB."""
    import torch
    n = 1 << 23
    X = np.arange(n, dtype=np.float32).reshape(n, 1)
    h = dm.prepare(dev(X), L1)
    Z = torch.zeros((n, 64), dtype=torch.float32, device="cuda")
    out = torch.empty((n, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(dm.DMError) as ex:
        h.matvec_static(Z, out=out)
    assert ex.value.status == dm.ERR_ARG
    h.free()
