"""Total variation products (the TV theorem of Appendix A.3): the l1 path with
the result halved, on distributions given as probability vectors.  Float
results against the FP64 oracle's TV matrix within half the l1 bounds;
integer data is rejected."""
import numpy as np
import pytest

import oracle
import synth

from gpu_helpers import U32, bound_ratio, dev, float_errors, method_scale_l1

pytestmark = pytest.mark.gpu
dm = pytest.importorskip("paper_2210_15114_amd")


@pytest.mark.parametrize("b", [1, 8])
def test_tv_matches_oracle(b):
    g = synth.rng(5050 + b)
    n, d = 3001, 10
    X = g.dirichlet(np.ones(d), size=n).astype(np.float32)
    Z = g.standard_normal((n, b)).astype(np.float32)
    h = dm.prepare(dev(X), dm.TV)
    Y = h.matvec(dev(Z)).cpu().numpy()
    h.sync()
    h.free()
    e, o = float_errors(X, Z, Y, oracle.TV)
    S = method_scale_l1(X, Z, np.arange(n))
    ratio = bound_ratio(np.abs(Y.reshape(n, -1).astype(np.float64) - o), (0.5 * (8 + 3 * d) * U32 * S))
    print("tv errors", e, "bound-ratio", ratio)
    assert e["spec"] <= 1e-6 and ratio <= 1.0


def test_tv_single_column_in_groups_is_half_of_l1():
    # n = 2^20 + 5 points of d = 20 coordinates: the single-column buffer holds
    # 15 coordinates, so the query runs in 2 groups.  Halving is exact, but two
    # float runs of the chained scan may differ in the last bits (the carries
    # combine a timing-dependent set of predecessor records), so the relation
    # is checked to a few FP32 units of the largest output
    g = synth.rng(5070)
    n, d = (1 << 20) + 5, 20
    X = g.dirichlet(np.ones(d), size=n).astype(np.float32)
    z = g.standard_normal(n).astype(np.float32)
    Xd, zd = dev(X), dev(z)
    ht, hl = dm.prepare(Xd, dm.TV), dm.prepare(Xd, dm.L1)
    yt = ht.matvec(zd).cpu().numpy()
    yl = hl.matvec(zd).cpu().numpy()
    ht.sync()
    hl.sync()
    err = np.abs(yt.astype(np.float64) - 0.5 * yl.astype(np.float64))
    assert err.max() <= 2 * d * U32 * np.abs(yl).max()
    rows = np.concatenate([np.arange(3), g.choice(n, 20, replace=False), np.arange(n - 3, n)])
    e, o = float_errors(X, z, yt, oracle.TV, rows)
    assert e["spec"] <= 1e-6 and e["per_row"] <= 1e-6


def test_tv_rejects_integer_points():
    X = np.ones((10, 3), dtype=np.int32)
    with pytest.raises(dm.DMError) as ex:
        dm.prepare(dev(X), dm.TV)
    assert ex.value.status == dm.ERR_DTYPE
