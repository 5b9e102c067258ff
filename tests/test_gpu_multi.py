"""GPU parity of the multi-dataset query (one captured graph over many point
sets of uneven n and d, float and integer mixed) against per-dataset results
and the CPU oracle.  Integer datasets are bit-exact; float datasets meet the
same bounds as the single-dataset path.  The graph is replayed several times
with different right-hand sides and eager work in between; every replay is
checked."""
import numpy as np
import pytest

import oracle
import synth
from oracle import L1

from gpu_helpers import U32, dev, float_errors, method_scale_l1

pytestmark = pytest.mark.gpu
dm = pytest.importorskip("paper_2210_15114_amd")


def _sets(seed, count=14):
    g = synth.rng(seed)
    specs = []
    for i in range(count):
        n = int(g.choice([1, 7, 300, 1025, 4096, 9000]))
        d = int(g.choice([1, 3, 16]))
        is_int = bool(i % 2)
        if is_int:
            X = g.integers(-2 ** 15, 2 ** 15, size=(n, d)).astype(np.int32)
        else:
            X = g.standard_normal((n, d)).astype(np.float32)
        specs.append(X)
    return specs


def _rhs(X, b, g):
    n = X.shape[0]
    if X.dtype == np.int32:
        return np.rint(4096 * g.standard_normal((n, b))).astype(np.int32)
    return g.standard_normal((n, b)).astype(np.float32)


def _check(X, Z, Y):
    if X.dtype == np.int32:
        o, ov = oracle.matvec_int(X, Z, L1)
        assert ov == 0
        assert np.array_equal(Y, o)
    else:
        e, o = float_errors(X, Z, Y, L1)
        S = method_scale_l1(X, Z, np.arange(X.shape[0]))
        err = np.abs(Y.astype(np.float64) - o)
        assert e["spec"] <= 1e-6
        assert (err <= (8 + 3 * X.shape[1]) * U32 * S + 1e-30).all()


@pytest.mark.parametrize("b", [1, 8, 64])
def test_multi_matches_oracle_and_replays(b):
    import torch
    Xs = _sets(900 + b)
    h = dm.prepare_multi([dev(X) for X in Xs])
    g = synth.rng(77 + b)
    for rep in range(3):
        Zs = [_rhs(X, b, g) for X in Xs]
        Zd = [dev(Z) for Z in Zs]
        outs = h.matvec(Zd)
        h.sync()
        junk = torch.randn(1000, device="cuda").sum().item()    # eager work between replays
        assert np.isfinite(junk)
        for X, Z, Y in zip(Xs, Zs, outs):
            _check(X, Z, Y.cpu().numpy())


def test_multi_equals_single_dataset_integers():
    Xs = [X for X in _sets(1234) if X.dtype == np.int32]
    g = synth.rng(5)
    Zs = [_rhs(X, 8, g) for X in Xs]
    h = dm.prepare_multi([dev(X) for X in Xs])
    outs = [o.cpu().numpy() for o in h.matvec([dev(Z) for Z in Zs])]
    h.sync()
    for X, Z, Y in zip(Xs, Zs, outs):
        hs = dm.prepare(dev(X), L1)
        Ys = hs.matvec(dev(Z)).cpu().numpy()
        hs.sync()
        assert np.array_equal(Y, Ys)


def test_multi_rejects_wrong_use():
    X = np.zeros((10, 2), np.float32)
    h = dm.prepare_multi([dev(X)])
    single = dm.prepare(dev(X), L1)
    import ctypes
    assert dm.lib().dm_matvec(h._ptr, ctypes.c_void_p(1), dm.F32, 1, ctypes.c_void_p(2), None) == dm.ERR_STATE
    z = (ctypes.c_void_p * 1)(1)
    o = (ctypes.c_void_p * 1)(2)
    assert dm.lib().dm_matvec_multi(single._ptr, z, 1, o, None) == dm.ERR_STATE


@pytest.mark.parametrize("b", [1, 8, 40])
def test_every_tile_variant_matches_the_oracle(b):
    """Each tile variant of the many-dataset pass (set explicitly), on the
    same datasets: integer sets bit-exact, float sets within the bounds; then
    the tuner times them all and keeps one."""
    Xs = _sets(1300 + b)
    g = synth.rng(1310 + b)
    Zs = [_rhs(X, b, g) for X in Xs]
    h = dm.prepare_multi([dev(X) for X in Xs])
    Zd = [dev(Z) for Z in Zs]
    count = dm.lib().dm_multi_variant_count()
    assert count >= 2
    for v in range(count):
        h.set_variant(b, v)
        assert h.get_variant(b) == v
        outs = h.matvec(Zd)
        h.sync()
        for X, Z, O in zip(Xs, Zs, outs):
            _check(X, Z, O.cpu().numpy())
    v, ms, outs = h.tune(Zd, reps=2)
    h.sync()
    assert 0 <= v < count and len(ms) == count and min(ms) > 0
    assert h.get_variant(b) == v
    for X, Z, O in zip(Xs, Zs, outs):
        _check(X, Z, O.cpu().numpy())
    h.free()
