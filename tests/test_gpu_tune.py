"""Tile variants of the l1 pass and the tuner that chooses among them.

Every variant computes the same method (Algorithm 2, Section 2) with a
different tile shape, so integer results must be bit-exact against the exact
oracle for every variant, and float results must meet the same bounds as the
default shape.  The tuner must return one of the variants, keep it for later
queries, and record it in the tuning cache so that a later handle of the same
configuration starts from it.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import L1

from gpu_helpers import U32, bound_ratio, dev, float_errors, method_scale_l1

pytestmark = pytest.mark.gpu
dm = pytest.importorskip("paper_2210_15114_amd")


def _int_data(n, d, b, seed, wide=False):
    g = synth.rng(seed)
    X = g.integers(-2 ** 15, 2 ** 15, size=(n, d)).astype(np.int32)
    Z = np.rint(4096 * g.standard_normal((n, b))).astype(np.int64 if wide else np.int32)
    return X, Z


@pytest.mark.parametrize("b", [1, 3, 8, 33, 64])
def test_every_variant_bit_exact_on_integers(b):
    X, Z = _int_data(9001, 3, b, 900 + b)
    o, ov = oracle.matvec_int(X, Z, L1)
    assert ov == 0
    h = dm.prepare(dev(X), L1)
    Zd = dev(Z)
    for v in range(dm.lib().dm_variant_count()):
        h.set_variant(b, v)
        assert h.get_variant(b) == v
        Y = h.matvec(Zd)
        h.sync()
        assert np.array_equal(Y.cpu().numpy(), o), "variant %d, b=%d" % (v, b)
    h.free()


@pytest.mark.parametrize("b", [1, 16])
def test_every_variant_bit_exact_int64_rhs(b):
    X, Z = _int_data(5003, 2, b, 950 + b, wide=True)
    o, ov = oracle.matvec_int(X, Z, L1)
    assert ov == 0
    h = dm.prepare(dev(X), L1)
    import torch
    for v in range(dm.lib().dm_variant_count()):
        h.set_variant(b, v, torch.int64)
        Y = h.matvec(dev(Z))
        h.sync()
        assert np.array_equal(Y.cpu().numpy(), o), "variant %d, b=%d" % (v, b)
    h.free()


@pytest.mark.parametrize("b", [1, 16, 64])
def test_every_variant_within_float_bounds(b):
    g = synth.rng(990 + b)
    n, d = 7001, 4
    X = g.standard_normal((n, d)).astype(np.float32)
    Z = g.standard_normal((n, b)).astype(np.float32)
    S = method_scale_l1(X, Z, np.arange(n))
    h = dm.prepare(dev(X), L1)
    Zd = dev(Z)
    o = None
    for v in range(dm.lib().dm_variant_count()):
        h.set_variant(b, v)
        Y = h.matvec(Zd).cpu().numpy()
        h.sync()
        e, o = float_errors(X, Z, Y, L1)
        ratio = bound_ratio(np.abs(Y.astype(np.float64) - o), ((8 + 3 * d) * U32 * S))
        print("variant", v, e, ratio)
        assert e["spec"] <= 1e-6 and e["per_row"] <= 1e-6, "variant %d" % v
        assert ratio <= 1.0, "variant %d" % v
    h.free()


def test_tune_keeps_choice_and_writes_cache(tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("DM_TUNE_CACHE", str(cache))
    X, Z = _int_data(20000, 3, 8, 975)
    o, ov = oracle.matvec_int(X, Z, L1)
    h = dm.prepare(dev(X), L1)
    chosen, ms = h.tune(8, reps=3)
    print("chosen", chosen, "ms per pass", ms)
    assert 0 <= chosen < dm.lib().dm_variant_count()
    assert len(ms) == dm.lib().dm_variant_count() and all(t > 0 for t in ms)
    assert ms[chosen] == min(ms)
    assert h.get_variant(8) == chosen
    Y = h.matvec(dev(Z))
    h.sync()
    assert np.array_equal(Y.cpu().numpy(), o)
    h.free()
    lines = cache.read_text().split("\n")
    assert any(line.startswith("dmtune1 ") and line.endswith(" %d" % chosen) for line in lines)
    # a new handle of the same configuration starts from the cached choice
    h2 = dm.prepare(dev(X), L1)
    assert h2.get_variant(8) == chosen
    h2.free()
