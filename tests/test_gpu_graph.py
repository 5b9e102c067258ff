"""The single-dataset query replayed from captured hipGraphs: the first call
with given (Z, Out, b) records the query, later ones replay it.  Every replay
is checked (integer data: bit-exact against the exact oracle), with new
right-hand-side values written into the same Z between replays, eager work
and synchronisations in between, more argument sets than the handle keeps
graphs (eviction), and the eager path (profiling on) agreeing bit for bit."""
import numpy as np
import pytest

import oracle
import synth
from oracle import L1

from gpu_helpers import dev

pytestmark = pytest.mark.gpu
dm = pytest.importorskip("paper_2210_15114_amd")


@pytest.mark.parametrize("metric", [L1, dm.L3, dm.L2SQ, dm.L4])
def test_replays_match_the_oracle(metric):
    import torch
    g = synth.rng(8100 + metric)
    n, d, b = 20001, 5, 8
    lim = 200 if metric in (dm.L3, dm.L4) else 3000
    X = g.integers(-lim, lim, size=(n, d)).astype(np.int32)
    h = dm.prepare(dev(X), metric)
    Zd = torch.empty((n, b), dtype=torch.int32, device="cuda")
    outs = [torch.empty((n, b), dtype=torch.int64, device="cuda") for _ in range(6)]
    rows = synth.subsample_rows(n, 40, 8101)
    for rep in range(9):
        Z = g.integers(-100, 100, size=(n, b)).astype(np.int32)
        Zd.copy_(torch.from_numpy(Z))
        o = outs[rep % len(outs)]          # 6 output buffers: graphs get evicted and recorded again
        h.matvec(Zd, out=o)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 16, device="cuda").sum()    # eager work between replays
        h.sync()
        ref, ov = oracle.matvec_int(X, Z, metric, rows)
        assert ov == 0
        assert np.array_equal(o.cpu().numpy()[rows], ref), ("replay", rep)
        del junk
    # the eager path (profiling on) gives the same integers
    h.profile(True)
    o2 = torch.empty_like(outs[0])
    h.matvec(Zd, out=o2)
    h.sync()
    h.profile(False)
    h.matvec(Zd, out=outs[0])
    h.sync()
    assert torch.equal(o2, outs[0])
    h.free()


def test_float_replays_within_bounds():
    import torch
    from gpu_helpers import float_errors
    g = synth.rng(8200)
    n, d, b = 50001, 7, 16
    X = g.standard_normal((n, d)).astype(np.float32)
    h = dm.prepare(dev(X), L1)
    Zd = torch.empty((n, b), dtype=torch.float32, device="cuda")
    out = torch.empty((n, b), dtype=torch.float32, device="cuda")
    rows = synth.subsample_rows(n, 24, 8201)
    for rep in range(4):
        Z = g.standard_normal((n, b)).astype(np.float32)
        Zd.copy_(torch.from_numpy(Z))
        h.matvec(Zd, out=out)
        h.sync()
        e, _ = float_errors(X, Z, out.cpu().numpy(), L1, rows)
        assert e["spec"] <= 1e-6 and e["per_row"] <= 1e-6, (rep, e)
    h.free()
