"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module only draws random numbers and arranges them into arrays.  It holds
none of the distance-matrix arithmetic: neither the oracle nor the HIP path
imports anything else in common.

All draws use NumPy's ``Generator(PCG64(seed))``.  Seeds are derived from a
fixed base per workload so every run of a workload sees the same bits:

    seed_X   = 2210151140 + workload_id
    seed_Z   = seed_X + 1000
    seed_sub = seed_X + 2000

Workloads (sizes follow the paper's empirical setup, Section 4 / Table 3, scaled
to the shapes the benchmark uses):

* 1 - n=2048, d=16, X ~ N(0,1) in FP64 (the GPU receives the FP32 rounding),
      one z ~ N(0,1); integer variant with X, z uniform in [-1000, 1000].
* 2 - n=2**20, d=64, mixture of 32 spherical Gaussians (means 5*N(0,I), unit
      covariance, equal weights), FP32; z ~ N(0,1).
* 3 - n=2**22, d=128, X ~ U[0,1) FP32; Z n x 64 ~ N(0,1) FP32.
* 4 - 512 datasets, n log-uniform in [2**10, 2**18], d in {3,16,64}, FP32
      N(0,1) or int32 uniform in [-2**15, 2**15]; b=8 right-hand sides.
* 5 - n=2**21, d=32, mixture of 50 Gaussians (same recipe as 2); block 40.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 2210151140


def seeds(workload: int) -> dict:
    sx = SEED_BASE + int(workload)
    return {"X": sx, "Z": sx + 1000, "sub": sx + 2000}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


# ----------------------------------------------------------------------------
# point clouds
# ----------------------------------------------------------------------------
def normal_points(n: int, d: int, seed: int, dtype=np.float64) -> np.ndarray:
    g = rng(seed)
    if np.dtype(dtype) == np.float32:
        return g.standard_normal((n, d), dtype=np.float32)
    return g.standard_normal((n, d))


def uniform_points(n: int, d: int, seed: int, dtype=np.float32) -> np.ndarray:
    g = rng(seed)
    if np.dtype(dtype) == np.float32:
        return g.random((n, d), dtype=np.float32)
    return g.random((n, d))


def int_points(n: int, d: int, lo: int, hi: int, seed: int, dtype=np.int64) -> np.ndarray:
    """Integers uniform on the closed range [lo, hi]."""
    g = rng(seed)
    return g.integers(lo, hi, size=(n, d), endpoint=True).astype(dtype)


def gaussian_mixture(n: int, d: int, k: int, seed: int, mean_scale: float = 5.0,
                     dtype=np.float32) -> np.ndarray:
    """k spherical unit-variance Gaussians with means mean_scale*N(0,I), equal weights."""
    g = rng(seed)
    means = mean_scale * g.standard_normal((k, d))
    comp = g.integers(0, k, size=n)
    if np.dtype(dtype) == np.float32:
        noise = g.standard_normal((n, d), dtype=np.float32)
        return noise + means.astype(np.float32)[comp]
    return g.standard_normal((n, d)) + means[comp]


def simplex_points(n: int, d: int, seed: int, alpha: float = 1.0, dtype=np.float32) -> np.ndarray:
    """Probability vectors: Dirichlet(alpha, ..., alpha) rows, every coordinate
    > 0 after rounding to dtype (a draw that rounds to 0 is raised to the
    smallest normal number of dtype)."""
    g = rng(seed)
    P = g.dirichlet(np.full(d, float(alpha)), size=n).astype(dtype)
    return np.maximum(P, np.finfo(dtype).tiny)


def square_matrix(d: int, seed: int, kind: str = "spd") -> np.ndarray:
    """A d x d FP64 matrix: "spd" = B B^T / d + I/2 (B ~ N(0,1)),
    "general" = N(0,1) / sqrt(d) entries (neither symmetric nor definite)."""
    g = rng(seed)
    B = g.standard_normal((d, d))
    if kind == "spd":
        return B @ B.T / d + 0.5 * np.eye(d)
    if kind == "general":
        return B / math.sqrt(d)
    raise ValueError(kind)


# ----------------------------------------------------------------------------
# right-hand sides
# ----------------------------------------------------------------------------
def rhs_normal(n: int, b: int, seed: int, dtype=np.float32) -> np.ndarray:
    g = rng(seed)
    if np.dtype(dtype) == np.float32:
        return g.standard_normal((n, b), dtype=np.float32)
    return g.standard_normal((n, b))


def rhs_int_gauss(n: int, b: int, seed: int, scale: float = 4096.0, dtype=np.int32) -> np.ndarray:
    """Integer right-hand sides with a Gaussian shape: round(scale * N(0,1))."""
    g = rng(seed)
    return np.rint(scale * g.standard_normal((n, b))).astype(dtype)


def rhs_positive(n: int, b: int, seed: int, spread: float = 1e-3, dtype=np.float32) -> np.ndarray:
    """Perron-like positive right-hand sides 1 + spread*N(0,1) (precision stress)."""
    g = rng(seed)
    return (1.0 + spread * g.standard_normal((n, b))).astype(dtype)


def subsample_rows(n: int, m: int, seed: int, extra=()) -> np.ndarray:
    """m distinct rows uniformly without replacement, plus the given extra rows; sorted."""
    g = rng(seed)
    m = min(m, n)
    base = g.choice(n, size=m, replace=False) if m < n else np.arange(n)
    rows = np.unique(np.concatenate([base.astype(np.int64), np.asarray(extra, dtype=np.int64)]))
    return rows[(rows >= 0) & (rows < n)]


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
def workload1(variant: str = "float"):
    s = seeds(1)
    n, d = 2048, 16
    if variant == "float":
        X = normal_points(n, d, s["X"], np.float64)
        z = rhs_normal(n, 1, s["Z"], np.float64)
        return X, z
    X = int_points(n, d, -1000, 1000, s["X"], np.int64)
    z = int_points(n, 1, -1000, 1000, s["Z"], np.int64)
    return X, z


def workload2(n: int = 1 << 20, d: int = 64, nq: int = 1):
    s = seeds(2)
    X = gaussian_mixture(n, d, 32, s["X"], 5.0, np.float32)
    Z = rhs_normal(n, nq, s["Z"], np.float32)
    return X, Z


def workload3(n: int = 1 << 22, d: int = 128, b: int = 64):
    s = seeds(3)
    X = uniform_points(n, d, s["X"], np.float32)
    Z = rhs_normal(n, b, s["Z"], np.float32)
    return X, Z


@dataclass
class DatasetSpec:
    n: int
    d: int
    is_int: bool
    seed: int


def workload4_specs(count: int = 512, lo: int = 1 << 10, hi: int = 1 << 18,
                    dims=(3, 16, 64)) -> list:
    s = seeds(4)
    g = rng(s["X"])
    u = g.uniform(math.log(lo), math.log(hi), size=count)
    ns = np.floor(np.exp(u)).astype(np.int64)
    ds = g.choice(np.asarray(dims), size=count)
    ints = g.integers(0, 2, size=count).astype(bool)
    return [DatasetSpec(int(ns[i]), int(ds[i]), bool(ints[i]), s["X"] + 17 * (i + 1))
            for i in range(count)]


def workload4_dataset(spec: DatasetSpec, b: int = 8):
    if spec.is_int:
        X = int_points(spec.n, spec.d, -(1 << 15), 1 << 15, spec.seed, np.int32)
        Z = rhs_int_gauss(spec.n, b, spec.seed + 1000, 4096.0, np.int32)
    else:
        X = normal_points(spec.n, spec.d, spec.seed, np.float32)
        Z = rhs_normal(spec.n, b, spec.seed + 1000, np.float32)
    return X, Z


def workload5(n: int = 1 << 21, d: int = 32):
    s = seeds(5)
    return gaussian_mixture(n, d, 50, s["X"], 5.0, np.float32)
