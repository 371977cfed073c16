"""Seeded synthetic workloads shaped like the paper's experiments.

This module holds no arithmetic of the method: it only draws point clouds and
right-hand sides with numpy's PCG64 ``default_rng``.  Both the GPU path and the
CPU oracle are fed from here.

The paper's runs use particles spread uniformly in the cube [-1,1]^3 (Sec. 5,
settings list; Sec. 5.1) with a random vector to multiply.  The workloads
below keep that cube and use either a cell-centred tensor grid or i.i.d.
uniform points.
"""
from __future__ import annotations

import numpy as np

CUBE_LO = (-1.0, -1.0, -1.0)
CUBE_SIDE = 2.0


def grid_points(k: int) -> np.ndarray:
    """k^3 cell-centred grid in [-1,1]^3: x_i = -1 + (2i+1)/k, (ix, iy, iz) row order."""
    c = -1.0 + (2.0 * np.arange(k) + 1.0) / k
    gx, gy, gz = np.meshgrid(c, c, c, indexing="ij")
    return np.ascontiguousarray(np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1))


def uniform_points(n: int, seed: int = 0) -> np.ndarray:
    """n i.i.d. points, uniform in [-1,1]^3 (FP64, C-contiguous n x 3)."""
    return np.ascontiguousarray(np.random.default_rng(seed).uniform(-1.0, 1.0, (n, 3)))


def clustered_points(n_uniform: int, n_ball: int, radius: float = 0.05,
                     centre=(0.3, -0.2, 0.1), seed: int = 0) -> np.ndarray:
    """n_uniform points uniform in [-1,1]^3 followed by n_ball points uniform in a ball
    (a dense cluster: the tree then mixes nearly empty leaves with full ones)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, (n_uniform, 3))
    d = rng.standard_normal((n_ball, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    b = np.asarray(centre) + radius * np.cbrt(rng.uniform(0.0, 1.0, (n_ball, 1))) * d
    return np.ascontiguousarray(np.concatenate([u, b], axis=0))


def two_density_points(n: int, frac_low: float, seed: int = 0) -> np.ndarray:
    """n points uniform in [-1,1]^3 whose first round(frac_low n) are folded into
    the half x <= 0 and the rest into x >= 0: two densities, so that leaves of
    one depth hold from a few points to several times as many."""
    p = uniform_points(n, seed)
    k = int(round(frac_low * n))
    p[:k, 0] = -np.abs(p[:k, 0])
    p[k:, 0] = np.abs(p[k:, 0])
    return np.ascontiguousarray(p)


def uniform_rhs(n: int, seed: int = 0, nrhs: int | None = None) -> np.ndarray:
    shape = (n,) if nrhs is None else (n, nrhs)
    return np.random.default_rng(seed).uniform(-1.0, 1.0, shape)


def normal_rhs(n: int, seed: int = 1, nrhs: int | None = None) -> np.ndarray:
    shape = (n,) if nrhs is None else (n, nrhs)
    return np.random.default_rng(seed).standard_normal(shape)


def sample_rows(n: int, count: int, seed: int = 3) -> np.ndarray:
    """Sorted distinct target rows for sampled checks at sizes the dense sum cannot cover."""
    count = min(count, n)
    return np.sort(np.random.default_rng(seed).choice(n, size=count, replace=False)).astype(np.int64)


# Named workloads.  Each entry: points, kernel, leaf size, ACA tolerance, RHS.
WORKLOADS = {
    # 16^3 grid, Laplace, leaf <= 64, tol 1e-10, one RHS U(-1,1) seed 0.
    "grid4096": dict(n=4096, points=("grid", 16), kernel="laplace", leaf_size=64, tol=1e-10,
                     rhs=("uniform", 0)),
    # 262,144 i.i.d. points, Laplace, leaf <= 64, tol 1e-8, one RHS N(0,1) seed 1.
    "uniform262k": dict(n=262144, points=("uniform", 0), kernel="laplace", leaf_size=64,
                        tol=1e-8, rhs=("normal", 1)),
    "uniform262k_yukawa": dict(n=262144, points=("uniform", 0), kernel="yukawa", leaf_size=64,
                               tol=1e-8, rhs=("normal", 1)),
    # 1,048,576 i.i.d. points, Laplace, tol 1e-7 (precision form).
    "uniform1m": dict(n=1048576, points=("uniform", 0), kernel="laplace", leaf_size=64, tol=1e-7,
                      rhs=("normal", 1)),
}


def make_points(spec) -> np.ndarray:
    kind, arg = spec
    if kind == "grid":
        return grid_points(arg)
    if kind == "uniform":
        raise ValueError("uniform points need n; use workload_points")
    raise ValueError(kind)


def workload_points(name: str) -> np.ndarray:
    w = WORKLOADS[name]
    kind, arg = w["points"]
    if kind == "grid":
        return grid_points(arg)
    return uniform_points(w["n"], seed=arg)


def workload_rhs(name: str, nrhs: int | None = None) -> np.ndarray:
    w = WORKLOADS[name]
    kind, seed = w["rhs"]
    if kind == "uniform":
        return uniform_rhs(w["n"], seed, nrhs)
    return normal_rhs(w["n"], seed, nrhs)


def batch_problem_sizes(count: int = 32, seed: int = 7, lo: int = 8192, hi: int = 131072):
    """Sizes of independent problems for the multi-problem form: uniform integers in [lo, hi]."""
    return np.random.default_rng(seed).integers(lo, hi, count, endpoint=True)


# The multi-problem workload: 32 independent clouds, Laplace, leaf <= 64,
# ACA tol 1e-7, FP32 factors, one RHS each.
BATCH_WORKLOAD = dict(count=32, kernel="laplace", leaf_size=64, tol=1e-7, factor_dtype="fp32")


def batch_workload(count: int = 32, seed: int = 7, lo: int = 8192, hi: int = 131072):
    """[(points_i, rhs_i)]: sizes from batch_problem_sizes, points of problem i uniform in
    [-1,1]^3 with seed 100 + i, right-hand side N(0,1) with seed 200 + i."""
    ns = batch_problem_sizes(count, seed, lo, hi)
    return [(uniform_points(int(v), 100 + i), normal_rhs(int(v), 200 + i)) for i, v in enumerate(ns)]
