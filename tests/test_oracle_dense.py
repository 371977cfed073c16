"""Pins of the oracle's dense reference (Sec. 3.1, eq. (Laplace3D)).

Each check is fixed by mathematics, not by re-running the oracle's formula:
closed-form kernel values, a cube-corner configuration whose potential is
known exactly, the two-point case, the zero diagonal, bitwise symmetry of
the entries and linearity.
"""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_kernel_closed_form_values(oracle_mod):
    with open(os.path.join(GOLDEN, "kernel_values.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        got = oracle_mod.kernel_eval(c["kernel"], [c["r"]], c["param"])[0]
        assert got == pytest.approx(c["f"], rel=1e-15, abs=0.0), c


def test_two_points(oracle_mod):
    d = 0.75
    pts = np.array([[0.1, -0.2, 0.3], [0.1 + d, -0.2, 0.3]])
    x = np.array([2.0, -3.0])
    y = oracle_mod.dense_matvec(pts, x)
    f = 1.0 / (4.0 * np.pi * d)
    np.testing.assert_allclose(y, [f * -3.0, f * 2.0], rtol=1e-15)


@pytest.mark.parametrize("s", [1.0, 0.25])
def test_cube_corners_potential(oracle_mod, s):
    # 8 unit charges on the corners of a cube of side s: each corner sees 3
    # charges at distance s, 3 at s*sqrt(2) and 1 at s*sqrt(3).
    c = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], dtype=float) * s
    y = oracle_mod.dense_matvec(c, np.ones(8))
    expect = (3.0 + 3.0 / np.sqrt(2.0) + 1.0 / np.sqrt(3.0)) / (4.0 * np.pi * s)
    np.testing.assert_allclose(y, expect, rtol=1e-14)
    # the same configuration for exp(-r)/r
    yk = oracle_mod.dense_matvec(c, np.ones(8), kernel="yukawa", param=1.0)
    ek = sum(m * np.exp(-d) / d for m, d in ((3, s), (3, s * np.sqrt(2)), (1, s * np.sqrt(3))))
    np.testing.assert_allclose(yk, ek, rtol=1e-14)


def test_entries_symmetric_and_zero_diagonal(oracle_mod):
    rng = np.random.default_rng(11)
    pts = rng.uniform(-1, 1, (200, 3))
    for kernel in ("laplace", "yukawa", "inv_r4", "cos_r"):
        for (i, j) in [(0, 1), (5, 199), (17, 42), (100, 3)]:
            ei = np.zeros(200)
            ej = np.zeros(200)
            ei[i] = 1.0
            ej[j] = 1.0
            col_j = oracle_mod.dense_matvec(pts, ej, kernel=kernel)
            col_i = oracle_mod.dense_matvec(pts, ei, kernel=kernel)
            assert col_j[i] == col_i[j]  # K(i,j) == K(j,i) bitwise
            assert col_j[j] == 0.0 and col_i[i] == 0.0  # K(i,i) = 0
            assert col_j[i] != 0.0


def test_coincident_distinct_points_contribute_nothing(oracle_mod):
    pts = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    y = oracle_mod.dense_matvec(pts, np.array([1.0, 1.0, 1.0]))
    f1 = 1.0 / (4.0 * np.pi)
    np.testing.assert_allclose(y, [f1, f1, 2 * f1], rtol=1e-15)


def test_linearity_and_rows(oracle_mod):
    rng = np.random.default_rng(5)
    pts = rng.uniform(-1, 1, (500, 3))
    a, b = rng.standard_normal(500), rng.standard_normal(500)
    ya = oracle_mod.dense_matvec(pts, a)
    yb = oracle_mod.dense_matvec(pts, b)
    yab = oracle_mod.dense_matvec(pts, 2.0 * a - 0.5 * b)
    np.testing.assert_allclose(yab, 2.0 * ya - 0.5 * yb, rtol=1e-12, atol=1e-12 * np.abs(ya).max())
    # sampled-row mode returns exactly the same numbers as the full product
    rows = np.array([0, 3, 250, 499])
    np.testing.assert_array_equal(oracle_mod.dense_rows(pts, a, rows), ya[rows])
    # several right-hand sides are independent columns
    Y = oracle_mod.dense_matvec(pts, np.stack([a, b], axis=1))
    np.testing.assert_array_equal(Y[:, 0], ya)
    np.testing.assert_array_equal(Y[:, 1], yb)
    # <a, K b> = <b, K a> (K symmetric), up to summation order
    assert abs(a @ yb - b @ ya) <= 1e-13 * np.linalg.norm(a) * np.linalg.norm(yb) * 10
