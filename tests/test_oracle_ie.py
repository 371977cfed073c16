"""Pins of the oracle's integral-equation pieces (Sec. 5.2).

- The self-cell integral C = int_{[-1/2,1/2]^3} 1/|u| du: its closed form
  against an independent route, the divergence theorem (div(u/|u|) = 2/|u|,
  so the volume integral is a quarter of the sum over the six faces of the
  smooth face integrals of 1/|u|), integrated by adaptive quadrature.
- GMRES: finite termination on an n x n system with restart >= n, agreement
  with LAPACK's solve on a nonsymmetric well-conditioned system with short
  restarts, the minimal-residual property (the estimates never increase
  within a cycle), and exact recovery of a known solution of the collocation
  system on the 16^3 grid with the dense kernel product.
"""
import numpy as np
import pytest

from oracle import ie
from paper_2307_16303_amd import inputs


def test_self_integral_closed_form():
    # one face at distance 1/2: int_{[-1/2,1/2]^2} (x^2 + y^2 + 1/4)^(-1/2) dx dy, a
    # smooth integrand, by a 200-point Gauss-Legendre product rule
    xg, wg = np.polynomial.legendre.leggauss(200)
    x, w = 0.5 * xg, 0.5 * wg
    X, Y = np.meshgrid(x, x)
    face = float(np.sum(np.outer(w, w) / np.sqrt(X * X + Y * Y + 0.25)))
    # volume integral = (1/2) sum over faces of (u . n)/|u| dS = (1/2) 6 (1/2) face
    via_faces = 1.5 * face
    assert ie.cube_self_integral() == pytest.approx(via_faces, rel=1e-13, abs=0.0)
    assert ie.cube_self_integral() == pytest.approx(2.38007736, abs=1e-8)


def test_gmres_finite_termination():
    rng = np.random.default_rng(91)
    A = rng.standard_normal((30, 30)) + 8.0 * np.eye(30)
    x_true = rng.standard_normal(30)
    f = A @ x_true
    x, it, hist = ie.gmres(lambda v: A @ v, f, rtol=1e-13, restart=40, max_iter=40)
    assert it <= 30
    assert np.linalg.norm(x - x_true) <= 1e-11 * np.linalg.norm(x_true)


def test_gmres_restarted_matches_lapack():
    rng = np.random.default_rng(92)
    n = 200
    A = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    f = rng.standard_normal(n)
    x, it, hist = ie.gmres(lambda v: A @ v, f, rtol=1e-12, restart=10, max_iter=500)
    ref = np.linalg.solve(A, f)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    assert np.linalg.norm(A @ x - f) <= 1e-12 * np.linalg.norm(f)
    assert it > 10  # several cycles ran


def test_gmres_residual_estimates_do_not_increase():
    rng = np.random.default_rng(93)
    n = 120
    A = np.diag(np.linspace(1.0, 5.0, n)) + 0.2 * rng.standard_normal((n, n)) / np.sqrt(n)
    f = rng.standard_normal(n)
    _, it, hist = ie.gmres(lambda v: A @ v, f, rtol=1e-12, restart=200, max_iter=200)
    # one cycle: the true residual first, then one estimate per iteration
    assert all(b <= a * (1 + 1e-12) for a, b in zip(hist[:-1], hist[1:-1]))


def test_collocation_system_recovers_a_known_solution(oracle_mod):
    k = 16
    pts = inputs.grid_points(k)
    diag, scale = ie.ie_coefficients(k)
    h = 2.0 / k
    assert diag == pytest.approx(1.0 + h * h * 2.38007736, rel=1e-8)
    assert scale == pytest.approx(4.0 * np.pi * h ** 3)

    def apply(v):
        return diag * v + scale * oracle_mod.dense_matvec(pts, v)

    sigma = inputs.normal_rhs(k ** 3, seed=94)
    f = apply(sigma)
    x, it, hist = ie.gmres(apply, f, rtol=1e-10, restart=30, max_iter=300)
    assert hist[-1] < 1e-10
    assert np.linalg.norm(x - sigma) <= 1e-8 * np.linalg.norm(sigma)
    print(f"[ie oracle] 16^3 grid: {it} iterations, forward error "
          f"{np.linalg.norm(x - sigma) / np.linalg.norm(sigma):.2e}")
