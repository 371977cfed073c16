"""Oracle side of the integral-equation solve (Sec. 5.2, eqs. (IE) and
(ILDiscrete)): the collocation system and a plain restarted GMRES.

TEST INFRASTRUCTURE ONLY.  Only ``tests/`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the GPU library.

Discretisation (the paper leaves the quadrature open; this is the reading the
repository takes): sigma(x) + int_B K(x, y) sigma(y) dy = f(x) on B = [-1,1]^3
with K = 1/|x - y|, piecewise-constant sigma on the N = k^3 cells of a uniform
grid (side h = 2/k), collocation at the cell centres x_i.  Off the diagonal the
cell integral is the midpoint rule h^3 / |x_i - x_j|; on the diagonal it is the
exact integral of 1/|x_i - y| over the cell, h^2 C with
C = int_{[-1/2,1/2]^3} du / |u| = 6 ln((1 + sqrt 3) / sqrt 2) - pi / 2.
So A sigma = (1 + h^2 C) sigma + h^3 K0 sigma, K0 the kernel matrix of 1/r
with a zero diagonal.  The library's Laplace kernel is 1/(4 pi r), so with
its product y = K~ sigma the off-diagonal term is 4 pi h^3 y.

GMRES(m) follows Saad and Schultz (1986): Arnoldi with modified Gram-Schmidt,
Givens rotations on the Hessenberg matrix, the least-squares solution at the
end of every cycle, restart from the true residual.
"""
from __future__ import annotations

import numpy as np

FOUR_PI = 4.0 * np.pi


def cube_self_integral() -> float:
    """int over the unit cube centred at the origin of 1/|u| (closed form)."""
    s3 = np.sqrt(3.0)
    return 6.0 * np.log((1.0 + s3) / np.sqrt(2.0)) - np.pi / 2.0


def ie_coefficients(k: int) -> tuple[float, float]:
    """(diagonal, scale of the 1/(4 pi r) product) of the collocation system on
    a k^3 grid of [-1,1]^3: A sigma = diag sigma + scale K_laplace sigma."""
    h = 2.0 / k
    return 1.0 + h * h * cube_self_integral(), FOUR_PI * h ** 3


def gmres(apply, f, x0=None, rtol: float = 1e-10, restart: int = 50, max_iter: int = 1000):
    """Solves apply(x) = f.  Returns (x, iterations, relative residual history);
    the history holds the true relative residual at the start of every cycle
    and the Givens estimate after every iteration."""
    f = np.asarray(f, dtype=np.float64)
    n = f.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    fn = float(np.linalg.norm(f))
    if fn == 0.0:
        return np.zeros(n), 0, [0.0]
    history = []
    it = 0
    while True:
        r = f - apply(x)
        beta = float(np.linalg.norm(r))
        history.append(beta / fn)
        if beta / fn < rtol or it >= max_iter:
            return x, it, history
        m = restart
        V = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        jj = 0
        for j in range(m):
            w = apply(V[:, j])
            it += 1
            for i in range(j + 1):  # modified Gram-Schmidt
                H[i, j] = float(w @ V[:, i])
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = float(np.linalg.norm(w))
            if H[j + 1, j] > 0.0:
                V[:, j + 1] = w / H[j + 1, j]
            for i in range(j):  # earlier rotations on the new column
                a, b = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * b
                H[i + 1, j] = -sn[i] * a + cs[i] * b
            a, b = H[j, j], H[j + 1, j]
            d = float(np.hypot(a, b))
            cs[j], sn[j] = (1.0, 0.0) if d == 0.0 else (a / d, b / d)
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            jj = j + 1
            history.append(abs(g[j + 1]) / fn)
            if abs(g[j + 1]) / fn < rtol or it >= max_iter or H[j, j] == 0.0:
                break
        # least squares: back substitution on the rotated Hessenberg matrix
        y = np.zeros(jj)
        for i in range(jj - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:jj] @ y[i + 1:]) / H[i, i]
        x = x + V[:, :jj] @ y
