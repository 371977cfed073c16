"""Pins of the oracle's ACA (Sec. 4.1, eq. (prank); Algorithm 1).

- Special cases with exact answers: the zero matrix (rank 0), an exactly
  representable rank-one matrix (rank 1, zero residual), a diagonal matrix
  (full rank, exact), random exact rank-r products (rank <= r + 1, residual at
  rounding level).
- The cross-approximation identity of eq. (prank): the stored U V^T equals
  K(X,tau) K(sigma,tau)^-1 K(sigma,Y) built from the recorded pivots.
- Kernel blocks of the 16^3 grid: Frobenius error within 10 tol, and the
  Eckart-Young lower bound rank_ACA >= r_delta(K_b) (numerical rank as defined
  in the footnote of Sec. 3.1) with delta the measured 2-norm error.
"""
import numpy as np
import pytest

from paper_2307_16303_amd import inputs

CUBE = dict(box_lo=inputs.CUBE_LO, box_side=inputs.CUBE_SIDE)


def test_zero_matrix(oracle_mod):
    U, V, rp, cp = oracle_mod.aca_dense(np.zeros((7, 5)), 1e-8)
    assert U.shape[1] == 0


def test_exact_rank_one(oracle_mod):
    b = np.array([1.0, -2.0, 4.0, 0.5, 8.0])
    c = np.array([2.0, 0.25, -4.0, 1.0])
    A = np.outer(b, c)
    U, V, rp, cp = oracle_mod.aca_dense(A, 1e-12)
    assert U.shape[1] == 1
    assert rp[0] == 0 and cp[0] == 2  # row 0 first; largest |A[0, j]| is at j = 2
    np.testing.assert_array_equal(U @ V.T, A)


def test_diagonal_full_rank(oracle_mod):
    d = np.array([3.0, -1.0, 2.0, 5.0, -7.0, 0.5])
    A = np.diag(d)
    U, V, rp, cp = oracle_mod.aca_dense(A, 1e-12)
    assert U.shape[1] == 6
    np.testing.assert_array_equal(U @ V.T, A)
    np.testing.assert_array_equal(rp, np.arange(6))  # argmax of a zero column -> lowest unused row
    np.testing.assert_array_equal(cp, np.arange(6))


@pytest.mark.parametrize("m,n,r", [(40, 30, 5), (100, 120, 12), (64, 64, 1), (9, 200, 9)])
def test_exact_low_rank(oracle_mod, m, n, r):
    rng = np.random.default_rng(m * n + r)
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    U, V, rp, cp = oracle_mod.aca_dense(A, 1e-12)
    k = U.shape[1]
    assert r <= k <= r + 1
    assert np.linalg.norm(A - U @ V.T) <= 1e-13 * np.linalg.norm(A) * 10
    assert len(set(rp.tolist())) == k and len(set(cp.tolist())) == k


def test_cross_identity_on_kernel_blocks(oracle_mod):
    g = inputs.grid_points(16)
    h = oracle_mod.HODLR3D(g, leaf_size=64, tol=1e-6, **CUBE)
    f = h.far()
    rp, cp = h.pivots()
    off = np.concatenate([[0], np.cumsum(f["rank"])])
    rng = np.random.default_rng(0)
    picks = list(rng.choice(np.nonzero(f["level"] == 2)[0], 20, replace=False)) + [0, 3]
    for b in picks:
        K = h.block_dense(b)
        U, V = h.block_factors(b)
        sig = rp[off[b]:off[b + 1]]
        tau = cp[off[b]:off[b + 1]]
        cross = K[:, tau] @ np.linalg.solve(K[np.ix_(sig, tau)], K[sig, :])
        assert np.linalg.norm(U @ V.T - cross) <= 1e-9 * np.linalg.norm(K)
        # the approximation interpolates the pivot rows and columns
        np.testing.assert_allclose((U @ V.T)[sig, :], K[sig, :], rtol=0, atol=1e-12 * np.abs(K).max())
        np.testing.assert_allclose((U @ V.T)[:, tau], K[:, tau], rtol=0, atol=1e-12 * np.abs(K).max())


@pytest.mark.parametrize("tol", [1e-6, 1e-10])
def test_kernel_blocks_error_and_eckart_young(oracle_mod, tol):
    g = inputs.grid_points(16)
    h = oracle_mod.HODLR3D(g, leaf_size=64, tol=tol, **CUBE)
    f = h.far()
    assert h.num_capped == 0
    rng = np.random.default_rng(1)
    picks = list(np.nonzero(f["level"] == 1)[0][:2]) + list(
        rng.choice(np.nonzero(f["level"] == 2)[0], 40, replace=False))
    worst = 0.0
    ratios = []
    for b in picks:
        K = h.block_dense(b)
        U, V = h.block_factors(b)
        R = K - U @ V.T
        fro = np.linalg.norm(R) / np.linalg.norm(K)
        worst = max(worst, fro)
        s = np.linalg.svd(K, compute_uv=False)
        delta = np.linalg.norm(R, 2) / s[0]
        r_delta = int(np.sum(s / s[0] > delta * (1 + 1e-8)))
        k = U.shape[1]
        assert k >= r_delta, (b, k, r_delta)
        r_tol = max(1, int(np.sum(s / s[0] > tol)))
        ratios.append(k / r_tol)
    assert worst <= 10 * tol, worst
    # ACA is near-optimal in rank on these blocks
    assert 0.8 <= np.median(ratios) <= 2.0, np.median(ratios)


def _coords(key, bits):
    x = y = z = 0
    for b in range(bits - 1, -1, -1):
        x = (x << 1) | ((key >> (3 * b + 2)) & 1)
        y = (y << 1) | ((key >> (3 * b + 1)) & 1)
        z = (z << 1) | ((key >> (3 * b)) & 1)
    return np.array([x, y, z])


def test_rank_growth_by_relation(oracle_mod):
    # Table tab:rankgrowth: at equal box size, vertex-sharing (V) blocks need a
    # higher rank than well-separated (W) ones, and W ranks fall with distance.
    g = inputs.grid_points(16)
    h = oracle_mod.HODLR3D(g, leaf_size=64, tol=1e-8, **CUBE)
    f = h.far()
    lv2 = f["level"] == 2
    cheb = np.array([np.abs(_coords(t, 2) - _coords(s, 2)).max()
                     for t, s in zip(f["t"][lv2], f["s"][lv2])])
    ranks = f["rank"][lv2]
    assert ranks[cheb == 1].mean() > ranks[cheb >= 2].mean()
    assert ranks[cheb >= 3].mean() <= ranks[cheb == 2].mean()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_norm_estimate_and_stopping_rule(oracle_mod, seed):
    # The running estimate equals |U V^T|_F^2 computed directly, which needs
    # every cross term (u_a.u_b)(v_a.v_b); the stop happens at the first term
    # with |u_k||v_k| <= tol |S_k|_F.
    rng = np.random.default_rng(seed)
    m, n = 60, 45
    # smooth, numerically low-rank, with strongly non-orthogonal ACA terms
    a = rng.uniform(0, 1, m)
    b = rng.uniform(2, 3, n)
    A = 1.0 / (a[:, None] + b[None, :]) + 0.3
    tol = 1e-9
    U, V, rp, cp, norm2 = oracle_mod.aca_dense(A, tol, return_norm=True)
    k = U.shape[1]
    assert 2 <= k < min(m, n)
    S = U @ V.T
    assert norm2 == pytest.approx(np.linalg.norm(S) ** 2, rel=1e-12)
    for j in range(1, k + 1):
        term = np.linalg.norm(U[:, j - 1]) * np.linalg.norm(V[:, j - 1])
        sj = np.linalg.norm(U[:, :j] @ V[:, :j].T)
        if j < k:
            assert term > tol * sj * (1 - 1e-9)
        else:
            assert term <= tol * sj * (1 + 1e-9)
