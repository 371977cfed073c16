"""Pins of the oracle's rank truncation (recompression of ACA factors).

Every check rests on something other than the truncation routine itself:
exact low-rank products, the Eckart-Young theorem through a dense SVD of the
product U V^T (not of the QR core the routine uses), and the rank rule.
"""
import numpy as np

import oracle


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_exact_low_rank_product_keeps_its_rank():
    rng = np.random.default_rng(11)
    for m, n, k, r in [(40, 30, 12, 5), (200, 64, 30, 1), (17, 19, 9, 8)]:
        A = rng.standard_normal((m, r)) @ rng.standard_normal((r, k))
        B = rng.standard_normal((n, k))
        Up, Vp, rr = oracle.truncate_factors(A, B, 1e-10)
        assert rr == r
        assert Up.shape == (m, r) and Vp.shape == (n, r)
        assert rel(Up @ Vp.T, A @ B.T) <= 1e-12


def test_error_is_the_eckart_young_tail_and_rank_is_minimal():
    rng = np.random.default_rng(12)
    m, n, k = 60, 45, 25
    # factors with geometrically decaying singular values, as ACA produces
    # (decay chosen so that no singular value sits on a threshold)
    qa, _ = np.linalg.qr(rng.standard_normal((m, k)))
    qb, _ = np.linalg.qr(rng.standard_normal((n, k)))
    s = 10.0 ** (-0.37 * np.arange(k))
    U = qa * s
    V = qb @ np.linalg.qr(rng.standard_normal((k, k)))[0]
    M = U @ V.T
    sd = np.linalg.svd(M, compute_uv=False)
    total = np.linalg.norm(sd)
    for tol in (1e-2, 1e-5, 1e-8):
        Up, Vp, r = oracle.truncate_factors(U, V, tol)
        tail = np.linalg.norm(sd[r:])
        err = np.linalg.norm(M - Up @ Vp.T)
        assert abs(err - tail) <= 1e-9 * total + 1e-6 * tail
        assert tail <= tol * total
        assert np.linalg.norm(sd[r - 1:]) > tol * total  # one rank less would not do


def test_no_op_cases():
    rng = np.random.default_rng(13)
    U1, V1 = rng.standard_normal((10, 1)), rng.standard_normal((7, 1))
    Up, Vp, r = oracle.truncate_factors(U1, V1, 0.5)
    assert r == 1 and np.array_equal(Up, U1) and np.array_equal(Vp, V1)
    U, V = rng.standard_normal((30, 6)), rng.standard_normal((20, 6))
    Up, Vp, r = oracle.truncate_factors(U, V, 1e-15)
    assert r == 6 and np.array_equal(Up, U) and np.array_equal(Vp, V)
    Z = np.zeros((5, 3))
    Up, Vp, r = oracle.truncate_factors(Z, Z, 1e-3)
    assert r == 3 and not Up.any()


def test_aca_factors_of_a_kernel_block_shrink_within_tol():
    # two separated 8x8x8 grids (a well-separated block), Laplace entries
    g = (np.arange(8) + 0.5) / 8
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    Y = X + np.array([2.0, 0.0, 0.0])
    pts = np.concatenate([X, Y])
    K = oracle.dense_rows(pts, np.eye(len(pts))[:, 512:], np.arange(512))
    U, V = oracle.aca_dense(K, 1e-8)[:2]
    Up, Vp, r = oracle.truncate_factors(U, V, 1e-8)
    assert r <= U.shape[1]
    assert rel(Up @ Vp.T, U @ V.T) <= 1e-8
    assert rel(Up @ Vp.T, K) <= 1e-7
