"""Pins of the oracle's reverse-mode derivative and the least-squares gradient solve."""

import numpy as np

import oracle as orc


def _fd_check(f, x, grad, n_probe=12, h=1e-6, seed=0):
    rng = np.random.default_rng(seed)
    for _ in range(n_probe):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        xp = x.copy()
        xm = x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (f(xp) - f(xm)) / (2 * h)
        assert abs(fd - grad[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, grad[idx])


def test_vjp_finite_differences():
    rng = np.random.default_rng(1)
    p, L = 8, 3
    a = rng.standard_normal((p, 4, 5))
    b = rng.standard_normal((p, 5, 3))
    g = rng.standard_normal((p, 4, 3))
    da, db = orc.w_product_vjp(a, b, g, L)
    _fd_check(lambda x: np.sum(g * orc.w_product(x, b, L)), a, da)
    _fd_check(lambda x: np.sum(g * orc.w_product(a, x, L)), b, db, seed=1)


def test_vjp_equals_products_with_transposes():
    # For this lifting, dA = G *_w B^T and dB = A^T *_w G: the per-group scale between
    # W^T and W^{-1} is a scalar per coefficient slice and commutes with the face-product.
    rng = np.random.default_rng(2)
    p, L = 16, 4
    a = rng.standard_normal((p, 3, 4))
    b = rng.standard_normal((p, 4, 6))
    g = rng.standard_normal((p, 3, 6))
    da, db = orc.w_product_vjp(a, b, g, L)
    np.testing.assert_allclose(da, orc.w_product(g, orc.transpose(b), L), atol=1e-12)
    np.testing.assert_allclose(db, orc.w_product(orc.transpose(a), g, L), atol=1e-12)


def test_lsq_gradient_finite_differences():
    rng = np.random.default_rng(3)
    p, L = 8, 3
    k = rng.standard_normal((p, 6, 6))
    x = rng.standard_normal((p, 6, 4))
    y = rng.standard_normal((p, 6, 4))
    f = lambda z: float(np.sum((orc.w_product(k, z, L) - y) ** 2))  # noqa: E731
    _fd_check(f, x, orc.lsq_grad(k, x, y, L), h=1e-5)


def test_gradient_descent_reaches_least_squares_solution():
    # With well-conditioned coefficient slices the fixed-step iteration converges to
    # K^{-1} *_w Y.
    rng = np.random.default_rng(4)
    p, L, n = 8, 2, 5
    k = orc.lift_inv(np.stack([np.eye(n) + 0.1 * rng.standard_normal((n, n)) for _ in range(p)]), L)
    x_true = rng.standard_normal((p, n, 3))
    y = orc.w_product(k, x_true, L)
    # Lipschitz constant of the gradient: 2 * max_c ||Khat_c||_2^2 (synthesis vectors are
    # orthogonal with per-group scale, so the operator norm is the largest slice norm).
    kh = orc.lift_fwd(k, L)
    lip = 2 * max(np.linalg.norm(kh[c], 2) ** 2 for c in range(p))
    x, losses = orc.deblur_gd(k, y, L, steps=400, eta=1.0 / lip)
    assert all(b <= a * (1 + 1e-12) + 1e-24 for a, b in zip(losses, losses[1:]))
    np.testing.assert_allclose(x, x_true, atol=1e-8)


def test_identical_slices_operator_only_sees_coarse_coefficients():
    # K with identical frontal slices has zero detail coefficients, so K *_w X depends on X
    # only through its s_L slices, and the gradient has zero detail coefficients.
    rng = np.random.default_rng(6)
    p, L = 16, 3
    g = rng.standard_normal((5, 5))
    k = np.repeat(g[None], p, axis=0)
    kh = orc.lift_fwd(k, L)
    assert not np.any(kh[p >> L:])
    x = rng.standard_normal((p, 5, 2))
    y = rng.standard_normal((p, 5, 2))
    gh = orc.lift_fwd(orc.lsq_grad(k, x, y, L), L)
    assert np.max(np.abs(gh[p >> L:])) < 1e-12
