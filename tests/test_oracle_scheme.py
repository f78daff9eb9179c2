"""Pins of the oracle's general predict/update lifting (Sec. II-A, W_j with
chosen P_j and U_j; Example 2.1; Remark 3.1).

Each pin is fixed by something other than the oracle's own code: the lazy
transform already pinned to Example 2.2, small cases worked by hand from the
level equations, the kept samples of Example 2.1, exactness of the linear
interpolate on linear data, perfect reconstruction (Lemma 2.1), linearity
(Lemma 2.2), the adjoint identities and a finite-difference derivative.
"""

import numpy as np
import pytest

import oracle as orc


def _x(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("L", [0, 1, 2, 3, 4])
def test_lazy_scheme_is_the_paper_transform(L):
    # P_j = I, U_j = I/2 reproduce Alg. 1 (pinned to Example 2.2) to the bit.
    x = _x((16, 3, 5), L)
    t = orc.lazy_scheme(L)
    assert np.array_equal(orc.lift_fwd_scheme(x, L, t), orc.lift_fwd(x, L))
    c = orc.lift_fwd(x, L)
    assert np.array_equal(orc.lift_inv_scheme(c, L, t), orc.lift_inv(c, L))


def test_lazy_scheme_transposes_match_the_derived_ones():
    # The explicit-matrix transposes against the level-by-level transposes of
    # the lazy transform, which are derived and pinned independently.
    g = _x((16, 2, 3), 5)
    t = orc.lazy_scheme(3)
    np.testing.assert_allclose(orc.lift_fwd_scheme_adj(g, 3, t), orc.lift_fwd_adj(g, 3),
                               rtol=0, atol=1e-14)
    np.testing.assert_allclose(orc.lift_inv_scheme_adj(g, 3, t), orc.lift_inv_adj(g, 3),
                               rtol=0, atol=1e-14)


def test_interpolating_level_by_hand():
    # f = (1, 2, 4, 8), one level: o = (1, 4), e = (2, 8).  Predict from the
    # kept neighbours: P e = (e[0], (e[0] + e[1]) / 2) = (2, 5) (the left end
    # extends e[0]), so d = (1 - 2, 4 - 5) = (-1, -1); U = 0 keeps s = e.
    f = np.array([1.0, 2.0, 4.0, 8.0])
    assert np.array_equal(orc.lift_fwd_scheme(f, 1, orc.interpolating_scheme(1)),
                          [2.0, 8.0, -1.0, -1.0])
    # CDF 5/3 update: U d = ((d0 + d1) / 4, (d1 + d1) / 4) = (-0.5, -0.5), s = e + U d.
    assert np.array_equal(orc.lift_fwd_scheme(f, 1, orc.cdf53_scheme(1)),
                          [1.5, 7.5, -1.0, -1.0])


def test_stencil_matrices_by_hand():
    # n = 3, interpolating predict: row m holds 1/2 at clamp(m-1) and at m.
    P, U = orc.scheme_operators(3, [0, 0.5, 0.5, 0, 0], [0, 0, 0.25, 0.25, 0])
    np.testing.assert_array_equal(P, [[1.0, 0, 0], [0.5, 0.5, 0], [0, 0.5, 0.5]])
    np.testing.assert_array_equal(U, [[0.25, 0.25, 0], [0, 0.25, 0.25], [0, 0, 0.5]])
    # One pair per tube: every tap lands on the only entry.
    P1, U1 = orc.scheme_operators(1, [1, 2, 3, 4, 5], [0.5, 0, 0, 0, 0.25])
    assert P1[0, 0] == 15.0 and U1[0, 0] == 0.75


@pytest.mark.parametrize("L", [1, 2, 3])
def test_example21_smooth_coefficients_are_kept_samples(L):
    # Example 2.1: with U = 0 the smooth coefficients are samples of the
    # signal itself; with the second entry of each pair kept, s_L holds
    # f[2^L - 1], f[2^(L+1) - 1], ...
    x = _x((16, 2, 2), 10 + L)
    c = orc.lift_fwd_scheme(x, L, orc.interpolating_scheme(L))
    step = 1 << L
    np.testing.assert_array_equal(c[:16 >> L], x[step - 1::step])


@pytest.mark.parametrize("L", [1, 2, 3])
def test_interpolating_details_vanish_on_linear_tubes(L):
    # The linear interpolate is exact for linear data, so away from the left
    # end (where the predict extends e[0]) every detail coefficient is zero,
    # at every level (the kept samples of a linear tube are again linear).
    p = 32
    tube = 3.0 - 0.75 * np.arange(p)
    c = orc.lift_fwd_scheme(tube, L, orc.interpolating_scheme(L))
    for j in range(1, L + 1):
        d = c[p >> j: p >> (j - 1)]
        np.testing.assert_allclose(d[1:], 0.0, atol=1e-13)
        # d[0] = f0 - f1 at level 1 (slope -0.75 per sample, times 2^(j-1)).
        assert abs(d[0] - 0.75 * (1 << (j - 1))) < 1e-13


def _random_scheme(L, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-0.6, 0.6, (L, 2, orc.SCHEME_TAPS))


@pytest.mark.parametrize("L,seed", [(1, 0), (2, 1), (3, 2), (4, 3)])
def test_perfect_reconstruction_any_scheme(L, seed):
    # Lemma 2.1 holds for any P_j, U_j: every lifting step is inverted exactly.
    t = _random_scheme(L, seed)
    x = _x((32, 3, 2), seed)
    c = orc.lift_fwd_scheme(x, L, t)
    np.testing.assert_allclose(orc.lift_inv_scheme(c, L, t), x, atol=1e-12)
    np.testing.assert_allclose(orc.lift_fwd_scheme(orc.lift_inv_scheme(x, L, t), L, t), x,
                               atol=1e-12)


def test_linearity_any_scheme():
    t = _random_scheme(3, 7)
    x, y = _x((16, 4), 1), _x((16, 4), 2)
    lhs = orc.lift_fwd_scheme(2.5 * x - 0.5 * y, 3, t)
    rhs = 2.5 * orc.lift_fwd_scheme(x, 3, t) - 0.5 * orc.lift_fwd_scheme(y, 3, t)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


@pytest.mark.parametrize("scheme", ["interp", "cdf53", "random"])
def test_adjoint_identities(scheme):
    # <W x, y> = <x, W^T y> and <W^{-1} x, y> = <x, W^{-T} y>, with W and
    # W^{-1} evaluated level by level and the transposes from the matrices.
    L = 3
    t = {"interp": orc.interpolating_scheme(L), "cdf53": orc.cdf53_scheme(L),
         "random": _random_scheme(L, 9)}[scheme]
    x, y = _x((24, 5), 3), _x((24, 5), 4)
    assert abs(np.sum(orc.lift_fwd_scheme(x, L, t) * y)
               - np.sum(x * orc.lift_fwd_scheme_adj(y, L, t))) < 1e-11
    assert abs(np.sum(orc.lift_inv_scheme(x, L, t) * y)
               - np.sum(x * orc.lift_inv_scheme_adj(y, L, t))) < 1e-11


def test_scheme_product_associative_and_lazy_case():
    t = orc.cdf53_scheme(2)
    a, b, c = _x((8, 3, 4), 1), _x((8, 4, 2), 2), _x((8, 2, 5), 3)
    lhs = orc.w_product_scheme(orc.w_product_scheme(a, b, 2, t), c, 2, t)
    rhs = orc.w_product_scheme(a, orc.w_product_scheme(b, c, 2, t), 2, t)
    np.testing.assert_allclose(lhs, rhs, atol=1e-11)
    np.testing.assert_array_equal(orc.w_product_scheme(a, b, 2, orc.lazy_scheme(2)),
                                  orc.w_product(a, b, 2))


def test_scheme_vjp_by_finite_differences():
    t = _random_scheme(2, 11)
    a, b, g = _x((8, 3, 4), 5), _x((8, 4, 2), 6), _x((8, 3, 2), 7)
    da, db = orc.w_product_scheme_vjp(a, b, g, 2, t)
    va, vb = _x(a.shape, 8), _x(b.shape, 9)
    h = 1e-6

    def loss(aa, bb):
        return np.sum(g * orc.w_product_scheme(aa, bb, 2, t))

    fd = (loss(a + h * va, b + h * vb) - loss(a - h * va, b - h * vb)) / (2 * h)
    assert abs(fd - (np.sum(da * va) + np.sum(db * vb))) < 1e-6 * max(1.0, abs(fd))


def test_taps_shape_is_checked():
    with pytest.raises(ValueError):
        orc.lift_fwd_scheme(np.zeros((8, 2)), 2, np.zeros((1, 2, 5)))


def test_scheme_matrix_by_hand_and_inverse():
    # One lazy level on p = 4 (pairs (x0, x1), (x2, x3)): s = (x0 + x1) / 2,
    # d = x0 - x1, coefficients in Mallat order (s_1 then d_1).
    expect = np.array([[0.5, 0.5, 0.0, 0.0],
                       [0.0, 0.0, 0.5, 0.5],
                       [1.0, -1.0, 0.0, 0.0],
                       [0.0, 0.0, 1.0, -1.0]])
    np.testing.assert_array_equal(orc.scheme_matrix(4, 1, orc.lazy_scheme(1)), expect)
    # Lemma 2.1 in matrix form, for any stencils: W^{-1} W = W W^{-1} = I.
    t = _random_scheme(3, 21)
    Wm = orc.scheme_matrix(16, 3, t)
    Wi = orc.scheme_inverse_matrix(16, 3, t)
    np.testing.assert_allclose(Wi @ Wm, np.eye(16), atol=1e-12)
    np.testing.assert_allclose(Wm @ Wi, np.eye(16), atol=1e-12)
