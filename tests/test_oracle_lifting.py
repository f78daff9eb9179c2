"""Pins of the oracle's lifting transforms (W, W^{-1}, W^T, W^{-T}) against the paper and closed forms."""

import numpy as np
import pytest

import oracle as orc
from pins import load_golden, dense_forward, dense_inverse, apply_mode3

EX = load_golden("example_2_2.json")


def _coeff_groups(c, L):
    p = c.shape[0]
    groups = {"s%d" % L: c[: p >> L]}
    for j in range(1, L + 1):
        groups["d%d" % j] = c[p >> j: p >> (j - 1)]
    return groups


def test_example_2_2_forward_all_levels_exact():
    # Example 2.2: level-1 and level-2 coefficients of A and B, exact dyadic values.
    for name in ("A", "B"):
        x = EX[name]
        c1 = _coeff_groups(orc.lift_fwd(x, 1), 1)
        assert np.array_equal(c1["s1"], EX[name + "_s1"])
        assert np.array_equal(c1["d1"], EX[name + "_d1"])
        c2 = _coeff_groups(orc.lift_fwd(x, 2), 2)
        assert np.array_equal(c2["s2"], EX[name + "_s2"])
        assert np.array_equal(c2["d2"], EX[name + "_d2"])
        assert np.array_equal(c2["d1"], EX[name + "_d1"])


def test_example_2_2_inverse_exact():
    # Example 2.2: C_s1 from (C_s2, C_d2), then C from (C_s1, C_d1).
    c = np.concatenate([EX["C_s2"], EX["C_d2"], EX["C_d1"]])
    assert np.array_equal(orc.lift_inv(c, 2), EX["C"])
    c_lvl1 = np.concatenate([EX["C_s2"], EX["C_d2"]])
    assert np.array_equal(orc.lift_inv(c_lvl1, 1), EX["C_s1"])


@pytest.mark.parametrize("p,L", [(1, 0), (2, 1), (4, 2), (8, 3), (12, 2), (16, 4), (24, 3), (32, 5), (6, 1)])
def test_forward_matches_closed_form(p, L):
    rng = np.random.default_rng(p * 31 + L)
    x = rng.standard_normal((p, 3, 2))
    np.testing.assert_allclose(orc.lift_fwd(x, L), apply_mode3(dense_forward(p, L), x), rtol=0, atol=1e-13)
    c = rng.standard_normal((p, 3, 2))
    np.testing.assert_allclose(orc.lift_inv(c, L), apply_mode3(dense_inverse(p, L), c), rtol=0, atol=1e-13)


@pytest.mark.parametrize("p,L", [(2, 1), (8, 3), (16, 2), (24, 3), (64, 6)])
def test_closed_forms_are_inverses(p, L):
    # The two independent closed forms are inverse to each other (Lemma 2.1 on the dense route).
    w = dense_forward(p, L)
    wi = dense_inverse(p, L)
    np.testing.assert_allclose(wi @ w, np.eye(p), atol=1e-14)
    np.testing.assert_allclose(w @ wi, np.eye(p), atol=1e-14)


@pytest.mark.parametrize("p,L", [(8, 3), (16, 4), (48, 4), (10, 1)])
def test_perfect_reconstruction_and_linearity(p, L):
    # Lemma 2.1 (both orders) and Lemma 2.2.
    rng = np.random.default_rng(7)
    f = rng.standard_normal((p, 4, 5))
    g = rng.standard_normal((p, 4, 5))
    np.testing.assert_allclose(orc.lift_inv(orc.lift_fwd(f, L), L), f, atol=1e-14)
    np.testing.assert_allclose(orc.lift_fwd(orc.lift_inv(f, L), L), f, atol=1e-14)
    a, b = 1.75, -0.3
    np.testing.assert_allclose(orc.lift_fwd(a * f + b * g, L),
                               a * orc.lift_fwd(f, L) + b * orc.lift_fwd(g, L), atol=1e-13)


def test_smooth_is_block_mean_and_details_sum_to_zero():
    # s_L is the mean over each 2^L block; each synthesis vector of a detail has zero sum,
    # so the tube sum equals 2^L * sum(s_L).
    rng = np.random.default_rng(3)
    p, L = 32, 3
    x = rng.standard_normal((p, 2, 2))
    c = orc.lift_fwd(x, L)
    m = p >> L
    for b in range(m):
        np.testing.assert_allclose(c[b], x[b * 8:(b + 1) * 8].mean(axis=0), atol=1e-15)
    np.testing.assert_allclose(x.sum(axis=0), (1 << L) * c[:m].sum(axis=0), atol=1e-13)


def test_constant_tube_has_zero_details():
    p, L = 16, 4
    x = np.repeat(np.array([[1.5, -2.0]])[None], p, axis=0)
    c = orc.lift_fwd(x, L)
    assert np.array_equal(c[0], x[0])
    assert not np.any(c[1:])


def test_level_zero_is_identity():
    x = np.random.default_rng(1).standard_normal((5, 3, 3))
    assert np.array_equal(orc.lift_fwd(x, 0), x)
    assert np.array_equal(orc.lift_inv(x, 0), x)
    assert np.array_equal(orc.lift_fwd_adj(x, 0), x)
    assert np.array_equal(orc.lift_inv_adj(x, 0), x)


@pytest.mark.parametrize("p,L", [(2, 1), (8, 3), (24, 3), (16, 4), (12, 2)])
def test_adjoints_match_dense_transposes(p, L):
    rng = np.random.default_rng(11)
    g = rng.standard_normal((p, 3, 4))
    np.testing.assert_allclose(orc.lift_fwd_adj(g, L), apply_mode3(dense_forward(p, L).T, g), atol=1e-13)
    np.testing.assert_allclose(orc.lift_inv_adj(g, L), apply_mode3(dense_inverse(p, L).T, g), atol=1e-13)


def test_adjoint_dot_product_identities():
    rng = np.random.default_rng(5)
    p, L = 32, 4
    x = rng.standard_normal((p, 6, 7))
    y = rng.standard_normal((p, 6, 7))
    lhs = np.sum(orc.lift_fwd(x, L) * y)
    rhs = np.sum(x * orc.lift_fwd_adj(y, L))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs) + 1e-12
    lhs = np.sum(orc.lift_inv(x, L) * y)
    rhs = np.sum(x * orc.lift_inv_adj(y, L))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs) + 1e-12


def test_transform_is_not_orthogonal_but_weighted_parseval_holds():
    # Remark 2.1: W is not orthogonal.  The exact energy identity has per-group weights.
    p, L = 16, 3
    w = dense_forward(p, L)
    assert not np.allclose(w @ w.T, np.eye(p))
    x = np.random.default_rng(9).standard_normal((p, 5, 4))
    c = orc.lift_fwd(x, L)
    wts = orc.coefficient_weights(p, L)
    e_spatial = np.sum(x * x)
    e_coeff = sum(wts[k] * np.sum(c[k] * c[k]) for k in range(p))
    assert abs(e_spatial - e_coeff) <= 1e-12 * e_spatial
    # the weights are the squared column norms of the closed-form inverse
    np.testing.assert_allclose(np.sum(dense_inverse(p, L) ** 2, axis=0), wts, atol=1e-14)


def test_transpose_invariance():
    # Thm 2.1: the transform commutes with the per-slice transpose.
    x = np.random.default_rng(2).standard_normal((16, 3, 5))
    np.testing.assert_array_equal(orc.lift_fwd(orc.transpose(x), 4), orc.transpose(orc.lift_fwd(x, 4)))
    np.testing.assert_array_equal(orc.lift_inv(orc.transpose(x), 4), orc.transpose(orc.lift_inv(x, 4)))


@pytest.mark.parametrize("p,L", [(6, 2), (0, 0), (8, -1), (12, 3)])
def test_rejects_bad_levels(p, L):
    with pytest.raises(ValueError):
        orc.check_levels(p, L)


def test_parseval_weights_of_the_test_helper():
    # The weights the GPU tests use to combine per-slice bars satisfy the
    # weighted Parseval identity with the oracle's transform, for every level.
    from gpu_helpers import parseval_weights
    rng = np.random.default_rng(17)
    for p, L in [(16, 0), (16, 1), (16, 4), (96, 5), (24, 3)]:
        x = rng.standard_normal((p, 3, 5))
        xh = orc.lift_fwd(x, L)
        w = parseval_weights(p, L)
        lhs = float(np.sum(x * x))
        rhs = float(np.sum(w * np.sum(xh * xh, axis=(1, 2))))
        assert abs(lhs - rhs) <= 1e-12 * lhs
