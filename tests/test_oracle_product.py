"""Pins of the oracle's face-product, w-product and its algebra (Def. 2.1-2.7, Thm 2.1-2.4)."""

import numpy as np
import pytest

import oracle as orc
from pins import load_golden, brute_w_product, dense_forward, apply_mode3

EX = load_golden("example_2_2.json")


def test_example_2_2_face_products_exact():
    ah = orc.lift_fwd(EX["A"], 2)
    bh = orc.lift_fwd(EX["B"], 2)
    ch = orc.face(ah, bh)
    assert np.array_equal(ch[0:1], EX["C_s2"])
    assert np.array_equal(ch[1:2], EX["C_d2"])
    assert np.array_equal(ch[2:4], EX["C_d1"])


def test_example_2_2_w_product_exact():
    assert np.array_equal(orc.w_product(EX["A"], EX["B"], 2), EX["C"])


def test_level_zero_is_batched_matmul():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((5, 4, 6))
    b = rng.standard_normal((5, 6, 3))
    np.testing.assert_allclose(orc.w_product(a, b, 0), np.matmul(a, b), atol=1e-14)


@pytest.mark.parametrize("p,L", [(2, 1), (4, 2), (8, 3), (6, 1), (8, 2)])
def test_brute_force_tiny(p, L):
    rng = np.random.default_rng(p + 10 * L)
    a = rng.standard_normal((p, 2, 3))
    b = rng.standard_normal((p, 3, 2))
    np.testing.assert_allclose(orc.w_product(a, b, L), brute_w_product(a, b, L), atol=1e-12)


def test_m_product_route():
    # The w-product is the transform-domain product for M = W_[L] (dense route).
    rng = np.random.default_rng(4)
    p, L = 16, 3
    a = rng.standard_normal((p, 5, 4))
    b = rng.standard_normal((p, 4, 3))
    w = dense_forward(p, L)
    ch = np.matmul(apply_mode3(w, a), apply_mode3(w, b))
    c = apply_mode3(np.linalg.inv(w), ch)
    np.testing.assert_allclose(orc.w_product(a, b, L), c, atol=1e-12)


def test_transpose_flags():
    rng = np.random.default_rng(8)
    a = rng.standard_normal((8, 4, 5))
    b = rng.standard_normal((8, 5, 3))
    ref = orc.w_product(a, b, 3)
    np.testing.assert_allclose(orc.w_product(orc.transpose(a), b, 3, trans_a=True), ref, atol=1e-13)
    np.testing.assert_allclose(orc.w_product(a, orc.transpose(b), 3, trans_b=True), ref, atol=1e-13)
    np.testing.assert_allclose(orc.w_product(orc.transpose(a), orc.transpose(b), 3, True, True), ref, atol=1e-13)


def test_transpose_reversal():
    # Thm 2.2: (A *_w B)^T = B^T *_w A^T.
    rng = np.random.default_rng(12)
    a = rng.standard_normal((16, 3, 4))
    b = rng.standard_normal((16, 4, 5))
    lhs = orc.transpose(orc.w_product(a, b, 4))
    rhs = orc.w_product(orc.transpose(b), orc.transpose(a), 4)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_associativity():
    # Thm 2.4.
    rng = np.random.default_rng(13)
    a = rng.standard_normal((16, 3, 4))
    b = rng.standard_normal((16, 4, 5))
    c = rng.standard_normal((16, 5, 2))
    lhs = orc.w_product(orc.w_product(a, b, 3), c, 3)
    rhs = orc.w_product(a, orc.w_product(b, c, 3), 3)
    np.testing.assert_allclose(lhs, rhs, atol=1e-11)


@pytest.mark.parametrize("p,L", [(2, 1), (8, 3), (16, 2)])
def test_identity(p, L):
    # Def. 2.3: A *_w I = I *_w A = A; the diagonal tube has the closed form
    # 1 + (L - 2 popcount(t mod 2^L)) / 2 (from the closed-form inverse).
    n = 4
    eye = orc.identity(n, p, L)
    for t in range(p):
        pop = bin(t % (1 << L)).count("1")
        np.testing.assert_allclose(eye[t], np.eye(n) * (1.0 + (L - 2 * pop) / 2.0), atol=1e-15)
    a = np.random.default_rng(1).standard_normal((p, n, n))
    np.testing.assert_allclose(orc.w_product(a, eye, L), a, atol=1e-13)
    np.testing.assert_allclose(orc.w_product(eye, a, L), a, atol=1e-13)


def test_inverse_and_reversal():
    # Def. 2.4, Lemma 2.3 and Thm 2.3.
    rng = np.random.default_rng(21)
    p, L, n = 8, 3, 4
    a = rng.standard_normal((p, n, n)) + 3 * np.eye(n)
    b = rng.standard_normal((p, n, n)) + 3 * np.eye(n)
    eye = orc.identity(n, p, L)
    ai = orc.inverse(a, L)
    np.testing.assert_allclose(orc.w_product(a, ai, L), eye, atol=1e-11)
    np.testing.assert_allclose(orc.w_product(ai, a, L), eye, atol=1e-11)
    np.testing.assert_allclose(orc.inverse(ai, L), a, atol=1e-11)
    lhs = orc.inverse(orc.w_product(a, b, L), L)
    rhs = orc.w_product(orc.inverse(b, L), ai, L)
    np.testing.assert_allclose(lhs, rhs, atol=1e-11)


def test_trace_properties():
    # Def. 2.7 and Lemma 2.5 (items 1-4); closed form Tr(C) = 2^L sum_k Tr(Chat_sL,k).
    rng = np.random.default_rng(31)
    p, L, n = 16, 3, 5
    a = rng.standard_normal((p, n, n))
    b = rng.standard_normal((p, n, n))
    assert abs(orc.trace(a) - orc.trace(orc.transpose(a))) < 1e-12
    assert abs(orc.trace(2 * a - 3 * b) - (2 * orc.trace(a) - 3 * orc.trace(b))) < 1e-11
    ab = orc.w_product(a, b, L)
    ba = orc.w_product(b, a, L)
    assert abs(orc.trace(ab) - orc.trace(ba)) < 1e-10
    assert abs(orc.trace(orc.w_product(orc.transpose(a), b, L))
               - orc.trace(orc.w_product(a, orc.transpose(b), L))) < 1e-10
    ch = orc.lift_fwd(ab, L)
    closed = (1 << L) * sum(np.trace(ch[k]) for k in range(p >> L))
    assert abs(orc.trace(ab) - closed) < 1e-10


def test_face_rejects_mismatched_slices():
    with pytest.raises(ValueError):
        orc.face(np.zeros((2, 2, 2)), np.zeros((3, 2, 2)))
