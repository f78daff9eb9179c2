"""Pins of the oracle's w-svd (Alg. 2, Thm 2.5) and Moore-Penrose inverse (Def. 2.6, Remark 2.2)."""

import numpy as np
import pytest

import oracle as orc
from pins import load_golden

RM = load_golden("remark_2_2.json")


def test_slice_svd_matches_gram_eigenvalues():
    # A second library route: the squared singular values are the eigenvalues of M^T M.
    rng = np.random.default_rng(2)
    for shape in [(6, 4), (5, 5), (7, 3)]:
        m = rng.standard_normal(shape)
        u, s, v = orc.slice_svd(m)
        ev = np.sort(np.linalg.eigvalsh(m.T @ m))[::-1]
        np.testing.assert_allclose(s ** 2, ev, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose((u * s) @ v.T, m, atol=1e-13)
        for i in range(s.size):
            assert u[np.argmax(np.abs(u[:, i])), i] > 0


@pytest.mark.parametrize("p,L,n1,n2", [(16, 2, 8, 6), (8, 3, 5, 7), (4, 1, 6, 6)])
def test_full_rank_reconstruction_and_orthogonality(p, L, n1, n2):
    # Thm 2.5 with r = min(n1, n2): A = U *_w Sigma *_w V^T exactly, and U^T *_w U = I_r.
    rng = np.random.default_rng(p + n1)
    a = rng.standard_normal((p, n1, n2))
    r = min(n1, n2)
    uh, sh, vh, ak = orc.w_svd(a, L, r)
    np.testing.assert_allclose(ak, a, atol=1e-12)
    u, sig, v = orc.spatial_factors(uh, sh, vh, L)
    usv = orc.w_product(orc.w_product(u, sig, L), orc.transpose(v), L)
    np.testing.assert_allclose(usv, a, atol=1e-11)
    eye = orc.identity(r, p, L)
    np.testing.assert_allclose(orc.w_product(orc.transpose(u), u, L), eye, atol=1e-12)
    np.testing.assert_allclose(orc.w_product(orc.transpose(v), v, L), eye, atol=1e-12)
    assert np.all(np.diff(sh, axis=1) <= 0) and np.all(sh >= 0)


@pytest.mark.parametrize("k", [1, 2, 4])
def test_truncation_error_weighted_parseval(k):
    # ||A - A_k||_F^2 = sum_c w_c sum_{i>k} sigma_{c,i}^2, with the weights of the
    # closed-form inverse (2^L on s_L, 2^j / 4 on d_j).  The unweighted bound of
    # Thm 2.5 does not hold for this non-orthogonal transform (Remark 2.1).
    rng = np.random.default_rng(40 + k)
    p, L = 16, 3
    a = rng.standard_normal((p, 7, 6))
    _, _, _, ak = orc.w_svd(a, L, k)
    ah = orc.lift_fwd(a, L)
    wts = orc.coefficient_weights(p, L)
    tail = 0.0
    for c in range(p):
        s = np.linalg.svd(ah[c], compute_uv=False)
        tail += wts[c] * np.sum(s[k:] ** 2)
    err = np.sum((a - ak) ** 2)
    assert abs(err - tail) <= 1e-11 * tail


def test_theorem_2_5_unweighted_bound_counterexample():
    # p = 2, L = 1, both slices I_2, r = 1: true error sqrt(2) exceeds the printed bound 1.
    a = np.stack([np.eye(2), np.eye(2)])
    _, _, _, ak = orc.w_svd(a, 1, 1)
    err = np.linalg.norm((a - ak).ravel())
    assert abs(err - np.sqrt(2.0)) < 1e-14


def test_remark_2_2_values():
    L = 1
    a, b = RM["A"], RM["B"]
    ah = orc.lift_fwd(a, L)
    bh = orc.lift_fwd(b, L)
    np.testing.assert_allclose(ah[0], RM["A_s"], atol=1e-15)
    np.testing.assert_allclose(ah[1], RM["A_d"], atol=1e-15)
    np.testing.assert_allclose(bh[0], RM["B_s"], atol=1e-15)
    np.testing.assert_allclose(bh[1], RM["B_d"], atol=1e-15)
    ab = orc.w_product(a, b, L)
    abh = orc.lift_fwd(ab, L)
    np.testing.assert_allclose(abh[0], RM["AB_s"], atol=1e-14)
    np.testing.assert_allclose(abh[1], RM["AB_d"], atol=1e-14)
    c = orc.w_pinv(ab, L)
    ch = orc.lift_fwd(c, L)
    np.testing.assert_allclose(ch[0], RM["C_s"], atol=1e-12)
    np.testing.assert_allclose(ch[1], RM["C_d"], atol=1e-12)
    np.testing.assert_allclose(c, RM["C"], atol=1e-12)
    ap = orc.w_pinv(a, L)
    bp = orc.w_pinv(b, L)
    aph = orc.lift_fwd(ap, L)
    bph = orc.lift_fwd(bp, L)
    np.testing.assert_allclose(aph[0], RM["Apinv_s"], atol=1e-12)
    np.testing.assert_allclose(aph[1], RM["Apinv_d"], atol=1e-12)
    np.testing.assert_allclose(bph[0], RM["Bpinv_s"], atol=1e-12)
    np.testing.assert_allclose(bph[1], RM["Bpinv_d"], atol=1e-12)
    d = orc.w_product(bp, ap, L)
    dh = orc.lift_fwd(d, L)
    np.testing.assert_allclose(dh[0], RM["D_s"], atol=1e-12)
    np.testing.assert_allclose(dh[1], RM["D_d"], atol=1e-12)
    np.testing.assert_allclose(d, RM["D"], atol=1e-12)
    assert not np.allclose(c, d)


def _penrose(a, x, L):
    axa = orc.w_product(orc.w_product(a, x, L), a, L)
    xax = orc.w_product(orc.w_product(x, a, L), x, L)
    ax = orc.w_product(a, x, L)
    xa = orc.w_product(x, a, L)
    return axa, xax, ax, xa


@pytest.mark.parametrize("shape,L", [((8, 4, 6), 3), ((16, 5, 3), 2), ((4, 6, 6), 2)])
def test_moore_penrose_conditions(shape, L):
    # Def. 2.6: the four conditions hold for the per-slice construction (Thm 2.6).
    rng = np.random.default_rng(sum(shape))
    a = rng.standard_normal(shape)
    a[:, :, -1] = a[:, :, 0]          # make slices rank deficient as well
    x = orc.w_pinv(a, L)
    axa, xax, ax, xa = _penrose(a, x, L)
    np.testing.assert_allclose(axa, a, atol=1e-11)
    np.testing.assert_allclose(xax, x, atol=1e-11)
    np.testing.assert_allclose(orc.transpose(ax), ax, atol=1e-11)
    np.testing.assert_allclose(orc.transpose(xa), xa, atol=1e-11)


def test_moore_penrose_properties():
    # Lemma 2.4 items 1-4.
    rng = np.random.default_rng(77)
    p, L = 8, 2
    a = rng.standard_normal((p, 4, 6))
    ap = orc.w_pinv(a, L)
    np.testing.assert_allclose(orc.w_pinv(ap, L), a, atol=1e-10)
    np.testing.assert_allclose(orc.w_pinv(orc.transpose(a), L), orc.transpose(ap), atol=1e-10)
    aat = orc.w_product(a, orc.transpose(a), L)
    np.testing.assert_allclose(orc.w_pinv(aat, L),
                               orc.w_product(orc.w_pinv(orc.transpose(a), L), ap, L), atol=1e-10)
    np.testing.assert_allclose(ap, orc.w_product(orc.transpose(a), orc.w_pinv(aat, L), L), atol=1e-10)


def test_w_svd_rejects_bad_rank():
    with pytest.raises(ValueError):
        orc.w_svd(np.zeros((2, 3, 3)), 1, 4)
    with pytest.raises(ValueError):
        orc.w_svd(np.zeros((2, 3, 3)), 1, 0)


def test_psnr_definition():
    x = np.zeros((2, 3, 4))
    y = x.copy()
    y[0, 0, 0] = 0.1
    # N = 24 samples, squared error 0.01 -> 10 log10(24 / 0.01)
    assert abs(orc.psnr(x, y) - 10 * np.log10(2400.0)) < 1e-12


def test_sparse_w_svd_equals_w_svd_at_one_level():
    # With L = 1 the kept slices s_1 and d_1 are all p coefficients.
    a = np.random.default_rng(50).standard_normal((8, 6, 5))
    full = orc.w_svd(a, 1, 3)
    sp = orc.w_svd_sparse(a, 1, 3)
    for x, y in zip(full, sp):
        np.testing.assert_allclose(x, y, atol=1e-13)


def test_sparse_w_svd_exact_on_tensors_without_fine_details():
    # Tubes constant on pairs of slices have d_1 = 0; at L = 2 sp-w-svd then keeps
    # everything there is, so it equals the full w-svd.
    rng = np.random.default_rng(51)
    half = rng.standard_normal((8, 7, 6))
    a = np.repeat(half, 2, axis=0)            # slices 2q and 2q+1 equal
    assert not np.any(orc.lift_fwd(a, 2)[8:])  # d_1 occupies slices [p/2, p)
    _, _, _, ak_full = orc.w_svd(a, 2, 4)
    _, _, _, ak_sp = orc.w_svd_sparse(a, 2, 4)
    np.testing.assert_allclose(ak_sp, ak_full, atol=1e-12)


def test_sparse_w_svd_error_identity():
    # ||A - A_k||^2 = sum over kept slices of w_c * (tail singular energy)
    #                 + sum over dropped slices of w_c * ||Ahat_c||^2.
    rng = np.random.default_rng(52)
    p, L, k = 32, 3, 2
    a = rng.standard_normal((p, 6, 5))
    _, _, _, ak = orc.w_svd_sparse(a, L, k)
    ah = orc.lift_fwd(a, L)
    w = orc.coefficient_weights(p, L)
    kept = 2 * (p >> L)
    expect = 0.0
    for c in range(p):
        if c < kept:
            s = np.linalg.svd(ah[c], compute_uv=False)
            expect += w[c] * np.sum(s[k:] ** 2)
        else:
            expect += w[c] * np.sum(ah[c] ** 2)
    err = np.sum((a - ak) ** 2)
    assert abs(err - expect) <= 1e-11 * expect


def test_sparse_w_svd_rejects_level_zero():
    with pytest.raises(ValueError):
        orc.w_svd_sparse(np.zeros((4, 3, 3)), 0, 1)


# ---- pseudo-inverse deblurring (Sec. IV-C) -------------------------------------

def test_toeplitz_blur_entries():
    # b = 3: first row 1/3, 2/9, 1/9, 0, ... (c(j) = (b - j) / (3b)), symmetric.
    t = orc.toeplitz_blur(5, 3)
    np.testing.assert_allclose(t[0], [1 / 3, 2 / 9, 1 / 9, 0, 0], atol=1e-15)
    np.testing.assert_allclose(t[2], [1 / 9, 2 / 9, 1 / 3, 2 / 9, 1 / 9], atol=1e-15)
    np.testing.assert_array_equal(t, t.T)


def test_input_generator_blur_matches_the_oracle():
    # The seeded input module builds the same blur as the oracle's definition.
    from paper_2601_08228_amd import synth
    for n, b in ((5, 3), (40, 10), (17, 1)):
        np.testing.assert_array_equal(synth.toeplitz_blur(n, b), orc.toeplitz_blur(n, b))


def test_sparse_pinv_is_pinv_without_fine_details():
    # Identical frontal slices have no detail coefficients at all; the sparse and
    # full pseudo-inverses then agree, and both equal the slice pinv repeated.
    rng = np.random.default_rng(60)
    m = rng.standard_normal((6, 4))
    a = np.stack([m] * 8)
    full = orc.w_pinv(a, 2)
    sp = orc.w_pinv_sparse(a, 2)
    np.testing.assert_allclose(sp, full, atol=1e-12)
    np.testing.assert_allclose(full, np.stack([np.linalg.pinv(m)] * 8), atol=1e-12)


def test_sparse_pinv_keeps_only_coarse_blocks():
    rng = np.random.default_rng(61)
    a = rng.standard_normal((16, 5, 5))
    sp_hat = orc.lift_fwd(orc.w_pinv_sparse(a, 2), 2)
    full_hat = orc.lift_fwd(orc.w_pinv(a, 2), 2)
    np.testing.assert_allclose(sp_hat[:8], full_hat[:8], atol=1e-12)   # s_2 and d_2
    assert np.abs(sp_hat[8:]).max() <= 1e-14 * np.abs(full_hat).max()  # d_1 dropped


def test_pinv_deblur_recovers_the_coarse_part():
    # With invertible slice blurs, A_V *_w X *_w A_H^T keeps only s_L of X (the
    # blur tensors have no detail coefficients) and the deblurring returns
    # exactly that coarse part: W^{-1}(Xhat_{s_L}, 0, ..., 0).
    rng = np.random.default_rng(62)
    p, n1, n2, L = 8, 7, 5, 2
    av = np.stack([np.eye(n1) + 0.2 * rng.standard_normal((n1, n1))] * p)
    ah = np.stack([np.eye(n2) + 0.2 * rng.standard_normal((n2, n2))] * p)
    x = rng.standard_normal((p, n1, n2))
    bt = orc.w_product(orc.w_product(av, x, L), ah, L, trans_b=True)
    xh = orc.lift_fwd(x, L)
    xh[p >> L:] = 0
    coarse = orc.lift_inv(xh, L)
    for sparse in (False, True):
        np.testing.assert_allclose(orc.pinv_deblur(bt, av, ah, L, sparse), coarse, atol=1e-11)


def test_pinv_deblur_is_least_squares():
    # For general (slice-varying) operators the deblurred X satisfies the normal
    # equations slice by slice in the wavelet domain: A^T (A X B^T - Y) B = 0.
    rng = np.random.default_rng(63)
    p, n1, n2, L = 4, 6, 4, 1
    av = rng.standard_normal((p, n1 + 2, n1))     # tall: full column rank
    ah = rng.standard_normal((p, n2 + 1, n2))
    y = rng.standard_normal((p, n1 + 2, n2 + 1))
    x = orc.w_product(orc.w_product(orc.w_pinv(av, L), y, L), orc.w_pinv(ah, L), L, trans_b=True)
    r = orc.w_product(orc.w_product(av, x, L), ah, L, trans_b=True) - y
    g = orc.w_product(orc.w_product(av, r, L, trans_a=True), ah, L)
    assert np.abs(g).max() <= 1e-10 * np.abs(y).max()
