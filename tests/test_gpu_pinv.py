"""GPU parity of the Moore-Penrose inverse (Def. 2.6, Thm 2.6) and of the
pseudo-inverse deblurring (Sec. IV-C) against the FP64 oracle.

Tolerances: a pseudo-inverse computed from a backward-stable SVD has a
relative error of order kappa * eps (kappa the condition number of the kept
part of the slice); the bars below are max(n1, n2) * kappa * eps of the data
type, with kappa taken from the oracle's singular values.
"""

import numpy as np
import pytest

import oracle as orc
from gpu_helpers import device, to_dev, host, rel_fro
from pins import load_golden

pytestmark = pytest.mark.gpu

EPS64 = np.finfo(np.float64).eps
EPS32 = float(np.finfo(np.float32).eps)


@pytest.fixture(scope="module")
def wp():
    device()
    import paper_2601_08228_amd as wp
    return wp


def _kappa(a, L):
    """Largest condition number over the nonzero coefficient slices of W(A)."""
    kap = 1.0
    for sl in orc.lift_fwd(a, L):
        s = np.linalg.svd(sl, compute_uv=False)
        if s.size and s[0] > 0:
            kap = max(kap, s[0] / s[-1])
    return kap


@pytest.mark.parametrize("shape,L", [((16, 40, 24), 2), ((16, 24, 40), 2), ((8, 9, 9), 3),
                                     ((4, 130, 70), 1), ((2, 300, 20), 1), ((4, 1, 6), 2),
                                     ((2, 700, 650), 1), ((2, 45, 1500), 1)])
def test_pinv_f64_shapes(wp, shape, L):
    # Both orientations (n1 < n2 runs on the transpose), square, slices with
    # more than 128 rows (the block Jacobi kernel in FP64; 1500 rows take its
    # 8-column blocks), a single row.
    import torch
    a = np.random.default_rng(sum(shape)).standard_normal(shape)
    out, info = wp.w_pinv(to_dev(a, torch.float64), L)
    torch.cuda.synchronize()
    assert tuple(out.shape) == (shape[0], shape[2], shape[1])
    assert host(info).min() > 0
    tol = max(shape[1:]) * _kappa(a, L) * EPS64
    assert rel_fro(host(out), orc.w_pinv(a, L)) <= tol


def test_pinv_moore_penrose_conditions(wp):
    # Thm 2.6: A X A = A, X A X = X, (A X)^T = A X, (X A)^T = X A under *_w.
    import torch
    a = np.random.default_rng(70).standard_normal((8, 20, 12))
    x, _ = wp.w_pinv(to_dev(a, torch.float64), 3)
    x = host(x)
    ax = orc.w_product(a, x, 3)
    xa = orc.w_product(x, a, 3)
    assert rel_fro(orc.w_product(ax, a, 3), a) <= 1e-12
    assert rel_fro(orc.w_product(x, ax, 3), x) <= 1e-12
    assert rel_fro(np.transpose(ax, (0, 2, 1)), ax) <= 1e-12
    assert rel_fro(np.transpose(xa, (0, 2, 1)), xa) <= 1e-12


def test_pinv_rank_deficient_cut(wp):
    # Slices A_c = B_c C with C of rank 5: every coefficient slice has rank <= 5,
    # the values beyond the fifth are rounding noise, cut at rtol.
    import torch
    rng = np.random.default_rng(71)
    c = rng.standard_normal((5, 18))
    a = np.einsum("pir,rj->pij", rng.standard_normal((8, 30, 5)), c)
    rtol = 1e-9
    out, info = wp.w_pinv(to_dev(a, torch.float64), 2, rtol=rtol)
    torch.cuda.synchronize()
    assert host(info).min() > 0
    assert np.isfinite(host(out)).all()
    assert rel_fro(host(out), orc.w_pinv(a, 2, rtol=rtol)) <= 1e-10


def test_pinv_zero_and_identical_slices(wp):
    # Identical frontal slices: every detail coefficient slice is exactly zero
    # (its pseudo-inverse is zero) and A^+ repeats the slice pinv.
    import torch
    m = np.random.default_rng(72).standard_normal((12, 7))
    a = np.stack([m] * 8)
    out, _ = wp.w_pinv(to_dev(a, torch.float64), 3)
    np.testing.assert_allclose(host(out), np.stack([np.linalg.pinv(m)] * 8), atol=1e-12)
    z, _ = wp.w_pinv(to_dev(np.zeros((4, 5, 3)), torch.float64), 2)
    assert np.array_equal(host(z), np.zeros((4, 3, 5)))


@pytest.mark.parametrize("shape,L", [((16, 40, 24), 2), ((32, 20, 14), 3), ((8, 24, 40), 1)])
def test_sparse_pinv_f64(wp, shape, L):
    import torch
    a = np.random.default_rng(73 + L).standard_normal(shape)
    out, info = wp.w_pinv(to_dev(a, torch.float64), L, sparse=True)
    torch.cuda.synchronize()
    assert host(info).shape == (2 * (shape[0] >> L),)
    assert host(info).min() > 0
    tol = max(shape[1:]) * _kappa(a, L) * EPS64
    assert rel_fro(host(out), orc.w_pinv_sparse(a, L)) <= tol
    fine = orc.lift_fwd(host(out), L)[2 * (shape[0] >> L):]
    if fine.size:   # L = 1: s_1 and d_1 are all the coefficients
        assert np.abs(fine).max() <= 1e-14 * np.abs(host(out)).max()


def test_pinv_f32(wp):
    import torch
    a = np.random.default_rng(74).standard_normal((16, 64, 40)).astype(np.float32)
    out, info = wp.w_pinv(to_dev(a, torch.float32), 2)
    torch.cuda.synchronize()
    assert host(info).min() > 0
    a64 = a.astype(np.float64)
    tol = 64 * _kappa(a64, 2) * EPS32
    assert rel_fro(host(out), orc.w_pinv(a64, 2)) <= tol


@pytest.mark.parametrize("sparse", [False, True])
def test_pinv_deblur_matches_oracle(wp, sparse):
    # The blur of Sec. IV-C (b = 10) at a reduced spatial size, on an
    # HSI-like image; B = A_V * X * A_H^T is built by the oracle.
    import torch
    from paper_2601_08228_amd import synth, deblur
    p, n1, n2, L = 16, 40, 30, 2
    av = synth.stack_slices(synth.toeplitz_blur(n1, 10), p)
    ah = synth.stack_slices(synth.toeplitz_blur(n2, 10), p)
    x = synth.hsi_like(n1, n2, p, seed=75)
    bt = orc.w_product(orc.w_product(av, x, L), ah, L, trans_b=True)
    ref = orc.pinv_deblur(bt, av, ah, L, sparse=sparse)
    got, (iv, ih) = deblur.pinv_deblur(to_dev(bt, torch.float64), to_dev(av, torch.float64),
                                       to_dev(ah, torch.float64), L, sparse=sparse)
    torch.cuda.synchronize()
    assert host(iv).min() > 0 and host(ih).min() > 0
    kap = _kappa(av, L) + _kappa(ah, L)
    assert rel_fro(host(got), ref) <= max(n1, n2) * kap * EPS64


def test_pinv_deblur_salinas_shape_sampled(wp):
    # Salinas-sized problem (512 x 217 x 204, L = 2, b = 10) in FP64: the
    # pseudo-inverses checked on sampled slices against numpy's pinv of the
    # blur matrix (identical slices: A_V^+ repeats pinv(A_v)), and the
    # deblurred coefficients on sampled slices against a direct solve.
    import torch
    from paper_2601_08228_amd import synth, deblur
    p, n1, n2, L = 204, 512, 217, 2
    tv, th = synth.toeplitz_blur(n1, 10), synth.toeplitz_blur(n2, 10)
    av = torch.from_numpy(synth.stack_slices(tv, p)).cuda()
    ah = torch.from_numpy(synth.stack_slices(th, p)).cuda()
    for sparse in (False, True):
        pv, iv = wp.w_pinv(av, L, sparse=sparse)
        torch.cuda.synchronize()
        assert host(iv).min() > 0
        ref = np.linalg.pinv(tv)
        for c in (0, 101, 203):
            assert rel_fro(pv[c].cpu().numpy(), ref) <= n1 * _kappa(tv[None], 0) * EPS64
    # Deblurring of a seeded B (both blur matrices are invertible).
    b = torch.from_numpy(synth.normal((p, n1, n2), seed=76)).cuda()
    x, _ = deblur.pinv_deblur(b, av, ah, L, sparse=True)
    xs = x.cpu().numpy()
    bh = b.cpu().numpy()
    # With identical-slice blurs only the coarse coefficient s_L of B is seen:
    # X = W^{-1}(A_v^{-1} Bhat_{s_L} A_h^{-T}, 0, ...).  Check it on slices.
    bhat = orc.lift_fwd(bh, L)
    xhat = orc.lift_fwd(xs, L)
    kap = _kappa(tv[None], 0) + _kappa(th[None], 0)
    for c in (0, 25, 50):
        want = np.linalg.solve(tv, np.linalg.solve(th, bhat[c].T).T)
        assert rel_fro(xhat[c], want) <= max(n1, n2) * kap * EPS64
    assert np.abs(xhat[p >> L:]).max() <= 1e-12 * np.abs(xhat).max()


def test_pinv_botswana_shape_sampled(wp):
    # Botswana-sized blur (1476 x 1476 per slice, the 8-column-block path of
    # the block Jacobi), 144 bands, L = 4, sparse: the kept s_4 slices of A_V^+
    # equal numpy's pinv of the blur matrix, the dropped details are zero.
    import torch
    from paper_2601_08228_amd import synth
    p, n, L = 144, 1476, 4
    tv = synth.toeplitz_blur(n, 10)
    av = torch.from_numpy(synth.stack_slices(tv, p)).cuda()
    pv, iv = wp.w_pinv(av, L, sparse=True)
    torch.cuda.synchronize()
    assert host(iv).min() > 0
    ref = np.linalg.pinv(tv)
    tol = n * _kappa(tv[None], 0) * EPS64
    for c in (0, 77, 143):
        assert rel_fro(pv[c].cpu().numpy(), ref) <= tol


def test_remark_2_2_printed_values(wp):
    # The example after Remark 2.2: (A *_w B)^+ and B^+ *_w A^+ for A (2x3x2),
    # B (3x2x2), L = 1, computed on the GPU (FP64) against the printed tensors
    # C and D; B's detail slice has rank 1 (one singular value cut).
    import torch
    rm = load_golden("remark_2_2.json")
    a, b = to_dev(rm["A"], torch.float64), to_dev(rm["B"], torch.float64)
    c, _ = wp.w_pinv(wp.w_product(a, b, 1), 1)
    ap, _ = wp.w_pinv(a, 1)
    bp, _ = wp.w_pinv(b, 1)
    d = wp.w_product(bp, ap, 1)
    np.testing.assert_allclose(host(c), rm["C"], atol=1e-12)
    np.testing.assert_allclose(host(d), rm["D"], atol=1e-12)
    np.testing.assert_allclose(host(wp.w_transform(ap, 1))[0], rm["Apinv_s"], atol=1e-12)
    np.testing.assert_allclose(host(wp.w_transform(bp, 1))[1], rm["Bpinv_d"], atol=1e-12)
