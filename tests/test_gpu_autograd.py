"""GPU parity of the hand-written adjoint (torch.autograd.Function) and the deblurring solve."""

import numpy as np
import pytest

import oracle as orc
from gpu_helpers import device, to_dev, host, cast, rel_fro

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wp():
    device()
    import paper_2601_08228_amd as wp
    return wp


def test_gradcheck_fp64_crop(wp):
    # Central finite differences in FP64 on the 16x16x8 crop of the deblurring
    # problem: K = 8 copies of the 16x16 Gaussian band, X[:8, :16, :16].
    import torch
    from paper_2601_08228_amd import synth
    k = synth.stack_slices(synth.gaussian_band(16), 8)
    x = synth.hsi_like(16, 16, 8, seed=5)
    tk = to_dev(k, torch.float64).requires_grad_(True)
    tx = to_dev(x, torch.float64).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: wp.w_product_ad(a, b, 3), (tk, tx),
                                    eps=1e-6, atol=1e-8, rtol=1e-6)


@pytest.mark.parametrize("gemm,tol", [("native", 1e-5), ("bf16x3", 1e-5), ("bf16", 1e-2)])
def test_vjp_f32_vs_oracle(wp, gemm, tol):
    import torch
    rng = np.random.default_rng(3)
    p, L = 32, 4
    a = cast(rng.standard_normal((p, 96, 80)), np.float32)
    b = cast(rng.standard_normal((p, 80, 72)), np.float32)
    g = cast(rng.standard_normal((p, 96, 72)), np.float32)
    ta = to_dev(a, torch.float32).requires_grad_(True)
    tb = to_dev(b, torch.float32).requires_grad_(True)
    c = wp.w_product_ad(ta, tb, L, gemm)
    c.backward(to_dev(g, torch.float32))
    da, db = orc.w_product_vjp(a, b, g, L)
    assert rel_fro(host(c), orc.w_product(a, b, L)) <= tol
    assert rel_fro(host(ta.grad), da) <= tol
    assert rel_fro(host(tb.grad), db) <= tol


def test_vjp_f64_vs_oracle(wp):
    import torch
    rng = np.random.default_rng(4)
    p, L = 16, 3
    a, b, g = (rng.standard_normal(s) for s in [(p, 40, 30), (p, 30, 20), (p, 40, 20)])
    ta = to_dev(a, torch.float64).requires_grad_(True)
    tb = to_dev(b, torch.float64).requires_grad_(True)
    wp.w_product_ad(ta, tb, L).backward(to_dev(g, torch.float64))
    da, db = orc.w_product_vjp(a, b, g, L)
    assert rel_fro(host(ta.grad), da) <= 1e-12
    assert rel_fro(host(tb.grad), db) <= 1e-12


def test_only_requested_gradients(wp):
    import torch
    a = to_dev(np.ones((4, 3, 3)), torch.float64).requires_grad_(True)
    b = to_dev(np.ones((4, 3, 3)), torch.float64)
    wp.w_product_ad(a, b, 2).sum().backward()
    assert a.grad is not None and b.grad is None


def _deblur_problem(n, p, seed):
    from paper_2601_08228_amd import synth
    g = synth.gaussian_band(n)
    k = cast(synth.stack_slices(g, p), np.float32)
    x = synth.hsi_like(n, n, p, seed=seed)
    noise = synth.normal((p, n, n), seed=seed + 100, scale=0.01)
    y = cast(orc.w_product(k, x, 3) + noise, np.float32)
    eta = 1.0 / (2.0 * np.linalg.norm(g, 2) ** 2)
    return k, x, y, eta


def test_deblur_gradient_full_size(wp):
    # 256x256x128 blur operator and hyperspectral-like tensor: the FP32 gradient at a
    # nonzero point against the oracle gradient (<= 1e-5).
    import torch
    from paper_2601_08228_amd import deblur
    k, x, y, _ = _deblur_problem(256, 128, seed=5)
    x0 = cast(0.5 * x, np.float32)
    grad = deblur.lsq_gradient(to_dev(k, torch.float32), to_dev(x0, torch.float32),
                               to_dev(y, torch.float32), 3)
    assert rel_fro(host(grad), orc.lsq_grad(k, x0, y, 3)) <= 1e-5


@pytest.mark.parametrize("gemm", ["native", "bf16x3"])
def test_deblur_trajectory(wp, gemm):
    # 50 fixed-step iterations at 64x64x128 (the full 256x256 trajectory is in the
    # benchmark); iterate and loss curve against the oracle trajectory.
    import torch
    from paper_2601_08228_amd import deblur
    k, x, y, eta = _deblur_problem(64, 128, seed=6)
    xs, losses = deblur.solve(to_dev(k, torch.float32), to_dev(y, torch.float32), 3, steps=50,
                              eta=eta, gemm=gemm)
    x_ref, loss_ref = orc.deblur_gd(k, y, 3, 50, eta)
    assert rel_fro(host(xs), x_ref) <= 1e-5
    np.testing.assert_allclose(losses, loss_ref[:len(losses)], rtol=1e-4)
    assert losses[-1] < losses[0]


@pytest.mark.parametrize("gemm", ["native", "bf16x3"])
def test_graphed_solve_matches_eager_every_replay(wp, gemm):
    # The captured step, replayed with eager steps and synchronisations in
    # between, gives the eager iterate bit for bit after every replay (same
    # kernels in the same order), and the loss still falls.
    import torch
    from paper_2601_08228_amd import deblur
    from paper_2601_08228_amd.autograd import WProduct
    k, x, y, eta = _deblur_problem(32, 64, seed=7)
    tk, ty = to_dev(k, torch.float32), to_dev(y, torch.float32)
    solver = deblur.GraphedSolver(tk, ty, 3, eta, gemm=gemm)
    xe = torch.zeros_like(ty)
    loss0 = solver.residual_norm2()
    for step in range(6):
        solver.run(1)
        xv = xe.clone().requires_grad_(True)
        c = WProduct.apply(tk, xv, 3, gemm)
        (g,) = torch.autograd.grad(c, xv, grad_outputs=2.0 * (c - ty))
        xe = (xv - eta * g).detach()
        torch.cuda.synchronize()
        assert torch.equal(solver.x.detach(), xe), step
    assert solver.residual_norm2() < loss0


@pytest.mark.parametrize("gemm", ["native", "bf16x3"])
def test_full_size_backward_512x512x256_sampled(wp, gemm):
    # The benchmark's forward + backward (A, B 512x512x256 N(0,1), L = 4,
    # cotangent N(0,1)): sampled rows of dA = G *_w B^T and sampled columns of
    # dB = A^T *_w G against the oracle's derivative restricted to those rows /
    # columns (a row of dA needs only that row of G, a column of dB only that
    # column of G).
    import torch
    from paper_2601_08228_amd import synth
    dev = device()
    a = synth.normal_device((256, 512, 512), 21, dev)
    b = synth.normal_device((256, 512, 512), 22, dev)
    g = synth.normal_device((256, 512, 512), 102, dev)
    ta = a.clone().requires_grad_(True)
    tb = b.clone().requires_grad_(True)
    wp.w_product_ad(ta, tb, 4, gemm).backward(g)
    torch.cuda.synchronize()
    a_h, b_h, g_h = (host(t).astype(np.float64) for t in (a, b, g))
    da, db = host(ta.grad).astype(np.float64), host(tb.grad).astype(np.float64)
    rng = np.random.default_rng(8)
    got, ref = [], []
    for i in rng.integers(0, 512, 4):
        da_i, _ = orc.w_product_vjp(a_h[:, i:i + 1, :], b_h, g_h[:, i:i + 1, :], 4)
        got.append(da[:, i, :])
        ref.append(da_i[:, 0, :])
    assert rel_fro(np.array(got), np.array(ref)) <= 1e-5
    got, ref = [], []
    for j in rng.integers(0, 512, 4):
        _, db_j = orc.w_product_vjp(a_h, b_h[:, :, j:j + 1], g_h[:, :, j:j + 1], 4)
        got.append(db[:, :, j])
        ref.append(db_j[:, :, 0])
    assert rel_fro(np.array(got), np.array(ref)) <= 1e-5


@pytest.fixture(scope="module")
def deblur_full():
    # The deblurring workload at its stated size (256x256x128, L = 3) and the
    # oracle's 50-step trajectory, computed once for both face-product modes.
    k, x, y, eta = _deblur_problem(256, 128, seed=5)
    x_ref, loss_ref = orc.deblur_gd(k, y, 3, 50, eta)
    return k, y, eta, x_ref, loss_ref


@pytest.mark.parametrize("gemm", ["native", "bf16x3"])
def test_deblur_trajectory_full_size(wp, deblur_full, gemm):
    import torch
    from paper_2601_08228_amd import deblur
    k, y, eta, x_ref, loss_ref = deblur_full
    xs, losses = deblur.solve(to_dev(k, torch.float32), to_dev(y, torch.float32), 3, steps=50,
                              eta=eta, gemm=gemm)
    assert rel_fro(host(xs), x_ref) <= 1e-5
    np.testing.assert_allclose(losses, loss_ref[:len(losses)], rtol=1e-4)
    assert losses[-1] < losses[0]
