"""GPU parity of the w-svd (Alg. 2, Thm 2.5) against the FP64 oracle."""

import numpy as np
import pytest

import oracle as orc
from gpu_helpers import device, to_dev, host, cast, rel_fro, svd_bars, UNIT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wp():
    device()
    import paper_2601_08228_amd as wp
    return wp


def _check_factors(res, a_coeff, k, bars, prec="f64"):
    """uhat diag(shat) vhat^T against the oracle's rank-k rebuild, slice by slice,
    each slice within its own derived rank-k bar; every sigma within the Weyl
    bar 4 mr u sigma_1 of its slice."""
    uh, sh, vh = host(res.uhat), host(res.shat), host(res.vhat)
    mr = max(a_coeff.shape[1:])
    for c in range(a_coeff.shape[0]):
        u, s, v = orc.slice_svd(a_coeff[c])
        np.testing.assert_allclose(sh[c], s[:k], rtol=0, atol=4 * mr * UNIT[prec] * s[0])
        rebuilt = (uh[c] * sh[c]) @ vh[c].T
        ref = (u[:, :k] * s[:k]) @ v[:, :k].T
        assert rel_fro(rebuilt, ref) <= bars["ak_slice"][c], (c, rel_fro(rebuilt, ref))


def test_config1_f64_full_rank(wp):
    # A 32x24x16 N(0,1), L = 2, full rank 24: A = U *_w S *_w V^T to 1e-12.
    import torch
    from paper_2601_08228_amd import synth
    a = synth.normal((16, 32, 24), seed=1)
    res = wp.w_svd(to_dev(a, torch.float64), 2, 24)
    torch.cuda.synchronize()
    info = host(res.info)
    assert info.min() > 0
    coeff = orc.lift_fwd(a, 2)
    bars = svd_bars(coeff, 24, "f64", L=2)
    assert bars["ak"] == 1e-12 and bars["shat"] == 1e-12
    assert rel_fro(host(res.ak), a) <= 1e-12
    _, sh_ref, _, _ = orc.w_svd(a, 2, 24)
    assert rel_fro(host(res.shat), sh_ref) <= bars["shat"]
    assert host(res.orth_err).max() <= bars["orth"]
    _check_factors(res, coeff, 24, bars)


# Register-resident kernel: both orientations (n1 < n2 runs on the transpose),
# odd column counts (a zero tournament column), 1 and 2 columns, rows spanning
# several lanes.  Block kernel: more than 128 rows (FP64).  Every bar is
# derived from the oracle's singular values of the coefficient slices.
@pytest.mark.parametrize("shape,k", [((8, 10, 20), 5), ((16, 21, 13), 7), ((4, 9, 9), 9),
                                     ((8, 65, 40), 3), ((2, 3, 70), 1), ((32, 7, 7), 4),
                                     ((4, 5, 1), 1), ((4, 2, 6), 2), ((8, 130, 100), 10),
                                     ((4, 300, 40), 6), ((2, 24, 520), 5)])
def test_f64_shapes(wp, shape, k):
    import torch
    p, n1, n2 = shape
    L = 2 if p % 4 == 0 else 1
    a = np.random.default_rng(n1 * n2).standard_normal(shape)
    res = wp.w_svd(to_dev(a, torch.float64), L, k)
    torch.cuda.synchronize()
    assert host(res.info).min() > 0
    _, sh_ref, _, ak_ref = orc.w_svd(a, L, k)
    coeff = orc.lift_fwd(a, L)
    bars = svd_bars(coeff, k, "f64", L=L)
    assert rel_fro(host(res.shat), sh_ref) <= bars["shat"]
    assert rel_fro(host(res.ak), ak_ref) <= bars["ak"]
    assert host(res.orth_err).max() <= bars["orth"]
    _check_factors(res, coeff, k, bars)
    # sign convention: largest-magnitude entry of every U column is positive
    uh = host(res.uhat)
    idx = np.argmax(np.abs(uh), axis=1)
    assert np.all(np.take_along_axis(uh, idx[:, None, :], axis=1) > 0)


def test_config3_hsi_f32(wp):
    # 256x256x192 hyperspectral-like tensor (12 components, noise 0.01), L = 3, k = 20.
    import torch
    from paper_2601_08228_amd import synth
    x = cast(synth.hsi_like(256, 256, 192, seed=3), np.float32)
    res = wp.w_svd(to_dev(x, torch.float32), 3, 20)
    torch.cuda.synchronize()
    info = host(res.info)
    assert info.min() > 0, info
    _, sh_ref, _, ak_ref = orc.w_svd(x, 3, 20)
    ak = host(res.ak)
    # The stated target of this workload (1e-5) is held directly; the derived
    # orthogonality bar applies to both factors.
    assert rel_fro(host(res.shat), sh_ref) <= 1e-5
    assert rel_fro(ak, ak_ref) <= 1e-5
    assert abs(orc.psnr(x, ak) - orc.psnr(x, ak_ref)) <= 0.01
    assert host(res.orth_err).max() <= svd_bars(orc.lift_fwd(x, 3)[:2], 20, "f32")["orth"]


def test_nonconvergence_is_reported(wp):
    # One sweep is not enough for a random 64x48 slice: info < 0, nothing hangs.
    import torch
    a = np.random.default_rng(1).standard_normal((4, 64, 48))
    res = wp.w_svd(to_dev(a, torch.float64), 2, 5, max_sweeps=1)
    torch.cuda.synchronize()
    assert np.all(host(res.info) == -1)


def test_nonfinite_input_terminates(wp):
    import torch
    a = np.random.default_rng(2).standard_normal((4, 16, 12))
    a[1, 3, 4] = np.nan
    res = wp.w_svd(to_dev(a, torch.float64), 1, 3)
    torch.cuda.synchronize()
    info = host(res.info)
    # slice 1 is mixed into coefficient slices 0 (s_1) and 2 (d_1)
    assert info[0] < 0 and info[2] < 0
    assert info[1] > 0 and info[3] > 0


def test_block_kernel_nonconvergence_is_reported(wp):
    # The block kernel (300 rows in FP64) with a one-sweep limit: info = -1 for
    # every slice, and the call returns.
    import torch
    a = np.random.default_rng(3).standard_normal((4, 300, 80))
    res = wp.w_svd(to_dev(a, torch.float64), 2, 5, max_sweeps=1)
    torch.cuda.synchronize()
    assert np.all(host(res.info) == -1)


def test_block_kernel_nonfinite_input_terminates(wp):
    import torch
    a = np.random.default_rng(4).standard_normal((4, 300, 70))
    a[1, 100, 7] = np.inf
    res = wp.w_svd(to_dev(a, torch.float64), 1, 3)
    torch.cuda.synchronize()
    info = host(res.info)
    assert info[0] < 0 and info[2] < 0          # the coefficient slices that mix slice 1
    assert info[1] > 0 and info[3] > 0


def test_block_kernel_zero_slices(wp):
    # Identical frontal slices: the detail coefficient slices are zero, skipped
    # by the block kernel (one sweep, converged), with zero singular values.
    import torch
    m = np.random.default_rng(5).standard_normal((300, 70))
    a = np.stack([m] * 4)
    res = wp.w_svd(to_dev(a, torch.float64), 2, 6)
    torch.cuda.synchronize()
    info, sh = host(res.info), host(res.shat)
    assert info.min() > 0 and np.all(info[1:] == 1)
    assert np.all(sh[1:] == 0)
    np.testing.assert_allclose(sh[0], np.linalg.svd(m, compute_uv=False)[:6], rtol=1e-12)
    assert rel_fro(host(res.ak), orc.w_svd(a, 2, 6)[3]) <= 1e-12


@pytest.mark.parametrize("shape,k", [((16, 100, 60), 10), ((8, 33, 64), 8), ((4, 256, 256), 20),
                                     ((4, 600, 300), 20), ((4, 1200, 90), 12)])
def test_f32_shapes(wp, shape, k):
    # (4, 600, 300): the recovered factor has 300 rows, (4, 1200, 90) 90 rows
    # of a 1200-row slice; both are polished like any other.
    import torch
    p, n1, n2 = shape
    L = 2
    a = cast(np.random.default_rng(n1 + n2).standard_normal(shape), np.float32)
    res = wp.w_svd(to_dev(a, torch.float32), L, k)
    torch.cuda.synchronize()
    assert host(res.info).min() > 0
    _, sh_ref, _, ak_ref = orc.w_svd(a, L, k)
    coeff = orc.lift_fwd(a, L)
    bars = svd_bars(coeff, k, "f32", L=L)
    assert rel_fro(host(res.shat), sh_ref) <= bars["shat"]
    assert rel_fro(host(res.ak), ak_ref) <= bars["ak"]
    assert host(res.orth_err).max() <= bars["orth"]
    _check_factors(res, coeff, k, bars, "f32")


def _gapped(p, n1, n2, k, seed, lead=10.0):
    """Slices with a prescribed spectrum: k values in [lead/2, lead], the rest in
    [0.05, 0.5], random orthogonal factors (test input, built with numpy QR)."""
    rng = np.random.default_rng(seed)
    nc = min(n1, n2)
    out = np.empty((p, n1, n2))
    for c in range(p):
        q1, _ = np.linalg.qr(rng.standard_normal((n1, nc)))
        q2, _ = np.linalg.qr(rng.standard_normal((n2, nc)))
        s = np.concatenate([rng.uniform(lead / 2, lead, k), rng.uniform(0.05, 0.5, nc - k)])
        out[c] = (q1 * np.sort(s)[::-1]) @ q2.T
    return out


# High rank (k > 64): the recovered factor is orthonormalised by the FP64
# Newton-Schulz steps on workspace Gram matrices; full rank reproduces A.
@pytest.mark.parametrize("k", [100, 256])
def test_f32_high_rank_gaussian(wp, k):
    import torch
    a = cast(np.random.default_rng(256 + k).standard_normal((16, 256, 256)), np.float32)
    res = wp.w_svd(to_dev(a, torch.float32), 2, k)
    torch.cuda.synchronize()
    assert host(res.info).min() > 0
    _, sh_ref, _, ak_ref = orc.w_svd(a, 2, k)
    coeff = orc.lift_fwd(a, 2)
    bars = svd_bars(coeff, k, "f32", L=2)
    assert rel_fro(host(res.shat), sh_ref) <= bars["shat"]
    assert rel_fro(host(res.ak), ak_ref) <= bars["ak"]
    if k == 256:
        assert rel_fro(host(res.ak), a) <= 1e-5
    assert host(res.orth_err).max() <= bars["orth"]


def test_f32_high_rank_gapped(wp):
    # A clear gap after sigma_100 (sigma_1 / gap <= 2.2).  At
    # L = 0 (no lifting) the coefficient slices are the slices themselves, so
    # the prescribed spectrum is the one decomposed.
    import torch
    k = 100
    a = cast(_gapped(16, 256, 200, k, seed=11), np.float32)
    res = wp.w_svd(to_dev(a, torch.float32), 0, k)
    torch.cuda.synchronize()
    assert host(res.info).min() > 0
    _, sh_ref, _, ak_ref = orc.w_svd(a, 0, k)
    bars = svd_bars(a, k, "f32", L=0)
    # Held at the stated FP32 target, below the derived bar (which is at
    # least 4 mr u = 6e-5 for 256 rows).
    assert rel_fro(host(res.shat), sh_ref) <= 1e-5
    assert rel_fro(host(res.ak), ak_ref) <= 1e-5
    assert host(res.orth_err).max() <= bars["orth"]
    _check_factors(res, a, k, bars, "f32")


@pytest.mark.parametrize("shape,k", [((4, 300, 200), 20), ((8, 100, 90), 90), ((4, 90, 140), 70)])
def test_f64_long_and_high_rank(wp, shape, k):
    # FP64: a 200-row recovered factor (block kernel), full rank 90 and rank 70
    # of a transposed slice (the recovered factor is U) through the k > 64 polish.
    import torch
    p, n1, n2 = shape
    a = np.random.default_rng(n1 * 7 + n2).standard_normal(shape)
    res = wp.w_svd(to_dev(a, torch.float64), 2, k)
    torch.cuda.synchronize()
    assert host(res.info).min() > 0
    _, sh_ref, _, ak_ref = orc.w_svd(a, 2, k)
    coeff = orc.lift_fwd(a, 2)
    bars = svd_bars(coeff, k, "f64", L=2)
    assert rel_fro(host(res.shat), sh_ref) <= bars["shat"]
    assert rel_fro(host(res.ak), ak_ref) <= bars["ak"]
    if k == min(n1, n2):
        assert rel_fro(host(res.ak), a) <= 1e-12
    assert host(res.orth_err).max() <= bars["orth"]
    _check_factors(res, coeff, k, bars)


# Register kernel with 64 or more slices of untransposed columns: the columns
# are staged through LDS half a slice at a time.  Heights that fill the
# second half only partly, odd column counts (a zero tournament column), both
# precisions.
@pytest.mark.parametrize("shape,dtype,k", [((64, 200, 150), "f32", 12), ((64, 129, 129), "f32", 9),
                                           ((64, 120, 77), "f64", 7), ((64, 40, 33), "f64", 5)])
def test_register_kernel_staged_columns(wp, shape, dtype, k):
    import torch
    p, n1, n2 = shape
    L = 2
    a = np.random.default_rng(n1 * 3 + n2).standard_normal(shape)
    td = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        a = cast(a, np.float32)
    res = wp.w_svd(to_dev(a, td), L, k)
    torch.cuda.synchronize()
    assert host(res.info).min() > 0
    _, sh_ref, _, ak_ref = orc.w_svd(a, L, k)
    bars = svd_bars(orc.lift_fwd(a, L), k, dtype, L=L)
    assert rel_fro(host(res.shat), sh_ref) <= bars["shat"]
    assert rel_fro(host(res.ak), ak_ref) <= bars["ak"]
    assert host(res.orth_err).max() <= bars["orth"]


# Register kernel with more leading columns than the freed exchange buffers
# stage at once (k = 150 > 128 columns of 256 rows): the factors leave the
# kernel in two chunks.  Both orientations (the second forms V from W).
@pytest.mark.parametrize("shape", [(64, 256, 160), (64, 160, 256)])
def test_register_kernel_chunked_factors(wp, shape):
    import torch
    p, n1, n2 = shape
    k = 150
    a = cast(_gapped(p, n1, n2, k, seed=17), np.float32)
    res = wp.w_svd(to_dev(a, torch.float32), 0, k)
    torch.cuda.synchronize()
    assert host(res.info).min() > 0
    _, sh_ref, _, ak_ref = orc.w_svd(a, 0, k)
    bars = svd_bars(a, k, "f32", L=0)
    assert rel_fro(host(res.shat), sh_ref) <= 1e-5
    assert rel_fro(host(res.ak), ak_ref) <= 1e-5
    assert host(res.orth_err).max() <= bars["orth"]
    _check_factors(res, a, k, bars, "f32")


# ---- sp-w-svd (Sec. IV-B): only s_L and d_L are decomposed ---------------------

@pytest.mark.parametrize("shape,L,k", [((32, 20, 14), 3, 5), ((16, 7, 9), 4, 3),
                                       ((8, 65, 40), 1, 3), ((24, 33, 30), 3, 30),
                                       ((64, 130, 100), 2, 10)])
def test_sparse_f64_shapes(wp, shape, L, k):
    import torch
    p, n1, n2 = shape
    a = np.random.default_rng(7 * n1 + n2).standard_normal(shape)
    res = wp.w_svd_sparse(to_dev(a, torch.float64), L, k)
    torch.cuda.synchronize()
    nk = 2 * (p >> L)
    assert res.uhat.shape == (nk, n1, k) and res.shat.shape == (nk, k)
    assert host(res.info).min() > 0
    uh_ref, sh_ref, vh_ref, ak_ref = orc.w_svd_sparse(a, L, k)
    coeff = orc.lift_fwd(a, L)[:nk]
    bars = svd_bars(coeff, k, "f64", L=L, p=p)
    assert rel_fro(host(res.shat), sh_ref) <= bars["shat"]
    ak = host(res.ak)
    assert rel_fro(ak, ak_ref) <= bars["ak"]
    assert host(res.orth_err).max() <= bars["orth"]
    _check_factors(res, coeff, k, bars)
    # the finer details of the rebuilt tensor are absent (up to rounding)
    if nk < p:
        assert np.abs(orc.lift_fwd(ak, L)[nk:]).max() <= 1e-12 * np.abs(ak).max()


def test_sparse_matches_full_at_one_level(wp):
    # At L = 1 the kept slices are all slices: both entry points run the same kernels.
    import torch
    a = cast(np.random.default_rng(9).standard_normal((16, 48, 40)), np.float32)
    x = to_dev(a, torch.float32)
    full = wp.w_svd(x, 1, 6)
    sp = wp.w_svd_sparse(x, 1, 6)
    torch.cuda.synchronize()
    for f, s in zip(full[:5], sp[:5]):
        assert torch.equal(f, s)


def test_sparse_table3_shape_f32(wp):
    # Table 3 shape: 256x192x96 hyperspectral-like tensor, L = 5 (m = 3, 6 kept
    # slices), rank 32, FP32.
    import torch
    from paper_2601_08228_amd import synth
    x = cast(synth.hsi_like(256, 192, 96, seed=31), np.float32)
    res = wp.w_svd_sparse(to_dev(x, torch.float32), 5, 32)
    torch.cuda.synchronize()
    assert host(res.info).min() > 0
    _, sh_ref, _, ak_ref = orc.w_svd_sparse(x, 5, 32)
    ak = host(res.ak)
    assert rel_fro(host(res.shat), sh_ref) <= 1e-5
    assert rel_fro(ak, ak_ref) <= 1e-5
    assert abs(orc.psnr(x, ak) - orc.psnr(x, ak_ref)) <= 0.01
    assert host(res.orth_err).max() <= svd_bars(orc.lift_fwd(x, 5)[:6], 32, "f32")["orth"]


@pytest.mark.parametrize("k", [96, 192])
def test_sparse_table3_shape_high_rank(wp, k):
    # Table 3 cube at rank 96 and at full rank 192: the 192-row recovered
    # factor goes through the k > 64 polish.
    import torch
    from paper_2601_08228_amd import synth
    x = cast(synth.hsi_like(256, 192, 96, seed=31), np.float32)
    res = wp.w_svd_sparse(to_dev(x, torch.float32), 5, k)
    torch.cuda.synchronize()
    assert host(res.info).min() > 0
    _, sh_ref, _, ak_ref = orc.w_svd_sparse(x, 5, k)
    bars = svd_bars(orc.lift_fwd(x, 5)[:6], k, "f32", L=5, p=96)
    assert rel_fro(host(res.shat), sh_ref) <= bars["shat"]
    assert rel_fro(host(res.ak), ak_ref) <= bars["ak"]
    assert host(res.orth_err).max() <= bars["orth"]


@pytest.mark.parametrize("shape,dtype", [((64, 96, 80), "f32"), ((8, 300, 70), "f64")])
def test_timed_entry_matches_and_times_the_jacobi(wp, shape, dtype):
    # w_svd_timed gives w_svd's results bit for bit (register and block
    # kernels) and records its two events around the Jacobi stage, inside the
    # whole call.
    import torch
    td = torch.float32 if dtype == "f32" else torch.float64
    a = to_dev(np.random.default_rng(12).standard_normal(shape), td)
    ref = wp.w_svd(a, 2, 6)
    e0, e1, c0, c1 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
    c0.record()
    got = wp.w_svd_timed(a, 2, 6, e0, e1)
    c1.record()
    torch.cuda.synchronize()
    for f, r in zip(got[:5], ref[:5]):
        assert torch.equal(f, r)
    jac, whole = e0.elapsed_time(e1), c0.elapsed_time(c1)
    assert 0 < jac <= whole
