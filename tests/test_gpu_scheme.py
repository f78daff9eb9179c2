"""GPU parity of the lifting with chosen predict / update stencils (Sec. II-A,
Example 2.1, Remark 3.1): the four passes, the w-product and its derivative,
against the FP64 oracle; the lazy stencils against the lazy kernels."""

import numpy as np
import pytest

import oracle as orc
from gpu_helpers import device, to_dev, host, cast, rel_fro

pytestmark = pytest.mark.gpu

KINDS = ["forward", "inverse", "adj", "iadj"]


@pytest.fixture(scope="module")
def wp():
    device()
    import paper_2601_08228_amd as wp
    return wp


def _oracle_pass(x, L, taps, kind):
    return {"forward": orc.lift_fwd_scheme, "inverse": orc.lift_inv_scheme,
            "adj": orc.lift_fwd_scheme_adj, "iadj": orc.lift_inv_scheme_adj}[kind](x, L, taps)


def _taps(name, L, seed=0):
    if name == "interp":
        return orc.interpolating_scheme(L)
    if name == "cdf53":
        return orc.cdf53_scheme(L)
    return np.random.default_rng(seed).uniform(-0.6, 0.6, (L, 2, orc.SCHEME_TAPS))


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("shape,L", [((16, 5, 7), 2), ((64, 33, 9), 4), ((8, 1, 1), 3),
                                     ((96, 20, 30), 5), ((16, 4, 4), 0)])
@pytest.mark.parametrize("name", ["interp", "cdf53", "random"])
def test_passes_f64(wp, kind, shape, L, name):
    # Ragged position counts (35, 297, 1, 600, 16), one position, m = 3 with
    # five levels, L = 0 (a copy).
    import torch
    taps = _taps(name, L, seed=L)
    x = np.random.default_rng(shape[0] + L).standard_normal(shape)
    got = wp.w_transform_scheme(to_dev(x, torch.float64), L, taps, kind)
    assert rel_fro(host(got), _oracle_pass(x, L, taps, kind)) <= 1e-13


@pytest.mark.parametrize("kind", KINDS)
def test_passes_f32_long_tubes(wp, kind):
    # 2048 slices, the FP32 limit (16 positions per workgroup, 128 KiB of LDS).
    import torch
    L = 6
    taps = orc.cdf53_scheme(L)
    x = cast(np.random.default_rng(3).standard_normal((2048, 5, 7)), np.float32)
    got = wp.w_transform_scheme(to_dev(x, torch.float32), L, taps, kind)
    assert rel_fro(host(got), _oracle_pass(x, L, taps, kind)) <= 1e-6


def test_passes_f64_max_levels(wp):
    # p = 1024 FP64 (the limit) with ten levels, every pass.
    import torch
    L = 10
    taps = _taps("random", L, seed=5)
    x = np.random.default_rng(4).standard_normal((1024, 3, 2))
    for kind in KINDS:
        got = wp.w_transform_scheme(to_dev(x, torch.float64), L, taps, kind)
        assert rel_fro(host(got), _oracle_pass(x, L, taps, kind)) <= 1e-12, kind


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_lazy_stencils_match_the_lazy_kernels(wp, dtype):
    # P = I, U = I/2 takes the same rounding steps as the lazy forward and
    # inverse passes (bit for bit); the transposes agree to rounding.
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    L = 4
    taps = orc.lazy_scheme(L)
    x = to_dev(np.random.default_rng(6).standard_normal((48, 17, 13)), td)
    assert torch.equal(wp.w_transform_scheme(x, L, taps, "forward"), wp.w_transform(x, L))
    assert torch.equal(wp.w_transform_scheme(x, L, taps, "inverse"), wp.w_itransform(x, L))
    tol = 1e-15 if dtype == "f64" else 1e-6
    assert rel_fro(host(wp.w_transform_scheme(x, L, taps, "adj")),
                   host(wp.w_transform_adj(x, L))) <= tol
    assert rel_fro(host(wp.w_transform_scheme(x, L, taps, "iadj")),
                   host(wp.w_itransform_adj(x, L))) <= tol


def test_split_passes(wp):
    # bf16 hi of the forward pass equals the rounding of the FP32 pass, and
    # hi + lo recovers it to about 2^-16 relative.
    import torch
    L = 3
    taps = orc.cdf53_scheme(L)
    x = to_dev(np.random.default_rng(7).standard_normal((32, 24, 10)), torch.float32)
    for kind in ("forward", "iadj"):
        full = wp.w_transform_scheme(x, L, taps, kind)
        hi, lo = wp.w_transform_scheme_split(x, L, taps, kind)
        assert torch.equal(hi, full.to(torch.bfloat16))
        assert rel_fro(host(hi.float() + lo.float()), host(full)) <= 2.0 ** -15


@pytest.mark.parametrize("gemm,tol", [("native", 1e-5), ("bf16x3", 1e-5), ("bf16", 2e-2)])
def test_product_f32(wp, gemm, tol):
    import torch
    L = 3
    taps = orc.cdf53_scheme(L)
    rng = np.random.default_rng(8)
    a = cast(rng.standard_normal((32, 70, 50)), np.float32)
    b = cast(rng.standard_normal((32, 50, 90)), np.float32)
    c = wp.w_product_scheme(to_dev(a, torch.float32), to_dev(b, torch.float32), L, taps, gemm=gemm)
    assert rel_fro(host(c), orc.w_product_scheme(a, b, L, taps)) <= tol


def test_product_f64_transposed_operands(wp):
    import torch
    L = 2
    taps = _taps("random", L, seed=9)
    rng = np.random.default_rng(9)
    a = rng.standard_normal((8, 13, 11))   # stored (p, n2, n1) with trans_a
    b = rng.standard_normal((8, 17, 13))   # stored (p, n3, n2) with trans_b
    c = wp.w_product_scheme(to_dev(a, torch.float64), to_dev(b, torch.float64), L, taps,
                            trans_a=True, trans_b=True)
    ref = orc.w_product_scheme(a, b, L, taps, trans_a=True, trans_b=True)
    assert rel_fro(host(c), ref) <= 1e-12


@pytest.mark.parametrize("gemm,dtype,tol", [("native", "f64", 1e-12), ("native", "f32", 1e-5),
                                            ("bf16x3", "f32", 1e-5)])
def test_derivative_vs_oracle(wp, gemm, dtype, tol):
    import torch
    from paper_2601_08228_amd import w_product_ad
    td = torch.float64 if dtype == "f64" else torch.float32
    L = 2
    taps = orc.cdf53_scheme(L)
    rng = np.random.default_rng(10)
    a = rng.standard_normal((16, 24, 20))
    b = rng.standard_normal((16, 20, 12))
    g = rng.standard_normal((16, 24, 12))
    if dtype == "f32":
        a, b, g = cast(a, np.float32), cast(b, np.float32), cast(g, np.float32)
    at = to_dev(a, td).requires_grad_(True)
    bt = to_dev(b, td).requires_grad_(True)
    c = w_product_ad(at, bt, L, gemm, taps)
    c.backward(to_dev(g, td))
    da, db = orc.w_product_scheme_vjp(a, b, g, L, taps)
    assert rel_fro(host(c), orc.w_product_scheme(a, b, L, taps)) <= tol
    assert rel_fro(host(at.grad), da) <= tol
    assert rel_fro(host(bt.grad), db) <= tol


def test_full_size_passes_sampled(wp):
    # The benchmark's tensor and launch shape (512x512x256 FP32, L = 4, CDF 5/3):
    # every pass checked on 1024 sampled tubes, which the oracle computes one
    # by one (a tube's transform involves that tube only).
    import torch
    from paper_2601_08228_amd import synth
    L = 4
    taps = orc.cdf53_scheme(L)
    x = synth.normal_device((256, 512, 512), 21, torch.device("cuda:0"))
    cols = np.random.default_rng(12).choice(512 * 512, size=1024, replace=False)
    idx = torch.as_tensor(cols, device=x.device)
    xs = x.reshape(256, -1)[:, idx].double().cpu().numpy()
    for kind in KINDS:
        got = wp.w_transform_scheme(x, L, taps, kind).reshape(256, -1)[:, idx]
        assert rel_fro(host(got), _oracle_pass(xs, L, taps, kind)) <= 1e-6, kind
