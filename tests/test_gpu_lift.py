"""GPU parity of the lifting passes (W, W^{-1}, W^T, W^{-T}, split epilogue) against the oracle."""

import numpy as np
import pytest

import oracle as orc
from gpu_helpers import device, to_dev, host, cast, rel_fro, bf16_rne, bf16_bits_to_f32
from pins import load_golden

pytestmark = pytest.mark.gpu
EX = load_golden("example_2_2.json")


@pytest.fixture(scope="module")
def wp():
    device()
    import paper_2601_08228_amd as wp
    return wp


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_example_2_2_bit_exact(wp, dt):
    import torch
    tdt = torch.float64 if dt == "f64" else torch.float32
    for name in ("A", "B"):
        x = to_dev(EX[name], tdt)
        c2 = host(wp.w_transform(x, 2))
        assert np.array_equal(c2, orc.lift_fwd(EX[name], 2))
        assert np.array_equal(c2[0:1], EX[name + "_s2"])
        c1 = host(wp.w_transform(x, 1))
        assert np.array_equal(c1[0:2], EX[name + "_s1"])
        assert np.array_equal(c1[2:4], EX[name + "_d1"])
    c = np.concatenate([EX["C_s2"], EX["C_d2"], EX["C_d1"]])
    assert np.array_equal(host(wp.w_itransform(to_dev(c, tdt), 2)), EX["C"])


# (p, n1, n2, L): tiles with ragged tails (n1*n2 not a multiple of the vector
# width), one and two register tiers, L = 0 and up to 10 levels.
SHAPES = [(4, 2, 3, 2), (16, 32, 24, 2), (48, 7, 9, 4), (64, 33, 31, 6), (128, 5, 12, 7),
          (256, 8, 8, 8), (512, 3, 5, 9), (1024, 4, 4, 10), (96, 17, 16, 5), (7, 9, 11, 0),
          (32, 130, 66, 5), (24, 64, 64, 3)]
KINDS = ["w_transform", "w_itransform", "w_transform_adj", "w_itransform_adj"]
ORACLE = {"w_transform": orc.lift_fwd, "w_itransform": orc.lift_inv,
          "w_transform_adj": orc.lift_fwd_adj, "w_itransform_adj": orc.lift_inv_adj}


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", KINDS)
def test_f64_bit_exact_vs_oracle(wp, shape, kind):
    # The FP64 passes evaluate the same level steps in the same order (the halving
    # is exact), so they agree with the oracle bit for bit.
    import torch
    p, n1, n2, L = shape
    x = np.random.default_rng(p * 7 + n1).standard_normal((p, n1, n2))
    out = host(getattr(wp, kind)(to_dev(x, torch.float64), L))
    assert np.array_equal(out, ORACLE[kind](x, L))


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", KINDS)
def test_f32_vs_oracle(wp, shape, kind):
    import torch
    p, n1, n2, L = shape
    x = cast(np.random.default_rng(p * 5 + n2).standard_normal((p, n1, n2)), np.float32)
    out = host(getattr(wp, kind)(to_dev(x, torch.float32), L))
    # each output is a short sum of L+1 terms with exact halvings: error ~ (L+1) u32
    assert rel_fro(out, ORACLE[kind](x, L)) <= 2e-7 * (L + 1)


@pytest.mark.parametrize("kind", ["w_transform_split", "w_itransform_adj_split"])
@pytest.mark.parametrize("shape", [(16, 32, 24, 2), (64, 33, 31, 6), (7, 9, 11, 0), (32, 64, 64, 3),
                                   (16, 12, 5, 2), (256, 64, 40, 8)])
def test_split_epilogue(wp, kind, shape):
    # hi = RNE_bf16(c) and lo = RNE_bf16(c - hi) of the FP32 coefficients the plain pass writes.
    import torch
    p, n1, n2, L = shape
    x = cast(np.random.default_rng(3).standard_normal((p, n1, n2)), np.float32)
    xd = to_dev(x, torch.float32)
    plain_kind = "w_transform" if kind == "w_transform_split" else "w_itransform_adj"
    c = host(getattr(wp, plain_kind)(xd, L))
    hi, lo = getattr(wp, kind)(xd, L)
    hi = bf16_bits_to_f32(hi)
    lo = bf16_bits_to_f32(lo)
    exp_hi = bf16_rne(c)
    assert np.array_equal(hi, exp_hi)
    assert np.array_equal(lo, bf16_rne(c - exp_hi))
    rel = np.abs((hi.astype(np.float64) + lo) - c) / np.maximum(np.abs(c), 1e-30)
    assert rel.max() <= 2.0 ** -16
    hi_only, none = getattr(wp, kind)(xd, L, with_lo=False)
    assert none is None and np.array_equal(bf16_bits_to_f32(hi_only), exp_hi)


def test_perfect_reconstruction_on_device(wp):
    import torch
    x = np.random.default_rng(9).standard_normal((128, 40, 24))
    xd = to_dev(x, torch.float64)
    back = host(wp.w_itransform(wp.w_transform(xd, 7), 7))
    assert rel_fro(back, x) <= 1e-15


def test_full_size_sampled_tubes(wp):
    # 512 x 512 x 256 FP32, L = 4 (the w-product benchmark shape): every output of the
    # pass run at full size, checked on 256 sampled tubes against the oracle.
    import torch
    p, n1, n2, L = 256, 512, 512, 4
    from paper_2601_08228_amd import synth
    xd = synth.normal_device((p, n1, n2), 11, device())
    rng = np.random.default_rng(0)
    ii = rng.integers(0, n1, 256)
    jj = rng.integers(0, n2, 256)
    for kind in KINDS:
        out = getattr(wp, kind)(xd, L)
        torch.cuda.synchronize()
        tubes_in = host(xd[:, ii, jj]).astype(np.float64)[:, :, None]
        tubes_out = host(out[:, ii, jj])[:, :, None]
        assert rel_fro(tubes_out, ORACLE[kind](tubes_in, L)) <= 1e-6, kind
