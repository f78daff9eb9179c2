"""GPU parity of the face-product GEMMs (FP64, FP32, BF16, bf16x3 MFMA) against the oracle."""

import numpy as np
import pytest

import oracle as orc
from gpu_helpers import device, to_dev, host, cast, rel_fro, bf16_rne

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wp():
    device()
    import paper_2601_08228_amd as wp
    return wp


def _operands(p, m, k, n, ta, tb, seed, dist="normal"):
    rng = np.random.default_rng(seed)
    draw = rng.standard_normal if dist == "normal" else (lambda s: rng.uniform(-1, 1, s))
    a = draw((p, k, m) if ta else (p, m, k))
    b = draw((p, n, k) if tb else (p, k, n))
    return a, b


# (p, m, k, n): several tiles plus ragged tails in every dimension, single-tile,
# degenerate 1-wide dimensions, and K shorter than one K-tile.  The last two
# have every dimension a multiple of 8, so the BF16 modes take the
# direct-to-LDS kernel in all four transpose combinations (tails of 8 rows
# and columns, K not a multiple of the 32-wide stage, many stages).
SHAPES = [(3, 130, 70, 200), (2, 64, 64, 64), (1, 1, 1, 1), (5, 17, 3, 9), (4, 257, 33, 129),
          (2, 300, 520, 260), (16, 32, 24, 20), (1, 7, 1000, 5), (2, 264, 200, 328),
          (1, 512, 1032, 256)]
TRANS = [(False, False), (True, False), (False, True), (True, True)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("tt", TRANS)
def test_f64(wp, shape, tt):
    import torch
    p, m, k, n = shape
    a, b = _operands(p, m, k, n, *tt, seed=m + k)
    out = host(wp.w_face_product(to_dev(a, torch.float64), to_dev(b, torch.float64), *tt))
    ref = orc.face(a, b, *tt)
    # FP64 MFMA with FP64 accumulation: a K-term dot product, error ~ K u64.
    assert rel_fro(out, ref) <= 1e-15 * max(k, 8)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("tt", TRANS)
def test_f32(wp, shape, tt):
    import torch
    p, m, k, n = shape
    a, b = _operands(p, m, k, n, *tt, seed=m * 3 + n)
    a, b = cast(a, np.float32), cast(b, np.float32)
    out = host(wp.w_face_product(to_dev(a, torch.float32), to_dev(b, torch.float32), *tt))
    assert rel_fro(out, orc.face(a, b, *tt)) <= 1e-7 * max(np.sqrt(k), 4)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("tt", TRANS)
@pytest.mark.parametrize("mode", ["bf16", "bf16x3"])
def test_split(wp, shape, tt, mode):
    # Operands are split by the lifting epilogue at L = 0 (no transform), so the
    # products are of the input values themselves.
    import torch
    p, m, k, n = shape
    a, b = _operands(p, m, k, n, *tt, seed=m + 2 * n, dist="uniform")
    a, b = cast(a, np.float32), cast(b, np.float32)
    ahi, alo = wp.w_transform_split(to_dev(a, torch.float32), 0)
    bhi, blo = wp.w_transform_split(to_dev(b, torch.float32), 0)
    out = host(wp.w_face_product_split(ahi, alo, bhi, blo, *tt, gemm=mode))
    a_hi = bf16_rne(a).astype(np.float64)
    b_hi = bf16_rne(b).astype(np.float64)
    a_lo = bf16_rne((a - a_hi).astype(np.float32)).astype(np.float64)
    b_lo = bf16_rne((b - b_hi).astype(np.float32)).astype(np.float64)
    if mode == "bf16":
        exact = orc.face(a_hi, b_hi, *tt)          # the products the mode defines
        assert rel_fro(out, exact) <= 1e-7 * max(np.sqrt(k), 4)
        assert rel_fro(out, orc.face(a, b, *tt)) <= 1e-2
    else:
        exact = orc.face(a_hi, b_hi, *tt) + orc.face(a_hi, b_lo, *tt) + orc.face(a_lo, b_hi, *tt)
        assert rel_fro(out, exact) <= 1e-7 * max(np.sqrt(k), 4)
        assert rel_fro(out, orc.face(a, b, *tt)) <= 1e-5


def test_deterministic(wp):
    import torch
    a, b = _operands(8, 200, 300, 100, False, False, seed=1)
    da, db = to_dev(a, torch.float32), to_dev(b, torch.float32)
    r1 = host(wp.w_face_product(da, db))
    r2 = host(wp.w_face_product(da, db))
    assert np.array_equal(r1, r2)


@pytest.mark.parametrize("tt", TRANS)
@pytest.mark.parametrize("mode", ["bf16", "bf16x3"])
def test_direct_kernel_repeatable_full_size(wp, tt, mode):
    # The benchmark shape (256 slices of 512x512x512) in every transpose
    # combination: repeated calls give the same bits.  (A fragment read whose
    # output shared a register with a later read's address once made the
    # transposed-A BF16 kernel differ from call to call.)
    import torch
    from paper_2601_08228_amd import synth
    dev = torch.device("cuda:0")
    a = synth.normal_device((256, 512, 512), 41, dev)
    b = synth.normal_device((256, 512, 512), 42, dev)
    ahi, alo = wp.w_transform_split(a, 0)
    bhi, blo = wp.w_transform_split(b, 0)
    if mode == "bf16":
        alo = blo = None
    ref = wp.w_face_product_split(ahi, alo, bhi, blo, *tt, gemm=mode)
    for _ in range(4):
        assert torch.equal(wp.w_face_product_split(ahi, alo, bhi, blo, *tt, gemm=mode), ref)
    # One sampled slice against the oracle's product of the same bf16 parts.
    s = 97
    ah = ahi[s].float().double().cpu().numpy()
    bh = bhi[s].float().double().cpu().numpy()
    exact = orc.face(ah[None], bh[None], *tt)[0]
    if mode == "bf16x3":
        al = alo[s].float().double().cpu().numpy()
        bl = blo[s].float().double().cpu().numpy()
        exact = exact + orc.face(ah[None], bl[None], *tt)[0] + orc.face(al[None], bh[None], *tt)[0]
    assert rel_fro(ref[s].double().cpu().numpy(), exact) <= 1e-7 * np.sqrt(512)


def test_unaligned_pitch_uses_scalar_loads(wp):
    # K = 3 makes the row pitch 12 bytes: the 16-byte load path must not be used.
    import torch
    a, b = _operands(6, 45, 3, 37, False, False, seed=2)
    out = host(wp.w_face_product(to_dev(a, torch.float64), to_dev(b, torch.float64)))
    assert rel_fro(out, orc.face(a, b)) <= 1e-15


# The single-call form with the GEMM mode and a workspace: native equals
# w_face_product bit for bit; the BF16 modes split the FP32 operands inside
# the call and match the split face-product of the same planes bit for bit,
# and the oracle within the mode's error.
@pytest.mark.parametrize("shape", [(3, 130, 70, 200), (2, 264, 200, 328), (4, 9, 5, 3)])
@pytest.mark.parametrize("tt", TRANS)
def test_gemm_single_call(wp, shape, tt):
    import torch
    p, m, k, n = shape
    a, b = _operands(p, m, k, n, *tt, seed=m + 5 * n)
    a, b = cast(a, np.float32), cast(b, np.float32)
    ta_, tb_ = to_dev(a, torch.float32), to_dev(b, torch.float32)
    ref = orc.face(a, b, *tt)
    nat = wp.w_face_product_gemm(ta_, tb_, *tt, gemm="native")
    assert torch.equal(nat, wp.w_face_product(ta_, tb_, *tt))
    for gemm, tol in (("bf16x3", 1e-5), ("bf16", 2e-2)):
        got = wp.w_face_product_gemm(ta_, tb_, *tt, gemm=gemm)
        hi_a, lo_a = wp.w_transform_split(ta_, 0)
        hi_b, lo_b = wp.w_transform_split(tb_, 0)
        split = wp.w_face_product_split(hi_a, lo_a, hi_b, lo_b, *tt, gemm=gemm)
        assert torch.equal(got, split), gemm
        assert rel_fro(host(got), ref) <= tol, gemm


def test_gemm_single_call_workspace_checks(wp):
    import torch
    from paper_2601_08228_amd._lib import WprodError
    a = to_dev(np.ones((2, 8, 8)), torch.float32)
    need = wp.w_face_product_workspace(8, 8, 8, 2, torch.float32, "bf16x3")
    assert need > 0 and wp.w_face_product_workspace(8, 8, 8, 2, torch.float32, "native") == 0
    with pytest.raises(ValueError):
        wp.w_face_product_gemm(a, a, gemm="bf16x3",
                               workspace=torch.empty(need - 1, dtype=torch.uint8, device=a.device))
    # BF16 modes need FP32 data (WP_EDTYPE from the library, nothing launched).
    d = to_dev(np.ones((2, 8, 8)), torch.float64)
    with pytest.raises(WprodError):
        wp.w_face_product_gemm(d, d, gemm="bf16x3")
