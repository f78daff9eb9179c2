"""The allocation-free w-product entry point (w_product_noalloc) against w_product.

Both run the same kernels on the same inputs, so the results must agree bit
for bit; the no-alloc call takes its workspace from the library's fixed
device scratch instead of a caller buffer.  Called through the C ABI
(ctypes on libwprod.so) with device tensors from torch: two calls in a row,
the second with a smaller input (the scratch keeps the first call's
contents), for every precision mode, plus the size limit.
"""

import ctypes

import numpy as np
import pytest

from gpu_helpers import device, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wp():
    device()
    import paper_2601_08228_amd as wp
    return wp


def _noalloc(lib, a, b, c, L, ta, tb, dtype, gemm):
    import torch
    p = a.shape[0]
    n1, n2 = (a.shape[2], a.shape[1]) if ta else (a.shape[1], a.shape[2])
    n3 = b.shape[1] if tb else b.shape[2]
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return lib.w_product_noalloc(a.data_ptr(), b.data_ptr(), c.data_ptr(), n1, n2, n3, p, L,
                                 int(ta), int(tb), dtype, gemm, stream)


# (p, n1, n2, n3, L, trans_a, trans_b): the first call, then a smaller one.
CALLS = [(32, 96, 80, 72, 3, False, False), (8, 40, 24, 30, 2, True, False)]
MODES = [("f64", "native"), ("f32", "native"), ("f32", "bf16x3"), ("f32", "bf16")]


@pytest.mark.parametrize("prec,gemm", MODES)
def test_noalloc_matches_w_product(wp, prec, gemm):
    import torch
    from paper_2601_08228_amd import _lib
    lib = _lib.load()
    td = torch.float64 if prec == "f64" else torch.float32
    dt = _lib.WP_F64 if prec == "f64" else _lib.WP_F32
    mode = _lib.GEMM_MODES[gemm]
    rng = np.random.default_rng(5)
    for p, n1, n2, n3, L, ta, tb in CALLS:
        print("noalloc call", prec, gemm, (p, n1, n2, n3, L, ta, tb), flush=True)
        a = to_dev(rng.standard_normal((p, n2, n1) if ta else (p, n1, n2)), td)
        b = to_dev(rng.standard_normal((p, n3, n2) if tb else (p, n2, n3)), td)
        ref = wp.w_product(a, b, L, ta, tb, gemm=gemm)
        c = torch.full((p, n1, n3), float("nan"), dtype=td, device=a.device)
        st = _noalloc(lib, a, b, c, L, ta, tb, dt, mode)
        assert st == _lib.WP_OK, lib.w_status_string(st)
        torch.cuda.synchronize()
        assert torch.equal(c, ref)


def test_noalloc_rejects_calls_beyond_its_scratch(wp):
    # Sizes whose workspace exceeds the fixed scratch: WP_ESCRATCH before any
    # launch (the claimed sizes are never touched), output untouched.
    import torch
    from paper_2601_08228_amd import _lib
    lib = _lib.load()
    limit = lib.w_product_noalloc_scratch_bytes()
    assert limit == 128 << 20
    p, n = 256, 512  # three 256 MiB FP32 coefficient tensors
    assert wp.w_product_workspace(n, n, n, p, 4, torch.float32, "native") > limit
    small = [torch.zeros(16, device=device()) for _ in range(3)]
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib.w_product_noalloc(small[0].data_ptr(), small[1].data_ptr(), small[2].data_ptr(),
                               n, n, n, p, 4, 0, 0, _lib.WP_F32, 0, stream)
    assert st == _lib.WP_ESCRATCH
    torch.cuda.synchronize()
    assert bool((small[2] == 0).all())
    # The largest call that fits still runs and matches.
    a = to_dev(np.random.default_rng(9).standard_normal((64, 128, 128)), torch.float32)
    need = wp.w_product_workspace(128, 128, 128, 64, 2, torch.float32, "bf16x3")
    assert need <= limit
    assert torch.equal(wp.w_product_noalloc(a, a, 2, gemm="bf16x3"),
                       wp.w_product(a, a, 2, gemm="bf16x3"))
