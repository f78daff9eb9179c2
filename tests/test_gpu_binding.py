"""The Python binding rejects caller buffers that do not fit a call, before any launch.

The C ABI cannot see the size, dtype or device of a buffer, so the binding
checks every caller-supplied `out` and `workspace` (device, dtype, shape,
contiguity, byte count) and raises ValueError; these tests hand it wrong
buffers and check that the call raises and leaves `out` untouched.
"""

import numpy as np
import pytest

from gpu_helpers import device, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wp():
    device()
    import paper_2601_08228_amd as wp
    return wp


def _pair():
    import torch
    rng = np.random.default_rng(1)
    return (to_dev(rng.standard_normal((4, 6, 5)), torch.float32),
            to_dev(rng.standard_normal((4, 5, 3)), torch.float32))


def test_w_product_out_checks(wp):
    import torch
    a, b = _pair()
    bad_outs = [torch.full((4, 6, 3), 7.0, dtype=torch.float64, device=a.device),   # dtype
                torch.full((4, 6, 2), 7.0, dtype=torch.float32, device=a.device),   # shape
                torch.full((4, 3, 6), 7.0, dtype=torch.float32, device=a.device).transpose(1, 2),
                torch.full((4, 6, 3), 7.0, dtype=torch.float32)]                     # host
    for out in bad_outs:
        with pytest.raises((ValueError, TypeError)):
            wp.w_product(a, b, 2, out=out)
        assert bool((out == 7.0).all())


def test_w_product_workspace_checks(wp):
    import torch
    a, b = _pair()
    need = wp.w_product_workspace(6, 5, 3, 4, 2, torch.float32, "native")
    bad = [torch.empty(need, dtype=torch.uint8),                                  # host memory
           torch.empty(need - 1, dtype=torch.uint8, device=a.device),             # too small
           torch.empty((need, 2), dtype=torch.uint8, device=a.device)[:, 0]]     # not contiguous
    for ws in bad:
        with pytest.raises(ValueError):
            wp.w_product(a, b, 2, workspace=ws)
    ok = torch.empty(need, dtype=torch.uint8, device=a.device)
    c = wp.w_product(a, b, 2, workspace=ok)
    assert torch.equal(c, wp.w_product(a, b, 2))


def test_svd_pinv_scheme_workspace_checks(wp):
    import torch
    a, _ = _pair()
    small = torch.empty(16, dtype=torch.uint8, device=a.device)
    host_ws = torch.empty(1 << 20, dtype=torch.uint8)
    for ws in (small, host_ws):
        with pytest.raises(ValueError):
            wp.w_svd(a, 2, 3, workspace=ws)
        with pytest.raises(ValueError):
            wp.w_svd_sparse(a, 2, 3, workspace=ws)
        with pytest.raises(ValueError):
            wp.w_pinv(a, 2, workspace=ws)
    taps = np.zeros((2, 2, 5))
    taps[:, 0, 2] = 1.0
    taps[:, 1, 2] = 0.5
    b = to_dev(np.ones((4, 5, 3)), torch.float32)
    with pytest.raises(ValueError):
        wp.w_product_scheme(a, b, 2, taps, workspace=small)
    with pytest.raises(ValueError):
        wp.w_transform_scheme(a, 2, taps, out=torch.empty((4, 6, 5), dtype=torch.float64,
                                                          device=a.device))


def test_lift_out_checks(wp):
    import torch
    a, _ = _pair()
    for out in (torch.empty((4, 6, 5), dtype=torch.float32),
                torch.empty((4, 5, 6), dtype=torch.float32, device=a.device)):
        with pytest.raises((ValueError, TypeError)):
            wp.w_transform(a, 2, out=out)
