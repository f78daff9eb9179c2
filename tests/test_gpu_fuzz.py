"""Seeded shape fuzz against the FP64 oracle.

The fixed-shape tests name the edge cases one by one (ragged tiles, one
position, L = 0, transposes, thin slices); these draw combinations of them at
random from fixed seeds: p = m 2^L with L = 0..4, slice sides 1..70 (so the
vector and scalar lifting paths, partial MFMA tiles and both Jacobi
orientations all occur), both transpose flags and every precision mode, each
against the oracle with the tolerance of its fixed-shape test (and, where a
draw falls outside an entry point's contract, its documented error).
"""

import numpy as np
import pytest

import oracle as orc
from gpu_helpers import device, to_dev, host, cast, rel_fro, svd_bars

pytestmark = pytest.mark.gpu

CASES = list(range(20))


@pytest.fixture(scope="module")
def wp():
    device()
    import paper_2601_08228_amd as wp
    return wp


def _draw(seed):
    rng = np.random.default_rng(seed)
    L = int(rng.integers(0, 5))
    p = int(rng.integers(1, 5)) << L
    n1, n2, n3 = (int(v) for v in rng.integers(1, 71, 3))
    return rng, p, n1, n2, n3, L


@pytest.mark.parametrize("case", CASES)
def test_lifting_passes(wp, case):
    # FP64 passes take the oracle's rounding steps (bit for bit); FP32 within
    # the rounding of L levels.
    import torch
    rng, p, n1, n2, _, L = _draw(100 + case)
    x = rng.standard_normal((p, n1, n2))
    passes = {"w_transform": orc.lift_fwd, "w_itransform": orc.lift_inv,
              "w_transform_adj": orc.lift_fwd_adj, "w_itransform_adj": orc.lift_inv_adj}
    for name, ref in passes.items():
        got = host(getattr(wp, name)(to_dev(x, torch.float64), L))
        assert np.array_equal(got, ref(x, L)), (name, p, n1, n2, L)
        x32 = cast(x, np.float32)
        got = host(getattr(wp, name)(to_dev(x32, torch.float32), L))
        assert rel_fro(got, ref(x32, L)) <= 2e-7 * (L + 1), (name, p, n1, n2, L)


@pytest.mark.parametrize("case", CASES)
def test_product(wp, case):
    import torch
    rng, p, n1, n2, n3, L = _draw(200 + case)
    ta, tb = bool(rng.integers(0, 2)), bool(rng.integers(0, 2))
    a = rng.standard_normal((p, n2, n1) if ta else (p, n1, n2))
    b = rng.standard_normal((p, n3, n2) if tb else (p, n2, n3))
    ref = orc.w_product(a, b, L, ta, tb)
    c = host(wp.w_product(to_dev(a, torch.float64), to_dev(b, torch.float64), L, ta, tb))
    assert rel_fro(c, ref) <= 1e-12, (p, n1, n2, n3, L, ta, tb)
    a32, b32 = cast(a, np.float32), cast(b, np.float32)
    ref32 = orc.w_product(a32, b32, L, ta, tb)
    for gemm, tol in (("native", 1e-5), ("bf16x3", 1e-5), ("bf16", 2e-2)):
        c = host(wp.w_product(to_dev(a32, torch.float32), to_dev(b32, torch.float32), L, ta, tb,
                              gemm=gemm))
        assert rel_fro(c, ref32) <= tol, (gemm, p, n1, n2, n3, L, ta, tb)


@pytest.mark.parametrize("case", CASES)
def test_derivative(wp, case):
    import torch
    from paper_2601_08228_amd import w_product_ad
    rng, p, n1, n2, n3, L = _draw(300 + case)
    a = rng.standard_normal((p, n1, n2))
    b = rng.standard_normal((p, n2, n3))
    g = rng.standard_normal((p, n1, n3))
    at = to_dev(a, torch.float64).requires_grad_(True)
    bt = to_dev(b, torch.float64).requires_grad_(True)
    w_product_ad(at, bt, L).backward(to_dev(g, torch.float64))
    da, db = orc.w_product_vjp(a, b, g, L)
    assert rel_fro(host(at.grad), da) <= 1e-12, (p, n1, n2, n3, L)
    assert rel_fro(host(bt.grad), db) <= 1e-12, (p, n1, n2, n3, L)


@pytest.mark.parametrize("case", CASES)
def test_svd(wp, case):
    # FP64 truncated w-svd: singular values, the rank-k rebuild and both
    # factors' orthogonality within the bars derived from the oracle's singular
    # values; full rank reproduces A.
    import torch
    rng, p, n1, n2, _, L = _draw(400 + case)
    a = rng.standard_normal((p, n1, n2))
    k = int(rng.integers(1, min(n1, n2) + 1))
    res = wp.w_svd(to_dev(a, torch.float64), L, k)
    assert host(res.info).min() > 0
    _, sh_ref, _, ak_ref = orc.w_svd(a, L, k)
    bars = svd_bars(orc.lift_fwd(a, L), k, "f64", L=L)
    assert rel_fro(host(res.shat), sh_ref) <= bars["shat"], (p, n1, n2, L, k)
    assert rel_fro(host(res.ak), ak_ref) <= bars["ak"], (p, n1, n2, L, k, bars["ak"])
    assert host(res.orth_err).max() <= bars["orth"], (p, n1, n2, L, k)
    if k == min(n1, n2):
        assert rel_fro(host(res.ak), a) <= 1e-12


@pytest.mark.parametrize("case", CASES)
def test_scheme_passes(wp, case):
    import torch
    rng, p, n1, n2, _, L = _draw(500 + case)
    taps = rng.uniform(-0.6, 0.6, (L, 2, orc.SCHEME_TAPS))
    x = rng.standard_normal((p, n1, n2))
    ref = {"forward": orc.lift_fwd_scheme, "inverse": orc.lift_inv_scheme,
           "adj": orc.lift_fwd_scheme_adj, "iadj": orc.lift_inv_scheme_adj}
    for kind, fn in ref.items():
        got = host(wp.w_transform_scheme(to_dev(x, torch.float64), L, taps, kind))
        assert rel_fro(got, fn(x, L, taps)) <= 1e-13, (kind, p, n1, n2, L)


@pytest.mark.parametrize("case", CASES)
def test_pinv(wp, case):
    # FP64 Moore-Penrose inverse, full and sparse (s_L, d_L only), against the
    # oracle within max(n1, n2) * kappa * eps (kappa of the kept slices).
    import torch
    rng, p, n1, n2, _, L = _draw(600 + case)
    a = rng.standard_normal((p, n1, n2))
    kap = 1.0
    for sl in orc.lift_fwd(a, L):
        s = np.linalg.svd(sl, compute_uv=False)
        kap = max(kap, s[0] / s[-1])
    tol = max(n1, n2) * kap * np.finfo(np.float64).eps
    for sparse, ref in ((False, orc.w_pinv), (True, orc.w_pinv_sparse)):
        if sparse and L == 0:
            # The sparse inverse keeps s_L and d_L, which needs a level.
            from paper_2601_08228_amd._lib import WprodError
            with pytest.raises(WprodError):
                wp.w_pinv(to_dev(a, torch.float64), L, sparse=True)
            continue
        out, info = wp.w_pinv(to_dev(a, torch.float64), L, sparse=sparse)
        assert host(info).min() > 0
        assert rel_fro(host(out), ref(a, L)) <= tol, (sparse, p, n1, n2, L)
