"""Host-side checks of the C ABI: the library loads, exports every declared symbol,
and rejects invalid arguments before touching the GPU (no compute call is made)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wprod.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\**\s+\**(w_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2601_08228_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libwprod.so not built")
    return _lib.load()


def test_header_declares_expected_entry_points():
    names = _declared_functions()
    for must in ["w_transform", "w_itransform", "w_transform_adj", "w_itransform_adj",
                 "w_transform_split", "w_itransform_adj_split", "w_face_product",
                 "w_face_product_split", "w_product", "w_product_workspace", "w_svd",
                 "w_svd_workspace", "w_svd_sparse", "w_svd_sparse_workspace", "w_pinv",
                 "w_pinv_workspace", "w_transform_scheme", "w_transform_scheme_split",
                 "w_product_scheme", "w_product_scheme_workspace", "w_status_string", "w_version"]:
        assert must in names, must


def test_library_exports_every_declared_symbol(lib):
    from paper_2601_08228_amd import _lib
    for name in _declared_functions():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, name


def test_status_strings(lib):
    for code in [0, -1, -2, -3, -4, -5, -6, -7]:
        s = lib.w_status_string(code).decode()
        assert s.startswith("WP_")
    assert lib.w_status_string(-99).decode() == "unknown wp_status"
    assert lib.w_version() >= 100


# Fake, never dereferenced addresses: every call below fails validation first.
A = ctypes.c_void_p(0x100000)
B = ctypes.c_void_p(0x200000)
C = ctypes.c_void_p(0x300000)
WS = ctypes.c_void_p(0x400000)
NULL = None


@pytest.mark.parametrize("fn", ["w_transform", "w_itransform", "w_transform_adj", "w_itransform_adj"])
def test_transform_validation(lib, fn):
    f = getattr(lib, fn)
    assert f(A, B, 4, 4, 6, 2, 1, NULL) == -1          # p not a multiple of 2^L
    assert f(A, B, 4, 4, 8, -1, 1, NULL) == -1         # negative level
    assert f(A, B, 4, 4, 2048, 11, 1, NULL) == -1      # more than 10 levels
    assert f(A, B, 0, 4, 8, 1, 1, NULL) == -1          # empty slice
    assert f(A, B, 4, 4, 0, 0, 1, NULL) == -1          # no slices
    assert f(A, B, 1 << 20, 1 << 20, 1 << 4, 1, 1, NULL) == -1  # too many elements
    assert f(A, B, 4, 4, 8, 1, 7, NULL) == -4          # unknown dtype
    assert f(NULL, B, 4, 4, 8, 1, 1, NULL) == -2
    assert f(A, NULL, 4, 4, 8, 1, 1, NULL) == -2
    # out overlaps in (4*4*8 floats = 512 bytes)
    assert f(A, ctypes.c_void_p(0x100000 + 256), 4, 4, 8, 1, 1, NULL) == -3
    assert f(A, A, 4, 4, 8, 1, 0, NULL) == -3


def test_split_validation(lib):
    for fn in ("w_transform_split", "w_itransform_adj_split"):
        f = getattr(lib, fn)
        assert f(A, B, C, 4, 4, 6, 2, NULL) == -1
        assert f(NULL, B, C, 4, 4, 8, 2, NULL) == -2
        assert f(A, NULL, C, 4, 4, 8, 2, NULL) == -2
        assert f(A, B, ctypes.c_void_p(0x200000 + 64), 4, 4, 8, 2, NULL) == -3  # hi/lo overlap
        assert f(A, ctypes.c_void_p(0x100000 + 64), NULL, 4, 4, 8, 2, NULL) == -3


def test_face_product_validation(lib):
    f = lib.w_face_product
    assert f(A, B, C, 4, 5, 6, 3, 0, 0, 5, NULL) == -4
    assert f(A, B, C, 4, 0, 6, 3, 0, 0, 1, NULL) == -1
    assert f(A, B, C, 4, 5, 6, 3, 2, 0, 1, NULL) == -1     # bad flag
    assert f(A, NULL, C, 4, 5, 6, 3, 0, 0, 1, NULL) == -2
    assert f(A, B, ctypes.c_void_p(0x200000 + 4), 4, 5, 6, 3, 0, 0, 1, NULL) == -3
    g = lib.w_face_product_split
    assert g(A, NULL, B, NULL, C, 4, 5, 6, 3, 0, 0, 0, NULL) == -4  # native mode invalid here
    assert g(A, NULL, B, NULL, C, 4, 5, 6, 3, 0, 0, 2, NULL) == -2  # bf16x3 needs lo planes
    assert g(NULL, NULL, B, NULL, C, 4, 5, 6, 3, 0, 0, 1, NULL) == -2
    assert g(A, NULL, B, NULL, ctypes.c_void_p(0x100000), 4, 5, 6, 3, 0, 0, 1, NULL) == -3


def test_product_validation_and_workspace(lib):
    ws_f32 = lib.w_product_workspace(4, 5, 6, 8, 3, 1, 0)
    ws_x3 = lib.w_product_workspace(4, 5, 6, 8, 3, 1, 2)
    ws_f64 = lib.w_product_workspace(4, 5, 6, 8, 3, 0, 0)
    assert ws_f32 >= 8 * (20 + 30 + 24) * 4
    assert ws_f64 >= 8 * (20 + 30 + 24) * 8
    assert ws_x3 >= 8 * (20 + 30) * 4 + 8 * 24 * 4
    assert lib.w_product_workspace(4, 5, 6, 8, 3, 0, 2) == 0     # bf16x3 needs F32
    assert lib.w_product_workspace(4, 5, 6, 6, 3, 1, 0) == 0     # bad level
    f = lib.w_product
    args = (4, 5, 6, 8, 3, 0, 0, 1, 0)
    assert f(A, B, C, *args, WS, ws_f32 - 1, NULL) == -5
    assert f(A, B, C, *args, NULL, ws_f32, NULL) == -2
    assert f(A, B, C, 4, 5, 6, 8, 3, 0, 0, 0, 2, WS, 1 << 30, NULL) == -4
    assert f(A, B, C, 4, 5, 6, 8, 3, 0, 0, 1, 9, WS, 1 << 30, NULL) == -4
    assert f(A, B, C, 4, 5, 6, 6, 3, 0, 0, 1, 0, WS, 1 << 30, NULL) == -1
    assert f(A, B, A, *args, WS, ws_f32, NULL) == -3                       # C aliases A
    assert f(A, B, C, *args, ctypes.c_void_p(0x300000 + 16), ws_f32, NULL) == -3  # ws overlaps C


def test_svd_validation(lib):
    need = lib.w_svd_workspace(8, 6, 16, 2, 3, 1)
    assert need > 0
    assert lib.w_svd_workspace(8, 6, 16, 2, 7, 1) == 0           # k > min(n1, n2)
    assert lib.w_svd_workspace(2049, 6, 16, 2, 3, 1) == 0        # n1 > 2048
    f = lib.w_svd
    U, S, V, AK = (ctypes.c_void_p(0x500000), ctypes.c_void_p(0x600000),
                   ctypes.c_void_p(0x700000), ctypes.c_void_p(0x800000))
    INFO, ORTH = ctypes.c_void_p(0x900000), ctypes.c_void_p(0xA00000)
    W = ctypes.c_void_p(0x10000000)
    assert f(A, 8, 6, 16, 2, 0, U, S, V, AK, 0, INFO, ORTH, 1, W, need, NULL) == -1
    assert f(A, 8, 6, 16, 2, 7, U, S, V, AK, 0, INFO, ORTH, 1, W, need, NULL) == -1
    assert f(A, 8, 6, 12, 3, 3, U, S, V, AK, 0, INFO, ORTH, 1, W, need, NULL) == -1
    assert f(A, 8, 6, 16, 2, 3, U, S, V, AK, 0, INFO, ORTH, 3, W, need, NULL) == -4
    assert f(A, 8, 6, 16, 2, 3, U, S, V, AK, 0, NULL, ORTH, 1, W, need, NULL) == -2
    assert f(A, 8, 6, 16, 2, 3, U, S, V, AK, 0, INFO, ORTH, 1, W, need - 1, NULL) == -5
    assert f(A, 8, 6, 16, 2, 3, A, S, V, AK, 0, INFO, ORTH, 1, W, need, NULL) == -3
    assert f(A, 8, 6, 16, 2, 3, U, U, V, AK, 0, INFO, ORTH, 1, W, need, NULL) == -3


def test_sparse_svd_validation(lib):
    need = lib.w_svd_sparse_workspace(8, 6, 16, 2, 3, 1)
    assert 0 < need < lib.w_svd_workspace(8, 6, 16, 2, 3, 1)   # 8 of 16 slices decomposed
    assert lib.w_svd_sparse_workspace(8, 6, 16, 0, 3, 1) == 0   # needs L >= 1
    assert lib.w_svd_sparse_workspace(8, 6, 16, 2, 7, 1) == 0   # k > min(n1, n2)
    f = lib.w_svd_sparse
    U, S, V, AK = (ctypes.c_void_p(0x500000), ctypes.c_void_p(0x600000),
                   ctypes.c_void_p(0x700000), ctypes.c_void_p(0x800000))
    INFO, ORTH = ctypes.c_void_p(0x900000), ctypes.c_void_p(0xA00000)
    W = ctypes.c_void_p(0x10000000)
    assert f(A, 8, 6, 16, 0, 3, U, S, V, AK, 0, INFO, ORTH, 1, W, need, NULL) == -1
    assert f(A, 8, 6, 12, 3, 3, U, S, V, AK, 0, INFO, ORTH, 1, W, need, NULL) == -1
    assert f(A, 8, 6, 16, 2, 3, U, S, V, AK, 0, INFO, ORTH, 2, W, need, NULL) == -4
    assert f(A, 8, 6, 16, 2, 3, NULL, S, V, AK, 0, INFO, ORTH, 1, W, need, NULL) == -2
    assert f(A, 8, 6, 16, 2, 3, U, S, V, AK, 0, INFO, ORTH, 1, W, need - 1, NULL) == -5
    # uhat holds 8 slices * 8 * 3 floats = 768 bytes; shat inside it is an alias.
    assert f(A, 8, 6, 16, 2, 3, U, ctypes.c_void_p(0x500000 + 764), V, AK, 0, INFO, ORTH, 1, W,
             need, NULL) == -3


def test_pinv_validation(lib):
    need = lib.w_pinv_workspace(8, 6, 16, 2, 0, 1)
    assert need > 0
    assert 0 < lib.w_pinv_workspace(8, 6, 16, 2, 1, 1) < need     # sparse: 8 of 16 slices
    assert lib.w_pinv_workspace(8, 6, 16, 0, 1, 1) == 0            # sparse needs L >= 1
    assert lib.w_pinv_workspace(8, 6, 12, 3, 0, 1) == 0            # p not divisible by 2^L
    assert lib.w_pinv_workspace(2100, 6, 16, 2, 0, 1) == 0         # n1 > 2048
    assert lib.w_pinv_workspace(8, 6, 16, 2, 0, 2) == 0            # bad dtype code
    f = lib.w_pinv
    OUT, INFO = ctypes.c_void_p(0x500000), ctypes.c_void_p(0x900000)
    W = ctypes.c_void_p(0x10000000)
    assert f(A, OUT, 8, 6, 12, 3, 0, 0.0, INFO, 1, W, need, NULL) == -1
    assert f(A, OUT, 8, 6, 16, 2, 0, -1e-3, INFO, 1, W, need, NULL) == -1
    assert f(A, OUT, 8, 6, 16, 2, 0, float("nan"), INFO, 1, W, need, NULL) == -1
    assert f(A, OUT, 8, 6, 16, 2, 0, 1.0, INFO, 1, W, need, NULL) == -1
    assert f(A, OUT, 8, 6, 16, 2, 0, 0.0, INFO, 2, W, need, NULL) == -4
    assert f(A, NULL, 8, 6, 16, 2, 0, 0.0, INFO, 1, W, need, NULL) == -2
    assert f(A, OUT, 8, 6, 16, 2, 0, 0.0, NULL, 1, W, need, NULL) == -2
    assert f(A, OUT, 8, 6, 16, 2, 0, 0.0, INFO, 1, W, need - 1, NULL) == -5
    # a holds 16 * 8 * 6 floats = 3072 bytes: an output starting inside it aliases.
    assert f(A, ctypes.c_void_p(0x100000 + 3068), 8, 6, 16, 2, 0, 0.0, INFO, 1, W, need,
             NULL) == -3
    # info (16 int32) overlapping the output.
    assert f(A, OUT, 8, 6, 16, 2, 0, 0.0, ctypes.c_void_p(0x500000 + 3068), 1, W, need,
             NULL) == -3


def _taps(L, fill=0.25):
    import numpy as np
    return np.full((L, 2, 5), fill)


def test_scheme_transform_validation(lib):
    import numpy as np
    f = lib.w_transform_scheme
    t = _taps(2)
    T = t.ctypes.data
    assert f(A, B, 4, 4, 12, 3, T, 0, 1, NULL) == -1               # p not divisible by 2^L
    assert f(A, B, 4, 4, 16, 2, T, 4, 1, NULL) == -1               # unknown kind
    assert f(A, B, 4, 4, 16, 2, T, 0, 2, NULL) == -4               # bad dtype
    assert f(A, B, 4, 4, 16, 2, None, 0, 1, NULL) == -2            # taps missing
    bad = _taps(2)
    bad[1, 1, 3] = np.nan
    assert f(A, B, 4, 4, 16, 2, bad.ctypes.data, 0, 1, NULL) == -1
    bad[1, 1, 3] = np.inf
    assert f(A, B, 4, 4, 16, 2, bad.ctypes.data, 0, 1, NULL) == -1
    assert f(A, B, 4, 4, 2048, 2, T, 0, 0, NULL) == -1             # FP64 tubes too long for LDS
    assert f(NULL, B, 4, 4, 16, 2, T, 0, 1, NULL) == -2
    # a holds 4 * 4 * 16 floats = 1024 bytes: an output starting inside it aliases.
    assert f(A, ctypes.c_void_p(0x100000 + 1020), 4, 4, 16, 2, T, 0, 1, NULL) == -3
    g = lib.w_transform_scheme_split
    assert g(A, B, C, 4, 4, 16, 2, T, 1, NULL) == -1               # split only for W and W^{-T}
    assert g(A, B, C, 4, 4, 16, 2, None, 0, NULL) == -2
    assert g(A, ctypes.c_void_p(0x100000 + 1000), C, 4, 4, 16, 2, T, 0, NULL) == -3


def test_scheme_product_validation(lib):
    import numpy as np
    t = _taps(2)
    assert lib.w_product_scheme_workspace(3, 4, 5, 16, 2, 1, 0) == \
        lib.w_product_workspace(3, 4, 5, 16, 2, 1, 0)
    assert lib.w_product_scheme_workspace(3, 4, 5, 4096, 2, 1, 0) == 0   # p too long
    need = lib.w_product_scheme_workspace(3, 4, 5, 16, 2, 1, 2)
    assert need > 0
    f = lib.w_product_scheme
    assert f(A, B, C, 3, 4, 5, 16, 2, t.ctypes.data, 0, 0, 1, 2, WS, need - 1, NULL) == -5
    assert f(A, B, C, 3, 4, 5, 16, 2, t.ctypes.data, 0, 0, 0, 2, WS, need, NULL) == -4
    assert f(A, B, C, 3, 4, 5, 16, 2, None, 0, 0, 1, 2, WS, need, NULL) == -2
    bad = _taps(2)
    bad[0, 0, 0] = np.nan
    assert f(A, B, C, 3, 4, 5, 16, 2, bad.ctypes.data, 0, 0, 1, 2, WS, need, NULL) == -1
    assert f(A, B, C, 3, 4, 5, 16, 2, t.ctypes.data, 2, 0, 1, 2, WS, need, NULL) == -1


def test_named_schemes_match_the_oracle():
    import numpy as np
    import oracle as orc
    from paper_2601_08228_amd import schemes
    for L in (1, 3):
        np.testing.assert_array_equal(schemes.lazy(L), orc.lazy_scheme(L))
        np.testing.assert_array_equal(schemes.interpolating(L), orc.interpolating_scheme(L))
        np.testing.assert_array_equal(schemes.cdf53(L), orc.cdf53_scheme(L))


def test_product_path_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2601_08228_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()
