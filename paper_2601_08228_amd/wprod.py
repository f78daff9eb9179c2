"""Python binding of libwprod.so: the C entry points under the same names.

Argument marshalling only: each function checks that its tensors are
contiguous device tensors of a supported dtype, allocates outputs (and the
workspace) with torch, and calls the library on torch's current stream.
Tensors use the library layout: shape (p, n1, n2), frontal slices first.
Split-precision coefficients are returned as torch.bfloat16 tensors holding
the hi / lo parts.
"""

import collections
import ctypes

import numpy as np
import torch

from . import _lib

__all__ = [
    "w_transform", "w_itransform", "w_transform_adj", "w_itransform_adj",
    "w_transform_split", "w_itransform_adj_split", "w_face_product",
    "w_face_product_split", "w_face_product_gemm", "w_face_product_workspace", "w_product",
    "w_product_workspace", "w_product_noalloc", "w_product_noalloc_scratch_bytes", "w_svd",
    "w_svd_timed", "w_svd_workspace", "w_svd_sparse",
    "w_svd_sparse_workspace", "SvdResult", "w_pinv",
    "w_pinv_workspace", "SCHEME_KINDS", "w_transform_scheme", "w_transform_scheme_split",
    "w_product_scheme", "w_product_scheme_workspace",
]

_DT = {torch.float64: _lib.WP_F64, torch.float32: _lib.WP_F32}


def _stream(t):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _dev_tensor(t, name, dtypes):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be a device tensor (got %s)" % (name, t.device))
    if t.dtype not in dtypes:
        raise ValueError("%s has dtype %s; expected one of %s" % (name, t.dtype, dtypes))
    if t.dim() != 3:
        raise ValueError("%s must have shape (p, n1, n2)" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def _out_tensor(out, name, shape, dtype, device):
    """Check a caller-supplied output: device tensor on `device`, dtype, shape, contiguous."""
    if not isinstance(out, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if out.device != device:
        raise ValueError("%s is on %s; expected %s" % (name, out.device, device))
    if out.dtype != dtype:
        raise ValueError("%s has dtype %s; expected %s" % (name, out.dtype, dtype))
    if tuple(out.shape) != tuple(shape):
        raise ValueError("%s has shape %s; expected %s" % (name, tuple(out.shape), tuple(shape)))
    if not out.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return out


def _workspace(ws, need, device):
    """Allocate the workspace, or check a caller-supplied one (contiguous, on
    `device`, at least `need` bytes); returns (tensor, size in bytes)."""
    if ws is None:
        ws = torch.empty(max(int(need), 1), dtype=torch.uint8, device=device)
    else:
        if not isinstance(ws, torch.Tensor):
            raise TypeError("workspace must be a torch.Tensor")
        if ws.device != device:
            raise ValueError("workspace is on %s; expected %s" % (ws.device, device))
        if not ws.is_contiguous():
            raise ValueError("workspace must be contiguous")
        if ws.numel() * ws.element_size() < need:
            raise ValueError("workspace holds %d bytes; %d needed"
                             % (ws.numel() * ws.element_size(), need))
    return ws, ws.numel() * ws.element_size()


def _lift(fn_name, x, L, out):
    _dev_tensor(x, "x", tuple(_DT))
    if out is None:
        out = torch.empty_like(x)
    else:
        _out_tensor(out, "out", x.shape, x.dtype, x.device)
    p, n1, n2 = x.shape
    with torch.cuda.device(x.device):
        st = getattr(_lib.load(), fn_name)(_ptr(x), _ptr(out), n1, n2, p, int(L), _DT[x.dtype],
                                           _stream(x))
    _lib.check(fn_name, st)
    return out


def w_transform(x, L, out=None):
    """Forward lifting W_[L] along mode 3 (Eq. (1)); coefficients in Eq. (1) order."""
    return _lift("w_transform", x, L, out)


def w_itransform(xhat, L, out=None):
    """Inverse lifting W_[L]^{-1} (Alg. 1 inverse steps)."""
    return _lift("w_itransform", xhat, L, out)


def w_transform_adj(g, L, out=None):
    """W_[L]^T applied to coefficient-space g (reverse-mode step)."""
    return _lift("w_transform_adj", g, L, out)


def w_itransform_adj(g, L, out=None):
    """W_[L]^{-T} applied to spatial g (reverse-mode step)."""
    return _lift("w_itransform_adj", g, L, out)


def _lift_split(fn_name, x, L, with_lo):
    _dev_tensor(x, "x", (torch.float32,))
    hi = torch.empty(x.shape, dtype=torch.bfloat16, device=x.device)
    lo = torch.empty(x.shape, dtype=torch.bfloat16, device=x.device) if with_lo else None
    p, n1, n2 = x.shape
    with torch.cuda.device(x.device):
        st = getattr(_lib.load(), fn_name)(_ptr(x), _ptr(hi), _ptr(lo), n1, n2, p, int(L), _stream(x))
    _lib.check(fn_name, st)
    return hi, lo


def w_transform_split(x, L, with_lo=True):
    """Forward lifting of float32 x with bf16 hi/lo outputs (lo omitted if with_lo=False)."""
    return _lift_split("w_transform_split", x, L, with_lo)


def w_itransform_adj_split(g, L, with_lo=True):
    """W^{-T} of float32 g with bf16 hi/lo outputs."""
    return _lift_split("w_itransform_adj_split", g, L, with_lo)


def _face_dims(a, b, trans_a, trans_b):
    if a.shape[0] != b.shape[0]:
        raise ValueError("operands have different numbers of slices")
    p = a.shape[0]
    n1, n2 = (a.shape[2], a.shape[1]) if trans_a else (a.shape[1], a.shape[2])
    kb, n3 = (b.shape[2], b.shape[1]) if trans_b else (b.shape[1], b.shape[2])
    if kb != n2:
        raise ValueError("inner dimensions differ: %d vs %d" % (n2, kb))
    return p, n1, n2, n3


def w_face_product(ah, bh, trans_a=False, trans_b=False, out=None):
    """Face-product (Def. 2.1): out[k] = op(ah[k]) @ op(bh[k]) on FP64 / FP32 MFMA."""
    _dev_tensor(ah, "ah", tuple(_DT))
    _dev_tensor(bh, "bh", (ah.dtype,))
    p, n1, n2, n3 = _face_dims(ah, bh, trans_a, trans_b)
    if out is None:
        out = torch.empty((p, n1, n3), dtype=ah.dtype, device=ah.device)
    else:
        _out_tensor(out, "out", (p, n1, n3), ah.dtype, ah.device)
    with torch.cuda.device(ah.device):
        st = _lib.load().w_face_product(_ptr(ah), _ptr(bh), _ptr(out), n1, n2, n3, p, int(trans_a),
                                        int(trans_b), _DT[ah.dtype], _stream(ah))
    _lib.check("w_face_product", st)
    return out


def w_face_product_split(a_hi, a_lo, b_hi, b_lo, trans_a=False, trans_b=False, gemm="bf16x3",
                         out=None):
    """Face-product of split operands on BF16 MFMA with FP32 accumulation (float32 result)."""
    mode = _lib.GEMM_MODES[gemm]
    if mode == 0:
        raise ValueError("split face-product needs gemm='bf16' or 'bf16x3'")
    _dev_tensor(a_hi, "a_hi", (torch.bfloat16,))
    _dev_tensor(b_hi, "b_hi", (torch.bfloat16,))
    if gemm == "bf16x3":
        _dev_tensor(a_lo, "a_lo", (torch.bfloat16,))
        _dev_tensor(b_lo, "b_lo", (torch.bfloat16,))
    else:
        a_lo = b_lo = None
    p, n1, n2, n3 = _face_dims(a_hi, b_hi, trans_a, trans_b)
    for t, name in ((a_lo, "a_lo"), (b_hi, "b_hi"), (b_lo, "b_lo")):
        if t is not None and t.device != a_hi.device:
            raise ValueError("%s is on %s; expected %s" % (name, t.device, a_hi.device))
    if out is None:
        out = torch.empty((p, n1, n3), dtype=torch.float32, device=a_hi.device)
    else:
        _out_tensor(out, "out", (p, n1, n3), torch.float32, a_hi.device)
    with torch.cuda.device(a_hi.device):
        st = _lib.load().w_face_product_split(_ptr(a_hi), _ptr(a_lo), _ptr(b_hi), _ptr(b_lo),
                                              _ptr(out), n1, n2, n3, p, int(trans_a),
                                              int(trans_b), mode, _stream(a_hi))
    _lib.check("w_face_product_split", st)
    return out


def w_face_product_workspace(n1, n2, n3, p, dtype=torch.float32, gemm="native"):
    return int(_lib.load().w_face_product_workspace(n1, n2, n3, p, _DT[dtype],
                                                    _lib.GEMM_MODES[gemm]))


def w_face_product_gemm(ah, bh, trans_a=False, trans_b=False, gemm="native", out=None,
                        workspace=None):
    """Face-product (Def. 2.1) in one call for every arithmetic: 'native' (FP64 /
    FP32 MFMA), or 'bf16' / 'bf16x3' of float32 coefficients, split into bf16
    hi / lo planes inside the call."""
    _dev_tensor(ah, "ah", tuple(_DT))
    _dev_tensor(bh, "bh", (ah.dtype,))
    if bh.device != ah.device:
        raise ValueError("bh is on %s; expected %s" % (bh.device, ah.device))
    p, n1, n2, n3 = _face_dims(ah, bh, trans_a, trans_b)
    mode = _lib.GEMM_MODES[gemm]
    if out is None:
        out = torch.empty((p, n1, n3), dtype=ah.dtype, device=ah.device)
    else:
        _out_tensor(out, "out", (p, n1, n3), ah.dtype, ah.device)
    need = w_face_product_workspace(n1, n2, n3, p, ah.dtype, gemm) if ah.dtype in _DT else 0
    workspace, nbytes = _workspace(workspace, need, ah.device)
    with torch.cuda.device(ah.device):
        st = _lib.load().w_face_product_gemm(_ptr(ah), _ptr(bh), _ptr(out), n1, n2, n3, p,
                                             int(trans_a), int(trans_b), _DT[ah.dtype], mode,
                                             _ptr(workspace), nbytes, _stream(ah))
    _lib.check("w_face_product_gemm", st)
    return out


def w_product_workspace(n1, n2, n3, p, L, dtype=torch.float32, gemm="native"):
    return int(_lib.load().w_product_workspace(n1, n2, n3, p, int(L), _DT[dtype],
                                               _lib.GEMM_MODES[gemm]))


def w_product(a, b, L, trans_a=False, trans_b=False, gemm="native", out=None, workspace=None):
    """w-product C = op(A) *_w op(B) (Def. 2.1, Alg. 1) in one library call."""
    _dev_tensor(a, "a", tuple(_DT))
    _dev_tensor(b, "b", (a.dtype,))
    if b.device != a.device:
        raise ValueError("b is on %s; expected %s" % (b.device, a.device))
    p, n1, n2, n3 = _face_dims(a, b, trans_a, trans_b)
    mode = _lib.GEMM_MODES[gemm]
    need = w_product_workspace(n1, n2, n3, p, L, a.dtype, gemm)
    workspace, nbytes = _workspace(workspace, need, a.device)
    if out is None:
        out = torch.empty((p, n1, n3), dtype=a.dtype, device=a.device)
    else:
        _out_tensor(out, "out", (p, n1, n3), a.dtype, a.device)
    with torch.cuda.device(a.device):
        st = _lib.load().w_product(_ptr(a), _ptr(b), _ptr(out), n1, n2, n3, p, int(L), int(trans_a),
                                   int(trans_b), _DT[a.dtype], mode, _ptr(workspace), nbytes,
                                   _stream(a))
    _lib.check("w_product", st)
    return out


def w_product_noalloc_scratch_bytes():
    return int(_lib.load().w_product_noalloc_scratch_bytes())


def w_product_noalloc(a, b, L, trans_a=False, trans_b=False, gemm="native", out=None):
    """w_product with the library's fixed device scratch instead of a workspace:
    the library allocates nothing (pass `out` to allocate nothing at all).
    Calls that overlap on one device race on that scratch."""
    _dev_tensor(a, "a", tuple(_DT))
    _dev_tensor(b, "b", (a.dtype,))
    if b.device != a.device:
        raise ValueError("b is on %s; expected %s" % (b.device, a.device))
    p, n1, n2, n3 = _face_dims(a, b, trans_a, trans_b)
    if out is None:
        out = torch.empty((p, n1, n3), dtype=a.dtype, device=a.device)
    else:
        _out_tensor(out, "out", (p, n1, n3), a.dtype, a.device)
    with torch.cuda.device(a.device):
        st = _lib.load().w_product_noalloc(_ptr(a), _ptr(b), _ptr(out), n1, n2, n3, p, int(L),
                                           int(trans_a), int(trans_b), _DT[a.dtype],
                                           _lib.GEMM_MODES[gemm], _stream(a))
    _lib.check("w_product_noalloc", st)
    return out


SvdResult = collections.namedtuple("SvdResult", "uhat shat vhat ak info orth_err")


def w_svd_workspace(n1, n2, p, L, k, dtype=torch.float32):
    return int(_lib.load().w_svd_workspace(n1, n2, p, int(L), int(k), _DT[dtype]))


def w_svd_sparse_workspace(n1, n2, p, L, k, dtype=torch.float32):
    return int(_lib.load().w_svd_sparse_workspace(n1, n2, p, int(L), int(k), _DT[dtype]))


def _svd_call(name, a, L, k, nsl, max_sweeps, want_ak, want_orth, workspace, events=()):
    _dev_tensor(a, "a", tuple(_DT))
    p, n1, n2 = a.shape
    k = int(k)
    dev = a.device
    nsl = max(int(nsl), 0)
    uhat = torch.empty((nsl, n1, k), dtype=a.dtype, device=dev)
    shat = torch.empty((nsl, k), dtype=a.dtype, device=dev)
    vhat = torch.empty((nsl, n2, k), dtype=a.dtype, device=dev)
    ak = torch.empty_like(a) if want_ak else None
    info = torch.empty((nsl,), dtype=torch.int32, device=dev)
    orth = torch.empty((2,), dtype=torch.float64, device=dev) if want_orth else None
    lib = _lib.load()
    ws_name = name[:-len("_timed")] if name.endswith("_timed") else name
    need = getattr(lib, ws_name + "_workspace")(n1, n2, p, int(L), k, _DT[a.dtype])
    workspace, nbytes = _workspace(workspace, need, dev)
    with torch.cuda.device(dev):
        st = getattr(lib, name)(_ptr(a), n1, n2, p, int(L), k, _ptr(uhat), _ptr(shat), _ptr(vhat),
                                _ptr(ak), int(max_sweeps), _ptr(info), _ptr(orth), _DT[a.dtype],
                                _ptr(workspace), nbytes, _stream(a), *events)
    _lib.check(name, st)
    return SvdResult(uhat, shat, vhat, ak, info, orth)


def w_svd(a, L, k, max_sweeps=0, want_ak=True, want_orth=True, workspace=None):
    """Truncated w-svd (Alg. 2): wavelet-domain factors, rank-k approximation, Jacobi info.

    Returns SvdResult(uhat (p,n1,k), shat (p,k), vhat (p,n2,k), ak (p,n1,n2) or None,
    info (p,) int32 device tensor, orth_err (2,) float64 device tensor or None).
    Nothing is synchronised; info[k] < 0 marks a slice that did not converge.
    """
    p = a.shape[0] if a.dim() == 3 else 0
    return _svd_call("w_svd", a, L, k, p, max_sweeps, want_ak, want_orth, workspace)


def w_svd_timed(a, L, k, jacobi_begin, jacobi_end, max_sweeps=0, want_ak=True, want_orth=True,
                workspace=None):
    """w_svd with two torch.cuda.Event objects (created with enable_timing=True)
    recorded on the current stream just before and after the Jacobi stage, so
    that jacobi_begin.elapsed_time(jacobi_end) times the decomposition alone."""
    evs = []
    for ev, name in ((jacobi_begin, "jacobi_begin"), (jacobi_end, "jacobi_end")):
        if not isinstance(ev, torch.cuda.Event):
            raise TypeError("%s must be a torch.cuda.Event" % name)
        if not ev.cuda_event:
            ev.record()  # torch creates the HIP event on its first record
        evs.append(ctypes.c_void_p(ev.cuda_event))
    p = a.shape[0] if a.dim() == 3 else 0
    return _svd_call("w_svd_timed", a, L, k, p, max_sweeps, want_ak, want_orth, workspace,
                     tuple(evs))


def w_svd_sparse(a, L, k, max_sweeps=0, want_ak=True, want_orth=True, workspace=None):
    """sp-w-svd (Sec. IV-B): w-svd of the s_L and d_L slices only, finer details dropped.

    Same results as w_svd, but the factors and info hold nk = 2 p / 2^L slices
    (s_L then d_L); ak is (p, n1, n2).  Needs L >= 1.
    """
    p = a.shape[0] if a.dim() == 3 else 0
    nsl = 2 * (p >> int(L)) if int(L) >= 1 else 0
    return _svd_call("w_svd_sparse", a, L, k, nsl, max_sweeps, want_ak, want_orth, workspace)


def w_pinv_workspace(n1, n2, p, L, sparse=False, dtype=torch.float64):
    return int(_lib.load().w_pinv_workspace(n1, n2, p, int(L), int(bool(sparse)), _DT[dtype]))


def w_pinv(a, L, sparse=False, rtol=0.0, workspace=None):
    """Moore-Penrose inverse A^+ (Def. 2.6): returns (out (p, n2, n1), info).

    sparse=True inverts only s_L and d_L (sp-w-product, Sec. IV-C).  rtol = 0
    selects max(n1, n2) * machine epsilon.  info (int32 device tensor, one per
    inverted coefficient slice) is negative for a slice whose SVD did not
    converge.  Nothing is synchronised.
    """
    _dev_tensor(a, "a", tuple(_DT))
    p, n1, n2 = a.shape
    nsl = (2 * (p >> int(L)) if int(L) >= 1 else 0) if sparse else p
    out = torch.empty((p, n2, n1), dtype=a.dtype, device=a.device)
    info = torch.empty((max(nsl, 0),), dtype=torch.int32, device=a.device)
    lib = _lib.load()
    need = lib.w_pinv_workspace(n1, n2, p, int(L), int(bool(sparse)), _DT[a.dtype])
    workspace, nbytes = _workspace(workspace, need, a.device)
    with torch.cuda.device(a.device):
        st = lib.w_pinv(_ptr(a), _ptr(out), n1, n2, p, int(L), int(bool(sparse)), float(rtol),
                        _ptr(info), _DT[a.dtype], _ptr(workspace), nbytes, _stream(a))
    _lib.check("w_pinv", st)
    return out, info


# ---- lifting with chosen predict / update stencils (Sec. II-A; Remark 3.1) ----

SCHEME_KINDS = {"forward": 0, "inverse": 1, "adj": 2, "iadj": 3}


def _taps(taps, L):
    """Host copy of the taps as a C-contiguous float64 array of shape (L, 2, 5)."""
    t = np.ascontiguousarray(np.asarray(taps, dtype=np.float64))
    if t.shape != (int(L), 2, 5):
        raise ValueError("taps must have shape (%d, 2, 5), got %s" % (int(L), t.shape))
    return t


def w_transform_scheme(x, L, taps, kind="forward", out=None):
    """One pass of the lifting with stencils taps (L, 2, 5): kind 'forward' (W),
    'inverse' (W^{-1}), 'adj' (W^T) or 'iadj' (W^{-T})."""
    _dev_tensor(x, "x", tuple(_DT))
    t = _taps(taps, L)
    if out is None:
        out = torch.empty_like(x)
    else:
        _out_tensor(out, "out", x.shape, x.dtype, x.device)
    p, n1, n2 = x.shape
    with torch.cuda.device(x.device):
        st = _lib.load().w_transform_scheme(_ptr(x), _ptr(out), n1, n2, p, int(L),
                                            t.ctypes.data, SCHEME_KINDS[kind], _DT[x.dtype],
                                            _stream(x))
    _lib.check("w_transform_scheme", st)
    return out


def w_transform_scheme_split(x, L, taps, kind="forward", with_lo=True):
    """'forward' or 'iadj' pass of float32 x with bf16 hi / lo outputs."""
    _dev_tensor(x, "x", (torch.float32,))
    t = _taps(taps, L)
    hi = torch.empty(x.shape, dtype=torch.bfloat16, device=x.device)
    lo = torch.empty(x.shape, dtype=torch.bfloat16, device=x.device) if with_lo else None
    p, n1, n2 = x.shape
    with torch.cuda.device(x.device):
        st = _lib.load().w_transform_scheme_split(_ptr(x), _ptr(hi), _ptr(lo), n1, n2, p, int(L),
                                                  t.ctypes.data, SCHEME_KINDS[kind], _stream(x))
    _lib.check("w_transform_scheme_split", st)
    return hi, lo


def w_product_scheme_workspace(n1, n2, n3, p, L, dtype=torch.float32, gemm="native"):
    return int(_lib.load().w_product_scheme_workspace(n1, n2, n3, p, int(L), _DT[dtype],
                                                      _lib.GEMM_MODES[gemm]))


def w_product_scheme(a, b, L, taps, trans_a=False, trans_b=False, gemm="native", out=None,
                     workspace=None):
    """w-product (Def. 2.1) under the lifting with stencils taps (L, 2, 5)."""
    _dev_tensor(a, "a", tuple(_DT))
    _dev_tensor(b, "b", (a.dtype,))
    if b.device != a.device:
        raise ValueError("b is on %s; expected %s" % (b.device, a.device))
    t = _taps(taps, L)
    p, n1, n2, n3 = _face_dims(a, b, trans_a, trans_b)
    mode = _lib.GEMM_MODES[gemm]
    need = w_product_scheme_workspace(n1, n2, n3, p, L, a.dtype, gemm)
    workspace, nbytes = _workspace(workspace, need, a.device)
    if out is None:
        out = torch.empty((p, n1, n3), dtype=a.dtype, device=a.device)
    else:
        _out_tensor(out, "out", (p, n1, n3), a.dtype, a.device)
    with torch.cuda.device(a.device):
        st = _lib.load().w_product_scheme(_ptr(a), _ptr(b), _ptr(out), n1, n2, n3, p, int(L),
                                          t.ctypes.data, int(trans_a), int(trans_b),
                                          _DT[a.dtype], mode, _ptr(workspace), nbytes,
                                          _stream(a))
    _lib.check("w_product_scheme", st)
    return out
