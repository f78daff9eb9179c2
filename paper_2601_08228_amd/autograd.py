"""Reverse-mode derivative of the w-product as a torch.autograd.Function.

Forward (Def. 2.1, Alg. 1): Ahat = W A, Bhat = W B, Chat = Ahat Delta Bhat,
C = W^{-1} Chat.  For a cotangent G of C the chain rule gives
Ghat = W^{-T} G, dAhat = Ghat Delta Bhat^T, dBhat = Ahat^T Delta Ghat and
dA = W^T dAhat, dB = W^T dBhat: two transposed lifting passes, two
transposed face-products and one W^{-T} pass, every one a library kernel.
The same holds for a lifting with chosen predict / update stencils, whose
W^T and W^{-T} passes the library also provides.
In the split-precision modes the saved coefficients are the bf16 hi/lo
planes written by the forward lifting, and W^{-T} G is split the same way.

`forward_kernels` / `backward_kernels` run exactly those library calls; an
optional `mark(name)` callback is invoked after each call (one kernel each),
which is how the benchmark brackets individual kernels with events.
"""

import torch

from . import wprod as _w

__all__ = ["WProduct", "w_product_ad", "forward_kernels", "backward_kernels"]


def _noop(_name):
    return None


def _lifts(L, scheme):
    """The lifting calls of one scheme: (fwd, inv, adj, iadj, fwd_split, iadj_split)."""
    if scheme is None:
        return (lambda x: _w.w_transform(x, L), lambda x: _w.w_itransform(x, L),
                lambda x: _w.w_transform_adj(x, L), lambda x: _w.w_itransform_adj(x, L),
                lambda x, lo: _w.w_transform_split(x, L, with_lo=lo),
                lambda x, lo: _w.w_itransform_adj_split(x, L, with_lo=lo))
    return (lambda x: _w.w_transform_scheme(x, L, scheme, "forward"),
            lambda x: _w.w_transform_scheme(x, L, scheme, "inverse"),
            lambda x: _w.w_transform_scheme(x, L, scheme, "adj"),
            lambda x: _w.w_transform_scheme(x, L, scheme, "iadj"),
            lambda x, lo: _w.w_transform_scheme_split(x, L, scheme, "forward", with_lo=lo),
            lambda x, lo: _w.w_transform_scheme_split(x, L, scheme, "iadj", with_lo=lo))


def forward_kernels(a, b, L, gemm="native", mark=_noop, scheme=None):
    """C = A *_w B; returns (C, saved coefficients for the backward pass).

    scheme: None for the lazy lifting, else the (L, 2, 5) predict / update taps
    of a general lifting (Sec. II-A; Remark 3.1)."""
    fwd, inv, _, _, fwd_split, _ = _lifts(L, scheme)
    if gemm == "native":
        ah = fwd(a)
        mark("lift_fwd")
        bh = fwd(b)
        mark("lift_fwd")
        ch = _w.w_face_product(ah, bh)
        mark("face")
        saved = (ah, None, bh, None)
    else:
        x3 = gemm == "bf16x3"
        ahi, alo = fwd_split(a, x3)
        mark("lift_fwd_split")
        bhi, blo = fwd_split(b, x3)
        mark("lift_fwd_split")
        ch = _w.w_face_product_split(ahi, alo, bhi, blo, gemm=gemm)
        mark("face")
        saved = (ahi, alo, bhi, blo)
    c = inv(ch)
    mark("lift_inv")
    return c, saved


def backward_kernels(saved, g, L, gemm="native", need_a=True, need_b=True, mark=_noop,
                     scheme=None):
    """(dA, dB) for the cotangent g of C, from the coefficients saved by forward_kernels."""
    _, _, adj, iadj, _, iadj_split = _lifts(L, scheme)
    a0, a1, b0, b1 = saved
    da = db = None
    if gemm == "native":
        gh = iadj(g)
        mark("lift_inv_adj")
        if need_a:
            dah = _w.w_face_product(gh, b0, trans_b=True)
            mark("face_tb")
            da = adj(dah)
            mark("lift_fwd_adj")
        if need_b:
            dbh = _w.w_face_product(a0, gh, trans_a=True)
            mark("face_ta")
            db = adj(dbh)
            mark("lift_fwd_adj")
    else:
        ghi, glo = iadj_split(g, gemm == "bf16x3")
        mark("lift_inv_adj_split")
        if need_a:
            dah = _w.w_face_product_split(ghi, glo, b0, b1, trans_b=True, gemm=gemm)
            mark("face_tb")
            da = adj(dah)
            mark("lift_fwd_adj")
        if need_b:
            dbh = _w.w_face_product_split(a0, a1, ghi, glo, trans_a=True, gemm=gemm)
            mark("face_ta")
            db = adj(dbh)
            mark("lift_fwd_adj")
    return da, db


class WProduct(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, b, L, gemm, scheme=None):
        c, saved = forward_kernels(a.contiguous(), b.contiguous(), int(L), gemm, scheme=scheme)
        ctx.L = int(L)
        ctx.gemm = gemm
        ctx.scheme = scheme
        ctx.n_saved = [t is not None for t in saved]
        ctx.save_for_backward(*[t for t in saved if t is not None])
        return c

    @staticmethod
    def backward(ctx, g):
        it = iter(ctx.saved_tensors)
        saved = tuple(next(it) if present else None for present in ctx.n_saved)
        da, db = backward_kernels(saved, g.contiguous(), ctx.L, ctx.gemm,
                                  ctx.needs_input_grad[0], ctx.needs_input_grad[1],
                                  scheme=ctx.scheme)
        return da, db, None, None, None


def w_product_ad(a, b, L, gemm="native", scheme=None):
    """Differentiable w-product A *_w B (gemm: 'native', 'bf16' or 'bf16x3'; scheme:
    None for the lazy lifting or (L, 2, 5) predict / update taps)."""
    return WProduct.apply(a, b, L, gemm, scheme)
