"""Least-squares deblurring min_X ||K *_w X - Y||_F^2 by fixed-step gradient descent.

The gradient 2 K^T *_w (K *_w X - Y) comes from the library's reverse-mode
w-product (WProduct): forward lifting of K and X, face-product, inverse
lifting, then W^{-T}, a transposed face-product and W^T.  The residual, the
loss and the update are elementwise tensor operations on the device.
"""

import torch

from .autograd import WProduct
from . import wprod as _w

__all__ = ["lsq_gradient", "solve", "GraphedSolver", "pinv_deblur"]


def lsq_gradient(k, x, y, L, gemm="native"):
    """Gradient of ||K *_w X - Y||_F^2 with respect to X (device tensors)."""
    xv = x.detach().clone().requires_grad_(True)
    r = WProduct.apply(k, xv, L, gemm) - y
    (r * r).sum().backward()
    return xv.grad


def solve(k, y, L, steps, eta, gemm="native", x0=None):
    """Run `steps` iterations X <- X - eta * grad from X0 (zeros by default).

    Returns the final iterate and the losses before each step (host floats,
    read back once at the end).
    """
    x = torch.zeros_like(y) if x0 is None else x0.detach().clone()
    losses = []
    for _ in range(steps):
        xv = x.requires_grad_(True)
        r = WProduct.apply(k, xv, L, gemm) - y
        loss = (r * r).sum()
        loss.backward()
        losses.append(loss.detach())
        with torch.no_grad():
            x = (xv - eta * xv.grad).detach()
    return x, [float(v) for v in torch.stack(losses).cpu()]


class GraphedSolver:
    """The gradient step of `solve` captured once in a HIP graph and replayed.

    The step (forward w-product through WProduct, residual, the reverse pass
    for X with cotangent 2 r, the update X <- X - eta * grad) is a dozen
    short kernels and host-side library calls; replaying the captured graph
    removes the per-launch host cost, which sets the pace of the eager loop
    for small problems and the split-precision modes.  The loss is a
    reduction and stays outside the graph (`residual_norm2` evaluates it on
    demand).  k, y and the iterate are static tensors; `x` always holds the
    current iterate.
    """

    def __init__(self, k, y, L, eta, gemm="native", x0=None, warmup=2):
        self.k, self.y, self.L, self.eta, self.gemm = k, y, int(L), float(eta), gemm
        start = torch.zeros_like(y) if x0 is None else x0.detach().clone()
        self.x = start.clone().requires_grad_(True)
        # Warm-up on a side stream (default priority): first-call set-up happens
        # outside the capture.
        side = torch.cuda.Stream(device=y.device)
        side.wait_stream(torch.cuda.current_stream(y.device))
        with torch.cuda.stream(side):
            for _ in range(warmup):
                self._step()
        torch.cuda.current_stream(y.device).wait_stream(side)
        with torch.no_grad():
            self.x.copy_(start)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._step()

    def _step(self):
        c = WProduct.apply(self.k, self.x, self.L, self.gemm)
        r = c - self.y
        (g,) = torch.autograd.grad(c, self.x, grad_outputs=2.0 * r)
        with torch.no_grad():
            self.x.sub_(self.eta * g)

    def run(self, steps):
        """Replay the step `steps` times on the current stream."""
        for _ in range(steps):
            self.graph.replay()
        return self.x.detach()

    def residual_norm2(self):
        """||K *_w X - Y||_F^2 at the current iterate (eager, not captured)."""
        with torch.no_grad():
            r = WProduct.apply(self.k, self.x.detach(), self.L, self.gemm) - self.y
            return float((r * r).sum())


def pinv_deblur(b, av, ah, L, sparse=False, gemm="native"):
    """X = A_V^+ *_w B *_w (A_H^T)^+ (Sec. IV-C) with library calls only:
    two pseudo-inverses (sparse=True: sp-w-product) and two w-products, the
    second with A_H^+ transposed ((A_H^T)^+ = (A_H^+)^T).

    Returns (X, (info_v, info_h)); the info tensors report Jacobi convergence.
    """
    pv, info_v = _w.w_pinv(av, L, sparse=sparse)
    ph, info_h = _w.w_pinv(ah, L, sparse=sparse)
    t = _w.w_product(pv, b, L, gemm=gemm)
    x = _w.w_product(t, ph, L, trans_b=True, gemm=gemm)
    return x, (info_v, info_h)
