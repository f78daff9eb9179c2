"""Shared helpers of the GPU parity tests (test-only)."""

import numpy as np
import pytest


def device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    return torch.device("cuda:0")


def to_dev(x, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=device())


def host(t):
    return t.detach().cpu().numpy()


def cast(x, np_dtype):
    """Values the path computes on (Q17 reading): cast, then upcast for the oracle."""
    return np.asarray(x).astype(np_dtype).astype(np.float64)


def rel_fro(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((x - ref).ravel())
    return num / den if den > 0 else num


def bf16_rne(x):
    """bfloat16 round-to-nearest-even of float32 values, returned as float32 (CPU reference)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def bf16_bits_to_f32(t):
    """torch.bfloat16 device tensor -> float32 numpy array of the same values."""
    return t.float().cpu().numpy()


UNIT = {"f64": 2.0 ** -53, "f32": 2.0 ** -24}
TARGET = {"f64": 1e-12, "f32": 1e-5}


def parseval_weights(p, L):
    """Weights w_c of the weighted Parseval identity of the lifting W_[L] for a
    p-slice tensor: ||x||^2 = sum_c w_c ||xhat_c||^2 over the coefficient slices
    c of Eq. (1), w = 2^L on s_L and 2^(j-2) on d_j (W = D H with H the
    orthonormal Haar transform and D diagonal)."""
    w = np.empty(p)
    w[:p >> L] = 2.0 ** L
    for j in range(1, L + 1):
        w[p >> j:p >> (j - 1)] = 2.0 ** (j - 2)
    return w


def svd_bars(coeff, k, prec, L=None, p=None):
    """Parity bars of a truncated w-svd, derived from the oracle's singular values.

    coeff: the decomposed coefficient slices (nsl, n1, n2) in FP64, the leading
    nsl of the p coefficient slices (p = nsl by default; sp-w-svd keeps s_L and
    d_L); prec 'f64' or 'f32' (u = unit roundoff of the path's data type); L:
    the level, to weight the slices (None: the worst slice sets the tensor
    bar).  The Jacobi SVD is backward stable with a backward error of at most
    about mr u ||A_c|| per slice (mr = max(n1, n2)), so:
      * sigma: |d sigma_i| <= 4 mr u sigma_1 (Weyl);
      * A_k (= U_k U_k^T A, the projection on the computed subspace): the
        subspace moves by at most 4 mr u sigma_1 / (sigma_k - sigma_{k+1})
        (Wedin), and A_k by as much relative to its norm; at full rank the
        projection is the identity and the gap factor is 1.  The spatial
        error then follows from the weighted Parseval identity of W:
        ||dA_k||^2 = sum_c w_c ||dA_k,c||^2 <= sum_c w_c bar_c^2 ||A_k,c||^2;
      * orthogonality: the Jacobi stops at |u_i.u_j| <= sqrt(mr) u, plus the
        rounding of the dot products, normalisation and storage, and the
        polish of the recovered factor stops at 4 (sqrt(n) + 2) u:
        4 (sqrt(mr) + 8) u covers both.
    Each bar is held at the target tolerance (1e-12 FP64, 1e-5 FP32) when the
    derived one is below it.  Returns a dict with the tensor bars 'shat', 'ak',
    'orth' and the per-slice rank-k bars 'ak_slice'.
    """
    coeff = np.asarray(coeff, dtype=np.float64)
    nsl, n1, n2 = coeff.shape
    mr, nc = max(n1, n2), min(n1, n2)
    u = UNIT[prec]
    tgt = TARGET[prec]
    per, norms2, sq_err = np.full(nsl, tgt), np.zeros(nsl), 0.0
    for c in range(nsl):
        s = np.linalg.svd(coeff[c], compute_uv=False)
        norms2[c] = float(np.sum(s[:k] ** 2))
        if s[0] == 0:
            continue
        if k < nc:
            gap = s[k - 1] - s[k]
            ratio = s[0] / gap if gap > 0 else np.inf
        else:
            ratio = 1.0
        per[c] = max(tgt, 4.0 * mr * u * ratio)
        sq_err += k * (4.0 * mr * u * s[0]) ** 2
    if L is None:
        ak = float(per.max())
    else:
        wts = parseval_weights(nsl if p is None else p, L)[:nsl]
        den = float(np.sum(wts * norms2))
        ak = max(tgt, float(np.sqrt(np.sum(wts * per ** 2 * norms2) / den))) if den > 0 else tgt
    sq_ref = float(np.sum(norms2))
    shat = max(tgt, float(np.sqrt(sq_err / sq_ref))) if sq_ref > 0 else tgt
    return {"shat": shat, "ak": ak, "orth": 4.0 * (np.sqrt(mr) + 8.0) * u, "ak_slice": per}
