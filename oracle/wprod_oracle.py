"""FP64 NumPy oracle of the w-product, its adjoint and the w-svd.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code,
header, table or helper with the HIP implementation; inputs reach it as plain
arrays.

Paper: Panchal & Behera, "Second-Generation Wavelet-inspired Tensor Product
with Applications in Hyperspectral Imaging" (arXiv 2601.08228).

Storage convention (same as the HIP library, chosen independently here):
a tensor A in R^{n1 x n2 x p} is held as an array of shape (p, n1, n2), so
``A[k]`` is the frontal slice A^(k+1) of Sec. II and ``A[:, i, j]`` is the
mode-3 tube A[i+1, j+1, :].  Coefficient tensors use the same shape with the
slices in the order of Eq. (1): s_L, d_L, d_{L-1}, ..., d_1.  With m = p/2^L,
s_L occupies slices [0, m) and d_j occupies [p/2^j, p/2^(j-1)).

Every function computes in float64 and returns float64 arrays.  Loops are
written out; NumPy is used for the slice-wise matrix products, the per-slice
SVD and elementwise arithmetic only.

Readings of the paper taken here (each listed in the design notes):
  * pairs are (slice 2q, slice 2q+1) with 0-based q; d = first - second and
    s = second + d/2 (Alg. 1 forward steps; fixed by Example 2.2, where
    A_d1^(1) = A^(1) - A^(2));
  * coefficients are packed as in Eq. (1), p slices in total (the codomain
    written after Def. 2.1 omits s_L and is read as a typo);
  * p must be a multiple of 2^L; L = 0 is allowed and means no transform;
  * the identity tensor is W^{-1} of "every coefficient slice is I"
    (s_L and all d_j; the intermediate s_j, j < L, are not coefficients);
  * pseudo-inverse and truncated SVD act per coefficient slice (Thm 2.5,
    Thm 2.6 and Remark 2.2, whose printed values this reading reproduces);
  * PSNR uses MPP^2 in the numerator; with data in [0, 1], MPP = 1;
  * general lifting (Sec. II-A with chosen P_j, U_j; Remark 3.1): the
    predicted entries are the first of each pair and the kept ones the second
    (the odd and even entries of Alg. 1, whose indices are 1-based), so that
    P_j = I, U_j = I/2 is exactly the lazy transform above; P_j and U_j are
    5-tap stencils with the sequence extended by its end values.
"""

import numpy as np

__all__ = [
    "check_levels", "lift_fwd", "lift_inv", "lift_fwd_adj", "lift_inv_adj",
    "face", "w_product", "w_product_vjp", "transpose", "identity", "inverse",
    "trace", "slice_svd", "w_svd", "w_svd_sparse", "spatial_factors", "w_pinv", "psnr",
    "lsq_grad", "deblur_gd", "coefficient_weights", "w_pinv_sparse", "toeplitz_blur",
    "pinv_deblur", "SCHEME_TAPS", "scheme_operators", "lift_fwd_scheme", "lift_inv_scheme",
    "scheme_matrix", "scheme_inverse_matrix", "lift_fwd_scheme_adj", "lift_inv_scheme_adj",
    "w_product_scheme", "w_product_scheme_vjp", "lazy_scheme", "interpolating_scheme",
    "cdf53_scheme",
]


def check_levels(p, L):
    """p = 2^L m with integers m >= 1, L >= 0 (Sec. II-A, Eq. (1))."""
    if L < 0 or p <= 0 or p % (1 << L) != 0:
        raise ValueError(f"p={p} is not a positive multiple of 2^L (L={L})")


def lift_fwd(x, L):
    """Forward lazy lifting W_[L] along mode 3 (Eq. (1); Alg. 1, forward part).

    With P_j = I and U_j = I/2 (Sec. II-A), each level splits the current
    smooth sequence into pairs (first, second), predicts d_j = first - second
    and updates s_j = second + d_j / 2.  Returns (s_L, d_L, ..., d_1) stacked
    along axis 0.
    """
    x = np.asarray(x, dtype=np.float64)
    p = x.shape[0]
    check_levels(p, L)
    s = x.copy()
    details = []                       # details[j-1] = d_j
    for _j in range(1, L + 1):
        first = s[0::2]
        second = s[1::2]
        d = first - second
        s = second + d / 2.0
        details.append(d)
    return np.concatenate([s] + details[::-1], axis=0)


def _split_coefficients(c, L):
    """Views (s_L, {j: d_j}) of a Mallat-ordered coefficient tensor."""
    p = c.shape[0]
    m = p >> L
    d = {j: c[p >> j: p >> (j - 1)] for j in range(1, L + 1)}
    return c[:m], d


def lift_inv(c, L):
    """Inverse lifting W_[L]^{-1} (Eq. (3) per-level inverse; Alg. 1, inverse part).

    For j = L down to 1: second = s_j - d_j / 2, first = d_j + second, and
    s_{j-1} interleaves (first, second).
    """
    c = np.asarray(c, dtype=np.float64)
    p = c.shape[0]
    check_levels(p, L)
    s, d = _split_coefficients(c, L)
    s = s.copy()
    for j in range(L, 0, -1):
        second = s - d[j] / 2.0
        first = d[j] + second
        nxt = np.empty((2 * s.shape[0],) + s.shape[1:], dtype=np.float64)
        nxt[0::2] = first
        nxt[1::2] = second
        s = nxt
    return s


def lift_fwd_adj(g, L):
    """Transpose W_[L]^T (not in the paper; needed by the adjoint of Def. 2.1).

    W_[L] = W_L ... W_1, so W_[L]^T = W_1^T ... W_L^T: the level-L step is
    transposed first.  One forward level maps (first, second) to
    (s, d) = (first/2 + second/2, first - second); its transpose maps
    (g_s, g_d) to (first, second) = (g_s/2 + g_d, g_s/2 - g_d).
    """
    g = np.asarray(g, dtype=np.float64)
    p = g.shape[0]
    check_levels(p, L)
    gs, gd = _split_coefficients(g, L)
    gs = gs.copy()
    for j in range(L, 0, -1):
        first = gs / 2.0 + gd[j]
        second = gs / 2.0 - gd[j]
        nxt = np.empty((2 * gs.shape[0],) + gs.shape[1:], dtype=np.float64)
        nxt[0::2] = first
        nxt[1::2] = second
        gs = nxt
    return gs


def lift_inv_adj(g, L):
    """Transpose of the inverse, W_[L]^{-T} (not in the paper).

    W^{-1} = W_1^{-1} ... W_L^{-1}, so W^{-T} = W_L^{-T} ... W_1^{-T}: the
    level-1 step is transposed first.  One inverse level maps (s, d) to
    (first, second) = (s + d/2, s - d/2); its transpose maps (g_first,
    g_second) to (g_s, g_d) = (g_first + g_second, (g_first - g_second)/2).
    Returns Mallat order like lift_fwd.
    """
    g = np.asarray(g, dtype=np.float64)
    p = g.shape[0]
    check_levels(p, L)
    s = g.copy()
    details = []
    for _j in range(1, L + 1):
        gf = s[0::2]
        gsec = s[1::2]
        details.append((gf - gsec) / 2.0)
        s = gf + gsec
    return np.concatenate([s] + details[::-1], axis=0)


def _op(m, trans):
    return m.T if trans else m


def face(ah, bh, trans_a=False, trans_b=False):
    """Face-product Delta: slice-wise matrix products (Def. 2.1; Alg. 1, middle part).

    ``trans_a`` / ``trans_b`` use the stored slices transposed (Def. 2.2),
    so the stored operand shapes are (p, n2, n1) / (p, n3, n2).
    """
    ah = np.asarray(ah, dtype=np.float64)
    bh = np.asarray(bh, dtype=np.float64)
    if ah.shape[0] != bh.shape[0]:
        raise ValueError("operands have different numbers of slices")
    out = []
    for k in range(ah.shape[0]):
        out.append(_op(ah[k], trans_a) @ _op(bh[k], trans_b))
    return np.stack(out, axis=0)


def w_product(a, b, L, trans_a=False, trans_b=False):
    """A *_w B = W^{-1}( W(A) Delta W(B) ) (Def. 2.1, Alg. 1).

    The transposes act per slice before the product; by Thm 2.1 it does not
    matter whether they are taken before or after the transform.
    """
    return lift_inv(face(lift_fwd(a, L), lift_fwd(b, L), trans_a, trans_b), L)


def w_product_vjp(a, b, g, L):
    """Reverse-mode derivative of C = A *_w B for the loss <G, C>.

    Chain rule through Def. 2.1: Ghat = W^{-T} G, dAhat = Ghat Delta Bhat^T,
    dBhat = Ahat^T Delta Ghat, dA = W^T dAhat, dB = W^T dBhat.
    """
    ah = lift_fwd(a, L)
    bh = lift_fwd(b, L)
    gh = lift_inv_adj(g, L)
    da = lift_fwd_adj(face(gh, bh, trans_b=True), L)
    db = lift_fwd_adj(face(ah, gh, trans_a=True), L)
    return da, db


def transpose(a):
    """Tensor transpose A^T[i, j, :] = A[j, i, :] (Def. 2.2)."""
    return np.ascontiguousarray(np.swapaxes(np.asarray(a, dtype=np.float64), 1, 2))


def identity(n, p, L):
    """Identity tensor: every coefficient slice equals I_n, mapped back by W^{-1} (Def. 2.3)."""
    check_levels(p, L)
    coeff = np.stack([np.eye(n) for _ in range(p)], axis=0)
    return lift_inv(coeff, L)


def inverse(a, L):
    """Tensor inverse: invert each coefficient slice, then W^{-1} (Def. 2.4)."""
    ah = lift_fwd(a, L)
    return lift_inv(np.stack([np.linalg.inv(ah[k]) for k in range(ah.shape[0])]), L)


def trace(a):
    """Tr(A) = sum over k and i of A[i, i, k] (Def. 2.7)."""
    a = np.asarray(a, dtype=np.float64)
    total = 0.0
    for k in range(a.shape[0]):
        total += float(np.trace(a[k]))
    return total


def slice_svd(m):
    """Thin SVD of one coefficient slice with a fixed sign convention.

    LAPACK (numpy.linalg.svd) in float64; singular values descending.  Signs
    are normalised so that the entry of largest magnitude in each left
    singular vector is positive (the lowest row index wins ties); the right
    vector is flipped with it, so U diag(s) V^T is unchanged.
    """
    u, s, vt = np.linalg.svd(np.asarray(m, dtype=np.float64), full_matrices=False)
    v = vt.T.copy()
    for i in range(s.shape[0]):
        col = u[:, i]
        piv = int(np.argmax(np.abs(col)))
        if col[piv] < 0:
            u[:, i] = -u[:, i]
            v[:, i] = -v[:, i]
    return u, s, v


def w_svd(a, L, k):
    """Truncated w-svd (Alg. 2; Thm 2.5).

    Each coefficient slice of W(A) is decomposed, the k largest singular
    triplets are kept and the slice is rebuilt as U_k diag(s_k) V_k^T; W^{-1}
    of the rebuilt coefficients is the rank-k approximation A_k.

    Returns (Uhat (p, n1, k), shat (p, k), Vhat (p, n2, k), Ak (p, n1, n2)):
    the wavelet-domain factors and the approximation.
    """
    a = np.asarray(a, dtype=np.float64)
    p, n1, n2 = a.shape
    if not 1 <= k <= min(n1, n2):
        raise ValueError("rank k out of range")
    ah = lift_fwd(a, L)
    uh = np.empty((p, n1, k))
    sh = np.empty((p, k))
    vh = np.empty((p, n2, k))
    ch = np.empty((p, n1, n2))
    for c in range(p):
        u, s, v = slice_svd(ah[c])
        uh[c] = u[:, :k]
        sh[c] = s[:k]
        vh[c] = v[:, :k]
        ch[c] = (u[:, :k] * s[:k]) @ v[:, :k].T
    return uh, sh, vh, lift_inv(ch, L)


def w_svd_sparse(a, L, k):
    """Sparse w-svd, sp-w-svd (Sec. IV-B, computational analysis).

    Only the coarsest coefficients carry the information kept: the s_L and
    d_L slices (slices [0, 2m) of W(A), m = p/2^L) are decomposed and
    truncated to rank k as in Alg. 2; the finer details d_j, j < L, are set
    to zero before W^{-1}.  Requires L >= 1.

    Returns (Uhat (2m, n1, k), shat (2m, k), Vhat (2m, n2, k), Ak (p, n1, n2)).
    """
    a = np.asarray(a, dtype=np.float64)
    p, n1, n2 = a.shape
    if L < 1:
        raise ValueError("sp-w-svd needs L >= 1")
    if not 1 <= k <= min(n1, n2):
        raise ValueError("rank k out of range")
    ah = lift_fwd(a, L)
    kept = 2 * (p >> L)
    uh = np.empty((kept, n1, k))
    sh = np.empty((kept, k))
    vh = np.empty((kept, n2, k))
    ch = np.zeros((p, n1, n2))
    for c in range(kept):
        u, s, v = slice_svd(ah[c])
        uh[c] = u[:, :k]
        sh[c] = s[:k]
        vh[c] = v[:, :k]
        ch[c] = (u[:, :k] * s[:k]) @ v[:, :k].T
    return uh, sh, vh, lift_inv(ch, L)


def spatial_factors(uh, sh, vh, L):
    """Spatial-domain factors U, Sigma, V of Thm 2.5: W^{-1} of each coefficient factor."""
    p, k = sh.shape
    sig = np.zeros((p, k, k))
    for c in range(p):
        sig[c] = np.diag(sh[c])
    return lift_inv(uh, L), lift_inv(sig, L), lift_inv(vh, L)


def w_pinv(a, L, rtol=None):
    """Moore-Penrose inverse under *_w (Def. 2.6, Thm 2.6).

    Per coefficient slice: V diag(1/s) U^T over the singular values above
    rtol * s_max (default rtol = max(n1, n2) * machine epsilon), then W^{-1}.
    The result has shape (p, n2, n1).
    """
    ah = lift_fwd(a, L)
    p, n1, n2 = ah.shape
    if rtol is None:
        rtol = max(n1, n2) * np.finfo(np.float64).eps
    out = np.empty((p, n2, n1))
    for c in range(p):
        u, s, vt = np.linalg.svd(ah[c], full_matrices=False)
        cut = rtol * (s[0] if s.size else 0.0)
        inv = np.array([1.0 / x if x > cut else 0.0 for x in s])
        out[c] = (vt.T * inv) @ u.T
    return lift_inv(out, L)


def w_pinv_sparse(a, L, rtol=None):
    """Sparse Moore-Penrose inverse (the sp-w-product deblurring of Sec. IV-C).

    As w_pinv, but only the coarsest coefficient blocks s_L and d_L (slices
    [0, 2p/2^L)) are inverted; the finer detail slices of the result are zero.
    Requires L >= 1.
    """
    ah = lift_fwd(a, L)
    p, n1, n2 = ah.shape
    if L < 1:
        raise ValueError("the sparse pseudo-inverse needs L >= 1")
    if rtol is None:
        rtol = max(n1, n2) * np.finfo(np.float64).eps
    out = np.zeros((p, n2, n1))
    for c in range(2 * (p >> L)):
        u, s, vt = np.linalg.svd(ah[c], full_matrices=False)
        cut = rtol * (s[0] if s.size else 0.0)
        inv = np.array([1.0 / x if x > cut else 0.0 for x in s])
        out[c] = (vt.T * inv) @ u.T
    return lift_inv(out, L)


def toeplitz_blur(n, b):
    """Linear blur matrix of Sec. IV-C: entry (i, j) = c(|i - j|) with
    c(j) = (b - j) / (3 b) for 0 <= j < b and 0 otherwise."""
    out = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            dist = abs(i - j)
            if dist < b:
                out[i, j] = (b - dist) / (3.0 * b)
    return out


def pinv_deblur(bt, av, ah, L, sparse=False):
    """Least-squares deblurring of Sec. IV-C: X = A_V^+ *_w B *_w (A_H^T)^+.

    bt: blurred tensor (p, n1, n2); av: (p, n1, n1); ah: (p, n2, n2).  With
    sparse=True the pseudo-inverses are the sparse ones (sp-w-product).
    (A_H^T)^+ = (A_H^+)^T, since the pseudo-inverse acts per coefficient slice
    and the transpose commutes with W (Thm 2.1).
    """
    pinv = w_pinv_sparse if sparse else w_pinv
    return w_product(w_product(pinv(av, L), bt, L), pinv(ah, L), L, trans_b=True)


def coefficient_weights(p, L):
    """Squared norms of the synthesis vectors: ||x||^2 = sum_c w_c ||xhat_c||^2.

    Not stated in the paper; it follows from the closed form of W^{-1}: each
    s_L coefficient is spread over 2^L samples with weight 1 and each d_j
    coefficient over 2^j samples with weight +-1/2, and these synthesis
    vectors are mutually orthogonal.  So w = 2^L on s_L and 2^j / 4 on d_j.
    """
    check_levels(p, L)
    w = np.empty(p)
    w[: p >> L] = float(1 << L)
    for j in range(1, L + 1):
        w[p >> j: p >> (j - 1)] = (1 << j) / 4.0
    return w


def psnr(x1, x2, mpp=1.0):
    """PSNR of Sec. IV-A with MPP^2 in the numerator: 10 log10(N MPP^2 / ||X1 - X2||_F^2)."""
    x1 = np.asarray(x1, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    err = float(np.sum((x1 - x2) ** 2))
    return 10.0 * np.log10(x1.size * mpp * mpp / err)


def lsq_grad(k, x, y, L):
    """Gradient of f(X) = ||K *_w X - Y||_F^2 with respect to X.

    df = 2 <R, K *_w dX> with R = K *_w X - Y, so by the chain rule through
    Def. 2.1 the gradient is W^T( Khat^T Delta W^{-T}(2R) ).
    """
    r = w_product(k, x, L) - np.asarray(y, dtype=np.float64)
    kh = lift_fwd(k, L)
    return lift_fwd_adj(face(kh, lift_inv_adj(2.0 * r, L), trans_a=True), L)


def deblur_gd(k, y, L, steps, eta, x0=None):
    """Fixed-step gradient descent X <- X - eta * grad f(X) for min ||K *_w X - Y||_F^2.

    Returns the final iterate and the loss before every step and after the last.
    """
    x = np.zeros_like(np.asarray(y, dtype=np.float64)) if x0 is None else np.array(x0, dtype=np.float64)
    losses = []
    for _t in range(steps):
        r = w_product(k, x, L) - y
        losses.append(float(np.sum(r * r)))
        x = x - eta * lsq_grad(k, x, y, L)
    r = w_product(k, x, L) - y
    losses.append(float(np.sum(r * r)))
    return x, losses


# ---- General predict / update lifting (Sec. II-A, W_j; Remark 3.1) -----------

SCHEME_TAPS = 5   # stencil taps at offsets -2, -1, 0, 1, 2


def _check_taps(taps, L):
    taps = np.asarray(taps, dtype=np.float64)
    if taps.shape != (L, 2, SCHEME_TAPS):
        raise ValueError(f"taps must have shape ({L}, 2, {SCHEME_TAPS}), got {taps.shape}")
    return taps


def scheme_operators(n, pred, upd):
    """P_j and U_j of one level as n x n matrices (n = pairs per tube).

    P(e)[m] = sum_t pred[t] e[clamp(m + t - 2)] and U(d)[m] likewise, the
    index clamped to [0, n - 1]: the sequence is extended by its end values.
    """
    P = np.zeros((n, n))
    U = np.zeros((n, n))
    for m in range(n):
        for t in range(SCHEME_TAPS):
            i = min(max(m + t - 2, 0), n - 1)
            P[m, i] += pred[t]
            U[m, i] += upd[t]
    return P, U


def _along0(mat, x):
    """Apply the matrix to every mode-3 tube (axis 0) of x."""
    return np.tensordot(mat, x, axes=(1, 0))


def lift_fwd_scheme(x, L, taps):
    """W_[L] with chosen predict and update operators (Sec. II-A, W_j).

    taps[j-1] = (predict stencil, update stencil) of level j.  Each level takes
    the first entry of every pair as o and the second as e, then
    d_j = o - P_j e and s_j = e + U_j d_j.  Returns (s_L, d_L, ..., d_1).
    """
    x = np.asarray(x, dtype=np.float64)
    check_levels(x.shape[0], L)
    taps = _check_taps(taps, L)
    s = x.copy()
    details = []
    for j in range(1, L + 1):
        o = s[0::2]
        e = s[1::2]
        P, U = scheme_operators(e.shape[0], taps[j - 1, 0], taps[j - 1, 1])
        d = o - _along0(P, e)
        s = e + _along0(U, d)
        details.append(d)
    return np.concatenate([s] + details[::-1], axis=0)


def lift_inv_scheme(c, L, taps):
    """W_[L]^{-1} with chosen P_j, U_j (Sec. II-A, W_j^{-1}): for j = L down to
    1, e = s_j - U_j d_j and o = d_j + P_j e, interleaved as (o, e) pairs."""
    c = np.asarray(c, dtype=np.float64)
    check_levels(c.shape[0], L)
    taps = _check_taps(taps, L)
    s, d = _split_coefficients(c, L)
    s = s.copy()
    for j in range(L, 0, -1):
        P, U = scheme_operators(s.shape[0], taps[j - 1, 0], taps[j - 1, 1])
        e = s - _along0(U, d[j])
        o = d[j] + _along0(P, e)
        nxt = np.empty((2 * s.shape[0],) + s.shape[1:], dtype=np.float64)
        nxt[0::2] = o
        nxt[1::2] = e
        s = nxt
    return s


def scheme_matrix(p, L, taps):
    """The p x p matrix of W_[L] (column i = W applied to the i-th unit tube)."""
    return lift_fwd_scheme(np.eye(p), L, taps)


def scheme_inverse_matrix(p, L, taps):
    """The p x p matrix of W_[L]^{-1}, column by column from lift_inv_scheme."""
    return lift_inv_scheme(np.eye(p), L, taps)


def lift_fwd_scheme_adj(g, L, taps):
    """W_[L]^T (not in the paper; the adjoint of Def. 2.1 needs it): the
    transpose of the explicit matrix, applied to every tube."""
    g = np.asarray(g, dtype=np.float64)
    return _along0(scheme_matrix(g.shape[0], L, taps).T, g)


def lift_inv_scheme_adj(g, L, taps):
    """W_[L]^{-T}: the transpose of the explicit inverse matrix."""
    g = np.asarray(g, dtype=np.float64)
    return _along0(scheme_inverse_matrix(g.shape[0], L, taps).T, g)


def w_product_scheme(a, b, L, taps, trans_a=False, trans_b=False):
    """A *_w B (Def. 2.1) with the lifting of chosen P_j, U_j (Remark 3.1)."""
    return lift_inv_scheme(face(lift_fwd_scheme(a, L, taps), lift_fwd_scheme(b, L, taps),
                                trans_a, trans_b), L, taps)


def w_product_scheme_vjp(a, b, g, L, taps):
    """Reverse-mode derivative of C = A *_w B under a general scheme (chain rule
    through Def. 2.1 with the explicit transposes)."""
    ah = lift_fwd_scheme(a, L, taps)
    bh = lift_fwd_scheme(b, L, taps)
    gh = lift_inv_scheme_adj(g, L, taps)
    da = lift_fwd_scheme_adj(face(gh, bh, trans_b=True), L, taps)
    db = lift_fwd_scheme_adj(face(ah, gh, trans_a=True), L, taps)
    return da, db


def lazy_scheme(L):
    """P_j = I, U_j = I/2 at every level: the lazy transform (Sec. II-A)."""
    t = np.zeros((L, 2, SCHEME_TAPS))
    t[:, 0, 2] = 1.0
    t[:, 1, 2] = 0.5
    return t


def interpolating_scheme(L):
    """Example 2.1: U_j = 0 and P_j the linear interpolate of the two kept
    neighbours.  The predicted entry o[m] = f[2m] lies between e[m-1] = f[2m-1]
    and e[m] = f[2m+1], so P(e)[m] = (e[m-1] + e[m]) / 2 (taps at -1 and 0)."""
    t = np.zeros((L, 2, SCHEME_TAPS))
    t[:, 0, 1] = 0.5
    t[:, 0, 2] = 0.5
    return t


def cdf53_scheme(L):
    """The interpolating predict with the update U(d)[m] = (d[m] + d[m+1]) / 4
    (taps at 0 and +1): the kept entry e[m] = f[2m+1] lies between the predicted
    o[m] and o[m+1].  This is the CDF 5/3 pair of lifting steps."""
    t = interpolating_scheme(L)
    t[:, 1, 2] = 0.25
    t[:, 1, 3] = 0.25
    return t
