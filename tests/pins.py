"""Independent routes used to pin the oracle (test-only helpers).

The dense transform matrices below are built from closed forms of the lazy
lifting (sums over dyadic blocks, derived by unrolling the level recursion of
Eq. (1) and its inverse), not by calling the oracle's level loops, so a wrong
sign, index or packing order in either route shows up as a mismatch.
"""

import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        raw = json.load(f)
    out = {}
    for key, val in raw.items():
        out[key] = np.array(val, dtype=np.float64) if isinstance(val, list) else val
    return out


def bit(t, j):
    return (t >> j) & 1


def dense_forward(p, L):
    """p x p matrix of W_[L] in Mallat order, from the block-sum closed form.

    s_L[b]  = 2^-L * sum of x[t] over the block t >> L == b;
    d_j[q]  = 2^-(j-1) * (sum over the first half of block q at scale 2^j
                          minus sum over its second half), i.e. the sign is
              + where bit (j-1) of t is 0 and - where it is 1.
    """
    m = p >> L
    w = np.zeros((p, p))
    for b in range(m):
        for t in range(p):
            if t >> L == b:
                w[b, t] = 2.0 ** (-L)
    for j in range(1, L + 1):
        off = p >> j
        for q in range(p >> j):
            for t in range(p):
                if t >> j == q:
                    w[off + q, t] = 2.0 ** (-(j - 1)) * (1.0 if bit(t, j - 1) == 0 else -1.0)
    return w


def dense_inverse(p, L):
    """p x p matrix of W_[L]^{-1}: x[t] = s_L[t>>L] + sum_j (1/2)(-1)^bit_{j-1}(t) d_j[t>>j]."""
    m = p >> L
    w = np.zeros((p, p))
    for t in range(p):
        w[t, t >> L] = 1.0
        for j in range(1, L + 1):
            off = p >> j
            w[t, off + (t >> j)] = 0.5 * (1.0 if bit(t, j - 1) == 0 else -1.0)
    assert m >= 1
    return w


def apply_mode3(mat, x):
    """(mat applied along axis 0): out[c] = sum_t mat[c, t] x[t]."""
    return np.einsum("ct,tij->cij", mat, x)


def brute_w_product(a, b, L):
    """C[k,i,j] = sum_{t,k1,k2} A[k1,i,t] B[k2,t,j] T[k,k1,k2], T[k,k1,k2] = sum_c Winv[k,c] W[c,k1] W[c,k2].

    Written with explicit loops; use only on tiny tensors.
    """
    p, n1, n2 = a.shape
    n3 = b.shape[2]
    w = dense_forward(p, L)
    wi = dense_inverse(p, L)
    t3 = np.zeros((p, p, p))
    for k in range(p):
        for k1 in range(p):
            for k2 in range(p):
                t3[k, k1, k2] = sum(wi[k, c] * w[c, k1] * w[c, k2] for c in range(p))
    out = np.zeros((p, n1, n3))
    for k in range(p):
        for i in range(n1):
            for j in range(n3):
                acc = 0.0
                for k1 in range(p):
                    for k2 in range(p):
                        if t3[k, k1, k2] == 0.0:
                            continue
                        for t in range(n2):
                            acc += a[k1, i, t] * b[k2, t, j] * t3[k, k1, k2]
                out[k, i, j] = acc
    return out


def rel_fro(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((x - ref).ravel())
    return num / den if den > 0 else num
