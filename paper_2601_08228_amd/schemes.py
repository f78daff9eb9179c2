"""Named predict / update stencils for the general lifting (Sec. II-A; Remark 3.1).

Each function returns the taps array of shape (L, 2, 5) taken by
w_transform_scheme and w_product_scheme: taps[j-1, 0] is the predict and
taps[j-1, 1] the update stencil of level j, tap t at offset t - 2.  At every
level o[m] is the first and e[m] the second entry of pair m; d = o - P e,
s = e + U d.
"""

import numpy as np

__all__ = ["lazy", "interpolating", "cdf53", "custom"]


def _empty(L):
    return np.zeros((int(L), 2, 5), dtype=np.float64)


def lazy(L):
    """P = I, U = I/2: the transform of Alg. 1 (same results as w_transform)."""
    t = _empty(L)
    t[:, 0, 2] = 1.0
    t[:, 1, 2] = 0.5
    return t


def interpolating(L):
    """Example 2.1: U = 0 and P the mean of the two kept neighbours of each
    predicted entry, e[m-1] and e[m] (offsets -1 and 0)."""
    t = _empty(L)
    t[:, 0, 1] = 0.5
    t[:, 0, 2] = 0.5
    return t


def cdf53(L):
    """Interpolating predict with the update (d[m] + d[m+1]) / 4 (the CDF 5/3
    lifting pair)."""
    t = interpolating(L)
    t[:, 1, 2] = 0.25
    t[:, 1, 3] = 0.25
    return t


def custom(levels):
    """Taps from a per-level list of (predict, update) 5-tap stencils, one
    entry per level (Remark 3.1: operators chosen level by level)."""
    t = np.asarray(levels, dtype=np.float64)
    if t.ndim != 3 or t.shape[1:] != (2, 5):
        raise ValueError("expected a list of (predict[5], update[5]) pairs")
    return np.ascontiguousarray(t)
