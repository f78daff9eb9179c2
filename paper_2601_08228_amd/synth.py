"""Seeded synthetic inputs for the w-product workloads.

This module only draws random numbers and builds input tensors; it holds none
of the w-product's arithmetic (no lifting, no face-product), so both the HIP
path and the FP64 oracle can be fed from it.  Every array is float64 of shape
(p, n1, n2) (frontal slices first) unless stated; callers cast to the path
dtype and give the oracle exactly the cast values.

The hyperspectral-like generator stands in for the paper's hyperspectral
images (Sec. IV, Tables 3 and 4), which are not available: smooth spectra,
spatially correlated abundance maps, values in [0, 1], few components.
"""

import numpy as np

__all__ = ["normal", "uniform", "hsi_like", "gaussian_band", "toeplitz_blur", "stack_slices",
           "normal_device",
           "uniform_device"]


def normal(shape, seed, scale=1.0):
    """i.i.d. N(0, scale^2) from numpy's PCG64 generator."""
    return np.random.default_rng(seed).standard_normal(shape) * scale


def uniform(shape, seed, lo=-1.0, hi=1.0):
    """i.i.d. U(lo, hi) from numpy's PCG64 generator."""
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


def _smooth_periodic(z, sigma_px):
    """Periodic Gaussian smoothing of a 2-D field through the FFT."""
    n1, n2 = z.shape
    f1 = np.fft.fftfreq(n1)[:, None]
    f2 = np.fft.fftfreq(n2)[None, :]
    kern = np.exp(-2.0 * (np.pi * sigma_px) ** 2 * (f1 ** 2 + f2 ** 2))
    return np.real(np.fft.ifft2(np.fft.fft2(z) * kern))


def hsi_like(n1, n2, p, seed, components=12, noise=0.01, sigma_px=8.0):
    """Hyperspectral-like tensor (p, n1, n2): sum of rank-1 map x spectrum terms.

    Draw order: all spatial maps, then all spectra, then the noise.
      map r:      N(0,1) field smoothed with a periodic Gaussian (sigma_px
                  pixels), min-max scaled to [0, 1];
      spectrum r: 3 Gaussian bumps over the p bands, centre ~ U(0, p-1),
                  width ~ U(p/40, p/8), amplitude ~ U(0.2, 1), scaled so its
                  maximum is 1;
      X = (1/R) sum_r spectrum_r[:, None, None] * map_r[None] + N(0, noise^2).
    """
    rng = np.random.default_rng(seed)
    maps = []
    for _r in range(components):
        m = _smooth_periodic(rng.standard_normal((n1, n2)), sigma_px)
        m = (m - m.min()) / (m.max() - m.min())
        maps.append(m)
    bands = np.arange(p, dtype=np.float64)
    sigs = []
    for _r in range(components):
        s = np.zeros(p)
        for _b in range(3):
            centre = rng.uniform(0.0, p - 1.0)
            width = rng.uniform(p / 40.0, p / 8.0)
            amp = rng.uniform(0.2, 1.0)
            s += amp * np.exp(-((bands - centre) ** 2) / (2.0 * width ** 2))
        sigs.append(s / s.max())
    x = np.zeros((p, n1, n2))
    for m, s in zip(maps, sigs):
        x += s[:, None, None] * m[None, :, :]
    x /= components
    if noise > 0:
        x += rng.standard_normal((p, n1, n2)) * noise
    return x


def gaussian_band(n, sigma=1.5, half_width=4):
    """Banded Gaussian blur matrix G (n x n), 2*half_width+1 diagonals.

    G[i, j] = exp(-(i-j)^2 / (2 sigma^2)) / Z for |i - j| <= half_width, with Z
    the sum of the kernel over its 2*half_width+1 taps, so interior rows sum
    to 1; rows near the border are truncated, not renormalised.
    """
    t = np.arange(-half_width, half_width + 1, dtype=np.float64)
    z = np.sum(np.exp(-(t ** 2) / (2.0 * sigma ** 2)))
    g = np.zeros((n, n))
    for i in range(n):
        for j in range(max(0, i - half_width), min(n, i + half_width + 1)):
            g[i, j] = np.exp(-((i - j) ** 2) / (2.0 * sigma ** 2)) / z
    return g


def toeplitz_blur(n, b):
    """Linear-decay blur matrix of the deblurring experiment (Sec. IV-C), n x n:
    T[i, j] = (b - |i - j|) / (3 b) for |i - j| < b, zero elsewhere."""
    dist = np.abs(np.arange(n)[:, None] - np.arange(n)[None, :]).astype(np.float64)
    return np.where(dist < b, (b - dist) / (3.0 * b), 0.0)


def stack_slices(mat, p):
    """Tensor whose p frontal slices all equal ``mat`` (shape (p, n1, n2))."""
    return np.repeat(np.asarray(mat, dtype=np.float64)[None], p, axis=0)


def normal_device(shape, seed, device, dtype=None, scale=1.0):
    """i.i.d. N(0, scale^2) drawn on the device by torch's seeded generator (for large inputs)."""
    import torch
    gen = torch.Generator(device=device).manual_seed(int(seed))
    x = torch.randn(shape, generator=gen, device=device, dtype=dtype or torch.float32)
    return x.mul_(scale) if scale != 1.0 else x


def uniform_device(shape, seed, device, lo=-1.0, hi=1.0, dtype=None):
    """i.i.d. U(lo, hi) drawn on the device by torch's seeded generator (for large inputs)."""
    import torch
    gen = torch.Generator(device=device).manual_seed(int(seed))
    x = torch.rand(shape, generator=gen, device=device, dtype=dtype or torch.float32)
    return x.mul_(hi - lo).add_(lo)
