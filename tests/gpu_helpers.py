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
