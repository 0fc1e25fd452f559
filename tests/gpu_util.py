"""Shared helpers of the GPU tests (inputs and comparisons; no solver code)."""
import numpy as np


def smooth_density(shape, seed, lo=0.5, hi=4.0):
    """Positive smooth periodic density with a few random Fourier modes."""
    rng = np.random.default_rng(seed)
    axes = np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in shape], indexing="ij")
    s = np.zeros(shape)
    for g in axes:
        for k in (1, 2):
            s += rng.standard_normal() * np.sin(k * g + rng.uniform(0, 6))
    s = (s - s.min()) / (s.max() - s.min() + 1e-300)
    return lo + (hi - lo) * s


def rel2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_host(t):
    return t.detach().cpu().numpy()
