"""Helpers shared by the GPU tests."""
import numpy as np
import torch


def to_dev(a) -> torch.Tensor:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.ndim == 1:
        a = a[None, :]
    return torch.from_numpy(a).to("cuda")


def rel_close(a, b, rtol):
    return abs(a - b) <= rtol * abs(b)


def grad_close(g, ref, rtol):
    """Per component |g - ref| <= rtol * max(|ref|, 1e-3 * max|ref|)."""
    g, ref = np.asarray(g), np.asarray(ref)
    tol = rtol * np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    return bool((np.abs(g - ref) <= tol).all()), np.abs(g - ref) / tol


def say(*a):
    print(*a, flush=True)
