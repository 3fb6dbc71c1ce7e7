"""Shared oracle helpers: exact sums, the NLL assembly, finite differences.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import math

import numpy as np
import torch

DT = torch.float64


def as_t(a, requires_grad: bool = False) -> torch.Tensor:
    t = torch.as_tensor(np.asarray(a, dtype=np.float64)).clone()
    if requires_grad:
        t.requires_grad_(True)
    return t


def fsum(t) -> float:
    """Exactly rounded sum of a float64 tensor/array (Shewchuk via math.fsum)."""
    if isinstance(t, torch.Tensor):
        t = t.detach().cpu().numpy()
    return math.fsum(np.asarray(t, dtype=np.float64).ravel().tolist())


def nll_value(log_p: torch.Tensor, n_events: int, log_norm: float) -> float:
    """NLL = -sum_i ln P~_i + N ln I, the sum taken exactly rounded.

    This is the unbinned negative log-likelihood of unweighted events with
    density P~/I; the paper's fitting loop minimises it (Sec. 1 and 4: the
    objective handed to Minuit).
    """
    return -fsum(log_p) + n_events * log_norm


def central_fd(f, theta, rel_step: float = 1e-6, idx=None) -> np.ndarray:
    """Central finite-difference gradient of a scalar function of theta.

    Step h_i = rel_step * max(|theta_i|, 1).
    """
    theta = np.asarray(theta, dtype=np.float64)
    idx = range(theta.size) if idx is None else idx
    g = np.zeros(theta.size)
    for i in idx:
        h = rel_step * max(abs(theta[i]), 1.0)
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        g[i] = (f(tp) - f(tm)) / ((tp[i] - theta[i]) + (theta[i] - tm[i]))
    return g
