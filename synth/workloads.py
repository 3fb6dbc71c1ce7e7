"""Model descriptions and generation points of the benchmark workloads, as the
JSON-able dicts the library and the oracle both accept.  Pure data."""
from __future__ import annotations

import numpy as np

from .samplers import CONFIG0_RANGE, CONFIG0_TRUTH, DALITZ_MASSES, DALITZ_RESONANCES


def mix1d_desc(lo: float = CONFIG0_RANGE[0], hi: float = CONFIG0_RANGE[1]) -> dict:
    """Gaussian(mu, sigma) with fraction f plus exponential(tau) on [lo, hi];
    theta = (mu, sigma, tau, f)."""
    return {"kind": "mix1d", "lo": lo, "hi": hi, "n_params": 4,
            "components": [{"type": "gauss", "params": [0, 1]}, {"type": "exp", "params": [2]}],
            "fracs": [3]}


def mix1d_truth() -> np.ndarray:
    return np.array(CONFIG0_TRUTH, dtype=np.float64)


def dalitz_desc(grid=(1024, 1024), free_lineshapes: bool = False, chunk: int | None = None) -> dict:
    """The eight-resonance three-body model; theta = (Re c, Im c) per resonance,
    then (m0, Gamma0) per resonance when the lineshapes are free."""
    M, m1, m2, m3 = DALITZ_MASSES
    d = {"kind": "dalitz3", "M": M, "m": [m1, m2, m3], "r_res": 1.5, "r_D": 5.0, "grid": list(grid),
         "free_lineshapes": bool(free_lineshapes),
         "resonances": [{"pair": p, "L": L, "m0": m0, "w0": w0} for (p, L, m0, w0, _c) in DALITZ_RESONANCES]}
    if chunk is not None:
        d["chunk"] = int(chunk)
    return d


def dalitz_truth(free_lineshapes: bool = False) -> np.ndarray:
    th = []
    for (_p, _L, _m0, _w0, c) in DALITZ_RESONANCES:
        th += [c[0], c[1]]
    if free_lineshapes:
        for (_p, _L, m0, w0, _c) in DALITZ_RESONANCES:
            th += [m0, w0]
    return np.array(th, dtype=np.float64)
