"""Workload of the time-dependent three-body model (a pi+ pi- pi0-like decay
with D0 mixing): description, generation point and synthetic events.  Pure
data and sampling."""
from __future__ import annotations

import math

import numpy as np

from .philox import key_from_seed, uniforms
from .samplers import BASE_SEED, dalitz_events

# daughters 1 = pi0, 2 = pi+, 3 = pi-: s12 = m^2(pi+ pi0), s13 = m^2(pi- pi0)
TDDP_MASSES = (1.86484, 0.1349766, 0.13957, 0.13957)
# (pair, L, m0, Gamma0, (Re c, Im c))
TDDP_RESONANCES = (
    ("12", 1, 0.7753, 0.1491, (1.0, 0.0)),
    ("13", 1, 0.7753, 0.1491, (0.588, 0.010)),
    ("23", 1, 0.7753, 0.1491, (0.714, -0.020)),
    ("12", 1, 1.465, 0.400, (-0.252, 0.189)),
    ("13", 1, 1.465, 0.400, (-0.179, 0.118)),
    ("23", 0, 0.990, 0.070, (0.080, -0.035)),
    ("23", 2, 1.2755, 0.1867, (0.194, -0.110)),
    ("23", 0, 0.500, 0.400, (0.210, 0.150)),
)
# Sixteen resonances, the size of the paper's pi+ pi- pi0 time-dependent
# example: rho(770), rho(1450) and rho(1700) in each of the three pairs, and
# six isoscalar states in pi+ pi- (f0(980), f0(1370), f0(1500), f0(1710),
# f2(1270), f0(500)) plus f2'(1525).
TDDP_RESONANCES16 = (
    ("12", 1, 0.7753, 0.1491, (1.0, 0.0)),
    ("13", 1, 0.7753, 0.1491, (0.588, 0.010)),
    ("23", 1, 0.7753, 0.1491, (0.714, -0.020)),
    ("12", 1, 1.465, 0.400, (-0.252, 0.189)),
    ("13", 1, 1.465, 0.400, (-0.179, 0.118)),
    ("23", 1, 1.465, 0.400, (0.213, -0.156)),
    ("12", 1, 1.720, 0.250, (0.310, -0.270)),
    ("13", 1, 1.720, 0.250, (0.220, 0.190)),
    ("23", 1, 1.720, 0.250, (-0.140, 0.330)),
    ("23", 0, 0.990, 0.070, (0.080, -0.035)),
    ("23", 0, 1.370, 0.350, (0.160, 0.120)),
    ("23", 0, 1.505, 0.109, (-0.090, 0.070)),
    ("23", 0, 1.720, 0.135, (0.050, -0.040)),
    ("23", 2, 1.2755, 0.1867, (0.194, -0.110)),
    ("23", 0, 0.500, 0.400, (0.210, 0.150)),
    ("23", 2, 1.525, 0.073, (0.060, 0.045)),
)
TDDP_TAU = 0.4101
TDDP_SIGMA_T = 0.1
TDDP_X, TDDP_Y = 0.0039, 0.0065


def tddp3_desc(grid=(1024, 1024), tau: float = TDDP_TAU, sigma_t: float = TDDP_SIGMA_T,
               resonances=TDDP_RESONANCES) -> dict:
    M, m1, m2, m3 = TDDP_MASSES
    return {"kind": "tddp3", "M": M, "m": [m1, m2, m3], "r_res": 1.5, "r_D": 5.0, "grid": list(grid),
            "tau": tau, "sigma_t": sigma_t,
            "resonances": [{"pair": p, "L": L, "m0": m0, "w0": w0} for (p, L, m0, w0, _c) in resonances]}


def tddp3_desc16(grid=(1024, 1024), tau: float = TDDP_TAU, sigma_t: float = TDDP_SIGMA_T) -> dict:
    """The sixteen-resonance model."""
    return tddp3_desc(grid, tau, sigma_t, TDDP_RESONANCES16)


def tddp3_truth(x: float = TDDP_X, y: float = TDDP_Y, resonances=TDDP_RESONANCES) -> np.ndarray:
    """theta = (c, cbar, x, y) with cbar = c."""
    c = [v for (_p, _L, _m0, _w0, cc) in resonances for v in cc]
    return np.array(c + c + [x, y], dtype=np.float64)


def tddp3_truth16(x: float = TDDP_X, y: float = TDDP_Y) -> np.ndarray:
    return tddp3_truth(x, y, TDDP_RESONANCES16)


def tddp3_events(n: int, seed: int = BASE_SEED, tau: float = TDDP_TAU, sigma_t: float = TDDP_SIGMA_T,
                 resonances=TDDP_RESONANCES) -> np.ndarray:
    """Events (3, n): Dalitz points from the three-body band sampler with the
    given masses and resonances, t = exponential(tau) + Gaussian(0, sigma_t)."""
    d = dalitz_events(n, seed=seed, masses=TDDP_MASSES, resonances=resonances)
    u, v = uniforms(n, key_from_seed(seed, 9), 0)
    w, _ = uniforms(n, key_from_seed(seed, 9), 1)
    t = -tau * np.log1p(-u) + sigma_t * np.sqrt(-2.0 * np.log1p(-v)) * np.cos(2.0 * math.pi * w)
    return np.vstack([d, t[None, :]])
