"""Seeded synthetic event samples shaped like the paper's three workload classes
(a 1-D peak over a smooth background, a three-body Dalitz plot, a four-body
decay with a decay time).  The paper's own BaBar samples are not public in
this form; these stand in for them.

The samplers draw from distributions directly (component choice, Box-Muller,
inverse CDFs, two-body decay kinematics) and never evaluate the fitted
densities or the likelihood: the events are inputs to the method, produced the
same way for the CPU oracle and for the device library.
"""
from __future__ import annotations

import math

import numpy as np

from .philox import key_from_seed, uniforms_at

BASE_SEED = 1710088260

# ---------------------------------------------------------------------------
# 1-D mixture: Gaussian peak + exponential background on [lo, hi]
# ---------------------------------------------------------------------------
CONFIG0_TRUTH = (0.2, 1.1, -0.3, 0.7)  # mu, sigma, tau, frac(gauss)
CONFIG0_RANGE = (-10.0, 10.0)


def mix1d_events(n: int, seed: int = BASE_SEED, fit: int = 0,
                 theta=CONFIG0_TRUTH, lo: float = -10.0, hi: float = 10.0):
    """n events x in [lo, hi] from  f*TruncGauss(mu, sigma) + (1-f)*TruncExp(tau).

    Event i, attempt a uses Philox counters (i, 2a) and (i, 2a+1): the first
    gives (u_component, u_1), the second (u_2, -).  Gaussian draws outside
    [lo, hi] are redrawn with the next attempt; exponential draws use the
    inverse CDF of the truncated exponential and always land inside.
    """
    mu, sigma, tau, frac = (float(t) for t in theta)
    key = key_from_seed(seed, fit)
    out = np.empty(n, dtype=np.float64)
    todo = np.arange(n, dtype=np.uint64)
    width = hi - lo
    attempt = 0
    while todo.size:
        uc, u1 = uniforms_at(todo, key, 2 * attempt, 0)
        u2, _ = uniforms_at(todo, key, 2 * attempt + 1, 0)
        is_g = uc < frac
        r = np.sqrt(-2.0 * np.log1p(-u1))
        xg = mu + sigma * r * np.cos(2.0 * math.pi * u2)
        if tau != 0.0:
            xe = lo + np.log1p(u1 * math.expm1(tau * width)) / tau
        else:
            xe = lo + u1 * width
        xe = np.clip(xe, lo, hi)
        x = np.where(is_g, xg, xe)
        ok = (x >= lo) & (x <= hi)
        out[todo[ok].astype(np.int64)] = x[ok]
        todo = todo[~ok]
        attempt += 1
        if attempt > 1000:
            raise RuntimeError("mix1d_events: range too narrow for the Gaussian")
    return out


def lognormal_sizes(n_fits: int, lo: int = 1000, hi: int = 2_000_000,
                    seed: int = BASE_SEED, stream: int = 7):
    """Per-fit event counts N_k = round(exp(U(ln lo, ln hi)))."""
    u, _ = uniforms_at(np.arange(n_fits, dtype=np.uint64), key_from_seed(seed, 0xFFFF), stream)
    return np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)


# ---------------------------------------------------------------------------
# Three-body decay M -> 1 2 3: phase space plus resonance bands
# ---------------------------------------------------------------------------
DALITZ_MASSES = (1.865, 0.494, 0.140, 0.135)  # parent, m1, m2, m3

# (pair, L, m0, width, (Re c, Im c)) -- the synthetic eight-resonance model
DALITZ_RESONANCES = (
    ("23", 1, 0.770, 0.150, (1.0, 0.0)),
    ("12", 1, 0.892, 0.050, (-0.4662, 0.1697)),
    ("13", 1, 0.892, 0.050, (0.3778, -0.1375)),
    ("12", 0, 1.430, 0.270, (0.0796, 0.1378)),
    ("13", 0, 1.430, 0.270, (-0.0651, -0.1127)),
    ("12", 2, 1.430, 0.100, (0.8751, 0.5052)),
    ("23", 1, 1.700, 0.250, (-0.2214, 1.2557)),
    ("13", 1, 1.900, 0.300, (0.4792, -0.8300)),
)
# mixture weights of the event generator: flat phase space, then one band per
# resonance (roughly the resonances' fit fractions)
_BAND_WEIGHTS = (0.454, 0.151, 0.101, 0.061, 0.040, 0.020, 0.030, 0.020)
_FLAT_WEIGHT = 0.15

_PAIR_IDX = {"12": (1, 2, 3), "13": (1, 3, 2), "23": (2, 3, 1)}


def _two_body(s, ma, mb, mc, M):
    """Energies and momenta of particle A and bachelor C in the AB rest frame."""
    rs = np.sqrt(s)
    ea = (s + ma * ma - mb * mb) / (2.0 * rs)
    ec = (M * M - s - mc * mc) / (2.0 * rs)
    pa = np.sqrt(np.maximum(ea * ea - ma * ma, 0.0))
    pc = np.sqrt(np.maximum(ec * ec - mc * mc, 0.0))
    return ea, ec, pa, pc


def dalitz_box(masses=DALITZ_MASSES):
    """Bounding box [(m1+m2)^2,(M-m3)^2] x [(m1+m3)^2,(M-m2)^2] of (s12, s13)."""
    M, m1, m2, m3 = masses
    return ((m1 + m2) ** 2, (M - m3) ** 2), ((m1 + m3) ** 2, (M - m2) ** 2)


def dalitz_events(n: int, seed: int = BASE_SEED, fit: int = 0,
                  masses=DALITZ_MASSES, resonances=DALITZ_RESONANCES,
                  flat_weight: float = _FLAT_WEIGHT, band_weights=_BAND_WEIGHTS):
    """n events (s12, s13) as an SoA array of shape (2, n).

    Each event picks a mixture component from a uniform draw: flat phase space
    (uniform in the Dalitz region, by rejection from the bounding box), or a
    band of resonance k (mass from a Cauchy of width Gamma_k truncated to the
    kinematic range of its pair, decay angle isotropic in the pair's rest
    frame, which is flat in the other invariant).
    """
    M, m1, m2, m3 = masses
    mass = {1: m1, 2: m2, 3: m3}
    msum = M * M + m1 * m1 + m2 * m2 + m3 * m3
    (a12, b12), (a13, b13) = dalitz_box(masses)
    w = np.array([flat_weight] + list(band_weights), dtype=np.float64)
    cw = np.cumsum(w / w.sum())
    key = key_from_seed(seed, fit)
    s12 = np.empty(n)
    s13 = np.empty(n)
    todo = np.arange(n, dtype=np.uint64)
    attempt = 0
    while todo.size:
        uc, u1 = uniforms_at(todo, key, 2 * attempt, 1)
        u2, _ = uniforms_at(todo, key, 2 * attempt + 1, 1)
        comp = np.searchsorted(cw, uc, side="right")
        comp = np.minimum(comp, len(w) - 1)
        x12 = np.full(todo.size, np.nan)
        x13 = np.full(todo.size, np.nan)
        # flat component: uniform in the box, keep if inside the region
        sel = comp == 0
        if sel.any():
            t12 = a12 + u1[sel] * (b12 - a12)
            t13 = a13 + u2[sel] * (b13 - a13)
            ea, ec, pa, pc = _two_body(t12, m1, m2, m3, M)
            cos = (m1 * m1 + m3 * m3 + 2.0 * ea * ec - t13) / (2.0 * pa * pc)
            inside = np.abs(cos) <= 1.0
            x12[np.flatnonzero(sel)[inside]] = t12[inside]
            x13[np.flatnonzero(sel)[inside]] = t13[inside]
        for k, (pair, _L, m0, gam, _c) in enumerate(resonances):
            sel = comp == k + 1
            if not sel.any():
                continue
            ia, ib, ic = _PAIR_IDX[pair]
            ma, mb, mc = mass[ia], mass[ib], mass[ic]
            mlo, mhi = ma + mb, M - mc
            hw = 0.5 * gam
            ta, tb = math.atan((mlo - m0) / hw), math.atan((mhi - m0) / hw)
            m = m0 + hw * np.tan(ta + u1[sel] * (tb - ta))
            m = np.clip(m, mlo, mhi)
            s = m * m
            ea, ec, pa, pc = _two_body(s, ma, mb, mc, M)
            cos = 2.0 * u2[sel] - 1.0
            s_ac = ma * ma + mc * mc + 2.0 * (ea * ec - pa * pc * cos)
            if pair == "12":
                v12, v13 = s, s_ac
            elif pair == "13":
                v13, v12 = s, s_ac
            else:  # pair 23, A=2, C=1: s_AC = s12
                v12 = s_ac
                v13 = msum - v12 - s
            x12[np.flatnonzero(sel)] = v12
            x13[np.flatnonzero(sel)] = v13
        ok = np.isfinite(x12)
        s12[todo[ok].astype(np.int64)] = x12[ok]
        s13[todo[ok].astype(np.int64)] = x13[ok]
        todo = todo[~ok]
        attempt += 1
        if attempt > 10000:
            raise RuntimeError("dalitz_events: rejection did not terminate")
    return np.stack([s12, s13])
