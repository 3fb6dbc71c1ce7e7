"""Four-body decay workload (time-dependent amplitude fit): model description,
generation point, phase-space sample and event sample.  The samplers draw
from distributions directly and never evaluate the fitted rate.

Final state K+ K- pi+ pi- from a D0 (masses 1.865; 0.494, 0.494, 0.140,
0.140), pairs (12) = K K and (34) = pi pi.  Phase-space density in
(m12, m34) is proportional to p(M; m12, m34) q(m12; m1, m2) q(m34; m3, m4)
(two-body momenta), angles are uniform.
"""
from __future__ import annotations

import math

import numpy as np

from .philox import key_from_seed, uniforms_at

TD4_MASSES = (1.865, 0.494, 0.494, 0.140, 0.140)
TD4_TAU = 0.41            # ps
TD4_SIGMA_T = 0.05        # ps
TD4_X, TD4_Y = 0.004, 0.006

# (L, m0, Gamma0); m0 = 0 marks a non-resonant (flat) entry
TD4_R12 = ((0, 0.0, 0.0), (1, 1.019461, 0.004249), (0, 1.370, 0.350))       # NR, phi(1020), f0(1370)
TD4_R34 = ((0, 0.0, 0.0), (1, 0.77526, 0.1491), (0, 0.990, 0.070))          # NR, rho(770), f0(980)
# (r12 index, r34 index, angular type)
TD4_AMPS = ((0, 0, 0), (0, 2, 0), (0, 1, 1), (2, 1, 1), (1, 0, 2),
            (1, 2, 2), (1, 1, 3), (1, 1, 4), (1, 1, 5), (2, 2, 0))
# coefficients of Abar (cbar) and A (c); the first of each is the reference
TD4_CBAR = ((1.0, 0.0), (0.35, -0.20), (0.80, 0.45), (-0.30, 0.55), (1.60, -0.40),
            (0.45, 0.30), (1.10, 0.25), (0.60, -0.70), (-0.50, 0.65), (0.25, 0.15))
TD4_C = ((0.25, 0.0), (0.05, 0.09), (-0.12, 0.20), (0.10, -0.04), (0.30, 0.22),
         (-0.08, 0.11), (0.21, -0.17), (-0.14, -0.10), (0.09, 0.16), (0.04, -0.06))


# The twenty-amplitude model: four entries per pair and every spin-compatible
# (r12, r34, angular type) combination once (S x S: type 0; S x V: 1; V x S: 2;
# V x V: 3, 4, 5), ten of them in Abar (Cabibbo-favoured, D0bar-like) and the
# other ten in A (doubly Cabibbo-suppressed), so A and Abar share no basis
# function.  Lineshapes are Breit-Wigners of the named resonances.
TD4S_R12 = ((0, 0.0, 0.0), (1, 1.019461, 0.004249), (0, 1.370, 0.350), (0, 1.505, 0.109))
#           NR              phi(1020)                 f0(1370)           f0(1500)
TD4S_R34 = ((0, 0.0, 0.0), (1, 0.77526, 0.1491), (0, 0.990, 0.070), (1, 0.78266, 0.00868))
#           NR              rho(770)              f0(980)            omega(782)
TD4S_ABAR = ((1, 1, 3), (1, 1, 4), (1, 1, 5), (1, 0, 2), (1, 2, 2),
             (0, 1, 1), (2, 1, 1), (0, 0, 0), (0, 2, 0), (2, 2, 0))
TD4S_A = ((1, 3, 3), (1, 3, 4), (1, 3, 5), (0, 3, 1), (2, 3, 1),
          (3, 1, 1), (3, 3, 1), (2, 0, 0), (3, 0, 0), (3, 2, 0))
TD4S_CBAR = ((1.0, 0.0), (0.55, -0.35), (-0.40, 0.60), (1.30, 0.25), (0.35, -0.45),
             (0.70, 0.40), (-0.25, 0.50), (0.60, -0.20), (0.45, 0.35), (-0.30, -0.25))
TD4S_C = ((0.20, 0.0), (0.06, 0.08), (-0.05, 0.09), (0.12, -0.07), (0.04, 0.10),
          (0.09, -0.11), (-0.07, 0.05), (0.10, 0.03), (-0.04, -0.08), (0.06, 0.05))


def td4_split_desc(sigma_t: float = TD4_SIGMA_T, r12=TD4S_R12, r34=TD4S_R34, chunk: int | None = None) -> dict:
    """The twenty-amplitude model: Abar's ten basis functions first, then A's."""
    d = td4_desc(sigma_t=sigma_t, r12=r12, r34=r34, chunk=chunk)
    d["amps"] = [list(a) + ["Abar"] for a in TD4S_ABAR] + [list(a) + ["A"] for a in TD4S_A]
    return d


def td4_split_truth() -> np.ndarray:
    """theta of the twenty-amplitude model: A's coefficients, Abar's, x, y."""
    th = []
    for c in TD4S_C:
        th += [c[0], c[1]]
    for c in TD4S_CBAR:
        th += [c[0], c[1]]
    th += [TD4_X, TD4_Y]
    return np.array(th, dtype=np.float64)


def td4_desc(sigma_t: float = TD4_SIGMA_T, r12=TD4_R12, r34=TD4_R34, chunk: int | None = None) -> dict:
    M, m1, m2, m3, m4 = TD4_MASSES
    d = {"kind": "td4", "M": M, "m": [m1, m2, m3, m4], "r_res": 1.5, "tau": TD4_TAU, "sigma_t": sigma_t,
         "r12": [{"L": L, "m0": m0, "w0": w0} for (L, m0, w0) in r12],
         "r34": [{"L": L, "m0": m0, "w0": w0} for (L, m0, w0) in r34],
         "amps": [list(a) for a in TD4_AMPS]}
    if chunk is not None:
        d["chunk"] = int(chunk)
    return d


def td4_truth() -> np.ndarray:
    th = []
    for c in TD4_C:
        th += [c[0], c[1]]
    for c in TD4_CBAR:
        th += [c[0], c[1]]
    th += [TD4_X, TD4_Y]
    return np.array(th, dtype=np.float64)


def _q(m, ma, mb):
    l = (m * m - (ma + mb) ** 2) * (m * m - (ma - mb) ** 2)
    return np.sqrt(np.maximum(l, 0.0)) / (2.0 * m)


def _ps_weight(m12, m34):
    M, m1, m2, m3, m4 = TD4_MASSES
    return _q(M, m12, m34) * _q(m12, m1, m2) * _q(m34, m3, m4)


_PS_MAX = None


def _ps_max():
    global _PS_MAX
    if _PS_MAX is None:
        M, m1, m2, m3, m4 = TD4_MASSES
        a = np.linspace(m1 + m2, M - m3 - m4, 801)
        b = np.linspace(m3 + m4, M - m1 - m2, 801)
        A, B = np.meshgrid(a, b, indexing="ij")
        w = np.where(A + B < M, _ps_weight(A, B), 0.0)
        _PS_MAX = 1.05 * float(w.max())
    return _PS_MAX


def td4_phase_space(n: int, seed: int = 1710088260, fit: int = 0, stream0: int = 100) -> np.ndarray:
    """Unweighted four-body phase-space points, array (5, n):
    m12, m34, cos theta12, cos theta34, phi."""
    M, m1, m2, m3, m4 = TD4_MASSES
    lo12, hi12 = m1 + m2, M - m3 - m4
    lo34, hi34 = m3 + m4, M - m1 - m2
    key = key_from_seed(seed, fit)
    out = np.empty((5, n))
    todo = np.arange(n, dtype=np.uint64)
    wmax = _ps_max()
    a = 0
    while todo.size:
        u1, u2 = uniforms_at(todo, key, stream0 + 3 * a, 2)
        u3, u4 = uniforms_at(todo, key, stream0 + 3 * a + 1, 2)
        u5, u6 = uniforms_at(todo, key, stream0 + 3 * a + 2, 2)
        m12 = lo12 + u1 * (hi12 - lo12)
        m34 = lo34 + u2 * (hi34 - lo34)
        ok = (m12 + m34 < M) & (u3 * wmax < _ps_weight(m12, m34))
        idx = todo[ok].astype(np.int64)
        out[0, idx] = m12[ok]
        out[1, idx] = m34[ok]
        out[2, idx] = 2.0 * u4[ok] - 1.0
        out[3, idx] = 2.0 * u5[ok] - 1.0
        out[4, idx] = (2.0 * u6[ok] - 1.0) * math.pi
        todo = todo[~ok]
        a += 1
    return out


def td4_events(n: int, seed: int = 1710088260, fit: int = 0, band_frac: float = 0.3) -> np.ndarray:
    """Events (6, n): phase-space kinematics with resonance bands (a fraction
    band_frac of events has m12 from a Cauchy of the phi(1020) width and
    another fraction m34 from the rho(770), each truncated to the kinematic
    range), decay time t = exponential(tau) + Gaussian(0, sigma_t)."""
    M, m1, m2, m3, m4 = TD4_MASSES
    ev = np.empty((6, n))
    ev[:5] = td4_phase_space(n, seed, fit, stream0=200)
    key = key_from_seed(seed, fit)
    i = np.arange(n, dtype=np.uint64)
    ua, ub = uniforms_at(i, key, 50, 3)
    uc, ud = uniforms_at(i, key, 51, 3)
    ue, uf = uniforms_at(i, key, 52, 3)
    # phi band in m12
    sel = ua < band_frac
    L, m0, w0 = TD4_R12[1]
    lo, hi = m1 + m2, M - ev[1, sel]
    ta, tb = np.arctan((lo - m0) / (0.5 * w0)), np.arctan((hi - m0) / (0.5 * w0))
    ev[0, sel] = np.clip(m0 + 0.5 * w0 * np.tan(ta + ub[sel] * (tb - ta)), lo, hi - 1e-12)
    # rho band in m34
    sel2 = (uc < band_frac) & ~sel
    L, m0, w0 = TD4_R34[1]
    lo, hi = m3 + m4, M - ev[0, sel2]
    ta, tb = np.arctan((lo - m0) / (0.5 * w0)), np.arctan((hi - m0) / (0.5 * w0))
    ev[1, sel2] = np.clip(m0 + 0.5 * w0 * np.tan(ta + ud[sel2] * (tb - ta)), lo, hi - 1e-12)
    # decay time with resolution
    t_true = -TD4_TAU * np.log1p(-ue)
    r = np.sqrt(-2.0 * np.log1p(-uf))
    ug, _ = uniforms_at(i, key, 53, 3)
    ev[5] = t_true + TD4_SIGMA_T * r * np.cos(2.0 * math.pi * ug)
    return ev
