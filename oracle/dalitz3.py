"""Oracle for the three-body Dalitz-plot amplitude model (the paper's amplitude
analyses of three-body decays, Sec. 1 and 5: a coherent sum of complex
resonance amplitudes whose magnitude squared is the density).

The paper gives no formulas; this module takes the standard isobar reading:

Kinematics.  Parent mass M, daughters m1, m2, m3; observables s12, s13 and
s23 = M^2 + m1^2 + m2^2 + m3^2 - s12 - s13.  A resonance sits in a pair AB
with bachelor C: pair "12" is (A, B, C) = (1, 2, 3), "13" is (1, 3, 2),
"23" is (2, 3, 1).  lambda(a, b, c) = a^2 + b^2 + c^2 - 2ab - 2ac - 2bc;
q = sqrt(lambda(s_AB, mA^2, mB^2)) / (2 sqrt(s_AB)) is the daughter momentum
and p = sqrt(lambda(M^2, s_AB, mC^2)) / (2 sqrt(s_AB)) the bachelor momentum,
both in the AB rest frame; q0 is q at s_AB = m0^2.  Negative lambda (only
possible by rounding at the edge of phase space) is read as 0.

Lineshape.  Blatt-Weisskopf factors with z = (q r)^2: F0 = 1,
F1 = 1/sqrt(1 + z), F2 = 1/sqrt(z^2 + 3z + 9).  Mass-dependent width
Gamma(s) = Gamma0 (q/q0)^(2L+1) (m0/sqrt(s)) [F_L(q r)/F_L(q0 r)]^2 and
T = 1 / (m0^2 - s - i m0 Gamma(s)).

Spin factors (Zemach, Lorentz-invariant form):
Z0 = 1; Z1 = s_AC - s_BC + (M^2 - mC^2)(mB^2 - mA^2)/s_AB;
Z2 = Z1^2 - X Y / 3 with X = lambda(s_AB, M^2, mC^2)/s_AB and
Y = lambda(s_AB, mA^2, mB^2)/s_AB.

Amplitude A_k = [F_L(q r_R)/F_L(q0 r_R)] F_L(p r_D) Z_L T and density
P~ = |sum_k c_k A_k|^2 with complex coefficients c_k.

Normalization I: midpoint rule on an nx x ny grid over the bounding box
[(m1+m2)^2, (M-m3)^2] x [(m1+m3)^2, (M-m2)^2]; a cell counts iff its centre
lies in the physical region, s23 in [s23-(s12), s23+(s12)] from the energies
of particles 2 and 3 in the (12) rest frame.  I = dA * sum_inside P~(centre).

Parameter vector: (Re c_k, Im c_k) for k = 0..K-1, then, when the model says
"free_lineshapes", (m0_k, Gamma0_k) for k = 0..K-1.

Pins (tests/test_oracle_dalitz3.py): q, p, Z1 and Z2 against explicit
four-vectors boosted into the pair rest frame; |T(m0^2)| = 1/(m0 Gamma0);
the narrow-width limit of the lineshape integral, pi/(m0 Gamma0); the grid
region area against 1-D quadrature of the s23 limits; the grid I against 2-D
adaptive quadrature; invariance of the NLL under a complex rescaling of all
coefficients (and the two gradient identities it implies); invariance under
relabelling daughters 2 and 3; autograd against central differences.

Toy generation (`generate`, the paper's Monte Carlo generation for toy
studies, Sec. 5): accept-reject on the kinematic box with counter-based
uniforms per event and attempt.  Pins: sample moments against quadrature of
P~, every event in the region, the per-event (prefix) property, a too-low
envelope reported.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .common import as_t, fsum, nll_value

_PAIRS = {"12": (1, 2, 3), "13": (1, 3, 2), "23": (2, 3, 1)}


class Dalitz:
    def __init__(self, desc: dict):
        if desc.get("kind") != "dalitz3":
            raise ValueError("not a dalitz3 model")
        self.M = float(desc["M"])
        self.m = {i + 1: float(v) for i, v in enumerate(desc["m"])}
        self.r_res = float(desc.get("r_res", 1.5))
        self.r_D = float(desc.get("r_D", 5.0))
        self.grid = tuple(int(g) for g in desc.get("grid", (1024, 1024)))
        self.free_ls = bool(desc.get("free_lineshapes", False))
        self.res = []
        for r in desc["resonances"]:
            if r["pair"] not in _PAIRS or int(r["L"]) not in (0, 1, 2):
                raise ValueError(f"bad resonance {r}")
            self.res.append((r["pair"], int(r["L"]), float(r["m0"]), float(r["w0"])))
        self.K = len(self.res)
        self.n_params = 4 * self.K if self.free_ls else 2 * self.K

    # -- kinematics ------------------------------------------------------
    @staticmethod
    def lam(a, b, c):
        return a * a + b * b + c * c - 2.0 * a * b - 2.0 * a * c - 2.0 * b * c

    def s23(self, s12, s13):
        M, m = self.M, self.m
        return M * M + m[1] ** 2 + m[2] ** 2 + m[3] ** 2 - s12 - s13

    def pair_invariants(self, pair, s12, s13):
        """(s_AB, s_AC, s_BC) for a pair."""
        s23 = self.s23(s12, s13)
        if pair == "12":
            return s12, s13, s23
        if pair == "13":
            return s13, s12, s23
        return s23, s12, s13  # pair 23: A=2, B=3, C=1

    @staticmethod
    def blatt_weisskopf(L, z):
        if L == 0:
            return torch.ones_like(z) if isinstance(z, torch.Tensor) else 1.0
        if L == 1:
            return 1.0 / torch.sqrt(1.0 + z) if isinstance(z, torch.Tensor) else 1.0 / math.sqrt(1.0 + z)
        return (1.0 / torch.sqrt(z * z + 3.0 * z + 9.0) if isinstance(z, torch.Tensor)
                else 1.0 / math.sqrt(z * z + 3.0 * z + 9.0))

    def momenta(self, pair, s_ab):
        """(q, p) in the AB rest frame."""
        ia, ib, ic = _PAIRS[pair]
        ma, mb, mc = self.m[ia], self.m[ib], self.m[ic]
        rs = torch.sqrt(s_ab)
        q = torch.sqrt(torch.clamp(self.lam(s_ab, ma * ma, mb * mb), min=0.0)) / (2.0 * rs)
        p = torch.sqrt(torch.clamp(self.lam(self.M ** 2 + 0.0 * s_ab, s_ab, mc * mc), min=0.0)) / (2.0 * rs)
        return q, p

    def q0(self, pair, m0):
        ia, ib, _ = _PAIRS[pair]
        ma, mb = self.m[ia], self.m[ib]
        return torch.sqrt(self.lam(m0 * m0, ma * ma, mb * mb)) / (2.0 * m0)

    def zemach(self, pair, L, s12, s13):
        ia, ib, ic = _PAIRS[pair]
        ma, mb, mc = self.m[ia], self.m[ib], self.m[ic]
        M = self.M
        s_ab, s_ac, s_bc = self.pair_invariants(pair, s12, s13)
        if L == 0:
            return torch.ones_like(s_ab)
        z1 = s_ac - s_bc + (M * M - mc * mc) * (mb * mb - ma * ma) / s_ab
        if L == 1:
            return z1
        x = self.lam(s_ab, M * M + 0.0 * s_ab, mc * mc) / s_ab
        y = self.lam(s_ab, ma * ma + 0.0 * s_ab, mb * mb) / s_ab
        return z1 * z1 - x * y / 3.0

    def lineshape(self, pair, L, m0, w0, s_ab):
        """Relativistic Breit-Wigner T(s) with mass-dependent width."""
        q, _ = self.momenta(pair, s_ab)
        q0 = self.q0(pair, m0)
        r = self.r_res
        fr = self.blatt_weisskopf(L, (q * r) ** 2) / self.blatt_weisskopf(L, (q0 * r) ** 2)
        gam = w0 * (q / q0) ** (2 * L + 1) * (m0 / torch.sqrt(s_ab)) * fr * fr
        return 1.0 / torch.complex(m0 * m0 - s_ab, -m0 * gam)

    def amplitude(self, k, s12, s13, m0, w0):
        pair, L, _, _ = self.res[k]
        s_ab, _, _ = self.pair_invariants(pair, s12, s13)
        q, p = self.momenta(pair, s_ab)
        q0 = self.q0(pair, m0)
        fr = self.blatt_weisskopf(L, (q * self.r_res) ** 2) / self.blatt_weisskopf(L, (q0 * self.r_res) ** 2)
        fd = self.blatt_weisskopf(L, (p * self.r_D) ** 2)
        z = self.zemach(pair, L, s12, s13)
        t = self.lineshape(pair, L, m0, w0, s_ab)
        return (fr * fd * z) * t

    # -- model -----------------------------------------------------------
    def unpack(self, theta):
        cs = [torch.complex(theta[2 * k], theta[2 * k + 1]) for k in range(self.K)]
        if self.free_ls:
            ls = [(theta[2 * self.K + 2 * k], theta[2 * self.K + 2 * k + 1]) for k in range(self.K)]
        else:
            ls = [(torch.tensor(m0, dtype=torch.float64), torch.tensor(w0, dtype=torch.float64))
                  for (_, _, m0, w0) in self.res]
        return cs, ls

    def density_unnorm(self, theta, s12, s13):
        cs, ls = self.unpack(theta)
        tot = torch.zeros(s12.shape, dtype=torch.complex128)
        for k in range(self.K):
            tot = tot + cs[k] * self.amplitude(k, s12, s13, *ls[k])
        return tot.real ** 2 + tot.imag ** 2

    # -- grid ------------------------------------------------------------
    def box(self):
        M, m = self.M, self.m
        return ((m[1] + m[2]) ** 2, (M - m[3]) ** 2), ((m[1] + m[3]) ** 2, (M - m[2]) ** 2)

    def inside(self, s12, s13):
        """Physical-region predicate at (s12, s13), from the (12) rest frame."""
        M, m = self.M, self.m
        rs = np.sqrt(s12)
        e2 = (s12 - m[1] ** 2 + m[2] ** 2) / (2.0 * rs)
        e3 = (M * M - s12 - m[3] ** 2) / (2.0 * rs)
        p2 = np.sqrt(np.maximum(e2 * e2 - m[2] ** 2, 0.0))
        p3 = np.sqrt(np.maximum(e3 * e3 - m[3] ** 2, 0.0))
        lo = (e2 + e3) ** 2 - (p2 + p3) ** 2
        hi = (e2 + e3) ** 2 - (p2 - p3) ** 2
        s23 = M * M + m[1] ** 2 + m[2] ** 2 + m[3] ** 2 - s12 - s13
        return (s23 >= lo) & (s23 <= hi)

    def grid_cells(self):
        """Centres of the inside cells and the cell area dA."""
        (a12, b12), (a13, b13) = self.box()
        nx, ny = self.grid
        d12 = (b12 - a12) / nx
        d13 = (b13 - a13) / ny
        c12 = a12 + (np.arange(nx) + 0.5) * d12
        c13 = a13 + (np.arange(ny) + 0.5) * d13
        g12, g13 = np.meshgrid(c12, c13, indexing="ij")
        ins = self.inside(g12, g13)
        return g12[ins], g13[ins], d12 * d13


def norm_tensor(model: Dalitz, theta: torch.Tensor, cells=None) -> torch.Tensor:
    c12, c13, da = cells if cells is not None else model.grid_cells()
    return da * model.density_unnorm(theta, as_t(c12), as_t(c13)).sum()


def norm_value(model: Dalitz, theta, cells=None) -> float:
    c12, c13, da = cells if cells is not None else model.grid_cells()
    with torch.no_grad():
        v = model.density_unnorm(as_t(theta), as_t(c12), as_t(c13))
    return da * fsum(v)


def nll(theta, ev, desc: dict, cells=None) -> float:
    """NLL = -sum ln P~(s12_i, s13_i) + N ln I, event sum exactly rounded."""
    model = Dalitz(desc)
    ev = np.asarray(ev)
    with torch.no_grad():
        p = model.density_unnorm(as_t(theta), as_t(ev[0]), as_t(ev[1]))
    norm = norm_value(model, theta, cells)
    return nll_value(torch.log(p), ev.shape[1], math.log(norm))


def nll_grad(theta, ev, desc: dict, cells=None):
    """(NLL, gradient by autograd)."""
    model = Dalitz(desc)
    ev = np.asarray(ev)
    th = as_t(theta, requires_grad=True)
    lp = torch.log(model.density_unnorm(th, as_t(ev[0]), as_t(ev[1])))
    nt = norm_tensor(model, th, cells)
    loss = -lp.sum() + ev.shape[1] * torch.log(nt)
    loss.backward()
    value = nll_value(lp.detach(), ev.shape[1], math.log(norm_value(model, theta, cells)))
    return value, th.grad.numpy().copy()


def config1_desc(grid=(1024, 1024), free_lineshapes: bool = False, resonances=None,
                 masses=(1.865, 0.494, 0.140, 0.135)) -> dict:
    """The eight-resonance synthetic Dalitz model (truth table in `truth_theta`)."""
    from_table = resonances if resonances is not None else RESONANCES
    return {"kind": "dalitz3", "M": masses[0], "m": list(masses[1:]),
            "r_res": 1.5, "r_D": 5.0, "grid": list(grid),
            "free_lineshapes": bool(free_lineshapes),
            "resonances": [{"pair": p, "L": L, "m0": m0, "w0": w0} for (p, L, m0, w0, _c) in from_table]}


def truth_theta(desc: dict, resonances=None) -> np.ndarray:
    table = resonances if resonances is not None else RESONANCES
    th = []
    for (_p, _L, _m0, _w0, c) in table:
        th += [c[0], c[1]]
    if desc.get("free_lineshapes"):
        for (_p, _L, m0, w0, _c) in table:
            th += [m0, w0]
    return np.array(th, dtype=np.float64)


# (pair, L, m0, Gamma0, (Re c, Im c)); the first coefficient is the reference
RESONANCES = (
    ("23", 1, 0.770, 0.150, (1.0, 0.0)),
    ("12", 1, 0.892, 0.050, (-0.4662, 0.1697)),
    ("13", 1, 0.892, 0.050, (0.3778, -0.1375)),
    ("12", 0, 1.430, 0.270, (0.0796, 0.1378)),
    ("13", 0, 1.430, 0.270, (-0.0651, -0.1127)),
    ("12", 2, 1.430, 0.100, (0.8751, 0.5052)),
    ("23", 1, 1.700, 0.250, (-0.2214, 1.2557)),
    ("13", 1, 1.900, 0.300, (0.4792, -0.8300)),
)


GEN_ENVELOPE_FACTOR = 1.2  # automatic envelope: this factor x the grid maximum
GEN_MAX_ATTEMPTS = 4096    # attempts per event before it is left unresolved (NaN)


def envelope(theta, desc: dict, cells=None) -> float:
    """Automatic accept-reject envelope: 1.2 x the largest P~ over the centres
    of the integration-grid cells inside the region."""
    model = Dalitz(desc)
    c12, c13, _ = cells if cells is not None else model.grid_cells()
    with torch.no_grad():
        return GEN_ENVELOPE_FACTOR * float(model.density_unnorm(as_t(theta), as_t(c12), as_t(c13)).max())


def generate(theta, desc: dict, n: int, seed: int, fit: int = 0, W: float | None = None):
    """Toy events (2, n) distributed as P~ by accept-reject, event by event.

    Event i, attempt a takes (u1, u2) from Philox counter (i, 2a, word 1) and
    u3 from (i, 2a + 1, word 1) under key (seed, fit).  The candidate
    s12 = lo12 + u1 (hi12 - lo12), s13 = lo13 + u2 (hi13 - lo13) on the
    kinematic box (bounds as products, (m1 + m2)(m1 + m2) and so on) is kept
    when it lies in the region and u3 W < P~; an event not kept within
    GEN_MAX_ATTEMPTS attempts stays NaN.  W defaults to `envelope`.
    Returns (events, W, number of kept events whose P~ exceeds W)."""
    from synth.philox import key_from_seed, uniforms_at
    model = Dalitz(desc)
    M, m = model.M, model.m
    lo12, hi12 = (m[1] + m[2]) * (m[1] + m[2]), (M - m[3]) * (M - m[3])
    lo13, hi13 = (m[1] + m[3]) * (m[1] + m[3]), (M - m[2]) * (M - m[2])
    if W is None:
        W = envelope(theta, desc)
    key = key_from_seed(seed, fit)
    out = np.full((2, n), np.nan)
    todo = np.arange(n, dtype=np.uint64)
    above = 0
    th = as_t(theta)
    for a in range(GEN_MAX_ATTEMPTS):
        if todo.size == 0:
            break
        u1, u2 = uniforms_at(todo, key, 2 * a, 1)
        u3, _ = uniforms_at(todo, key, 2 * a + 1, 1)
        s12 = lo12 + u1 * (hi12 - lo12)
        s13 = lo13 + u2 * (hi13 - lo13)
        ins = model.inside(s12, s13)
        keep = np.zeros(todo.size, dtype=bool)
        if ins.any():
            with torch.no_grad():
                pv = model.density_unnorm(th, as_t(s12[ins]), as_t(s13[ins])).numpy()
            k = u3[ins] * W < pv
            keep[np.flatnonzero(ins)[k]] = True
            above += int((pv[k] > W).sum())
        idx = todo[keep].astype(np.int64)
        out[0, idx] = s12[keep]
        out[1, idx] = s13[keep]
        todo = todo[~keep]
    return out, W, above
