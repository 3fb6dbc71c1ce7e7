"""Oracle for the time-dependent three-body Dalitz-plot model (the paper's
pi+ pi- pi0 time-dependent amplitude fit with mixing, Sec. 1 Table 2 and
Fig. 2; the paper gives no formulas, so everything here is a reading).

Final state D0 -> h1 h2 h3 whose daughters 2 and 3 are each other's charge
conjugates (m2 = m3): the CP-conjugate decay Dbar0 -> h1 h3 h2 reaches the
point (s12, s13) where D0 reaches (s13, s12).  Observables (s12, s13, t).

Amplitudes.  A_k is the three-body isobar amplitude of oracle.dalitz3
(relativistic Breit-Wigner with mass-dependent width, Blatt-Weisskopf
barriers, Zemach spin factors; fixed masses and widths), and
  A(s12, s13) = sum_k c_k A_k(s12, s13),
  Abar(s12, s13) = sum_k cbar_k A_k(s13, s12),
two coefficient sets (cbar = c is CP conservation in the decay).

Time dependence and resolution are those of oracle.td4 (q/p = 1,
Gamma = 1/tau, mixing parameters x, y, Gaussian resolution sigma_t through
h(a; t)):
  R = 1/2 [(|A|^2 + |Abar|^2) Hc + (|A|^2 - |Abar|^2) Hcos
           - 2 Re(conj(A) Abar) Hs - 2 Im(conj(A) Abar) Hsin]
with Hc, Hs = (h(G(1-y)) +- h(G(1+y)))/2 and Hcos + i Hsin = h(G(1 - i x)).

Normalization: the t integral over the real line (1/(G(1-y^2)) etc., as in
oracle.td4) times the Dalitz-plot integral by the midpoint rule on the
model's grid (cells counted when their centre lies inside the region, as in
oracle.dalitz3):
  I = dA sum_cells 1/2 [(|A|^2+|Abar|^2) cy + (|A|^2-|Abar|^2) cx
                        - 2 Re(conj(A) Abar) y cy - 2 Im(conj(A) Abar) x cx],
  cy = 1/(G(1-y^2)), cx = 1/(G(1+x^2)).

theta = (Re c_k, Im c_k)_k, (Re cbar_k, Im cbar_k)_k, x, y.

Pins (tests/test_oracle_tddp3.py): at x = y = 0 the model factorizes into
the three-body density times the resolved exponential, so the NLL equals the
oracle.dalitz3 NLL of the coefficients c minus sum_i ln h(G; t_i) plus N ln
tau; the integral over t of the convolved rate equals the t-integrated rate
at points with x, y and both amplitudes nonzero (signs of the mixing terms);
with m2 = m3 the Dbar0 amplitude of a resonance in one pair equals the
three-body amplitude of the same resonance in the mirrored pair (12 <-> 13,
23 itself); autograd against central differences.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .common import as_t, fsum, nll_value
from .dalitz3 import Dalitz
from .td4 import h_conv


class TDDP:
    def __init__(self, desc: dict):
        if desc.get("kind") != "tddp3":
            raise ValueError("not a tddp3 model")
        if float(desc["m"][1]) != float(desc["m"][2]):
            raise ValueError("daughters 2 and 3 must be charge conjugates (equal masses)")
        self.dal = Dalitz(dict(desc, kind="dalitz3", free_lineshapes=False))
        self.tau = float(desc["tau"])
        self.sigma = float(desc["sigma_t"])
        self.K = self.dal.K
        self.P = 4 * self.K + 2

    def basis(self, s12, s13):
        """(A_k(s12, s13), A_k(s13, s12)) for every resonance."""
        d = self.dal
        ls = [(torch.tensor(m0, dtype=torch.float64), torch.tensor(w0, dtype=torch.float64))
              for (_, _, m0, w0) in d.res]
        a = [d.amplitude(k, s12, s13, *ls[k]) for k in range(self.K)]
        b = [d.amplitude(k, s13, s12, *ls[k]) for k in range(self.K)]
        return a, b

    def amplitudes(self, theta, s12, s13):
        K = self.K
        a, b = self.basis(s12, s13)
        A = sum(torch.complex(theta[2 * k], theta[2 * k + 1]) * a[k] for k in range(K))
        Ab = sum(torch.complex(theta[2 * K + 2 * k], theta[2 * K + 2 * k + 1]) * b[k] for k in range(K))
        return A, Ab

    def _mix(self, theta):
        return theta[self.P - 2], theta[self.P - 1]

    def rate(self, theta, ev):
        """R convolved with the resolution, per event (s12, s13, t)."""
        A, Ab = self.amplitudes(theta, ev[0], ev[1])
        t = ev[2]
        x, y = self._mix(theta)
        G = 1.0 / self.tau
        hp = h_conv(torch.complex(G * (1.0 - y), 0.0 * y), t, self.sigma).real
        hm = h_conv(torch.complex(G * (1.0 + y), 0.0 * y), t, self.sigma).real
        hc = h_conv(torch.complex(G + 0.0 * x, -G * x), t, self.sigma)
        a2 = A.real ** 2 + A.imag ** 2
        b2 = Ab.real ** 2 + Ab.imag ** 2
        z = A.conj() * Ab
        return 0.5 * ((a2 + b2) * 0.5 * (hp + hm) + (a2 - b2) * hc.real
                      - 2.0 * z.real * 0.5 * (hp - hm) - 2.0 * z.imag * hc.imag)

    def unconvolved_rate(self, theta, s12, s13, t):
        """R before the resolution convolution (t >= 0)."""
        A, Ab = self.amplitudes(theta, s12, s13)
        x, y = self._mix(theta)
        gt = t / self.tau
        a2 = A.real ** 2 + A.imag ** 2
        b2 = Ab.real ** 2 + Ab.imag ** 2
        z = A.conj() * Ab
        return 0.5 * torch.exp(-gt) * ((a2 + b2) * torch.cosh(y * gt) + (a2 - b2) * torch.cos(x * gt)
                                       - 2.0 * z.real * torch.sinh(y * gt) - 2.0 * z.imag * torch.sin(x * gt))

    def integrated_rate(self, theta, s12, s13):
        """The t-integral of R at each Dalitz point."""
        A, Ab = self.amplitudes(theta, s12, s13)
        x, y = self._mix(theta)
        G = 1.0 / self.tau
        a2 = A.real ** 2 + A.imag ** 2
        b2 = Ab.real ** 2 + Ab.imag ** 2
        z = A.conj() * Ab
        cy = 1.0 / (G * (1.0 - y * y))
        cx = 1.0 / (G * (1.0 + x * x))
        return 0.5 * ((a2 + b2) * cy + (a2 - b2) * cx - 2.0 * z.real * y * cy - 2.0 * z.imag * x * cx)


def norm_tensor(model: TDDP, theta, cells=None) -> torch.Tensor:
    c12, c13, da = cells if cells is not None else model.dal.grid_cells()
    return da * model.integrated_rate(theta, as_t(c12), as_t(c13)).sum()


def norm_value(model: TDDP, theta, cells=None) -> float:
    c12, c13, da = cells if cells is not None else model.dal.grid_cells()
    with torch.no_grad():
        v = model.integrated_rate(as_t(theta), as_t(c12), as_t(c13))
    return da * fsum(v)


def nll(theta, ev, desc: dict, cells=None) -> float:
    """NLL = -sum ln R(s12_i, s13_i, t_i) + N ln I, the event sum exactly rounded."""
    model = TDDP(desc)
    ev = np.asarray(ev)
    with torch.no_grad():
        r = model.rate(as_t(theta), as_t(ev))
    return nll_value(torch.log(r), ev.shape[1], math.log(norm_value(model, theta, cells)))


def nll_grad(theta, ev, desc: dict, cells=None):
    """(NLL, gradient by autograd)."""
    model = TDDP(desc)
    ev = np.asarray(ev)
    th = as_t(theta, requires_grad=True)
    lr = torch.log(model.rate(th, as_t(ev)))
    nt = norm_tensor(model, th, cells)
    loss = -lr.sum() + ev.shape[1] * torch.log(nt)
    loss.backward()
    value = nll_value(lr.detach(), ev.shape[1], math.log(norm_value(model, theta, cells)))
    return value, th.grad.numpy().copy()


# (pair, L, m0, Gamma0, (Re c, Im c)) of a pi+ pi- pi0-like model: daughters
# 1 = pi0, 2 = pi+, 3 = pi-, so s12 = m^2(pi+ pi0) and s13 = m^2(pi- pi0).
RESONANCES = (
    ("12", 1, 0.7753, 0.1491, (1.0, 0.0)),      # rho+
    ("13", 1, 0.7753, 0.1491, (0.588, 0.010)),  # rho-
    ("23", 1, 0.7753, 0.1491, (0.714, -0.020)),  # rho0
    ("12", 1, 1.465, 0.400, (-0.252, 0.189)),   # rho(1450)+
    ("13", 1, 1.465, 0.400, (-0.179, 0.118)),   # rho(1450)-
    ("23", 0, 0.990, 0.070, (0.080, -0.035)),   # f0(980)
    ("23", 2, 1.2755, 0.1867, (0.194, -0.110)),  # f2(1270)
    ("23", 0, 0.500, 0.400, (0.210, 0.150)),    # f0(500)
)
MASSES = (1.86484, 0.1349766, 0.13957, 0.13957)
TAU = 0.4101
SIGMA_T = 0.1
X_MIX, Y_MIX = 0.0039, 0.0065


def pipipi0_desc(grid=(1024, 1024), resonances=None, tau: float = TAU, sigma_t: float = SIGMA_T) -> dict:
    """The eight-resonance time-dependent pi+ pi- pi0-like model."""
    table = resonances if resonances is not None else RESONANCES
    M, m1, m2, m3 = MASSES
    return {"kind": "tddp3", "M": M, "m": [m1, m2, m3], "r_res": 1.5, "r_D": 5.0, "grid": list(grid),
            "tau": tau, "sigma_t": sigma_t,
            "resonances": [{"pair": p, "L": L, "m0": m0, "w0": w0} for (p, L, m0, w0, _c) in table]}


def truth_theta(resonances=None, x: float = X_MIX, y: float = Y_MIX) -> np.ndarray:
    """theta with cbar = c (CP conservation in the decay)."""
    table = resonances if resonances is not None else RESONANCES
    c = [v for (_p, _L, _m0, _w0, cc) in table for v in cc]
    return np.array(c + c + [x, y], dtype=np.float64)


GEN_ENVELOPE_FACTOR = 1.2  # automatic envelope: this factor x the grid maximum of (|A| + |Abar|)^2
GEN_MAX_ATTEMPTS = 4096


def envelope(theta, desc: dict, cells=None) -> float:
    """1.2 x the largest (|A| + |Abar|)^2 over the integration-grid cell centres."""
    model = TDDP(desc)
    c12, c13, _ = cells if cells is not None else model.dal.grid_cells()
    with torch.no_grad():
        A, Ab = model.amplitudes(as_t(theta), as_t(c12), as_t(c13))
        return GEN_ENVELOPE_FACTOR * float(((A.abs() + Ab.abs()) ** 2).max())


def generate(theta, desc: dict, n: int, seed: int, fit: int = 0, W: float | None = None):
    """Toy events (3, n) distributed as the model by accept-reject, event by
    event.  The unconvolved rate obeys R(s12, s13, t) <= e^{-lam t} (|A| + |Abar|)^2
    with lam = G (1 - |y|) (|sinh| <= cosh, |cos|, |sin| <= 1 and cosh >= 1
    bound the bracket by cosh(y G t) (2 max(|A|^2, |Abar|^2) + 4 |A||Abar|), and
    e^{-Gt} cosh(y G t) <= e^{-lam t}), so: event i, attempt a takes
    (u1, u2) from Philox counter (i, 2a, word 2) and (u3, u4) from
    (i, 2a + 1, word 2) under key (seed, fit); s12 = lo12 + u1 (hi12 - lo12),
    s13 = lo13 + u2 (hi13 - lo13) on the kinematic box, t_true = -ln(1 - u3)/lam;
    the candidate is kept when it lies in the region and
    u4 W e^{-lam t_true} < R(s12, s13, t_true).  The measured time adds a
    Gaussian of width sigma_t from counter (i, 0, word 3) (Box-Muller).  An
    event not kept within GEN_MAX_ATTEMPTS attempts stays NaN.
    Returns (events, W, number of kept events whose (|A| + |Abar|)^2 exceeds W)."""
    from synth.philox import key_from_seed, uniforms_at
    model = TDDP(desc)
    d = model.dal
    M, m = d.M, d.m
    lo12, hi12 = (m[1] + m[2]) * (m[1] + m[2]), (M - m[3]) * (M - m[3])
    lo13, hi13 = (m[1] + m[3]) * (m[1] + m[3]), (M - m[2]) * (M - m[2])
    if W is None:
        W = envelope(theta, desc)
    y = float(theta[model.P - 1])
    lam = (1.0 - abs(y)) / model.tau
    key = key_from_seed(seed, fit)
    out = np.full((3, n), np.nan)
    todo = np.arange(n, dtype=np.uint64)
    above = 0
    th = as_t(theta)
    for a in range(GEN_MAX_ATTEMPTS):
        if todo.size == 0:
            break
        u1, u2 = uniforms_at(todo, key, 2 * a, 2)
        u3, u4 = uniforms_at(todo, key, 2 * a + 1, 2)
        s12 = lo12 + u1 * (hi12 - lo12)
        s13 = lo13 + u2 * (hi13 - lo13)
        tt = -np.log1p(-u3) / lam
        ins = d.inside(s12, s13)
        keep = np.zeros(todo.size, dtype=bool)
        if ins.any():
            with torch.no_grad():
                r = model.unconvolved_rate(th, as_t(s12[ins]), as_t(s13[ins]), as_t(tt[ins])).numpy()
                A, Ab = model.amplitudes(th, as_t(s12[ins]), as_t(s13[ins]))
                env = ((A.abs() + Ab.abs()) ** 2).numpy()
            k = u4[ins] * W * np.exp(-lam * tt[ins]) < r
            keep[np.flatnonzero(ins)[k]] = True
            above += int((env[k] > W).sum())
        idx = todo[keep].astype(np.int64)
        out[0, idx] = s12[keep]
        out[1, idx] = s13[keep]
        out[2, idx] = tt[keep]
        todo = todo[~keep]
    i = np.arange(n, dtype=np.uint64)
    v1, v2 = uniforms_at(i, key, 0, 3)
    out[2] = out[2] + model.sigma * np.sqrt(-2.0 * np.log1p(-v1)) * np.cos(2.0 * math.pi * v2)
    return out, W, above
