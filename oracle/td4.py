"""Oracle for the time-dependent four-body amplitude model (the paper's
four-body time-dependent amplitude analyses, Abstract and Sec. 5; the paper
gives no formulas, so everything here is a reading).

Final state D0 -> h1 h2 h3 h4 with pairs (12) and (34); observables
(m12, m34, cos theta12, cos theta34, phi, t): two pair masses, the two
helicity angles, the angle between the decay planes and the decay time.

Amplitudes.  Basis functions B_k = a12[r1_k](m12) a34[r2_k](m34) Omega_k with
  a[r](m) = 1 for a non-resonant entry (m0 = 0), else
  [F_L(q r)/F_L(q0 r)] T(m^2), T = 1/(m0^2 - s - i m0 Gamma(s)) with the
  mass-dependent width of the three-body model (q: daughter momentum in the
  pair frame, Blatt-Weisskopf F_0 = 1, F_1 = (1+z)^-1/2),
  Omega by helicity structure: 0 S x S: 1;  1 S x V: c34;  2 V x S: c12;
  3 V x V (lambda 0): c12 c34;  4 V x V (lambda +1): 1/2 s12 s34 e^{i phi};
  5 V x V (lambda -1): 1/2 s12 s34 e^{-i phi}   (s = sqrt(1 - c^2)).
Every basis function enters the D0 amplitude A, the Dbar0 amplitude Abar, or
both (an optional fourth entry "A", "Abar" or "both" of each amplitude;
"both" when absent): A = sum_{k in A} c_k B_k, Abar = sum_{k in Abar} cbar_k B_k.
With "both" everywhere the two sums share one basis and differ only in their
coefficients; with disjoint sets, A and Abar are built from distinct basis
functions (the doubly Cabibbo-suppressed and the Cabibbo-favoured amplitudes
of a four-body analysis, Sec. 5, read as ten distinct functions each).

Time dependence (q/p = 1, Gamma = 1/tau, mixing x, y):
  R(x, t) = 1/2 e^{-Gamma t} [(|A|^2 + |Abar|^2) cosh(y Gamma t) + (|A|^2 - |Abar|^2) cos(x Gamma t)
            - 2 Re(A* Abar) sinh(y Gamma t) - 2 Im(A* Abar) sin(x Gamma t)]   (t >= 0),
convolved with a Gaussian resolution of width sigma_t: with
  h(a; t) = [e^{-a u} theta(u)] (x) G_sigma (t) = 1/2 exp(a^2 sigma^2/2 - a t) erfc((a sigma^2 - t)/(sigma sqrt2)),
e^{-Gamma t} cosh -> (h(G(1-y)) + h(G(1+y)))/2, sinh -> (h(G(1-y)) - h(G(1+y)))/2,
cos -> Re h(G(1 - i x)), sin -> Im h(G(1 - i x)).  h is evaluated through the
Faddeeva function w (scipy.special.wofz here): with z = (a sigma^2 - t)/(sigma sqrt2),
h = 1/2 e^{-t^2/(2 sigma^2)} w(i z) for Re z >= 0, and
h = e^{a^2 sigma^2/2 - a t} - 1/2 e^{-t^2/(2 sigma^2)} w(-i z) otherwise.

Normalization: the t integral over the real line keeps the unconvolved
integrals 1/(G(1-y^2)), y/(G(1-y^2)), 1/(G(1+x^2)), x/(G(1+x^2)); I is the
average over an unweighted phase-space sample of
  1/2 [(|A|^2+|Abar|^2)/(G(1-y^2)) + (|A|^2-|Abar|^2)/(G(1+x^2))
       - 2 Re(A* Abar) y/(G(1-y^2)) - 2 Im(A* Abar) x/(G(1+x^2))].

theta = (Re c_k, Im c_k) for the members of A in description order, then
(Re cbar_k, Im cbar_k) for the members of Abar in description order, then x, y.

Pins (tests/test_oracle_td4.py): h against direct quadrature of the
convolution (real and complex a, t from -0.3 to 5 ps), the sigma -> 0 limit,
the integral of h over t equal to 1/a, the t-integral of R against the
normalization formula, factorization at x = y = 0, orthogonality of the six
angular functions on the angle space, the pole-mass value of T, and
autograd against central differences.
"""
from __future__ import annotations

import math

import numpy as np
import torch
from scipy.special import wofz

from .common import as_t, fsum, nll_value

SQRT_2PI = math.sqrt(2.0 * math.pi)


class _H(torch.autograd.Function):
    """h(a; t) for a complex scalar a (0-d complex128) and a vector t."""

    @staticmethod
    def forward(ctx, a, t, sigma):
        av = complex(a.detach())
        tv = t.detach().numpy()
        z = (av * sigma * sigma - tv) / (sigma * math.sqrt(2.0))
        g = np.exp(-tv * tv / (2.0 * sigma * sigma))
        h = np.empty(tv.shape, dtype=np.complex128)
        up = z.real >= 0.0
        h[up] = 0.5 * g[up] * wofz(1j * z[up])
        dn = ~up
        h[dn] = np.exp(av * av * sigma * sigma / 2.0 - av * tv[dn]) - 0.5 * g[dn] * wofz(-1j * z[dn])
        ht = torch.from_numpy(h.astype(np.complex128))
        ctx.save_for_backward(ht, t)
        ctx.sigma = sigma
        ctx.a = av
        return ht

    @staticmethod
    def backward(ctx, grad):
        h, t = ctx.saved_tensors
        s = ctx.sigma
        # dh/da = (a s^2 - t) h - s/sqrt(2 pi) exp(-t^2/(2 s^2))
        dh = (ctx.a * s * s - t) * h - (s / SQRT_2PI) * torch.exp(-t * t / (2.0 * s * s))
        ga = (grad * dh.conj()).sum()
        return ga, None, None


def h_conv(a, t, sigma: float):
    if not isinstance(a, torch.Tensor):
        a = torch.tensor(complex(a), dtype=torch.complex128)
    if not torch.is_complex(a):
        a = torch.complex(a, torch.zeros_like(a))
    return _H.apply(a, t, sigma)


class TD4:
    def __init__(self, desc: dict):
        if desc.get("kind") != "td4":
            raise ValueError("not a td4 model")
        self.M = float(desc["M"])
        self.m = [float(v) for v in desc["m"]]
        self.r = float(desc.get("r_res", 1.5))
        self.tau = float(desc["tau"])
        self.sigma = float(desc["sigma_t"])
        self.r12 = [(int(e["L"]), float(e["m0"]), float(e["w0"])) for e in desc["r12"]]
        self.r34 = [(int(e["L"]), float(e["m0"]), float(e["w0"])) for e in desc["r34"]]
        self.amps = [tuple(int(v) for v in a[:3]) for a in desc["amps"]]
        self.K = len(self.amps)
        sides = [a[3] if len(a) > 3 else "both" for a in desc["amps"]]
        if any(sd not in ("both", "A", "Abar") for sd in sides):
            raise ValueError("an amplitude's sum must be \"both\", \"A\" or \"Abar\"")
        self.in_a = [k for k in range(self.K) if sides[k] in ("both", "A")]
        self.in_b = [k for k in range(self.K) if sides[k] in ("both", "Abar")]
        self.P = 2 * len(self.in_a) + 2 * len(self.in_b) + 2

    @staticmethod
    def lam(a, b, c):
        return a * a + b * b + c * c - 2 * a * b - 2 * a * c - 2 * b * c

    @staticmethod
    def bw_factor(L, z):
        return torch.ones_like(z) if L == 0 else 1.0 / torch.sqrt(1.0 + z)

    def pair_amp(self, m, ma, mb, res):
        L, m0, w0 = res
        if m0 == 0.0:
            return torch.ones(m.shape, dtype=torch.complex128)
        s = m * m
        q = torch.sqrt(torch.clamp(self.lam(s, ma * ma, mb * mb), min=0.0)) / (2.0 * m)
        q0 = math.sqrt(self.lam(m0 * m0, ma * ma, mb * mb)) / (2.0 * m0)
        fr = self.bw_factor(L, (q * self.r) ** 2) / self.bw_factor(L, torch.tensor((q0 * self.r) ** 2, dtype=torch.float64))
        gam = w0 * (q / q0) ** (2 * L + 1) * (m0 / m) * fr * fr
        t = 1.0 / torch.complex(m0 * m0 - s, -m0 * gam)
        return fr * t

    @staticmethod
    def omega(typ, c12, c34, phi):
        one = torch.ones(c12.shape, dtype=torch.complex128)
        if typ == 0:
            return one
        if typ == 1:
            return c34 * one
        if typ == 2:
            return c12 * one
        if typ == 3:
            return c12 * c34 * one
        s = 0.5 * torch.sqrt(1.0 - c12 * c12) * torch.sqrt(1.0 - c34 * c34)
        if typ == 4:
            return torch.polar(s, phi)
        if typ == 5:
            return torch.polar(s, -phi)
        raise ValueError(typ)

    def basis(self, kin):
        """B_k for kinematics kin = (m12, m34, c12, c34, phi) tensors."""
        m12, m34, c12, c34, phi = kin
        m1, m2, m3, m4 = self.m
        a12 = [self.pair_amp(m12, m1, m2, r) for r in self.r12]
        a34 = [self.pair_amp(m34, m3, m4, r) for r in self.r34]
        return [a12[i] * a34[j] * self.omega(typ, c12, c34, phi) for (i, j, typ) in self.amps]

    def amplitudes(self, theta, B):
        off = 2 * len(self.in_a)
        A = torch.zeros_like(B[0])
        for j, k in enumerate(self.in_a):
            A = A + torch.complex(theta[2 * j], theta[2 * j + 1]) * B[k]
        Ab = torch.zeros_like(B[0])
        for j, k in enumerate(self.in_b):
            Ab = Ab + torch.complex(theta[off + 2 * j], theta[off + 2 * j + 1]) * B[k]
        return A, Ab

    def rate(self, theta, ev):
        """R(x, t) convolved with the resolution, per event."""
        B = self.basis(ev[:5])
        A, Ab = self.amplitudes(theta, B)
        t = ev[5]
        x, y = theta[self.P - 2], theta[self.P - 1]
        G = 1.0 / self.tau
        one = torch.ones((), dtype=torch.float64)
        hp = h_conv(torch.complex(G * (1.0 - y), 0.0 * y), t, self.sigma).real
        hm = h_conv(torch.complex(G * (1.0 + y), 0.0 * y), t, self.sigma).real
        hc = h_conv(torch.complex(G * one, -G * x), t, self.sigma)
        a2 = A.real ** 2 + A.imag ** 2
        b2 = Ab.real ** 2 + Ab.imag ** 2
        z = A.conj() * Ab
        return 0.5 * ((a2 + b2) * 0.5 * (hp + hm) + (a2 - b2) * hc.real
                      - 2.0 * z.real * 0.5 * (hp - hm) - 2.0 * z.imag * hc.imag)

    def integrated_rate(self, theta, kin):
        """The t-integral of R at each phase-space point."""
        B = self.basis(kin)
        A, Ab = self.amplitudes(theta, B)
        x, y = theta[self.P - 2], theta[self.P - 1]
        G = 1.0 / self.tau
        a2 = A.real ** 2 + A.imag ** 2
        b2 = Ab.real ** 2 + Ab.imag ** 2
        z = A.conj() * Ab
        cy = 1.0 / (G * (1.0 - y * y))
        cx = 1.0 / (G * (1.0 + x * x))
        return 0.5 * ((a2 + b2) * cy + (a2 - b2) * cx - 2.0 * z.real * y * cy - 2.0 * z.imag * x * cx)


def nll(theta, ev, mc, desc) -> float:
    model = TD4(desc)
    with torch.no_grad():
        th = as_t(theta)
        r = model.rate(th, as_t(ev))
        norm = fsum(model.integrated_rate(th, as_t(mc))) / mc.shape[1]
    return nll_value(torch.log(r), ev.shape[1], math.log(norm))


def nll_grad(theta, ev, mc, desc):
    model = TD4(desc)
    th = as_t(theta, requires_grad=True)
    lr = torch.log(model.rate(th, as_t(ev)))
    ir = model.integrated_rate(th, as_t(mc))
    loss = -lr.sum() + ev.shape[1] * torch.log(ir.mean())
    loss.backward()
    with torch.no_grad():
        norm = fsum(ir.detach()) / mc.shape[1]
    return nll_value(lr.detach(), ev.shape[1], math.log(norm)), th.grad.numpy().copy()


def unconvolved_rate(model: TD4, theta, kin, t):
    """R(x, t) before the resolution convolution (t >= 0)."""
    B = model.basis(kin)
    A, Ab = model.amplitudes(theta, B)
    x, y = theta[model.P - 2], theta[model.P - 1]
    G = 1.0 / model.tau
    a2 = A.real ** 2 + A.imag ** 2
    b2 = Ab.real ** 2 + Ab.imag ** 2
    z = A.conj() * Ab
    gt = G * t
    return 0.5 * torch.exp(-gt) * ((a2 + b2) * torch.cosh(y * gt) + (a2 - b2) * torch.cos(x * gt)
                                   - 2.0 * z.real * torch.sinh(y * gt) - 2.0 * z.imag * torch.sin(x * gt))


def generate(theta, desc, n: int, seed: int = 1710088260, fit: int = 0, batch: int = 200_000):
    """Events (6, n) distributed as the model at theta, by accept-reject.

    Proposal: an unweighted phase-space point times t_true ~ Exp(G(1 - |y|));
    since e^{-Gt}cosh(yGt) <= e^{-G(1-|y|)t} and every interference term is
    bounded by |A||Abar|, R(x, t) <= e^{-G(1-|y|)t} (|A| + |Abar|)^2, so a
    candidate is kept with probability R / (e^{-G(1-|y|)t} W), W an upper
    bound of (|A| + |Abar|)^2 over phase space (1.5 x the largest value on a
    large phase-space sample; a candidate above W raises an error).  The
    measured time is t_true plus a Gaussian of width sigma_t (Box-Muller)."""
    from synth import td4_phase_space
    from synth.philox import key_from_seed, uniforms_at
    model = TD4(desc)
    th = as_t(theta)
    G = 1.0 / model.tau
    y = float(theta[model.P - 1])
    lam = G * (1.0 - abs(y))
    with torch.no_grad():
        ps = torch.from_numpy(td4_phase_space(batch, seed, fit, stream0=5000))
        A, Ab = model.amplitudes(th, model.basis(ps))
        W = 1.5 * float(((A.abs() + Ab.abs()) ** 2).max())
    key = key_from_seed(seed, fit)
    out = np.empty((6, n))
    got = 0
    rnd = 0
    while got < n:
        kin = td4_phase_space(batch, seed, fit, stream0=10_000 + 1000 * rnd)  # 3 streams per attempt
        i = np.arange(batch, dtype=np.uint64)
        u1, u2 = uniforms_at(i, key, 3000 + 2 * rnd, 0)
        u3, u4 = uniforms_at(i, key, 3001 + 2 * rnd, 0)
        tt = -np.log1p(-u1) / lam
        with torch.no_grad():
            kt = torch.from_numpy(kin)
            r = unconvolved_rate(model, th, kt, torch.from_numpy(tt)).numpy()
            A, Ab = model.amplitudes(th, model.basis(kt))
            env = ((A.abs() + Ab.abs()) ** 2).numpy()
        if (env > W).any():
            raise RuntimeError("amplitude bound exceeded; raise the safety factor")
        keep = u2 * W * np.exp(-lam * tt) < r
        idx = np.nonzero(keep)[0][: n - got]
        out[:5, got:got + idx.size] = kin[:, idx]
        gauss = np.sqrt(-2.0 * np.log1p(-u3[idx])) * np.cos(2.0 * math.pi * u4[idx])
        out[5, got:got + idx.size] = tt[idx] + model.sigma * gauss
        got += idx.size
        rnd += 1
    return out


def _q(m, ma, mb):
    l = (m * m - (ma + mb) * (ma + mb)) * (m * m - (ma - mb) * (ma - mb))
    return np.sqrt(np.maximum(l, 0.0)) / (2.0 * m)


def ps_weight(desc, m12, m34):
    """Four-body phase-space density in (m12, m34) with the angles uniform:
    q(M; m12, m34) q(m12; m1, m2) q(m34; m3, m4) (q: two-body momentum)."""
    M = float(desc["M"])
    m1, m2, m3, m4 = (float(v) for v in desc["m"])
    return _q(M, m12, m34) * _q(m12, m1, m2) * _q(m34, m3, m4)


def ps_wmax(desc) -> float:
    """1.05 x the largest phase-space weight on an 801 x 801 grid of the box."""
    M = float(desc["M"])
    m1, m2, m3, m4 = (float(v) for v in desc["m"])
    a = np.linspace(m1 + m2, M - m3 - m4, 801)
    b = np.linspace(m3 + m4, M - m1 - m2, 801)
    A, B = np.meshgrid(a, b, indexing="ij")
    w = np.where(A + B < M, ps_weight(desc, A, B), 0.0)
    return 1.05 * float(w.max())


GEN_MAX_ATTEMPTS = 65536  # attempts per event before it is left unresolved


def pair_proposal(lo: float, hi: float, entries):
    """Proposal density of one pair mass for the toy generator: probability
    1/2 uniform on [lo, hi] and 1/2 split equally over the pair's resonant
    entries (all of it uniform when there are none); entry r through a
    Student-t density of two degrees of freedom, (1 + x^2)^(-3/2) / 2 with
    x = (m - m0)/s, s = w0/2 (m0 +- s is the peak's half maximum), truncated
    to [lo, hi].  Its distribution function is (1 + v)/2, v = x/sqrt(1 + x^2),
    so a truncated draw is v uniform between the ends' values and
    x = v / sqrt(1 - v^2)."""
    m, s, vlo, vhi = [], [], [], []
    for e in entries:
        if float(e["m0"]) == 0.0:  # flat (non-resonant) entry
            continue
        m0, sc = float(e["m0"]), 0.5 * float(e["w0"])
        xlo, xhi = (lo - m0) / sc, (hi - m0) / sc
        m.append(m0)
        s.append(sc)
        vlo.append(xlo / math.sqrt(1.0 + xlo * xlo))
        vhi.append(xhi / math.sqrt(1.0 + xhi * xhi))
    return {"lo": lo, "hi": hi, "n": len(m), "wu": 0.5 if m else 1.0, "m": m, "s": s, "vlo": vlo, "vhi": vhi}


def proposal_draw(p, usel, upos):
    """Masses drawn from the pair proposal with component selectors usel and
    positions upos (arrays of uniforms)."""
    out = p["lo"] + upos * (p["hi"] - p["lo"])
    if p["n"] == 0:
        return out
    n, wu = p["n"], p["wu"]
    r = np.minimum(((usel - wu) / (1.0 - wu) * n).astype(np.int64), n - 1)
    res = usel >= wu
    for k in range(n):
        sel = res & (r == k)
        v = p["vlo"][k] + upos[sel] * (p["vhi"][k] - p["vlo"][k])
        out[sel] = p["m"][k] + p["s"][k] * (v / np.sqrt(1.0 - v * v))
    return out


def proposal_density(p, m):
    """The pair proposal's density at the masses m."""
    q = np.full(np.shape(m), (1.0 if p["n"] == 0 else p["wu"]) / (p["hi"] - p["lo"]))
    if p["n"]:
        wr = (1.0 - p["wu"]) / p["n"]
        for k in range(p["n"]):
            x = (m - p["m"][k]) / p["s"][k]
            t = 1.0 + x * x
            q = q + wr / ((p["s"][k] * (p["vhi"][k] - p["vlo"][k])) * (t * np.sqrt(t)))
    return q


def generate_events(theta, desc, n: int, seed: int, fit: int = 0, W: float = None, batch_env: int = 200_000):
    """Toy events (6, n) of the model, event by event, by accept-reject with
    importance sampling of the pair masses: attempt a of event i takes
    (u1, u2) ... (u9, u10) from Philox counters (i, 5a + j, word 4),
    j = 0..4, key (seed, fit); m12 from the r12 proposal (`pair_proposal`)
    with selector u1 and position u3, m34 from the r34 proposal with u2 and
    u4, c12 = 2 u5 - 1, c34 = 2 u6 - 1, phi = (2 u7 - 1) pi,
    t = -ln(1 - u8)/lam with lam = G (1 - |y|); kept when m12 + m34 < M and
    u9 W q12(m12) q34(m34) e^{-lam t} < w(m12, m34) R, w the phase-space
    weight and R the unconvolved rate (at most e^{-lam t} (|A| + |Abar|)^2,
    as in `generate`), so that the kept events follow w R; W bounds
    w (|A| + |Abar|)^2 / (q12 q34), by default 1.2 x its largest value on a
    phase-space sample.  The measured time adds sigma_t times a Box-Muller
    normal from counter (i, 0, 5).  Returns (events, W, number of kept events
    above W)."""
    from synth import td4_phase_space
    from synth.philox import key_from_seed, uniforms_at
    model = TD4(desc)
    th = as_t(theta)
    M = model.M
    m1, m2, m3, m4 = model.m
    p12 = pair_proposal(m1 + m2, M - m3 - m4, desc["r12"])
    p34 = pair_proposal(m3 + m4, M - m1 - m2, desc["r34"])
    G = 1.0 / model.tau
    y = float(theta[model.P - 1])
    lam = G * (1.0 - abs(y))

    def ratio(kin):
        with torch.no_grad():
            A, Ab = model.amplitudes(th, model.basis(torch.from_numpy(kin)))
            env = ((A.abs() + Ab.abs()) ** 2).numpy()
        return ps_weight(desc, kin[0], kin[1]) * env / (proposal_density(p12, kin[0]) * proposal_density(p34, kin[1]))

    if W is None:
        W = 1.2 * float(ratio(td4_phase_space(batch_env, seed, fit, stream0=5000)).max())
    key = key_from_seed(seed, fit)
    out = np.full((6, n), np.nan)
    todo = np.arange(n, dtype=np.uint64)
    above = 0
    for a in range(GEN_MAX_ATTEMPTS):
        if todo.size == 0:
            break
        u1, u2 = uniforms_at(todo, key, 5 * a, 4)
        u3, u4 = uniforms_at(todo, key, 5 * a + 1, 4)
        u5, u6 = uniforms_at(todo, key, 5 * a + 2, 4)
        u7, u8 = uniforms_at(todo, key, 5 * a + 3, 4)
        u9, _ = uniforms_at(todo, key, 5 * a + 4, 4)
        m12 = proposal_draw(p12, u1, u3)
        m34 = proposal_draw(p34, u2, u4)
        w = np.where(m12 + m34 < M, ps_weight(desc, m12, m34), 0.0)
        ok = w > 0.0
        keep = np.zeros(todo.size, dtype=bool)
        if ok.any():
            kin = np.stack([m12[ok], m34[ok], 2.0 * u5[ok] - 1.0, 2.0 * u6[ok] - 1.0, (2.0 * u7[ok] - 1.0) * math.pi])
            t = -np.log1p(-u8[ok]) / lam
            with torch.no_grad():
                r = unconvolved_rate(model, th, torch.from_numpy(kin), torch.from_numpy(t)).numpy()
            q12, q34 = proposal_density(p12, kin[0]), proposal_density(p34, kin[1])
            k = u9[ok] * W * q12 * q34 * np.exp(-lam * t) < w[ok] * r
            sel = np.flatnonzero(ok)[k]
            keep[sel] = True
            if k.any():
                above += int((ratio(kin[:, k]) > W).sum())
            idx = todo[sel].astype(np.int64)
            out[:5, idx] = kin[:, k]
            out[5, idx] = t[k]
        todo = todo[~keep]
    i = np.arange(n, dtype=np.uint64)
    v1, v2 = uniforms_at(i, key, 0, 5)
    out[5] = out[5] + model.sigma * np.sqrt(-2.0 * np.log1p(-v1)) * np.cos(2.0 * math.pi * v2)
    return out, W, above
