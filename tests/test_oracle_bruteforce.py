"""Brute-force pins of the composed amplitude NLLs (CPU only).

Each model is evaluated here a second time, at 50 significant digits with
mpmath, on ten events, from formulas other than the ones the oracle uses
wherever a second formula exists:

* two-body momenta from rest-frame energies, E_A = (s + mA^2 - mB^2)/(2 sqrt s)
  and q = sqrt(E_A^2 - mA^2), instead of the Kallen function;
* the Zemach factors from the rest-frame scalar product of the daughter and
  bachelor momenta, Z1 = -4 q.p and Z2 = Z1^2 - 16 |q|^2 |p|^2 / 3, with q.p
  read off s_AC (the oracle uses the invariant form);
* the physical region from the cosine of the angle between daughters 2 and 3
  in the (12) rest frame lying in [-1, 1] (the oracle compares s23 with its
  two limits);
* the decay-time dependence by numerical convolution of the unconvolved rate
  with the Gaussian resolution, and its time integral by quadrature (the
  oracle maps each term onto h(a; t) through the Faddeeva function and uses
  the closed-form integrals).

Then NLL = -sum ln P~ + N ln I with I summed over a small grid (three-body
models) or averaged over a small phase-space sample (four-body model), as the
normalization definitions say.  The oracle's NLL must agree to 1e-13
relative: a dropped term, a wrong sign or index, a transposed pair or a
mis-scaled normalization fails.

Also here: the oracle's decay-time function h(a; t), evaluated through
scipy's Faddeeva function on two branches, against mpmath's complementary
error function of complex argument on a 200-point grid that reaches
|z| > 10 and Im z < 0, and scipy's w(z) itself against mpmath.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import torch

import synth
from oracle import dalitz3 as OD, td4 as OT, tddp3 as OP

mp.mp.dps = 50
NEV = 10
PAIRS = {"12": (1, 2, 3), "13": (1, 3, 2), "23": (2, 3, 1)}


def F(L, z):
    """Blatt-Weisskopf barrier factor of spin L at z = (q r)^2."""
    if L == 0:
        return mp.mpf(1)
    if L == 1:
        return 1 / mp.sqrt(1 + z)
    return 1 / mp.sqrt(z * z + 3 * z + 9)


def rest_momentum(s, ma, mb):
    """|q| of daughter a in the rest frame of a pair of mass^2 s, and E_a."""
    rs = mp.sqrt(s)
    ea = (s + ma * ma - mb * mb) / (2 * rs)
    return mp.sqrt(max(ea * ea - ma * ma, mp.mpf(0))), ea


class ThreeBody:
    """Isobar amplitudes of a three-body decay at 50 digits."""

    def __init__(self, desc, theta=None, free=False):
        self.M = mp.mpf(desc["M"])
        self.m = {i + 1: mp.mpf(v) for i, v in enumerate(desc["m"])}
        self.r = mp.mpf(desc.get("r_res", 1.5))
        self.rD = mp.mpf(desc.get("r_D", 5.0))
        self.res = []
        K = len(desc["resonances"])
        for k, r in enumerate(desc["resonances"]):
            m0, w0 = mp.mpf(r["m0"]), mp.mpf(r["w0"])
            if free:
                m0, w0 = mp.mpf(theta[2 * K + 2 * k]), mp.mpf(theta[2 * K + 2 * k + 1])
            self.res.append((r["pair"], int(r["L"]), m0, w0))

    def s23(self, s12, s13):
        m = self.m
        return self.M ** 2 + m[1] ** 2 + m[2] ** 2 + m[3] ** 2 - s12 - s13

    def amp(self, k, s12, s13):
        pair, L, m0, w0 = self.res[k]
        a, b, c = PAIRS[pair]
        ma, mb, mc = self.m[a], self.m[b], self.m[c]
        sij = {(1, 2): s12, (1, 3): s13, (2, 3): self.s23(s12, s13)}
        inv = lambda i, j: sij[(min(i, j), max(i, j))]
        s, s_ac = inv(a, b), inv(a, c)
        q, ea = rest_momentum(s, ma, mb)
        # bachelor energy and momentum in the pair rest frame
        ec = (self.M ** 2 - s - mc * mc) / (2 * mp.sqrt(s))
        p = mp.sqrt(max(ec * ec - mc * mc, mp.mpf(0)))
        q0, _ = rest_momentum(m0 * m0, ma, mb)
        qp = (ma * ma + mc * mc + 2 * ea * ec - s_ac) / 2  # q_vec . p_vec
        z1 = -4 * qp
        Z = (mp.mpf(1), z1, z1 * z1 - mp.mpf(16) / 3 * q * q * p * p)[L]
        fr = F(L, (q * self.r) ** 2) / F(L, (q0 * self.r) ** 2)
        gam = w0 * (q / q0) ** (2 * L + 1) * (m0 / mp.sqrt(s)) * fr * fr
        T = 1 / mp.mpc(m0 * m0 - s, -m0 * gam)
        return fr * F(L, (p * self.rD) ** 2) * Z * T

    def coherent(self, coef, s12, s13):
        return mp.fsum(coef[k] * self.amp(k, s12, s13) for k in range(len(self.res)))

    def inside(self, s12, s13):
        """|cos| <= 1 for the angle between daughters 2 and 3 in the (12)
        frame; also the distance from the boundary."""
        m = self.m
        p2, e2 = rest_momentum(s12, m[2], m[1])
        e3 = (self.M ** 2 - s12 - m[3] ** 2) / (2 * mp.sqrt(s12))
        p3 = mp.sqrt(max(e3 * e3 - m[3] ** 2, mp.mpf(0)))
        cs = (m[2] ** 2 + m[3] ** 2 + 2 * e2 * e3 - self.s23(s12, s13)) / (2 * p2 * p3)
        return abs(cs) <= 1, abs(abs(cs) - 1)

    def grid(self, nx, ny):
        """Inside cell centres and the cell area of an nx x ny grid."""
        M, m = self.M, self.m
        a12, b12 = (m[1] + m[2]) ** 2, (M - m[3]) ** 2
        a13, b13 = (m[1] + m[3]) ** 2, (M - m[2]) ** 2
        d12, d13 = (b12 - a12) / nx, (b13 - a13) / ny
        cells = []
        for i in range(nx):
            for j in range(ny):
                c12, c13 = a12 + (i + mp.mpf(0.5)) * d12, a13 + (j + mp.mpf(0.5)) * d13
                ins, dist = self.inside(c12, c13)
                # the double-precision predicate of the oracle decides these
                # centres the same way only away from the boundary
                assert dist > mp.mpf(1e-9), (i, j)
                if ins:
                    cells.append((c12, c13))
        return cells, d12 * d13


def coefs(theta, K, off=0):
    return [mp.mpc(theta[off + 2 * k], theta[off + 2 * k + 1]) for k in range(K)]


def rel(a, b):
    return abs(a - b) / abs(b)


# ----------------------------------------------------------- three-body model
@pytest.mark.parametrize("free", [False, True])
def test_dalitz3_nll_brute_force(free):
    desc = OD.config1_desc(grid=(24, 24), free_lineshapes=free)
    th = OD.truth_theta(desc)
    th = th * (1.0 + 0.02 * np.sin(1.3 * np.arange(th.size) + 0.4))
    ev = synth.dalitz_events(NEV, seed=4711)
    bf = ThreeBody(desc, th, free)
    K = len(desc["resonances"])
    c = coefs(th, K)
    lp = [mp.log(abs(bf.coherent(c, mp.mpf(ev[0, i]), mp.mpf(ev[1, i]))) ** 2) for i in range(NEV)]
    cells, dA = bf.grid(24, 24)
    norm = dA * mp.fsum(abs(bf.coherent(c, a, b)) ** 2 for (a, b) in cells)
    ref = -mp.fsum(lp) + NEV * mp.log(norm)
    got = OD.nll(th, ev, desc)
    assert rel(mp.mpf(OD.norm_value(OD.Dalitz(desc), th)), norm) < 1e-13
    assert rel(mp.mpf(got), ref) < 1e-13, (got, ref)


# ----------------------------------------------------- decay-time functions
def convolved(rate_u, t, sigma, G):
    """int_0^inf rate_u(u) G_sigma(t - u) du by quadrature."""
    t, s = mp.mpf(t), mp.mpf(sigma)
    g = lambda u: rate_u(u) * mp.exp(-(t - u) ** 2 / (2 * s * s)) / (s * mp.sqrt(2 * mp.pi))
    pts = sorted({mp.mpf(0), max(mp.mpf(0), t - 12 * s), max(mp.mpf(0), t), max(mp.mpf(0), t + 12 * s)})
    return mp.quad(g, pts + [mp.inf])


def mixing_rate(A, Ab, x, y, G):
    """The unconvolved rate as a function of u >= 0."""
    a2, b2 = abs(A) ** 2, abs(Ab) ** 2
    z = mp.conj(A) * Ab
    x, y = mp.mpf(x), mp.mpf(y)

    def r(u):
        gu = G * u
        return mp.exp(-gu) / 2 * ((a2 + b2) * mp.cosh(y * gu) + (a2 - b2) * mp.cos(x * gu)
                                  - 2 * z.real * mp.sinh(y * gu) - 2 * z.imag * mp.sin(x * gu))
    return r


def time_integrals(x, y, G):
    """Integrals over u >= 0 of e^{-Gu} times cosh, cos, sinh, sin."""
    x, y = mp.mpf(x), mp.mpf(y)
    f = lambda h: mp.quad(lambda u: mp.exp(-G * u) * h(u), [0, 1 / G, 10 / G, mp.inf])
    return (f(lambda u: mp.cosh(y * G * u)), f(lambda u: mp.cos(x * G * u)),
            f(lambda u: mp.sinh(y * G * u)), f(lambda u: mp.sin(x * G * u)))


def integrated(A, Ab, ti):
    a2, b2 = abs(A) ** 2, abs(Ab) ** 2
    z = mp.conj(A) * Ab
    ch, co, sh, si = ti
    return ((a2 + b2) * ch + (a2 - b2) * co - 2 * z.real * sh - 2 * z.imag * si) / 2


# ------------------------------------------- time-dependent three-body model
@pytest.mark.parametrize("xy", [(0.0039, 0.0065), (0.3, -0.2)])
def test_tddp3_nll_brute_force(xy):
    desc = OP.pipipi0_desc(grid=(16, 16))
    th = OP.truth_theta(x=xy[0], y=xy[1])
    K = len(desc["resonances"])
    th[2 * K:4 * K] *= 1.0 + 0.1 * np.cos(np.arange(2 * K))  # cbar != c
    ev = synth.tddp3_events(NEV, seed=4712, sigma_t=desc["sigma_t"])
    bf = ThreeBody(desc)
    c, cb = coefs(th, K), coefs(th, K, 2 * K)
    G = 1 / mp.mpf(desc["tau"])
    x, y = th[-2], th[-1]

    def amps(s12, s13):
        return bf.coherent(c, s12, s13), bf.coherent(cb, s13, s12)  # Dbar0 at the mirrored point

    lp = []
    for i in range(NEV):
        A, Ab = amps(mp.mpf(ev[0, i]), mp.mpf(ev[1, i]))
        lp.append(mp.log(convolved(mixing_rate(A, Ab, x, y, G), ev[2, i], desc["sigma_t"], G)))
    ti = time_integrals(x, y, G)
    cells, dA = bf.grid(16, 16)
    norm = dA * mp.fsum(integrated(*amps(a, b), ti) for (a, b) in cells)
    ref = -mp.fsum(lp) + NEV * mp.log(norm)
    got = OP.nll(th, ev, desc)
    assert rel(mp.mpf(got), ref) < 1e-13, (got, ref)


# ---------------------------------------------- time-dependent four-body model
class FourBody:
    def __init__(self, desc):
        self.m = [mp.mpf(v) for v in desc["m"]]
        self.r = mp.mpf(desc.get("r_res", 1.5))
        self.r12 = [(int(e["L"]), mp.mpf(e["m0"]), mp.mpf(e["w0"])) for e in desc["r12"]]
        self.r34 = [(int(e["L"]), mp.mpf(e["m0"]), mp.mpf(e["w0"])) for e in desc["r34"]]
        self.amps = [tuple(int(v) for v in a[:3]) for a in desc["amps"]]
        self.sides = [a[3] if len(a) > 3 else "both" for a in desc["amps"]]

    def lineshape(self, m, ma, mb, e):
        L, m0, w0 = e
        if m0 == 0:
            return mp.mpc(1)
        q, _ = rest_momentum(m * m, ma, mb)
        q0, _ = rest_momentum(m0 * m0, ma, mb)
        fr = F(L, (q * self.r) ** 2) / F(L, (q0 * self.r) ** 2)
        gam = w0 * (q / q0) ** (2 * L + 1) * (m0 / m) * fr * fr
        return fr / mp.mpc(m0 * m0 - m * m, -m0 * gam)

    @staticmethod
    def angular(typ, c12, c34, phi):
        s = mp.sqrt(1 - c12 * c12) * mp.sqrt(1 - c34 * c34) / 2
        return (mp.mpc(1), c34, c12, c12 * c34, s * mp.expjpi(phi / mp.pi), s * mp.expjpi(-phi / mp.pi))[typ]

    def basis(self, kin, amps):
        m12, m34, c12, c34, phi = (mp.mpf(v) for v in kin)
        m1, m2, m3, m4 = self.m
        a12 = [self.lineshape(m12, m1, m2, e) for e in self.r12]
        a34 = [self.lineshape(m34, m3, m4, e) for e in self.r34]
        return [a12[i] * a34[j] * self.angular(typ, c12, c34, phi) for (i, j, typ) in amps]


def four_body_coefs(bf, th):
    """Per basis function its coefficient in A and in Abar (0 where it is not
    a member): theta lists the members of A in description order, then those
    of Abar, then x and y."""
    K = len(bf.amps)
    members_a = [k for k in range(K) if bf.sides[k] != "Abar"]
    members_b = [k for k in range(K) if bf.sides[k] != "A"]
    c, cb = [mp.mpc(0)] * K, [mp.mpc(0)] * K
    for j, k in enumerate(members_a):
        c[k] = mp.mpc(th[2 * j], th[2 * j + 1])
    off = 2 * len(members_a)
    for j, k in enumerate(members_b):
        cb[k] = mp.mpc(th[off + 2 * j], th[off + 2 * j + 1])
    assert off + 2 * len(members_b) + 2 == len(th)
    return c, cb


@pytest.mark.parametrize("model,xy", [("shared", (0.004, 0.006)), ("shared", (0.25, 0.3)),
                                      ("split", (0.004, 0.006)), ("split", (-0.2, 0.35))])
def test_td4_nll_brute_force(model, xy):
    """Ten shared basis functions with two coefficient sets, and twenty
    distinct ones split ten into A and ten into Abar."""
    desc = synth.td4_desc() if model == "shared" else synth.td4_split_desc()
    th = synth.td4_truth() if model == "shared" else synth.td4_split_truth()
    th[-2:] = xy
    ev = synth.td4_events(NEV, seed=4713)
    mc = synth.td4_phase_space(40, seed=4714)
    bf = FourBody(desc)
    K = len(desc["amps"])
    c, cb = four_body_coefs(bf, th)
    G = 1 / mp.mpf(desc["tau"])

    def amps(kin):
        B = bf.basis(kin, bf.amps)
        return mp.fsum(c[k] * B[k] for k in range(K)), mp.fsum(cb[k] * B[k] for k in range(K))

    lp = []
    for i in range(NEV):
        A, Ab = amps(ev[:5, i])
        lp.append(mp.log(convolved(mixing_rate(A, Ab, xy[0], xy[1], G), ev[5, i], desc["sigma_t"], G)))
    ti = time_integrals(xy[0], xy[1], G)
    norm = mp.fsum(integrated(*amps(mc[:, j]), ti) for j in range(mc.shape[1])) / mc.shape[1]
    ref = -mp.fsum(lp) + NEV * mp.log(norm)
    got = OT.nll(th, ev, mc, desc)
    assert rel(mp.mpf(got), ref) < 1e-13, (got, ref)


# ------------------------------------------------------------ Faddeeva pins
def h_mp(a, t, sigma):
    """h(a; t) = 1/2 exp(a^2 s^2/2 - a t) erfc((a s^2 - t)/(s sqrt 2)) at 50 digits."""
    a, t, s = mp.mpc(a), mp.mpf(t), mp.mpf(sigma)
    return mp.exp(a * a * s * s / 2 - a * t) * mp.erfc((a * s * s - t) / (s * mp.sqrt(2))) / 2


def h_grid():
    """200 (a, t, sigma) points: real a = G(1 -+ y) and complex a = G(1 - i x)
    at the workloads' and at large mixing, t from -0.6 to 8 ps, sigma 0.05
    and 0.1 ps."""
    G = 1 / 0.41
    avals = [G * 0.994, G * 1.006, complex(G, -G * 0.004), complex(G, -G * 0.3), complex(G * 0.7, G * 0.5)]
    tvals = np.concatenate([np.linspace(-0.6, 0.2, 8), np.linspace(0.25, 8.0, 12)])
    return [(a, t, s) for a in avals for s in (0.05, 0.1) for t in tvals]


def test_h_against_mpmath_on_a_grid():
    pts = h_grid()
    assert len(pts) == 200
    zs = [(complex(a) * s * s - t) / (s * math.sqrt(2.0)) for (a, t, s) in pts]
    assert sum(abs(z) > 10 for z in zs) >= 20 and sum(z.imag < 0 for z in zs) >= 60
    worst = 0.0
    for (a, t, s) in pts:
        got = complex(OT.h_conv(complex(a), torch.tensor([t], dtype=torch.float64), s).numpy()[0])
        ref = h_mp(a, t, s)
        err = float(abs(mp.mpc(got) - ref) / abs(ref))
        worst = max(worst, err)
        assert err < 1e-13, (a, t, s, got, ref)
    print("largest relative error of h:", worst)


def test_scipy_faddeeva_against_mpmath():
    """w(z) = exp(-z^2) erfc(-i z) on 200 points of both half planes, |z| up
    to 30 (the oracle only calls it in the upper half plane)."""
    from scipy.special import wofz
    rng = np.random.default_rng(11)
    r = np.concatenate([rng.uniform(0.0, 3.0, 80), rng.uniform(3.0, 30.0, 120)])
    ang = rng.uniform(-math.pi, math.pi, 200)
    z = r * np.exp(1j * ang)
    # in the lower half plane w grows like exp(y^2 - x^2); stay where it is finite
    z = np.where((z.imag < 0) & (z.imag ** 2 - z.real ** 2 > 600), np.conj(z), z)
    assert (np.abs(z) > 10).sum() >= 80 and (z.imag < 0).sum() >= 50
    for zz in z:
        ref = mp.exp(-mp.mpc(zz) ** 2) * mp.erfc(-1j * mp.mpc(zz))
        got = wofz(zz)
        assert abs(mp.mpc(got) - ref) / abs(ref) < 2e-13, (zz, got, ref)
