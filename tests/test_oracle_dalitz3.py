"""Pins of the Dalitz-plot oracle against explicit four-vector kinematics,
closed-form lineshape properties, quadrature, invariances and finite
differences (CPU only)."""
import math

import numpy as np
import pytest
import torch
from scipy import integrate

import synth
from oracle import common, dalitz3 as D

DESC = D.config1_desc()
MODEL = D.Dalitz(DESC)
TH = D.truth_theta(DESC)


def four_vectors(s12, s13, M, m1, m2, m3):
    """Momenta of the three daughters in the parent rest frame, built from
    energies E_i = (M^2 + m_i^2 - s_jk)/(2M) and momentum balance."""
    s23 = M * M + m1 * m1 + m2 * m2 + m3 * m3 - s12 - s13
    e1 = (M * M + m1 * m1 - s23) / (2 * M)
    e2 = (M * M + m2 * m2 - s13) / (2 * M)
    e3 = (M * M + m3 * m3 - s12) / (2 * M)
    p1 = np.sqrt(e1 * e1 - m1 * m1)
    p2 = np.sqrt(e2 * e2 - m2 * m2)
    p3 = np.sqrt(e3 * e3 - m3 * m3)
    cos12 = (p3 * p3 - p1 * p1 - p2 * p2) / (2 * p1 * p2)
    sin12 = np.sqrt(np.maximum(1 - cos12 ** 2, 0))
    z = np.zeros_like(s12)
    v1 = np.stack([e1, z, z, p1], -1)
    v2 = np.stack([e2, p2 * sin12, z, p2 * cos12], -1)
    v3 = np.stack([e3, -v1[:, 1] - v2[:, 1], z, -v1[:, 3] - v2[:, 3]], -1)
    return {1: v1, 2: v2, 3: v3}


def boost_to_rest(v, P):
    """Lorentz-boost four-vectors v into the rest frame of four-vector P."""
    beta = P[:, 1:] / P[:, :1]
    b2 = (beta * beta).sum(-1, keepdims=True)
    gam = 1 / np.sqrt(1 - b2)
    bp = (beta * v[:, 1:]).sum(-1, keepdims=True)
    e = gam * (v[:, :1] - bp)
    coef = (gam - 1) * bp / b2 - gam * v[:, :1]
    return np.concatenate([e, v[:, 1:] + coef * beta], -1)


@pytest.mark.parametrize("pair", ["12", "13", "23"])
def test_momenta_and_zemach_vs_four_vectors(pair):
    ev = synth.dalitz_events(2000, seed=3)
    M, m1, m2, m3 = synth.DALITZ_MASSES
    vs = four_vectors(ev[0], ev[1], M, m1, m2, m3)
    ia, ib, ic = {"12": (1, 2, 3), "13": (1, 3, 2), "23": (2, 3, 1)}[pair]
    P = vs[ia] + vs[ib]
    pa = boost_to_rest(vs[ia], P)[:, 1:]
    pc = boost_to_rest(vs[ic], P)[:, 1:]
    qa = np.linalg.norm(pa, axis=-1)
    qc = np.linalg.norm(pc, axis=-1)
    s12, s13 = torch.tensor(ev[0]), torch.tensor(ev[1])
    s_ab, _, _ = MODEL.pair_invariants(pair, s12, s13)
    q, p = MODEL.momenta(pair, s_ab)
    assert np.allclose(q.numpy(), qa, rtol=1e-9, atol=0)
    assert np.allclose(p.numpy(), qc, rtol=1e-9, atol=0)
    dot = (pa * pc).sum(-1)
    z1 = MODEL.zemach(pair, 1, s12, s13).numpy()
    z2 = MODEL.zemach(pair, 2, s12, s13).numpy()
    scale = 4 * qa * qc
    assert np.allclose(z1, -4 * dot, rtol=0, atol=1e-9 * scale.max())
    cos = dot / (qa * qc)
    assert np.allclose(z2, 16 * qa ** 2 * qc ** 2 * (cos ** 2 - 1 / 3), rtol=0, atol=1e-9 * scale.max() ** 2)


@pytest.mark.parametrize("k", range(8))
def test_lineshape_at_pole_mass(k):
    """Gamma(m0^2) = Gamma0, so T(m0^2) = i/(m0 Gamma0)."""
    pair, L, m0, w0 = MODEL.res[k]
    t = MODEL.lineshape(pair, L, torch.tensor(m0), torch.tensor(w0), torch.tensor([m0 * m0]))
    assert abs(float(t.real[0])) < 1e-13 / (m0 * w0)
    assert abs(float(t.imag[0]) * m0 * w0 - 1) < 1e-13


@pytest.mark.parametrize("pair,L,m0", [("23", 1, 0.77), ("12", 0, 1.2), ("12", 2, 1.43)])
def test_narrow_width_lineshape_integral(pair, L, m0):
    """As Gamma0 -> 0 the integral of |T|^2 over s tends to pi/(m0 Gamma0)."""
    w0 = 1e-4
    ia, ib, ic = {"12": (1, 2, 3), "13": (1, 3, 2), "23": (2, 3, 1)}[pair]
    M = MODEL.M
    lo, hi = (MODEL.m[ia] + MODEL.m[ib]) ** 2, (M - MODEL.m[ic]) ** 2

    def f(s):
        t = MODEL.lineshape(pair, L, torch.tensor(m0), torch.tensor(w0), torch.tensor([s]))
        return float(t.real[0] ** 2 + t.imag[0] ** 2)
    val = 0.0
    pts = [lo, m0 * m0 - 50 * m0 * w0, m0 * m0, m0 * m0 + 50 * m0 * w0, hi]
    for a, b in zip(pts[:-1], pts[1:]):
        val += integrate.quad(f, a, b, limit=400, epsabs=0, epsrel=1e-11)[0]
    assert abs(val * m0 * w0 / math.pi - 1) < 2e-3


def test_grid_area_vs_quadrature():
    """Inside cells x dA against the region area: int 4 p1* p3* ds12, with the
    momenta of particles 1 and 3 in the (12) rest frame."""
    M, m1, m2, m3 = synth.DALITZ_MASSES

    def width(s):
        rs = math.sqrt(s)
        e1 = (s + m1 * m1 - m2 * m2) / (2 * rs)
        e3 = (M * M - s - m3 * m3) / (2 * rs)
        return 4 * math.sqrt(max(e1 * e1 - m1 * m1, 0)) * math.sqrt(max(e3 * e3 - m3 * m3, 0))
    area = integrate.quad(width, (m1 + m2) ** 2, (M - m3) ** 2, limit=200, epsabs=0, epsrel=1e-12)[0]
    c12, c13, da = MODEL.grid_cells()
    assert c12.size == 497806
    assert abs(c12.size * da / area - 1) < 2e-4


def test_grid_norm_vs_quadrature():
    """Midpoint-grid I against a composite Gauss-Legendre rule over the
    region (slices in s12, exact s13 limits per slice)."""
    M, m1, m2, m3 = synth.DALITZ_MASSES
    x, w = np.polynomial.legendre.leggauss(8)
    (a12, b12), _ = MODEL.box()
    edges = np.linspace(a12, b12, 161)
    s12n = ((edges[:-1, None] + edges[1:, None]) / 2 + (edges[1:, None] - edges[:-1, None]) / 2 * x).ravel()
    w12 = ((edges[1:, None] - edges[:-1, None]) / 2 * w).ravel()
    rs = np.sqrt(s12n)
    e1 = (s12n + m1 * m1 - m2 * m2) / (2 * rs)
    e3 = (M * M - s12n - m3 * m3) / (2 * rs)
    p1 = np.sqrt(e1 * e1 - m1 * m1)
    p3 = np.sqrt(e3 * e3 - m3 * m3)
    lo = m1 * m1 + m3 * m3 + 2 * (e1 * e3 - p1 * p3)
    hi = m1 * m1 + m3 * m3 + 2 * (e1 * e3 + p1 * p3)
    t = np.linspace(0, 1, 161)
    u = ((t[:-1, None] + t[1:, None]) / 2 + (t[1:, None] - t[:-1, None]) / 2 * x).ravel()
    wu = ((t[1:, None] - t[:-1, None]) / 2 * w).ravel()
    S12 = np.repeat(s12n, u.size)
    S13 = (lo[:, None] + (hi - lo)[:, None] * u[None, :]).ravel()
    W = (w12[:, None] * (hi - lo)[:, None] * wu[None, :]).ravel()
    with torch.no_grad():
        pv = MODEL.density_unnorm(torch.tensor(TH), torch.tensor(S12), torch.tensor(S13)).numpy()
    quad = float((pv * W).sum())
    grid = D.norm_value(MODEL, TH)
    assert abs(grid / quad - 1) < 1e-3, (grid, quad)


def test_coefficient_rescaling_invariance():
    ev = synth.dalitz_events(3000, seed=5)
    cells = D.Dalitz(D.config1_desc(grid=(128, 128))).grid_cells()
    d = D.config1_desc(grid=(128, 128))
    a, g = D.nll_grad(TH, ev, d, cells)
    rot = 1.7 * complex(math.cos(0.9), math.sin(0.9))
    c = TH[0::2] + 1j * TH[1::2]
    c2 = rot * c
    th2 = np.empty_like(TH)
    th2[0::2], th2[1::2] = c2.real, c2.imag
    b = D.nll(th2, ev, d, cells)
    assert abs(a - b) < 1e-12 * abs(a)
    gr, gi = g[0::2], g[1::2]
    norm = np.abs(g).max() * np.abs(c).max()
    assert abs((c.real * gr + c.imag * gi).sum()) < 1e-10 * norm
    assert abs((-c.imag * gr + c.real * gi).sum()) < 1e-10 * norm


def test_relabel_daughters_two_and_three():
    """Swapping daughters 2 and 3 (masses, pair names, s12 <-> s13) leaves
    P~ unchanged once odd-L coefficients in pair 23 change sign (A <-> B)."""
    M, m1, m2, m3 = synth.DALITZ_MASSES
    swap = {"12": "13", "13": "12", "23": "23"}
    table2 = []
    for (pair, L, m0, w0, c) in D.RESONANCES:
        sgn = -1.0 if (pair == "23" and L % 2 == 1) else 1.0
        table2.append((swap[pair], L, m0, w0, (sgn * c[0], sgn * c[1])))
    d2 = D.config1_desc(resonances=table2, masses=(M, m1, m3, m2))
    th2 = D.truth_theta(d2, resonances=table2)
    ev = synth.dalitz_events(3000, seed=6)
    with torch.no_grad():
        p1 = MODEL.density_unnorm(torch.tensor(TH), torch.tensor(ev[0]), torch.tensor(ev[1])).numpy()
        p2 = D.Dalitz(d2).density_unnorm(torch.tensor(th2), torch.tensor(ev[1]), torch.tensor(ev[0])).numpy()
    assert np.allclose(p1, p2, rtol=1e-11, atol=0)


@pytest.mark.parametrize("free", [False, True])
def test_autograd_vs_central_fd(free):
    d = D.config1_desc(grid=(96, 96), free_lineshapes=free)
    th = D.truth_theta(d)
    th = th + 0.03 * np.sin(np.arange(th.size) + 1.0) * np.maximum(np.abs(th), 0.05)
    ev = synth.dalitz_events(2000, seed=7)
    cells = D.Dalitz(d).grid_cells()
    _, g = D.nll_grad(th, ev, d, cells)
    # events where the amplitude sum nearly vanishes make the third derivative
    # large in the small coefficients; a relative step of 2e-7 keeps both the
    # truncation and the rounding error of the difference below the bound
    fd = common.central_fd(lambda t: D.nll(t, ev, d, cells), th, rel_step=2e-7)
    tol = 1e-6 * np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max())
    assert (np.abs(g - fd) <= tol).all(), np.abs(g - fd) / tol


def _hankel_abs(L, x):
    """|x h_L(x)| with h_L = j_L + i y_L, the spherical Hankel function."""
    from scipy.special import spherical_jn, spherical_yn
    return x * np.hypot(spherical_jn(L, x), spherical_yn(L, x))


@pytest.mark.parametrize("k", range(8))
def test_width_and_barriers_vs_spherical_hankel(k):
    """Penetration factor P_L(x) = x / |x h_L(x)|^2 gives the running width
    Gamma(s) = Gamma0 (m0/sqrt s) P_L(q r)/P_L(q0 r), and the barrier factor
    is F_L(x) = 1 / (x^L |x h_L(x)|); both from the scattering solutions, not
    from the polynomial forms the oracle uses."""
    pair, L, m0, w0 = MODEL.res[k]
    ev = synth.dalitz_events(500, seed=8)
    s12, s13 = torch.tensor(ev[0]), torch.tensor(ev[1])
    s_ab, _, _ = MODEL.pair_invariants(pair, s12, s13)
    t = MODEL.lineshape(pair, L, torch.tensor(m0), torch.tensor(w0), s_ab)
    inv = 1.0 / t
    q, p = MODEL.momenta(pair, s_ab)
    q0 = float(MODEL.q0(pair, torch.tensor(m0)))
    r, rd = MODEL.r_res, MODEL.r_D
    q, p, s = q.numpy(), p.numpy(), s_ab.numpy()
    pen = lambda x: x / _hankel_abs(L, x) ** 2
    gam = w0 * (m0 / np.sqrt(s)) * pen(q * r) / pen(q0 * r)
    assert np.allclose(inv.real.numpy(), m0 * m0 - s, rtol=1e-12, atol=1e-12)
    assert np.allclose(-inv.imag.numpy() / m0, gam, rtol=1e-10, atol=0)
    bf = lambda x: 1.0 / (x ** L * _hankel_abs(L, x))
    z = MODEL.zemach(pair, L, s12, s13).numpy()
    amp = MODEL.amplitude(k, s12, s13, torch.tensor(m0), torch.tensor(w0)).numpy()
    expect = bf(q * r) / bf(q0 * r) * bf(p * rd) * z * t.numpy()
    assert np.allclose(amp, expect, rtol=1e-10, atol=1e-14 * np.abs(expect).max())


# ------------------------------------------------------------ toy generation
@pytest.fixture(scope="module")
def toy_sample():
    d = D.config1_desc(grid=(256, 256))
    th = D.truth_theta(d)
    ev, W, above = D.generate(th, d, 12_000, seed=5, fit=2)
    return d, th, ev, W, above


def test_generated_moments_match_the_density(toy_sample):
    """Sample means of s12, s13, s12^2 and s12 s13 agree with their
    expectations under P~ (fine-grid quadrature over the region) within 4
    standard errors: a swapped coordinate, a wrong box, an inverted accept
    test or a dropped region cut moves them by many."""
    d, th, ev, W, above = toy_sample
    assert above == 0 and np.isfinite(ev).all()
    model = D.Dalitz(dict(d, grid=[1024, 1024]))
    c12, c13, _ = model.grid_cells()
    with torch.no_grad():
        w = model.density_unnorm(common.as_t(th), common.as_t(c12), common.as_t(c13)).numpy()
    w = w / w.sum()
    for f in (lambda a, b: a, lambda a, b: b, lambda a, b: a * a, lambda a, b: a * b):
        x = f(ev[0], ev[1])
        expect = float((w * f(c12, c13)).sum())
        se = x.std() / math.sqrt(x.size)
        assert abs(x.mean() - expect) < 4.0 * se, (x.mean(), expect, se)


def test_generated_events_lie_in_the_region(toy_sample):
    d, th, ev, W, above = toy_sample
    model = D.Dalitz(d)
    assert model.inside(ev[0], ev[1]).all()


def test_generation_is_per_event(toy_sample):
    """Event i depends only on (theta, seed, fit, W, i): a shorter run is a
    prefix, another fit index gives other events."""
    d, th, ev, W, above = toy_sample
    head, W2, _ = D.generate(th, d, 500, seed=5, fit=2, W=W)
    assert W2 == W and np.array_equal(head, ev[:, :500])
    other, _, _ = D.generate(th, d, 500, seed=5, fit=3, W=W)
    assert not np.any(other[0] == ev[0, :500])


def test_low_envelope_is_reported():
    d = D.config1_desc(grid=(128, 128))
    th = D.truth_theta(d)
    W = D.envelope(th, d)
    _, _, above = D.generate(th, d, 2000, seed=6, W=0.2 * W)
    assert above > 0
