"""Pins of the time-dependent four-body oracle (CPU only)."""
import math

import numpy as np
import pytest
import torch
from scipy import integrate

import synth
from oracle import common, td4 as OT

DESC = synth.td4_desc()
TH = synth.td4_truth()
MODEL = OT.TD4(DESC)
SIG = synth.TD4_SIGMA_T


def h(a, t, sigma=SIG):
    return OT.h_conv(complex(a), torch.tensor(np.atleast_1d(t), dtype=torch.float64), sigma).numpy()


@pytest.mark.parametrize("a", [2.439 * (1 - 0.006), 2.439 * (1 + 0.3), complex(2.439, -2.439 * 0.004),
                               complex(1.2, 0.9)])
@pytest.mark.parametrize("t", [-0.3, -0.05, 0.0, 0.004, 0.3, 2.0, 5.0])
def test_h_against_direct_convolution(a, t):
    """h(a; t) = int_0^inf e^{-a u} G_sigma(t - u) du by adaptive quadrature."""
    g = lambda u: math.exp(-(t - u) ** 2 / (2 * SIG * SIG)) / (SIG * math.sqrt(2 * math.pi))
    lo, hi = max(0.0, t - 12 * SIG), max(0.0, t + 12 * SIG)
    re = integrate.quad(lambda u: (np.exp(-a * u)).real * g(u), lo, hi, epsabs=1e-16, epsrel=1e-13, limit=200)[0]
    im = integrate.quad(lambda u: (np.exp(-a * u)).imag * g(u), lo, hi, epsabs=1e-16, epsrel=1e-13, limit=200)[0]
    got = h(a, t)[0]
    ref = complex(re, im)
    assert abs(got - ref) <= 1e-11 * max(abs(ref), 1e-30) + 1e-300


@pytest.mark.parametrize("a", [2.4, complex(2.4, -0.3)])
def test_h_sigma_to_zero_and_unit_integral(a):
    t = np.array([0.5, 1.0, 3.0])
    assert np.allclose(h(a, t, sigma=1e-4), np.exp(-a * t), rtol=1e-10)
    re = integrate.quad(lambda v: h(a, v)[0].real, -1, 40, limit=400, epsabs=1e-14)[0]
    im = integrate.quad(lambda v: h(a, v)[0].imag, -1, 40, limit=400, epsabs=1e-14)[0]
    assert abs(complex(re, im) - 1 / a) < 1e-10


def _one_point():
    kin = synth.td4_phase_space(1, seed=5)
    return [torch.tensor(kin[i]) for i in range(5)]


@pytest.mark.parametrize("xy", [(0.004, 0.006), (0.2, -0.3), (0.0, 0.0)])
def test_time_integral_of_rate_equals_normalization_formula(xy):
    th = TH.copy()
    th[-2:] = xy
    kin = _one_point()
    tht = torch.tensor(th)

    def rate(t):
        ev = torch.stack([k.reshape(1) for k in kin] + [torch.tensor([t])])
        with torch.no_grad():
            return float(MODEL.rate(tht, ev)[0])
    val = integrate.quad(rate, -1.0, 30.0, limit=500, epsabs=1e-15, epsrel=1e-12, points=[0.0, 0.5])[0]
    with torch.no_grad():
        ref = float(MODEL.integrated_rate(tht, torch.stack([k.reshape(1) for k in kin]))[0])
    assert abs(val / ref - 1) < 1e-9


def test_no_mixing_factorizes():
    """x = y = 0: R(x, t) = |A(x)|^2 h(Gamma; t)."""
    th = TH.copy()
    th[-2:] = 0.0
    ev = synth.td4_events(200, seed=6)
    with torch.no_grad():
        r = MODEL.rate(torch.tensor(th), torch.tensor(ev)).numpy()
        A, _ = MODEL.amplitudes(torch.tensor(th), MODEL.basis(torch.tensor(ev[:5])))
    hg = h(1 / synth.TD4_TAU, ev[5]).real
    assert np.allclose(r, (A.abs() ** 2).numpy() * hg, rtol=1e-12)


def test_angular_functions_orthogonal():
    """The six helicity structures are orthogonal on (c12, c34, phi)."""
    x, w = np.polynomial.legendre.leggauss(12)
    pf = np.linspace(-math.pi, math.pi, 33)[:-1] + math.pi / 32
    C12, C34, PHI = np.meshgrid(x, x, pf, indexing="ij")
    W = (w[:, None, None] * w[None, :, None]) * (2 * math.pi / 32)
    tens = [OT.TD4.omega(k, torch.tensor(C12), torch.tensor(C34), torch.tensor(PHI)).numpy() for k in range(6)]
    gram = np.array([[np.sum(W * a * np.conj(b)) for b in tens] for a in tens])
    off = gram - np.diag(np.diag(gram))
    assert np.abs(off).max() < 1e-12 * np.abs(np.diag(gram)).max()
    assert np.abs(gram[0, 0] - 8 * math.pi) < 1e-12


def test_lineshape_pole():
    from synth.td4 import TD4_R34
    L, m0, w0 = TD4_R34[1]
    amp = MODEL.pair_amp(torch.tensor([m0]), 0.140, 0.140, (L, m0, w0))
    assert abs(amp[0] - 1j / (m0 * w0)) < 1e-12 / (m0 * w0)


def test_autograd_vs_central_fd():
    ev = synth.td4_events(1500, seed=7)
    mc = synth.td4_phase_space(3000, seed=8)
    th = TH * (1 + 0.05 * np.sin(np.arange(TH.size)))
    th[-2:] = [0.05, -0.04]
    _, g = OT.nll_grad(th, ev, mc, DESC)
    fd = common.central_fd(lambda q: OT.nll(q, ev, mc, DESC), th, rel_step=1e-6)
    tol = 1e-6 * np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max())
    assert (np.abs(g - fd) <= tol).all(), np.abs(g - fd) / tol


def test_split_model_equals_shared_basis_with_zero_coefficients():
    """Twenty distinct basis functions, ten in A and ten in Abar, give the NLL
    and gradient of the same twenty functions entering both sums, with the
    coefficients of the non-members set to zero (the split layout lists A's
    members, then Abar's, then x and y)."""
    ds, ths = synth.td4_split_desc(), synth.td4_split_truth()
    ths = ths * (1 + 0.05 * np.cos(np.arange(ths.size)))
    ths[-2:] = [0.04, -0.03]
    db = dict(ds, amps=[a[:3] for a in ds["amps"]])
    K = len(ds["amps"])
    in_a = [k for k, a in enumerate(ds["amps"]) if a[3] == "A"]
    in_b = [k for k, a in enumerate(ds["amps"]) if a[3] == "Abar"]
    thb = np.zeros(4 * K + 2)
    for j, k in enumerate(in_a):
        thb[2 * k:2 * k + 2] = ths[2 * j:2 * j + 2]
    for j, k in enumerate(in_b):
        thb[2 * K + 2 * k:2 * K + 2 * k + 2] = ths[2 * len(in_a) + 2 * j:2 * len(in_a) + 2 * j + 2]
    thb[-2:] = ths[-2:]
    ev = synth.td4_events(400, seed=17)
    mc = synth.td4_phase_space(2000, seed=18)
    vs, gs = OT.nll_grad(ths, ev, mc, ds)
    vb, gb = OT.nll_grad(thb, ev, mc, db)
    assert abs(vs - vb) <= 1e-13 * abs(vb)
    gmap = np.r_[np.concatenate([gb[2 * k:2 * k + 2] for k in in_a]),
                 np.concatenate([gb[2 * K + 2 * k:2 * K + 2 * k + 2] for k in in_b]), gb[-2:]]
    assert np.allclose(gs, gmap, rtol=1e-12, atol=1e-12 * np.abs(gmap).max())


def test_phase_space_marginal():
    """m12 marginal of the phase-space sample against 1-D quadrature of the
    phase-space density (chi-square over 20 bins)."""
    M, m1, m2, m3, m4 = synth.TD4_MASSES
    ps = synth.td4_phase_space(200_000, seed=9)
    q = lambda m, a, b: math.sqrt(max((m * m - (a + b) ** 2) * (m * m - (a - b) ** 2), 0.0)) / (2 * m)
    dens = lambda m12: integrate.quad(lambda m34: q(M, m12, m34) * q(m12, m1, m2) * q(m34, m3, m4),
                                      m3 + m4, M - m12, limit=200)[0]
    edges = np.linspace(m1 + m2, M - m3 - m4, 21)
    probs = np.array([integrate.quad(dens, a, b, limit=200)[0] for a, b in zip(edges[:-1], edges[1:])])
    probs /= probs.sum()
    counts, _ = np.histogram(ps[0], edges)
    exp = probs * ps.shape[1]
    keep = exp > 20
    chi2 = (((counts - exp) ** 2) / exp)[keep].sum()
    assert chi2 < 50, chi2  # 19 dof


SMALL = synth.td4_desc(r12=((0, 0.0, 0.0), (0, 1.370, 0.350)))
SMALL["amps"] = [[0, 0, 0], [0, 1, 1], [0, 2, 0], [1, 1, 1], [1, 0, 0], [1, 2, 0]]
SMALL_TH = np.array([0.25, 0.0, -0.12, 0.20, 0.05, 0.09, 0.10, -0.04, 0.3, 0.22, -0.08, 0.11,
                     1.0, 0.0, 0.8, 0.45, 0.35, -0.2, -0.3, 0.55, 1.6, -0.4, 0.45, 0.3, 0.004, 0.006])


def test_generator_time_distribution_without_mixing():
    """x = y = 0: R(x, t) = |A(x)|^2 e^{-Gt}, so t_true ~ Exp(G) for every point and
    the measured t (plus a zero-mean Gaussian) has mean tau and variance tau^2 + sigma^2."""
    th = SMALL_TH.copy()
    th[-2:] = 0.0
    ev = OT.generate(th, SMALL, 4000, seed=11)
    n = ev.shape[1]
    tau, s = synth.TD4_TAU, synth.TD4_SIGMA_T
    sd = math.sqrt(tau * tau + s * s)
    assert abs(ev[5].mean() - tau) < 4 * sd / math.sqrt(n)
    assert abs(ev[5].var() / (sd * sd) - 1) < 4 * math.sqrt(8.0 / n)  # exponential kurtosis 9


def test_generator_kinematics_follow_the_amplitude():
    """The m34 histogram of generated events against a phase-space sample
    reweighted by the time-integrated rate (chi-square over 12 bins)."""
    ev = OT.generate(SMALL_TH, SMALL, 4000, seed=12)
    ps = synth.td4_phase_space(200_000, seed=13)
    model = OT.TD4(SMALL)
    with torch.no_grad():
        w = model.integrated_rate(torch.tensor(SMALL_TH), torch.tensor(ps)).numpy()
    edges = np.quantile(ev[1], np.linspace(0, 1, 13))
    edges[0], edges[-1] = 0.0, 10.0
    counts, _ = np.histogram(ev[1], edges)
    prob, _ = np.histogram(ps[1], edges, weights=w)
    exp = prob / prob.sum() * ev.shape[1]
    chi2 = (((counts - exp) ** 2) / exp).sum()
    assert chi2 < 35, chi2  # 11 dof


# ------------------------------------------------ per-event generator (the device's definition)
@pytest.fixture(scope="module")
def per_event_toys():
    ev, W, above = OT.generate_events(SMALL_TH, SMALL, 4000, seed=14)
    th0 = SMALL_TH.copy()
    th0[-2:] = 0.0
    ev0, _, above0 = OT.generate_events(th0, SMALL, 4000, seed=15)
    return ev, W, above, ev0, above0


def test_per_event_generator_time_without_mixing(per_event_toys):
    _, _, _, ev0, above0 = per_event_toys
    assert above0 == 0 and np.isfinite(ev0).all()
    n = ev0.shape[1]
    tau, s = synth.TD4_TAU, synth.TD4_SIGMA_T
    sd = math.sqrt(tau * tau + s * s)
    assert abs(ev0[5].mean() - tau) < 4 * sd / math.sqrt(n)
    assert abs(ev0[5].var() / (sd * sd) - 1) < 4 * math.sqrt(8.0 / n)


def test_per_event_generator_kinematics(per_event_toys):
    ev, W, above, _, _ = per_event_toys
    assert above == 0 and np.isfinite(ev).all()
    ps = synth.td4_phase_space(200_000, seed=16)
    model = OT.TD4(SMALL)
    with torch.no_grad():
        w = model.integrated_rate(torch.tensor(SMALL_TH), torch.tensor(ps)).numpy()
    for row in (0, 1, 2):
        edges = np.quantile(ev[row], np.linspace(0, 1, 13))
        edges[0], edges[-1] = -10.0, 10.0
        counts, _ = np.histogram(ev[row], edges)
        prob, _ = np.histogram(ps[row], edges, weights=w)
        exp = prob / prob.sum() * ev.shape[1]
        chi2 = (((counts - exp) ** 2) / exp).sum()
        assert chi2 < 35, (row, chi2)  # 11 dof


def test_per_event_generator_prefix(per_event_toys):
    ev, W, _, _, _ = per_event_toys
    head, W2, _ = OT.generate_events(SMALL_TH, SMALL, 200, seed=14, W=W)
    assert W2 == W and np.array_equal(head, ev[:, :200])
