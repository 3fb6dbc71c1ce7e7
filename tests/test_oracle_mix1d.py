"""Pins of the 1-D mixture oracle against quadrature, textbook MLEs,
invariances and finite differences (CPU only)."""
import math
import os

import mpmath
import numpy as np
import pytest
import torch
from scipy import integrate, optimize

import synth
from oracle import common, mix1d

TRUTH = np.array(synth.CONFIG0_TRUTH)
D0 = mix1d.config0_desc()

# a four-component model on a positive range exercising argus and bw
D4 = {"kind": "mix1d", "lo": 5.20, "hi": 5.30, "n_params": 10,
      "components": [{"type": "argus", "params": [0, 1]},
                     {"type": "bw", "params": [2, 3]},
                     {"type": "gauss", "params": [4, 5]},
                     {"type": "exp", "params": [6]}],
      "fracs": [7, 8, 9]}
TH4 = np.array([5.29, -20.0, 5.2795, 0.004, 5.28, 0.003, -3.0, 0.4, 0.2, 0.25])


def dens(theta, desc):
    th = common.as_t(theta)

    def f(x):
        with torch.no_grad():
            return float(mix1d.density(th, torch.tensor([x], dtype=torch.float64), desc)[0])
    return f


@pytest.mark.parametrize("desc,theta,points", [
    (D0, TRUTH, [0.2]),
    (D0, [1.5, 0.3, 0.4, 0.25], [1.5]),
    (D0, [-9.0, 2.0, 0.0, 0.5], [-9.0]),
    (D4, TH4, [5.28, 5.2795]),
])
def test_density_integrates_to_one(desc, theta, points):
    lo, hi = desc["lo"], desc["hi"]
    val, err = integrate.quad(dens(theta, desc), lo, hi, points=points, limit=500,
                              epsabs=1e-13, epsrel=1e-13)
    assert abs(val - 1.0) < 1e-10, (val, err)


@pytest.mark.parametrize("kind,p,lo,hi", [
    ("gauss", (0.2, 1.1), -10, 10), ("gauss", (9.5, 0.7), -10, 10),
    ("exp", (-0.3,), -10, 10), ("exp", (2e-13,), -10, 10), ("exp", (1.7,), -1, 2),
    ("argus", (5.29, -20.0), 5.2, 5.3), ("argus", (5.29, -3.0), 0.0, 5.25),
    ("bw", (5.2795, 0.004), 5.2, 5.3), ("bw", (1.0, 0.5), -2, 2),
])
def test_component_integral_vs_mpmath(kind, p, lo, hi):
    """Closed-form integrals against 30-digit adaptive quadrature of the shape."""
    mpmath.mp.dps = 30
    pt = [torch.tensor(v, dtype=torch.float64) for v in p]
    closed = float(mix1d.component_integral(kind, pt, lo, hi))

    def shape(x):
        xt = torch.tensor([float(x)], dtype=torch.float64)
        return mpmath.mpf(float(mix1d.component_shape(kind, xt, pt)[0]))
    brk = [lo, hi]
    if kind in ("gauss", "bw"):
        brk = sorted({lo, hi, min(max(p[0], lo), hi)})
    if kind == "argus":
        brk = sorted({lo, min(hi, p[0]), hi})
    q = mpmath.quad(shape, brk, maxdegree=10)
    assert abs(closed - float(q)) <= 1e-11 * abs(float(q))


def test_shape_definitions():
    """Defining properties of each shape: Gaussian at mu +- sigma is e^-1/2 of
    the peak; exp ratio over unit step is e^tau; BW is half maximum at
    m0 +- gamma/2 (full width gamma); argus vanishes at and above m0."""
    t = lambda *v: [torch.tensor(a, dtype=torch.float64) for a in v]
    x = torch.tensor([0.2 - 1.1, 0.2, 0.2 + 1.1], dtype=torch.float64)
    g = mix1d.component_shape("gauss", x, t(0.2, 1.1))
    assert abs(float(g[0] / g[1]) - math.exp(-0.5)) < 1e-15 and abs(float(g[2] / g[1]) - math.exp(-0.5)) < 1e-15
    e = mix1d.component_shape("exp", torch.tensor([1.0, 2.0], dtype=torch.float64), t(-0.3))
    assert abs(float(e[1] / e[0]) - math.exp(-0.3)) < 1e-15
    b = mix1d.component_shape("bw", torch.tensor([5.0 - 0.02, 5.0, 5.0 + 0.02], dtype=torch.float64), t(5.0, 0.04))
    assert abs(float(b[0] / b[1]) - 0.5) < 1e-12 and abs(float(b[2] / b[1]) - 0.5) < 1e-12
    a = mix1d.component_shape("argus", torch.tensor([5.29, 5.295, 5.0], dtype=torch.float64), t(5.29, -20.0))
    assert float(a[0]) == 0.0 and float(a[1]) == 0.0 and float(a[2]) > 0


def test_brute_force_ten_events():
    """50-digit NLL on 10 events with component integrals by quadrature."""
    mpmath.mp.dps = 50
    x = synth.mix1d_events(10, seed=99)
    mu, sg, tau, f = (mpmath.mpf(v) for v in TRUTH)
    g = lambda v: mpmath.exp(-(v - mu) ** 2 / (2 * sg ** 2))
    e = lambda v: mpmath.exp(tau * v)
    ng = mpmath.quad(g, [-10, mu, 10])
    ne = mpmath.quad(e, [-10, 10])
    ref = -sum(mpmath.log(f * g(mpmath.mpf(v)) / ng + (1 - f) * e(mpmath.mpf(v)) / ne) for v in x)
    got = mix1d.nll(TRUTH, x, D0)
    assert abs(got - float(ref)) <= 1e-14 * abs(float(ref))


def test_gaussian_mle_is_stationary():
    """f = 1: the MLE of a (negligibly truncated) Gaussian is the sample mean
    and the biased sample standard deviation; the gradient vanishes there."""
    x = 0.2 + 1.1 * np.random.default_rng(5).standard_normal(20000)
    mu, sd = x.mean(), x.std()
    _, g = mix1d.nll_grad([mu, sd, -0.3, 1.0], x, D0)
    scale = x.size / sd
    assert abs(g[0]) < 1e-9 * scale and abs(g[1]) < 1e-9 * scale
    assert abs(g[2]) < 1e-12  # tau drops out when f = 1


def test_exponential_mle_is_stationary():
    """f = 0: the truncated-exponential MLE solves mean(x) = E_tau[x]; solve
    that moment equation with quadrature moments and check the gradient."""
    x = synth.mix1d_events(5000, theta=(0.0, 1.0, -0.3, 0.0))
    xbar = x.mean()

    def mean_tau(tau):
        num = integrate.quad(lambda v: v * math.exp(tau * v), -10, 10, epsabs=1e-15, epsrel=1e-13)[0]
        den = integrate.quad(lambda v: math.exp(tau * v), -10, 10, epsabs=1e-15, epsrel=1e-13)[0]
        return num / den
    tau_hat = optimize.brentq(lambda t: mean_tau(t) - xbar, -2.0, -0.01, xtol=1e-15)
    _, g = mix1d.nll_grad([0.0, 1.0, tau_hat, 0.0], x, D0)
    assert abs(g[2]) < 1e-7 * x.size


def test_translation_invariance():
    x = synth.mix1d_events(3000)
    c = 3.75
    d = mix1d.config0_desc(-10 + c, 10 + c)
    a = mix1d.nll(TRUTH, x, D0)
    b = mix1d.nll([TRUTH[0] + c, TRUTH[1], TRUTH[2], TRUTH[3]], x + c, d)
    assert abs(a - b) < 1e-12 * abs(a)


@pytest.mark.parametrize("desc,theta", [(D0, TRUTH * np.array([1.3, 0.9, 1.2, 0.95])), (D4, TH4)])
def test_autograd_vs_central_fd(desc, theta):
    lo, hi = desc["lo"], desc["hi"]
    if desc is D0:
        x = synth.mix1d_events(4000)
    else:
        # keep events away from the argus endpoint m0, where the shape has a
        # square-root kink that a finite difference cannot straddle
        x = np.linspace(lo + 1e-4, hi - 1e-4, 2000)
        x = x[np.abs(x - theta[0]) > 1e-3]
    _, g = mix1d.nll_grad(theta, x, desc)
    # D4 has widths of a few 1e-3 at positions ~5.3: a relative step of 1e-6
    # would leave an O((h/width)^2) ~ 1e-6 truncation error, so use 1e-7 there
    step = 1e-6 if desc is D0 else 1e-7
    fd = common.central_fd(lambda t: mix1d.nll(t, x, desc), theta, rel_step=step)
    tol = 1e-6 * np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max())
    assert (np.abs(g - fd) <= tol).all(), (g, fd)


@pytest.mark.slow
def test_pulls_unit_width():
    """Fits of 1000 toys of 100k events each, drawn at the truth by the input
    sampler (not by this oracle's density): the pulls (fit - truth)/error of
    the four parameters have mean within 0.1 (3.2 statistical standard
    deviations) and width within 0.05 of one (2.2 deviations).  A dropped
    normalization term, a wrong sign in a component or a Hessian off by a
    factor would shift the means or scale the widths far beyond that."""
    import multiprocessing as mp
    n_toys = 1000
    jobs = [(100_000, 5150, t, TRUTH) for t in range(n_toys)]
    with mp.get_context("spawn").Pool(min(8, os.cpu_count() or 1)) as pool:
        pulls = np.array(pool.map(mix1d.toy_pull, jobs, chunksize=8))
    mean, width = pulls.mean(0), pulls.std(0, ddof=1)
    print("pull means", mean, "widths", width)
    assert (np.abs(mean) < 0.1).all(), mean
    assert (np.abs(width - 1.0) < 0.05).all(), width


# ------------------------------------------------ extended and binned data
def _ext(desc, idx):
    return dict(desc, n_params=idx + 1, **{"yield": idx})


def test_extended_yield_mle_is_the_event_count():
    """d/dnu (nu - N ln nu) vanishes at nu = N, and the extended NLL exceeds
    the plain one by exactly that term, which is smallest there."""
    d = mix1d.config0_desc()
    de = _ext(d, 4)
    x = synth.mix1d_events(500, seed=3)
    th = np.array(list(synth.CONFIG0_TRUTH) + [500.0])
    v, g = mix1d.nll_grad(th, x, de)
    assert abs(g[4]) < 1e-12
    v0 = mix1d.nll(th[:4], x, d)
    assert abs((v - v0) - (500.0 - 500.0 * math.log(500.0))) < 1e-9
    for s in (0.999, 1.001):
        assert mix1d.nll(np.r_[th[:4], 500.0 * s], x, de) > v


def test_binned_poisson_with_events_at_bin_centres():
    """Events placed at bin centres (several per bin for some bins): the
    binned Poisson NLL equals N Delta sum_b P_b - N ln(N Delta) plus the
    unbinned NLL of those events."""
    d = mix1d.config0_desc()
    nb = 400
    rng = np.random.default_rng(4)
    counts = np.zeros(nb)
    idx = rng.integers(0, nb, 300)
    np.add.at(counts, idx, 1.0)
    x = mix1d.bin_centres(d, nb)[idx]
    th = np.array(synth.CONFIG0_TRUTH) * np.array([1.1, 0.95, 1.05, 0.97])
    N = counts.sum()
    delta = 20.0 / nb
    with torch.no_grad():
        psum = float(mix1d.density(common.as_t(th), common.as_t(mix1d.bin_centres(d, nb)), d).sum())
    expect = N * delta * psum - N * math.log(N * delta) + mix1d.nll(th, x, d)
    v, _ = mix1d.binned_value_grad(th, counts, d, "poisson")
    assert abs(v - expect) < 1e-9 * abs(expect)


def test_extended_binned_yield_mle():
    """Extended binned Poisson: d/dnu vanishes at nu = W / (Delta sum_b P_b)."""
    d = _ext(mix1d.config0_desc(), 4)
    nb = 250
    counts = np.histogram(synth.mix1d_events(4000, seed=5), bins=nb, range=(-10.0, 10.0))[0].astype(np.float64)
    th4 = np.array(synth.CONFIG0_TRUTH)
    with torch.no_grad():
        psum = float(mix1d.density(common.as_t(th4), common.as_t(mix1d.bin_centres(d, nb)), d).sum())
    nu = counts.sum() / ((20.0 / nb) * psum)
    _, g = mix1d.binned_value_grad(np.r_[th4, nu], counts, d, "poisson")
    assert abs(g[4]) < 1e-10


def test_chi2_neyman_value_at_nonzero_residuals():
    """Hand-computed Neyman chi^2 on four bins of a flat density (exponential
    with tau = 0 on [0, 4]: P = 1/4, so nu_b = N / 4 at every bin).  Counts
    (5, 0, 2, 4): the empty bin is left out, each residual is divided by the
    observed count.  Extended, nu = 12 (nu_b = 3):
        (5-3)^2/5 + (2-3)^2/2 + (4-3)^2/4 = 0.8 + 0.5 + 0.25 = 1.55,
    where dividing by nu_b (Pearson) would give 2 over the filled bins.
    d/dnu = -1/2 sum (n_b - nu_b)/n_b = -0.075; d/dtau at tau = 0 follows from
    d nu_b/dtau = nu_b (x_b - 2): -2 sum (n_b - nu_b)/n_b nu_b (x_b - 2) = 2.85.
    Not extended, N = 11 (nu_b = 2.75): 2.25^2/5 + 0.75^2/2 + 1.25^2/4 = 1.684375.
    The Poisson NLL of the extended case is 12 - 11 ln 3."""
    flat = {"kind": "mix1d", "lo": 0.0, "hi": 4.0, "n_params": 2,
            "components": [{"type": "exp", "params": [0]}], "fracs": [], "yield": 1}
    counts = [5.0, 0.0, 2.0, 4.0]
    v, g = mix1d.binned_value_grad(np.array([0.0, 12.0]), counts, flat, "chi2")
    assert abs(v - 1.55) < 1e-15 and abs(g[0] - 2.85) < 1e-14 and abs(g[1] + 0.075) < 1e-15, (v, g)
    plain = dict(flat, n_params=1)
    plain.pop("yield")
    v, _ = mix1d.binned_value_grad(np.array([0.0]), counts, plain, "chi2")
    assert abs(v - 1.684375) < 1e-15, v
    v, _ = mix1d.binned_value_grad(np.array([0.0, 12.0]), counts, flat, "poisson")
    assert abs(v - (12.0 - 11.0 * math.log(3.0))) < 1e-14, v


def test_chi2_vanishes_at_the_expected_counts():
    d = _ext(mix1d.config0_desc(), 4)
    nb = 64
    th = np.r_[np.array(synth.CONFIG0_TRUTH), 1.0e4]
    with torch.no_grad():
        p = mix1d.density(common.as_t(th), common.as_t(mix1d.bin_centres(d, nb)), d).numpy()
    counts = th[4] * (20.0 / nb) * p
    v, g = mix1d.binned_value_grad(th, counts, d, "chi2")
    assert v < 1e-20 and np.max(np.abs(g)) < 1e-12


@pytest.mark.parametrize("stat", ["poisson", "chi2"])
@pytest.mark.parametrize("ext", [False, True])
def test_binned_autograd_vs_central_fd(stat, ext):
    d = mix1d.config0_desc()
    if ext:
        d = _ext(d, 4)
    nb = 120
    counts = np.histogram(synth.mix1d_events(3000, seed=6), bins=nb, range=(-10.0, 10.0))[0].astype(np.float64)
    th = np.array(synth.CONFIG0_TRUTH) * np.array([1.1, 0.95, 1.05, 0.97])
    if ext:
        th = np.r_[th, 2900.0]
    _, g = mix1d.binned_value_grad(th, counts, d, stat)
    fd = common.central_fd(lambda t: mix1d.binned_value_grad(t, counts, d, stat)[0], th, rel_step=1e-6)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-6 * np.max(np.abs(fd)))
