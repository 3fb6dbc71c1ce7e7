"""Oracle for one-observable mixture models (the paper's basic and combination
PDFs, Sec. 1 and Fig. 1: components added with fractions into a final PDF).

Model description (dict)::

    {"kind": "mix1d", "lo": -10, "hi": 10, "n_params": 4,
     "components": [{"type": "gauss", "params": [0, 1]},
                    {"type": "exp",   "params": [2]}],
     "fracs": [3]}

Integers are indices into the parameter vector theta.  Component types and
their parameters:

* gauss  (mu, sigma):   exp(-(x-mu)^2 / (2 sigma^2))
* exp    (tau):         exp(tau x)
* argus  (m0, c):       x sqrt(1 - x^2/m0^2) exp(c (1 - x^2/m0^2)), x < m0; 0 above
* bw     (m0, gamma):   1 / ((x - m0)^2 + gamma^2/4)   (non-relativistic)

Each component is divided by its integral over [lo, hi]; with K components
and K-1 fractions f_k the density is
P(x) = sum_{k<K-1} f_k c_k(x)/N_k + (1 - sum f) c_{K-1}(x)/N_{K-1},
so the overall normalization I is 1 and NLL = -sum_i ln P(x_i).

Integrals used here (each a closed form):
* gauss: sigma sqrt(pi/2) [erf((hi-mu)/(sigma sqrt2)) - erf((lo-mu)/(sigma sqrt2))]
* exp:   exp(tau lo) expm1(tau (hi-lo)) / tau, and hi-lo at tau = 0
* argus: with w = 1 - x^2/m0^2, x dx = -(m0^2/2) dw, the integral is
         (m0^2/2) int_{w(hi)}^{w(lo)} w^(1/2) e^(c w) dw, a regularized lower
         incomplete gamma function P(3/2, .) for c < 0
* bw:    (2/gamma) [atan(2(hi-m0)/gamma) - atan(2(lo-m0)/gamma)]

Extended likelihood (optional "yield": i): with nu = theta[i] expected events
the NLL of N events gains nu - N ln nu.  Binned data (the paper's binned
DataSet): counts n_b of uniform bins on [lo, hi], expected nu_b = N Delta
P(x_b) at the bin centres (N = nu, or the total count when not extended);
Poisson NLL sum_b (nu_b - n_b ln nu_b) without the constant ln n_b!, or chi^2
over the filled bins.

Pins (tests/test_oracle_mix1d.py): adaptive quadrature of every normalized
component and of the mixture; mpmath brute force on 10 events with
normalizations taken by quadrature; the Gaussian maximum-likelihood
estimate (sample mean and biased variance) is a stationary point; the
truncated-exponential MLE from a quadrature moment equation is a stationary
point; translation invariance; autograd against central differences;
extended: the yield's MLE is N; binned: a histogram with one event at each
of N bin centres reproduces the unbinned NLL up to the closed-form terms
N Delta sum_b P_b - N ln(N Delta), the extended Poisson yield MLE is
W / (Delta sum_b P_b), chi^2 vanishes with zero gradient when the counts are
the expected counts.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .common import as_t, fsum, nll_value

_KINDS = {"gauss": 2, "exp": 1, "argus": 2, "bw": 2}


def parse(desc: dict):
    if desc.get("kind") != "mix1d":
        raise ValueError("not a mix1d model")
    lo, hi = float(desc["lo"]), float(desc["hi"])
    if not hi > lo:
        raise ValueError("empty range")
    comps = []
    for c in desc["components"]:
        t = c["type"]
        if t not in _KINDS or len(c["params"]) != _KINDS[t]:
            raise ValueError(f"bad component {c}")
        if t == "argus" and lo < 0:
            raise ValueError("argus needs lo >= 0")
        comps.append((t, [int(i) for i in c["params"]]))
    fracs = [int(i) for i in desc.get("fracs", [])]
    if len(fracs) != len(comps) - 1:
        raise ValueError("need K-1 fractions")
    return lo, hi, comps, fracs


def component_shape(kind: str, x: torch.Tensor, p) -> torch.Tensor:
    """Unnormalized component value at x."""
    if kind == "gauss":
        mu, sigma = p
        return torch.exp(-((x - mu) ** 2) / (2.0 * sigma ** 2))
    if kind == "exp":
        (tau,) = p
        return torch.exp(tau * x)
    if kind == "argus":
        m0, c = p
        w = 1.0 - (x / m0) ** 2
        inside = w > 0
        wc = torch.where(inside, w, torch.ones_like(w))
        val = x * torch.sqrt(wc) * torch.exp(c * wc)
        return torch.where(inside, val, torch.zeros_like(val))
    if kind == "bw":
        m0, gam = p
        return 1.0 / ((x - m0) ** 2 + gam ** 2 / 4.0)
    raise ValueError(kind)


def component_integral(kind: str, p, lo: float, hi: float) -> torch.Tensor:
    """Integral of the unnormalized component over [lo, hi]."""
    if kind == "gauss":
        mu, sigma = p
        r2 = math.sqrt(2.0)
        return sigma * math.sqrt(math.pi / 2.0) * (
            torch.erf((hi - mu) / (sigma * r2)) - torch.erf((lo - mu) / (sigma * r2)))
    if kind == "exp":
        (tau,) = p
        width = hi - lo
        if abs(float(torch.as_tensor(tau).detach())) < 1e-12:
            return width * (1.0 + 0.5 * tau * (hi + lo))
        return torch.exp(tau * lo) * torch.expm1(tau * width) / tau
    if kind == "argus":
        m0, c = p
        if float(torch.as_tensor(c).detach()) >= 0.0:
            raise ValueError("argus needs c < 0")
        k = -c
        w_lo = 1.0 - (lo / m0) ** 2
        w_hi = torch.clamp(1.0 - (hi / m0) ** 2, min=0.0)
        w_lo = torch.clamp(w_lo, min=0.0)
        g32 = math.gamma(1.5)

        def lower(wv):
            # int_0^W w^(1/2) e^(-k w) dw = k^(-3/2) Gamma(3/2) P(3/2, k W)
            return k ** -1.5 * g32 * torch.special.gammainc(
                torch.tensor(1.5, dtype=torch.float64), k * wv)

        return 0.5 * m0 ** 2 * (lower(w_lo) - lower(w_hi))
    if kind == "bw":
        m0, gam = p
        return (2.0 / gam) * (torch.atan(2.0 * (hi - m0) / gam) - torch.atan(2.0 * (lo - m0) / gam))
    raise ValueError(kind)


def density(theta: torch.Tensor, x: torch.Tensor, desc: dict) -> torch.Tensor:
    """Normalized mixture density P(x | theta) on [lo, hi]."""
    lo, hi, comps, fracs = parse(desc)
    total = torch.zeros_like(x)
    rest = torch.ones((), dtype=torch.float64)
    for k, (kind, idx) in enumerate(comps):
        p = [theta[i] for i in idx]
        term = component_shape(kind, x, p) / component_integral(kind, p, lo, hi)
        if k < len(comps) - 1:
            f = theta[fracs[k]]
            rest = rest - f
            total = total + f * term
        else:
            total = total + rest * term
    return total


def yield_index(desc: dict):
    """Index of the expected-yield parameter of an extended model, or None."""
    return int(desc["yield"]) if "yield" in desc else None


def extended_term(theta, n: int, desc: dict):
    """nu - N ln nu for an extended model (Poisson probability of observing N
    events when nu are expected, up to the constant ln N!), else 0."""
    i = yield_index(desc)
    if i is None:
        return 0.0
    nu = theta[i]
    return nu - n * torch.log(nu) if isinstance(nu, torch.Tensor) else nu - n * math.log(nu)


def nll(theta, x, desc: dict) -> float:
    """NLL value, events summed exactly rounded (I = 1 by construction); an
    extended model adds nu - N ln nu."""
    with torch.no_grad():
        p = density(as_t(theta), as_t(x), desc)
        v = nll_value(torch.log(p), int(np.size(x)), 0.0)
    return v + float(extended_term(np.asarray(theta, dtype=np.float64), int(np.size(x)), desc))


def nll_grad(theta, x, desc: dict):
    """(NLL, dNLL/dtheta) with the gradient from autograd."""
    th = as_t(theta, requires_grad=True)
    p = density(th, as_t(x), desc)
    lp = torch.log(p)
    loss = -lp.sum() + extended_term(th, int(np.size(x)), desc)
    loss.backward()
    v = nll_value(lp.detach(), int(np.size(x)), 0.0)
    v += float(extended_term(np.asarray(theta, dtype=np.float64), int(np.size(x)), desc))
    return v, th.grad.numpy().copy()


def bin_centres(desc: dict, n_bins: int) -> np.ndarray:
    lo, hi, _, _ = parse(desc)
    delta = (hi - lo) / n_bins
    return lo + (np.arange(n_bins) + 0.5) * delta


def binned_tensor(theta: torch.Tensor, counts, desc: dict, stat: str) -> torch.Tensor:
    """Binned statistic of histogram counts on n_bins uniform bins over
    [lo, hi]: expected counts nu_b = N Delta P(x_b) at the bin centres, N the
    yield of an extended model or the total count; "poisson":
    sum_b (nu_b - n_b ln nu_b); "chi2": sum over n_b > 0 of (n_b - nu_b)^2 / n_b."""
    lo, hi, _, _ = parse(desc)
    n = as_t(np.asarray(counts, dtype=np.float64))
    nb = n.numel()
    delta = (hi - lo) / nb
    p = density(theta, as_t(bin_centres(desc, nb)), desc)
    i = yield_index(desc)
    N = theta[i] if i is not None else n.sum()
    nu = N * delta * p
    if stat == "poisson":
        filled = n > 0
        return nu.sum() - (n[filled] * torch.log(nu[filled])).sum()
    filled = n > 0
    return ((n[filled] - nu[filled]) ** 2 / n[filled]).sum()


def binned_value_grad(theta, counts, desc: dict, stat: str):
    """(statistic, gradient by autograd)."""
    th = as_t(theta, requires_grad=True)
    v = binned_tensor(th, counts, desc, stat)
    v.backward()
    return float(v.detach()), th.grad.numpy().copy()


def nll_tensor(theta: torch.Tensor, x: torch.Tensor, desc: dict) -> torch.Tensor:
    """The NLL as a differentiable tensor (event sum in plain float64)."""
    return -torch.log(density(theta, x, desc)).sum() + extended_term(theta, int(x.numel()), desc)


def fit(x, theta0, desc: dict, bounds=None):
    """Maximum-likelihood fit of events x: scipy's L-BFGS-B on this module's
    NLL and autograd gradient, then errors sqrt(diag(H^-1)) from the autograd
    Hessian H of the NLL at the minimum (an NLL has error definition 1/2, so
    H^-1 is the covariance).  Returns (theta, errors, nll)."""
    from scipy import optimize
    res = optimize.minimize(lambda t: nll_grad(t, x, desc), np.asarray(theta0, dtype=np.float64), jac=True,
                            method="L-BFGS-B", bounds=bounds, options={"ftol": 1e-15, "gtol": 1e-9, "maxiter": 2000})
    xt = as_t(x)
    h = torch.autograd.functional.hessian(lambda t: nll_tensor(t, xt, desc), as_t(res.x)).numpy()
    cov = np.linalg.inv(0.5 * (h + h.T))
    return res.x, np.sqrt(np.diag(cov)), float(res.fun)


CONFIG0_BOUNDS = [(-5.0, 5.0), (0.1, 5.0), (-3.0, 3.0), (0.01, 0.99)]


def toy_pull(args):
    """Pull (fitted - truth) / error of one config-0 toy: n events drawn at
    the truth by the input sampler under key (seed, fit), fitted from the
    truth.  args = (n, seed, fit, truth); for pull studies in worker
    processes."""
    import synth
    n, seed, fit_index, truth = args
    torch.set_num_threads(1)
    x = synth.mix1d_events(n, seed=seed, fit=fit_index)
    th, err, _ = fit(x, truth, config0_desc(), bounds=CONFIG0_BOUNDS)
    return (th - np.asarray(truth)) / err


def config0_desc(lo: float = -10.0, hi: float = 10.0) -> dict:
    """The 1-D fit: f Gaussian(mu, sigma) + (1-f) exponential(tau) on [lo, hi]."""
    return {"kind": "mix1d", "lo": lo, "hi": hi, "n_params": 4,
            "components": [{"type": "gauss", "params": [0, 1]},
                           {"type": "exp", "params": [2]}],
            "fracs": [3]}


def max_density(theta, desc: dict, n_scan: int = 200001) -> float:
    lo, hi, _, _ = parse(desc)
    x = torch.linspace(lo, hi, n_scan, dtype=torch.float64)
    with torch.no_grad():
        return float(density(as_t(theta), x, desc).max())
