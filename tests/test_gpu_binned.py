"""Binned data and extended likelihoods of 1-D mixtures against the oracle:
Poisson NLL and chi^2 of histogram counts, with and without a yield
parameter, values and gradients; the extended unbinned NLL; binned fits."""
import numpy as np
import pytest
import torch

import synth
from oracle import mix1d as OM
from tests.gpu_util import grad_close, rel_close, say, to_dev

pytestmark = pytest.mark.gpu

D0 = OM.config0_desc()
TRUTH = np.array(synth.CONFIG0_TRUTH)
OFF = TRUTH * np.array([1.1, 0.95, 1.05, 0.97])
D4 = {"kind": "mix1d", "lo": 5.20, "hi": 5.30, "n_params": 10,
      "components": [{"type": "argus", "params": [0, 1]},
                     {"type": "bw", "params": [2, 3]},
                     {"type": "gauss", "params": [4, 5]},
                     {"type": "exp", "params": [6]}],
      "fracs": [7, 8, 9]}
TH4 = np.array([5.29, -20.0, 5.2795, 0.004, 5.28, 0.003, -3.0, 0.4, 0.2, 0.25])


def ext(desc):
    i = desc["n_params"]
    return dict(desc, n_params=i + 1, **{"yield": i})


def hist(x, desc, nb):
    return np.histogram(x, bins=nb, range=(desc["lo"], desc["hi"]))[0].astype(np.float64)


@pytest.mark.parametrize("stat", ["poisson", "chi2"])
@pytest.mark.parametrize("extended", [False, True])
@pytest.mark.parametrize("nb", [1, 100, 2048 + 17, 100_000])
def test_config0_binned_parity(stat, extended, nb):
    from paper_1710_08826_amd import Model
    say("binned config0", stat, "extended" if extended else "", "nb =", nb)
    d = ext(D0) if extended else D0
    m = Model(d)
    counts = hist(synth.mix1d_events(200_000, seed=21), D0, nb)
    th = np.r_[OFF, 1.9e5] if extended else OFF
    v, g = m.nll_binned(th, to_dev(counts)[0], stat, grad=True)
    vo, go = OM.binned_value_grad(th, counts, d, stat)
    assert rel_close(v, vo, 1e-12), (v, vo)
    ok, r = grad_close(g, go, 1e-10)
    assert ok, r
    assert rel_close(m.nll_binned(th, to_dev(counts)[0], stat), v, 1e-14)


@pytest.mark.parametrize("stat", ["poisson", "chi2"])
def test_four_component_binned_parity(stat):
    from paper_1710_08826_amd import Model
    say("binned four components", stat)
    m = Model(ext(D4))
    rng = np.random.default_rng(22)
    counts = rng.poisson(50.0, 3000).astype(np.float64)
    counts[::7] = 0.0
    th = np.r_[TH4, 1.4e5]
    v, g = m.nll_binned(th, to_dev(counts)[0], stat, grad=True)
    vo, go = OM.binned_value_grad(th, counts, ext(D4), stat)
    assert rel_close(v, vo, 1e-12), (v, vo)
    ok, r = grad_close(g, go, 1e-10)
    assert ok, r


@pytest.mark.parametrize("n", [1, 3 * 1024 + 5, 100_000])
def test_extended_unbinned_parity(n):
    from paper_1710_08826_amd import Model
    say("extended unbinned n =", n)
    m = Model(ext(D0))
    x = synth.mix1d_events(n, seed=23)
    th = np.r_[OFF, 1.05 * n]
    v, g = m.nll(th, to_dev(x), grad=True)
    vo, go = OM.nll_grad(th, x, ext(D0))
    assert rel_close(v, vo, 1e-12), (v, vo)
    ok, r = grad_close(g, go, 1e-10)
    assert ok, r


def test_binned_fits_recover_the_truth():
    """Extended Poisson (2000 bins) and chi^2 (100 bins, every bin well
    filled: Neyman's chi^2 is biased where counts are small) fits of a
    1M-event histogram: parameters within 4 errors of the truth and of the
    unbinned fit, yield near N."""
    from paper_1710_08826_amd import Model, generate_mix1d
    say("binned fits")
    n = 1_000_000
    ev = generate_mix1d(n, 1710088260, 3, TRUTH)
    ub = Model(D0).fit(TRUTH * 1.05, ev)
    m = Model(ext(D0))
    start = np.r_[TRUTH * 1.05, 0.9 * n]
    for stat, nb in (("poisson", 2000), ("chi2", 100)):
        counts = torch.histc(ev[0], bins=nb, min=-10.0, max=10.0).to(torch.float64)
        assert float(counts.sum()) == n and (stat == "poisson" or float(counts.min()) > 30)
        r = m.fit_binned(start, counts, stat)
        pull = (r.theta[:4] - TRUTH) / r.errors[:4]
        say("  ", stat, r.theta, r.errors, r.n_iter)
        assert np.all(np.abs(pull) < 4.0), pull
        assert np.all(np.abs(r.theta[:4] - ub.theta) < 4.0 * ub.errors)
        assert abs(r.theta[4] - n) < 4.0 * r.errors[4]


def test_binned_errors():
    from paper_1710_08826_amd import FitNLLError, Model
    m = Model(D0)
    c = to_dev(np.ones(10))[0]
    with pytest.raises(KeyError):
        m.nll_binned(TRUTH, c, "likelihood")
    import ctypes as C
    from paper_1710_08826_amd import _lib
    st = m._lib.fn_nll_binned(m._h, TRUTH.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(c.data_ptr()), 10,
                              7, None, None, None)
    assert st == _lib.FN_E_INVALID
    with pytest.raises(FitNLLError):  # no events in a non-extended chi^2 / Poisson fit
        m.nll_binned(TRUTH, to_dev(np.zeros(10))[0], "poisson")
    import oracle.dalitz3 as OD
    md = Model(OD.config1_desc(grid=(64, 64)))
    with pytest.raises(FitNLLError):
        md.nll_binned(OD.truth_theta(OD.config1_desc()), c, "poisson")
