"""Parity of the device 1-D mixture NLL (+ adjoint gradient) with the oracle."""
import numpy as np
import pytest

import synth
from oracle import common, mix1d as OM
from tests.gpu_util import grad_close, rel_close, say, to_dev

pytestmark = pytest.mark.gpu

D0 = OM.config0_desc()
TRUTH = np.array(synth.CONFIG0_TRUTH)
OFF = TRUTH * np.array([1.15, 0.9, 1.2, 0.95])  # a non-stationary point
D4 = {"kind": "mix1d", "lo": 5.20, "hi": 5.30, "n_params": 10,
      "components": [{"type": "argus", "params": [0, 1]},
                     {"type": "bw", "params": [2, 3]},
                     {"type": "gauss", "params": [4, 5]},
                     {"type": "exp", "params": [6]}],
      "fracs": [7, 8, 9]}
TH4 = np.array([5.29, -20.0, 5.2795, 0.004, 5.28, 0.003, -3.0, 0.4, 0.2, 0.25])


@pytest.fixture(scope="module")
def m0():
    from paper_1710_08826_amd import Model
    return Model(D0)


@pytest.mark.parametrize("n", [1, 255, 2048, 2049, 3 * 2048 + 17, 100_000])
def test_config0_nll_and_grad(m0, n):
    say("mix1d config0 n =", n)
    x = synth.mix1d_events(n, seed=11)
    ev = to_dev(x)
    for th in (TRUTH, OFF):
        v, g = m0.nll(th, ev, grad=True)
        vo, go = OM.nll_grad(th, x, D0)
        assert rel_close(v, vo, 1e-12), (v, vo)
        ok, r = grad_close(g, go, 1e-10)
        assert ok, r
        assert rel_close(m0.nll(th, ev), v, 1e-14)  # NLL-only kernel agrees


def test_config0_grad_vs_central_fd(m0):
    x = synth.mix1d_events(20000, seed=12)
    ev = to_dev(x)
    _, g = m0.nll(OFF, ev, grad=True)
    fd = common.central_fd(lambda t: OM.nll(t, x, D0), OFF)
    ok, r = grad_close(g, fd, 1e-6)
    assert ok, r


def test_empty_sample(m0):
    import torch
    ev = torch.zeros((1, 0), dtype=torch.float64, device="cuda")
    v, g = m0.nll(TRUTH, ev, grad=True)
    assert v == 0.0 and (g == 0).all()


def test_four_component_model():
    from paper_1710_08826_amd import Model
    m = Model(D4)
    x = np.linspace(5.2 + 1e-5, 5.3 - 1e-5, 5003)
    ev = to_dev(x)
    v, g = m.nll(TH4, ev, grad=True)
    vo, go = OM.nll_grad(TH4, x, D4)
    assert rel_close(v, vo, 1e-12), (v, vo)
    ok, r = grad_close(g, go, 1e-10)
    assert ok, r
    p = m.eval(TH4, ev).cpu().numpy()
    import torch
    with torch.no_grad():
        po = OM.density(common.as_t(TH4), common.as_t(x), D4).numpy()
    assert np.allclose(p, po, rtol=1e-12, atol=0)


def test_bitwise_repeatable(m0):
    ev = to_dev(synth.mix1d_events(300_001, seed=13))
    ref = m0.nll(OFF, ev, grad=True)
    for _ in range(10):
        v, g = m0.nll(OFF, ev, grad=True)
        assert v == ref[0] and np.array_equal(g, ref[1])


def test_invalid_parameters_raise_nonfinite(m0):
    from paper_1710_08826_amd import FitNLLError
    from paper_1710_08826_amd._lib import FN_E_NONFINITE
    ev = to_dev(synth.mix1d_events(1000))
    for bad in ([0.2, -1.0, -0.3, 0.7], [0.2, 1.1, -0.3, 5.0], [np.nan, 1.1, -0.3, 0.7]):
        with pytest.raises(FitNLLError) as e:
            m0.nll(bad, ev)
        assert e.value.status == FN_E_NONFINITE


def test_events_check(m0):
    x = synth.mix1d_events(5000)
    x[[3, 100, 4999]] = [11.0, -10.5, np.nan]
    assert m0.check_events(to_dev(x)) == 3
    assert m0.check_events(to_dev(synth.mix1d_events(5000))) == 0


def test_fit_matches_oracle_fit(m0):
    """Device BFGS (adjoint and finite-difference gradients) and the oracle's
    quasi-Newton fit land on the same minimum within 1e-3 sigma."""
    from scipy import optimize
    x = synth.mix1d_events(100_000, seed=21)
    ev = to_dev(x)
    start = TRUTH * 1.1
    ra = m0.fit(start, ev, grad_mode="adjoint")
    rf = m0.fit(start, ev, grad_mode="fd")
    res = optimize.minimize(lambda t: OM.nll_grad(t, x, D0), start, jac=True, method="L-BFGS-B",
                            bounds=[(-5, 5), (0.1, 5), (-3, 3), (0.01, 0.99)],
                            options={"ftol": 1e-15, "gtol": 1e-9, "maxiter": 1000})
    say("adjoint", ra.theta, ra.errors, ra.n_iter, ra.n_calls)
    say("fd     ", rf.theta, rf.errors, rf.n_iter, rf.n_calls)
    say("oracle ", res.x)
    assert (np.abs(ra.theta - res.x) < 1e-3 * ra.errors).all()
    assert (np.abs(rf.theta - res.x) < 1e-3 * ra.errors).all()
    assert (np.abs(ra.errors / rf.errors - 1) < 1e-3).all()
    assert (np.abs(ra.theta - TRUTH) < 5 * ra.errors).all()


def test_tiny_densities_far_tails():
    """A narrow Gaussian over events spread on [-8, 8]: densities down to
    e^-525 (the product of two of them underflows a double), where the passes'
    running product of densities must renormalize after every event; NLL and
    gradient match the oracle's sum of logarithms.  Densities that are exactly
    zero (events 160 sigma out, where exp underflows) make the NLL +inf."""
    from paper_1710_08826_amd import FitNLLError, Model
    from paper_1710_08826_amd._lib import FN_E_NONFINITE
    d = {"kind": "mix1d", "lo": -10.0, "hi": 10.0, "n_params": 2,
         "components": [{"type": "gauss", "params": [0, 1]}], "fracs": []}
    m = Model(d)
    rng = np.random.default_rng(23)
    x = rng.uniform(-8.0, 8.0, 5000)
    th = np.array([0.1, 0.25])  # x - mu up to 8.1 = 32 sigma: ln P down to -525
    v, g = m.nll(th, to_dev(x), grad=True)
    vo, go = OM.nll_grad(th, x, d)
    assert np.isfinite(v) and v > 1e5
    assert rel_close(v, vo, 1e-12), (v, vo)
    ok, r = grad_close(g, go, 1e-10)
    assert ok, r
    th_narrow = np.array([0.1, 0.05])  # up to 162 sigma: exp(-13000) = 0 for the far events
    with pytest.raises(FitNLLError) as e:
        m.nll(th_narrow, to_dev(x))
    assert e.value.status == FN_E_NONFINITE
