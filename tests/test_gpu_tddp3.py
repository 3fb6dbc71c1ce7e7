"""Parity of the time-dependent Dalitz-plot NLL, normalization and adjoint
gradient with the oracle (oracle/tddp3.py)."""
import math

import numpy as np
import pytest

import synth
from oracle import common, tddp3 as T
from tests.gpu_util import grad_close, rel_close, say, to_dev

pytestmark = pytest.mark.gpu


def events(n, seed, desc):
    return synth.tddp3_events(n, seed, desc["tau"], desc["sigma_t"])


def theta(x=0.02, y=0.03):
    th = T.truth_theta(x=x, y=y)
    th[16:32] = np.roll(th[16:32], 2) * 0.9 + 0.01   # cbar != c
    return th


D256 = T.pipipi0_desc(grid=(256, 256))


@pytest.fixture(scope="module")
def m256():
    from paper_1710_08826_amd import Model
    return Model(D256)


@pytest.fixture(scope="module")
def cells256():
    return T.TDDP(D256).dal.grid_cells()


def test_norm_matches_oracle(m256, cells256):
    say("tddp3 norm")
    for th in (theta(), theta(0.3, -0.2)):
        I, dI = m256.norm(th)
        Io = T.norm_value(T.TDDP(D256), th, cells256)
        assert rel_close(I, Io, 1e-12), (I, Io)


@pytest.mark.parametrize("n", [1, 1000, 3 * 1024 + 17, 50_000])
def test_nll_and_gradient(m256, cells256, n):
    say("tddp3 n =", n)
    ev = events(n, 61, D256)
    for th in (theta(), theta(0.3, -0.2)):
        v, g = m256.nll(th, to_dev(ev), grad=True)
        vo, go = T.nll_grad(th, ev, D256, cells256)
        assert rel_close(v, vo, 1e-12), (v, vo, (v - vo) / vo)
        ok, r = grad_close(g, go, 1e-10)
        assert ok, r
        assert rel_close(m256.nll(th, to_dev(ev)), v, 1e-14)


def test_gradient_vs_central_fd():
    from paper_1710_08826_amd import Model
    d = T.pipipi0_desc(grid=(64, 64))
    m = Model(d)
    ev = events(2000, 62, d)
    th = theta(0.05, 0.04)
    _, g = m.nll(th, to_dev(ev), grad=True)
    fd = common.central_fd(lambda t: T.nll(t, ev, d), th, rel_step=1e-6)
    ok, r = grad_close(g, fd, 1e-6)
    assert ok, r


def test_full_size():
    """1M events on the 1024 x 1024 grid, the benchmark's configuration."""
    from paper_1710_08826_amd import Model
    d = T.pipipi0_desc()
    m = Model(d)
    ev = events(1_000_000, 63, d)
    th = theta()
    v = m.nll(th, to_dev(ev))
    vo = T.nll(th, ev, d)
    assert rel_close(v, vo, 1e-12), (v, vo)


def test_bitwise_repeatable_and_empty(m256):
    ev = to_dev(events(20_000, 64, D256))
    th = theta()
    a = m256.nll(th, ev, grad=True)
    b = m256.nll(th, ev, grad=True)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])
    import torch
    v, g = m256.nll(th, torch.zeros((3, 0), dtype=torch.float64, device="cuda"), grad=True)
    assert v == 0.0 and not np.any(g)


def test_invalid_descriptions_and_calls(m256):
    from paper_1710_08826_amd import FitNLLError, Model
    bad = [dict(D256, m=[0.135, 0.1396, 0.1350]), dict(D256, grid=[256, 128]), dict(D256, tau=0.0),
           dict(D256, sigma_t=-1.0), dict(D256, free_lineshapes=True)]
    for d in bad:
        with pytest.raises(FitNLLError):
            Model(d)
    with pytest.raises(FitNLLError):
        m256.eval(theta(), to_dev(events(10, 65, D256)))


def test_generation_matches_oracle(m256):
    """Device toy events against the oracle generator (same per-event
    accept-reject definition, same envelope): Dalitz coordinates bitwise,
    decay times to rounding, except where an accept decision falls within
    rounding of the rate."""
    say("tddp3 generate")
    th = theta(0.3, 0.2)
    W = T.envelope(th, D256)
    ev, used = m256.generate(th, 3000, seed=31, fit=2, envelope=W)
    assert used == W
    orc, _, above = T.generate(th, D256, 3000, seed=31, fit=2, W=W)
    assert above == 0
    dev = ev.cpu().numpy()
    same = np.all(dev[:2] == orc[:2], axis=0)
    assert same.mean() >= 0.999, same.mean()
    assert np.allclose(dev[2][same], orc[2][same], rtol=0.0, atol=1e-13)
    _, Wa = m256.generate(th, 0, seed=1)
    assert rel_close(Wa, W, 1e-12), (Wa, W)


def test_fit_to_generated_events_recovers_the_truth():
    """Host BFGS fit of 200k device-generated events at a point with large
    mixing (x = 0.05, y = 0.04): c_0 fixed (the NLL is invariant under a common
    complex rescaling of c and cbar) and cbar fixed at its true value; every
    free parameter within 4 errors of the truth."""
    from paper_1710_08826_amd import Model
    say("tddp3 fit")
    d = T.pipipi0_desc(grid=(512, 512))
    m = Model(d)
    th = T.truth_theta(x=0.05, y=0.04)
    ev, _ = m.generate(th, 200_000, seed=41)
    free = np.zeros(th.size, dtype=np.int32)
    free[2:16] = 1
    free[-2:] = 1
    start = th.copy()
    start[2:16] *= 1.03
    start[-2:] = [0.03, 0.02]
    r = m.fit(start, ev, free=free)
    pull = (r.theta - th)[free == 1] / r.errors[free == 1]
    say("  x, y =", r.theta[-2:], "+-", r.errors[-2:], "max pull", np.max(np.abs(pull)))
    assert np.all(np.abs(pull) < 4.0), pull
