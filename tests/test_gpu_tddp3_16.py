"""Parity of the time-dependent Dalitz-plot model at the size of the paper's
pi+ pi- pi0 example (sixteen resonances: rho(770), rho(1450), rho(1700) in
each pair and seven isoscalar states in pi+ pi-): NLL, normalization and
adjoint gradient against the oracle on a coarse grid at several sample sizes,
central differences, and the 1M-event, 1024 x 1024-grid configuration the
benchmark times (NLL and gradient)."""
import numpy as np
import pytest

import synth
from oracle import common, tddp3 as T
from tests.gpu_util import grad_close, rel_close, say, to_dev

pytestmark = pytest.mark.gpu

D128 = synth.tddp3_desc16(grid=(128, 128))


def events(n, seed):
    return synth.tddp3_events(n, seed, resonances=synth.TDDP_RESONANCES16)


def theta(x=0.02, y=0.03):
    th = synth.tddp3_truth16(x=x, y=y)
    K = 16
    th[2 * K:4 * K] = np.roll(th[2 * K:4 * K], 2) * 0.9 + 0.01  # cbar != c
    return th


@pytest.fixture(scope="module")
def m128():
    from paper_1710_08826_amd import Model
    return Model(D128)


@pytest.fixture(scope="module")
def cells128():
    return T.TDDP(D128).dal.grid_cells()


def test_layout(m128):
    assert m128.n_params == 4 * 16 + 2


def test_norm_matches_oracle(m128, cells128):
    say("tddp3-16 norm")
    for th in (theta(), theta(0.3, -0.2)):
        I, _ = m128.norm(th)
        assert rel_close(I, T.norm_value(T.TDDP(D128), th, cells128), 1e-12)


@pytest.mark.parametrize("n", [1, 3 * 4096 + 17, 50_000])
def test_nll_and_gradient(m128, cells128, n):
    say("tddp3-16 n =", n)
    ev = events(n, 161)
    for th in (theta(), theta(0.3, -0.2)):
        v, g = m128.nll(th, to_dev(ev), grad=True)
        vo, go = T.nll_grad(th, ev, D128, cells128)
        assert rel_close(v, vo, 1e-12), (v, vo, (v - vo) / vo)
        ok, r = grad_close(g, go, 1e-10)
        assert ok, r.max()
        assert rel_close(m128.nll(th, to_dev(ev)), v, 1e-14)


def test_gradient_vs_central_fd():
    from paper_1710_08826_amd import Model
    d = synth.tddp3_desc16(grid=(48, 48))
    m = Model(d)
    ev = events(2000, 162)
    th = theta(0.05, 0.04)
    _, g = m.nll(th, to_dev(ev), grad=True)
    fd = common.central_fd(lambda t: T.nll(t, ev, d), th, rel_step=1e-6)
    ok, r = grad_close(g, fd, 1e-6)
    assert ok, r.max()


def test_full_size():
    """1M events on the 1024 x 1024 grid with the gradient."""
    from paper_1710_08826_amd import Model
    say("tddp3-16 full size")
    d = synth.tddp3_desc16()
    m = Model(d)
    ev = events(1_000_000, 163)
    th = theta()
    v, g = m.nll(th, to_dev(ev), grad=True)
    say("tddp3-16 full size: oracle")
    vo, go = T.nll_grad(th, ev, d)
    assert rel_close(v, vo, 1e-12), (v, vo)
    ok, r = grad_close(g, go, 1e-10)
    assert ok, r.max()
