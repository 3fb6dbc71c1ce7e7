"""Parity of the device time-dependent four-body NLL, normalization, adjoint
gradient and per-event density with the oracle, from a few events to the full
workload (10M events, 5M-point normalization sample)."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from oracle import common, td4 as OT
from tests.gpu_util import grad_close, rel_close, say, to_dev

pytestmark = pytest.mark.gpu

DESC = synth.td4_desc()
TH = synth.td4_truth()
N_MC = 20_000


def offset(th):
    t = th + 0.05 * np.sin(np.arange(th.size) + 1.0) * np.maximum(np.abs(th), 0.05)
    t[-2:] = [0.03, -0.02]
    return t


@pytest.fixture(scope="module")
def mc():
    return synth.td4_phase_space(N_MC, seed=41)


@pytest.fixture(scope="module")
def model(mc):
    from paper_1710_08826_amd import Model
    m = Model(DESC)
    m.set_norm_sample(to_dev(mc))
    return m


def oracle_norm(th, mc):
    model = OT.TD4(DESC)
    tht = torch.tensor(th, requires_grad=True)
    ir = model.integrated_rate(tht, torch.tensor(mc))
    ir.mean().backward()
    return common.fsum(ir.detach()) / mc.shape[1], tht.grad.numpy().copy()


def test_norm_matches_oracle(model, mc):
    say("td4 norm")
    for th in (TH, offset(TH)):
        I, dI = model.norm(th)
        Io, dIo = oracle_norm(th, mc)
        assert rel_close(I, Io, 1e-12), (I, Io)
        ok, r = grad_close(dI, dIo, 1e-11)
        assert ok, r.max()


@pytest.mark.parametrize("n", [1, 1000, 3 * 1024 + 17, 20_000])
def test_nll_and_gradient(model, mc, n):
    say("td4 nll n =", n)
    ev = synth.td4_events(n, seed=43)
    evd = to_dev(ev)
    for th in (TH, offset(TH)):
        v, g = model.nll(th, evd, grad=True)
        vo, go = OT.nll_grad(th, ev, mc, DESC)
        assert rel_close(v, vo, 1e-12), (v, vo, (v - vo) / vo)
        ok, r = grad_close(g, go, 1e-10)
        assert ok, r.max()
        # the value-only kernel sums the same tree; its instantiation may contract differently
        assert rel_close(model.nll(th, evd), v, 1e-14)


def test_gradient_vs_central_differences(model, mc):
    say("td4 fd")
    ev = synth.td4_events(3000, seed=44)
    evd = to_dev(ev)
    th = offset(TH)
    _, g = model.nll(th, evd, grad=True)
    fd = common.central_fd(lambda q: OT.nll(q, ev, mc, DESC), th, rel_step=1e-6)
    ok, r = grad_close(g, fd, 1e-6)
    assert ok, r.max()


def test_eval_is_normalized_rate(model, mc):
    say("td4 eval")
    ev = synth.td4_events(5000, seed=45)
    th = offset(TH)
    p = model.eval(th, to_dev(ev)).cpu().numpy()
    om = OT.TD4(DESC)
    tht, evt = torch.tensor(th), torch.tensor(ev)
    with torch.no_grad():
        r = om.rate(tht, evt).numpy()
        # condition scale of R: the same sums with every term taken in magnitude, so
        # that interference minima (R far below its terms) are judged on the terms' size
        B = om.basis(evt[:5])
        K = om.K
        aa = sum(abs(complex(th[2 * k], th[2 * k + 1])) * B[k].abs() for k in range(K)).numpy()
        bb = sum(abs(complex(th[2 * K + 2 * k], th[2 * K + 2 * k + 1])) * B[k].abs() for k in range(K)).numpy()
        G = 1.0 / synth.TD4_TAU
        x, y = th[-2:]
        hp = OT.h_conv(complex(G * (1 - y)), evt[5], om.sigma).real.abs().numpy()
        hm = OT.h_conv(complex(G * (1 + y)), evt[5], om.sigma).real.abs().numpy()
        hc = OT.h_conv(complex(G, -G * x), evt[5], om.sigma).abs().numpy()
    cond = 0.5 * ((aa ** 2 + bb ** 2) * (hp + hm + hc) + 2 * aa * bb * (hp + hm + hc))
    I, _ = oracle_norm(th, mc)
    err = np.abs(p - r / I) / (cond / I)
    k = int(np.argmax(err))
    assert err.max() <= 1e-12, (err.max(), k, ev[:, k], p[k], r[k] / I)
    # and the plain relative error is within 1e-12 for all but a few events at interference minima
    rel = np.abs(p - r / I) / (r / I)
    assert (rel <= 1e-12).mean() >= 0.999, np.sort(rel)[-8:]


def test_empty_sample_and_determinism(model):
    say("td4 empty/determinism")
    v, g = model.nll(TH, torch.empty((6, 0), dtype=torch.float64, device="cuda"), grad=True)
    assert v == 0.0 and (g == 0.0).all()
    evd = to_dev(synth.td4_events(50_000, seed=46))
    a = model.nll(offset(TH), evd, grad=True)
    b = model.nll(offset(TH), evd, grad=True)
    assert a[0] == b[0] and (a[1] == b[1]).all()


def test_domain_check(model):
    say("td4 domain check")
    ev = synth.td4_events(1000, seed=47)
    assert model.check_events(to_dev(ev)) == 0
    bad = ev.copy()
    bad[0, 3] = 0.5          # m12 below m1 + m2
    bad[2, 10] = 1.5         # |cos| > 1
    bad[4, 20] = 4.0         # |phi| > pi
    bad[5, 30] = np.inf      # t not finite
    bad[1, 40] = 1.8         # m12 + m34 > M
    assert model.check_events(to_dev(bad)) == 5


def test_errors():
    from paper_1710_08826_amd import FitNLLError as FitError, Model
    m = Model(DESC)
    ev = to_dev(synth.td4_events(10, seed=48))
    with pytest.raises(FitError, match="normalization sample"):
        m.nll(TH, ev)
    bad = dict(DESC)
    bad["amps"] = DESC["amps"] + [[5, 0, 0]]
    with pytest.raises(FitError):
        Model(bad)
    bad = dict(DESC)
    bad["sigma_t"] = 0.0
    with pytest.raises(FitError, match="sigma_t"):
        Model(bad)
    fx = m.fixed()
    assert fx.size == 2 * (len(DESC["r12"]) + len(DESC["r34"])) + 1 and fx[-1] == DESC["sigma_t"]


@pytest.fixture(scope="module")
def full():
    say("td4 full-size inputs: 10M events, 5M-point sample")
    return synth.td4_events(10_000_000, seed=49), synth.td4_phase_space(5_000_000, seed=50)


def test_full_size(full):
    from paper_1710_08826_amd import Model
    ev, mc = full
    m = Model(DESC)
    m.set_norm_sample(to_dev(mc))
    th = offset(TH)
    evd = to_dev(ev)
    say("td4 full size: device")
    v, g = m.nll(th, evd, grad=True)
    say("td4 full size: oracle")
    vo, go = OT.nll_grad(th, ev, mc, DESC)
    assert rel_close(v, vo, 1e-12), (v, vo, (v - vo) / vo)
    ok, r = grad_close(g, go, 1e-10)
    assert ok, r.max()
