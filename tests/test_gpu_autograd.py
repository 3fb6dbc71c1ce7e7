"""The NLL as a torch.autograd.Function (the Python bindings' differentiable
objective): gradients through NLLFunction equal the library's adjoint
gradient bitwise and the oracle's autograd gradient to 1e-10, for theta on
the CPU and on the GPU."""
import numpy as np
import pytest
import torch

import synth
from oracle import dalitz3 as OD, mix1d as OM
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def _check(model, theta, ev_dev, vo, go, device):
    from paper_1710_08826_amd import NLLFunction
    v_ref, g_ref = model.nll(theta, ev_dev, grad=True)
    th = torch.tensor(theta, dtype=torch.float64, device=device, requires_grad=True)
    v = NLLFunction.apply(th, model, ev_dev)
    assert v.device == th.device
    (g,) = torch.autograd.grad(2.5 * v, th)
    assert g.device == th.device
    assert float(v) == v_ref
    assert np.array_equal(g.cpu().numpy(), 2.5 * g_ref)
    assert abs(float(v) - vo) <= 1e-12 * abs(vo)
    gg = g.cpu().numpy() / 2.5
    assert np.allclose(gg, go, rtol=1e-10, atol=1e-10 * np.abs(go).max()), (gg, go)


@pytest.mark.parametrize("device", ["cpu", "cuda"])
def test_nllfunction_mix1d(device):
    from paper_1710_08826_amd import Model
    d = OM.config0_desc()
    x = synth.mix1d_events(20_000, seed=41)
    th = np.array(synth.CONFIG0_TRUTH) * np.array([1.05, 0.97, 1.1, 0.98])
    vo, go = OM.nll_grad(th, x, d)
    _check(Model(d), th, to_dev(x), vo, go, device)


@pytest.mark.parametrize("device", ["cpu", "cuda"])
def test_nllfunction_dalitz(device):
    from paper_1710_08826_amd import Model
    d = OD.config1_desc(grid=(128, 128), free_lineshapes=True)
    th = OD.truth_theta(d) * 1.01
    ev = synth.dalitz_events(5_000, seed=42)
    vo, go = OD.nll_grad(th, ev, d)
    say("oracle", vo)
    _check(Model(d), th, to_dev(ev), vo, go, device)


def test_nllfunction_in_torch_optimizer():
    """A few steps of a torch optimizer on the device NLL move downhill."""
    from paper_1710_08826_amd import Model, NLLFunction
    d = OM.config0_desc()
    m = Model(d)
    ev = to_dev(synth.mix1d_events(50_000, seed=43))
    th = torch.tensor(np.array(synth.CONFIG0_TRUTH) * 1.1, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.LBFGS([th], lr=0.5, max_iter=40, line_search_fn="strong_wolfe")
    v0 = float(NLLFunction.apply(th, m, ev))

    def closure():
        opt.zero_grad()
        v = NLLFunction.apply(th, m, ev)
        v.backward()
        return v

    opt.step(closure)
    v1 = float(NLLFunction.apply(th, m, ev))
    one = m.fit(np.array(synth.CONFIG0_TRUTH) * 1.1, ev)
    say("nll", v0, "->", v1, "fit", one.nll)
    assert v1 < v0 and abs(v1 - one.nll) < 1e-4
