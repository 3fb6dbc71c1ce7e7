"""Device toy generation of Dalitz-plot events against the oracle generator
(the same per-event accept-reject definition): events equal bitwise except
where the accept decision u3 W < P~ falls within rounding of P~, the
automatic envelope, the per-event property, errors."""
import numpy as np
import pytest
import torch

from oracle import dalitz3 as OD
from tests.gpu_util import rel_close, say

pytestmark = pytest.mark.gpu

D1 = OD.config1_desc()
TH1 = OD.truth_theta(D1)
D3 = OD.config1_desc(free_lineshapes=True)


def offset(th):
    return th + 0.03 * np.sin(np.arange(th.size) + 1.0) * np.maximum(np.abs(th), 0.05)


@pytest.fixture(scope="module")
def m1():
    from paper_1710_08826_amd import Model
    return Model(D1)


def _compare(dev, orc, model):
    same = np.all(dev == orc, axis=0)
    say("  events equal bitwise:", int(same.sum()), "of", same.size)
    assert same.mean() >= 0.999
    assert model.inside(dev[0][~same], dev[1][~same]).all()


@pytest.mark.parametrize("n", [1, 3000, 20_000 + 77])
def test_events_match_oracle(m1, n):
    say("dalitz generate n =", n)
    W = OD.envelope(TH1, D1)
    ev, used = m1.generate(TH1, n, seed=11, fit=5, envelope=W)
    assert used == W
    orc, _, above = OD.generate(TH1, D1, n, seed=11, fit=5, W=W)
    assert above == 0
    _compare(ev.cpu().numpy(), orc, OD.Dalitz(D1))


def test_automatic_envelope_and_free_lineshapes():
    from paper_1710_08826_amd import Model
    say("dalitz generate free lineshapes")
    m3 = Model(D3)
    th = offset(OD.truth_theta(D3))
    ev, W = m3.generate(th, 5000, seed=12)
    Wo = OD.envelope(th, D3)
    assert rel_close(W, Wo, 1e-12), (W, Wo)
    orc, _, _ = OD.generate(th, D3, 5000, seed=12, W=W)
    _compare(ev.cpu().numpy(), orc, OD.Dalitz(D3))


def test_per_event_and_full_size(m1):
    """1M events (the benchmark's size): a 10k run is their prefix; every
    event is finite and inside the region."""
    say("dalitz generate 1M")
    ev, W = m1.generate(TH1, 1_000_000, seed=13)
    head, W2 = m1.generate(TH1, 10_000, seed=13)
    assert W2 == W and torch.equal(head, ev[:, :10_000])
    e = ev.cpu().numpy()
    assert np.isfinite(e).all() and OD.Dalitz(D1).inside(e[0], e[1]).all()
    assert m1.check_events(ev) == 0


def test_generation_errors(m1):
    from paper_1710_08826_amd import FitNLLError, Model
    import synth
    with pytest.raises(FitNLLError):
        m1.generate(TH1, 100, seed=1, envelope=-1.0)
    with pytest.raises(FitNLLError):
        Model(synth.mix1d_desc()).generate(synth.mix1d_truth(), 100, seed=1)
    W = OD.envelope(TH1, D1)
    with pytest.raises(FitNLLError, match="above the envelope"):
        m1.generate(TH1, 20_000, seed=1, envelope=0.2 * W)
    ev, _ = m1.generate(TH1, 0, seed=1)
    assert ev.shape == (2, 0)
