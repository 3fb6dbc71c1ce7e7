"""Device generation for the four-body model: the phase-space normalization
sample equals the input sampler's (same counters), and toy events match the
oracle's per-event generator (same accept-reject definition and envelope)."""
import numpy as np
import pytest

import synth
from oracle import td4 as OT
from tests.gpu_util import rel_close, say, to_dev
from tests.test_oracle_td4 import SMALL, SMALL_TH

pytestmark = pytest.mark.gpu


def test_norm_sample_matches_the_input_sampler():
    """The normalization from a device-generated sample equals the one from
    the same points generated on the host and copied in."""
    from paper_1710_08826_amd import Model
    say("td4 phase-space sample")
    m = Model(SMALL)
    n = 200_000
    m.generate_norm_sample(n, seed=71, fit=3)
    I_gen, _ = m.norm(SMALL_TH)
    m.set_norm_sample(to_dev(synth.td4_phase_space(n, seed=71, fit=3)))
    I_set, _ = m.norm(SMALL_TH)
    assert I_gen == I_set, (I_gen, I_set)


def test_events_match_the_oracle_generator():
    from paper_1710_08826_amd import Model
    say("td4 generate")
    m = Model(SMALL)
    m.generate_norm_sample(100_000, seed=72)
    _, W_auto = m.generate(SMALL_TH, 0, seed=1)
    assert W_auto > 0
    n = 400
    _, W, _ = OT.generate_events(SMALL_TH, SMALL, 0, seed=73, fit=1)  # the oracle's envelope
    ev, used = m.generate(SMALL_TH, n, seed=73, fit=1, envelope=W)
    assert used == W
    orc, _, above = OT.generate_events(SMALL_TH, SMALL, n, seed=73, fit=1, W=W)
    assert above == 0
    dev = ev.cpu().numpy()
    same = np.all(dev[:5] == orc[:5], axis=0)
    say("  equal:", int(same.sum()), "of", n)
    assert same.mean() >= 0.99
    assert np.allclose(dev[5][same], orc[5][same], rtol=0.0, atol=1e-13)
    assert np.isfinite(dev).all()
