"""Parity with the oracle for model structures other than the benchmark ones:
the per-event passes are compiled for each model's structure, so every
structure is its own kernel."""
import numpy as np
import pytest

import synth
from oracle import dalitz3 as OD, td4 as OT
from tests.gpu_util import grad_close, rel_close, say, to_dev

pytestmark = pytest.mark.gpu

# Dalitz structures: one pair with spins 0 and 2; a single spin-1 resonance; all three pairs with spin 2
DALITZ_SHAPES = {
    "one_pair_L0_L2": (("13", 0, 1.430, 0.270, (1.0, 0.0)), ("13", 2, 1.430, 0.100, (0.6, -0.3))),
    "single_L1": (("12", 1, 0.892, 0.050, (1.0, 0.0)),),
    "spin2_all_pairs": (("12", 2, 1.430, 0.100, (1.0, 0.0)), ("13", 2, 1.430, 0.100, (0.4, 0.2)),
                        ("23", 2, 1.270, 0.185, (-0.3, 0.5))),
}


@pytest.mark.parametrize("name", sorted(DALITZ_SHAPES))
@pytest.mark.parametrize("free", [False, True])
def test_dalitz_structures(name, free):
    from paper_1710_08826_amd import Model
    res = DALITZ_SHAPES[name]
    desc = OD.config1_desc(grid=(256, 256), free_lineshapes=free, resonances=res)
    th = OD.truth_theta(desc, resonances=res) * (1.0 + 0.02 * np.cos(np.arange(2 * len(res) * (2 if free else 1))))
    say("dalitz shape", name, "free" if free else "fixed")
    m = Model(desc)
    ev = synth.dalitz_events(3 * m.chunk + 11, seed=71)
    cells = OD.Dalitz(desc).grid_cells()
    v, g = m.nll(th, to_dev(ev), grad=True)
    vo, go = OD.nll_grad(th, ev, desc, cells)
    assert rel_close(v, vo, 1e-12), (v, vo)
    if len(res) == 1 and not free:
        # one resonance, fixed lineshape: |c|^2 cancels between P~ and I, so the
        # gradient vanishes; its two cancelling terms are each about 2 N / |c|
        scale = 2 * ev.shape[1] / np.hypot(th[0], th[1])
        assert np.abs(g).max() <= 1e-12 * scale and np.abs(g - go).max() <= 1e-12 * scale
        return
    ok, r = grad_close(g, go, 1e-9)
    assert ok, r.max()


def test_td4_small_shape():
    """Three amplitudes, no spin-1 entry in pair (12), no phi-dependent factor."""
    from paper_1710_08826_amd import Model
    d = synth.td4_desc(r12=((0, 0.0, 0.0),))
    d["amps"] = [[0, 0, 0], [0, 1, 1], [0, 2, 0]]
    th = np.array([0.5, 0.0, -0.3, 0.35, 0.2, 0.25, 1.0, 0.0, 0.8, 0.45, 0.35, -0.3, 0.2, 0.15])
    mc = synth.td4_phase_space(20_000, seed=72)
    ev = synth.td4_events(3 * 1024 + 7, seed=73)
    say("td4 small shape")
    m = Model(d)
    m.set_norm_sample(to_dev(mc))
    v, g = m.nll(th, to_dev(ev), grad=True)
    vo, go = OT.nll_grad(th, ev, mc, d)
    assert rel_close(v, vo, 1e-12), (v, vo)
    ok, r = grad_close(g, go, 1e-10)
    assert ok, r.max()


def test_td4_spin1_and_phi_everywhere():
    """Every amplitude a product of two resonant spin-1 entries with a phi-dependent factor."""
    from paper_1710_08826_amd import Model
    d = synth.td4_desc(r12=((1, 1.019461, 0.004249),), r34=((1, 0.77526, 0.1491),))
    d["amps"] = [[0, 0, 4], [0, 0, 5], [0, 0, 3]]
    th = np.array([0.3, 0.1, -0.2, 0.25, 0.15, -0.05, 1.0, 0.0, 0.6, -0.4, 0.3, 0.2, 0.05, -0.03])
    mc = synth.td4_phase_space(20_000, seed=74)
    ev = synth.td4_events(2 * 1024 + 3, seed=75)
    say("td4 spin-1 shape")
    m = Model(d)
    m.set_norm_sample(to_dev(mc))
    v, g = m.nll(th, to_dev(ev), grad=True)
    vo, go = OT.nll_grad(th, ev, mc, d)
    assert rel_close(v, vo, 1e-12), (v, vo)
    ok, r = grad_close(g, go, 1e-10)
    assert ok, r.max()
