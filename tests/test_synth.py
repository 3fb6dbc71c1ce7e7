"""Input generators: Philox known answers and sampler sanity (CPU)."""
import os

import numpy as np

import synth
from synth.philox import philox4x32

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answers():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(w, 16) for w in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = philox4x32(tuple(r[0:4]), tuple(r[4:6]))
        assert [int(o) for o in out] == r[6:10]


def test_uniforms_range_and_determinism():
    a, b = synth.uniforms(100000, synth.key_from_seed(1), 0)
    assert a.min() >= 0 and a.max() < 1 and b.min() >= 0 and b.max() < 1
    assert abs(a.mean() - 0.5) < 0.005 and abs(b.var() - 1 / 12) < 0.002
    a2, _ = synth.uniforms(100000, synth.key_from_seed(1), 0)
    assert np.array_equal(a, a2)


def test_mix1d_events_in_range_and_mixture():
    x = synth.mix1d_events(200000)
    assert x.min() >= -10 and x.max() <= 10
    # the Gaussian component holds ~70% of events within +-5 sigma of mu
    near = np.abs(x - 0.2) < 5 * 1.1
    frac_exp_near = (1 - 0.7) * (np.exp(-0.3 * -5.3) - np.exp(-0.3 * 5.7)) / (np.exp(3) - np.exp(-3))
    assert abs(near.mean() - (0.7 + frac_exp_near)) < 0.01


def test_dalitz_events_inside_region():
    ev = synth.dalitz_events(50000)
    M, m1, m2, m3 = synth.DALITZ_MASSES
    s12, s13 = ev
    s23 = M * M + m1 * m1 + m2 * m2 + m3 * m3 - s12 - s13
    # every invariant mass lies within its two-body threshold and endpoint
    assert (s12 >= (m1 + m2) ** 2 - 1e-12).all() and (s12 <= (M - m3) ** 2 + 1e-12).all()
    assert (s13 >= (m1 + m3) ** 2 - 1e-12).all() and (s13 <= (M - m2) ** 2 + 1e-12).all()
    assert (s23 >= (m2 + m3) ** 2 - 1e-12).all() and (s23 <= (M - m1) ** 2 + 1e-12).all()
    # rho-like band in s23 around 0.77^2 is populated
    assert ((s23 > 0.5) & (s23 < 0.7)).mean() > 0.2


def test_sizes_distribution():
    n = synth.lognormal_sizes(4096)
    assert n.min() >= 1000 and n.max() <= 2_000_000
    assert 3.0e4 < np.median(n) < 6.0e4
