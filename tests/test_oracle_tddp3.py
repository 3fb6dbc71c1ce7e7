"""Pins of the time-dependent Dalitz-plot oracle (oracle/tddp3.py)."""
import math

import numpy as np
import pytest
import torch
from scipy import integrate

import synth
from oracle import common, dalitz3 as OD, tddp3 as T
from oracle.td4 import h_conv


def events(n, seed, desc):
    return synth.tddp3_events(n, seed, desc["tau"], desc["sigma_t"])


def dalitz_desc(desc):
    d = {k: v for k, v in desc.items() if k not in ("tau", "sigma_t")}
    return dict(d, kind="dalitz3", free_lineshapes=False)


def test_factorizes_without_mixing():
    """x = y = 0: R = |A|^2 h(G; t) and I = tau x the three-body integral, so
    NLL = NLL_dalitz3(c) - sum ln h(G; t_i) + N ln tau for any cbar."""
    desc = T.pipipi0_desc(grid=(96, 96))
    ev = events(400, 1, desc)
    th = T.truth_theta(x=0.0, y=0.0)
    th[16:32] = th[16:32] * 0.7 + 0.05   # cbar plays no role without mixing
    v = T.nll(th, ev, desc)
    vd = OD.nll(th[:16], ev[:2], dalitz_desc(desc))
    with torch.no_grad():
        h = h_conv(torch.tensor(1.0 / desc["tau"] + 0j), torch.from_numpy(ev[2]), desc["sigma_t"]).real
    expect = vd - common.fsum(torch.log(h)) + ev.shape[1] * math.log(desc["tau"])
    assert abs(v - expect) < 1e-11 * abs(expect), (v, expect)


def test_norm_without_mixing_is_tau_times_dalitz_norm():
    desc = T.pipipi0_desc(grid=(128, 128))
    th = T.truth_theta(x=0.0, y=0.0)
    m = T.TDDP(desc)
    a = T.norm_value(m, th)
    b = desc["tau"] * OD.norm_value(OD.Dalitz(dalitz_desc(desc)), th[:16])
    assert abs(a - b) < 1e-12 * b


@pytest.mark.parametrize("pt", [(0.6, 1.5), (1.2, 0.9), (2.0, 0.45)])
def test_time_integrals_match_the_integrated_rate(pt):
    """With large mixing and both amplitudes present, the integral over t of
    the unconvolved rate (t >= 0) and of the convolved rate (all t) equal
    the t-integrated rate: this fixes the signs of the mixing terms."""
    desc = T.pipipi0_desc(grid=(16, 16))
    m = T.TDDP(desc)
    th = T.truth_theta(x=0.4, y=0.25)
    th[16:32] = np.roll(th[16:32], 2) * 0.8   # cbar != c
    s12, s13 = (torch.tensor([v], dtype=torch.float64) for v in pt)
    assert OD.Dalitz(dalitz_desc(desc)).inside(np.array([pt[0]]), np.array([pt[1]]))[0]
    tt = torch.as_tensor(th)
    with torch.no_grad():
        want = float(m.integrated_rate(tt, s12, s13))

        def ru(t):
            return float(m.unconvolved_rate(tt, s12, s13, torch.tensor([t], dtype=torch.float64)))

        def rc(t):
            ev = torch.stack([s12, s13, torch.tensor([t], dtype=torch.float64)])
            return float(m.rate(tt, ev))

        a, _ = integrate.quad(ru, 0.0, 40.0 * desc["tau"], limit=400, epsabs=0.0, epsrel=1e-11)
        b, _ = integrate.quad(rc, -12.0 * desc["sigma_t"], 40.0 * desc["tau"], limit=400, epsabs=0.0,
                              epsrel=1e-10, points=[0.0])
    assert abs(a - want) < 1e-9 * abs(want), (a, want)
    assert abs(b - want) < 1e-8 * abs(want), (b, want)


def test_autograd_vs_central_fd():
    desc = T.pipipi0_desc(grid=(48, 48))
    ev = events(300, 2, desc)
    th = T.truth_theta(x=0.05, y=0.03)
    th[16:32] = th[16:32] * 0.9 + 0.02
    _, g = T.nll_grad(th, ev, desc)
    fd = common.central_fd(lambda t: T.nll(t, ev, desc), th, rel_step=1e-6)
    assert np.allclose(g, fd, rtol=2e-6, atol=2e-6 * np.max(np.abs(fd)))


def test_needs_conjugate_daughters():
    d = T.pipipi0_desc()
    d["m"] = [0.135, 0.1396, 0.494]
    with pytest.raises(ValueError):
        T.TDDP(d)


def test_conjugate_amplitude_is_the_mirrored_resonance():
    """With m2 = m3, the Dbar0 amplitude of a resonance in pair 12 at
    (s12, s13) is the D0 amplitude of the same resonance in pair 13 there
    (the daughters 2 and 3 exchanged): |Abar|^2 of a one-resonance model
    equals the three-body density of the mirrored model."""
    base = T.pipipi0_desc(grid=(16, 16))
    for pair, mirror in (("12", "13"), ("13", "12"), ("23", "23")):
        res = ((pair, 1, 0.7753, 0.1491, (1.0, 0.0)),)
        d = T.pipipi0_desc(grid=(16, 16), resonances=res)
        m = T.TDDP(d)
        ev = synth.dalitz_events(200, seed=3, masses=T.MASSES, resonances=T.RESONANCES)
        th = torch.tensor([0.3, -0.2, 0.8, 0.5, 0.01, 0.02], dtype=torch.float64)
        with torch.no_grad():
            A, Ab = m.amplitudes(th, torch.from_numpy(ev[0]), torch.from_numpy(ev[1]))
            dm = dict(dalitz_desc(base), resonances=[{"pair": mirror, "L": 1, "m0": 0.7753, "w0": 0.1491}])
            p = OD.Dalitz(dm).density_unnorm(torch.tensor([0.8, 0.5], dtype=torch.float64),
                                             torch.from_numpy(ev[0]), torch.from_numpy(ev[1]))
        b2 = (Ab.real ** 2 + Ab.imag ** 2).numpy()
        assert np.allclose(b2, p.numpy(), rtol=1e-12, atol=0.0), pair


# ------------------------------------------------------------ toy generation
@pytest.fixture(scope="module")
def toys():
    desc = T.pipipi0_desc(grid=(128, 128))
    th = T.truth_theta(x=0.3, y=0.2)
    th[16:32] = np.roll(th[16:32], 2) * 0.8
    ev, W, above = T.generate(th, desc, 5000, seed=21, fit=1)
    return desc, th, ev, W, above


def test_generated_time_and_dalitz_moments(toys):
    """Mean measured decay time and mean s12, s13 against quadrature of the
    model: the t moments come from closed forms (int t e^{-at} dt = 1/a^2 for
    each exponential of the rate), the Dalitz sums from a fine grid."""
    desc, th, ev, W, above = toys
    assert above == 0 and np.isfinite(ev).all()
    m = T.TDDP(dict(desc, grid=[512, 512]))
    c12, c13, _ = m.dal.grid_cells()
    G = 1.0 / m.tau
    x, y = th[-2], th[-1]
    with torch.no_grad():
        A, Ab = m.amplitudes(common.as_t(th), common.as_t(c12), common.as_t(c13))
    a2, b2 = (A.abs() ** 2).numpy(), (Ab.abs() ** 2).numpy()
    z = (A.conj() * Ab).numpy()
    # zeroth and first t moments of e^{-Gt} cosh, cos, sinh, sin
    ap, am, ac = G * (1 - y), G * (1 + y), G * (1 - 1j * x)
    m0 = (0.5 * (1 / ap + 1 / am), (1 / ac).real, 0.5 * (1 / ap - 1 / am), (1 / ac).imag)
    m1 = (0.5 * (1 / ap ** 2 + 1 / am ** 2), (1 / ac ** 2).real, 0.5 * (1 / ap ** 2 - 1 / am ** 2), (1 / ac ** 2).imag)

    def moment(mm):
        return 0.5 * ((a2 + b2) * mm[0] + (a2 - b2) * mm[1] - 2 * z.real * mm[2] - 2 * z.imag * mm[3])

    w0, w1 = moment(m0), moment(m1)
    checks = [(ev[2], w1.sum() / w0.sum()), (ev[0], (w0 * c12).sum() / w0.sum()), (ev[1], (w0 * c13).sum() / w0.sum())]
    for sample, expect in checks:
        se = sample.std() / math.sqrt(sample.size)
        assert abs(sample.mean() - expect) < 4.0 * se, (sample.mean(), expect, se)


def test_generation_is_per_event(toys):
    desc, th, ev, W, above = toys
    head, W2, _ = T.generate(th, desc, 300, seed=21, fit=1, W=W)
    assert W2 == W and np.array_equal(head, ev[:, :300])
    assert T.TDDP(desc).dal.inside(ev[0], ev[1]).all()
