"""Systematic-variation batches of the td4 model: every fit's NLL and gradient
equal the single-fit path's with the same fixed constants (bitwise) and the
oracle's (to 1e-12); batched fits converge, and a fit's result is the same
alone and inside the batch."""
import numpy as np
import pytest
import torch

import synth
from oracle import td4 as OT
from tests.gpu_util import grad_close, rel_close, say, to_dev

pytestmark = pytest.mark.gpu

DESC = synth.td4_desc()
TH = synth.td4_truth()
P = TH.size


def variation(fx, f):
    """Deterministic +- shifts of the fixed constants for fit f (f = 0: nominal)."""
    v = fx.copy()
    if f == 0:
        return v
    s = 1.0 if f % 2 else -1.0
    k = (f - 1) // 2 % 4
    if k == 0:
        v[2 * 3 + 2] += s * 0.0008       # rho(770) mass (r34 entry 1)
    elif k == 1:
        v[2 * 3 + 3] *= 1.0 + s * 0.05   # rho(770) width
    elif k == 2:
        v[3] *= 1.0 + s * 0.1            # phi(1020) width (r12 entry 1)
    else:
        v[-1] *= 1.0 + s * 0.1           # time resolution
    return v


def desc_for(fx):
    d = dict(DESC)
    d["r12"] = [{"L": e["L"], "m0": fx[2 * i], "w0": fx[2 * i + 1]} for i, e in enumerate(DESC["r12"])]
    o = 2 * len(DESC["r12"])
    d["r34"] = [{"L": e["L"], "m0": fx[o + 2 * i], "w0": fx[o + 2 * i + 1]} for i, e in enumerate(DESC["r34"])]
    d["sigma_t"] = fx[-1]
    return d


@pytest.fixture(scope="module")
def setup():
    from paper_1710_08826_amd import Model
    mc = synth.td4_phase_space(30_000, seed=61)
    m = Model(DESC)
    mcd = to_dev(mc)
    m.set_norm_sample(mcd)
    return m, mc, mcd


def thetas(F):
    return np.stack([TH * (1 + 0.04 * np.sin(np.arange(P) + f)) for f in range(F)])


def test_batched_nll_matches_single_and_oracle(setup):
    from paper_1710_08826_amd import Model, VariationBatch
    m, mc, mcd = setup
    F = 9
    fx0 = m.fixed()
    b = VariationBatch(m, F)
    for f in range(F):
        b.set_fixed(f, variation(fx0, f))
    ev = synth.td4_events(20_000, seed=62)
    evd = to_dev(ev)
    th = thetas(F)
    say("td4 vbatch nll")
    v, g = b.nll(th, evd, grad=True)
    v2 = b.nll(th, evd)
    assert np.all(np.abs(v2 - v) <= 1e-14 * np.abs(v))  # value-only kernel: same tree
    for f in range(F):
        single = Model(desc_for(variation(fx0, f)))
        single.set_norm_sample(mcd)
        vs, gs = single.nll(th[f], evd, grad=True)
        assert vs == v[f] and (gs == g[f]).all(), f
        if f in (0, 3, 8):
            vo, go = OT.nll_grad(th[f], ev, mc, desc_for(variation(fx0, f)))
            assert rel_close(v[f], vo, 1e-12), (f, v[f], vo)
            ok, r = grad_close(g[f], go, 1e-10)
            assert ok, (f, r.max())


# A well-conditioned fit: three amplitudes of distinct shapes, mixing large
# enough to constrain Abar, c_0 and cbar_0 fixed (they carry the global phase
# and scale and the relative phase that trades against a rotation of (x, y)).
SMALL = synth.td4_desc(r12=((0, 0.0, 0.0),))
SMALL["amps"] = [[0, 0, 0], [0, 1, 1], [0, 2, 0]]
SMALL_TH = np.array([0.5, 0.0, -0.3, 0.35, 0.2, 0.25, 1.0, 0.0, 0.8, 0.45, 0.35, -0.3, 0.2, 0.15])
SMALL_FREE = np.array([0, 0, 1, 1, 1, 1, 0, 0, 1, 1, 1, 1, 1, 1], np.int32)


def small_variation(fx, f):
    v = fx.copy()
    if f:
        s = 1.0 if f % 2 else -1.0
        k = (f - 1) // 2 % 3
        if k == 0:
            v[2 + 2] += s * 0.002          # rho(770) mass (r34 entry 1)
        elif k == 1:
            v[2 + 3] *= 1.0 + s * 0.05     # rho(770) width
        else:
            v[-1] *= 1.0 + s * 0.1         # time resolution
    return v


def test_batched_fits_converge_and_match_alone():
    """Events drawn from the model itself (oracle accept-reject); six variation
    fits from a common offset start."""
    from paper_1710_08826_amd import Model, VariationBatch
    Ps = SMALL_TH.size
    m = Model(SMALL)
    m.set_norm_sample(to_dev(synth.td4_phase_space(50_000, seed=65)))
    say("td4 generating model events")
    ev = to_dev(OT.generate(SMALL_TH, SMALL, 20_000, seed=66))
    F = 6
    fx0 = m.fixed()
    free = SMALL_FREE
    th0 = np.stack([SMALL_TH * (1 + 0.05 * np.sin(np.arange(Ps) + f)) for f in range(F)])
    th0[:, free == 0] = SMALL_TH[free == 0]
    b = VariationBatch(m, F)
    for f in range(F):
        b.set_fixed(f, small_variation(fx0, f))
    say("td4 vbatch fit F =", F)
    r = b.fit(th0, ev, free=free, tol=1e-7, max_iter=1000)
    say("status", r.status, "iters", r.iters, "evals", r.n_evals)
    assert (r.status == 2).all()
    assert (r.nll <= b.nll(th0, ev)).all()
    # the same minimum and errors as the host minimizer (nominal fit)
    ref = m.fit(th0[0], ev, free=free, tol=1e-7, max_iter=1000)
    say("host fit nll", ref.nll, "batch", r.nll[0])
    assert abs(r.nll[0] - ref.nll) < 1e-5
    sig = np.where(free == 1, ref.errors, 1.0)
    assert (np.abs(r.theta[0] - ref.theta) / sig).max() < 0.02
    assert np.allclose(r.errors[0][free == 1], ref.errors[free == 1], rtol=0.02)
    # the generation point lies within the statistical errors of the nominal fit
    pull = ((ref.theta - SMALL_TH) / sig)[free == 1]
    assert np.abs(pull).max() < 4.0, pull
    # fit 4 alone in a batch of one: same trajectory, same bits
    one = VariationBatch(m, 1)
    one.set_fixed(0, small_variation(fx0, 4))
    r1 = one.fit(th0[4:5], ev, free=free, tol=1e-7, max_iter=1000)
    assert r1.status[0] == 2 and r1.iters[0] == r.iters[4] and r1.n_evals[0] == r.n_evals[4]
    assert r1.nll[0] == r.nll[4] and (r1.theta[0] == r.theta[4]).all()
    # graph replay and plain launches give the same result
    r2 = one.fit(th0[4:5], ev, free=free, tol=1e-7, max_iter=1000, use_graph=False)
    assert r2.nll[0] == r1.nll[0] and (r2.theta[0] == r1.theta[0]).all()


def test_errors(setup):
    from paper_1710_08826_amd import FitNLLError, VariationBatch
    m, mc, mcd = setup
    b = VariationBatch(m, 2)
    fx = m.fixed()
    bad = fx.copy()
    bad[-1] = -1.0
    with pytest.raises(FitNLLError, match="sigma_t"):
        b.set_fixed(0, bad)
    with pytest.raises(FitNLLError):
        b.set_fixed(2, fx)
    with pytest.raises(ValueError):
        b.nll(TH[None, :], to_dev(synth.td4_events(10, seed=64)))
