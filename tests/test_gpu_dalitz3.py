"""Parity of the device Dalitz-plot NLL, normalization and adjoint gradient
with the oracle (fixed lineshapes with the cached normalization matrix, and
free masses/widths with the full grid every call)."""
import numpy as np
import pytest
import torch

import synth
from oracle import common, dalitz3 as OD
from tests.gpu_util import grad_close, rel_close, say, to_dev

pytestmark = pytest.mark.gpu

D1 = OD.config1_desc()
TH1 = OD.truth_theta(D1)
D3 = OD.config1_desc(free_lineshapes=True)
TH3 = OD.truth_theta(D3)


def offset(th):
    return th + 0.03 * np.sin(np.arange(th.size) + 1.0) * np.maximum(np.abs(th), 0.05)


@pytest.fixture(scope="module")
def cells1():
    return OD.Dalitz(D1).grid_cells()


@pytest.fixture(scope="module")
def m1():
    from paper_1710_08826_amd import Model
    return Model(D1)


@pytest.fixture(scope="module")
def m3():
    from paper_1710_08826_amd import Model
    return Model(D3)


def test_norm_matches_oracle_grid(m1, m3, cells1):
    say("dalitz norm")
    for th in (TH1, offset(TH1)):
        I, dI = m1.norm(th)
        Io = OD.norm_value(OD.Dalitz(D1), th, cells1)
        assert rel_close(I, Io, 1e-12), (I, Io)
    th3 = offset(TH3)
    I3, _ = m3.norm(th3)
    assert rel_close(I3, OD.norm_value(OD.Dalitz(D3), th3, cells1), 1e-12)


@pytest.mark.parametrize("n", [1, 1000, 3 * 2048 + 17, 100_000])
def test_config1_nll_and_coefficient_gradient(m1, cells1, n):
    say("dalitz config1 n =", n)
    ev = synth.dalitz_events(n, seed=31)
    evd = to_dev(ev)
    for th in (TH1, offset(TH1)):
        v, g = m1.nll(th, evd, grad=True)
        vo, go = OD.nll_grad(th, ev, D1, cells1)
        assert rel_close(v, vo, 1e-12), (v, vo, (v - vo) / vo)
        ok, r = grad_close(g, go, 1e-10)
        assert ok, r
        assert rel_close(m1.nll(th, evd), v, 1e-14)  # NLL-only kernel agrees


@pytest.mark.parametrize("n", [1, 5000, 2 * 4096 + 5])
def test_config3_nll_and_full_gradient(m3, cells1, n):
    say("dalitz config3 n =", n)
    ev = synth.dalitz_events(n, seed=32)
    evd = to_dev(ev)
    th = offset(TH3)
    v, g = m3.nll(th, evd, grad=True)
    vo, go = OD.nll_grad(th, ev, D3, cells1)
    assert rel_close(v, vo, 1e-12), (v, vo)
    ok, r = grad_close(g, go, 1e-9)
    assert ok, r


def test_config3_gradient_vs_central_fd(m3):
    """Adjoint against central differences of the oracle NLL (coarse grid so
    the 2P oracle evaluations stay fast)."""
    from paper_1710_08826_amd import Model
    d = OD.config1_desc(grid=(128, 128), free_lineshapes=True)
    m = Model(d)
    ev = synth.dalitz_events(4000, seed=33)
    th = offset(OD.truth_theta(d))
    _, g = m.nll(th, to_dev(ev), grad=True)
    cells = OD.Dalitz(d).grid_cells()
    fd = common.central_fd(lambda t: OD.nll(t, ev, d, cells), th, rel_step=1e-6)  # config 3's h = 1e-6
    ok, r = grad_close(g, fd, 1e-6)
    assert ok, r


@pytest.mark.parametrize("grid", [(37, 23), (1200, 7), (1, 1)])
def test_free_lineshapes_on_uneven_grids(grid):
    """The list of inside cells on grids where it is shorter than one
    workgroup's 1024 cells, spans many grid columns per workgroup (columns of
    a few cells each), or holds the single centre cell: NLL, normalization
    and full gradient against the oracle on the same grid."""
    from paper_1710_08826_amd import Model
    say("uneven grid", grid)
    d = OD.config1_desc(grid=grid, free_lineshapes=True)
    m = Model(d)
    cells = OD.Dalitz(d).grid_cells()
    assert cells[0].size >= 1
    ev = synth.dalitz_events(3000, seed=36)
    th = offset(OD.truth_theta(d))
    v, g = m.nll(th, to_dev(ev), grad=True)
    vo, go = OD.nll_grad(th, ev, d, cells)
    assert rel_close(v, vo, 1e-12), (v, vo)
    ok, r = grad_close(g, go, 1e-10)
    assert ok, r
    I, _ = m.norm(th)
    assert rel_close(I, OD.norm_value(OD.Dalitz(d), th, cells), 1e-12)


def test_full_size_config1(m1, cells1):
    """1M events, the benchmark's configuration."""
    ev = synth.dalitz_events(1_000_000, seed=34)
    th = offset(TH1)
    v, g = m1.nll(th, to_dev(ev), grad=True)
    vo, go = OD.nll_grad(th, ev, D1, cells1)
    assert rel_close(v, vo, 1e-12), (v, vo)
    ok, r = grad_close(g, go, 1e-10)
    assert ok, r


def test_full_size_config3(m3, cells1):
    """4M events with masses and widths free (32 parameters, the full grid
    every call), at the model's default chunk as the benchmark runs it."""
    ev = synth.dalitz_events(4_000_000, seed=37)
    th = offset(TH3)
    say("dalitz config3 full size: device")
    v, g = m3.nll(th, to_dev(ev), grad=True)
    say("dalitz config3 full size: oracle")
    vo, go = OD.nll_grad(th, ev, D3, cells1)
    assert rel_close(v, vo, 1e-12), (v, vo)
    ok, r = grad_close(g, go, 1e-9)
    assert ok, r


def test_presummed_level2(cells1):
    """2.5M events at chunk 1024 give 2442 event rows of 17 sums (332 KB), more
    than the level-2 step reads through one compute unit: workgroups of 16 rows
    pre-sum them first.  The result matches the oracle, and a level-2 step over
    the 154 rows of chunk 16384 (no pre-summation), within rounding."""
    from paper_1710_08826_amd import Model
    ev = synth.dalitz_events(2_500_000, seed=38)
    evd = to_dev(ev)
    th = offset(TH1)
    say("dalitz presummed level 2: device")
    m_small = Model(dict(D1, chunk=1024))
    m_big = Model(dict(D1, chunk=16384))
    v, g = m_small.nll(th, evd, grad=True)
    vb, gb = m_big.nll(th, evd, grad=True)
    assert m_small.chunk == 1024 and m_big.chunk == 16384
    assert rel_close(v, vb, 1e-13), (v, vb)
    ok, r = grad_close(g, gb, 1e-12)
    assert ok, r
    say("dalitz presummed level 2: oracle")
    vo, go = OD.nll_grad(th, ev, D1, cells1)
    assert rel_close(v, vo, 1e-12), (v, vo)
    ok, r = grad_close(g, go, 1e-10)
    assert ok, r


def test_eval_matches_oracle_density(m1, cells1):
    ev = synth.dalitz_events(2000, seed=35)
    p = m1.eval(TH1, to_dev(ev)).cpu().numpy()
    model = OD.Dalitz(D1)
    with torch.no_grad():
        po = model.density_unnorm(common.as_t(TH1), common.as_t(ev[0]), common.as_t(ev[1])).numpy()
    po = po / OD.norm_value(model, TH1, cells1)
    assert np.allclose(p, po, rtol=1e-12, atol=0)


def test_bitwise_repeatable(m3):
    ev = to_dev(synth.dalitz_events(50_000, seed=36))
    th = offset(TH3)
    ref = m3.nll(th, ev, grad=True)
    for _ in range(5):
        v, g = m3.nll(th, ev, grad=True)
        assert v == ref[0] and np.array_equal(g, ref[1])


def test_back_to_back_async_evaluations(m1):
    """Evaluations queued without waiting, alternating parameters, sample
    sizes (so numbers of partial-sum rows) and gradient level, each equal
    bitwise to the same evaluation run on its own."""
    say("dalitz back-to-back async")
    sizes = [100_000, 3 * 2048 + 17, 1, 50_000]
    evs = [to_dev(synth.dalitz_events(n, seed=40 + i)) for i, n in enumerate(sizes)]
    ths = [torch.from_numpy(th).cuda() for th in (TH1, offset(TH1))]
    P = m1.n_params
    ref = {}
    for e in range(len(evs)):
        for t in range(2):
            for g in (True, False):
                out = torch.empty(1 + P, dtype=torch.float64, device="cuda")
                m1.nll_async(ths[t], evs[e], out, g)
                torch.cuda.synchronize()
                ref[e, t, g] = out.cpu().numpy()
    plan = [(i % len(evs), (i // 2) % 2, i % 3 != 0) for i in range(48)]
    outs = torch.empty(len(plan), 1 + P, dtype=torch.float64, device="cuda")
    for i, (e, t, g) in enumerate(plan):
        m1.nll_async(ths[t], evs[e], outs[i], g)
    torch.cuda.synchronize()
    got = outs.cpu().numpy()
    for i, (e, t, g) in enumerate(plan):
        k = 1 + P if g else 1
        assert np.array_equal(got[i, :k], ref[e, t, g][:k]), (i, e, t, g)


def test_empty_sample(m1, m3):
    """No events: NLL = 0 and, for free lineshapes too, a zero gradient
    (N ln I and N dI/I vanish); the level-2 step still runs on its own."""
    say("dalitz empty sample")
    empty = torch.zeros((2, 0), dtype=torch.float64, device="cuda")
    for m, th in ((m1, TH1), (m3, offset(TH3))):
        v, g = m.nll(th, empty, grad=True)
        assert v == 0.0 and not np.any(g), (v, g)


def test_events_check(m1):
    ev = synth.dalitz_events(3000, seed=37)
    assert m1.check_events(to_dev(ev)) == 0
    ev[:, 5] = [0.3, 1.0]      # below the s12 threshold
    ev[:, 6] = [2.9, 2.9]      # inside the box, outside the region
    assert m1.check_events(to_dev(ev)) == 2


def test_invalid_model_descriptions():
    from paper_1710_08826_amd import FitNLLError, Model
    bad = [dict(D1, kind="nope"), dict(D1, grid=[0, 10]), dict(D1, resonances=[]),
           dict(D1, resonances=[{"pair": "14", "L": 1, "m0": 1.0, "w0": 0.1}]),
           dict(D1, chunk=1000)]
    for d in bad:
        with pytest.raises(FitNLLError):
            Model(d)
