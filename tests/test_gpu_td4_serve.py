"""Continuous serving of systematic-variation fits of the four-body model
(fn_vbatch_serve): requests with their own fixed constants and start points
arrive over time, are admitted into free slots at step boundaries and share
the events passes of the fits already running; every result is bitwise the
same as the request run alone in a batch of one, and admissions happen while
other fits are running."""
import numpy as np
import pytest

import synth
from oracle import td4 as OT
from tests.gpu_util import say, to_dev
from tests.test_gpu_td4_batch import SMALL, SMALL_FREE, SMALL_TH, small_variation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    from paper_1710_08826_amd import Model
    m = Model(SMALL)
    m.set_norm_sample(to_dev(synth.td4_phase_space(30_000, seed=165)))
    say("td4 serve: generating model events")
    ev = to_dev(OT.generate(SMALL_TH, SMALL, 10_000, seed=166))
    return m, ev


def requests(m, n):
    fx0 = m.fixed()
    Ps = SMALL_TH.size
    out = []
    for i in range(n):
        th0 = SMALL_TH * (1 + 0.04 * np.sin(np.arange(Ps) + 3 * i))
        th0[SMALL_FREE == 0] = SMALL_TH[SMALL_FREE == 0]
        fixed = None if i % 4 == 0 else small_variation(fx0, i % 7)
        out.append((100 + i, 0.0005 * i, fixed, th0))
    return out


def test_served_results_equal_alone(setup):
    from paper_1710_08826_amd import VariationBatch
    m, ev = setup
    reqs = requests(m, 10)
    b = VariationBatch(m, 3)  # fewer slots than requests: later ones wait and are admitted as slots free
    say("td4 serve: 10 requests, 3 slots")
    r = b.serve(reqs, ev, free=SMALL_FREE, tol=1e-7, max_iter=1000, poll_every=2)
    say("status", r["status"], "iters", r["iters"])
    assert (r["status"] == 2).all()
    assert list(r["id"]) == [q[0] for q in reqs]
    assert (r["t_done"] > r["t_admit"]).all()
    assert (r["t_admit"] >= np.array([q[1] for q in reqs]) - 1e-9).all()
    # continuous batching: some request was admitted while another was running
    overlap = any(r["t_admit"][j] > r["t_admit"][i] and r["t_admit"][j] < r["t_done"][i]
                  for i in range(len(reqs)) for j in range(len(reqs)) if i != j)
    assert overlap
    # with 3 slots, at most 3 requests run at any admission time
    for j in range(len(reqs)):
        t = r["t_admit"][j]
        assert ((r["t_admit"] <= t) & (r["t_done"] > t)).sum() <= 3
    for i in (0, 3, 9):
        _, _, fixed, th0 = reqs[i]
        one = VariationBatch(m, 1)
        one.set_fixed(0, fixed)
        r1 = one.fit(th0[None, :], ev, free=SMALL_FREE, tol=1e-7, max_iter=1000)
        assert r1.status[0] == 2
        assert r1.nll[0] == r["nll"][i] and (r1.theta[0] == r["theta"][i]).all(), i
        assert r1.iters[0] == r["iters"][i] and r1.n_evals[0] == r["n_evals"][i]
        assert (r1.errors[0] == r["errors"][i]).all()


def test_serve_rejects_bad_requests(setup):
    from paper_1710_08826_amd import FitNLLError, VariationBatch
    m, ev = setup
    b = VariationBatch(m, 2)
    reqs = requests(m, 2)
    bad = m.fixed()
    bad[-1] = -1.0
    with pytest.raises(FitNLLError, match="sigma_t"):
        b.serve([reqs[0], (7, 0.0, bad, reqs[1][3])], ev, free=SMALL_FREE)
    with pytest.raises(FitNLLError, match="arrival"):
        b.serve([(8, -1.0, None, reqs[1][3])], ev, free=SMALL_FREE)
    # an empty request list returns at once
    r = b.serve([], ev)
    assert r["status"].size == 0
