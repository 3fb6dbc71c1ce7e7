"""Continuous-batching server: every request completes, results equal the
request served alone (bitwise) and the single-fit minimum, the memory budget
queues requests and rejects ones that can never fit."""
import numpy as np
import pytest

import synth
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

TRUTH = synth.mix1d_truth()
START = TRUTH * np.array([1.1, 0.9, 1.15, 0.95])


def requests(n, seed=31, rate=2000.0):
    sizes = synth.lognormal_sizes(n, lo=1000, hi=60_000, seed=seed)
    u, _ = synth.uniforms(n, synth.key_from_seed(seed, 1), 3)
    arrivals = np.cumsum(-np.log1p(-u) / rate)
    return [dict(id=i, n_events=int(sizes[i]), seed=seed, fit=i, theta_gen=TRUTH, theta0=START,
                 arrival_s=float(arrivals[i])) for i in range(n)]


@pytest.fixture(scope="module")
def model():
    from paper_1710_08826_amd import Model
    return Model(synth.mix1d_desc())


def test_serve_mix_equals_alone(model):
    from paper_1710_08826_amd import Server
    reqs = requests(48)
    srv = Server(model, max_slots=16, max_events_per_fit=60_000, budget_bytes=64 << 20)
    srv.submit(reqs)
    n = srv.run(poll_every=2)
    res = {r.id: r for r in srv.results()}
    say("served", n, "p50 latency", np.median([r.latency for r in res.values()]))
    assert n == 48 and all(r.status == 2 for r in res.values())
    assert all(r.t_admit >= r.t_arrival - 1e-9 and r.t_done > r.t_admit for r in res.values())
    for i in (0, 17, 47):
        alone = Server(model, max_slots=1, max_events_per_fit=60_000, budget_bytes=8 << 20)
        q = dict(reqs[i], arrival_s=0.0)
        alone.submit([q])
        alone.run(poll_every=3)
        (a,) = alone.results()
        assert a.status == 2 and np.array_equal(a.theta, res[i].theta) and a.nll == res[i].nll
        assert a.iters == res[i].iters


def test_serve_matches_single_fit(model):
    from paper_1710_08826_amd import Server, generate_mix1d
    reqs = requests(6, seed=32)
    srv = Server(model, max_slots=4, max_events_per_fit=60_000, budget_bytes=16 << 20)
    srv.submit(reqs)
    srv.run(poll_every=4)
    for r in srv.results():
        q = reqs[r.id]
        ev = generate_mix1d(q["n_events"], q["seed"], q["fit"], TRUTH)
        one = model.fit(START, ev)
        assert (np.abs(r.theta - one.theta) < 2e-3 * one.errors).all(), (r.theta, one.theta)


def test_budget_queues_and_rejects(model):
    from paper_1710_08826_amd import Server
    from paper_1710_08826_amd._lib import FN_E_BUDGET
    reqs = requests(12, seed=33)
    for q in reqs:
        q["n_events"] = 20_000
        q["arrival_s"] = 0.0
    reqs.append(dict(reqs[0], id=99, n_events=50_000))
    # room for two 20k-event requests (160 kB each) at a time; the 50k one
    # (400 kB) exceeds the whole budget and can never be admitted
    srv = Server(model, max_slots=8, max_events_per_fit=60_000, budget_bytes=2 * 20_000 * 8 + 1024)
    srv.submit(reqs)
    srv.run(poll_every=2)
    res = {r.id: r for r in srv.results()}
    assert res[99].status == FN_E_BUDGET
    assert all(res[i].status == 2 for i in range(12))
    admits = sorted(res[i].t_admit for i in range(12))
    dones = sorted(res[i].t_done for i in range(12))
    # never more than two admitted and unfinished at once
    for t in admits:
        live = sum(1 for i in range(12) if res[i].t_admit <= t < res[i].t_done)
        assert live <= 2
