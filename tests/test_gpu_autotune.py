"""Autotuner of the summation chunk and, for the Dalitz passes, of the events
per thread and loop iteration: among the timed candidates within 2% of the
fastest it takes one event per thread if any, then the largest chunk; the
choice becomes the model's, and the evaluations that follow still match the
oracle; an invalid call leaves the model's choice alone.  Two events per
thread give bitwise the sums of one (each thread adds its events in index
order either way)."""
import ctypes as C

import numpy as np
import pytest

import synth
from oracle import dalitz3 as OD, mix1d as OM
from tests.gpu_util import grad_close, rel_close, say, to_dev

pytestmark = pytest.mark.gpu


def _info_chunk(m):
    p, o, c = C.c_int32(), C.c_int32(), C.c_int32()
    assert m._lib.fn_model_info(m._h, C.byref(p), C.byref(o), C.byref(c)) == 0
    return c.value


def test_dalitz_autotune_then_parity():
    from paper_1710_08826_amd import Model
    say("autotune dalitz")
    d = OD.config1_desc()
    th = OD.truth_theta(d)
    m = Model(d)
    x = synth.dalitz_events(200_000, seed=51)
    ev = to_dev(x)
    chunk, table = m.autotune(th, ev, reps=10)
    full = m.tune_table
    say("  chunk", chunk, "events per thread", m.events_per_thread, {k: round(v, 1) for k, v in full.items()})
    # candidates: the powers of two 256..16384, and the multiples of 256 that
    # give j x (compute units) workgroups for the 200k events, j = 1..8
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count

    def ceil_div(a, b):
        return -(-a // b)

    pow2 = {256 << k for k in range(7)}
    multiples = {max(256, ceil_div(ceil_div(200_000, j * cus), 256) * 256) for j in range(1, 9)}
    assert set(table) == pow2 | multiples, sorted(table)
    assert set(full) == {(c, e) for c in table for e in (1, 2)}, sorted(full)
    assert all(np.isfinite(v) and v > 0 for v in full.values())
    fastest = min(full.values())
    tie = {k for k, v in full.items() if v <= 1.02 * fastest}
    ept = 1 if any(e == 1 for _, e in tie) else 2
    assert m.events_per_thread == ept
    assert chunk == max(c for c, e in tie if e == ept)
    assert table == {c: t for (c, e), t in full.items() if e == ept}
    assert m.chunk == chunk == _info_chunk(m)
    v, g = m.nll(th, ev, grad=True)
    vo, go = OD.nll_grad(th, x, d)
    assert rel_close(v, vo, 1e-12), (v, vo)
    ok, r = grad_close(g, go, 1e-10)
    assert ok, r


def test_mix1d_autotune_and_errors():
    from paper_1710_08826_amd import FitNLLError, Model
    say("autotune mix1d")
    d = OM.config0_desc()
    th = np.array(synth.CONFIG0_TRUTH)
    m = Model(d)
    before = m.chunk
    with pytest.raises(FitNLLError):
        m.autotune(th, to_dev(synth.mix1d_events(0, seed=1)))
    assert _info_chunk(m) == before
    x = synth.mix1d_events(100_000, seed=52)
    chunk, _ = m.autotune(th, to_dev(x), reps=5)
    assert _info_chunk(m) == chunk
    v, g = m.nll(th, to_dev(x), grad=True)
    vo, go = OM.nll_grad(th, x, d)
    assert rel_close(v, vo, 1e-12)
    ok, r = grad_close(g, go, 1e-10)
    assert ok, r


@pytest.mark.parametrize("free", [False, True])
def test_two_events_per_thread_bitwise(free):
    """Models that differ only in events per thread: NLL and gradient bitwise
    equal on a ragged size, a size below one workgroup's threads and one
    event, and equal to the oracle."""
    from paper_1710_08826_amd import FitNLLError, Model
    say("two events per thread, free lineshapes", free)
    d = synth.dalitz_desc(free_lineshapes=free)
    th0 = synth.dalitz_truth(free_lineshapes=free)
    th = th0 * (1.0 + 0.01 * np.cos(np.arange(th0.size)))
    m1 = Model(dict(d, chunk=1024))
    m2 = Model(dict(d, chunk=1024, events_per_thread=2))
    assert m2.events_per_thread == 2
    for n in (3 * 1024 + 517, 200, 1):
        x = synth.dalitz_events(n, seed=53 + n)
        ev = to_dev(x)
        v1, g1 = m1.nll(th, ev, grad=True)
        v2, g2 = m2.nll(th, ev, grad=True)
        assert v1 == v2 and (g1 == g2).all(), (n, v1, v2)
        assert m2.nll(th, ev) == m1.nll(th, ev)
    x = synth.dalitz_events(3 * 1024 + 517, seed=53 + 3 * 1024 + 517)
    v2, g2 = m2.nll(th, to_dev(x), grad=True)
    vo, go = OD.nll_grad(th, x, d)
    assert rel_close(v2, vo, 1e-12), (v2, vo)
    ok, r = grad_close(g2, go, 1e-9)
    assert ok, r
    with pytest.raises(FitNLLError, match="events_per_thread"):
        Model(dict(d, events_per_thread=3))
    with pytest.raises(FitNLLError, match="events_per_thread"):
        Model(dict(OM.config0_desc(), events_per_thread=2))
