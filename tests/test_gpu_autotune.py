"""Chunk autotuner: the chosen chunk is the largest of the timed candidates
within 2% of the fastest,
becomes the model's chunk, and the evaluations that follow still match the
oracle; an invalid call leaves the model's chunk alone."""
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
    say("  chunk", chunk, {k: round(v, 1) for k, v in table.items()})
    # candidates: the powers of two 256..16384, and the multiples of 256 that
    # give j x (compute units) workgroups for the 200k events, j = 1..8
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count

    def ceil_div(a, b):
        return -(-a // b)

    pow2 = {256 << k for k in range(7)}
    multiples = {max(256, ceil_div(ceil_div(200_000, j * cus), 256) * 256) for j in range(1, 9)}
    assert set(table) == pow2 | multiples, sorted(table)
    assert chunk in table and table[chunk] <= 1.02 * min(table.values())
    assert all(table[c] > 1.02 * min(table.values()) for c in table if c > chunk)
    assert all(np.isfinite(v) and v > 0 for v in table.values())
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
