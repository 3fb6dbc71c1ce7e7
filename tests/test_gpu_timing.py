"""Kernel timing (fn_model_timing / fn_model_kernel_time): timed event-pass
launches go through a different dispatch call (one that records the kernel's
own start and end into HIP events), so every model kind is checked to give
bitwise the same NLL and gradient with every launch timed as untimed, and to
report one positive duration per timed launch."""
import numpy as np
import pytest

import synth
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def _check(m, th, ev, calls=3):
    ref = [m.nll(th, ev, grad=g) for g in (False, True)]
    m.set_timing(True, 1)
    m.kernel_time()  # reset
    for _ in range(calls):
        v0 = m.nll(th, ev)
        v1, g1 = m.nll(th, ev, grad=True)
        assert v0 == ref[0]
        assert v1 == ref[1][0] and np.array_equal(g1, ref[1][1])
    ms, launches = m.kernel_time()
    m.set_timing(False)
    assert launches == 2 * calls, launches
    assert ms > 0.0 and np.isfinite(ms)
    # sampled: every other launch
    m.set_timing(True, 2)
    for _ in range(calls):
        m.nll(th, ev, grad=True)
    _, launches = m.kernel_time()
    m.set_timing(False)
    assert launches == (calls + 1) // 2, launches
    return ms / launches


def test_timed_launches_match_untimed():
    from paper_1710_08826_amd import Model
    cases = [
        ("mix1d", synth.mix1d_desc(), synth.mix1d_truth(), synth.mix1d_events(50_000, seed=81), None),
        ("dalitz3", synth.dalitz_desc(), synth.dalitz_truth(), synth.dalitz_events(30_000, seed=82), None),
        ("dalitz3 free", synth.dalitz_desc(free_lineshapes=True), synth.dalitz_truth(free_lineshapes=True),
         synth.dalitz_events(30_000, seed=83), None),
        ("tddp3", synth.tddp3_desc(), synth.tddp3_truth(), synth.tddp3_events(20_000, seed=84), None),
        ("td4", synth.td4_desc(), synth.td4_truth(), synth.td4_events(20_000, seed=85),
         synth.td4_phase_space(50_000, seed=86)),
    ]
    for name, desc, th, x, mc in cases:
        say("timing", name)
        m = Model(desc)
        if mc is not None:
            m.set_norm_sample(to_dev(mc))
        per = _check(m, th, to_dev(x))
        say("  ms per timed launch", per)


def test_empty_sample_is_not_timed():
    from paper_1710_08826_amd import Model
    import torch
    m = Model(synth.dalitz_desc())
    ev = torch.zeros((2, 0), dtype=torch.float64, device="cuda")
    m.set_timing(True, 1)
    m.nll(synth.dalitz_truth(), ev, grad=True)
    assert m.kernel_time() == (0.0, 0)
    m.set_timing(False)


def test_span_mode_counts_graph_replays_and_keeps_results():
    """Span mode (dalitz3): every launch measures itself on the device, also
    inside captured graphs; results are bitwise the untimed ones, one span per
    launch (direct calls and graph replays), each span positive and of the
    order of the event-timed duration; other model kinds refuse the mode."""
    import torch
    from paper_1710_08826_amd import FitNLLError, Model
    for free in (False, True):
        say("span timing, free lineshapes", free)
        d = synth.dalitz_desc(free_lineshapes=free)
        th = synth.dalitz_truth(free_lineshapes=free)
        m = Model(d)
        ev = to_dev(synth.dalitz_events(200_000, seed=87))
        ref = m.nll(th, ev, grad=True)
        ms_ev = _check(m, th, ev)
        m.set_timing(True, span=True)
        v, g = m.nll(th, ev, grad=True)
        assert v == ref[0] and np.array_equal(g, ref[1])
        tdev = torch.from_numpy(th).cuda()
        out = torch.empty(1 + m.n_params, dtype=torch.float64, device="cuda")
        s = torch.cuda.Stream()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=s, capture_error_mode="thread_local"):
            m.nll_async(tdev, ev, out, True)
        replays = 7
        for _ in range(replays):
            graph.replay()
        torch.cuda.synchronize()
        assert out[0].item() == ref[0] and np.array_equal(out[1:].cpu().numpy(), ref[1])
        ms, launches = m.kernel_time()
        assert launches == 1 + replays, launches
        per = ms / launches
        say("  span ms per launch", per, "event-timed", ms_ev)
        assert 0.0 < per < 3.0 * ms_ev
        assert m.kernel_time() == (0.0, 0)  # reset by the query
        m.set_timing(False)
        m.nll(th, ev, grad=True)
        assert m.kernel_time() == (0.0, 0)
    mm = Model(synth.mix1d_desc())
    with pytest.raises(FitNLLError, match="span"):
        mm.set_timing(True, span=True)
