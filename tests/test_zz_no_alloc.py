"""The allocation-free NLL entry point (fn_nll_async_noalloc, partial rows in
the library's static scratch array) against fn_nll_async on the same models,
events and parameters: bitwise equal outputs on two calls in a row, the
second with a smaller input, for every model kind, with and without the
gradient; the first call of a fresh model also builds the cached
normalization through the scratch array.  A request larger than the array is
rejected with FN_E_INVALID and leaves later calls working."""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def pair(desc, mc=None):
    """Two fresh models of one description: one for each entry point."""
    from paper_1710_08826_amd import Model
    ms = [Model(desc), Model(desc)]
    if mc is not None:
        for m in ms:
            m.set_norm_sample(mc)
    return ms


def compare(m_ref, m_na, th, ev_big, n_small, label):
    P = m_ref.n_params
    tdev = torch.from_numpy(np.asarray(th, dtype=np.float64)).cuda()
    for with_grad in (True, False):
        for n in (ev_big.shape[1], n_small):
            ev = ev_big[:, :n]
            say(f"noalloc {label}: n = {n}, grad = {with_grad}")
            o_ref = torch.full((1 + P,), -1.0, dtype=torch.float64, device="cuda")
            o_na = torch.full((1 + P,), -2.0, dtype=torch.float64, device="cuda")
            if not with_grad:
                o_na[1:] = -1.0  # gradient entries are left untouched by both
            m_ref.nll_async(tdev, ev, o_ref, with_grad=with_grad)
            m_na.nll_async_noalloc(tdev, ev, o_na, with_grad=with_grad)
            torch.cuda.synchronize()
            a, b = o_ref.cpu().numpy(), o_na.cpu().numpy()
            assert np.isfinite(a[0]), a[0]
            assert np.array_equal(a, b), (label, n, with_grad, a[:4], b[:4])


def test_dalitz_cached_normalization():
    desc = synth.dalitz_desc()
    m_ref, m_na = pair(desc)
    ev = to_dev(synth.dalitz_events(1_000_000, seed=71))
    compare(m_ref, m_na, synth.dalitz_truth() * 1.01, ev, 100_003, "dalitz3 cached M")


def test_dalitz_free_lineshapes():
    desc = synth.dalitz_desc(grid=(256, 256), free_lineshapes=True)
    m_ref, m_na = pair(desc)
    ev = to_dev(synth.dalitz_events(200_000, seed=72))
    th = synth.dalitz_truth(free_lineshapes=True) * (1.0 + 0.01 * np.cos(np.arange(4 * 8)))
    compare(m_ref, m_na, th, ev, 30_001, "dalitz3 free lineshapes")


def test_mix1d():
    m_ref, m_na = pair(synth.mix1d_desc())
    ev = to_dev(synth.mix1d_events(100_000, seed=73))
    compare(m_ref, m_na, np.array(synth.CONFIG0_TRUTH) * 1.03, ev, 5_001, "mix1d")


def test_td4():
    desc = synth.td4_desc()
    mc = to_dev(synth.td4_phase_space(50_000, seed=74))
    m_ref, m_na = pair(desc, mc)
    ev = to_dev(synth.td4_events(20_000, seed=75))
    compare(m_ref, m_na, synth.td4_truth(), ev, 3_001, "td4")


def test_tddp3():
    desc = synth.tddp3_desc(grid=(256, 256))
    m_ref, m_na = pair(desc)
    ev = to_dev(synth.tddp3_events(50_000, 76, desc["tau"], desc["sigma_t"]))
    compare(m_ref, m_na, synth.tddp3_truth(x=0.02, y=0.03), ev, 7_001, "tddp3")


def test_too_large_is_rejected_and_later_calls_work():
    from paper_1710_08826_amd import Model
    from paper_1710_08826_amd._lib import FitNLLError
    desc = dict(synth.dalitz_desc(), chunk=256)
    m = Model(desc)
    P = m.n_params
    # 2^21 doubles hold fewer than 2^21 / (1 + P) rows of 1 + P doubles
    n_big = 256 * ((1 << 21) // (1 + P) + 2)
    say(f"noalloc rejects n = {n_big}")
    ev = torch.zeros((2, n_big), dtype=torch.float64, device="cuda")
    tdev = torch.from_numpy(synth.dalitz_truth()).cuda()
    out = torch.zeros(1 + P, dtype=torch.float64, device="cuda")
    with pytest.raises(FitNLLError) as ei:
        m.nll_async_noalloc(tdev, ev, out)
    assert ei.value.status == -1 and "scratch" in str(ei.value)
    del ev
    small = to_dev(synth.dalitz_events(10_000, seed=77))
    ref = torch.zeros(1 + P, dtype=torch.float64, device="cuda")
    m.nll_async(tdev, small, ref)
    m.nll_async_noalloc(tdev, small, out)
    torch.cuda.synchronize()
    assert np.array_equal(ref.cpu().numpy(), out.cpu().numpy())
