"""The oracle's arithmetic is float64 whatever torch's default dtype is: each
model's NLL and gradient are bitwise the same with the default set to float32
(the interpreter's own default, as in bench.py's CPU baseline) and to float64
(what tests/conftest.py sets)."""
import numpy as np
import pytest
import torch

import synth
from oracle import dalitz3 as OD, mix1d as OM, td4 as OT, tddp3 as OP


def cases():
    x = synth.mix1d_events(300, seed=1)
    yield "mix1d", lambda: OM.nll_grad(np.array(synth.CONFIG0_TRUTH) * 1.02, x, OM.config0_desc())
    d = OD.config1_desc(grid=(32, 32), free_lineshapes=True)
    ev = synth.dalitz_events(200, seed=2)
    yield "dalitz3", lambda: OD.nll_grad(OD.truth_theta(d) * 1.01, ev, d)
    dp = OP.pipipi0_desc(grid=(16, 16))
    evp = synth.tddp3_events(200, seed=3, sigma_t=dp["sigma_t"])
    yield "tddp3", lambda: OP.nll_grad(OP.truth_theta(x=0.02, y=0.01), evp, dp)
    mc = synth.td4_phase_space(500, seed=4)
    ev4 = synth.td4_events(200, seed=5)
    for desc, th in ((synth.td4_desc(), synth.td4_truth()), (synth.td4_split_desc(), synth.td4_split_truth())):
        yield "td4", (lambda desc=desc, th=th: OT.nll_grad(th, ev4, mc, desc))


@pytest.mark.parametrize("name,fn", list(cases()))
def test_oracle_independent_of_default_dtype(name, fn):
    saved = torch.get_default_dtype()
    try:
        torch.set_default_dtype(torch.float64)
        v64, g64 = fn()
        torch.set_default_dtype(torch.float32)
        v32, g32 = fn()
    finally:
        torch.set_default_dtype(saved)
    assert v64 == v32 and np.array_equal(g64, g32), (name, v64 - v32)
