"""Seeded synthetic inputs shared by the CPU oracle tests and the device library.

Holds random-number generation and sampling only; no part of the likelihood.
"""
from .philox import philox4x32, uniforms, uniforms_at, key_from_seed  # noqa: F401
from .samplers import (  # noqa: F401
    BASE_SEED, CONFIG0_TRUTH, CONFIG0_RANGE, DALITZ_MASSES, DALITZ_RESONANCES,
    mix1d_events, lognormal_sizes, dalitz_events, dalitz_box,
)
from .workloads import mix1d_desc, mix1d_truth, dalitz_desc, dalitz_truth  # noqa: F401,E402
from .td4 import (  # noqa: F401,E402
    TD4_MASSES, TD4_TAU, TD4_SIGMA_T, td4_desc, td4_truth, td4_phase_space, td4_events,
    td4_split_desc, td4_split_truth,
)
from .tddp3 import (  # noqa: F401,E402
    TDDP_MASSES, TDDP_RESONANCES, TDDP_RESONANCES16, tddp3_desc, tddp3_truth, tddp3_events,
    tddp3_desc16, tddp3_truth16,
)
