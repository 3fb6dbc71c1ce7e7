"""MI355X-native unbinned maximum-likelihood engine (GooFit 2.0's fitting
hot path): HIP kernels for gfx950 behind the C ABI in include/fitnll.h, with a
thin Python binding.  Import is cheap; the shared library loads on first use.
"""
from ._lib import FitNLLError, load  # noqa: F401

__all__ = ["FitNLLError", "load", "Model", "NLLFunction", "FitResult", "Batch", "VariationBatch", "generate_mix1d",
           "Server"]


def __getattr__(name):
    if name in ("Model", "NLLFunction", "FitResult", "context", "Batch", "BatchResults", "VariationBatch",
                "generate_mix1d", "Server", "ServeResult"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
