"""CPU FP64 oracle for the unbinned negative log-likelihood engine.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, readable statement
of what the device library must compute: the composed densities, their
normalization integrals, NLL = -sum_i ln P~(x_i) + N ln I, and its gradient.
Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import it; the device library never does, and the two share no code.

Conventions
-----------
* float64 everywhere (torch CPU tensors; complex128 for amplitudes).
* Event sums of the NLL value use ``math.fsum`` (exactly rounded).
* Gradients come from torch autograd on the same expressions (exact up to
  rounding) and, independently, from central finite differences.
* Model descriptions are the same JSON-able dicts the library takes; this
  package parses them with its own code.

Parity status per function is listed in each module header.
"""
from . import common, mix1d, dalitz3  # noqa: F401
