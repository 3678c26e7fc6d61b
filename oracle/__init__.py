"""CPU oracle for the explicit WaveHoltz hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
CPU-baseline leg of the benchmark import it; the GPU library never does, and
the two share no code.  ``core`` holds the FP64 time stepping, the filter and
the outer iterations; ``closed_forms`` holds the closed-form results used to
pin the oracle (discrete filter function, sine-mode eigenvalues, DST-I
solutions, a sparse direct solve of the discrete Helmholtz problem).
"""
from . import core  # noqa: F401
from . import closed_forms  # noqa: F401
