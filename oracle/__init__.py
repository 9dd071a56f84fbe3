"""CPU oracle for the MB4 step on the periodic 2D lattice NLS.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import it.  It shares no code with the GPU library.
"""
from .mb4_oracle import (  # noqa: F401
    ALPHA1_PAPER, C_PAPER, EPS_PAPER, LatticeNLS, MB4Constants, MB4Oracle,
    NewtonDivergence, energy_drift, hopping_matrix, method_constants,
    oracle_for)
