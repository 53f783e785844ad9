"""CPU oracle for the adaptive s-step GMRES hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline leg of the benchmark may use it; the HIP library never does, and the
two share no code.  See `sstep_gmres` for the algorithm, written from the
paper (Xu, Alonso, Darve, arXiv 2303.08953).
"""
from .sstep_gmres import *  # noqa: F401,F403
from . import sstep_gmres  # noqa: F401
