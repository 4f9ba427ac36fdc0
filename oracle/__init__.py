"""FP64 CPU oracle of the modified MRT lattice Boltzmann model.

Test infrastructure: imported only by the tests, the smoke check and the CPU
baseline of the benchmark.  It shares no code with the HIP path.
"""
from .lbm import *  # noqa: F401,F403
from . import lbm  # noqa: F401
