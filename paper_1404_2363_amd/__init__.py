"""MI355X (gfx950) modified-MRT lattice Boltzmann solver for the anisotropic
convection-diffusion equation.

``workloads`` draws seeded inputs; ``solver.Solver`` runs them through the HIP
library ``liblbm_cde.so`` (C ABI in ``include/lbm_cde.h``, binding in
``_lib``).  Build the library with ``paper_1404_2363_amd.build.build()``.
"""
__all__ = ["workloads", "solver", "build"]
