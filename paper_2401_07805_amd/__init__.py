"""Matrix-free variable-coefficient pressure-Poisson operator for MI355X (gfx950).

The operator a(p,q) = int (1/rho(phi)) grad p . grad q on Q_k hexahedra, with the
reciprocal density interpolation 1/rho = H(phi)/rho_l + (1-H(phi))/rho_g over a
tanh conservative level set, applied matrix-free by sum factorisation and
solved by Jacobi-preconditioned CG, in FP64 or with FP32 inner solves.  The
compute path is the HIP library libvpp.so (C ABI in include/vpp.h); this package
only marshals arguments to it.
"""
from ._lib import LIB_PATH, declared_functions, load  # noqa: F401
from .api import AmrProblem, Batch, PoissonSolve, Problem, VppError, config_candidates, poisson_solve  # noqa: F401

__all__ = ["Problem", "AmrProblem", "Batch", "PoissonSolve", "poisson_solve", "VppError", "config_candidates", "load",
           "LIB_PATH", "declared_functions"]
