"""Seeded synthetic inputs for approximate selected inversion.

This package produces the inputs of the method and nothing else: symmetric
sparse matrices of the shapes, sizes and value distributions of the paper's
workloads (grid diffusion operators, shifted indefinite Laplacians, random
diagonally dominant graphs), fill-reducing orderings, and the incomplete
block LDL^T factors (L, D, P) that the method takes as given (the paper takes
them from a separate block-ILDL package; its method starts from the factors).

Both the GPU library and the CPU oracle consume what this package produces;
it holds none of the arithmetic of SelInv, NInv, Mix, SPAI, the low-rank
correction or the learned correction. For the indefinite shifted Laplacian it
also gives the exact A^-1 products and diag(A^-1) in closed form: the
reference quantities that the paper obtains from a direct solver.
"""
from .matrices import (laplace2d, diffusion3d_7pt, shifted_laplace2d_indefinite,
                       random_dd_symmetric, stencil27_3d, kkt_matrix, dodd, covariance_grid,
                       saddle2d)
from .ordering import rcm, nested_dissection_grid, nested_multicolor_grid, apply_symmetric_perm
from .ildl import ildl_bk, IldlFactors
from .exact import ShiftedLaplace2DExact

__all__ = [
    "laplace2d", "diffusion3d_7pt", "shifted_laplace2d_indefinite",
    "random_dd_symmetric", "stencil27_3d", "kkt_matrix", "dodd", "covariance_grid", "saddle2d",
    "rcm", "nested_dissection_grid", "nested_multicolor_grid", "apply_symmetric_perm",
    "ildl_bk", "IldlFactors", "ShiftedLaplace2DExact",
]
