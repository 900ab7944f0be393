"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package only *builds inputs*: sparse matrices in CSR form, subdomain
partitions, deflation vectors and right-hand sides.  It contains none of the
solver's arithmetic (no projection, no multigrid, no Krylov recurrence), so
both the CPU oracle and the GPU library can consume its output without sharing
any solver code.

Problems follow the paper's benchmark section: the 3D Poisson problem
(-Laplace u = 1 on the unit cube, homogeneous Dirichlet conditions) discretised
with the 7-point stencil, constant ("subdomain") and linear deflation vectors,
and box partitions of the grid into subdomains.  Nonsymmetric inputs: a
first-order upwind convection-diffusion operator and a stabilised Q1 Oseen
operator with four unknowns per node.
"""
from .poisson import poisson7, grid_coords
from .partition import box_partition, slab_partition
from .deflation import constant_deflation, linear_deflation
from .configs import (Problem, config_small_poisson, config_lognormal_poisson,
                      config_batched, batched_recipe, concat_problems,
                      make_problem, tiny_problem, config_oseen, config_oseen_schur)
from .oseen import oseen_q1, field_deflation
from .convdiff import convection_diffusion7

__all__ = [
    "poisson7", "grid_coords", "box_partition", "slab_partition",
    "constant_deflation", "linear_deflation", "Problem",
    "config_small_poisson", "config_lognormal_poisson", "config_batched",
    "batched_recipe", "concat_problems", "make_problem", "tiny_problem",
    "config_oseen", "config_oseen_schur", "oseen_q1", "field_deflation", "convection_diffusion7",
]
