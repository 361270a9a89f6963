"""MI355X (gfx950) oblique-projection FEAST: HIP kernels behind a C ABI.

The shared library ``libfeast_mi355x.so`` implements the filter of eq. (8-4)
(shifted LU factorisations and solves, weighted node sum), the oblique
projection of Section 3 and Algorithm 5 (dense pencils, and sparse ones in CSR
form factored as band matrices); ``binding`` marshals torch tensors
into it.  Build it with ``python -m paper_1404_1768_amd.build``.
"""
from .binding import (FEAST_OK, FEAST_SINGULAR, FEAST_REFINE_STAGNATED, FEAST_EINVAL,  # noqa: F401
                      FEAST_EDEVICE, FEAST_ENOMEM, FEAST_ENUMERIC, FEAST_ESCRATCH, TRAPEZOID,
                      GAUSS_LEGENDRE,
                      FP64, MIXED, FeastError, Plan, SolveResult, feast_filter, feast_project,
                      feast_solve, feast_nodes, feast_reduced_eig, feast_stop_rule, load,
                      zgemm_batched, zgetrf_batched, zgetrs_batched, zgetrs_batched_noalloc, LIB_PATH, feast_eig,
                      Batch, BatchResult, enclosing_circle, region_inside, solve_region, csr_order)
