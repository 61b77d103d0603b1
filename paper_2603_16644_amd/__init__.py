"""MI355X (gfx950) randomized preconditioned normal equations for tall
least-squares problems (Garrison & Ipsen, arXiv 2603.16644).

The solver lives in the HIP library libpne.so behind the C ABI of
include/pne.h; this package is its Python binding.
"""
from ._lib import (PREC, BatchPlan, Opts, PneError, autotune_batched, cond_est, cond_est_qr, hpne_solve, lib, make_opts, nne_solve, pne_gram,
                   pne_sketch, pne_sketch_srft, pne_solve, pne_solve_batched, pne_solve_noalloc, qr_ls_solve, sketch_precond)

__all__ = ["PREC", "BatchPlan", "Opts", "PneError", "autotune_batched", "cond_est", "cond_est_qr", "hpne_solve", "lib", "make_opts", "nne_solve",
           "pne_gram", "pne_sketch", "pne_sketch_srft",
           "pne_solve", "pne_solve_batched", "pne_solve_noalloc", "qr_ls_solve", "sketch_precond"]
