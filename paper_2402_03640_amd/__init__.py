"""hipmsat: the gradient-based MaxSAT solve loop of Hosny & Reda (arXiv 2402.03640)
as hand-written HIP kernels for MI355X (gfx950), behind a C ABI.

The Python names mirror the C entry points of ``include/hipmsat.h``:
``load_cnf``, ``load_cnf_dimacs``, ``solve``, ``evaluate``, ``eval_relaxed``.
"""
from ._lib import (ADAM, LOSS_ALL, LOSS_UNSAT, RESIDENT, SGD, CancelFlag, Cnf, HipMsatError, Plan,
                   SolveOutput, SolverState, eval_relaxed, eval_relaxed_noalloc, evaluate, lib, load_cnf, load_cnf_dimacs, solve,
                   schedule_count, solve_batch, time_kernels, tune, tune_candidates, version)

__all__ = ["ADAM", "SGD", "LOSS_UNSAT", "LOSS_ALL", "RESIDENT", "CancelFlag", "Cnf", "HipMsatError", "Plan",
           "SolveOutput", "SolverState", "eval_relaxed", "eval_relaxed_noalloc", "evaluate", "lib", "load_cnf", "load_cnf_dimacs",
           "schedule_count", "solve", "solve_batch", "time_kernels", "tune", "tune_candidates", "version"]
