"""Solvers of the oracle: direct solve of the assembled system, and flexible CG
with the preconditioners of Section 6 (none, mean-based, hierarchical Schur).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import bgs, hsc, krylov
from .sg import SGSystem, assemble, matvec, unvec, vec


def solve_direct(sys: SGSystem, F: np.ndarray) -> np.ndarray:
    """Sparse direct solve of the assembled global system (small sizes)."""
    A = assemble(sys).tocsc()
    return unvec(spla.spsolve(A, vec(F)), sys.n)


def mean_solver(sys: SGSystem, inner="exact", inner_rtol=1e-4, inner_maxit=1000, degree=4):
    if inner == "exact":
        return hsc.ExactMeanSolver(sys)
    return hsc.PCGMeanSolver(sys, inner_rtol, inner_maxit, degree)


def solve_fcg(sys: SGSystem, F: np.ndarray, precond: str = "hsc", inner="exact",
              rtol: float = 1e-8, maxit: int = 200, inner_rtol: float = 1e-4,
              inner_maxit: int = 1000, degree: int = 4, X0=None):
    """FCG on the SG system with M in {none, mean, hsc, bgs}; returns (FCGResult, counters, solver)."""
    solver = mean_solver(sys, inner, inner_rtol, inner_maxit, degree)
    counters = hsc.Counters()
    if precond == "hsc":
        def M(R):
            return hsc.hsc_apply(sys, R, solver, counters)
    elif precond == "mean":
        def M(R):
            return hsc.mean_apply(sys, R, solver)
    elif precond == "bgs":
        def M(R):
            return bgs.bgs_apply(sys, R, solver, counters)
    elif precond == "none":
        def M(R):
            return R.copy()
    else:
        raise ValueError(precond)
    res = krylov.fcg(lambda U: matvec(sys, U), M, F, rtol, maxit, X0=X0)
    return res, counters, solver


def true_relres(sys: SGSystem, F: np.ndarray, U: np.ndarray) -> float:
    R = F - matvec(sys, U)
    return float(np.linalg.norm(R) / np.linalg.norm(F))


def error_bound_constant(problem) -> float:
    """c with ||u - u*||_2 <= c ||f - A u||_2 for the exact solution u* of A u* = f.

    A = sum_e C_e (x) K^e (eq. (global-matrix) regrouped by element) with the
    element chaos matrices C_e = theta0 I + sum_k a_k(e) G_k and the
    unit-coefficient element stiffness K^e >= 0. If C_e >= m I for every e
    (m = ``problem.coefficient_margin()``), then A >= m (I (x) K_Lap), so
    ||A^-1||_2 <= 1 / (m lambda_1) with lambda_1 = (8 - 4c - 4c^2) / 3,
    c = cos(pi / n_e), the smallest eigenvalue of the unit-coefficient Q1
    Laplacian on the interior nodes (sine mode (1, 1)). Infinite if m <= 0.
    """
    m = float(problem.coefficient_margin())
    if not m > 0.0:
        return float("inf")
    c = np.cos(np.pi / problem.n_e)
    lam1 = (8.0 - 4.0 * c - 4.0 * c * c) / 3.0
    return 1.0 / (m * lam1)
