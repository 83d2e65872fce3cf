"""A-priori reduction to the Schur complement of the top degree (Section 5).

Test infrastructure: a plain CPU reference written from the definitions, not
part of the product path.

With the unknowns split into the chaos functions of degree < p ("low") and
of degree p ("top"), the global system [[A_{P-1}, B_P], [C_P, D_P]] is reduced
by eliminating the top block:

    S_{P-1} u_low = g,   S_{P-1} = A_{P-1} - B_P D_P^-1 C_P,
                         g       = f_low - B_P D_P^-1 f_top,

solved by flexible CG preconditioned by Algorithm 1 run over the levels
1..p-1 only; afterwards u_top = D_P^-1 (f_top - C_P u_low). D_P is block
diagonal with K_0 blocks (normalised basis), so D_P^-1 is one mean solve per
top-degree column.
"""

from __future__ import annotations

import numpy as np

from . import hsc, krylov
from .sg import SGSystem, level_block


def _split(sys: SGSystem):
    lo = int(sys.off[sys.p])
    return slice(0, lo), slice(lo, sys.P)


def schur_apply(sys: SGSystem, X: np.ndarray, solve_mean) -> np.ndarray:
    """S_{P-1} X for a block X of shape (n, off[p])."""
    low, top = _split(sys)
    A_low = level_block(sys, low, low)
    B_top = level_block(sys, low, top)
    C_top = level_block(sys, top, low)
    return A_low(X) - B_top(solve_mean(C_top(X)))


def schur_rhs(sys: SGSystem, F: np.ndarray, solve_mean) -> np.ndarray:
    """g = f_low - B_P D_P^-1 f_top for a right-hand side F of shape (n, P)."""
    low, top = _split(sys)
    return F[:, low] - level_block(sys, low, top)(solve_mean(F[:, top]))


def recover_top(sys: SGSystem, F: np.ndarray, U_low: np.ndarray, solve_mean) -> np.ndarray:
    """u_top = D_P^-1 (f_top - C_P u_low)."""
    low, top = _split(sys)
    return solve_mean(F[:, top] - level_block(sys, top, low)(U_low))


def schur_dense(A_dense: np.ndarray, n: int, P_low: int) -> np.ndarray:
    """Dense S = A_11 - A_12 A_22^-1 A_21 from the assembled global matrix (small sizes)."""
    m = n * P_low
    A11, A12, A21, A22 = A_dense[:m, :m], A_dense[:m, m:], A_dense[m:, :m], A_dense[m:, m:]
    return A11 - A12 @ np.linalg.solve(A22, A21)


def solve_reduced(sys: SGSystem, F: np.ndarray, solve_mean, rtol: float = 1e-8, maxit: int = 200):
    """FCG on the reduced system with M_{P-1}, then recovery of the top degree.

    Returns (U of shape (n, P), FCGResult of the reduced iteration). Needs p >= 1.
    The stopping test is the relative residual of the reduced system.
    """
    low, top = _split(sys)
    g = schur_rhs(sys, F, solve_mean)
    res = krylov.fcg(lambda X: schur_apply(sys, X, solve_mean),
                     lambda R: hsc.hsc_apply(sys, R, solve_mean, ptop=sys.p - 1), g, rtol, maxit)
    U = np.zeros_like(F, dtype=np.float64)
    U[:, low] = res.x
    U[:, top] = recover_top(sys, F, res.x, solve_mean)
    return U, res
