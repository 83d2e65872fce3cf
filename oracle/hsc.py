"""Hierarchical Schur complement preconditioner (Section 4, Algorithm 1) and the
mean-based preconditioner (Section 6).

Level structure (eq. (global-matrix-hierarchy)): ``A_l = [[A_{l-1}, B_l],
[C_l, D_l]]`` where the trailing block collects the chaos functions of degree
exactly l. Here B_l is the full block ``A[deg < l, deg = l]`` and C_l the
full block ``A[deg = l, deg < l]``, applied matrix-free; nothing exploits
which of their rows are zero.

Reading of the post-correction (the solve counts of Section 6,
n_ds = 2 (n_db - 1) + 1): the up sweep performs a fresh solve
``u_l^l = D_l^-1 (r_l^l - C_l u_{l-1})`` where r_l^l is the degree-l part of
r_l as left by the pre-correction of level l + 1.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse.linalg as spla

from . import krylov
from .sg import SGSystem, level_block


def diagonal_blocks_are_mean(sys: SGSystem) -> bool:
    """Lemma of Section 3 for the normalised basis: D_l is block diagonal with K_0 blocks.

    True when every G_k (k >= 1) has no entry between two functions of the
    same degree (so D_l has no off-diagonal blocks and no K_k, k >= 1, on
    its diagonal) and G_0 is the identity.
    """
    off = sys.off
    if not np.array_equal(sys.G[0], np.eye(sys.P)):
        return False
    for Gk in sys.G[1:]:
        for l in range(sys.p + 1):
            if np.any(Gk[off[l]:off[l + 1], off[l]:off[l + 1]]):
                return False
    return True


@dataclass
class Counters:
    block_matvecs: int = 0
    block_solves: int = 0


def count_blocks(sys: SGSystem, rows: slice, cols: slice) -> int:
    pat = sum(np.abs(G[rows, cols]) for G in sys.G)
    return int(np.count_nonzero(pat))


class ExactMeanSolver:
    """D_l^-1 column by column with a sparse LU factorisation of K_0 (M_0 = exact LU)."""

    def __init__(self, sys: SGSystem):
        self.lu = spla.splu(sys.K[0].tocsc())

    def __call__(self, B: np.ndarray, X0=None) -> np.ndarray:
        # a direct solve has no use for an initial guess
        if B.shape[1] == 0:
            return B.copy()
        return self.lu.solve(np.asarray(B, dtype=np.float64))


class PCGMeanSolver:
    """D_l^-1 by independent inner PCG solves with the Chebyshev preconditioner."""

    def __init__(self, sys: SGSystem, rtol: float, maxit: int, degree: int):
        self.K0 = sys.K[0]
        self.prec = krylov.make_chebyshev(sys.K[0], sys.n_e, sys.theta0, degree)
        self.rtol = rtol
        self.maxit = maxit
        self.iterations = []

    def __call__(self, B: np.ndarray, X0=None) -> np.ndarray:
        st = krylov.InnerStats()
        X = krylov.pcg_columns(self.K0, B, self.prec, self.rtol, self.maxit, st, X0)
        self.iterations.append(st.iterations)
        return X


def hsc_apply(sys: SGSystem, R: np.ndarray, solve_mean, counters: Counters = None, ptop: int = None,
              warm: bool = False, blocks=None, solve_level=None) -> np.ndarray:
    """One action of M_P (Algorithm 1) on a residual block R of shape (n, P).

    ``solve_mean(V, X0=None)`` applies the inverse of the K_0 diagonal blocks
    to each column of V (an iterative solver starts from X0 if given). With
    ``ptop`` < p the levels run only up to ptop and R has the
    ``off[ptop + 1]`` columns of degree <= ptop (the preconditioner M_{P-1}
    of the reduced system of Section 5). ``warm``: each solve of the up sweep
    starts from the down-sweep solution y_l of its level (the algorithm fixes
    what is solved, not the inner solver's initial guess). ``blocks(rows,
    cols)`` (default: ``level_block``) gives the sub-block operators B_l, C_l,
    and ``solve_level(l, V)`` (default: ``solve_mean(V)``) applies D_l^-1, for
    systems whose D_l are not block diagonal (the lognormal coefficient of
    Section 6).
    """
    blk = blocks if blocks is not None else (lambda rows, cols: level_block(sys, rows, cols))

    def dsolve(l, V, X0=None):
        if solve_level is not None:
            return solve_level(l, V)
        return solve_mean(V, X0) if X0 is not None else solve_mean(V)

    off = sys.off
    p = sys.p if ptop is None else ptop
    r = np.array(R, dtype=np.float64, copy=True)
    u = np.zeros_like(r)
    cnt = counters if counters is not None else Counters()
    ys = {}
    # Down sweep: pre-corrections on levels p..1.
    for l in range(p, 0, -1):
        lo, hi = int(off[l]), int(off[l + 1])
        y = ys[l] = dsolve(l, r[:, lo:hi])
        cnt.block_solves += hi - lo
        B_l = blk(slice(0, lo), slice(lo, hi))
        r[:, :lo] -= B_l(y)
        cnt.block_matvecs += count_blocks(sys, slice(0, lo), slice(lo, hi))
    # Mean-value problem A_0 u_0 = g_0.
    u[:, 0:1] = dsolve(0, r[:, 0:1])
    cnt.block_solves += 1
    # Up sweep: post-corrections on levels 1..p.
    for l in range(1, p + 1):
        lo, hi = int(off[l]), int(off[l + 1])
        C_l = blk(slice(lo, hi), slice(0, lo))
        w = r[:, lo:hi] - C_l(u[:, :lo])
        cnt.block_matvecs += count_blocks(sys, slice(lo, hi), slice(0, lo))
        u[:, lo:hi] = dsolve(l, w, ys[l]) if warm else dsolve(l, w)
        cnt.block_solves += hi - lo
    return u


def mean_apply(sys: SGSystem, R: np.ndarray, solve_mean) -> np.ndarray:
    """Mean-based preconditioner M_m = I (x) K_0^-1 (Powell and Elman; Section 6)."""
    return solve_mean(np.asarray(R, dtype=np.float64))


def hsc_dense_p1(A_dense: np.ndarray, n: int, P: int) -> np.ndarray:
    """Dense M_1 for p = 1 from the block inverse of eq. (block-inverse) with S replaced by A_0.

    M = [[I, 0], [-D^-1 C, I]] diag(A_0^-1, D^-1) [[I, -B D^-1], [0, I]].
    """
    A0 = A_dense[:n, :n]
    B = A_dense[:n, n:]
    C = A_dense[n:, :n]
    D = A_dense[n:, n:]
    Di = np.linalg.inv(D)
    I0 = np.eye(n)
    I1 = np.eye(n * (P - 1))
    Lo = np.block([[I0, np.zeros((n, n * (P - 1)))], [-Di @ C, I1]])
    Mi = np.block([[np.linalg.inv(A0), np.zeros((n, n * (P - 1)))], [np.zeros((n * (P - 1), n)), Di]])
    Up = np.block([[I0, -B @ Di], [np.zeros((n * (P - 1), n)), I1]])
    return Lo @ Mi @ Up
