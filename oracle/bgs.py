"""Block symmetric Gauss-Seidel preconditioner M_bGS (Section 6): the
comparator of the hierarchical Schur complement preconditioner.

Test infrastructure: a plain CPU reference written from the definition, not
part of the product path.

One action from a zero initial guess, blocks = chaos functions in the graded
order, every diagonal block A_aa = K_0 inverted by ``solve_mean``:

  forward,  a = 0 .. P-1:  x_a = A_aa^-1 (r_a - sum_{b<a} A_ab x_b)
  backward, a = P-1 .. 0:  x_a = A_aa^-1 (r_a - sum_{b<a} A_ab xf_b - sum_{b>a} A_ab x_b)

where xf are the forward values and x on the right of the backward sweep the
already updated ones, i.e. M_bGS = (D + U)^-1 D (D + L)^-1 for A = L + D + U.
The lower products are recomputed in the backward sweep, which gives the
paper's work count: 2 n_db block solves and 1.5 times the block products of
one hierarchical Schur complement action.
"""

from __future__ import annotations

import numpy as np

from .hsc import Counters
from .sg import SGSystem


def _row_products(sys: SGSystem, a: int, X: np.ndarray, cols) -> tuple:
    """sum_{b in cols} A_ab X[:, b] = sum_k K_k (sum_b G_k[a, b] X[:, b]) and the number of nonzero blocks used."""
    out = np.zeros(X.shape[0])
    used = np.zeros(len(cols), dtype=bool)
    for k, (Gk, Kk) in enumerate(zip(sys.G, sys.K)):
        g = Gk[a, cols]
        nz = g != 0.0
        if np.any(nz):
            used |= nz
            out += Kk @ (X[:, cols][:, nz] @ g[nz])
    return out, int(np.count_nonzero(used))


def bgs_apply(sys: SGSystem, R: np.ndarray, solve_mean, counters: Counters = None, row_products=None,
              solve_block=None) -> np.ndarray:
    """One action of M_bGS on a residual block R of shape (n, P).

    ``row_products(a, X, cols)`` (default: from the K_k and G_k) and
    ``solve_block(a, v)`` (default: ``solve_mean``, for A_aa = K_0) serve
    systems whose diagonal blocks are not K_0 (the lognormal coefficient of
    Section 6).
    """
    rowp = row_products if row_products is not None else (lambda a, X, cols: _row_products(sys, a, X, cols))

    def bsolve(a, v):
        if solve_block is not None:
            return solve_block(a, v)
        return solve_mean(v[:, None])[:, 0]

    P = sys.P
    cnt = counters if counters is not None else Counters()
    R = np.asarray(R, dtype=np.float64)
    xf = np.zeros_like(R)
    for a in range(P):
        lower, m = rowp(a, xf, list(range(a)))
        cnt.block_matvecs += m
        xf[:, a] = bsolve(a, R[:, a] - lower)
        cnt.block_solves += 1
    x = np.zeros_like(R)
    for a in range(P - 1, -1, -1):
        lower, m1 = rowp(a, xf, list(range(a)))
        upper, m2 = rowp(a, x, list(range(a + 1, P)))
        cnt.block_matvecs += m1 + m2
        x[:, a] = bsolve(a, R[:, a] - lower - upper)
        cnt.block_solves += 1
    return x


def bgs_dense(A_dense: np.ndarray, n: int, P: int) -> np.ndarray:
    """Dense M_bGS = (D + U)^-1 D (D + L)^-1 from the block splitting of the assembled matrix."""
    N = n * P
    blk = np.arange(N) // n
    Lm = np.where(blk[:, None] > blk[None, :], A_dense, 0.0)
    Um = np.where(blk[:, None] < blk[None, :], A_dense, 0.0)
    Dm = A_dense - Lm - Um
    return np.linalg.solve(Dm + Um, Dm @ np.linalg.inv(Dm + Lm))
