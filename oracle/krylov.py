"""Krylov solvers of the oracle.

* Flexible CG with one stored direction (Notay's FCG, cited in Section 5 as
  the method for a variable preconditioner; Section 6 reports its iteration
  counts). Stopping reading: Euclidean norm of the recursive residual of the
  unpreconditioned system relative to ||f||_2, zero initial guess unless a
  start is given.
* Inner solves on K_0 (the "independent loops of preconditioned Krylov
  subspace iterations for each diagonal block" of Section 5): PCG whose
  preconditioner is a Chebyshev polynomial in the Jacobi-scaled K_0 (the
  paper leaves the mean-value preconditioner M_0 open; this is one choice).
  The Chebyshev recurrence is the classical Chebyshev acceleration for an
  SPD matrix with spectrum in [lmin, lmax] (Saad, Iterative Methods for
  Sparse Linear Systems, 2nd ed., Sec. 12.3), started from zero.
* The Lanczos condition estimate from CG coefficients (Section 6).
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np


def dot(a, b) -> float:
    return float(np.sum(a * b))


# ---------------------------------------------------------------------------
# Spectrum of the Jacobi-scaled mean matrix
# ---------------------------------------------------------------------------

def jacobi_scaled_spectrum(n_e: int):
    """Extreme eigenvalues of D^-1 K_0 for the Q1 stencil on an n_e x n_e grid.

    K_0 = theta0 * K_Lap with the constant 9-point stencil (8/3 centre, -1/3
    for all eight neighbours) on interior nodes; its eigenvectors are the
    discrete sine modes sin(i pi x1) sin(j pi x2), 1 <= i, j <= n_e - 1, with
    eigenvalue (8 - 2 c_i - 2 c_j - 4 c_i c_j) / 3, c_i = cos(i pi h). D is the
    diagonal theta0 * 8/3, so D^-1 K_0 has eigenvalues
    (8 - 2 c_i - 2 c_j - 4 c_i c_j) / 8, independent of theta0.
    """
    m = n_e - 1
    c = np.cos(np.arange(1, m + 1) * math.pi / n_e)
    lam = (8.0 - 2.0 * c[:, None] - 2.0 * c[None, :] - 4.0 * c[:, None] * c[None, :]) / 8.0
    return float(lam.min()), float(lam.max())


@dataclass
class Chebyshev:
    """Degree-d Chebyshev polynomial preconditioner for K_0 (Jacobi scaled).

    ``apply(R)`` returns z_d of the Chebyshev iteration for
    (D^-1 K_0) z = D^-1 r from z_0 = 0: d updates of z, d - 1 products with
    K_0. The result is p(D^-1 K_0) D^-1 r for a fixed polynomial p, an SPD
    operator when [lmin, lmax] contains the spectrum.
    """
    K0: object
    diag: float
    lmin: float
    lmax: float
    degree: int

    def apply(self, R: np.ndarray) -> np.ndarray:
        theta = 0.5 * (self.lmax + self.lmin)
        delta = 0.5 * (self.lmax - self.lmin)
        S = R / self.diag
        W = S / theta
        Z = W.copy()
        if delta <= 0.0:
            return Z
        sigma1 = theta / delta
        rho = 1.0 / sigma1
        for _ in range(1, self.degree):
            S = S - (self.K0 @ W) / self.diag
            rho_new = 1.0 / (2.0 * sigma1 - rho)
            W = (rho_new * rho) * W + (2.0 * rho_new / delta) * S
            Z = Z + W
            rho = rho_new
        return Z


def make_chebyshev(K0, n_e: int, theta0: float, degree: int) -> Chebyshev:
    lmin, lmax = jacobi_scaled_spectrum(n_e)
    return Chebyshev(K0=K0, diag=theta0 * 8.0 / 3.0, lmin=lmin, lmax=lmax, degree=degree)


# ---------------------------------------------------------------------------
# Inner PCG on K_0, one independent solve per column
# ---------------------------------------------------------------------------

@dataclass
class InnerStats:
    iterations: np.ndarray = None   # per column


def pcg_columns(K0, B: np.ndarray, prec: Chebyshev, rtol: float, maxit: int, stats=None, X0=None):
    """Independent PCG solves K_0 x_j = b_j, one per column of B (shape (n, m)).

    Initial guess zero, or the columns of X0 (then r = b - K_0 x0, and a
    column whose initial residual already passes the test returns x0 without
    iterating). Column j stops once its recursive residual satisfies
    ||r_j|| <= rtol ||b_j|| (checked after each update, before the next
    preconditioner application) or after ``maxit`` products with K_0.
    A zero column gives x_j = 0 without iterating, whatever the initial
    guess. rtol <= 0 runs exactly ``maxit`` iterations.
    """
    n, m = B.shape
    X = np.zeros_like(B)
    its = np.zeros(m, dtype=np.int64)
    for j in range(m):
        b = B[:, j]
        bn = math.sqrt(dot(b, b))
        if bn == 0.0:
            continue
        if X0 is None:
            x = np.zeros(n)
            r = b.copy()
        else:
            x = np.array(X0[:, j], dtype=np.float64)
            r = b - K0 @ x
            if math.sqrt(dot(r, r)) <= rtol * bn:
                X[:, j] = x
                continue
        z = prec.apply(r[:, None])[:, 0]
        p = z.copy()
        gamma = dot(r, z)
        for it in range(maxit):
            q = K0 @ p
            alpha = gamma / dot(p, q)
            x = x + alpha * p
            r = r - alpha * q
            its[j] = it + 1
            if math.sqrt(dot(r, r)) <= rtol * bn:
                break
            if it + 1 == maxit:
                break
            z = prec.apply(r[:, None])[:, 0]
            gamma_new = dot(r, z)
            beta = gamma_new / gamma
            p = z + beta * p
            gamma = gamma_new
        X[:, j] = x
    if stats is not None:
        stats.iterations = its
    return X


# ---------------------------------------------------------------------------
# Outer flexible CG
# ---------------------------------------------------------------------------

@dataclass
class FCGResult:
    x: np.ndarray
    iterations: int
    converged: bool
    relres: float
    history: list = field(default_factory=list)
    history_time: list = field(default_factory=list)  # time.perf_counter() at each history entry
    alphas: list = field(default_factory=list)
    betas: list = field(default_factory=list)
    breakdown: bool = False


def fcg(apply_A, apply_M, F: np.ndarray, rtol: float, maxit: int, X0=None) -> FCGResult:
    """Flexible CG with one stored direction (truncation m = 1).

        z_i = M(r_i)
        p_i = z_i - (z_i . q_{i-1}) / (p_{i-1} . q_{i-1}) p_{i-1}   (p_0 = z_0)
        q_i = A p_i,  alpha_i = (p_i . r_i) / (p_i . q_i)
        x += alpha_i p_i,  r -= alpha_i q_i

    Stops when ||r||_2 <= rtol ||f||_2. A non-positive or non-finite p.q is
    reported as a breakdown.
    """
    X = np.zeros_like(F) if X0 is None else X0.copy()
    R = F - apply_A(X) if X0 is not None else F.copy()
    fn = math.sqrt(dot(F, F))
    res = FCGResult(x=X, iterations=0, converged=False, relres=0.0)
    if fn == 0.0:
        res.x = np.zeros_like(F)
        res.converged = True
        return res
    relres = math.sqrt(dot(R, R)) / fn
    res.history.append(relres)
    res.history_time.append(time.perf_counter())
    if relres <= rtol:
        res.converged = True
        res.relres = relres
        return res
    P = Q = None
    pq_prev = None
    for it in range(maxit):
        Z = apply_M(R)
        if P is None:
            P = Z
        else:
            beta = -dot(Z, Q) / pq_prev
            res.betas.append(beta)
            P = Z + beta * P
        Q = apply_A(P)
        pq = dot(P, Q)
        if not (pq > 0.0) or not math.isfinite(pq):
            res.breakdown = True
            break
        alpha = dot(P, R) / pq
        res.alphas.append(alpha)
        X = X + alpha * P
        R = R - alpha * Q
        pq_prev = pq
        res.iterations = it + 1
        relres = math.sqrt(dot(R, R)) / fn
        res.history.append(relres)
        res.history_time.append(time.perf_counter())
        if relres <= rtol:
            res.converged = True
            break
    res.x = X
    res.relres = relres
    return res


def pcg(apply_A, apply_M, F: np.ndarray, rtol: float, maxit: int) -> FCGResult:
    """Standard preconditioned CG (for comparison with FCG under a fixed preconditioner)."""
    X = np.zeros_like(F)
    R = F.copy()
    fn = math.sqrt(dot(F, F))
    res = FCGResult(x=X, iterations=0, converged=False, relres=1.0)
    Z = apply_M(R)
    P = Z.copy()
    gamma = dot(R, Z)
    for it in range(maxit):
        Q = apply_A(P)
        alpha = gamma / dot(P, Q)
        X = X + alpha * P
        R = R - alpha * Q
        res.iterations = it + 1
        res.relres = math.sqrt(dot(R, R)) / fn
        if res.relres <= rtol:
            res.converged = True
            break
        Z = apply_M(R)
        gamma_new = dot(R, Z)
        P = Z + (gamma_new / gamma) * P
        gamma = gamma_new
    res.x = X
    return res


def lanczos_kappa(alphas, betas) -> float:
    """Condition estimate from the Lanczos tridiagonal built from CG coefficients.

    T_00 = 1/alpha_0, T_ii = 1/alpha_i + beta_i/alpha_{i-1},
    T_{i-1,i} = sqrt(beta_i)/alpha_{i-1}, where beta_i builds p_i from p_{i-1}.
    """
    m = len(alphas)
    if m == 0:
        return 1.0
    T = np.zeros((m, m))
    T[0, 0] = 1.0 / alphas[0]
    for i in range(1, m):
        b = abs(betas[i - 1])
        T[i, i] = 1.0 / alphas[i] + b / alphas[i - 1]
        T[i - 1, i] = T[i, i - 1] = math.sqrt(b) / alphas[i - 1]
    ev = np.linalg.eigvalsh(T)
    return float(ev.max() / ev.min())
