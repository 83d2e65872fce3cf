"""Lognormal diffusion coefficient in the Hermite chaos (Section 6, second set
of experiments; Tables 6-9).

Test infrastructure: a plain CPU reference written from the definitions, not
part of the product path; the GPU library's lognormal calls are checked
against it.

The coefficient is ``k(x, xi) = exp(g(x, xi))`` with a Gaussian field
``g = mu_g + sum_k g_k(x) xi_k`` (KL terms ``g_k = sigma_g sqrt(lambda_k)
phi_k`` of the separable exponential covariance, the same KL data as the
other examples). Readings (the paper names only the lognormal CoV and that the
coefficient is expanded to twice the solution's degree, in Hermite
polynomials):

* the covariance belongs to the underlying Gaussian field, whose variance is
  fixed by the lognormal moments: ``sigma_g^2 = ln(1 + CoV^2)`` and
  ``mu_g = ln(mean) - sigma_g^2 / 2`` (mean 1 as in the other examples);
* the chaos expansion of ``exp(g)`` in the normalised Hermite basis has the
  closed-form coefficients
  ``k_i(x) = exp(mu_g + sum_k g_k^2 / 2) prod_k g_k^{i_k} / sqrt(i_k!)``
  (a generating-function identity), kept for ``|i| <= 2p``;
* the global matrix is ``A = sum_i G_i (x) K_i`` with
  ``(G_i)_{ab} = E[psi_i psi_a psi_b]`` and ``K_i`` the stiffness of ``k_i``
  (element values at the element level, like the KL terms). All diagonal
  blocks of a degree level couple, so the hierarchical preconditioner solves
  with the full level blocks D_l and block Gauss-Seidel with the full
  diagonal blocks A_aa; here both are exact (sparse LU), the paper's "direct"
  variant.

One-dimensional triple products of the normalised probabilists' Hermite
polynomials (a classical closed form): with ``s = (a + b + c) / 2`` an
integer and ``s >= a, b, c``,
``E[psi_a psi_b psi_c] = sqrt(a! b! c!) / ((s - a)! (s - b)! (s - c)!)``,
else zero.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import chaos, fe, hsc, krylov
from .sg import SGSystem, unvec, vec


def hermite_triple(a: int, b: int, c: int) -> float:
    """E[psi_a psi_b psi_c] for the normalised 1D Hermite basis (closed form)."""
    two_s = a + b + c
    if two_s % 2:
        return 0.0
    s = two_s // 2
    if s < a or s < b or s < c:
        return 0.0
    f = math.factorial
    return math.sqrt(f(a) * f(b) * f(c)) / (f(s - a) * f(s - b) * f(s - c))


def triple_matrices(coef_idx: np.ndarray, alpha: np.ndarray) -> list:
    """G_i[a, b] = prod_d E[psi_{i_d} psi_{a_d} psi_{b_d}] for every coefficient index i."""
    dmax = int(max(coef_idx.max(initial=0), alpha.max(initial=0)))
    T = np.zeros((dmax + 1, dmax + 1, dmax + 1))
    for i in range(dmax + 1):
        for a in range(dmax + 1):
            for b in range(dmax + 1):
                T[i, a, b] = hermite_triple(i, a, b)
    Gs = []
    for ci in coef_idx:
        G = np.ones((alpha.shape[0], alpha.shape[0]))
        for d in range(alpha.shape[1]):
            G *= T[ci[d]][alpha[:, d][:, None], alpha[:, d][None, :]]
        Gs.append(G)
    return Gs


def gpc_coefficients(mu_g: np.ndarray, g: np.ndarray, coef_idx: np.ndarray) -> np.ndarray:
    """k_i on the elements for each coefficient index i: shape (len(coef_idx), ...) of mu_g."""
    base = np.exp(mu_g + 0.5 * np.sum(g * g, axis=0))
    out = np.empty((coef_idx.shape[0],) + base.shape)
    for j, ci in enumerate(coef_idx):
        term = base.copy()
        for k, e in enumerate(ci):
            if e:
                term = term * g[k] ** e / math.sqrt(math.factorial(int(e)))
        out[j] = term
    return out


@dataclass
class LognormalSystem:
    sys: SGSystem          # the K_i and G_i lists (matrix-free form)
    A: sp.csr_matrix       # the assembled global matrix sum_i G_i (x) K_i
    coef: np.ndarray       # (terms, n_e, n_e) element values of the k_i
    coef_idx: np.ndarray   # coefficient multi-indices, |i| <= 2p


def build(problem, cov: float, mean: float = 1.0) -> LognormalSystem:
    """Lognormal system on the mesh and KL data of ``problem`` (its sigma and
    family are not used: the Gaussian field's variance comes from ``cov``)."""
    n_e, M, p = problem.n_e, problem.M, problem.p
    sg2 = math.log(1.0 + cov * cov)
    mu_g = np.full((n_e, n_e), math.log(mean) - 0.5 * sg2)
    g = math.sqrt(sg2) * problem.s[:, None, None] * problem.phi
    coef_idx = chaos.multi_indices(M, 2 * p)
    alpha = chaos.multi_indices(M, p)
    coef = gpc_coefficients(mu_g, g, coef_idx)
    K = [fe.assemble_stiffness(c, n_e) for c in coef]
    G = triple_matrices(coef_idx, alpha)
    sys = SGSystem(n_e=n_e, M=M, p=p, theta0=float(coef[0].mean()), K=K, G=G, alpha=alpha,
                   off=chaos.level_offsets(M, p), K_phi=[])
    return LognormalSystem(sys=sys, A=_assemble(sys), coef=coef, coef_idx=coef_idx)


def _assemble(sys: SGSystem) -> sp.csr_matrix:
    """Block (a, b) of A is the stiffness of the field sum_i G_i[a, b] k_i: K is
    linear in the coefficient, so every block is one combination of the K_i's
    values on the common 9-point pattern."""
    pat = sum(abs(Kk) for Kk in sys.K).tocsr()
    pat.sort_indices()
    r, c = pat.nonzero()
    vals = np.stack([np.asarray(Kk[r, c]).ravel() for Kk in sys.K])  # (terms, nnz)
    Gst = np.stack(sys.G)                                              # (terms, P, P)
    n, P = sys.n, sys.P
    blocks = np.einsum("tab,te->abe", Gst, vals)                       # (P, P, nnz)
    a_idx, b_idx = np.nonzero(np.any(blocks != 0.0, axis=2))
    rows = (a_idx[:, None] * n + r[None, :]).ravel()
    cols = (b_idx[:, None] * n + c[None, :]).ravel()
    data = blocks[a_idx, b_idx].ravel()
    return sp.csr_matrix((data, (rows, cols)), shape=(n * P, n * P))


class LognormalPreconditioners:
    """M_m, M_bGS and M_HS (Section 6) for the assembled lognormal matrix.

    M_m: ``I (x) K_0^-1`` with K_0 the stiffness of the mean coefficient k_0.
    M_bGS: block symmetric Gauss-Seidel over the chaos blocks, exact A_aa.
    M_HS: Algorithm 1 with exact D_l and the full off-diagonal level blocks.
    """

    def __init__(self, ls: LognormalSystem):
        self.ls = ls
        s = ls.sys
        self.n, self.P, self.off = s.n, s.P, s.off
        A = ls.A.tocsc()
        self.A = ls.A
        self.lu0 = spla.splu(s.K[0].tocsc())
        self.lu_level = []
        for l in range(s.p + 1):
            lo, hi = int(self.off[l]) * self.n, int(self.off[l + 1]) * self.n
            self.lu_level.append(spla.splu(A[lo:hi, lo:hi].tocsc()))
        self.lu_block = [spla.splu(A[a * self.n:(a + 1) * self.n, a * self.n:(a + 1) * self.n].tocsc())
                         for a in range(self.P)]

    def _sub(self, rows: slice, cols: slice):
        n = self.n
        Ab = self.A[rows.start * n:rows.stop * n, cols.start * n:cols.stop * n]

        def apply(V):
            return unvec(Ab @ vec(V), n)
        return apply

    def solve_level(self, l: int, V: np.ndarray) -> np.ndarray:
        return unvec(self.lu_level[l].solve(vec(V)), self.n)

    def mean(self, R: np.ndarray) -> np.ndarray:
        return self.lu0.solve(np.asarray(R, dtype=np.float64))

    def hsc(self, R: np.ndarray) -> np.ndarray:
        return hsc.hsc_apply(self.ls.sys, R, None, blocks=self._sub, solve_level=self.solve_level)

    def bgs(self, R: np.ndarray) -> np.ndarray:
        from . import bgs
        n = self.n

        def row_products(a, X, cols):
            if not cols:
                return np.zeros(n), 0
            c0, c1 = cols[0], cols[-1] + 1
            Ab = self.A[a * n:(a + 1) * n, c0 * n:c1 * n]
            return Ab @ vec(X[:, c0:c1]), 0

        def solve_block(a, v):
            return self.lu_block[a].solve(v)
        return bgs.bgs_apply(self.ls.sys, R, None, row_products=row_products, solve_block=solve_block)


def solve_fcg(ls: LognormalSystem, F: np.ndarray, precond: str, rtol: float = 1e-8, maxit: int = 500,
              pcs: LognormalPreconditioners = None):
    """Flexible CG on the assembled lognormal system; returns (FCGResult, preconditioners)."""
    pcs = pcs if pcs is not None else LognormalPreconditioners(ls)
    M = {"mean": pcs.mean, "bgs": pcs.bgs, "hsc": pcs.hsc, "none": lambda R: R.copy()}[precond]
    n = ls.sys.n
    res = krylov.fcg(lambda U: unvec(ls.A @ vec(U), n), M, F, rtol, maxit)
    return res, pcs
