"""The global stochastic Galerkin operator (Sections 2 and 3).

The system ``sum_j sum_i c_ijk K_i u_j = f_k`` (eq. (global-system)) is held
as the list of stiffness matrices K_0..K_M and the Galerkin matrices
G_0..G_M. With the unknown stored as an ``n x P`` matrix U whose column j is
the block u_j, the operator is

    Y = sum_k K_k U G_k^T,   i.e.  vec(Y) = (sum_k G_k (x) K_k) vec(U),

which is the block matrix of eq. (global-matrix) with blocks
``K^(j,k) = sum_i c_ijk K_i`` (eq. (global-matrix-block)).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import chaos, fe


@dataclass
class SGSystem:
    n_e: int
    M: int
    p: int
    theta0: float
    K: list            # K_0..K_M, CSR (n, n)
    G: list            # G_0..G_M, dense (P, P)
    alpha: np.ndarray  # (P, M) multi-indices
    off: np.ndarray    # level offsets, length p + 2
    K_phi: list        # stiffness of sigma * phi_k (derivative of K_k w.r.t. s_k), k = 1..M

    @property
    def n(self) -> int:
        return (self.n_e - 1) ** 2

    @property
    def P(self) -> int:
        return self.alpha.shape[0]


def build_system(problem) -> SGSystem:
    """Assemble K_k and G_k for a problem from the input generators.

    K_0 is the stiffness of the mean coefficient theta0; K_k (k >= 1) is the
    stiffness of the KL term sigma * s_k * phi_k (eq. (KL-expansion) with
    k_i = sqrt(lambda_i) v_i, scaled by sigma). The G_k belong to the
    problem's chaos family (Hermite if the problem names none).
    """
    n_e, M, p = problem.n_e, problem.M, problem.p
    K = [fe.assemble_stiffness(np.full((n_e, n_e), problem.theta0), n_e)]
    K_phi = []
    for k in range(M):
        K.append(fe.assemble_stiffness(problem.sigma * problem.s[k] * problem.phi[k], n_e))
        K_phi.append(fe.assemble_stiffness(problem.sigma * problem.phi[k], n_e))
    family = getattr(problem, "family", "hermite")
    return SGSystem(
        n_e=n_e, M=M, p=p, theta0=problem.theta0, K=K,
        G=chaos.galerkin_matrices(M, p, family=family), alpha=chaos.multi_indices(M, p),
        off=chaos.level_offsets(M, p), K_phi=K_phi,
    )


def matvec(sys: SGSystem, U: np.ndarray) -> np.ndarray:
    """MAT-VEC (Remark after eq. (global-matrix-block)): Y = sum_k (K_k U) G_k^T.

    U has shape (n, P). Only the K_k and the c_ijk are used; the global
    matrix is never formed.
    """
    Y = np.zeros_like(U)
    for Kk, Gk in zip(sys.K, sys.G):
        Y += (Kk @ U) @ Gk.T
    return Y


def assemble(sys: SGSystem) -> sp.csr_matrix:
    """The global matrix of eq. (global-matrix): sum_k G_k (x) K_k (small sizes only)."""
    A = None
    for Kk, Gk in zip(sys.K, sys.G):
        term = sp.kron(sp.csr_matrix(Gk), Kk, format="csr")
        A = term if A is None else A + term
    return A.tocsr()


def vec(U: np.ndarray) -> np.ndarray:
    """Stack the columns of U: the paper's vector [u_0; ...; u_M]."""
    return np.asarray(U).reshape(-1, order="F")


def unvec(x: np.ndarray, n: int) -> np.ndarray:
    return np.asarray(x).reshape(n, -1, order="F")


def block_counts(sys: SGSystem):
    """(n_b, n_db) of Section 6: non-zero blocks and diagonal blocks of the global matrix."""
    pat = chaos.block_pattern(sys.G) != 0
    return int(pat.sum()), int(sys.P)


def level_block(sys: SGSystem, rows: slice, cols: slice):
    """Matrix-free sub-block of the global matrix: V |-> sum_k K_k V G_k[rows, cols]^T.

    Maps an (n, |cols|) block to an (n, |rows|) block. Used for B_l, C_l and
    D_l of eq. (global-matrix-hierarchy) at sizes where assembling is too big.
    """
    def apply(V: np.ndarray) -> np.ndarray:
        out = np.zeros((V.shape[0], rows.stop - rows.start))
        for Kk, Gk in zip(sys.K, sys.G):
            Gs = Gk[rows, cols]
            if np.any(Gs):
                out += (Kk @ V) @ Gs.T
        return out
    return apply
