"""Quantity of interest and its gradient with respect to the coefficient parameters.

The parameters are theta = (theta0, s_1..s_M): the mean coefficient and the
KL amplitudes sqrt(lambda_k) of eq. (KL-expansion); sigma and the modes are
fixed. The SG matrix is linear in theta:
dA/dtheta0 = I (x) K_Lap and dA/ds_k = G_k (x) K[sigma phi_k].

For Q(U) the textbook adjoint identity gives dQ/dtheta = -<Lambda, (dA/dtheta) U>
with A Lambda = dQ/dU (A is symmetric). The quantity of interest (reading of
the subdomain statistics): E[u] is the mean chaos block and Var[u] the sum of
squares of the other blocks (normalised basis), so

    Q = w_mean . U[:, 0] + sum_{j >= 1} w_var . U[:, j]^2 .
"""

from __future__ import annotations

import numpy as np

from . import fe
from .sg import SGSystem


def qoi(U: np.ndarray, w_mean: np.ndarray, w_var: np.ndarray) -> float:
    return float(w_mean @ U[:, 0] + np.sum(w_var[:, None] * U[:, 1:] ** 2))


def qoi_parts(U, w_mean, w_var):
    return float(w_mean @ U[:, 0]), float(np.sum(w_var[:, None] * U[:, 1:] ** 2))


def qoi_grad_u(U: np.ndarray, w_mean: np.ndarray, w_var: np.ndarray) -> np.ndarray:
    Gq = np.zeros_like(U)
    Gq[:, 0] = w_mean
    Gq[:, 1:] = 2.0 * w_var[:, None] * U[:, 1:]
    return Gq


def parameter_contractions(sys: SGSystem, Lam: np.ndarray, U: np.ndarray) -> np.ndarray:
    """-<Lambda, (dA/dtheta_i) U>_F for theta = (theta0, s_1..s_M)."""
    KL = fe.laplacian(sys.n_e)
    g = np.zeros(1 + sys.M)
    g[0] = -np.sum(Lam * (KL @ U))
    for k in range(sys.M):
        g[1 + k] = -np.sum(Lam * ((sys.K_phi[k] @ U) @ sys.G[k + 1].T))
    return g


def adjoint_gradient(sys: SGSystem, U: np.ndarray, w_mean, w_var, solve) -> tuple:
    """(Q, grad, Lambda): ``solve(RHS)`` returns A^-1 RHS for an (n, P) block."""
    Q = qoi(U, w_mean, w_var)
    Lam = solve(qoi_grad_u(U, w_mean, w_var))
    return Q, parameter_contractions(sys, Lam, U), Lam
