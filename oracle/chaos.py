"""Polynomial chaos (Section 2, eq. (gPC-u), eq. (global-system)).

The chaos basis is the tensor product of univariate polynomials of total
degree at most p in M independent variables; there are
``(M + p)! / (M! p!)`` of them (Section 2). Two families:

* ``"hermite"``: standard Gaussian variables and the normalised probabilists'
  Hermite polynomials ``He_a(xi) / sqrt(a!)``;
* ``"legendre"``: variables uniform on ``[-1, 1]`` and the normalised
  Legendre polynomials ``sqrt(2a + 1) P_a(xi)`` (Section 2; the examples of
  Section 6). Reading: the support [-1, 1] is the one under which the
  paper's remark that ellipticity is no longer guaranteed above a
  coefficient of variation of 55 % holds for its setup, and it reproduces
  the iteration counts and condition estimates of its Tables 1-4 (a test
  pins this); CoV = sigma / theta0 is then a nominal value.

Both bases are orthonormal, ``E[psi_a psi_b] = delta_ab``, so every diagonal
block of the global matrix is exactly K_0.

Ordering reading: indices are graded by total degree (the level structure of
Section 3 needs degree-l functions to follow all lower degrees); within one
degree they are in descending lexicographic order, ``(d, 0, ..., 0)`` first.
"""

from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from numpy.polynomial import hermite_e, legendre

FAMILIES = ("hermite", "legendre")


def multi_indices(M: int, p: int) -> np.ndarray:
    """All alpha in N^M with |alpha| <= p, graded, descending lex within a degree."""
    out = []

    def rec(prefix, remaining, k):
        if k == M:
            if remaining == 0:
                out_deg.append(tuple(prefix))
            return
        for v in range(remaining, -1, -1):
            rec(prefix + [v], remaining - v, k + 1)

    for d in range(p + 1):
        out_deg = []
        rec([], d, 0)
        out.extend(out_deg)
    if M == 0:
        out = [()]
    return np.array(out, dtype=np.int64).reshape(len(out), M)


def level_offsets(M: int, p: int) -> np.ndarray:
    """Start index of each degree: off[l] .. off[l+1]-1 are the degree-l functions."""
    off = [0]
    for d in range(p + 1):
        off.append(off[-1] + math.comb(M + d - 1, d) if M > 0 else off[-1] + (1 if d == 0 else 0))
    return np.array(off, dtype=np.int64)


@lru_cache(maxsize=None)
def _gauss_hermite(nq: int):
    x, w = hermite_e.hermegauss(nq)
    return x, w / w.sum()


def he(a: int, x: np.ndarray) -> np.ndarray:
    c = np.zeros(a + 1)
    c[a] = 1.0
    return hermite_e.hermeval(x, c)


@lru_cache(maxsize=None)
def _gauss_legendre(nq: int):
    t, w = legendre.leggauss(nq)
    return t, w / w.sum()


def normalized_legendre(a: int, xi: np.ndarray) -> np.ndarray:
    """sqrt(2a + 1) P_a(xi): orthonormal for xi uniform on [-1, 1]."""
    c = np.zeros(a + 1)
    c[a] = 1.0
    return math.sqrt(2 * a + 1) * legendre.legval(np.asarray(xi), c)


def normalized_moment(exponent: int, a: int, b: int, family: str = "hermite") -> float:
    """E[xi^exponent psi_a(xi) psi_b(xi)] for the 1D normalised basis of a family.

    Gauss quadrature of the family's own measure (probability-normalised
    weights) with enough points to integrate the polynomial of degree
    exponent + a + b exactly.
    """
    nq = (exponent + a + b) // 2 + 2
    if family == "hermite":
        x, w = _gauss_hermite(nq)
        val = np.sum(w * x ** exponent * he(a, x) * he(b, x))
        return float(val / math.sqrt(math.factorial(a) * math.factorial(b)))
    if family == "legendre":
        x, w = _gauss_legendre(nq)
        return float(np.sum(w * x ** exponent * normalized_legendre(a, x) * normalized_legendre(b, x)))
    raise ValueError(family)


def galerkin_matrices(M: int, p: int, snap: float = 1e-12, family: str = "hermite"):
    """G_0..G_M with (G_k)_{ab} = E[xi_k psi_a psi_b], xi_0 = 1 (eq. (global-system)).

    The expectation factorises over the independent variables: the factor of
    dimension k carries xi_k, every other factor is E[psi_a psi_b] of that
    dimension. The xi_k factor comes from a quadrature table. Values below
    ``snap`` in magnitude are orthogonality zeros and are set to exactly 0.
    Returns a list of dense (P, P) arrays.
    """
    alpha = multi_indices(M, p)
    P = alpha.shape[0]
    # The basis is orthonormal by construction, so the factor of a dimension
    # without xi_k is the identity (checked against quadrature in the tests).
    m0 = np.eye(p + 1)
    # E[xi psi_a psi_b] is symmetric in (a, b): evaluate a <= b and mirror.
    m1 = np.zeros((p + 1, p + 1))
    for a in range(p + 1):
        for b in range(a, p + 1):
            m1[a, b] = m1[b, a] = normalized_moment(1, a, b, family)
    Gs = []
    for k in range(M + 1):
        G = np.ones((P, P))
        for dim in range(M):
            A = alpha[:, dim]
            T = m1 if dim == k - 1 else m0
            G *= T[A[:, None], A[None, :]]
        G[np.abs(G) <= snap] = 0.0
        Gs.append(G)
    return Gs


def block_pattern(Gs) -> np.ndarray:
    """The matrix c_P of Section 2: entry (j, k) = sum_i c_ijk (block sparsity)."""
    return sum(np.abs(G) for G in Gs)
