"""Q1 finite elements on the unit square (Section 2, eq. (global-system)).

The stiffness matrix of KL term i is ``(K_i)_{lm} = int_D k_i(x) grad phi_l .
grad phi_m dx`` (the bilinear form of Section 2 with the coefficient field
k_i). Coefficients are constant per element (their value at the element is
given as input), so ``K_i = sum_e k_i(e) K^e`` is exact. Homogeneous
Dirichlet data: only interior nodes carry unknowns.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# Local corner order of an element: counter-clockwise from the lower-left.
CORNERS = ((0, 0), (1, 0), (1, 1), (0, 1))


def q1_shape_gradients(xi: float, eta: float) -> np.ndarray:
    """Gradients of the four bilinear shape functions on the unit reference square.

    N_c(xi, eta) = (xi or 1-xi) * (eta or 1-eta) for the corner c = (cx, cy).
    """
    g = np.zeros((4, 2))
    for c, (cx, cy) in enumerate(CORNERS):
        fx = xi if cx else 1.0 - xi
        fy = eta if cy else 1.0 - eta
        dfx = 1.0 if cx else -1.0
        dfy = 1.0 if cy else -1.0
        g[c] = (dfx * fy, fx * dfy)
    return g


def q1_element_stiffness() -> np.ndarray:
    """int_e grad N_a . grad N_b for a square element.

    In 2D the integral is independent of the element size (the h^-2 of the
    gradients cancels the h^2 of the area), so the reference square is used.
    The integrand is a polynomial of degree 2 per direction; the 2x2 Gauss
    rule is exact for it.
    """
    gp = np.array([-1.0, 1.0]) / np.sqrt(3.0) * 0.5 + 0.5
    Ke = np.zeros((4, 4))
    for xi in gp:
        for eta in gp:
            g = q1_shape_gradients(xi, eta)
            Ke += 0.25 * g @ g.T
    return Ke


def interior_numbering(n_e: int) -> np.ndarray:
    """Map grid node (iy, ix), 0..n_e each, to its interior index or -1."""
    idx = -np.ones((n_e + 1, n_e + 1), dtype=np.int64)
    m = n_e - 1
    for iy in range(1, n_e):
        for ix in range(1, n_e):
            idx[iy, ix] = (iy - 1) * m + (ix - 1)
    return idx


def assemble_stiffness(coef: np.ndarray, n_e: int) -> sp.csr_matrix:
    """K = sum_e coef[e] K^e over interior nodes (element loop, vectorised over e).

    ``coef`` has shape (n_e, n_e) indexed [ey, ex].
    """
    Ke = q1_element_stiffness()
    num = interior_numbering(n_e)
    ey, ex = np.meshgrid(np.arange(n_e), np.arange(n_e), indexing="ij")
    ey = ey.ravel()
    ex = ex.ravel()
    c = np.asarray(coef, dtype=np.float64).reshape(n_e, n_e)[ey, ex]
    rows, cols, vals = [], [], []
    for a, (ax, ay) in enumerate(CORNERS):
        ga = num[ey + ay, ex + ax]
        for b, (bx, by) in enumerate(CORNERS):
            gb = num[ey + by, ex + bx]
            keep = (ga >= 0) & (gb >= 0)
            rows.append(ga[keep])
            cols.append(gb[keep])
            vals.append(c[keep] * Ke[a, b])
    n = (n_e - 1) ** 2
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    K.sum_duplicates()
    return K


def laplacian(n_e: int) -> sp.csr_matrix:
    """Stiffness matrix of the unit coefficient."""
    return assemble_stiffness(np.ones((n_e, n_e)), n_e)
