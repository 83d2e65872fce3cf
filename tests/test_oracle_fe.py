"""Pins of the oracle's finite-element layer."""

import math

import numpy as np
import pytest

from oracle import fe, krylov


def test_element_stiffness_closed_form():
    Ke = fe.q1_element_stiffness()
    expect = np.array([[4, -1, -2, -1], [-1, 4, -1, -2], [-2, -1, 4, -1], [-1, -2, -1, 4]]) / 6.0
    assert np.max(np.abs(Ke - expect)) < 1e-15


def _energy_by_integration(coef, u_nodes, n_e):
    """sum_e coef(e) int_e |grad u_h|^2 for the bilinear interpolant (3x3 Gauss per element)."""
    h = 1.0 / n_e
    full = np.zeros((n_e + 1, n_e + 1))
    full[1:-1, 1:-1] = u_nodes.reshape(n_e - 1, n_e - 1)
    g, w = np.polynomial.legendre.leggauss(3)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    total = 0.0
    for ey in range(n_e):
        for ex in range(n_e):
            u00, u10 = full[ey, ex], full[ey, ex + 1]
            u01, u11 = full[ey + 1, ex], full[ey + 1, ex + 1]
            acc = 0.0
            for xi, wx in zip(g, w):
                for eta, wy in zip(g, w):
                    dx = ((u10 - u00) * (1 - eta) + (u11 - u01) * eta) / h
                    dy = ((u01 - u00) * (1 - xi) + (u11 - u10) * xi) / h
                    acc += wx * wy * (dx * dx + dy * dy)
            total += coef[ey, ex] * acc * h * h
    return total


@pytest.mark.parametrize("n_e", [3, 5, 8])
def test_assembled_energy_equals_integral(n_e):
    rng = np.random.default_rng(n_e)
    coef = rng.uniform(0.5, 2.0, (n_e, n_e))
    K = fe.assemble_stiffness(coef, n_e)
    u = rng.standard_normal((n_e - 1) ** 2)
    assert abs(u @ (K @ u) - _energy_by_integration(coef, u, n_e)) < 1e-12 * abs(u @ (K @ u))
    assert abs(K - K.T).max() == 0.0


@pytest.mark.parametrize("n_e", [4, 7, 12])
def test_laplacian_spectrum_closed_form(n_e):
    KL = fe.laplacian(n_e).toarray()
    ev = np.sort(np.linalg.eigvalsh(KL))
    c = np.cos(np.arange(1, n_e) * math.pi / n_e)
    lam = np.sort(((8 - 2 * c[:, None] - 2 * c[None, :] - 4 * c[:, None] * c[None, :]) / 3).ravel())
    assert np.max(np.abs(ev - lam)) < 1e-12
    lmin, lmax = krylov.jacobi_scaled_spectrum(n_e)
    d = np.diag(KL)
    assert np.allclose(d, 8.0 / 3.0)
    ev_s = np.linalg.eigvalsh(KL / d[:, None])
    assert abs(ev_s.min() - lmin) < 1e-13 and abs(ev_s.max() - lmax) < 1e-13


def test_laplacian_stencil():
    n_e = 6
    KL = fe.laplacian(n_e).toarray()
    m = n_e - 1
    i = 2 * m + 2  # interior node away from the boundary
    row = KL[i].reshape(m, m)
    expect = np.zeros((m, m))
    expect[1:4, 1:4] = -1.0 / 3.0
    expect[2, 2] = 8.0 / 3.0
    assert np.max(np.abs(row - expect)) < 1e-15
