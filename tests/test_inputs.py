"""Checks of the seeded input generators (KL data, weights, workload sets)."""

import math

import numpy as np
import pytest
from scipy.optimize import brentq

from sg_inputs import batch_problems, kl_1d, kl_2d, named_problem, qoi_weights


def _exponential_kernel_eigenvalues(L, count):
    """Eigenvalues of exp(-|x-y|/L) on an interval of length 1 (closed form).

    With c = 1/L and half-length a = 1/2: even modes solve c - w tan(w a) = 0,
    odd modes w + c tan(w a) = 0; lambda = 2c / (w^2 + c^2).
    """
    c, a = 1.0 / L, 0.5
    out = []
    k = 0
    while len(out) < count:
        lo, hi = 2 * k * math.pi + 1e-12, 2 * k * math.pi + math.pi - 1e-12
        w = brentq(lambda w: c - w * math.tan(w * a), lo, hi)
        out.append(2 * c / (w * w + c * c))
        lo, hi = (2 * k + 1) * math.pi + 1e-12, (2 * k + 2) * math.pi - 1e-12
        w = brentq(lambda w: w + c * math.tan(w * a), lo, hi)
        out.append(2 * c / (w * w + c * c))
        k += 1
    return np.array(out[:count])


@pytest.mark.parametrize("L", [0.3, 0.5, 1.0])
def test_kl_1d_against_closed_form(L):
    mu, E = kl_1d(256, L, 6)
    exact = _exponential_kernel_eigenvalues(L, 6)
    err256 = np.abs(mu - exact) / exact
    assert np.max(err256) < 5e-4
    # second-order convergence of the trapezoid Nystrom method
    mu2, _ = kl_1d(512, L, 6)
    err512 = np.abs(mu2 - exact) / exact
    assert np.all(err512[1:] < err256[1:] / 3.5)
    w = np.full(257, 1 / 256)
    w[[0, -1]] *= 0.5
    G = (E * w) @ E.T
    assert np.max(np.abs(G - np.eye(6))) < 1e-12
    assert np.all(E[:, 0] > 0)


def test_kl_2d_mode_order_and_ties():
    lam, phi, modes = kl_2d(16, 0.5, 4)
    assert modes == [(0, 0), (0, 1), (1, 0), (0, 2)]
    assert lam[1] == lam[2]
    lam, phi, modes = kl_2d(256, 0.3, 10)
    assert modes == [(0, 0), (0, 1), (1, 0), (1, 1), (0, 2), (2, 0), (0, 3), (3, 0), (1, 2), (2, 1)]
    assert np.all(np.diff(lam) <= 0)


def test_qoi_weights():
    wm, wv = qoi_weights(10)
    assert abs(wm.sum() - 1) < 1e-15
    assert np.count_nonzero(wv) == 9  # x in {0.4, 0.5, 0.6}^2
    assert np.allclose(wv[wv > 0], 0.01)


def test_named_problem_sizes():
    pr = named_problem("small")
    assert (pr.n, pr.P) == (225, 15)
    assert pr.coefficient_margin() > 0


def test_batch_problem_generator():
    a = batch_problems(seed=0, count=12)
    b = batch_problems(seed=0, count=12)
    for x, y in zip(a, b):
        assert (x.n_e, x.M, x.p, x.sigma) == (y.n_e, y.M, y.p, y.sigma)
        assert x.P <= 495 and x.coefficient_margin() > 0
        assert 0.1 <= x.sigma <= 0.3 and 0.2 <= x.L <= 1.0


def test_coefficient_margin_matches_element_eigenvalues():
    """Cross-check the rotation-invariance bound against eigenvalues of theta0 I + sum a_k G_k."""
    from oracle import chaos
    pr = named_problem("small", n_e=8, M=3, p=3, sigma=0.3)
    Gs = chaos.galerkin_matrices(pr.M, pr.p)
    a = pr.element_coefficients()
    worst = min(np.linalg.eigvalsh(pr.theta0 * Gs[0] + sum(a[k, ey, ex] * Gs[k + 1] for k in range(pr.M))).min()
                for ey in range(8) for ex in range(8))
    assert abs(worst - pr.coefficient_margin()) < 1e-12
