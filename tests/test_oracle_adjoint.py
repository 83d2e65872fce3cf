"""Pins of the oracle's quantity of interest and adjoint gradient."""

import numpy as np
import pytest
from numpy.polynomial import hermite_e

from oracle import adjoint, fe, sg, solve
from sg_inputs import Problem, named_problem, nodal_rhs, qoi_weights


def _Q_of(prob, w_mean, w_var):
    s = sg.build_system(prob)
    U = solve.solve_direct(s, prob.load_block().T.copy())
    return adjoint.qoi(U, w_mean, w_var), s, U


def _perturbed(prob, i, h):
    import copy
    q = copy.deepcopy(prob)
    if i == 0:
        q.theta0 = q.theta0 + h
    else:
        q.s = q.s.copy()
        q.s[i - 1] += h
    return q


def test_adjoint_matches_central_differences():
    prob = named_problem("small", n_e=8, M=3, p=2, sigma=0.25, L=0.4)
    w_mean, w_var = qoi_weights(prob.n_e, 0.25, 0.75)
    Q, s, U = _Q_of(prob, w_mean, w_var)
    _, g, _ = adjoint.adjoint_gradient(s, U, w_mean, w_var, lambda R: solve.solve_direct(s, R))
    h = 1e-5
    fd = np.zeros_like(g)
    for i in range(1 + prob.M):
        qp = _Q_of(_perturbed(prob, i, h), w_mean, w_var)[0]
        qm = _Q_of(_perturbed(prob, i, -h), w_mean, w_var)[0]
        fd[i] = (qp - qm) / (2 * h)
    assert np.max(np.abs(g - fd)) <= 1e-7 * np.max(np.abs(fd))


def test_euler_homogeneity():
    """A is linear in (theta0, s), so theta0 dQ/dtheta0 + sum s_k dQ/ds_k = -Q_mean - 2 Q_var."""
    prob = named_problem("small", n_e=10, M=4, p=3)
    w_mean, w_var = qoi_weights(prob.n_e)
    Q, s, U = _Q_of(prob, w_mean, w_var)
    _, g, _ = adjoint.adjoint_gradient(s, U, w_mean, w_var, lambda R: solve.solve_direct(s, R))
    qm, qv = adjoint.qoi_parts(U, w_mean, w_var)
    lhs = prob.theta0 * g[0] + np.dot(prob.s, g[1:])
    assert abs(lhs - (-qm - 2 * qv)) <= 1e-12 * abs(qm + 2 * qv)


def test_mean_problem_gradient():
    """p = 0: u = K_0^-1 f / theta0-scaling gives dQ/dtheta0 = -Q/theta0 and no s dependence."""
    prob = named_problem("small", n_e=10, M=3, p=0, theta0=1.4)
    w_mean, w_var = qoi_weights(prob.n_e)
    Q, s, U = _Q_of(prob, w_mean, w_var)
    _, g, _ = adjoint.adjoint_gradient(s, U, w_mean, w_var, lambda R: solve.solve_direct(s, R))
    assert abs(g[0] + Q / prob.theta0) <= 1e-13 * abs(Q)
    assert np.all(g[1:] == 0.0)


@pytest.mark.parametrize("p", [2, 4])
def test_constant_mode_analytic_derivative(p):
    n_e, theta0, sigma = 8, 1.0, 0.2
    prob = Problem(name="const", n_e=n_e, M=1, p=p, theta0=theta0, sigma=sigma, L=1.0,
                   s=np.array([0.9]), phi=np.ones((1, n_e, n_e)), f_nodal=nodal_rhs(n_e))
    c = sigma * 0.9
    w_mean, w_var = qoi_weights(n_e, 0.2, 0.8)
    Q, s, U = _Q_of(prob, w_mean, w_var)
    _, g, _ = adjoint.adjoint_gradient(s, U, w_mean, w_var, lambda R: solve.solve_direct(s, R))
    x, w = hermite_e.hermegauss(p + 1)
    w = w / w.sum()
    v = np.linalg.solve(fe.laplacian(n_e).toarray(), prob.load_block()[0])
    a = theta0 + c * x
    S1, S2 = np.sum(w / a), np.sum(w / a ** 2)
    dS1_dt, dS2_dt = -np.sum(w / a ** 2), -2 * np.sum(w / a ** 3)
    dS1_dc, dS2_dc = -np.sum(w * x / a ** 2), -2 * np.sum(w * x / a ** 3)
    m, q = w_mean @ v, w_var @ v ** 2
    assert abs(Q - (S1 * m + (S2 - S1 ** 2) * q)) <= 1e-12 * abs(Q)
    dQ_dt = dS1_dt * m + (dS2_dt - 2 * S1 * dS1_dt) * q
    dQ_dc = dS1_dc * m + (dS2_dc - 2 * S1 * dS1_dc) * q
    assert abs(g[0] - dQ_dt) <= 1e-11 * abs(dQ_dt)
    assert abs(g[1] - sigma * dQ_dc) <= 1e-11 * abs(sigma * dQ_dc)
