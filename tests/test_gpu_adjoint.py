"""Adjoint gradient of the quantity of interest (hand-written adjoint through
the C-ABI and the torch.autograd.Function) on the differentiation recipe:
against the oracle's adjoint on the 32^2 instance and against central finite
differences of the GPU solve on the 512^2 instance."""

import copy

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from oracle import adjoint, sg, solve  # noqa: E402
from sg_inputs import named_problem, qoi_weights  # noqa: E402


def _b():
    from paper_1205_1864_amd import binding
    return binding


def _spec(prob, rtol):
    b = _b()
    from paper_1205_1864_amd.autograd import QoISpec
    wm, wv = qoi_weights(prob.n_e)
    return QoISpec(problem=prob, F=b.to_device_block(prob.load_block()), w_mean=b.to_device_vec(wm),
                   w_var=b.to_device_vec(wv), opts=b.Options(inner_precision=64, cheb_degree=8, inner_rtol=1e-10,
                                                             inner_maxit=4000), rtol=rtol, maxit=400)


def _q_and_grad(prob, spec):
    from paper_1205_1864_amd.autograd import SGQoI
    theta = torch.tensor(np.concatenate([[prob.theta0], prob.s]), dtype=torch.float64, requires_grad=True)
    Q = SGQoI.apply(theta, spec)
    Q.backward()
    return float(Q.detach()), theta.grad.numpy().copy()


@pytest.mark.timeout(600)
def test_adjoint_gradient_matches_oracle_adjoint_32():
    """32^2 instance of the differentiation recipe (M = 8, p = 3, P = 165)."""
    prob = named_problem("grad_small")
    spec = _spec(prob, rtol=1e-12)
    Q, g = _q_and_grad(prob, spec)
    s = sg.build_system(prob)
    F = prob.load_block().T.copy()
    wm, wv = qoi_weights(prob.n_e)

    def oracle_solve(R):
        res, _, _ = solve.solve_fcg(s, R, "hsc", "exact", rtol=1e-13, maxit=400)
        return res.x

    Qo, go, _ = adjoint.adjoint_gradient(s, oracle_solve(F), wm, wv, oracle_solve)
    assert abs(Q - Qo) <= 1e-10 * abs(Qo)
    assert np.max(np.abs(g - go)) <= 1e-8 * np.max(np.abs(go)), (g, go)


@pytest.mark.timeout(900)
def test_adjoint_gradient_matches_finite_differences_512():
    """512^2 differentiation recipe (M = 8, p = 3, 43M unknowns): central differences
    with h = 1e-6 of tight GPU solves agree with the adjoint gradient to 1e-5 in
    every one of the 1 + M components (theta0 and the eight KL amplitudes), each
    relative to itself (with a floor of 1e-3 of the largest component) and
    normwise."""
    prob = named_problem("grad")
    spec = _spec(prob, rtol=1e-12)
    Q, g = _q_and_grad(prob, spec)
    assert spec.last_stats["forward"]["rc"] == 0 and spec.last_stats["adjoint"]["rc"] == 0
    b = _b()
    h = 1e-6
    fds = []
    for i in range(prob.M + 1):  # theta0, then every KL amplitude
        qs = []
        for sgn in (+1, -1):
            pr = copy.copy(prob)
            if i == 0:
                pr.theta0 = prob.theta0 + sgn * h
            else:
                s_ = np.array(prob.s, dtype=np.float64).copy()
                s_[i - 1] += sgn * h
                pr.s = s_
            solver = b.SGSolver(pr, spec.opts)
            U, st = solver.sg_solve(spec.F, rtol=1e-12, maxit=400)
            assert st["rc"] == 0
            qs.append(solver.sg_qoi(U, spec.w_mean, spec.w_var))
            solver.close()
        fd = (qs[0] - qs[1]) / (2 * h)
        print(f"component {i}: adjoint {g[i]:.10e} central difference {fd:.10e}", flush=True)
        assert abs(fd - g[i]) <= 1e-5 * max(abs(g[i]), 1e-3 * np.max(np.abs(g))), (i, fd, g[i])
        fds.append(fd)
    fds = np.array(fds)
    assert np.max(np.abs(g - fds)) <= 1e-5 * np.max(np.abs(fds))
