"""Legendre chaos (uniform variables on [-1, 1], the examples of Section 6)
through the C-ABI against the CPU oracle."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import adjoint, bgs, hsc, krylov, sg, solve  # noqa: E402
from sg_inputs import named_problem, qoi_weights, random_block  # noqa: E402


def _b():
    from paper_1205_1864_amd import binding
    return binding


def _dev(A):
    return _b().to_device_block(A)


@pytest.mark.parametrize("kw", [dict(n_e=10, M=4, p=4), dict(n_e=64, M=5, p=3), dict(n_e=128, M=3, p=4),
                                dict(n_e=33, M=6, p=2)])
def test_matvec_parity(kw):
    prob = named_problem("paper_legendre", **kw)
    print(f"legendre matvec n_e={prob.n_e} M={prob.M} p={prob.p}", flush=True)
    s = sg.build_system(prob)
    solver = _b().SGSolver(prob)
    U = random_block(prob.P, prob.n, seed=3)
    Y = solver.sg_matvec(_dev(U)).cpu().numpy()
    Yo = sg.matvec(s, U.T).T
    assert np.linalg.norm(Y - Yo) <= 1e-12 * np.linalg.norm(Yo)


def test_matvec_parity_scale():
    prob = named_problem("scale_legendre")
    print("legendre matvec 256^2 M=10 p=3", flush=True)
    s = sg.build_system(prob)
    solver = _b().SGSolver(prob)
    U = random_block(prob.P, prob.n, seed=1)
    Y = solver.sg_matvec(_dev(U)).cpu().numpy()
    Yo = sg.matvec(s, U.T).T
    assert np.linalg.norm(Y - Yo) <= 1e-12 * np.linalg.norm(Yo)


@pytest.mark.parametrize("which", ["hsc", "mean", "bgs"])
def test_preconditioner_tight_parity(which):
    b = _b()
    prob = named_problem("paper_legendre", n_e=24, M=3, p=3)
    s = sg.build_system(prob)
    solver = b.SGSolver(prob, b.Options(inner_precision=64, inner_rtol=1e-13, inner_maxit=2000))
    R = random_block(prob.P, prob.n, seed=8)
    apply = {"hsc": solver.sg_apply_hsc, "mean": solver.sg_apply_mean, "bgs": solver.sg_apply_bgs}[which]
    Z = apply(_dev(R)).cpu().numpy()
    ex = hsc.ExactMeanSolver(s)
    ref = {"hsc": lambda: hsc.hsc_apply(s, R.T, ex), "mean": lambda: hsc.mean_apply(s, R.T, ex),
           "bgs": lambda: bgs.bgs_apply(s, R.T, ex)}[which]
    Zo = ref().T
    assert np.linalg.norm(Z - Zo) <= 1e-9 * np.linalg.norm(Zo)


@pytest.mark.parametrize("pc", ["mean", "bgs", "hsc"])
def test_paper_example_solves(pc):
    """The Section 6 example (10 x 10 mesh, N = 4, degree 4, CoV 50 %): with
    (nearly) exact inner solves the GPU flexible CG takes the oracle's
    iterations, with the oracle's Lanczos condition estimate, and reaches the
    direct solution."""
    b = _b()
    prob = named_problem("paper_legendre")
    s = sg.build_system(prob)
    F = prob.load_block()
    solver = b.SGSolver(prob, b.Options(inner_precision=64, precond=pc, inner_rtol=1e-14, inner_maxit=3000))
    U, st = solver.sg_solve(_dev(F), rtol=1e-8, maxit=100)
    res, _, _ = solve.solve_fcg(s, F.T.copy(), pc, "exact", rtol=1e-8, maxit=100)
    assert st["rc"] == 0
    assert st["outer_it"] == res.iterations
    kappa_o = krylov.lanczos_kappa(res.alphas, res.betas)
    assert abs(st["kappa_est"] - kappa_o) <= 1e-6 * kappa_o
    Ud = solve.solve_direct(s, F.T.copy())
    A = sg.assemble(s).toarray()
    ev = np.linalg.eigvalsh(A)
    assert np.linalg.norm(U.cpu().numpy().T - Ud) <= ev.max() / ev.min() * 1.05e-8 * np.linalg.norm(Ud)


@pytest.mark.parametrize("prec", [64, 32])
def test_solve_scale_converges(prec):
    """256^2, M = 10, p = 3 with Legendre chaos: the production solve reaches the
    tolerance; its true residual is checked on the oracle's operator."""
    b = _b()
    prob = named_problem("scale_legendre")
    print(f"legendre solve 256^2 inner FP{prec}", flush=True)
    solver = b.SGSolver(prob, b.Options(inner_precision=prec, cheb_degree=8, inner_rtol=1e-4, inner_maxit=2000))
    F = prob.load_block()
    U, st = solver.sg_solve(_dev(F), rtol=1e-8, maxit=100)
    assert st["rc"] == 0 and st["true_relres"] <= 1.05e-8
    s = sg.build_system(prob)
    assert solve.true_relres(s, F.T, U.cpu().numpy().T) <= 1.05e-8


def test_adjoint_gradient_matches_oracle_adjoint():
    """32^2, M = 4, p = 3: the adjoint gradient of the subdomain QoI against the oracle's."""
    b = _b()
    prob = named_problem("paper_legendre", n_e=32, M=4, p=3, sigma=0.4)
    s = sg.build_system(prob)
    solver = b.SGSolver(prob, b.Options(inner_precision=64, inner_rtol=1e-12, inner_maxit=3000))
    F = prob.load_block()
    wm, wv = qoi_weights(prob.n_e)
    U, _ = solver.sg_solve(_dev(F), rtol=1e-12, maxit=200)
    Q, grad, ast = solver.sg_adjoint_grad(U, b.to_device_vec(wm), b.to_device_vec(wv), rtol=1e-12, maxit=200)

    def oracle_solve(R):
        res, _, _ = solve.solve_fcg(s, R, "hsc", "exact", rtol=1e-13, maxit=400)
        return res.x

    Qo, go, _ = adjoint.adjoint_gradient(s, oracle_solve(F.T.copy()), wm, wv, oracle_solve)
    assert abs(Q - Qo) <= 1e-10 * abs(Qo)
    g = np.asarray(grad)
    assert np.max(np.abs(g - go)) <= 1e-8 * np.max(np.abs(go)), (g, go)
