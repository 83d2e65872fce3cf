"""A-priori reduction to the Schur complement of the top degree (Section 5)
through the C-ABI, against the CPU oracle."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import hsc, schur, sg, solve  # noqa: E402
from sg_inputs import named_problem  # noqa: E402


def _b():
    from paper_1205_1864_amd import binding
    return binding


def _dev(A):
    return _b().to_device_block(A)


@pytest.mark.parametrize("name,kw,pc", [("small", {}, "hsc"), ("small", dict(M=3, p=3), "hsc"),
                                        ("paper_legendre", {}, "hsc"), ("small", dict(M=3, p=1), "hsc"),
                                        ("small", {}, "mean")])
def test_reduced_solve_matches_oracle(name, kw, pc):
    """Tight inner solves: the reduced iteration takes the oracle's iterations
    and reaches its solution; with HSC, as many as the unreduced solve."""
    b = _b()
    prob = named_problem(name, **kw)
    s = sg.build_system(prob)
    F = prob.load_block()
    opts = b.Options(inner_precision=64, precond=pc, inner_rtol=1e-14, inner_maxit=3000)
    solver = b.SGSolver(prob, opts)
    U, st = solver.sg_solve_reduced(_dev(F), rtol=1e-8, maxit=100, op_rtol=1e-14)
    assert st["rc"] == 0
    ex = hsc.ExactMeanSolver(s)
    if pc == "hsc":
        Uo, res = schur.solve_reduced(s, F.T.copy(), ex, rtol=1e-8)
    else:
        from oracle import krylov
        g = schur.schur_rhs(s, F.T.copy(), ex)
        res = krylov.fcg(lambda X: schur.schur_apply(s, X, ex), lambda R: hsc.mean_apply(s, R, ex), g, 1e-8, 100)
        Uo = np.zeros_like(F.T)
        lo = int(s.off[s.p])
        Uo[:, :lo] = res.x
        Uo[:, lo:] = schur.recover_top(s, F.T.copy(), res.x, ex)
    assert st["outer_it"] == res.iterations
    assert np.linalg.norm(U.cpu().numpy().T - Uo) <= 1e-9 * np.linalg.norm(Uo)
    if pc == "hsc":
        _, sf = solver.sg_solve(_dev(F), rtol=1e-8, maxit=100)
        assert st["outer_it"] == sf["outer_it"]


@pytest.mark.parametrize("family", ["hermite", "legendre"])
def test_reduced_solve_scale(family):
    """256^2, M = 10, p = 3 with the production preconditioner (inner PCG to
    1e-4) and the top-degree solves of the reduction to 1e-11."""
    b = _b()
    prob = named_problem("scale" if family == "hermite" else "scale_legendre")
    print(f"reduced solve 256^2 {family}", flush=True)
    solver = b.SGSolver(prob, b.Options(inner_precision=64, cheb_degree=8, inner_rtol=1e-4, inner_maxit=3000))
    F = prob.load_block()
    U, st = solver.sg_solve_reduced(_dev(F), rtol=1e-8, maxit=100, op_rtol=1e-11)
    assert st["rc"] == 0
    assert st["true_relres"] <= 1.05e-8
    s = sg.build_system(prob)
    assert solve.true_relres(s, F.T, U.cpu().numpy().T) <= 1.05e-8


def test_reduced_solve_rejections():
    b = _b()
    prob = named_problem("small")
    F = _dev(prob.load_block())
    with pytest.raises(b.SGError):
        b.SGSolver(named_problem("small", p=0)).sg_solve_reduced(_dev(named_problem("small", p=0).load_block()))
    with pytest.raises(b.SGError):
        b.SGSolver(prob, b.Options(inner_precision=32)).sg_solve_reduced(F)
    with pytest.raises(b.SGError):
        b.SGSolver(prob, b.Options(precond="bgs")).sg_solve_reduced(F)
    with pytest.raises(b.SGError):
        b.SGSolver(prob).sg_solve_reduced(F, op_rtol=0.0)
