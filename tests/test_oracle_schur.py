"""Pins of the oracle's a-priori reduction to the Schur complement (Section 5)."""

import numpy as np
import pytest

from oracle import hsc, schur, sg, solve
from sg_inputs import named_problem


def _tiny(**kw):
    prob = named_problem("small", n_e=5, M=2, p=2, **kw)
    return prob, sg.build_system(prob)


def test_matrix_free_schur_equals_dense_elimination():
    """S X from the matrix-free blocks equals the dense A11 - A12 A22^-1 A21 of
    the assembled global matrix (dense LU of the top block)."""
    prob, s = _tiny()
    A = sg.assemble(s).toarray()
    P_low = int(s.off[s.p])
    S = schur.schur_dense(A, s.n, P_low)
    X = np.random.default_rng(0).standard_normal((s.n, P_low))
    Y = schur.schur_apply(s, X, hsc.ExactMeanSolver(s))
    Yd = (S @ sg.vec(X)).reshape(s.n, P_low, order="F")
    assert np.linalg.norm(Y - Yd) <= 1e-12 * np.linalg.norm(Yd)


def test_schur_complement_spd_and_not_worse_conditioned():
    """The Schur complement of an SPD matrix is SPD and its condition number
    does not exceed the original one."""
    for kw in (dict(), dict(sigma=0.35)):
        prob, s = _tiny(**kw)
        A = sg.assemble(s).toarray()
        S = schur.schur_dense(A, s.n, int(s.off[s.p]))
        assert np.allclose(S, S.T, atol=1e-13 * np.abs(S).max())
        ea, es = np.linalg.eigvalsh(A), np.linalg.eigvalsh(S)
        assert es.min() > 0
        assert es.max() / es.min() <= ea.max() / ea.min() * (1 + 1e-10)


@pytest.mark.parametrize("name,kw", [("small", {}), ("small", dict(M=3, p=3)), ("paper_legendre", {}),
                                     ("paper_legendre", dict(M=2, p=3))])
def test_reduced_solve_matches_direct_and_full_iterations(name, kw):
    """With exact inner solves the reduced iteration reaches the direct
    solution, and takes as many iterations as the unreduced HSC-preconditioned
    flexible CG (the paper's observation for its examples)."""
    prob = named_problem(name, **kw)
    s = sg.build_system(prob)
    F = prob.load_block().T.copy()
    ex = hsc.ExactMeanSolver(s)
    U, res = schur.solve_reduced(s, F, ex, rtol=1e-8)
    assert res.converged
    Ud = solve.solve_direct(s, F)
    A = sg.assemble(s).toarray()
    ev = np.linalg.eigvalsh(A)
    assert np.linalg.norm(U - Ud) <= ev.max() / ev.min() * 1e-8 * np.linalg.norm(Ud)
    # the top block is solved exactly, so the full residual is the reduced one
    g = schur.schur_rhs(s, F, ex)
    assert solve.true_relres(s, F, U) <= 1.05e-8 * np.linalg.norm(g) / np.linalg.norm(F)
    full, _, _ = solve.solve_fcg(s, F, "hsc", "exact", rtol=1e-8)
    assert res.iterations == full.iterations


def test_degree_one_reduces_to_the_mean_level():
    """p = 1: the reduced unknown is u_0 alone, M_{P-1} is K_0^-1, and
    S = K_0 - sum_k G_k[0, k] G_k[k, 0] K_k K_0^-1 K_k."""
    prob = named_problem("small", n_e=6, M=3, p=1)
    s = sg.build_system(prob)
    ex = hsc.ExactMeanSolver(s)
    X = np.random.default_rng(1).standard_normal((s.n, 1))
    K0 = s.K[0].toarray()
    S = K0.copy()
    for k in range(1, prob.M + 1):
        g = s.G[k][0, k] * s.G[k][k, 0]
        Kk = s.K[k].toarray()
        S -= g * Kk @ np.linalg.solve(K0, Kk)
    assert np.linalg.norm(schur.schur_apply(s, X, ex) - S @ X) <= 1e-12 * np.linalg.norm(S @ X)
    R = np.random.default_rng(2).standard_normal((s.n, 1))
    assert np.allclose(hsc.hsc_apply(s, R, ex, ptop=0), np.linalg.solve(K0, R), rtol=1e-12, atol=0)
