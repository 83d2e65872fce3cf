"""Pins of the oracle's block symmetric Gauss-Seidel preconditioner (Section 6 comparator)."""

import numpy as np

from oracle import bgs, hsc, sg, solve
from sg_inputs import named_problem


def _sys(**kw):
    prob = named_problem("small", **kw)
    return prob, sg.build_system(prob)


def test_bgs_equals_matrix_splitting_form():
    """The block sweeps equal (D + U)^-1 D (D + L)^-1 of the assembled matrix (tiny system)."""
    prob, s = _sys(n_e=5, M=2, p=2)
    A = sg.assemble(s).toarray()
    Md = bgs.bgs_dense(A, s.n, s.P)
    R = np.random.default_rng(1).standard_normal((s.n, s.P))
    Z = bgs.bgs_apply(s, R, hsc.ExactMeanSolver(s))
    Zd = sg.unvec(Md @ sg.vec(R), s.n)
    assert np.linalg.norm(Z - Zd) <= 1e-12 * np.linalg.norm(Zd)


def test_bgs_is_symmetric_positive_definite():
    prob, s = _sys(n_e=5, M=2, p=2)
    A = sg.assemble(s).toarray()
    Md = bgs.bgs_dense(A, s.n, s.P)
    assert np.linalg.norm(Md - Md.T) <= 1e-12 * np.linalg.norm(Md)
    assert np.linalg.eigvalsh(0.5 * (Md + Md.T)).min() > 0.0


def test_bgs_work_counts_are_the_papers():
    """2 n_db block solves and 1.5 times the block products of one HSC action (Section 6)."""
    prob, s = _sys(n_e=6, M=3, p=3)
    R = np.random.default_rng(2).standard_normal((s.n, s.P))
    cb, ch = hsc.Counters(), hsc.Counters()
    mean = hsc.ExactMeanSolver(s)
    bgs.bgs_apply(s, R, mean, cb)
    hsc.hsc_apply(s, R, mean, ch)
    assert cb.block_solves == 2 * s.P
    assert 2 * cb.block_matvecs == 3 * ch.block_matvecs


def test_bgs_reduces_to_mean_solve_at_degree_zero():
    prob, s = _sys(n_e=7, M=3, p=0)
    R = np.random.default_rng(3).standard_normal((s.n, s.P))
    mean = hsc.ExactMeanSolver(s)
    assert np.allclose(bgs.bgs_apply(s, R, mean), mean(R), rtol=0, atol=1e-13)


def test_bgs_preconditioned_fcg_converges_to_direct_solution():
    prob, s = _sys()
    F = prob.load_block().T.copy()
    res, cnt, _ = solve.solve_fcg(s, F, "bgs", "exact", rtol=1e-10)
    Ud = solve.solve_direct(s, F)
    assert res.converged
    assert np.linalg.norm(res.x - Ud) <= 1e-8 * np.linalg.norm(Ud)
