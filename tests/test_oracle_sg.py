"""Pins of the oracle's global SG operator and solves."""

import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp
from numpy.polynomial import hermite_e

from oracle import chaos, fe, krylov, sg, solve
from sg_inputs import Problem, named_problem, nodal_rhs


def _tiny(n_e=4, M=2, p=2, sigma=0.3, L=0.5):
    return named_problem("small", n_e=n_e, M=M, p=p, sigma=sigma, L=L)


def test_galerkin_system_by_tensor_quadrature():
    """A = E[psi psi^T (x) K(xi)] evaluated on a tensor Gauss-Hermite grid (brute force)."""
    prob = _tiny(n_e=4, M=2, p=2)
    s = sg.build_system(prob)
    A = s and sg.assemble(s).toarray()
    alpha = chaos.multi_indices(prob.M, prob.p)
    x, w = hermite_e.hermegauss(prob.p + 2)
    w = w / w.sum()
    Aq = np.zeros_like(A)
    for idx in itertools.product(range(len(x)), repeat=prob.M):
        xi = x[list(idx)]
        wq = np.prod(w[list(idx)])
        psi = np.array([np.prod([hermite_e.hermeval(xi[d], np.eye(prob.p + 1)[a[d]])
                                 / math.sqrt(math.factorial(a[d])) for d in range(prob.M)])
                        for a in alpha])
        coef = prob.theta0 + prob.sigma * np.einsum("k,kij->ij", prob.s * xi, prob.phi)
        Kq = fe.assemble_stiffness(coef, prob.n_e).toarray()
        Aq += wq * np.kron(np.outer(psi, psi), Kq)
    assert np.max(np.abs(A - Aq)) < 1e-12 * np.max(np.abs(A))


@pytest.mark.parametrize("name_kw", [dict(n_e=16, M=4, p=2), dict(n_e=6, M=3, p=3), dict(n_e=5, M=1, p=4)])
def test_matrix_free_matches_assembled(name_kw):
    prob = named_problem("small", **name_kw)
    s = sg.build_system(prob)
    A = sg.assemble(s)
    U = np.random.default_rng(1).standard_normal((s.n, s.P))
    Y1 = sg.matvec(s, U)
    Y2 = sg.unvec(A @ sg.vec(U), s.n)
    assert np.linalg.norm(Y1 - Y2) <= 1e-14 * np.linalg.norm(Y2)


def test_diagonal_blocks_are_mean_bitwise_and_symmetry():
    prob = named_problem("small")
    s = sg.build_system(prob)
    A = sg.assemble(s).tocsr()
    n, P = s.n, s.P
    K0 = s.K[0].toarray()
    for a in range(P):
        blk = A[a * n:(a + 1) * n, a * n:(a + 1) * n].toarray()
        assert np.array_equal(blk, K0)
    # within a level all off-diagonal blocks vanish (Lemma of Section 3)
    for l in range(s.p + 1):
        lo, hi = s.off[l], s.off[l + 1]
        for a in range(lo, hi):
            for b in range(lo, hi):
                if a != b:
                    assert A[a * n:(a + 1) * n, b * n:(b + 1) * n].nnz == 0 or \
                        not np.any(A[a * n:(a + 1) * n, b * n:(b + 1) * n].toarray())
    # C_l = B_l^T (symmetric K_k, Remark of Section 3)
    assert abs(A - A.T).max() == 0.0


def test_coupling_rows_of_linear_kl():
    """B_l = A[deg < l, deg = l] is non-zero only in the degree l-1 rows."""
    prob = named_problem("small", n_e=5, M=3, p=3)
    s = sg.build_system(prob)
    pat = chaos.block_pattern(s.G) != 0
    for l in range(1, s.p + 1):
        assert not np.any(pat[: s.off[l - 1], s.off[l]:s.off[l + 1]])
        assert np.any(pat[s.off[l - 1]:s.off[l], s.off[l]:s.off[l + 1]])


def test_mean_problem_special_case():
    """p = 0 (P = 1): the SG system is the deterministic mean problem K_0 u = f."""
    prob = named_problem("small", p=0)
    s = sg.build_system(prob)
    A = sg.assemble(s)
    assert abs(A - s.K[0]).max() == 0.0
    F = prob.load_block().T.copy()
    res, _, _ = solve.solve_fcg(s, F, "hsc", "exact", rtol=1e-12)
    u = np.linalg.solve(s.K[0].toarray(), F[:, 0])
    assert res.iterations == 1
    assert np.linalg.norm(res.x[:, 0] - u) <= 1e-12 * np.linalg.norm(u)


def test_zero_variance_special_case():
    """sigma = 0: u_0 = K_0^-1 f, higher blocks vanish, and HSC is exact (one iteration)."""
    prob = named_problem("small", sigma=0.0)
    s = sg.build_system(prob)
    F = prob.load_block().T.copy()
    res, _, _ = solve.solve_fcg(s, F, "hsc", "exact", rtol=1e-10)
    u = np.linalg.solve(s.K[0].toarray(), F[:, 0])
    assert res.iterations == 1
    assert np.linalg.norm(res.x[:, 0] - u) <= 1e-12 * np.linalg.norm(u)
    assert np.max(np.abs(res.x[:, 1:])) == 0.0


def _constant_mode_problem(n_e, p, theta0, c):
    phi = np.ones((1, n_e, n_e))
    return Problem(name="const", n_e=n_e, M=1, p=p, theta0=theta0, sigma=c, L=1.0,
                   s=np.array([1.0]), phi=phi, f_nodal=nodal_rhs(n_e))


@pytest.mark.parametrize("p", [1, 3, 5])
def test_constant_mode_gauss_quadrature_closed_form(p):
    """a = theta0 + c xi: E[u] and sum_j u_j^2 from the (p+1)-point Gauss-Hermite rule."""
    n_e, theta0, c = 8, 1.0, 0.2
    prob = _constant_mode_problem(n_e, p, theta0, c)
    s = sg.build_system(prob)
    F = prob.load_block().T.copy()
    x, w = hermite_e.hermegauss(p + 1)
    w = w / w.sum()
    v = np.linalg.solve(fe.laplacian(n_e).toarray(), F[:, 0])
    S1 = np.sum(w / (theta0 + c * x))
    S2 = np.sum(w / (theta0 + c * x) ** 2)
    Ud = solve.solve_direct(s, F)
    res, _, _ = solve.solve_fcg(s, F, "hsc", "exact", rtol=1e-13)
    for U in (Ud, res.x):
        assert np.linalg.norm(U[:, 0] - S1 * v) <= 1e-11 * np.linalg.norm(v)
        var = np.sum(U[:, 1:] ** 2, axis=1)
        assert np.linalg.norm(var - (S2 - S1 ** 2) * v ** 2) <= 1e-10 * np.linalg.norm(v ** 2)


def test_fcg_hsc_matches_direct_small():
    prob = named_problem("small")
    s = sg.build_system(prob)
    F = prob.load_block().T.copy()
    Ud = solve.solve_direct(s, F)
    res, cnt, _ = solve.solve_fcg(s, F, "hsc", "exact", rtol=1e-8)
    assert res.converged
    A = sg.assemble(s).toarray()
    ev = np.linalg.eigvalsh(A)
    assert ev.min() > 0
    kappa = ev.max() / ev.min()
    err = np.linalg.norm(res.x - Ud) / np.linalg.norm(Ud)
    assert err <= kappa * 1e-8
    assert solve.true_relres(s, F, res.x) <= 1e-8 * 1.05


def test_fcg_equals_pcg_with_fixed_preconditioner():
    """With exact inner solves M_P is fixed and SPD, so FCG and PCG take the same steps."""
    prob = named_problem("small")
    s = sg.build_system(prob)
    F = prob.load_block().T.copy()
    from oracle import hsc
    ex = hsc.ExactMeanSolver(s)
    for M in (lambda R: hsc.hsc_apply(s, R, ex), lambda R: hsc.mean_apply(s, R, ex)):
        r1 = krylov.fcg(lambda U: sg.matvec(s, U), M, F, 1e-10, 100)
        r2 = krylov.pcg(lambda U: sg.matvec(s, U), M, F, 1e-10, 100)
        assert abs(r1.iterations - r2.iterations) <= 1
        assert np.linalg.norm(r1.x - r2.x) <= 1e-8 * np.linalg.norm(r2.x)


@pytest.mark.parametrize("kw", [dict(), dict(n_e=12, M=3, p=3, sigma=0.3),
                                dict(n_e=10, M=4, p=4, family="legendre", sigma=0.5, L=0.5)])
def test_error_bound_constant_bounds_the_inverse(kw):
    """||A^-1||_2 <= c (the margin bound A >= m I (x) K_Lap) against the dense
    spectrum, and c is not loose by more than a small factor."""
    from oracle import solve
    prob = named_problem("small", **kw)
    s = sg.build_system(prob)
    lmin = float(np.linalg.eigvalsh(sg.assemble(s).toarray()).min())
    c = solve.error_bound_constant(prob)
    assert 1.0 <= lmin * c <= 3.0
