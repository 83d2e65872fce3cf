"""Pins of the oracle's Legendre chaos (uniform variables on [-1, 1]).

The Hermite family is pinned in test_oracle_chaos.py and test_oracle_sg.py;
here the same checks are made for the family of the paper's examples
(Section 6), plus the paper's own iteration counts and condition estimates.
"""

import itertools
import math
import os

import numpy as np
import pytest
from numpy.polynomial import legendre

from oracle import chaos, fe, krylov, sg, solve
from sg_inputs import Problem, named_problem, nodal_rhs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "legendre_tables.txt")


def test_three_term_recurrence_and_orthonormality():
    """xi P_n = ((n + 1) P_{n+1} + n P_{n-1}) / (2n + 1), so for the normalised
    polynomials E[xi psi_n psi_{n+1}] = (n + 1) / sqrt((2n + 1)(2n + 3)), and
    every other pair gives zero."""
    for a in range(8):
        for b in range(8):
            assert abs(chaos.normalized_moment(0, a, b, "legendre") - (a == b)) < 1e-13
            m = max(a, b)
            expect = m / math.sqrt((2 * m - 1) * (2 * m + 1)) if abs(a - b) == 1 else 0.0
            assert abs(chaos.normalized_moment(1, a, b, "legendre") - expect) < 1e-13


@pytest.mark.parametrize("M,p", [(2, 3), (4, 4), (6, 2)])
def test_galerkin_matrix_entries(M, p):
    al = chaos.multi_indices(M, p)
    Gs = chaos.galerkin_matrices(M, p, family="legendre")
    assert np.array_equal(Gs[0], np.eye(al.shape[0]))
    for k in range(1, M + 1):
        G = Gs[k]
        assert np.array_equal(G, G.T)
        diff = al[:, None, :] - al[None, :, :]
        only_k = (np.abs(diff).sum(axis=2) == 1) & (np.abs(diff[:, :, k - 1]) == 1)
        m = np.maximum(al[:, None, k - 1], al[None, :, k - 1])
        expect = np.where(only_k, m / np.sqrt(np.maximum((2 * m - 1) * (2 * m + 1), 1)), 0.0)
        assert np.max(np.abs(G - expect)) < 1e-13
        assert np.array_equal(G != 0, only_k)


def test_galerkin_system_by_tensor_quadrature():
    """A = E[psi psi^T (x) K(xi)] on a tensor Gauss-Legendre grid (brute force)."""
    prob = named_problem("paper_legendre", n_e=4, M=2, p=2, sigma=0.4)
    s = sg.build_system(prob)
    A = sg.assemble(s).toarray()
    alpha = chaos.multi_indices(prob.M, prob.p)
    x, w = legendre.leggauss(prob.p + 2)
    w = w / w.sum()
    Aq = np.zeros_like(A)
    for idx in itertools.product(range(len(x)), repeat=prob.M):
        xi = x[list(idx)]
        wq = np.prod(w[list(idx)])
        psi = np.array([np.prod([math.sqrt(2 * a[d] + 1) * legendre.legval(xi[d], np.eye(prob.p + 1)[a[d]])
                                 for d in range(prob.M)]) for a in alpha])
        coef = prob.theta0 + prob.sigma * np.einsum("k,kij->ij", prob.s * xi, prob.phi)
        Kq = fe.assemble_stiffness(coef, prob.n_e).toarray()
        Aq += wq * np.kron(np.outer(psi, psi), Kq)
    assert np.max(np.abs(A - Aq)) <= 1e-12 * np.max(np.abs(A))


@pytest.mark.parametrize("p", [1, 3, 5])
def test_constant_mode_gauss_legendre_rule(p):
    """a = theta0 + c xi, xi ~ U[-1, 1]: the Galerkin solution equals the
    (p+1)-point Gauss-Legendre rule, E[u] = sum_q w_q / (theta0 + c x_q) K_Lap^-1 f
    and sum_{j>=1} u_j^2 = [sum_q w_q / a_q^2 - (sum_q w_q / a_q)^2] (K_Lap^-1 f)^2."""
    n_e, theta0, c = 8, 1.0, 0.6
    prob = Problem(name="const", n_e=n_e, M=1, p=p, theta0=theta0, sigma=c, L=1.0, s=np.array([1.0]),
                   phi=np.ones((1, n_e, n_e)), f_nodal=nodal_rhs(n_e), family="legendre")
    s = sg.build_system(prob)
    F = prob.load_block().T.copy()
    x, w = legendre.leggauss(p + 1)
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


def _golden_rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            rows.append((int(t[0]), t[1], float(t[2]), [(int(t[3]), float(t[4])), (int(t[5]), float(t[6])),
                                                        (int(t[7]), float(t[8]))]))
    return rows


def _row_param(r):
    # rows with P >= 210 chaos functions (Table 1 N >= 6, Table 2 P >= 6) take
    # 5-10 s each: run with SGPC_RUN_SLOW=1
    big = (r[1] == "N" and r[2] >= 6) or (r[1] == "P" and r[2] >= 6)
    return pytest.param(r, marks=pytest.mark.slow if big else (), id=f"T{r[0]}-{r[1]}{r[2]:g}")


@pytest.mark.parametrize("row", [_row_param(r) for r in _golden_rows()])
def test_paper_tables_1_to_4(row):
    """The oracle's flexible CG with exact inner solves against the paper's
    Tables 1-4. The KL data are computed here with a Nystrom method and the
    Dirichlet nodes are eliminated, so the counts may differ slightly: each
    count is at most the paper's and at most two below it, and each condition
    estimate within 20 % of the paper's (the largest gap, -16 %, is the
    mean-based estimate on the 5 x 5 mesh, where the KL data are coarsest).
    One entry is allowed three below: the mean-based count at N = 5 (15 against
    18). The separable exponential kernel gives the KL modes (0, 2) and (2, 0)
    exactly equal eigenvalues; N = 4 takes one of them and N = 5 both, while
    the paper's KL, computed numerically on its mesh, need not tie them, so its
    fifth mode can differ (test_kl_dimension_interlacing pins the N sequence).
    Unit-variance uniform variables on [-sqrt(3), sqrt(3)] instead would give
    two to three times the paper's iteration counts."""
    _, key, val, ref = row
    kw = {}
    if key == "N":
        kw["M"] = int(val)
    elif key == "P":
        kw["p"] = int(val)
    elif key == "CoV":
        kw["sigma"] = val / 100.0
    elif key == "h":
        kw["n_e"] = int(val)
    prob = named_problem("paper_legendre", **kw)
    s = sg.build_system(prob)
    F = prob.load_block().T.copy()
    for pc, (it_ref, kappa_ref) in zip(("mean", "bgs", "hsc"), ref):
        res, _, _ = solve.solve_fcg(s, F, pc, "exact", rtol=1e-8, maxit=100)
        assert res.converged
        slack = 3 if (key, val, pc) == ("N", 5.0, "mean") else 2
        assert it_ref - slack <= res.iterations <= it_ref, (pc, res.iterations, it_ref)
        kappa = krylov.lanczos_kappa(res.alphas, res.betas)
        assert abs(kappa - kappa_ref) <= 0.20 * kappa_ref, (pc, kappa, kappa_ref)


def test_kl_dimension_interlacing():
    """The N - 1 term system is a compression of the N term one (its chaos
    space and KL terms are a subset), so the extreme generalised eigenvalues of
    (A, M_m^-1) spread out as N grows (Cauchy interlacing) and the condition
    number of M_m A does not decrease. The Lanczos estimates from a seeded
    random right-hand side (no symmetry of f = 1 to hide part of the spectrum)
    follow that, within 2 %, over N = 1..5 (degree 4, CoV 50 %)."""
    kappas = []
    for N in range(1, 6):
        prob = named_problem("paper_legendre", M=N)
        s = sg.build_system(prob)
        R = np.random.default_rng(7).standard_normal((s.n, s.P))
        res, _, _ = solve.solve_fcg(s, R, "mean", "exact", rtol=1e-8, maxit=100)
        assert res.converged
        kappas.append(krylov.lanczos_kappa(res.alphas, res.betas))
    for a, b in zip(kappas, kappas[1:]):
        assert b >= 0.98 * a, kappas
