"""Pins of the oracle's preconditioners and inner solver."""

import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

from oracle import fe, hsc, krylov, sg
from sg_inputs import named_problem


def _dense_operator(apply, n):
    return np.column_stack([apply(np.eye(n)[:, j]) for j in range(n)])


def _hsc_dense(s):
    ex = hsc.ExactMeanSolver(s)
    N = s.n * s.P

    def ap(v):
        return sg.vec(hsc.hsc_apply(s, sg.unvec(v, s.n), ex))
    return _dense_operator(ap, N)


def test_hsc_p1_equals_block_inverse_formula():
    """p = 1: Algorithm 1 is the block inverse of eq. (block-inverse) with S replaced by A_0."""
    prob = named_problem("small", n_e=4, M=2, p=1, sigma=0.3)
    s = sg.build_system(prob)
    A = sg.assemble(s).toarray()
    M_alg = _hsc_dense(s)
    M_ref = hsc.hsc_dense_p1(A, s.n, s.P)
    assert np.max(np.abs(M_alg - M_ref)) <= 1e-13 * np.max(np.abs(M_ref))


@pytest.mark.parametrize("p", [2, 3])
def test_hsc_symmetric_positive_definite(p):
    """Theorem 1: with exact solves M_P is SPD for SPD A_P."""
    prob = named_problem("small", n_e=4, M=2, p=p, sigma=0.3)
    s = sg.build_system(prob)
    Md = _hsc_dense(s)
    assert np.max(np.abs(Md - Md.T)) <= 1e-12 * np.max(np.abs(Md))
    ev = np.linalg.eigvalsh(0.5 * (Md + Md.T))
    assert ev.min() > 0
    A = sg.assemble(s).toarray()
    evp = np.linalg.eigvals(Md @ A).real
    assert evp.min() > 0


def test_hsc_zero_degree_is_mean_inverse():
    prob = named_problem("small", n_e=6, p=0)
    s = sg.build_system(prob)
    R = np.random.default_rng(3).standard_normal((s.n, 1))
    Z = hsc.hsc_apply(s, R, hsc.ExactMeanSolver(s))
    ref = np.linalg.solve(s.K[0].toarray(), R)
    assert np.linalg.norm(Z - ref) <= 1e-13 * np.linalg.norm(ref)


def test_pre_correction_touches_only_previous_degree():
    prob = named_problem("small", n_e=5, M=3, p=3)
    s = sg.build_system(prob)
    rng = np.random.default_rng(4)
    for l in range(1, s.p + 1):
        lo, hi = s.off[l], s.off[l + 1]
        y = rng.standard_normal((s.n, hi - lo))
        out = sg.level_block(s, slice(0, lo), slice(lo, hi))(y)
        assert not np.any(out[:, : s.off[l - 1]])
        assert np.any(out[:, s.off[l - 1]:lo])


@pytest.mark.parametrize("degree", [1, 2, 4, 7])
def test_chebyshev_residual_polynomial(degree):
    """On an eigenvector of D^-1 K_0 with eigenvalue lam, 1 - lam p(lam) = T_d((theta-lam)/delta)/T_d(theta/delta)."""
    n_e = 8
    K0 = fe.assemble_stiffness(np.full((n_e, n_e), 1.7), n_e)
    prec = krylov.make_chebyshev(K0, n_e, 1.7, degree)
    theta = 0.5 * (prec.lmax + prec.lmin)
    delta = 0.5 * (prec.lmax - prec.lmin)
    m = n_e - 1
    x = np.arange(1, n_e) / n_e
    Td = np.zeros(degree + 1)
    Td[degree] = 1.0
    for (i, j) in [(1, 1), (2, 5), (m, 1), (m, m), (3, 3)]:
        v = np.outer(np.sin(j * math.pi * x), np.sin(i * math.pi * x)).ravel()
        lam = ((8 - 2 * math.cos(i * math.pi / n_e) - 2 * math.cos(j * math.pi / n_e)
                - 4 * math.cos(i * math.pi / n_e) * math.cos(j * math.pi / n_e)) / 8.0)
        z = prec.apply((prec.diag * v)[:, None])[:, 0]
        p_lam = z @ v / (v @ v)
        assert np.linalg.norm(z - p_lam * v) <= 1e-12 * np.linalg.norm(z)
        expect = npcheb.chebval((theta - lam) / delta, Td) / npcheb.chebval(theta / delta, Td)
        assert abs((1.0 - lam * p_lam) - expect) < 1e-12


def test_chebyshev_preconditioner_is_spd():
    n_e = 6
    K0 = fe.laplacian(n_e)
    prec = krylov.make_chebyshev(K0, n_e, 1.0, 4)
    Md = _dense_operator(lambda v: prec.apply(v[:, None])[:, 0], K0.shape[0])
    assert np.max(np.abs(Md - Md.T)) < 1e-13
    assert np.linalg.eigvalsh(Md).min() > 0


def test_inner_pcg_converges_and_masks_zero_columns():
    n_e = 20
    K0 = fe.assemble_stiffness(np.full((n_e, n_e), 1.3), n_e)
    prec = krylov.make_chebyshev(K0, n_e, 1.3, 4)
    rng = np.random.default_rng(5)
    B = rng.standard_normal((K0.shape[0], 4))
    B[:, 2] = 0.0
    st = krylov.InnerStats()
    X = krylov.pcg_columns(K0, B, prec, 1e-10, 500, st)
    ref = np.linalg.solve(K0.toarray(), B)
    assert st.iterations[2] == 0 and np.all(X[:, 2] == 0.0)
    for j in (0, 1, 3):
        assert np.linalg.norm(B[:, j] - K0 @ X[:, j]) <= 1.01e-10 * np.linalg.norm(B[:, j])
        assert np.linalg.norm(X[:, j] - ref[:, j]) <= 1e-7 * np.linalg.norm(ref[:, j])
    # a higher degree needs fewer iterations
    st2 = krylov.InnerStats()
    krylov.pcg_columns(K0, B, krylov.make_chebyshev(K0, n_e, 1.3, 8), 1e-10, 500, st2)
    assert st2.iterations[0] < st.iterations[0]


def test_lanczos_kappa_exact_on_diagonal_matrix():
    d = np.array([1.0, 2.0, 3.5, 10.0, 40.0])
    A = np.diag(d)
    b = np.ones(5)
    # alphas / betas of plain CG
    x = np.zeros(5); rr = b.copy(); p = rr.copy(); g = rr @ rr
    al, be = [], []
    for _ in range(5):
        q = A @ p; a = g / (p @ q); al.append(a)
        x += a * p; rr -= a * q; gn = rr @ rr
        if gn < 1e-28:
            break
        be.append(gn / g); p = rr + (gn / g) * p; g = gn
    assert abs(krylov.lanczos_kappa(al, be) - 40.0) < 1e-8


def test_mean_preconditioner_is_block_inverse():
    prob = named_problem("small", n_e=6, M=2, p=2)
    s = sg.build_system(prob)
    R = np.random.default_rng(6).standard_normal((s.n, s.P))
    Z = hsc.mean_apply(s, R, hsc.ExactMeanSolver(s))
    assert np.linalg.norm(s.K[0] @ Z - R) <= 1e-12 * np.linalg.norm(R)
    assert hsc.diagonal_blocks_are_mean(s)


def test_inner_pcg_initial_guess():
    """PCG from an initial guess x0: the textbook shift x = x0 + d, K_0 d = b - K_0 x0."""
    n_e = 18
    K0 = fe.assemble_stiffness(np.full((n_e, n_e), 0.9), n_e)
    prec = krylov.make_chebyshev(K0, n_e, 0.9, 3)
    rng = np.random.default_rng(11)
    n = K0.shape[0]
    B = rng.standard_normal((n, 4))
    B[:, 1] = 0.0
    X0 = rng.standard_normal((n, 4))
    ref = np.linalg.solve(K0.toarray(), B)
    # exact initial guess: no iteration, x0 returned; a zero column gives 0 whatever x0
    st = krylov.InnerStats()
    X = krylov.pcg_columns(K0, B, prec, 1e-10, 500, st, ref)
    assert np.all(st.iterations == 0)
    assert np.array_equal(X[:, [0, 2, 3]], ref[:, [0, 2, 3]]) and np.all(X[:, 1] == 0.0)
    X = krylov.pcg_columns(K0, B, prec, 1e-10, 500, None, X0)
    assert np.all(X[:, 1] == 0.0)
    # fixed iteration count: the iterates from x0 are x0 plus those of the shifted system from 0
    for m in (1, 4):
        Xw = krylov.pcg_columns(K0, B, prec, 0.0, m, None, X0)
        D = krylov.pcg_columns(K0, B - K0 @ X0, prec, 0.0, m)
        for j in (0, 2, 3):
            assert np.linalg.norm(Xw[:, j] - (X0[:, j] + D[:, j])) <= 1e-12 * np.linalg.norm(Xw[:, j])
    # to tolerance from a random guess, and fewer iterations from a close one
    st_w, st_c = krylov.InnerStats(), krylov.InnerStats()
    Xw = krylov.pcg_columns(K0, B, prec, 1e-10, 500, st_w, X0)
    krylov.pcg_columns(K0, B, prec, 1e-10, 500, st_c, ref + 1e-4 * X0)
    for j in (0, 2, 3):
        assert np.linalg.norm(B[:, j] - K0 @ Xw[:, j]) <= 1.01e-10 * np.linalg.norm(B[:, j])
    st0 = krylov.InnerStats()
    krylov.pcg_columns(K0, B, prec, 1e-10, 500, st0)
    assert np.all(st_c.iterations[[0, 2, 3]] < st0.iterations[[0, 2, 3]])


def test_hsc_warm_up_sweep():
    """Starting the up-sweep solves from y_l changes nothing with exact solves and,
    with inner PCG to a tight tolerance, gives the same action in fewer inner iterations."""
    prob = named_problem("small", n_e=14, M=3, p=3, sigma=0.3)
    s = sg.build_system(prob)
    R = np.random.default_rng(4).standard_normal((s.n, s.P))
    ex = hsc.ExactMeanSolver(s)
    Zx = hsc.hsc_apply(s, R, ex)
    assert np.array_equal(hsc.hsc_apply(s, R, ex, warm=True), Zx)
    cold = hsc.PCGMeanSolver(s, 1e-12, 2000, 4)
    warm = hsc.PCGMeanSolver(s, 1e-12, 2000, 4)
    Zc = hsc.hsc_apply(s, R, cold)
    Zw = hsc.hsc_apply(s, R, warm, warm=True)
    assert np.linalg.norm(Zw - Zx) <= 1e-9 * np.linalg.norm(Zx)
    assert np.linalg.norm(Zc - Zx) <= 1e-9 * np.linalg.norm(Zx)
    up = slice(prob.p + 1, None)  # the up-sweep solves are the last p calls
    assert sum(int(v.sum()) for v in warm.iterations[up]) < sum(int(v.sum()) for v in cold.iterations[up])
