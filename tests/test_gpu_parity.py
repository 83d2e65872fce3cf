"""GPU path (through the C-ABI) against the CPU oracle."""

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import bgs, hsc, krylov, sg, solve  # noqa: E402
from sg_inputs import named_problem, random_block  # noqa: E402


def _b():
    from paper_1205_1864_amd import binding
    return binding


def _sys(**kw):
    prob = named_problem("small", **kw)
    return prob, sg.build_system(prob)


def _dev(A):
    return _b().to_device_block(A)


SHAPES = [dict(), dict(n_e=7, M=3, p=3), dict(n_e=33, M=5, p=2), dict(n_e=19, M=2, p=4),
          dict(n_e=10, M=3, p=0), dict(n_e=9, M=0, p=2), dict(n_e=40, M=6, p=3, sigma=0.15),
          # grid widths that take the register-strip kernel (multiples of 64, up to 512)
          dict(n_e=64, M=4, p=2), dict(n_e=64, M=12, p=2, sigma=0.1), dict(n_e=128, M=3, p=4),
          dict(n_e=64, M=0, p=3), dict(n_e=64, M=1, p=5), dict(n_e=192, M=7, p=2),
          dict(n_e=512, M=2, p=2), dict(n_e=64, M=13, p=2, sigma=0.1)]


@pytest.mark.parametrize("kw", SHAPES)
def test_matvec_parity(kw):
    b = _b()
    prob, s = _sys(**kw)
    print(f"matvec parity n_e={prob.n_e} M={prob.M} p={prob.p}", flush=True)
    solver = b.SGSolver(prob)
    U = random_block(prob.P, prob.n, seed=11)
    Y = solver.sg_matvec(_dev(U)).cpu().numpy()
    Yo = sg.matvec(s, U.T).T
    assert np.linalg.norm(Y - Yo) <= 1e-12 * np.linalg.norm(Yo)


@pytest.mark.parametrize("kw", SHAPES)
@pytest.mark.parametrize("rows", [1, 5, 16])
def test_matvec_parity_staged(kw, rows, monkeypatch):
    """The row-staged operator kernel (forced, with pieces of 1, 5 and 16 node
    rows) against the oracle on every shape."""
    monkeypatch.setenv("SGPC_MV_STAGE", str(rows))
    b = _b()
    prob, s = _sys(**kw)
    print(f"staged matvec parity n_e={prob.n_e} M={prob.M} p={prob.p} rows={rows}", flush=True)
    solver = b.SGSolver(prob)
    U = random_block(prob.P, prob.n, seed=11)
    Y = solver.sg_matvec(_dev(U)).cpu().numpy()
    Yo = sg.matvec(s, U.T).T
    assert np.linalg.norm(Y - Yo) <= 1e-12 * np.linalg.norm(Yo)


@pytest.mark.parametrize("rows", [0, 10])
def test_matvec_parity_scale(rows, monkeypatch):
    monkeypatch.setenv("SGPC_MV_STAGE", str(rows))
    b = _b()
    prob = named_problem("scale")
    print(f"matvec parity 256^2 M=10 p=3 staged rows={rows}", flush=True)
    s = sg.build_system(prob)
    solver = b.SGSolver(prob)
    U = random_block(prob.P, prob.n, seed=0)
    Y = solver.sg_matvec(_dev(U)).cpu().numpy()
    Yo = sg.matvec(s, U.T).T
    assert np.linalg.norm(Y - Yo) <= 1e-12 * np.linalg.norm(Yo)


@pytest.mark.parametrize("prec,tol", [(64, 1e-11), (32, 2e-5)])
@pytest.mark.parametrize("degree,tile", [(4, 0), (1, 16), (6, 32)])
def test_inner_solve_fixed_iterations(prec, tol, degree, tile):
    b = _b()
    prob, s = _sys(n_e=45, M=2, p=2)
    print(f"inner solve prec={prec} degree={degree} tile={tile}", flush=True)
    solver = b.SGSolver(prob, b.Options(inner_precision=prec, cheb_degree=degree, inner_maxit=9,
                                        inner_rtol=0.0, tile=tile))
    B = random_block(5, prob.n, seed=3)
    B[2] = 0.0
    X, its = solver.sg_inner_solve(_dev(B))
    X = X.cpu().numpy()
    prec_o = krylov.make_chebyshev(s.K[0], prob.n_e, prob.theta0, degree)
    st = krylov.InnerStats()
    Xo = krylov.pcg_columns(s.K[0], B.T, prec_o, 0.0, 9, st).T
    assert list(its) == list(st.iterations)
    assert np.all(X[2] == 0.0)
    for c in (0, 1, 3, 4):
        assert np.linalg.norm(X[c] - Xo[c]) <= tol * np.linalg.norm(Xo[c])


@pytest.mark.parametrize("prec,tol", [(64, 1e-11), (32, 2e-5)])
@pytest.mark.parametrize("n_e", [4, 33, 34, 49, 50, 130])
@pytest.mark.parametrize("degree", [1, 2, 3, 4, 5, 8, 12, 16])
def test_inner_solve_band_geometry(prec, tol, n_e, degree):
    """Banded inner tiles at the edges of their geometry: a grid smaller than
    the halo (n_e = 4); a tile plus its halo and the extra node exactly one
    wavefront wide (nx = 64 - 2d: n_e = 49 at degree 8, 33 at degree 16) and
    one column more (n_e = 50, 34); several ragged tiles in both directions
    (n_e = 130); every halo capacity (degree <= 4, 8, 12, 16)."""
    b = _b()
    prob, s = _sys(n_e=n_e, M=2, p=1)
    print(f"inner band prec={prec} n_e={n_e} degree={degree}", flush=True)
    solver = b.SGSolver(prob, b.Options(inner_precision=prec, cheb_degree=degree, inner_maxit=7,
                                        inner_rtol=0.0, tile=32))
    B = random_block(3, prob.n, seed=n_e + degree)
    X, its = solver.sg_inner_solve(_dev(B))
    X = X.cpu().numpy()
    prec_o = krylov.make_chebyshev(s.K[0], prob.n_e, prob.theta0, degree)
    st = krylov.InnerStats()
    Xo = krylov.pcg_columns(s.K[0], B.T, prec_o, 0.0, 7, st).T
    assert list(its) == list(st.iterations)
    for c in range(3):
        assert np.linalg.norm(X[c] - Xo[c]) <= tol * np.linalg.norm(Xo[c])


@pytest.mark.parametrize("prec,tol", [(64, 1e-11), (32, 2e-5)])
@pytest.mark.parametrize("degree", [2, 8, 16])
@pytest.mark.parametrize("tile", [0, 32])
def test_inner_solve_tall_grid(prec, tol, degree, tile):
    """Several bands in y at every band height: 299 unknown rows take three
    128-row bands (FP64) or two 256-row bands (FP32), the last one ragged, with
    tile = 32; with tile = 0 the three-column launch is small enough for the
    64-row bands (five per tile column) that load the next tile ahead."""
    b = _b()
    prob, s = _sys(n_e=300, M=2, p=1)
    print(f"inner tall prec={prec} degree={degree} tile={tile}", flush=True)
    solver = b.SGSolver(prob, b.Options(inner_precision=prec, cheb_degree=degree, inner_maxit=6,
                                        inner_rtol=0.0, tile=tile))
    B = random_block(3, prob.n, seed=300 + degree)
    X, its = solver.sg_inner_solve(_dev(B))
    X = X.cpu().numpy()
    prec_o = krylov.make_chebyshev(s.K[0], prob.n_e, prob.theta0, degree)
    st = krylov.InnerStats()
    Xo = krylov.pcg_columns(s.K[0], B.T, prec_o, 0.0, 6, st).T
    assert list(its) == list(st.iterations)
    for c in range(3):
        assert np.linalg.norm(X[c] - Xo[c]) <= tol * np.linalg.norm(Xo[c])


@pytest.mark.parametrize("prec,tol", [(64, 1e-11), (32, 2e-5)])
def test_inner_solve_small_launch_band_height(prec, tol):
    """The automatic band height of a small launch on the benchmark's grid: ten
    columns of 255 x 255 unknowns at degree 16 make 140 tiles of 128 rows or
    280 of 64 rows; on 256 compute units the launch takes 128-row bands (one
    tile per block) in both precisions, the FP32 kernel's middle height."""
    b = _b()
    prob, s = _sys(n_e=256, M=3, p=2)
    assert prob.P == 10
    print(f"inner small launch prec={prec}", flush=True)
    solver = b.SGSolver(prob, b.Options(inner_precision=prec, cheb_degree=16, inner_maxit=5,
                                        inner_rtol=0.0, tile=0))
    B = random_block(10, prob.n, seed=256)
    X, its = solver.sg_inner_solve(_dev(B))
    X = X.cpu().numpy()
    prec_o = krylov.make_chebyshev(s.K[0], prob.n_e, prob.theta0, 16)
    st = krylov.InnerStats()
    Xo = krylov.pcg_columns(s.K[0], B.T, prec_o, 0.0, 5, st).T
    assert list(its) == list(st.iterations)
    for c in range(10):
        assert np.linalg.norm(X[c] - Xo[c]) <= tol * np.linalg.norm(Xo[c])


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("degree", [16, 3])
def test_inner_schedules_bitwise_equal(prec, degree, monkeypatch):
    """The inner launch schedules (the automatic grid, a cap of 128 blocks, and
    whole columns per block, whose column phases need no device-scope counters)
    run the same arithmetic per column: bitwise equal iterates and iteration
    counts, for the 220 top-level columns of the 256^2 benchmark grid, at fixed
    iteration counts and to a tolerance; the first schedule's fixed-iteration
    iterates also agree with the oracle's PCG on sampled columns."""
    b = _b()
    prob = named_problem("scale")
    B = random_block(220, prob.n, seed=3)
    Bd = _dev(B)
    res = []
    for mb in ("0", "128", "-1"):
        print(f"inner schedule max_blocks={mb} prec={prec} degree={degree}", flush=True)
        monkeypatch.setenv("SGPC_PCG_MAX_BLOCKS", mb)
        solver = b.SGSolver(prob, b.Options(inner_precision=prec, cheb_degree=degree, inner_maxit=12, inner_rtol=0.0))
        X12, its12 = solver.sg_inner_solve(Bd)
        solver.set_opts(b.Options(inner_precision=prec, cheb_degree=degree, inner_maxit=2000, inner_rtol=1e-4))
        Xt, itst = solver.sg_inner_solve(Bd)
        res.append((X12.cpu(), list(its12), Xt.cpu(), list(itst)))
        solver.close()
    for X12, its12, Xt, itst in res[1:]:
        assert bool((X12 == res[0][0]).all()) and its12 == res[0][1]
        assert bool((Xt == res[0][2]).all()) and itst == res[0][3]
    assert all(i == 12 for i in res[0][1])
    K0 = sg.build_system(prob).K[0]
    prec_o = krylov.make_chebyshev(K0, prob.n_e, prob.theta0, degree)
    cols = [0, 97, 219]
    st = krylov.InnerStats()
    Xo = krylov.pcg_columns(K0, B[cols].T, prec_o, 0.0, 12, st).T
    tol = 1e-11 if prec == 64 else 2e-5
    for j, c in enumerate(cols):
        assert np.linalg.norm(res[0][0][c].numpy() - Xo[j]) <= tol * np.linalg.norm(Xo[j])


@pytest.mark.parametrize("pc,prec,warm", [("hsc", 64, False), ("hsc", 32, True), ("bgs", 64, True),
                                         ("mean", 32, False)])
def test_solve_graph_replay_equals_eager(pc, prec, warm):
    """use_graph: the preconditioner action captured once and replayed in every
    outer iteration (eager FCG work and host synchronisation between replays)
    gives the eager solve bit for bit, with the same counters, in two solves in
    a row (the second replays the first one's graph) and after the options
    change (the graph is captured again)."""
    import torch
    b = _b()
    prob, s = _sys(n_e=40, M=4, p=3)
    print(f"graph replay pc={pc} prec={prec} warm={warm}", flush=True)
    F = _dev(prob.load_block())
    base = dict(inner_precision=prec, precond=pc, cheb_degree=8, inner_rtol=1e-4, warm_start=warm)
    eager = b.SGSolver(prob, b.Options(**base))
    graph = b.SGSolver(prob, b.Options(**base, use_graph=True))
    assert graph.stream.cuda_stream != 0
    keys = ("outer_it", "inner_it_total", "n_blockmv", "n_blocksolve", "inner_launches")
    for degree in (8, 5):
        if degree != 8:
            eager.set_opts(b.Options(**dict(base, cheb_degree=degree)))
            graph.set_opts(b.Options(**dict(base, cheb_degree=degree), use_graph=True))
        Ue, se = eager.sg_solve(F, rtol=1e-8, maxit=100)
        for rep in range(2):
            Ug, sg_ = graph.sg_solve(F, rtol=1e-8, maxit=100)
            torch.cuda.synchronize()
            assert se["rc"] == 0 and sg_["rc"] == 0
            assert bool((Ug == Ue).all()), (degree, rep, float((Ug - Ue).abs().max()))
            assert all(sg_[k] == se[k] for k in keys), ({k: (sg_[k], se[k]) for k in keys})
            assert sg_["inner_it_max"] == se["inner_it_max"]
            # with a graph, ms_inner times the replayed actions as a whole
            assert sg_["ms_inner"] >= 0.5 * se["ms_inner"] and sg_["ms_inner"] <= 2.0 * sg_["ms_precond"] + 1.0
    assert solve.true_relres(s, prob.load_block().T, Ug.cpu().numpy().T) <= 1.05e-8
    eager.close()
    graph.close()


@pytest.mark.parametrize("prec", [64, 32])
def test_inner_solve_to_tolerance(prec):
    b = _b()
    prob, s = _sys(n_e=64, M=2, p=3)
    rtol = 1e-6 if prec == 64 else 1e-4
    solver = b.SGSolver(prob, b.Options(inner_precision=prec, cheb_degree=4, inner_maxit=500, inner_rtol=rtol))
    B = random_block(7, prob.n, seed=4)
    X, its = solver.sg_inner_solve(_dev(B))
    X = X.cpu().numpy()
    prec_o = krylov.make_chebyshev(s.K[0], prob.n_e, prob.theta0, 4)
    st = krylov.InnerStats()
    krylov.pcg_columns(s.K[0], B.T, prec_o, rtol, 500, st)
    for c in range(7):
        r = B[c] - s.K[0] @ X[c]
        assert np.linalg.norm(r) <= rtol * 1.2 * np.linalg.norm(B[c])
        assert abs(int(its[c]) - int(st.iterations[c])) <= 1


@pytest.mark.parametrize("kw", [dict(), dict(n_e=21, M=3, p=3), dict(n_e=12, M=5, p=2),
                                dict(n_e=64, M=5, p=3), dict(n_e=128, M=10, p=2)])
def test_coupling_parity(kw):
    b = _b()
    prob, s = _sys(**kw)
    print(f"coupling parity n_e={prob.n_e} M={prob.M} p={prob.p}", flush=True)
    solver = b.SGSolver(prob)
    rng = np.random.default_rng(7)
    for l in range(1, prob.p + 1):
        for d in (0, 1):
            R = rng.standard_normal((prob.P, prob.n))
            V = rng.standard_normal((prob.P, prob.n))
            Rg = solver.sg_coupling(l, d, _dev(R), _dev(V)).cpu().numpy()
            Ro = R.T.copy()
            lo, hi = s.off[l], s.off[l + 1]
            if d == 0:
                Ro[:, :lo] -= sg.level_block(s, slice(0, lo), slice(lo, hi))(V.T[:, lo:hi])
            else:
                Ro[:, lo:hi] -= sg.level_block(s, slice(lo, hi), slice(0, lo))(V.T[:, :lo])
            assert np.linalg.norm(Rg - Ro.T) <= 1e-13 * np.linalg.norm(Ro)


@pytest.mark.parametrize("which", ["hsc", "mean", "bgs"])
@pytest.mark.parametrize("kw", [dict(n_e=24, M=3, p=3), dict(n_e=64, M=4, p=2), dict(n_e=19, M=2, p=4)])
def test_preconditioner_tight_parity(which, kw):
    b = _b()
    prob, s = _sys(**kw)
    solver = b.SGSolver(prob, b.Options(inner_precision=64, inner_rtol=1e-13, inner_maxit=2000))
    R = random_block(prob.P, prob.n, seed=8)
    apply = {"hsc": solver.sg_apply_hsc, "mean": solver.sg_apply_mean, "bgs": solver.sg_apply_bgs}[which]
    Z = apply(_dev(R)).cpu().numpy()
    ex = hsc.ExactMeanSolver(s)
    ref = {"hsc": lambda: hsc.hsc_apply(s, R.T, ex), "mean": lambda: hsc.mean_apply(s, R.T, ex),
           "bgs": lambda: bgs.bgs_apply(s, R.T, ex)}[which]
    Zo = ref().T
    assert np.linalg.norm(Z - Zo) <= 1e-9 * np.linalg.norm(Zo)


@pytest.mark.parametrize("which", ["hsc", "bgs"])
@pytest.mark.parametrize("kw", [dict(n_e=24, M=3, p=3), dict(n_e=64, M=4, p=2), dict(n_e=19, M=2, p=4)])
def test_preconditioner_tight_parity_warm(which, kw):
    """Warm-started up-sweep (backward-sweep) solves reach the same action."""
    b = _b()
    prob, s = _sys(**kw)
    solver = b.SGSolver(prob, b.Options(inner_precision=64, inner_rtol=1e-13, inner_maxit=2000, warm_start=True))
    R = random_block(prob.P, prob.n, seed=9)
    apply = solver.sg_apply_hsc if which == "hsc" else solver.sg_apply_bgs
    Z = apply(_dev(R)).cpu().numpy()
    ex = hsc.ExactMeanSolver(s)
    Zo = (hsc.hsc_apply(s, R.T, ex) if which == "hsc" else bgs.bgs_apply(s, R.T, ex)).T
    assert np.linalg.norm(Z - Zo) <= 1e-9 * np.linalg.norm(Zo)


@pytest.mark.parametrize("prec,tol", [(64, 1e-11), (32, 1e-4)])
@pytest.mark.parametrize("n_e", [4, 52, 130])
@pytest.mark.parametrize("degree,tile", [(1, 0), (2, 0), (4, 0), (8, 0), (4, 16)])
def test_hsc_warm_fixed_iterations(prec, tol, n_e, degree, tile):
    """Three inner iterations per solve, up sweep from y_l: element-wise against the
    oracle's Algorithm 1 with the same inner PCG from the same initial guesses (16 x 16
    tiles start from zero)."""
    b = _b()
    prob, s = _sys(n_e=n_e, M=2, p=2, sigma=0.3)
    solver = b.SGSolver(prob, b.Options(inner_precision=prec, cheb_degree=degree, inner_maxit=3, inner_rtol=0.0,
                                        tile=tile, warm_start=True))
    R = random_block(prob.P, prob.n, seed=12)
    Z = solver.sg_apply_hsc(_dev(R)).cpu().numpy()
    inner = hsc.PCGMeanSolver(s, 0.0, 3, degree)
    Zo = hsc.hsc_apply(s, R.T, inner, warm=tile != 16).T
    assert np.linalg.norm(Z - Zo) <= tol * np.linalg.norm(Zo)
    if tile != 16 and prec == 64 and n_e >= 52:
        # a cold start gives a different action (three iterations are far from converged here)
        Zc = hsc.hsc_apply(s, R.T, hsc.PCGMeanSolver(s, 0.0, 3, degree)).T
        assert np.linalg.norm(Z - Zc) > 1e3 * tol * np.linalg.norm(Zo)


def test_warm_start_saves_inner_iterations():
    b = _b()
    prob, s = _sys(n_e=64, M=4, p=3, sigma=0.3)
    F = prob.load_block()
    out = {}
    for warm in (False, True):
        solver = b.SGSolver(prob, b.Options(inner_precision=64, cheb_degree=8, inner_rtol=1e-4, warm_start=warm))
        U, st = solver.sg_solve(_dev(F), rtol=1e-8, maxit=100)
        assert st["rc"] == 0 and st["true_relres"] <= 1.05e-8
        out[warm] = (U.cpu().numpy(), st)
    (Uc, sc), (Uw, sw) = out[False], out[True]
    assert abs(sc["outer_it"] - sw["outer_it"]) <= 1
    assert sw["inner_it_total"] < sc["inner_it_total"]
    assert np.linalg.norm(Uw - Uc) <= 1e-6 * np.linalg.norm(Uc)


@pytest.mark.parametrize("prec,pc,warm", [(64, "hsc", False), (32, "hsc", False), (64, "mean", False),
                                          (32, "mean", False), (64, "bgs", False), (32, "bgs", False),
                                          (64, "hsc", True), (32, "hsc", True), (64, "bgs", True), (32, "bgs", True)])
def test_solve_small(prec, pc, warm):
    b = _b()
    prob, s = _sys()
    F = prob.load_block()
    solver = b.SGSolver(prob, b.Options(inner_precision=prec, precond=pc, inner_rtol=1e-4, warm_start=warm))
    U, st = solver.sg_solve(_dev(F), rtol=1e-8, maxit=100)
    U = U.cpu().numpy()
    assert st["rc"] == 0
    Ud = solve.solve_direct(s, F.T.copy())
    tr = solve.true_relres(s, F.T, U.T)
    assert tr <= 1.05e-8
    assert abs(st["true_relres"] - tr) <= 1e-3 * tr + 1e-15
    A = sg.assemble(s).toarray()
    ev = np.linalg.eigvalsh(A)
    assert np.linalg.norm(U.T - Ud) / np.linalg.norm(Ud) <= ev.max() / ev.min() * 1e-8
    P = prob.P
    n_b = int(np.count_nonzero(sum(np.abs(G) for G in s.G)))
    if pc == "hsc":
        assert st["n_blocksolve"] == st["outer_it"] * (2 * (P - 1) + 1)
        assert st["n_blockmv"] == st["outer_it"] * (n_b - P)
    if pc == "bgs":
        # the top level is solved once; the lower level products of the forward
        # sweep are kept, so one action costs one pass over the off-diagonal blocks
        top = int(s.off[prob.p + 1] - s.off[prob.p])
        assert st["n_blocksolve"] == st["outer_it"] * (2 * P - top)
        assert st["n_blockmv"] == st["outer_it"] * (n_b - P)


def test_solve_bgs_matches_oracle_iterates():
    """bGS-preconditioned FCG with (nearly) exact inner solves follows the oracle's."""
    b = _b()
    prob, s = _sys(n_e=20, M=3, p=3)
    F = prob.load_block()
    solver = b.SGSolver(prob, b.Options(inner_precision=64, precond="bgs", inner_rtol=1e-14, inner_maxit=3000))
    U, st = solver.sg_solve(_dev(F), rtol=1e-10, maxit=80)
    res, cnt, _ = solve.solve_fcg(s, F.T.copy(), "bgs", "exact", rtol=1e-10, maxit=80)
    assert st["rc"] == 0
    assert st["outer_it"] == res.iterations
    assert np.linalg.norm(U.cpu().numpy().T - res.x) <= 1e-10 * np.linalg.norm(res.x)
    # the oracle recomputes the lower products in the backward sweep (1.5x) and
    # solves every block twice; the GPU keeps both the top-level and the lower values
    assert cnt.block_solves == 2 * prob.P * res.iterations


def test_solve_tight_matches_oracle_iterates():
    """With (nearly) exact inner solves the GPU FCG follows the oracle's FCG."""
    b = _b()
    prob, s = _sys()
    F = prob.load_block()
    solver = b.SGSolver(prob, b.Options(inner_precision=64, inner_rtol=1e-14, inner_maxit=3000))
    U, st = solver.sg_solve(_dev(F), rtol=1e-10, maxit=50)
    res, _, _ = solve.solve_fcg(s, F.T.copy(), "hsc", "exact", rtol=1e-10)
    assert st["outer_it"] == res.iterations
    assert np.linalg.norm(U.cpu().numpy().T - res.x) <= 1e-10 * np.linalg.norm(res.x)


def test_solve_edge_cases():
    b = _b()
    prob, s = _sys(n_e=12, M=2, p=2)
    solver = b.SGSolver(prob)
    Z = np.zeros((prob.P, prob.n))
    U, st = solver.sg_solve(_dev(Z))
    assert st["rc"] == 0 and st["outer_it"] == 0 and float(U.abs().max()) == 0.0
    F = prob.load_block()
    U, st = solver.sg_solve(_dev(F), rtol=1e-12, maxit=1)
    assert st["rc"] == b.SG_NOT_CONVERGED and st["outer_it"] == 1
    Fn = F.copy()
    Fn[0, 3] = np.nan
    with pytest.raises(b.SGError):
        solver.sg_solve(_dev(Fn))


def test_argument_errors():
    """Aliased or out-of-range arguments are rejected before any work is enqueued."""
    from sg_inputs import qoi_weights
    b = _b()
    prob, s = _sys(n_e=12, M=2, p=2)
    solver = b.SGSolver(prob)
    Bd = _dev(random_block(2, prob.n, seed=5))
    with pytest.raises(b.SGError, match="distinct"):
        solver.sg_inner_solve(Bd, X=Bd)
    F = _dev(prob.load_block())
    with pytest.raises(b.SGError, match="distinct"):
        solver.sg_solve(F, U=F)
    U, st = solver.sg_solve(F, rtol=1e-10)
    wm, wv = (_b().to_device_vec(w) for w in qoi_weights(prob.n_e))
    with pytest.raises(b.SGError, match="Lambda"):
        solver.sg_adjoint_grad(U, wm, wv, Lambda=U)
    with pytest.raises(b.SGError, match="rtol"):
        solver.sg_adjoint_grad(U, wm, wv, rtol=-1.0)
    with pytest.raises(b.SGError, match="ncols"):
        solver.sg_inner_solve(_dev(random_block(prob.P + 1, prob.n, seed=6)))
    Q, g, st = solver.sg_adjoint_grad(U, wm, wv, rtol=1e-10)
    assert st["rc"] == 0 and np.all(np.isfinite(g))


def test_adjoint_parity_small():
    from oracle import adjoint
    from sg_inputs import qoi_weights
    b = _b()
    prob, s = _sys(n_e=16, M=4, p=3)
    F = prob.load_block()
    wm, wv = qoi_weights(prob.n_e)
    solver = b.SGSolver(prob, b.Options(inner_precision=64, inner_rtol=1e-12))
    U, st = solver.sg_solve(_dev(F), rtol=1e-12)
    Q, g, st2 = solver.sg_adjoint_grad(U, b.to_device_vec(wm), b.to_device_vec(wv), rtol=1e-12)
    Ud = solve.solve_direct(s, F.T.copy())
    Qo, go, _ = adjoint.adjoint_gradient(s, Ud, wm, wv, lambda R: solve.solve_direct(s, R))
    assert abs(Q - Qo) <= 1e-10 * abs(Qo)
    assert np.max(np.abs(g - go)) <= 1e-8 * np.max(np.abs(go))


@pytest.mark.parametrize("kw,prec", [(dict(n_e=64, M=4, p=2), 64), (dict(n_e=128, M=3, p=3), 32),
                                     (dict(n_e=33, M=5, p=2), 64)])
def test_autotune_keeps_parity(kw, prec):
    """The tuned schedules compute the same operator and solves (to rounding)."""
    b = _b()
    prob, s = _sys(**kw)
    solver = b.SGSolver(prob, b.Options(inner_precision=prec, cheb_degree=8, inner_rtol=1e-4))
    rep = solver.sg_autotune(3)
    assert rep["candidates"] >= 2 and rep["pcg_tile"] in (16, 32) and rep["pcg_ms"] > 0
    assert rep["mv_variant"] in (0, 1, 2, 3, 4)
    U = random_block(prob.P, prob.n, seed=4)
    Y = solver.sg_matvec(_dev(U)).cpu().numpy()
    Yo = sg.matvec(s, U.T.copy()).T
    assert np.linalg.norm(Y - Yo) <= 1e-12 * np.linalg.norm(Yo)
    F = prob.load_block()
    Ux, st = solver.sg_solve(_dev(F), rtol=1e-8, maxit=100)
    assert st["rc"] == 0 and solve.true_relres(s, F.T, Ux.cpu().numpy().T) <= 1.05e-8


@pytest.mark.parametrize("prec", [64, 32])
def test_solve_scale_benchmark_configuration(prec):
    """256^2, M = 10, p = 3, Hermite chaos, in the benchmark's launch configuration
    (Chebyshev degree 16, autotuned schedules): the solve reaches 1e-8, its true
    residual on the oracle's operator agrees, and the solution matches the
    oracle's own solve (FCG with Algorithm 1 and exact LU inner solves, to 1e-10)
    within the a-posteriori bound (||r_gpu|| + ||r_oracle||) ||A^-1||, with
    ||A^-1|| bounded through the coefficient margin (oracle.solve.error_bound_constant)."""
    from gpu_common import oracle_solution
    b = _b()
    print(f"benchmark configuration solve 256^2 inner FP{prec}: oracle reference", flush=True)
    prob, s, F, Uo, ro = oracle_solution("scale")
    print(f"benchmark configuration solve 256^2 inner FP{prec}: GPU solve", flush=True)
    solver = b.SGSolver(prob, b.Options(inner_precision=prec, cheb_degree=16, precond="hsc", inner_rtol=1e-4,
                                        inner_maxit=2000))
    try:
        solver.sg_autotune(3)
        U, st = solver.sg_solve(_dev(F.T), rtol=1e-8, maxit=100)
        assert st["rc"] == 0 and st["true_relres"] <= 1.05e-8
        Ug = U.cpu().numpy().T
    finally:
        solver.close()
    tr = solve.true_relres(s, F, Ug)
    assert tr <= 1.05e-8
    assert abs(st["true_relres"] - tr) <= 1e-3 * tr
    fn = float(np.linalg.norm(F))
    bound = (tr * fn + ro) * solve.error_bound_constant(prob) / float(np.linalg.norm(Uo))
    err = float(np.linalg.norm(Ug - Uo) / np.linalg.norm(Uo))
    print(f"FP{prec} inner: |u - u_oracle| / |u_oracle| = {err:.3e}, bound {bound:.3e}", flush=True)
    assert bound < 1e-6
    assert err <= bound


def test_solve_indefinite_reports_breakdown():
    """A Gaussian coefficient with sigma large enough makes the Galerkin matrix
    indefinite (Section 2's lower bound k_min fails; the coefficient margin is
    negative). With the right-hand side along the eigenvector of the most
    negative eigenvalue (dense spectrum of the oracle's assembled matrix), the
    first curvature p^T A p = lambda_min |f|^2 < 0: the solve stops with
    SG_BREAKDOWN and returns the last finite iterate, the zero start."""
    b = _b()
    prob, s = _sys(n_e=4, M=1, p=3, sigma=2.0)
    assert prob.coefficient_margin() < 0
    A = sg.assemble(s).toarray()
    w, V = np.linalg.eigh(A)
    assert w[0] < -1.0
    F = sg.unvec(V[:, 0], s.n).T.copy()  # (P, n)
    print("indefinite system: breakdown", flush=True)
    solver = b.SGSolver(prob, b.Options(precond="none"))
    try:
        U, st = solver.sg_solve(_dev(F), rtol=1e-8, maxit=10)
    finally:
        solver.close()
    assert st["rc"] == b.SG_BREAKDOWN and st["status"] == b.SG_BREAKDOWN
    assert st["outer_it"] == 0
    assert float(U.abs().max()) == 0.0
