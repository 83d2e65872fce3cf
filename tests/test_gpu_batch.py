"""Multi-problem batch (ragged inner launches, device-side outer CG scalars,
graph replay) through the C-ABI: against single-problem solves of the same
library, against the oracle's direct solve, and graph against eager."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import sg, solve  # noqa: E402
from sg_inputs import batch_problems, make_problem  # noqa: E402


def _b():
    from paper_1205_1864_amd import binding
    return binding


# grids that take every SG-operator path (generic tiles, y-marching kernel at
# multiples of 64), chaos degrees 0..3, both chaos families, one zero right-hand side
MIXED = [dict(n_e=16, M=4, p=2, sigma=0.2, L=0.5), dict(n_e=64, M=3, p=3, sigma=0.25, L=0.3),
         dict(n_e=21, M=2, p=1, sigma=0.2, L=0.6), dict(n_e=32, M=5, p=2, sigma=0.15, L=0.4),
         dict(n_e=12, M=3, p=0, sigma=0.2, L=0.5), dict(n_e=128, M=2, p=2, sigma=0.2, L=0.8),
         dict(n_e=24, M=3, p=3, sigma=0.2, L=0.5),
         dict(n_e=20, M=3, p=3, sigma=0.4, L=0.5, family="legendre")]
ZERO_RHS = 4


def _problems():
    return [make_problem(f"b{i}", **kw) for i, kw in enumerate(MIXED)]


def _rhs(probs):
    b = _b()
    F = []
    for i, pr in enumerate(probs):
        f = pr.load_block()
        if i == ZERO_RHS:
            f = np.zeros_like(f)
        F.append(b.to_device_block(f))
    return F


@pytest.mark.parametrize("prec,pc,warm,tile", [(64, "hsc", False, 0), (32, "hsc", False, 0), (64, "mean", False, 0),
                                               (64, "bgs", False, 0), (32, "bgs", False, 0), (64, "hsc", True, 0),
                                               (32, "hsc", True, 0), (64, "bgs", True, 0), (64, "hsc", False, 16),
                                               (32, "bgs", False, 16)])
def test_batch_matches_single_solves(prec, pc, warm, tile):
    b = _b()
    probs = _problems()
    print(f"batch vs single prec={prec} pc={pc} warm={warm} tile={tile}", flush=True)
    opts = b.Options(inner_precision=prec, precond=pc, inner_rtol=1e-4, warm_start=warm, tile=tile)
    batch = b.SGBatch(probs, opts)
    F = _rhs(probs)
    U, stats, info = batch.sg_batch_solve(F, rtol=1e-8, maxit=100, use_graph=True)
    assert info["rc"] == 0
    for i, pr in enumerate(probs):
        st = stats[i]
        if i == ZERO_RHS:
            assert st["status"] == 0 and st["outer_it"] == 0 and float(U[i].abs().max()) == 0.0
            continue
        single = b.SGSolver(pr, opts)
        Us, ss = single.sg_solve(F[i], rtol=1e-8, maxit=100)
        assert st["status"] == 0 and ss["rc"] == 0
        assert st["true_relres"] <= 1.05e-8
        assert abs(st["outer_it"] - ss["outer_it"]) <= (0 if prec == 64 else 1)
        d = float((U[i] - Us).norm() / Us.norm())
        # same arithmetic per column; only the order of the outer FP64 reductions differs
        assert d <= (1e-11 if prec == 64 else 1e-7), (i, d)
        if pc == "hsc":
            P = pr.P
            assert st["n_blocksolve"] == st["outer_it"] * (2 * (P - 1) + 1)
            assert st["n_blockmv"] == ss["n_blockmv"] // max(1, ss["outer_it"]) * st["outer_it"]
        if pc == "bgs":
            assert st["n_blocksolve"] == ss["n_blocksolve"] // max(1, ss["outer_it"]) * st["outer_it"]
            assert st["n_blockmv"] == ss["n_blockmv"] // max(1, ss["outer_it"]) * st["outer_it"]
        assert st["inner_it_total"] > 0


def test_batch_against_oracle_direct_solve():
    b = _b()
    kws = [dict(n_e=16, M=4, p=2, sigma=0.2, L=0.5), dict(n_e=12, M=3, p=3, sigma=0.25, L=0.3),
           dict(n_e=9, M=2, p=1, sigma=0.2, L=0.6)]
    probs = [make_problem(f"o{i}", **kw) for i, kw in enumerate(kws)]
    batch = b.SGBatch(probs, b.Options(inner_precision=32, inner_rtol=1e-4))
    F = [b.to_device_block(pr.load_block()) for pr in probs]
    U, stats, info = batch.sg_batch_solve(F, rtol=1e-8, maxit=100)
    assert info["rc"] == 0
    for pr, u, st in zip(probs, U, stats):
        s = sg.build_system(pr)
        Fh = pr.load_block()
        Ud = solve.solve_direct(s, Fh.T.copy())
        ev = np.linalg.eigvalsh(sg.assemble(s).toarray())
        tr = solve.true_relres(s, Fh.T, u.cpu().numpy().T)
        assert tr <= 1.05e-8 and abs(st["true_relres"] - tr) <= 1e-3 * tr
        err = np.linalg.norm(u.cpu().numpy().T - Ud) / np.linalg.norm(Ud)
        assert err <= ev.max() / ev.min() * 1.05e-8


@pytest.mark.parametrize("prec,pc", [(32, "hsc"), (64, "hsc"), (64, "mean"), (32, "bgs")])
def test_batch_autotune_keeps_parity(prec, pc):
    """The tuned batch schedules (every member's SG operator; tile kind, band
    height and block cap of the ragged inner launches) solve the same systems:
    every member reaches 1e-8 on the oracle's operator and matches the oracle's
    direct solve within its condition number times 1.05e-8."""
    b = _b()
    kws = [dict(n_e=16, M=4, p=2, sigma=0.2, L=0.5), dict(n_e=12, M=3, p=3, sigma=0.25, L=0.3),
           dict(n_e=9, M=2, p=1, sigma=0.2, L=0.6), dict(n_e=33, M=3, p=2, sigma=0.2, L=0.4)]
    probs = [make_problem(f"t{i}", **kw) for i, kw in enumerate(kws)]
    print(f"batch autotune prec={prec} pc={pc}", flush=True)
    batch = b.SGBatch(probs, b.Options(inner_precision=prec, precond=pc, inner_rtol=1e-4))
    rep = batch.sg_batch_autotune(3)
    assert rep["candidates"] >= 2 + len(probs) and rep["pcg_ms"] > 0 and rep["mv_ms"] > 0
    assert rep["pcg_tile"] in (16, 32) and rep["pcg_rows"] in (16, 64, 128, 256)
    assert rep["mv_variant"] in (0, 1, 2, 3, 4)
    F = [b.to_device_block(pr.load_block()) for pr in probs]
    for use_graph in (True, False):
        U, stats, info = batch.sg_batch_solve(F, rtol=1e-8, maxit=100, use_graph=use_graph)
        assert info["rc"] == 0
        for pr, u, st in zip(probs, U, stats):
            s = sg.build_system(pr)
            Fh = pr.load_block()
            tr = solve.true_relres(s, Fh.T, u.cpu().numpy().T)
            assert tr <= 1.05e-8 and abs(st["true_relres"] - tr) <= 1e-3 * tr
            Ud = solve.solve_direct(s, Fh.T.copy())
            ev = np.linalg.eigvalsh(sg.assemble(s).toarray())
            err = np.linalg.norm(u.cpu().numpy().T - Ud) / np.linalg.norm(Ud)
            assert err <= ev.max() / ev.min() * 1.05e-8
    batch.close()


def test_batch_graph_replay_equals_eager():
    """The captured outer iteration replays exactly the eager launches: bitwise equal results."""
    b = _b()
    probs = _problems()
    batch = b.SGBatch(probs, b.Options(inner_precision=32, inner_rtol=1e-4))
    F = _rhs(probs)
    Ug, sg_, _ = batch.sg_batch_solve(F, rtol=1e-8, maxit=100, use_graph=True)
    Ue, se, _ = batch.sg_batch_solve(F, rtol=1e-8, maxit=100, use_graph=False)
    Ug2, _, _ = batch.sg_batch_solve(F, rtol=1e-8, maxit=100, use_graph=True)  # replays the existing graph
    for a, c, a2, x, y in zip(Ug, Ue, Ug2, sg_, se):
        assert bool((a == c).all()) and bool((a2 == c).all())
        assert x["outer_it"] == y["outer_it"] and x["inner_it_total"] == y["inner_it_total"]


def test_batch_seeded_uneven_set_converges():
    """A seeded uneven batch (the multi-problem recipe at reduced sizes) converges per problem."""
    b = _b()
    probs = batch_problems(seed=3, count=10, grids=(16, 32, 64), max_P=120)
    batch = b.SGBatch(probs, b.Options(inner_precision=32, inner_rtol=1e-4))
    F = [b.to_device_block(pr.load_block()) for pr in probs]
    U, stats, info = batch.sg_batch_solve(F, rtol=1e-8, maxit=100)
    assert info["rc"] == 0
    for st in stats:
        assert st["status"] == 0 and st["true_relres"] <= 1.05e-8 and 1 <= st["outer_it"] <= 30


def test_batch_not_converged_and_rejection():
    b = _b()
    probs = _problems()[:3]
    batch = b.SGBatch(probs, b.Options(inner_precision=64))
    F = _rhs(probs)
    U, stats, info = batch.sg_batch_solve(F, rtol=1e-12, maxit=1)
    assert info["rc"] == b.SG_NOT_CONVERGED
    assert all(st["outer_it"] == 1 and st["status"] == b.SG_NOT_CONVERGED for st in stats)
    with pytest.raises(b.SGError):
        b.SGBatch(probs, b.Options(precond="none"))


@pytest.mark.timeout(900)
def test_batch_full_recipe_members_against_oracle():
    """The 48-problem uneven recipe (grids 32^2..256^2, P <= 495, FP32 inner / FP64 outer)
    in one batch, in the benchmark's configuration (Chebyshev degree 16): every
    member converges; the true residual of every member, recomputed with the
    oracle's own operator, meets the stopping test; and the members small enough
    for a direct solve agree with the oracle within the bound of the stopping test."""
    b = _b()
    probs = batch_problems(seed=0, count=48)
    batch = b.SGBatch(probs, b.Options(inner_precision=32, cheb_degree=16, inner_rtol=1e-4, inner_maxit=2000))
    F = [b.to_device_block(pr.load_block()) for pr in probs]
    U, stats, info = batch.sg_batch_solve(F, rtol=1e-8, maxit=100)
    batch.close()
    assert info["rc"] == 0
    assert all(st["status"] == 0 and st["true_relres"] <= 1.05e-8 for st in stats)
    for i, pr in enumerate(probs):
        print(f"batch member {i}: n_e={pr.n_e} M={pr.M} p={pr.p} oracle residual", flush=True)
        s = sg.build_system(pr)
        tr = solve.true_relres(s, pr.load_block().T, U[i].cpu().numpy().T)
        assert tr <= 1.05e-8, (i, tr)
        assert abs(tr - stats[i]["true_relres"]) <= 1e-3 * tr, (i, tr, stats[i]["true_relres"])
    small = sorted(range(len(probs)), key=lambda i: probs[i].n * probs[i].P)[:4]
    for i in small:
        pr = probs[i]
        s = sg.build_system(pr)
        Fh = pr.load_block()
        Ud = solve.solve_direct(s, Fh.T.copy())
        err = np.linalg.norm(U[i].cpu().numpy().T - Ud) / np.linalg.norm(Ud)
        # ||u - u*|| / ||u*|| <= kappa(A) ||r|| / ||f||; kappa(A) <= 4 for these coefficient margins
        assert err <= 4.0 * 1.05e-8, (i, err)
