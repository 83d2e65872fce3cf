"""Benchmark of the SG solver hot path on one MI355X.

Workload (timed step): the hierarchical-Schur-preconditioned flexible CG solve
of the 256^2 Q1 problem with M = 10 KL terms and Hermite degree p = 3
(P = 286, 18.6M unknowns) to relative residual 1e-8, FP64 inner PCG with a
degree-16 Jacobi-Chebyshev preconditioner stopped at 1e-4. Inputs are seeded
and synthetic and resident in HBM before timing starts.

Also reported (outside the timed steps): the SG matvec bandwidth (cold and
warm Infinity Cache), the FP32-inner, mean-preconditioned and block symmetric
Gauss-Seidel-preconditioned solves, the solve through the a-priori Schur
reduction of the top degree, the same solve with Legendre chaos, the
adjoint gradient of the 512^2 differentiation case, the 48-problem uneven
batch (FP32 inner / FP64 outer, graph replay) against the same problems
solved one after another, the roofline of the dominant kernel, and the CPU
oracle's own solve of the timed workload on the host (flexible CG with the
hierarchical Schur preconditioner and exact sparse-LU inner solves, to 1e-10),
which is both the CPU baseline and the reference every GPU solution is
compared with.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "SG solve s to relres 1e-8 + matvec HBM GB/s (256², M=10, p=3); adjoint grad s"
HBM_PEAK_GBS = 8000.0
CHEB_DEGREE = 16  # updates of the Chebyshev preconditioner of the inner PCG (fastest measured; 8 as an extra)
# HBM bytes per launch measured with separate FETCH_SIZE and WRITE_SIZE counter
# runs of this benchmark, scaled by the same counters of a 512 MiB elementwise
# kernel (profiles/hbm_traffic_solve_256sq_M10_p3.txt). Emptied when the
# kernel changes.
# pcg_kernel<double, BandTile<double, 128 | 64, 15, 16>, 1>, average over a solve's launches, by the
# inner schedule's block cap (-1: whole columns per block where they fill the device; 0: automatic grid)
PCG_TRAFFIC_BYTES = {-1: 14.30e9}
# one SG matvec, by schedule (mv_variant, mv_param): the row-staged kernel with 10-row pieces,
# and the y-marching kernel it replaced
MATVEC_TRAFFIC_BYTES = {(4, 10): 354.2e6, (2, 2): 570.4e6, (2, 1): 543.0e6}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _ensure_built():
    """Build the library if it is missing, or if its recorded source hash says it
    was built from other sources (a library without a recorded hash is used as is)."""
    from paper_1205_1864_amd.build import LIB, SRCHASH, build, built_from_current_sources
    if not os.path.exists(LIB):
        log("library missing: building")
        build()
    elif os.path.exists(SRCHASH) and not built_from_current_sources():
        log("library built from other sources: rebuilding")
        build()


def time_matvec(solver, U, Y, reps, cold, flush=None):
    import torch
    stream = solver.stream
    times = []
    for _ in range(reps):
        if cold:
            flush.add_(1.0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        solver.sg_matvec(U, Y)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times)), times


def bench_batch(degree, count=48, seed=0):
    """The uneven batch solved together (graph replay; default, then autotuned
    schedules) and one problem after another (default schedules)."""
    import torch
    from paper_1205_1864_amd.binding import Options, SGBatch, SGSolver, to_device_block
    from sg_inputs import batch_problems
    probs = batch_problems(seed=seed, count=count)
    opts = Options(inner_precision=32, cheb_degree=degree, precond="hsc", inner_maxit=2000)
    log(f"batch: {count} problems, {sum(p.n * p.P for p in probs) / 1e6:.1f}M unknowns")
    batch = SGBatch(probs, opts)
    F = [to_device_block(p.load_block()) for p in probs]
    U = batch.empty()

    def timed():
        batch.sg_batch_solve(F, U, rtol=1e-8, maxit=100)  # warm-up; captures the graph
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st, info = batch.sg_batch_solve(F, U, rtol=1e-8, maxit=100)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, st, info

    t_default, _, _ = timed()
    log(f"batch, default schedules: {t_default:.3f} s ({count / t_default:.2f} solves/s)")
    tune = batch.sg_batch_autotune(3)
    log(f"batch autotuned: {tune}")
    t_batch, st, info = timed()
    log(f"batch: {t_batch:.3f} s ({count / t_batch:.2f} solves/s), rc {info['rc']}")
    batch.close()
    del batch
    torch.cuda.empty_cache()
    # the same problems one after another (setup not timed)
    t_seq, diffs, seq_outer = 0.0, [], []
    for i, pr in enumerate(probs):
        sv = SGSolver(pr, opts)
        Us = sv.empty()
        if i == 0:
            sv.sg_solve(F[i], Us, rtol=1e-8, maxit=100)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, ss = sv.sg_solve(F[i], Us, rtol=1e-8, maxit=100)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t1
        diffs.append(float(torch.linalg.norm(U[i] - Us) / torch.linalg.norm(Us)))
        seq_outer.append(ss["outer_it"])
        sv.close()
        del sv, Us
    log(f"sequential: {t_seq:.3f} s ({count / t_seq:.2f} solves/s)")
    return {
        "batch_count": count, "batch_unknowns": int(sum(p.n * p.P for p in probs)),
        "batch_s": t_batch, "batch_solves_per_s": count / t_batch, "batch_default_schedule_s": t_default,
        "batch_schedule": tune,
        "batch_sequential_s": t_seq, "batch_sequential_solves_per_s": count / t_seq,
        "batch_speedup_vs_sequential": t_seq / t_batch, "batch_rc": info["rc"],
        "batch_outer_it": [s["outer_it"] for s in st], "batch_sequential_outer_it": seq_outer,
        "batch_max_true_relres": max(s["true_relres"] for s in st),
        "batch_max_rel_diff_vs_sequential": max(diffs),
    }


def oracle_reference(prob, rtol=1e-10):
    """The oracle's own solve of the timed workload on the host cores.

    Flexible CG preconditioned by Algorithm 1 with exact sparse-LU solves of
    the K_0 blocks (the oracle as it stands), run to relres ``rtol``. Returns
    the solution (n x P), the time from the start of the iteration until the
    recursive residual first reached 1e-8 (the GPU metric), the setup times and
    the a-posteriori constant of the error bound (oracle.solve.error_bound_constant).
    """
    from oracle import hsc, krylov, sg
    from oracle.sg import matvec
    t0 = time.perf_counter()
    c0 = time.process_time()
    s = sg.build_system(prob)
    t_build = time.perf_counter() - t0
    F = prob.load_block().T.copy()
    t1 = time.perf_counter()
    ex = hsc.ExactMeanSolver(s)
    t_lu = time.perf_counter() - t1
    t2 = time.perf_counter()
    res = krylov.fcg(lambda U: matvec(s, U), lambda R: hsc.hsc_apply(s, R, ex), F, rtol, 200)
    t_solve = time.perf_counter() - t2
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    hit = [i for i, r in enumerate(res.history) if r <= 1e-8]
    t_1e8 = res.history_time[hit[0]] - t2 if hit else float("nan")
    r_true = F - matvec(s, res.x)
    return {
        "U": res.x, "fnorm": float(np.linalg.norm(F)), "unorm": float(np.linalg.norm(res.x)),
        "rnorm_true": float(np.linalg.norm(r_true)), "outer_it": res.iterations,
        "outer_it_1e8": hit[0] if hit else None, "history": res.history,
        "t_1e8": t_1e8, "t_solve": t_solve, "t_build": t_build, "t_lu": t_lu,
        "cores": len(os.sched_getaffinity(0)), "effective_cores": round(cpu / wall, 2),
    }


def compare_with_oracle(U_dev, true_relres, ref, Uo_dev, cbound):
    """Relative difference of a GPU solution from the oracle's, and its rigorous bound
    (||r_gpu|| + ||r_oracle||) c / ||u_oracle||."""
    import torch
    err = float(torch.linalg.norm(U_dev - Uo_dev) / ref["unorm"])
    bound = (true_relres * ref["fnorm"] + ref["rnorm_true"]) * cbound / ref["unorm"]
    return err, bound


def cpu_baseline_entry(ref):
    return {
        "value": ref["t_1e8"], "unit": "s",
        "cores": ref["cores"], "effective_cores": ref["effective_cores"],
        "kind": "oracle",
        "sample": (f"the oracle's whole solve of the timed workload (256^2, M=10, p=3): flexible CG with "
                   f"Algorithm 1 and exact sparse-LU K_0 solves; value = time of the iteration until its "
                   f"recursive residual first reached 1e-8 ({ref['outer_it_1e8']} iterations); the run "
                   f"continued to 1e-10 ({ref['outer_it']} iterations, {ref['t_solve']:.1f} s) to serve as "
                   f"the parity reference; not included: assembly {ref['t_build']:.1f} s, LU factorisation "
                   f"{ref['t_lu']:.1f} s"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="only the timed solve and the matvec")
    ap.add_argument("--pcg-blocks", type=int, default=None,
                    help="fix the inner PCG schedule instead of autotuning it (0: automatic grid, -1: whole "
                         "columns per block); for counter runs of one schedule")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    _ensure_built()
    from paper_1205_1864_amd.binding import Options, SGSolver, to_device_block, to_device_vec
    from sg_inputs import named_problem, qoi_weights, random_block

    torch.cuda.set_device(0)
    prob = named_problem("scale")
    F = to_device_block(prob.load_block())
    ref = Uo = cbound = None
    if not args.no_cpu:
        from oracle.solve import error_bound_constant
        cbound = error_bound_constant(prob)
        # the oracle first: its solution is the reference of every GPU solve below
        log("cpu oracle: FCG-HSC with exact LU inner solves to 1e-10")
        ref = oracle_reference(prob)
        log(f"cpu oracle: {ref['t_1e8']:.1f} s to 1e-8, {ref['t_solve']:.1f} s to 1e-10, "
            f"history {['%.1e' % h for h in ref['history']]}")
        Uo = to_device_block(ref.pop("U").T)

    def vs_oracle(key, U_dev, true_relres, into):
        if Uo is None:
            return
        err, bound = compare_with_oracle(U_dev, true_relres, ref, Uo, cbound)
        into[f"rel_err_vs_oracle_{key}"] = err
        into[f"rel_err_bound_{key}"] = bound
        log(f"{key}: |u - u_oracle| / |u_oracle| = {err:.2e} (bound {bound:.2e})")
    opts64 = Options(inner_precision=64, cheb_degree=CHEB_DEGREE, inner_maxit=2000, precond="hsc", inner_rtol=1e-4)
    if args.pcg_blocks is not None:  # the handle's default inner schedule, read at set-up
        os.environ["SGPC_PCG_MAX_BLOCKS"] = str(args.pcg_blocks)
    solver = SGSolver(prob, opts64)
    # not timed: picks the launch schedules for this problem (only the SG operator's when the
    # inner schedule is fixed)
    schedule = solver.sg_autotune(1 if args.pcg_blocks is not None else 3)
    log(f"autotune: {schedule}")
    U = solver.empty()

    # ---- timed steps: the HSC-FCG solve
    for _ in range(args.warmup):
        _, wst = solver.sg_solve(F, U, rtol=1e-8, maxit=100)
        log(f"warm-up solve: {wst['ms']:.1f} ms, outer {wst['outer_it']}, inner {wst['inner_it_total']}")
    torch.cuda.synchronize()
    ms_inner = bytes_inner = 0.0
    launches = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st = solver.sg_solve(F, U, rtol=1e-8, maxit=100)
        ms_inner += st["ms_inner"]
        bytes_inner += st["inner_bytes"]
        launches += st["inner_launches"]
        log(f"timed solve: {st['ms']:.1f} ms, outer {st['outer_it']}, relres {st['true_relres']:.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    solve_s = elapsed / max(1, args.steps)
    U64 = U.clone()

    # ---- SG matvec bandwidth
    alg_bytes_mv = 2.0 * prob.n * prob.P * 8 + prob.M * prob.n_e ** 2 * 8
    Ur = to_device_block(random_block(prob.P, prob.n, seed=0))
    Yr = solver.empty()
    time_matvec(solver, Ur, Yr, 5, cold=False)
    warm_ms, _ = time_matvec(solver, Ur, Yr, 50, cold=False)
    flush = torch.zeros(512 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
    cold_ms, _ = time_matvec(solver, Ur, Yr, 50, cold=True, flush=flush)
    del flush
    log(f"matvec cold {cold_ms:.3f} ms warm {warm_ms:.3f} ms")
    mv_cold = alg_bytes_mv / (cold_ms * 1e-3) / 1e9
    mv_warm = alg_bytes_mv / (warm_ms * 1e-3) / 1e9

    extra = {
        "outer_it": st["outer_it"], "true_relres": st["true_relres"], "kappa_est": st["kappa_est"],
        "inner_it_total": st["inner_it_total"], "inner_it_max_per_level": st["inner_it_max"][: prob.p + 1],
        "n_blockmv": st["n_blockmv"], "n_blocksolve": st["n_blocksolve"],
        "ms_precond": st["ms_precond"], "ms_matvec_in_solve": st["ms_matvec"],
        "matvec_ms_cold": cold_ms, "matvec_ms_warm": warm_ms,
        "matvec_GBs_cold": mv_cold, "matvec_GBs_warm": mv_warm,
        "matvec_frac_cold": mv_cold / HBM_PEAK_GBS, "matvec_alg_bytes": alg_bytes_mv,
        "error_bound_constant": cbound,
    }
    vs_oracle("hsc_fp64", U64, st["true_relres"], extra)

    def run_extras():
        # FP32 inner (precision variant) and mean-based comparators
        for label, o in [("hsc_fp32", Options(inner_precision=32, cheb_degree=CHEB_DEGREE, precond="hsc", inner_maxit=2000)),
                         ("mean_fp64", Options(inner_precision=64, cheb_degree=CHEB_DEGREE, precond="mean", inner_maxit=2000)),
                         ("mean_fp32", Options(inner_precision=32, cheb_degree=CHEB_DEGREE, precond="mean", inner_maxit=2000)),
                         ("bgs_fp64", Options(inner_precision=64, cheb_degree=CHEB_DEGREE, precond="bgs", inner_maxit=2000)),
                         # up-sweep (backward-sweep) inner solves started from the down-sweep values
                         ("hsc_fp64_warm", Options(inner_precision=64, cheb_degree=CHEB_DEGREE, precond="hsc",
                                                   inner_maxit=2000, warm_start=True)),
                         ("bgs_fp64_warm", Options(inner_precision=64, cheb_degree=CHEB_DEGREE, precond="bgs",
                                                   inner_maxit=2000, warm_start=True)),
                         # the same solves with a degree-8 Chebyshev preconditioner
                         ("hsc_fp64_d8", Options(inner_precision=64, cheb_degree=8, precond="hsc", inner_maxit=2000)),
                         ("hsc_fp32_d8", Options(inner_precision=32, cheb_degree=8, precond="hsc", inner_maxit=2000)),
                         # the preconditioner action captured once and replayed from a HIP graph
                         ("hsc_fp64_graph", Options(inner_precision=64, cheb_degree=CHEB_DEGREE, precond="hsc",
                                                    inner_maxit=2000, use_graph=True)),
                         ("hsc_fp32_graph", Options(inner_precision=32, cheb_degree=CHEB_DEGREE, precond="hsc",
                                                    inner_maxit=2000, use_graph=True))]:
            sv = SGSolver(prob, o)
            sv.sg_autotune(3)
            Uv = sv.empty()
            sv.sg_solve(F, Uv, rtol=1e-8, maxit=200)  # warm-up (and the capture of a graph)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, sv_st = sv.sg_solve(F, Uv, rtol=1e-8, maxit=200)
            torch.cuda.synchronize()
            extra[f"solve_s_{label}"] = time.perf_counter() - t1
            log(f"{label}: {extra[f'solve_s_{label}']:.3f} s, outer {sv_st['outer_it']}")
            extra[f"outer_it_{label}"] = sv_st["outer_it"]
            extra[f"inner_it_total_{label}"] = sv_st["inner_it_total"]
            extra[f"n_blocksolve_{label}"] = sv_st["n_blocksolve"]
            extra[f"true_relres_{label}"] = sv_st["true_relres"]
            extra[f"rel_diff_vs_fp64_hsc_{label}"] = float(torch.linalg.norm(Uv - U64) / torch.linalg.norm(U64))
            vs_oracle(label, Uv, sv_st["true_relres"], extra)
            # algorithmic inner-PCG bandwidth of this variant (library byte count over its HIP-event
            # time; a replayed graph is timed per action, so it has no per-launch figure)
            if sv_st["ms_inner"] > 0 and not o.use_graph:
                gbs = sv_st["inner_bytes"] / (sv_st["ms_inner"] * 1e-3) / 1e9
                extra[f"pcg_GBs_{label}"] = gbs
                extra[f"pcg_frac_{label}"] = gbs / HBM_PEAK_GBS
            if label == "hsc_fp32":
                # FP32-inner error of one preconditioner action against the FP64 one
                Rr = to_device_block(random_block(prob.P, prob.n, seed=5))
                z32 = sv.sg_apply_hsc(Rr)
                z64 = solver.sg_apply_hsc(Rr)
                extra["hsc_action_rel_err_fp32"] = float(torch.linalg.norm(z32 - z64) / torch.linalg.norm(z64))
            sv.close()
            del sv, Uv
            torch.cuda.empty_cache()

        # a-priori reduction to the Schur complement of the top degree (Section 5):
        # the same problem, top-degree solves of the reduced operator to 1e-11
        sr = SGSolver(prob, Options(inner_precision=64, cheb_degree=CHEB_DEGREE, precond="hsc", inner_maxit=3000))
        sr.sg_autotune(3)
        Ur = sr.empty()
        sr.sg_solve_reduced(F, Ur, rtol=1e-8, maxit=200, op_rtol=1e-11)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, rst = sr.sg_solve_reduced(F, Ur, rtol=1e-8, maxit=200, op_rtol=1e-11)
        torch.cuda.synchronize()
        extra["solve_s_hsc_reduced"] = time.perf_counter() - t1
        extra["outer_it_hsc_reduced"] = rst["outer_it"]
        extra["true_relres_hsc_reduced"] = rst["true_relres"]
        extra["rel_diff_vs_fp64_hsc_hsc_reduced"] = float(torch.linalg.norm(Ur - U64) / torch.linalg.norm(U64))
        vs_oracle("hsc_reduced", Ur, rst["true_relres"], extra)
        log(f"hsc reduced: {extra['solve_s_hsc_reduced']:.3f} s, outer {rst['outer_it']}")
        sr.close()
        del sr, Ur
        torch.cuda.empty_cache()

        # Legendre chaos (uniform variables on [-1, 1]) on the same grid and KL data
        pl = named_problem("scale_legendre")
        sl = SGSolver(pl, Options(inner_precision=64, cheb_degree=CHEB_DEGREE, precond="hsc", inner_maxit=2000))
        sl.sg_autotune(3)
        Fl = to_device_block(pl.load_block())
        Ul = sl.empty()
        sl.sg_solve(Fl, Ul, rtol=1e-8, maxit=200)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, lst = sl.sg_solve(Fl, Ul, rtol=1e-8, maxit=200)
        torch.cuda.synchronize()
        extra["solve_s_hsc_legendre"] = time.perf_counter() - t1
        extra["outer_it_hsc_legendre"] = lst["outer_it"]
        extra["kappa_est_hsc_legendre"] = lst["kappa_est"]
        extra["true_relres_hsc_legendre"] = lst["true_relres"]
        log(f"hsc legendre: {extra['solve_s_hsc_legendre']:.3f} s, outer {lst['outer_it']}")
        sl.close()
        del sl, Ul, Fl
        torch.cuda.empty_cache()

        # adjoint gradient, 512^2, M = 8, p = 3
        pg = named_problem("grad")
        sg_ = SGSolver(pg, Options(inner_precision=64, cheb_degree=CHEB_DEGREE, precond="hsc", inner_maxit=2000))
        sg_.sg_autotune(3)
        Fg = to_device_block(pg.load_block())
        wm, wv = qoi_weights(pg.n_e)
        wm_d, wv_d = to_device_vec(wm), to_device_vec(wv)
        Ug = sg_.empty()
        sg_.sg_solve(Fg, Ug, rtol=1e-8, maxit=100)  # warm-up
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        _, fst = sg_.sg_solve(Fg, Ug, rtol=1e-8, maxit=100)
        Q, grad, ast = sg_.sg_adjoint_grad(Ug, wm_d, wv_d, rtol=1e-8, maxit=100)
        torch.cuda.synchronize()
        extra["adjoint_grad_s"] = time.perf_counter() - t2
        log(f"adjoint 512^2: {extra['adjoint_grad_s']:.3f} s")
        extra["adjoint_outer_it"] = [fst["outer_it"], ast["outer_it"]]
        extra["adjoint_Q"] = Q
        extra["adjoint_grad"] = [float(g) for g in grad]
        sg_.close()
        del sg_, Ug, Fg
        torch.cuda.empty_cache()

        # multi-problem batch: 48 seeded uneven problems, FP32 inner / FP64 outer
        extra.update(bench_batch(CHEB_DEGREE))
        torch.cuda.empty_cache()

        # lognormal-coefficient operator (Section 6, Tables 6-9): the paper's finest
        # mesh of Table 9 (h = 1/30, N = 4, degree 4) and a 256^2 grid at degree 2
        from paper_1205_1864_amd.binding import LognormalOperator
        for label, kw in (("logn_30sq_N4_p4", dict(n_e=30, M=4, p=4)), ("logn_256sq_N4_p2", dict(n_e=256, M=4, p=2))):
            pr = named_problem("small", L=0.5, **kw)
            op = LognormalOperator(pr, 1.0, 1.0)
            Ul = to_device_block(random_block(op.P, op.n, seed=1))
            Yl = torch.empty_like(Ul)
            stream = torch.cuda.current_stream()
            for _ in range(3):
                op.matvec(Ul, Yl)
            ts = []
            for _ in range(20):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                op.matvec(Ul, Yl)
                e1.record(stream)
                e1.synchronize()
                ts.append(e0.elapsed_time(e1))
            ms = float(np.median(ts))
            # algorithmic bytes: U and Y once, every stored block field once
            nbytes = 2.0 * op.n * op.P * 8 + op.nblocks * pr.n_e * pr.n_e * 8.0
            extra[f"{label}_matvec_ms"] = ms
            extra[f"{label}_blocks"] = op.nblocks
            extra[f"{label}_GBs"] = nbytes / (ms * 1e-3) / 1e9
            extra[f"{label}_frac"] = extra[f"{label}_GBs"] / HBM_PEAK_GBS
            log(f"{label}: {ms:.3f} ms, {op.nblocks} blocks, {extra[f'{label}_GBs']:.0f} GB/s")
            op.close()
            del op, Ul, Yl
            torch.cuda.empty_cache()
        # the lognormal solve of Tables 6-9 (10 x 10 mesh, N = 4, degree 4, CoV 100 %;
        # the paper prints 16 M_HS iterations and kappa 4.17) and a 64^2 grid
        for label, kw in (("logn_solve_10sq_N4_p4", dict(n_e=10, M=4, p=4)),
                          ("logn_solve_64sq_N4_p3", dict(n_e=64, M=4, p=3))):
            pr = named_problem("small", L=0.5, **kw)
            op = LognormalOperator(pr, 1.0, 1.0)
            Fl = to_device_block(pr.load_block())
            Ul, _ = op.solve(Fl, rtol=1e-8, precond="hsc")  # warm-up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            Ul, lst = op.solve(Fl, Ul, rtol=1e-8)
            torch.cuda.synchronize()
            extra[f"{label}_s"] = time.perf_counter() - t1
            extra[f"{label}_outer_it"] = lst["outer_it"]
            extra[f"{label}_inner_it"] = lst["inner_it"]
            extra[f"{label}_kappa_est"] = lst["kappa_est"]
            extra[f"{label}_relres"] = lst["relres"]
            log(f"{label}: {extra[f'{label}_s']:.3f} s, outer {lst['outer_it']}, kappa {lst['kappa_est']:.4f}")
            op.close()
            del op, Ul, Fl
            torch.cuda.empty_cache()
        torch.cuda.empty_cache()


    if not args.no_extra:
        try:
            run_extras()
        except Exception as exc:  # an extra never costs the headline line
            import traceback
            traceback.print_exc()
            extra["extras_error"] = repr(exc)
    achieved = bytes_inner / (ms_inner * 1e-3) / 1e9 if ms_inner > 0 else 0.0
    # the counter traffic belongs to the schedules it was measured with
    pcg_traffic = PCG_TRAFFIC_BYTES.get(schedule["pcg_max_blocks"]) if schedule["pcg_tile"] == 32 else None
    mv_traffic = MATVEC_TRAFFIC_BYTES.get((schedule["mv_variant"], schedule["mv_param"]))
    mv_kernel = {4: "sgop_stage_kernel", 3: "sgop_piece_kernel<double>", 2: "sgop_march_kernel<double>",
                 1: "sgop_strip_dyn_kernel<double>", 0: "sgop_strip_kernel<double>"}.get(
                     schedule["mv_variant"], f"SG operator variant {schedule['mv_variant']}")
    roofline = {
        "kernel": "pcg_kernel (persistent batched inner PCG, all launches of the timed solves)",
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS, "traffic": pcg_traffic, "traffic_unit": "bytes per launch",
        "avg_launch_ms": ms_inner / max(1, launches), "launches": launches,
        "alg_bytes_per_launch": bytes_inner / max(1, launches),
    }
    roofline_mv = {
        "kernel": f"{mv_kernel} (SG matvec)", "bound": "hbm", "achieved": mv_cold, "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": mv_cold / HBM_PEAK_GBS, "traffic": mv_traffic,
        "traffic_unit": "bytes per launch", "avg_launch_ms": cold_ms,
        "alg_bytes_per_launch": alg_bytes_mv,
    }
    out = {
        "metric": METRIC, "value": solve_s, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": solve_s * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "HSC-FCG solve, 256^2 Q1, M=10, p=3 (P=286, 18.6M unknowns), "
                               f"FP64 inner PCG Jacobi-Chebyshev d={CHEB_DEGREE} to 1e-4, outer to 1e-8",
                   "cheb_degree": CHEB_DEGREE, "schedule": schedule, "n_e": prob.n_e, "M": prob.M, "p": prob.p, "P": prob.P, "sigma": prob.sigma, "L": prob.L},
        "roofline": roofline, "roofline_matvec": roofline_mv, "extra": extra,
    }
    if ref is not None:
        out["cpu_baseline"] = cpu_baseline_entry(ref)
        extra["oracle_outer_it"] = ref["outer_it"]
        extra["oracle_relres_history"] = ref["history"]
        extra["oracle_true_relres"] = ref["rnorm_true"] / ref["fnorm"]
    # explicit teardown: every handle is released and the device idle before exit
    solver.close()
    del solver
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
