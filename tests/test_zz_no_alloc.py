"""The allocation-free inner solve (sg_inner_solve_static) against sg_inner_solve.

Both run the same kernels on the same inputs, so the solutions and iteration
counts must agree bit for bit; two calls in a row, the second with fewer
columns (the static scratch keeps the previous call's contents)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from sg_inputs import named_problem, random_block  # noqa: E402


@pytest.mark.parametrize("prec", [64, 32])
def test_inner_solve_static_matches_workspace_solve(prec):
    from paper_1205_1864_amd import binding as b
    prob = named_problem("small", n_e=64, M=4, p=3)
    print(f"inner_solve_static n_e=64 M=4 p=3 P={prob.P} FP{prec}", flush=True)
    solver = b.SGSolver(prob, b.Options(inner_precision=prec, cheb_degree=8, inner_rtol=1e-6, inner_maxit=500))
    try:
        for ncols, seed in ((prob.P, 1), (5, 2)):
            B = b.to_device_block(random_block(ncols, prob.n, seed=seed))
            X_ws, it_ws = solver.sg_inner_solve(B)
            X_st, it_st = solver.sg_inner_solve_static(B)
            assert np.array_equal(it_ws, it_st)
            assert np.all(it_st > 0) and np.all(it_st < 500)
            assert np.array_equal(X_ws.cpu().numpy(), X_st.cpu().numpy())
    finally:
        solver.close()


def test_inner_solve_static_rejects_oversize():
    from paper_1205_1864_amd import binding as b
    prob = named_problem("scale")
    print("inner_solve_static size check 256^2", flush=True)
    solver = b.SGSolver(prob, b.Options(inner_precision=64, cheb_degree=16))
    try:
        B = b.to_device_block(random_block(40, prob.n, seed=3))
        with pytest.raises(b.SGError) as ei:
            solver.sg_inner_solve_static(B)
        assert ei.value.code == b.SG_ENOMEM and "scratch" in str(ei.value)
    finally:
        solver.close()
