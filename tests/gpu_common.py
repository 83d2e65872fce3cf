"""Shared helpers of the GPU parity tests."""

import functools

import numpy as np

from oracle import sg
from sg_inputs import named_problem


@functools.lru_cache(maxsize=None)
def system(name, **kw):
    prob = named_problem(name, **dict(kw))
    return prob, sg.build_system(prob)


def cached_system(name, **kw):
    return system(name, **kw)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@functools.lru_cache(maxsize=None)
def oracle_solution(name, rtol=1e-10):
    """The oracle's solve of a named workload: flexible CG preconditioned by
    Algorithm 1 with exact sparse-LU K_0 solves, to relres ``rtol``. Returns
    (problem, system, F (n x P), U (n x P), ||f - A U||_2)."""
    from oracle import solve
    prob, s = system(name)
    F = prob.load_block().T.copy()
    res, _, _ = solve.solve_fcg(s, F, precond="hsc", inner="exact", rtol=rtol, maxit=100)
    assert res.converged
    r = F - sg.matvec(s, res.x)
    return prob, s, F, res.x, float(np.linalg.norm(r))
