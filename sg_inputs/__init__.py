"""Seeded synthetic inputs for the stochastic Galerkin model problem.

This package only *generates inputs*: mesh geometry, the Karhunen-Loeve (KL)
data of the random coefficient, right-hand sides, quantity-of-interest
weights, random test vectors and the parameter sets of the workloads. It holds
none of the solver's arithmetic (no stiffness assembly, no Galerkin products,
no preconditioner), so both the CPU oracle and the GPU path may use it.

Model problem: Section 2 of the paper (random diffusion equation on the unit
square, homogeneous Dirichlet data, linear KL expansion of the coefficient with
an exponential covariance, eq. (cov)).
"""

from .problems import (  # noqa: F401
    Problem,
    kl_1d,
    kl_2d,
    make_problem,
    named_problem,
    nodal_rhs,
    qoi_weights,
    random_block,
    batch_problems,
    n_chaos,
)
