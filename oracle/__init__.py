"""CPU oracle for the stochastic Galerkin (SG) solver -- TEST INFRASTRUCTURE ONLY.

A plain, slow FP64 implementation (NumPy / SciPy) of what the GPU path
computes, written from the paper (Sousedik, Ghanem, Phipps: "Hierarchical
Schur complement preconditioner for the stochastic Galerkin finite element
methods"). It shares no code with the GPU library: only ``tests/``, the
package smoke check and the CPU-baseline leg of the benchmark may import it.

Modules
-------
fe       Q1 finite elements: element stiffness, assembled K_k (Section 2).
chaos    Hermite chaos: graded multi-indices, Galerkin matrices
         G_k = E[xi_k psi_a psi_b] by Gauss-Hermite quadrature (eq.
         (global-system), eq. (global-matrix-block)).
sg       The global SG operator: assembled Kronecker form (eq.
         (global-matrix)) and the matrix-free MAT-VEC form (Remark after
         eq. (global-matrix-block)); level structure (eq.
         (global-matrix-hierarchy)).
krylov   Flexible CG (Section 5), inner PCG with a Jacobi-scaled Chebyshev
         polynomial preconditioner, Lanczos condition estimate (Section 6).
hsc      Algorithm 1 (hierarchical Schur complement preconditioner) and the
         mean-based preconditioner (Section 6).
adjoint  Quantity of interest, adjoint gradient and finite differences.
bgs      Block symmetric Gauss-Seidel preconditioner (Section 6).
schur    A-priori reduction to the Schur complement of the top degree
         (Section 5).
lognormal
         Lognormal coefficient expanded in Hermite chaos to twice the
         solution's degree, with the full-level-block preconditioners
         (Section 6, Tables 6-9).

Every function cites the passage it follows. Readings of points where the
paper is silent are stated where they are used.
"""
