/*
 * sg.h -- C interface of the MI355X stochastic Galerkin (SG) solver library.
 *
 * Problem (Section 2 of Sousedik, Ghanem, Phipps, "Hierarchical Schur
 * complement preconditioner for the stochastic Galerkin finite element
 * methods"): -div(a(x, xi) grad u) = f on the unit square, u = 0 on the
 * boundary, with a linear Karhunen-Loeve coefficient
 *     a(x, xi) = theta0 + sigma * sum_{k=1..M} s_k phi_k(x) xi_k,
 * xi_k independent (standard Gaussian or uniform on [-1, 1]), Q1 elements on
 * an n_e x n_e grid and a normalised chaos of total degree <= p
 * (P = (M+p)!/(M! p!) functions). The discrete system is sum_k (G_k (x) K_k) vec(U) = vec(F)
 * (eq. (global-system), eq. (global-matrix)).
 *
 * Layout conventions used by every call
 *   n = (n_e - 1)^2 interior nodes, node (ix, iy), 1 <= ix, iy <= n_e - 1,
 *   has index (iy - 1)(n_e - 1) + (ix - 1) (x1 fastest).
 *   A block of chaos coefficients is an n x P column-major FP64 array in
 *   device memory, leading dimension n: column j holds chaos coefficient j.
 *   Chaos functions are graded by total degree; within one degree they are
 *   in descending lexicographic order of their multi-indices ((d,0,..,0)
 *   first). Level l (degree l) occupies columns level_off[l]..level_off[l+1]-1.
 *   Element arrays are indexed [ey][ex] (x1 fastest).
 *
 * Memory and streams
 *   The caller owns every array. The library allocates no device memory: it
 *   works inside a caller-provided device workspace whose size is returned
 *   by sg_workspace_bytes. Host inputs are copied during the call; no
 *   pointer is retained after a call returns except the workspace. All
 *   device work is issued on the stream given to sg_setup. Calls that return
 *   host scalars (sg_solve, sg_adjoint_grad, sg_inner_solve, sg_qoi)
 *   synchronise that stream; the others are asynchronous.
 *   A handle is not thread-safe; use one handle per stream.
 *
 * Status codes
 *   SG_OK (0); negative: the call was rejected and did nothing
 *   (SG_EINVAL invalid argument, SG_EDEVICE HIP runtime error,
 *   SG_ENOMEM workspace too small); positive: a solver outcome with the
 *   outputs filled (SG_NOT_CONVERGED: the last iterate is returned;
 *   SG_BREAKDOWN: a non-positive or non-finite curvature p^T A p was met,
 *   the last finite iterate is returned). sg_last_error() describes the
 *   most recent failure of the calling thread.
 */
#ifndef SG_H
#define SG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SG_OK = 0,
  SG_EINVAL = -1,
  SG_EDEVICE = -2,
  SG_ENOMEM = -3,
  SG_NOT_CONVERGED = 1,
  SG_BREAKDOWN = 2
};

enum { SG_PC_NONE = 0, SG_PC_MEAN = 1, SG_PC_HSC = 2, SG_PC_BGS = 3 };

typedef struct sg_ctx* sg_handle;

/* Problem description (Section 2; eq. (KL-expansion) with k_i = sqrt(lambda_i) v_i).
 * theta0 > 0 is the mean coefficient, sigma >= 0 the standard-deviation
 * scale, s[M] the KL amplitudes sqrt(lambda_k) and phi[M][n_e][n_e] the
 * element values of the KL modes (both host arrays, copied by sg_setup).
 * The element coefficient of KL term k is a_k(e) = sigma * s[k] * phi[k][e];
 * coefficients are constant per element. family selects the distribution of
 * the random variables and the chaos basis (Section 2):
 *   SG_FAMILY_HERMITE   standard Gaussian variables, normalised Hermite
 *                       polynomials He_a / sqrt(a!);
 *   SG_FAMILY_LEGENDRE  variables uniform on [-1, 1], normalised Legendre
 *                       polynomials sqrt(2a + 1) P_a (the examples of Section 6).
 * Requires n_e >= 3, M >= 0, p >= 0, P <= 2^20. */
enum { SG_FAMILY_HERMITE = 0, SG_FAMILY_LEGENDRE = 1 };

typedef struct sg_problem {
  int32_t n_e;
  int32_t M;
  int32_t p;
  int32_t family;
  double theta0;
  double sigma;
  const double* s;
  const double* phi;
} sg_problem;

/* Solver options.
 *   inner_precision   64 or 32: arithmetic of the inner K_0 solves and the
 *                     coupling products of the preconditioner (the outer
 *                     CG and the SG matvec are always FP64).
 *   cheb_degree       d >= 1: updates of the Chebyshev polynomial
 *                     preconditioner of the inner PCG (d - 1 products with
 *                     K_0 per application).
 *   inner_maxit       cap on inner PCG iterations per solve (>= 1).
 *   precond           SG_PC_NONE, SG_PC_MEAN, SG_PC_HSC or SG_PC_BGS for sg_solve.
 *   tile              spatial tiles of the inner solver: 32 = banded tiles (up to
 *                     64 columns including the Chebyshev halo; 128 rows in FP64,
 *                     256 in FP32; degrees <= 16),
 *                     16 = 16 x 16 tiles, 0 = automatic (banded tiles, with
 *                     64-row bands for launches of fewer tiles than compute
 *                     units; 16 x 16 tiles above degree 16).
 *   warm_start        0: every inner solve starts from zero. 1: the inner
 *                     solves of the up sweep of Algorithm 1 start from the
 *                     down-sweep solution of the same level, and those of the
 *                     backward sweep of block Gauss-Seidel from the forward
 *                     sweep's (banded tiles; 16 x 16 tiles start from zero).
 *                     The stopping test stays relative to the right-hand side.
 *   inner_rtol        relative residual at which an inner solve stops
 *                     (recursive residual, Euclidean norm); <= 0 runs
 *                     exactly inner_maxit iterations.
 *   use_graph         0 or 1: sg_solve captures one preconditioner action
 *                     (all its inner launches, couplings and read-backs) into
 *                     a HIP graph on the handle's stream the first time it is
 *                     applied and replays the graph in every later outer
 *                     iteration and solve (until the options or the schedule
 *                     change). Needs a stream other than the default one. The
 *                     inner launches of a captured action are ordinary (not
 *                     cooperative) launches of at most the resident grid.
 *                     Results are the same bit for bit.
 *   reserved          must be 0. */
typedef struct sg_opts {
  int32_t inner_precision;
  int32_t cheb_degree;
  int32_t inner_maxit;
  int32_t precond;
  int32_t tile;
  int32_t warm_start;
  double inner_rtol;
  int32_t use_graph;
  int32_t reserved;
} sg_opts;

/* Statistics of a solve. Counters are totals over the call. */
typedef struct sg_stats {
  int32_t outer_it;           /* outer FCG iterations */
  int32_t status;             /* same code as returned */
  int64_t inner_it_total;     /* inner PCG iterations summed over all solves */
  int64_t n_blockmv;          /* block products in preconditioner actions (n_m per HSC action) */
  int64_t n_blocksolve;       /* block solves in preconditioner actions (n_ds per HSC action) */
  int32_t inner_it_max[16];   /* max inner iterations per level (level l < 16) */
  double relres;              /* final recursive relative residual ||r||_2 / ||f||_2 */
  double true_relres;         /* ||f - A u||_2 / ||f||_2 recomputed at exit */
  double kappa_est;           /* Lanczos condition estimate from the FCG coefficients */
  double ms;                  /* wall time of the call in milliseconds */
  double ms_precond;          /* time in preconditioner actions */
  double ms_matvec;           /* time in SG matvecs */
  double ms_inner;            /* device time of the inner PCG launches (HIP events on the stream; with
                                 use_graph, of the replayed preconditioner actions as a whole) */
  double inner_bytes;         /* algorithmic bytes of those launches: per column (9 its + 6) n w
                                 with banded tiles, (10 its + 6) n w with 16 x 16 tiles (3 n w
                                 when it stops at once; n w more from a warm start) */
  int64_t inner_launches;     /* number of inner PCG launches */
} sg_stats;

/* Device workspace needed by sg_setup for this problem and options. */
int sg_workspace_bytes(const sg_problem* prob, const sg_opts* opts, size_t* bytes);

/* Validate, build the chaos tables and upload the coefficients into the
 * workspace (device pointer, at least sg_workspace_bytes long, 256-byte
 * aligned). `stream` is a hipStream_t (NULL = default stream). */
int sg_setup(const sg_problem* prob, const sg_opts* opts, void* workspace, size_t workspace_bytes,
             void* stream, sg_handle* out);

/* Sizes: n, P, level offsets level_off[p+2] and, if alpha is not NULL, the
 * multi-indices alpha[P][M] (host arrays). */
int sg_sizes(sg_handle h, int64_t* n, int32_t* P, int32_t* level_off, int32_t* alpha);

/* Replace the options of a handle (same inner precision as at setup). */
int sg_set_opts(sg_handle h, const sg_opts* opts);

/* Y = sum_k K_k U G_k^T (the MAT-VEC of the Remark after eq.
 * (global-matrix-block)); U and Y are distinct n x P device blocks. FP64. */
int sg_matvec(sg_handle h, const double* U, double* Y);

/* Z = M_P R: one action of the hierarchical Schur complement preconditioner
 * (Algorithm 1) with inexact diagonal-block solves by inner PCG (Section 5).
 * R and Z are distinct n x P device blocks. */
int sg_apply_hsc(sg_handle h, const double* R, double* Z);

/* Z = (I (x) K_0^-1) R approximately: the mean-based preconditioner (Section 6),
 * one inner PCG solve per column. */
int sg_apply_mean(sg_handle h, const double* R, double* Z);

/* Z = M_bGS R: one action of the block symmetric Gauss-Seidel preconditioner
 * (the comparator of Section 6) from a zero initial guess, blocks in the
 * graded chaos order, diagonal blocks K_0 inverted by the inner PCG. Blocks of
 * equal degree do not couple (linear KL expansion), so each sweep runs level
 * by level: forward l = 0..p with z_l = D_l^-1 (r_l - C_l z_{l-1}), backward
 * l = p-1..0 with z_l = D_l^-1 (r_l - C_l z'_{l-1} - B_{l+1} z_{l+1}), where
 * z' are the forward values (their product is kept, not recomputed) and the
 * top level keeps its forward value. R and Z are distinct n x P device blocks. */
int sg_apply_bgs(sg_handle h, const double* R, double* Z);

/* Inner solves on the diagonal blocks (Section 5): for columns c = 0..ncols-1,
 * PCG on K_0 x_c = b_c with the Jacobi-scaled Chebyshev preconditioner, in
 * the handle's inner precision (FP64 data in and out). B and X are distinct
 * n x ncols device blocks (ld = n), 0 <= ncols <= P. iters[ncols] (host, may
 * be NULL) receives the iteration count of each column. */
int sg_inner_solve(sg_handle h, const double* B, double* X, int32_t ncols, int32_t* iters);

/* sg_inner_solve without any device allocation, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid it): the inner solver's state vectors, the FP32
 * copies of B and X (FP32 inner precision), the per-tile partial sums and the
 * per-column counters live in a fixed 64 MiB device array of the library (one
 * copy per device, held until the process ends) instead of the handle's
 * workspace. Same arguments, results and synchronisation as sg_inner_solve.
 * SG_ENOMEM if ncols columns need more than 64 MiB of that scratch (per column
 * 6 n w bytes, 8 n w in FP32, plus partial sums; at n = 65025 in FP64 at most
 * 20 columns). Every call on one device shares its array: calls that overlap
 * on one device (other streams, other host threads) race and must be
 * serialised by the caller. */
int sg_inner_solve_static(sg_handle h, const double* B, double* X, int32_t ncols, int32_t* iters);

/* Coupling products of Algorithm 1 on level l (1 <= l <= p), FP64:
 *   dir = 0 (pre-correction):  R[:, level l-1] -= (B_l Y)[:, level l-1]
 *            with Y read from the level-l columns of Y;
 *   dir = 1 (post-correction): R[:, level l] -= (C_l Z)[:, level l]
 *            with Z read from the level-(l-1) columns of Z.
 * R, Y/Z are n x P device blocks. */
int sg_coupling(sg_handle h, int32_t level, int32_t dir, double* R, const double* V);

/* Solve A U = F by flexible CG (Section 5) preconditioned as opts.precond,
 * to ||f - A u||_2 <= rtol ||f||_2 (recursive residual) or maxit outer
 * iterations. use_x0 != 0 starts from the contents of U, else from zero.
 * stats (host, may be NULL) is filled. */
int sg_solve(sg_handle h, const double* F, double* U, double rtol, int32_t maxit, int32_t use_x0,
             sg_stats* stats);

/* Solve A U = F through the a-priori reduction to the Schur complement of the
 * top chaos degree (Section 5, eq. (global-Schur-system)): flexible CG on
 *   S u_low = f_low - B_p D_p^-1 f_top,  S = A_{P-1} - B_p D_p^-1 C_p,
 * over the columns of degree < p, preconditioned by Algorithm 1 over the
 * levels 1..p-1 (opts.precond = SG_PC_HSC) or by the mean-based preconditioner
 * (SG_PC_MEAN), to ||g - S u_low||_2 <= rtol ||g||_2 or maxit iterations; then
 * u_top = D_p^-1 (f_top - C_p u_low). The D_p solves of the operator, of the
 * right-hand side and of the recovery run the inner PCG to op_rtol (0 < op_rtol
 * < 1; the reduction is exact only for exact D_p solves), the preconditioner's
 * to opts.inner_rtol. Needs p >= 1 and opts.inner_precision = 64. F and U are
 * distinct n x P device blocks; U is overwritten (zero start). stats (host, may
 * be NULL) counts the reduced iteration; its true_relres is that of the full
 * system. */
int sg_solve_reduced(sg_handle h, const double* F, double* U, double rtol, int32_t maxit, double op_rtol,
                     sg_stats* stats);

/* Quantity of interest Q = w_mean . U[:,0] + sum_{j>=1} w_var . U[:,j]^2
 * (w_mean, w_var: n-vectors on the device); result to *Q (host). */
int sg_qoi(sg_handle h, const double* U, const double* w_mean, const double* w_var, double* Q);

/* Gradient of Q with respect to theta = (theta0, s_1..s_M) at the solution U
 * of A U = F: solves the adjoint system A Lambda = dQ/dU with the same
 * preconditioned FCG (A is symmetric) to rtol, then contracts
 * dQ/dtheta_i = -<Lambda, (dA/dtheta_i) U>. Q (host) and grad[1+M] (host)
 * receive the results; Lambda (device n x P, may be NULL, distinct from U)
 * receives the adjoint solution. rtol >= 0 and maxit >= 0 as for sg_solve. */
int sg_adjoint_grad(sg_handle h, const double* U, const double* w_mean, const double* w_var,
                    double rtol, int32_t maxit, double* Q, double* grad, double* Lambda,
                    sg_stats* stats);

/* Schedule autotuner. Times candidate launch schedules on this handle's own
 * grid and chaos sizes and keeps the fastest for all later calls:
 *   flags bit 0: the SG operator (piece kernel with 8, 16 or 32 node rows
 *                per piece and all resident waves or 4 per CU, when M <= 12;
 *                y-marching kernel with 1, 2 or 4 grid segments per XCD or the
 *                automatic count; band kernels with 32..128 row chunks per
 *                band, where the grid shape allows them);
 *   flags bit 1: the inner PCG (tile kind 16 or 32 where the Chebyshev halo
 *                allows 32; block count automatic, half the CUs, or whole
 *                columns per block), timed on
 *                the columns of the largest chaos level with a constant
 *                right-hand side.
 * Runs on the handle's stream inside its workspace (the FCG vectors and the
 * inner solver's state are overwritten) and synchronises it. The schedules
 * differ only in the order of floating-point sums. report (host, may be NULL)
 * receives the choice. */
typedef struct sg_tune_report {
  int32_t mv_variant;      /* 0, 1: band kernels; 2: y-marching kernel; 3: piece kernel;
                              4: row-staged kernel (node rows of all chaos columns in LDS) */
  int32_t mv_param;        /* row chunks per band (variants 0, 1); segments per XCD (2; 0 = automatic);
                              100 * rows per piece + waves per CU (3; 0 waves = all resident);
                              node rows per piece (4) */
  int32_t pcg_tile;        /* inner tile kind (32 banded, 16 square) */
  int32_t pcg_max_blocks;  /* cap on the blocks of an inner launch (0 = as many as fit; -1 = whole
                              columns per block for launches whose columns fill at least 3/4 of the
                              resident blocks, no cap for smaller ones) */
  double mv_ms;            /* median time of one SG matvec with the chosen schedule */
  double pcg_ms;           /* time of the inner test solve with the chosen schedule */
  int32_t candidates;      /* schedules timed */
  int32_t pcg_rows;        /* band height of banded inner tiles (sg_batch_autotune; 16 for 16 x 16
                              tiles); 0 from sg_autotune, whose launches pick it by their size */
} sg_tune_report;

int sg_autotune(sg_handle h, int32_t flags, sg_tune_report* report);

/* Release the handle (the workspace stays with the caller). */
void sg_destroy(sg_handle h);

/* ---- Multi-problem batch.
 * Many independent problems (each as in sg_setup: its own grid, KL terms and
 * chaos degree) solved together by the flexible CG of Section 5 with the
 * preconditioner opts.precond (SG_PC_HSC, Algorithm 1, SG_PC_MEAN or
 * SG_PC_BGS, Section 6); all problems share the options. One outer iteration of the
 * batch runs, for all problems that have not stopped yet: the diagonal-block
 * solves of each step of Algorithm 1 for every problem in one inner launch,
 * the coupling products and SG matvecs of each problem, and batched vector
 * updates whose scalars stay on the device. A problem stops on its own test
 * (same stopping rule as sg_solve, zero initial guess) and is skipped from
 * then on. */
typedef struct sg_batch_ctx* sg_batch;

/* Device workspace for a batch of `count` problems (probs[count], host). */
int sg_batch_workspace_bytes(int32_t count, const sg_problem* probs, const sg_opts* opts, size_t* bytes);

/* Set up the batch inside the workspace (device, 256-byte aligned, at least
 * sg_batch_workspace_bytes long); all work goes to `stream`. */
int sg_batch_setup(int32_t count, const sg_problem* probs, const sg_opts* opts, void* workspace,
                   size_t workspace_bytes, void* stream, sg_batch* out);

/* n and P of problem i of the batch. */
int sg_batch_sizes(sg_batch b, int32_t i, int64_t* n, int32_t* P);

/* Solve problem i: F[i] (right-hand side) and U[i] (solution) are n_i x P_i
 * device blocks in the layout of sg_solve; F and U are host arrays of
 * `count` device pointers. use_graph != 0 captures one outer iteration of the
 * batch into a HIP graph at the second iteration and replays it afterwards
 * (the batch's stream must then not be the default stream: SG_EINVAL).
 * stats[count] (host, may be NULL) receives each problem's statistics (ms is
 * the wall time of the whole batch); *ms_total (may be NULL) the same time.
 * Returns SG_OK if every problem converged, else the first non-OK outcome
 * (SG_BREAKDOWN before SG_NOT_CONVERGED); per-problem outcomes are in stats. */
int sg_batch_solve(sg_batch b, const double* const* F, double* const* U, double rtol, int32_t maxit,
                   int32_t use_graph, sg_stats* stats, double* ms_total);

/* Release the batch and its per-problem handles (the workspace stays with the caller). */
/* Schedule autotuner of a batch (the batch counterpart of sg_autotune):
 *   flags bit 0: every member's SG operator, as sg_autotune's bit 0 on the
 *                member's own sizes;
 *   flags bit 1: the ragged inner launches: banded tiles with the default or
 *                64-row bands, and 16 x 16 tiles when opts.tile is 0, each
 *                with all or half of the compute units, timed on one inner
 *                solve of every column set a preconditioner action uses, with
 *                a constant right-hand side in every problem.
 * Overwrites the members' vectors, drops a captured graph and synchronises
 * the stream; the candidates differ only in the order of floating-point sums.
 * report (host, may be NULL) receives the choice: the inner schedule, and
 * the SG-operator schedule of the largest member with mv_ms summed over the
 * members. */
int sg_batch_autotune(sg_batch b, int32_t flags, sg_tune_report* report);

void sg_batch_destroy(sg_batch b);

/* Lognormal coefficient (Section 6, second set of experiments; Tables 6-9).
 * The coefficient is k(x, xi) = exp(g(x, xi)) with the Gaussian field
 * g = mu_g + sum_k g_k(x) xi_k, g_k(e) = sigma_g s[k] phi[k][e], expanded in
 * the normalised Hermite chaos to total degree 2p; the solution has degree p.
 * The fields of sg_problem mean here: theta0 > 0 the mean of k, sigma >= 0 its
 * coefficient of variation, s and phi the KL data of the Gaussian field;
 * family must be SG_FAMILY_HERMITE; 3 <= n_e <= 4096, M <= 16, p <= 8,
 * P^2 <= 2^22, C(M+2p, 2p) <= 2^20 coefficient terms and that count times
 * n_e^2 <= 2.5e8 (the host builds the terms' element fields). sigma_g^2 = ln(1 + sigma^2) and mu_g = ln(theta0) - sigma_g^2/2
 * give k that mean and CoV. The global matrix A = sum_i G_i (x) K_i with
 * (G_i)_ab = E[psi_i psi_a psi_b] couples every pair of chaos blocks that
 * some term reaches (block dense); the library stores each such block's
 * element coefficient field c_ab = sum_i (G_i)_ab k_i (nblocks x n_e^2 FP64 in
 * the workspace, computed at setup).
 *   sg_logn_workspace_bytes  device bytes the handle needs;
 *   sg_logn_setup            tables and block fields into `workspace` (device,
 *                            256-byte aligned, caller-owned, at least the
 *                            queried size), work on `stream`; synchronises it;
 *   sg_logn_sizes            n, P and the number of stored blocks (host outputs,
 *                            each may be NULL);
 *   sg_logn_matvec           Y = A U for distinct n x P FP64 device blocks in the
 *                            layout of sg_matvec (asynchronous on the stream);
 *   sg_logn_destroy          frees the host handle (not the workspace).
 *   sg_logn_solve            A U = F (distinct n x P device blocks; U is overwritten,
 *                            zero start) by flexible CG (Section 5) to
 *                            ||f - A u||_2 <= rtol ||f||_2 (recursive residual) or maxit
 *                            iterations, preconditioned (Section 6) by
 *                            SG_PC_HSC: Algorithm 1 with the full level blocks D_l
 *                              (they couple here);
 *                            SG_PC_BGS: block symmetric Gauss-Seidel over the chaos
 *                              blocks, diagonal blocks A_aa = K(c_aa);
 *                            SG_PC_MEAN: I (x) K(k_0)^-1, k_0 the mean coefficient.
 *                            Each block solve is a Jacobi-preconditioned CG to
 *                            inner_rtol (0 < inner_rtol < 1) or inner_maxit
 *                            iterations (one per column for the mean-based
 *                            preconditioner); the paper found direct and iterative D_l
 *                            solves to the outer tolerance equivalent. Host outputs
 *                            (each may be NULL): outer iterations, total inner
 *                            iterations, final relative residual and the Lanczos
 *                            condition estimate of the preconditioned operator.
 *                            Synchronises the stream. Returns SG_OK,
 *                            SG_NOT_CONVERGED or SG_BREAKDOWN as sg_solve.
 */
typedef struct sg_logn_ctx* sg_logn_handle;
int sg_logn_workspace_bytes(const sg_problem* prob, size_t* bytes);
int sg_logn_setup(const sg_problem* prob, void* workspace, size_t workspace_bytes, void* stream,
                  sg_logn_handle* out);
int sg_logn_sizes(sg_logn_handle h, int64_t* n, int32_t* P, int32_t* nblocks);
int sg_logn_matvec(sg_logn_handle h, const double* U, double* Y);
int sg_logn_solve(sg_logn_handle h, int32_t precond, const double* F, double* U, double rtol, int32_t maxit,
                  double inner_rtol, int32_t inner_maxit, int32_t* outer_it, int64_t* inner_it, double* relres,
                  double* kappa);
void sg_logn_destroy(sg_logn_handle h);

/* Thread-local description of the last failure (never NULL). */
const char* sg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SG_H */
