/*
 * hinv.h -- C ABI of libhinv, Hessian actions for Bayesian inversion of the
 * Poisson log-coefficient problem on MI355X (gfx950).
 *
 * The operations follow the problem statement of Villa, Petra & Ghattas,
 * "hIPPYlib: an extensible software framework for large-scale inverse
 * problems governed by PDEs; Part I" (ACM TOMS; arXiv:1909.03948):
 *
 *   forward   -div(e^m grad u) = 0 in (0,1)^2, u = 0 on y = 0, u = 1 on y = 1,
 *             zero flux on x = 0, 1                     (Sec. 5.1, Eq. equ:poi)
 *   cost      J(m) = 1/2 sigma^-2 |B u - d|^2 + 1/2 |m - m_pr|^2_R
 *                                                       (Sec. 5.1, Eq. eq:cost-elliptic)
 *   gradient  adjoint solve + g = R (m - m_pr) + C(u)^T p (App. A, Eqs. eq:firstadj,
 *                                                        eq:firstcontrol)
 *   Hessian   incremental forward / adjoint solves and the Hessian action
 *             (App. A, Eqs. eq:incrementals1-3; Sec. 2.1, Eq. eq:abstract_hessianAction)
 *   prior     R = K_A M^-1 K_A, K_A = gamma K + delta M + beta M_boundary
 *             (Sec. 5.1, Eq. eq:PoissonPrior; Sec. 2.3), prior draws through the
 *             rectangular mass factor (Sec. 4.3.1, Eq. eq:sample_prior; App. C)
 *   MAP       inexact Newton-CG (Alg. 1)
 *   low rank  double-pass randomized generalized eigensolver with PreCholQR
 *             (Alg. 2, Alg. 4; Eq. eq:eigenproblem_1)
 *   samples   y = (I - V S V^T R) x (Sec. 4.3.2, Eq. eq:sample_post)
 *
 * Discretization: P1 state and parameter on the N x N right-diagonal
 * triangulation of the unit square; node k(i,j) = j (N+1) + i; the diagonal of
 * cell (i,j) joins (i,j) and (i+1,j+1); triangle t = 2 (j N + i) + s, s = 0 for
 * the lower and 1 for the upper triangle; e^m is integrated with the centroid
 * rule, c_T = exp((m_a + m_r + m_b) / 3).
 *
 * Conventions
 *   - Every function returns an int status (HINV_OK or a negative HINV_E*).
 *     On error the detail string is available from hinv_last_error(ctx).
 *   - Vector arguments are DEVICE pointers to FP64 data owned by the caller.
 *     A vector of the parameter or state space has n = (N+1)^2 entries in node
 *     order.  A multivector of nrhs columns is column-major with leading
 *     dimension ld >= n (column c starts at ptr + c * ld).  The library never
 *     frees or retains caller memory beyond the call.
 *   - State-like vectors (u) hold their Dirichlet values; adjoint-like and
 *     incremental vectors (p, uhat, phat) are zero on the Dirichlet nodes.
 *   - All work is ordered on the context's HIP stream (a full Hessian action
 *     forks its prior term onto an internal stream with an event and joins it
 *     back before it returns).  Functions that return host values (cost, info
 *     structs, eigenvalues) synchronize that stream.
 *   - A context is not thread-safe; use one context per host thread.
 *   - Iterative solves stop at |b - A x|_2 / |b|_2 <= rtol per column, the
 *     residual evaluated in FP64.  A column that does not get there within the
 *     iteration limit makes the call return HINV_ENOCONV; outputs are still
 *     written and info->status holds the same code.  A NaN or infinite
 *     residual (a non-finite entry in an input, or one met during the solve)
 *     stops its column at once: the call returns HINV_ENOCONV and
 *     info->max_relres is NaN.
 */
#ifndef HINV_H
#define HINV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define HINV_OK        0
#define HINV_EINVAL   -1   /* invalid argument (null pointer, bad size or mode) */
#define HINV_ENOMEM   -2   /* device allocation failed */
#define HINV_EHIP     -3   /* HIP runtime error */
#define HINV_ENOCONV  -4   /* an iterative solve missed its tolerance */
#define HINV_ESTATE   -5   /* call out of order (e.g. Hessian before hinv_linearize) */
#define HINV_ENEGEIG  -6   /* eigenvalue <= -1 passed to the posterior sampler */
#define HINV_EBREAK   -7   /* Cholesky breakdown in PreCholQR (rank-deficient probe block) */

/* Hessian modes (App. A; Gauss-Newton per the footnote to Eq. eq:laplace_approx) */
#define HINV_HESS_FULL       0  /* misfit + prior */
#define HINV_HESS_MISFIT     1  /* data-misfit part only */
#define HINV_HESS_GN_FULL    2  /* Gauss-Newton misfit + prior */
#define HINV_HESS_GN_MISFIT  3  /* Gauss-Newton misfit only */

/* solver precision */
#define HINV_PREC_FP64     0  /* FP64 CG preconditioned by an FP32 multigrid V-cycle */
#define HINV_PREC_FP32_IR  1  /* FP32 multigrid-PCG inside FP64 iterative refinement */
#define HINV_PREC_AUTO     2  /* per call: FP64 below 8 right-hand sides (latency bound),
                                 FP32_IR from 8 up (bandwidth bound) */

/* precision of the T = Q^T (A Q) block product of the eigensolver */
#define HINV_TPROD_FP64    0  /* FP64 matrix cores */
#define HINV_TPROD_BF16    1  /* BF16 inputs, FP32 accumulation */

typedef struct hinv_ctx hinv_ctx;
typedef struct hinv_problem hinv_problem;
typedef struct hinv_batch hinv_batch;
typedef struct hinv_cnn hinv_cnn;

typedef struct {
    int    N;          /* cells per side, a power of two >= 4 */
    double gamma;      /* prior diffusion weight (> 0) */
    double delta;      /* prior reaction weight (> 0) */
    double beta;       /* Robin coefficient; NaN selects sqrt(gamma*delta)/1.42 */
    double m_prior;    /* constant prior mean */
    int    q;          /* number of observations (>= 0) */
    const double* obs_xy; /* HOST array [2q]: (x0, y0, x1, y1, ...) in [0,1]^2 */
    const double* d_obs;  /* HOST array [q] of data, may be NULL (zeros) */
    double sigma;      /* noise standard deviation (> 0) */
    int    precision;  /* HINV_PREC_* for the state-equation solves */
    double rtol;       /* relative residual of every solve, e.g. 1e-10 */
    int    max_iter;   /* iteration cap per solve (0: 200) */
    /* Anisotropic tensor of the prior's diffusion term, -gamma div(Theta grad m)
     * (Sec. 5.1, Eq. eq:PoissonPrior): Theta = theta1 v v^T + theta2 w w^T with
     * v = (sin alpha, cos alpha), w = (cos alpha, -sin alpha) -- the s.p.d.
     * tensor with the eigenvalues and directions the section states (the matrix
     * printed there is not s.p.d. for its own parameters).  theta1 <= 0 selects
     * Theta = I.  The mesh needs 0 <= Theta_12 <= min(Theta_11, Theta_22) (its
     * diagonals lie along the principal direction; HINV_EINVAL otherwise), which
     * holds for theta1 >= theta2 > 0 and 0 <= alpha <= pi/2, e.g. the paper's
     * theta = (2, 0.5), alpha = pi/4. */
    double theta1, theta2, alpha;
    /* Degree of the state space: 0 or 1 -- P1 on the parameter's nodes;
     * 2 -- P2, the pairing of Sec. 5.1 (quadratic state, linear parameter).
     * With 2, every state-space vector (u, adjoint p, uhat, phat, and the
     * arguments of hinv_state_apply / hinv_state_solve) has ns = (2N+1)^2
     * entries, node J (2N+1) + I at (I h/2, J h/2) (vertices and edge
     * midpoints); the parameter-space vectors keep n = (N+1)^2.  Its solves
     * are FP64 PCG with a two-level preconditioner (P2 Chebyshev-Jacobi
     * smoothing around one V-cycle of the P1 operator, the exact Galerkin
     * coarse space) whatever the precision setting.  Batches, flexible CG and
     * the CNN pair harvest take P1 problems only (HINV_EINVAL). */
    int state_degree;
} hinv_problem_desc;

typedef struct {
    int    status;        /* HINV_OK or HINV_ENOCONV */
    int    solves;        /* number of solves (columns x systems) */
    int    iterations;    /* total PCG iterations, all precisions and refinement steps */
    int    refinements;   /* FP64 refinement steps */
    int    fallbacks;     /* FP32_IR solves that switched to FP64 after stagnating */
    double max_relres;    /* largest final FP64 relative residual over the solves */
} hinv_solve_info;

typedef struct {
    double rel_tol;      /* stop when |g_i| <= rel_tol |g_0| (default 1e-6) */
    double abs_tol;      /* ... or |g_i| <= abs_tol (default 0) */
    int    max_iter;     /* Newton iterations (default 50) */
    int    max_backtrack;/* Armijo backtracking steps (default 10) */
    double c_armijo;     /* Armijo constant (default 1e-4) */
    int    max_cg;       /* CG iterations per Newton step (default 500) */
    int    gn_iters;     /* the first gn_iters Newton steps use the Gauss-Newton Hessian,
                            the later ones the full Hessian (default 5; >= max_iter:
                            Gauss-Newton throughout) */
} hinv_newton_opts;

#define HINV_NEWTON_MAXREC 64
typedef struct {
    int    status;        /* HINV_OK, HINV_ENOCONV (max_iter) or HINV_ESTATE (line search failed) */
    int    iterations;    /* Newton iterations taken */
    int    converged;
    int    hessian_applies; /* total Hessian actions in the CG loops */
    double cost[HINV_NEWTON_MAXREC + 1];
    double gnorm[HINV_NEWTON_MAXREC + 1];
    int    cg_iters[HINV_NEWTON_MAXREC];
    double alpha[HINV_NEWTON_MAXREC];
    hinv_solve_info solves; /* accumulated over all PDE solves */
} hinv_newton_info;

/* Device memory for the library's workspaces, supplied by the caller (e.g. a
 * framework's caching allocator).  Every device buffer the library owns -- the
 * multigrid hierarchies, solver and eigensolver workspaces, reduction scratch
 * -- is obtained through it; the library never frees caller-owned vectors.
 *   alloc: returns `bytes` bytes of device memory on the context's device, for
 *          work the library enqueues on `stream` (the context's stream), or
 *          NULL on failure (the call then returns HINV_ENOMEM);
 *   free:  returns memory obtained from alloc, stream-ordered: work already
 *          enqueued on `stream` may still use it, so it must not be handed to
 *          work that is not ordered after that stream (the semantics of
 *          hipFreeAsync, or of a caching allocator that records the stream).
 * Workspaces grow to the largest call and are kept until the object that owns
 * them is destroyed: repeated calls of one shape allocate nothing. */
typedef struct hinv_allocator {
    void* (*alloc)(size_t bytes, void* stream, void* user);
    void (*free)(void* ptr, size_t bytes, void* stream, void* user);
    void* user;
} hinv_allocator;

/* ---- context ------------------------------------------------------------- */
/* Creates a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the legacy default stream).  alloc: device allocator
 * (copied; both callbacks non-NULL) or NULL for hipMalloc / hipFree, in which
 * case a buffer is freed only after the context's stream has finished with it.
 * Problems, batches and networks of a context must be destroyed before it. */
int hinv_ctx_create(int device, void* hip_stream, const hinv_allocator* alloc, hinv_ctx** out);
int hinv_ctx_destroy(hinv_ctx* ctx);
/* Switches the stream later calls enqueue on; waits for the previous stream
 * first, so buffers it still uses can be returned on the new one. */
int hinv_ctx_set_stream(hinv_ctx* ctx, void* hip_stream);
const char* hinv_last_error(const hinv_ctx* ctx);
const char* hinv_status_string(int status);

/* ---- kernel timing (roofline reports) ------------------------------------- */
#define HINV_KCLASS_MG_DOWN     0  /* finest-level pre-smooth + residual + restriction */
#define HINV_KCLASS_MG_UP       1  /* finest-level prolongation + post-smooth (+ r^T z) */
#define HINV_KCLASS_MG_BOTTOM   2  /* all levels N <= 32, one workgroup per column */
#define HINV_KCLASS_PCG_APPLY   3  /* p = z + beta p, q = A p */
#define HINV_KCLASS_PCG_UPDATE  4  /* x += alpha p, r -= alpha q */
#define HINV_KCLASS_GRAM        5  /* tall-skinny block product X^T Y on the matrix cores */
/* Classes 0, 1, 3 and 4 count launches of one to seven columns (single
 * right-hand sides); the same kernels launched for eight or more columns
 * (batched solves) are timed apart in these classes: */
#define HINV_KCLASS_MG_DOWN_BATCHED     6
#define HINV_KCLASS_MG_UP_BATCHED       7
#define HINV_KCLASS_PCG_APPLY_BATCHED   8
#define HINV_KCLASS_PCG_UPDATE_BATCHED  9
/* Enables (enable = 1) or disables sampled timing of one kernel class: every
 * `period`-th launch (period >= 1) is bracketed by HIP events on the context's
 * stream, at most 2048 launches per class.  Enabling clears the record. */
int hinv_ctx_kernel_timer(hinv_ctx* ctx, int kclass, int enable, int period);
/* Synchronizes the stream and returns, for the timed launches of a class:
 * their number, their summed duration (ms) and their summed algorithmic work
 * (bytes moved for the stencil and vector kernels -- each array counted once
 * per launch -- or flops for HINV_KCLASS_GRAM); `launches_total` is the number
 * of launches of the class while enabled. */
int hinv_ctx_kernel_timer_read(hinv_ctx* ctx, int kclass, int* timed, long* launches_total,
                               double* total_ms, double* total_work);

/* ---- launch-shape tuner ---------------------------------------------------- */
/* The first solve of each (operator, mesh size, column count, precision) times
 * candidate launch shapes on its own right-hand sides -- tile sizes of the
 * V-cycle kernels, the RHS-block width (columns one V-cycle workgroup sweeps:
 * 1, 2, 4, 8, 16) and node blocks per workgroup of the PCG vector kernels --
 * and keeps the fastest for the hierarchy's lifetime.  With the environment
 * variable HINV_TUNE_CACHE naming a file, the choices are appended to it as
 * JSON lines keyed by device architecture, compute units, operator kind, mesh
 * size, stacked instances, columns and precision, and later processes take
 * them from there instead of timing again (HINV_AUTOTUNE=0 disables both).
 * Returns the process-wide counts of shapes timed and taken from the file. */
int hinv_tuner_counts(long long* timed, long long* cached);

/* ---- problem -------------------------------------------------------------- */
/* Builds mesh data, prior multigrid hierarchy and observation operator.
 * Observation points are located in their cells on the device; the host only
 * sorts the resulting node indices to build the transpose. */
int hinv_problem_create(hinv_ctx* ctx, const hinv_problem_desc* d, hinv_problem** out);
int hinv_problem_destroy(hinv_problem* p);
/* n = (N+1)^2 */
int hinv_problem_size(const hinv_problem* p, int* n);
/* Entries of a state-space vector: (N+1)^2 for a P1 state, (2N+1)^2 for a P2
 * state (hinv_problem_desc.state_degree; Sec. 5.1). */
int hinv_problem_state_size(const hinv_problem* p, int* ns);
/* Replaces the data vector d (host array of q values) and/or sigma (> 0). */
int hinv_set_data(hinv_problem* p, const double* d_obs_host, double sigma);
/* Overrides precision and tolerance of the state-equation solves. */
int hinv_set_solver(hinv_problem* p, int precision, double rtol, int max_iter);

/* ---- forward problem and cost (Sec. 5.1) ----------------------------------- */
/* u[n]: solution of the forward problem at m[n] (Dirichlet values included). */
int hinv_forward(hinv_problem* p, const double* m, double* u, hinv_solve_info* info);
/* Host outputs: misfit = 1/2 sigma^-2 |B u - d|^2, reg = 1/2 (m-m_pr)^T R (m-m_pr). */
int hinv_cost(hinv_problem* p, const double* m, const double* u, double* misfit, double* reg);
/* Observations B u (q values, device). */
int hinv_observe(hinv_problem* p, const double* u, double* Bu);

/* ---- adjoint and gradient (App. A) -------------------------------------- */
/* p[n]: adjoint state; g[n]: gradient of J at m (u from hinv_forward). */
int hinv_gradient(hinv_problem* p, const double* m, const double* u, double* adj, double* g,
                  hinv_solve_info* info);

/* ---- Hessian action (App. A) ---------------------------------------------- */
/* Fixes the point (m, u, p) of later Hessian actions; builds the multigrid
 * hierarchy of A(m). u and adj must be the forward and adjoint solutions at m. */
int hinv_linearize(hinv_problem* p, const double* m, const double* u, const double* adj);
/* Incremental forward: uhat[:,c] solves A uhat = -C(u) mhat[:,c] (Eq. eq:incrementals1). */
int hinv_inc_forward(hinv_problem* p, int nrhs, const double* mhat, int ldm,
                     double* uhat, int ldu, hinv_solve_info* info);
/* Incremental adjoint: phat solves A phat = -(B^T B uhat / sigma^2 + C(p) mhat)
 * (Eq. eq:incrementals2); gauss_newton = 1 drops C(p) mhat. */
int hinv_inc_adjoint(hinv_problem* p, int nrhs, int gauss_newton, const double* mhat, int ldm,
                     const double* uhat, int ldu, double* phat, int ldp, hinv_solve_info* info);
/* out[:,c] = H mhat[:,c] in the given HINV_HESS_* mode (Eq. eq:incrementals3).
 * All nrhs columns go through one batched multi-right-hand-side solve.  The
 * incremental adjoint's right-hand side carries uhat, so when the solves run
 * in FP32 refinement (HINV_PREC_FP32_IR, or HINV_PREC_AUTO with 8 or more
 * columns) the incremental forward solve aims at rtol / 10 (a column whose
 * FP64 residual stops falling above that but at or below rtol is accepted);
 * the adjoint solve, and every solve of hinv_inc_forward / hinv_inc_adjoint,
 * run to rtol. */
int hinv_hessian_apply(hinv_problem* p, int mode, int nrhs, const double* mhat, int ldm,
                       double* out, int ldo, hinv_solve_info* info);

/* ---- prior (Sec. 5.1, Sec. 2.3, Sec. 4.3.1) ------------------------------- */
/* y = R x and y = R^{-1} x, column by column (all nrhs at once). */
int hinv_prior_apply(hinv_problem* p, int nrhs, const double* x, int ldx, double* y, int ldy);
int hinv_prior_solve(hinv_problem* p, int nrhs, const double* x, int ldx, double* y, int ldy,
                     hinv_solve_info* info);
/* y = R x exactly as hinv_prior_apply, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): the call allocates nothing.  Its intermediate vectors live in a
 * fixed scratch array of 8 388 608 doubles (64 MiB) that the library holds on
 * every GPU it runs on until the process ends (its address is looked up when
 * a context is created on that GPU).  Limit: 6 n nrhs <= 8 388 608, e.g.
 * nrhs <= 1 at N = 1024, 5 at N = 512, 21 at N = 256; larger calls return
 * HINV_EINVAL and write nothing.  Every scratch element is written before it
 * is read, so nothing carries over from earlier calls.  All calls on one GPU
 * share the array: calls that overlap in time on one GPU (other streams,
 * contexts or host threads) race and give undefined results. */
int hinv_prior_apply_noalloc(hinv_problem* p, int nrhs, const double* x, int ldx, double* y, int ldy);
/* out[:,s] = m_pr + K_A^{-1} C_M eta[:,s]: a draw from N(m_pr, R^{-1}).
 * eta: device, ns columns of 6 N^2 i.i.d. N(0,1) values with leading dimension
 * ldeta; entry 3 t + e sits at the midpoint of edge e of triangle t, edges
 * e0 = (a, r), e1 = (r, b), e2 = (a, b) with r the right-angle vertex. */
int hinv_prior_sample(hinv_problem* p, int ns, const double* eta, int ldeta, double* out, int ldo,
                      hinv_solve_info* info);

/* White noise for prior and posterior draws, generated on the device:
 * eta[:, s] (ns columns of 6 N^2 N(0,1) values, leading dimension ld) for the
 * samples first .. first+ns-1.  Philox4x64-10 (Salmon et al., SC'11) keyed by
 * (seed, stream); sample S uses the stream words [S L, (S+1) L), L = 6 N^2,
 * word w coming from counter block w / 4 + 1; Box-Muller on each word pair
 * (w0, w1): u1 = ((w0 >> 11) + 1) 2^-53, u2 = (w1 >> 11) 2^-53,
 * sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2).  Any sample can be drawn alone. */
int hinv_white_noise(hinv_problem* p, uint64_t seed, uint64_t stream, int64_t first, int ns,
                     double* eta, int ld);

/* ---- MAP point (Alg. 1) ---------------------------------------------------- */
/* m0 may be NULL (start from m_pr).  opts may be NULL (defaults).  On return
 * the problem is linearized at m_map. */
int hinv_map_newton(hinv_problem* p, const double* m0, double* m_map,
                    const hinv_newton_opts* opts, hinv_newton_info* info);

/* ---- low-rank posterior (Alg. 2, Alg. 4) --------------------------------- */
/* Double-pass randomized eigensolver for H_misfit v = lambda R v at the current
 * linearization point.  omega: device n x s block (s = k + oversampling).
 * mode: HINV_HESS_MISFIT or HINV_HESS_GN_MISFIT.  tprod: HINV_TPROD_*.
 * lambda: HOST array [k] (descending); V: device n x k, R-orthonormal.
 * A block Y = R^-1 A omega of numerical rank r < s (e.g. the Gauss-Newton
 * Hessian, of rank <= q, probed with s > q vectors, or a zero column in
 * omega) is orthonormalized on its r leading directions (eigendecomposition
 * of Y^T Y, directions below 100 rtol^2 of the largest dropped) and the
 * second pass runs on r columns.  Errors: HINV_EINVAL unless
 * 1 <= k <= s <= min(512, n); HINV_EBREAK when r < k or a Cholesky factor
 * still meets a non-positive pivot; lambda and V are then not written, and
 * the problem stays usable. */
int hinv_lowrank_eig(hinv_problem* p, int mode, int tprod, int s, const double* omega, int ldo,
                     int k, double* lambda_host, double* V, int ldv, hinv_solve_info* info);
/* Single-pass randomized eigensolver for H_misfit v = lambda R v (Alg. 3): one
 * pass of the Hessian over omega (n x s), Y = R^-1 H omega, PreCholQR of Y
 * (Alg. 4) giving Q (Q^T R Q = I) and Qbar = R Q; T is the least-squares
 * solution over symmetric s x s matrices of T (Qbar^T omega) = Qbar^T Y in the
 * Frobenius norm (Eq. eq:Tsinglepass), computed from its normal equations in
 * the eigenbasis of W W^T, W = Qbar^T omega; T = S Lambda S^T, V = Q S_k.
 * s Hessian actions instead of the double pass's 2 s, less accurate where the
 * spectrum beyond s is not negligible.  Arguments, layout and errors as in
 * hinv_lowrank_eig (FP64 block products; W must be nonsingular, which a
 * Gaussian omega gives with probability one). */
int hinv_lowrank_eig_single(hinv_problem* p, int mode, int s, const double* omega, int ldo, int k,
                            double* lambda_host, double* V, int ldv, hinv_solve_info* info);

/* Pointwise variance of the prior (Sec. 4.4.1, Eq. eq:prior_mvar): diag[n]
 * (device) = sum_i mu_i vbar_i (.) vbar_i, the (mu_i, vbar_i) being the s
 * eigenpairs of R^-1 from Alg. 2 with A = R^-1, B = I and no oversampling
 * (2 s prior solves).  omega: device n x s Gaussian block (ld ldo); mu_host:
 * HOST [s] (descending) or NULL.  Errors: HINV_EINVAL unless
 * 1 <= s <= min(512, n); HINV_EBREAK if Y = R^-1 omega has rank below s. */
int hinv_prior_variance(hinv_problem* p, int s, const double* omega, int ldo, double* diag, double* mu_host,
                        hinv_solve_info* info);

/* Pointwise variance of the Laplace posterior (Sec. 4.4.2, Eq. eq:post_mvar):
 * diag[n] = prior_diag - sum_i lambda_i / (1 + lambda_i) v_i (.) v_i with the
 * eigenpairs of hinv_lowrank_eig (lambda: HOST [k]; V: device n x k, ld ldv;
 * prior_diag, diag: device [n], may alias).  HINV_ENEGEIG if some
 * lambda_i <= -1.  Synchronizes the stream. */
int hinv_posterior_variance(hinv_problem* p, const double* prior_diag, int k, const double* lambda_host,
                            const double* V, int ldv, double* diag);

/* out[:,j] = m_map + (I - V S V^T R) x_j with x_j = K_A^{-1} C_M eta[:,j] and
 * S = diag(1 - (1 + lambda)^{-1/2}) (Eq. eq:sample_post).  lambda: HOST [k]. */
int hinv_posterior_sample(hinv_problem* p, const double* m_map, int k, const double* lambda_host,
                          const double* V, int ldv, int ns, const double* eta, int ldeta,
                          double* out, int ldo, hinv_solve_info* info);

/* The same samples with their white noise drawn on the device: sample j of
 * the call is sample first + j of the counter-based stream (seed, stream) of
 * hinv_white_noise, so any range of samples can be drawn alone and equals the
 * corresponding columns of a larger call.  The noise is generated and used in
 * internal chunks of up to 256 samples (6 N^2 x 256 doubles of workspace,
 * 12.9 GB at N = 1024); R V is formed once per call.  out: device n x ns,
 * ld ldo.  Errors as in hinv_posterior_sample. */
int hinv_posterior_sample_seeded(hinv_problem* p, const double* m_map, int k, const double* lambda_host,
                                 const double* V, int ldv, uint64_t seed, uint64_t stream, int64_t first, int ns,
                                 double* out, int ldo, hinv_solve_info* info);

/* ---- batches of independent inversions ------------------------------------ */
/* Many independent problems (own mesh size N_i, prior gamma_i / delta_i / beta_i,
 * observations and linearization point) whose Hessian actions and double
 * passes advance together.  Problems of one mesh size share a stacked
 * multigrid hierarchy: every solve of a Hessian action (two per column, App. A)
 * and every prior solve runs once per mesh size with the columns of all its
 * problems in one multi-right-hand-side PCG.  The solver settings are those of
 * probs[0], with the smallest rtol and largest max_iter of all members.
 * The problems must stay alive, on this context, while the batch exists; a
 * problem may appear once.  Columns per mesh size (members x nrhs, or
 * members x s) are limited to 4096. */
int hinv_batch_create(hinv_ctx* ctx, int nprob, hinv_problem* const* probs, hinv_batch** out);
int hinv_batch_destroy(hinv_batch* b);
/* out[i] (device, n_i x nrhs, leading dimension n_i) = H_i mhat[i] for every
 * problem i, at its current linearization point (HINV_ESTATE if a problem is
 * not linearized).  mhat, out: HOST arrays of nprob device pointers.  Modes as
 * in hinv_hessian_apply (Sec. 4.1, App. A). */
int hinv_batch_hessian_apply(hinv_batch* b, int mode, int nrhs, const double* const* mhat,
                             double* const* out, hinv_solve_info* info);
/* Double pass (Alg. 2 with Alg. 4) for every problem with s probe vectors and
 * rank k: omega[i] (device, n_i x s, ld n_i), V[i] (device, n_i x k, ld n_i),
 * lambda_host (HOST, nprob x k, row i = problem i, descending).  Mode and
 * tprod as in hinv_lowrank_eig.  HINV_EBREAK if any member's PreCholQR breaks
 * down; lambda_host and V are then unspecified (the mesh-size groups run one
 * after another and the call stops at the failing one). */
int hinv_batch_lowrank_eig(hinv_batch* b, int mode, int tprod, int s, const double* const* omega,
                           int k, double* lambda_host, double* const* V, hinv_solve_info* info);

/* ---- state operator at the linearization point ------------------------------ */
/* y = A(m) x restricted to the free rows (zero on the Dirichlet rows y = 0, 1):
 * the stiffness of the weak form (Sec. 5.1) with coefficient e^m, m the
 * linearization point.  Device, column-major, ld >= n. */
int hinv_state_apply(hinv_problem* p, int nrhs, const double* x, int ldx, double* y, int ldy);
/* A(m) x = b on the free rows (Dirichlet entries of x are zero) by multigrid
 * PCG with the problem's precision and tolerance. */
int hinv_state_solve(hinv_problem* p, int nrhs, const double* b, int ldb, double* x, int ldx,
                     hinv_solve_info* info);

typedef struct hinv_fcg_info {
    int status;               /* HINV_OK or HINV_ENOCONV */
    int iterations;           /* flexible-CG iterations */
    int fallback;             /* 1: stalled, multigrid PCG finished the solve */
    int fallback_iterations;  /* PCG iterations of the fallback */
    double relres;            /* final |b - A x| / |b| (recomputed) */
} hinv_fcg_info;

/* Flexible CG (Notay, SIAM J. Sci. Comput. 2000) on A(m) x = b, one
 * right-hand side, FP64: each new direction is A-orthogonalized against the
 * last `truncation` directions (1..32).  Preconditioner: one multigrid V-cycle
 * z = V(r), and when net is not NULL the network's correction of the residual
 * t = r - A z that the V-cycle leaves, c = s y(t / s, m, mask) with s the rms
 * of t, added at the step that minimizes the A-norm of the remaining error:
 * z += omega c, omega = c^T t / c^T A c (skipped unless positive).  Less than a 10x residual drop over 20 iterations hands the rest to
 * multigrid PCG.  b, x: device vectors of length n. */
int hinv_state_solve_fcg(hinv_problem* p, hinv_cnn* net, const double* b, double* x, double rtol,
                         int max_iter, int truncation, hinv_fcg_info* info);

/* ---- learned correction: residual CNN ------------------------------------- */
/* Six 3x3 convolutions with zero padding (3 -> 32, four residual 32 -> 32 with
 * ReLU, 32 -> 1), BF16 weights and activations on the matrix cores, FP32
 * accumulation, FP32 master parameters and Adam (beta 0.9 / 0.999, eps 1e-8).
 * Parameters are packed per layer as W[c_out][c_in][3][3] then b[c_out]; a new
 * network has all parameters zero. */
int hinv_cnn_create(hinv_ctx* ctx, hinv_cnn** out);
int hinv_cnn_destroy(hinv_cnn* net);
int hinv_cnn_param_count(void);
int hinv_cnn_set_params(hinv_cnn* net, const float* host, int count); /* resets Adam */
int hinv_cnn_get_params(hinv_cnn* net, float* host, int count);
/* in: device FP32 [B][3][S][S] (channel, row, column); out: device FP32 [B][S][S]. */
int hinv_cnn_forward(hinv_cnn* net, int B, int S, const float* in, float* out);
/* Loss and its gradient; grad_host (HOST, may be NULL) receives the gradient in
 * the packed layout.  tchan = 1: target device FP32 [B][S][S], loss = mean over
 * the batch of |y - t|^2 / |t|^2.  tchan = 4: target [B][4][S][S] =
 * (t, wE, wN, diag), loss = mean of d^T A d / t^T A t with d = (y - t) on the
 * free nodes (input channel 2) and A the 5-point stencil with east / north
 * edge weights wE, wN and diagonal diag (neighbours outside the image zero). */
int hinv_cnn_gradient(hinv_cnn* net, int B, int S, const float* in, const float* target, int tchan,
                      double* loss, float* grad_host);
/* gradient and one Adam step with learning rate lr; loss before the step. */
int hinv_cnn_train_step(hinv_cnn* net, int B, int S, const float* in, const float* target, int tchan,
                        float lr, double* loss);
/* npairs training pairs from the problem's incremental forward solves at its
 * linearization point (App. A): b = -C(u) mhat for random mhat, x_k after
 * k = 0..7 multigrid-PCG iterations, r = b - A x_k, r' = r - A V(r),
 * e' = A^-1 r'.  Each pair is cut to a crop x crop window at a seeded position
 * and scaled by the rms s of r' there: in[i] = (r' / s, m, free mask)
 * (device FP32 [npairs][3][crop][crop]), target[i] = (e' / s, wE, wN, diag)
 * ([npairs][4][crop][crop]: the stencil of A(m) on the window, for the energy
 * loss). */
int hinv_cnn_harvest(hinv_problem* p, int npairs, uint64_t seed, int crop, float* in, float* target,
                     hinv_solve_info* info);

#ifdef __cplusplus
}
#endif
#endif /* HINV_H */
