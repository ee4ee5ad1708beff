/*
 * imsmg.h - C ABI of the MI355X (gfx950) solver library libimsmg.so.
 *
 * Solves the immersed system A x = b (eq:systemMulti: A symmetric positive
 * definite, A_ij = a_h(phi_i, phi_j)) by conjugate gradients preconditioned
 * with the multigrid V-cycle of Algorithm alg:MGV (the paragraph after the
 * algorithm: symmetric V-cycle as CG preconditioner).  The V-cycle uses
 *   - level operators A_l and restrictions R_l, prolongation R_l^T
 *     (eq:coarsening; Galerkin coarse operators per Remark rem:gridParamCorr),
 *   - additive Schwarz smoothing M^{-1} = sum_j P_j A_j^{-1} P_j^T over the
 *     given index blocks, damped by gamma = 1 / max_K N_K (eq:applyCS) or by
 *     per-block weights,
 *   - blocks factorized with the tiny-eigenvalue removal of the smoothers
 *     subsection (eigenvalue below 1e-16 x largest diagonal entry: the
 *     dominant function of that eigenvector leaves the block),
 *   - a direct solve on the coarsest level (Algorithm alg:MGV, l = 1).
 *
 * Call order: imsmg_create -> imsmg_setup -> [imsmg_set_patch_weights]
 *             -> imsmg_factor_patches -> (imsmg_vcycle | imsmg_pcg_solve)*
 *             -> imsmg_destroy.   A new setup invalidates the factorization.
 *
 * Levels are numbered 0 (coarsest) .. nlevels-1 (finest).  On every level the
 * active functions are numbered in ascending lattice index (x fastest); CSR
 * columns are sorted; the CSR pattern of A_l must lie inside the stencil
 * (|lattice offset| <= reach per axis).
 *
 * Memory: every array passed to imsmg_setup is a HOST array and is copied;
 * the caller may free it on return.  Vectors passed to imsmg_vcycle,
 * imsmg_pcg_solve and the imsmg_apply_* calls are DEVICE pointers (FP64,
 * compact numbering of the level) owned by the caller, on the context's
 * device; the library never frees caller memory.  Work is ordered on the
 * context's stream and every call returns after it has completed.
 *
 * Errors: every call returns IMSMG_OK (0) or a negative code;
 * imsmg_last_error(ctx) describes the last failure.  A context must not be
 * used by two threads at once.
 */
#ifndef IMSMG_H
#define IMSMG_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  IMSMG_OK = 0,
  IMSMG_ERR_INVALID_ARG = -1,  /* shape, pointer or ordering mismatch */
  IMSMG_ERR_OOM = -2,
  IMSMG_ERR_HIP = -3,          /* a HIP runtime call failed */
  IMSMG_ERR_NOT_SPD = -4,      /* non-positive operator diagonal (setup), block / coarse factorization, or CG breakdown (p.Ap <= 0) */
  IMSMG_ERR_NOT_CONVERGED = -5,/* true relative residual above rtol at the end; x holds the last iterate */
  IMSMG_ERR_NAN = -6,          /* NaN / Inf met in the iteration */
  IMSMG_ERR_STATE = -7         /* call out of order (e.g. solve before factor) */
};

enum { IMSMG_FP64 = 0, IMSMG_MIXED = 1 };

typedef struct imsmg_ctx imsmg_ctx;

/* CSR matrix (host arrays). */
typedef struct {
  int32_t nrows, ncols;
  int64_t nnz;
  const int32_t *rowptr; /* nrows + 1 */
  const int32_t *col;    /* nnz, sorted per row */
  const double *val;     /* nnz */
} imsmg_csr;

/* Schwarz index blocks of one level (host arrays): block j is
 * idx[ptr[j] .. ptr[j+1]), sorted compact indices.
 * colour (optional, may be NULL): colour of every block in [0, 4096) for the
 * multiplicative smoother (smoothers subsection, "Multiplicative Schwarz":
 * blocks of one colour must not share an element, so they are applied
 * together and the residual is updated once per colour).  Setup checks, on
 * the element incidence, that no two blocks of one colour share an active
 * element (IMSMG_ERR_INVALID_ARG otherwise).  NULL: blocks are coloured
 * greedily in block order (smallest colour unused on their elements).
 * Singleton blocks that the factorization adds for DOFs left in no block take
 * the smallest colour >= max(colour) + 1 unused on their elements. */
typedef struct {
  int32_t nblocks;
  const int32_t *ptr;
  const int32_t *idx;
  const int32_t *colour;
} imsmg_patches;

/* Element incidence of one level (host arrays, optional): for every active
 * element e the compact indices of the active functions non-zero on it,
 * eidx[eptr[e] .. eptr[e+1]).  Used for N_K in gamma = 1 / max_K N_K.
 * The per-block damping features also need, per active element, its lattice
 * index elem[e] (x fastest over shape = elements per axis) and its volume
 * fraction eta[e] = |K cap Omega| / |K| in [0, 1] (NULL: all 1). */
typedef struct {
  int32_t nelements;
  const int32_t *eptr;
  const int32_t *eidx;
  int32_t shape[3];      /* elements per axis (unused axes: 1); read when elem != NULL */
  const int32_t *elem;   /* nelements lattice indices, or NULL */
  const double *eta;     /* nelements volume fractions, or NULL */
} imsmg_elements;

/* Function lattice of one level.
 *
 * dof_to_lattice == NULL makes the level a general sparse level: no function
 * lattice and no common stencil (locally refined discretizations: truncated
 * hierarchical B-splines of Figure fig:THB on meshes coarsened by Algorithm
 * alg:coarsen).  Its operator is kept as CSR with any pattern (columns
 * sorted and unique, positive diagonal), R and R^T as sparse rows, and the
 * smoother's blocks and element incidence as given; dim, shape, reach and
 * two_scale are ignored (two_scale must be NULL).  Either every level of a
 * setup is general or none is.  General levels support the additive and
 * the multiplicative smoother (colours: as given with the blocks, else
 * greedy from the element incidence), diagonal coarse smoothing, V and W
 * cycles, FP64 and mixed precision, single right-hand sides; learned
 * weights, block_gemm and the multi-column and batched calls return
 * IMSMG_ERR_INVALID_ARG. */
typedef struct {
  int32_t dim;                  /* 2 or 3 */
  int32_t shape[3];             /* functions per axis (unused axes: 1) */
  int32_t reach;                /* stencil half width (B-splines and Lagrange: degree p) */
  const int32_t *dof_to_lattice;/* nrows, strictly increasing (host) */
  /* Optional (may be NULL): the 1D two-scale matrix of R_l when R_l is the
   * tensor product of one 1D matrix restricted to active rows and columns
   * (eq:coarsening on a tensor grid).  Dense row-major, rows = functions per
   * axis of level l-1, cols = shape[0] of this level.  When given, setup
   * checks it against the CSR R_l entry by entry and then applies R_l and
   * R_l^T without stored indices or values. */
  const double *two_scale;
} imsmg_lattice;

typedef struct {
  int32_t precision;   /* IMSMG_FP64 or IMSMG_MIXED (FP32 V-cycle operators, FP64 CG) */
  int32_t nu_pre;      /* smoothing steps before / after the coarse correction (>= 1) */
  int32_t nu_post;
  int32_t max_iter;    /* CG iteration cap */
  int32_t check_every; /* host reads the convergence flag every this many iterations */
  int32_t use_graph;   /* replay each block of check_every iterations as one hipGraph */
  int32_t timing;      /* 0: off; n >= 1: record HIP events around each plain smoothing step of the
                          finest level, whose kernel (fused residual + trivial rows) is launched
                          n times back to back inside the event pair (the step reads x_a and r
                          and writes x_b and rh only, so the repeats leave the same result;
                          n > 1 spreads the events' own overhead over n launches); at most 64 */
  double gamma;        /* > 0: uniform damping on all levels; <= 0: 1 / max_K N_K per level */
  int32_t compress;    /* 1: rows equal to the level's interior stencil (1e-14 relative) read that
                          stencil instead of their own values (default 1) */
  int32_t use_learned; /* 1: imsmg_factor_patches damps every block of every level without given
                          weights by the loaded damping network (imsmg_load_mlp), subject to the
                          stability check and to the iteration judge (the weights are kept only
                          if PCG on a fixed probe needs fewer iterations than with gamma);
                          2: the same without the judge; default 0 */
  int32_t autotune;    /* 1: imsmg_factor_patches times the general-row smoother with 2, 4 and 8
                          lanes per row on each level (HIP events, a few launches each) and keeps
                          the fastest; 0: 4 lanes.  The lane count fixes the summation order of
                          that product, so contexts tuned differently round differently (each
                          context stays bitwise reproducible); default 0 */
  int32_t block_gemm;  /* general Schwarz blocks in the multi-right-hand-side solve
                          (imsmg_vcycle_multi, imsmg_pcg_solve_multi): 0 the assembled FP64
                          CSR product (default); 1 one patch GEMM W_j R_j per block on the
                          matrix cores with FP64 operands; 2 the same with BF16 operands and
                          FP32 accumulation.  1 and 2 apply on levels whose general blocks all
                          have <= 16 functions (others keep 0); the single-column solve always
                          uses 0 */
  int32_t flexible_cg; /* 1: imsmg_pcg_solve takes beta_k = (r_{k+1}.z_{k+1} - r_{k+1}.z_k) / (r_k.z_k)
                          (Polak-Ribiere form, robust to a preconditioner that changes between
                          iterations; one more dot product, reduced inside the update kernel);
                          0: beta_k = r_{k+1}.z_{k+1} / (r_k.z_k) (default).  The two agree in
                          exact arithmetic for the fixed SPD V-cycle.  The multi-column and
                          batched solves use 0 and reject 1 */
  int32_t smoother;    /* finest level: IMSMG_ADDITIVE (default; additive Schwarz damped by gamma or
                          the block weights) or IMSMG_MULTIPLICATIVE (multiplicative Schwarz,
                          eq:multiplicativeSchwarz1, colour by colour: forward colour order before
                          the coarse correction, reversed after it; undamped).  With blocks of one
                          function each (passed by the caller) these are Jacobi and Gauss-Seidel */
  int32_t coarse_smoother; /* the levels between the finest and the coarsest: -1 (default) as
                          `smoother`, else IMSMG_ADDITIVE or IMSMG_MULTIPLICATIVE.  Remark
                          rem:coarseGS: diagonal smoothers suffice there (pass one-function blocks
                          for those levels).  The multi-column and batched solves, per-block
                          weights and use_learned need the additive smoother on every level */
  int32_t cycle;       /* 1: V-cycle (Algorithm alg:MGV, default); 2: W-cycle (two coarse cycles
                          on every level above level 1, the second on the residual of the first) */
  int32_t flag_min_rows; /* levels with at least this many rows read the solve's convergence flag
                          in every kernel (skip the tail of a graph replay after convergence);
                          smaller levels do not (one dependent load less); default 65536 */
  int32_t ncomp;       /* components per lattice function: 1 (scalar problems, default) or 3 (3D
                          linear elasticity, eq:weakMulti with a displacement vector).  With ncomp
                          > 1 every level's unknowns are component-major, DOF c N + i = component
                          c of the level's lattice function i (N = operator size / ncomp; the
                          lattice's dof_to_lattice lists the N functions); the CSR holds every
                          component pair; R_l is block diagonal with one equal block per
                          component; every Schwarz block holds DOFs of one component (the
                          smoothers subsection's separate blocks per component); elements list
                          the DOFs of every component.  Supported: additive and multiplicative
                          Schwarz, V- or W-cycles, FP64 or FP32 level operators, single
                          right-hand side; rejected (IMSMG_ERR_INVALID_ARG): learned weights,
                          block_gemm, the multi-column and batched calls, 2D lattices */
} imsmg_options;

enum { IMSMG_ADDITIVE = 0, IMSMG_MULTIPLICATIVE = 1 };

typedef struct {
  int32_t status;        /* IMSMG_OK or an error code */
  int32_t iterations;
  double rel_res;        /* ||r_k|| / ||r_0|| (recursive residual) */
  double true_rel_res;   /* ||b - A x|| / ||b|| recomputed at the end */
  double solve_ms;       /* wall time of the call */
  int32_t restarts;      /* CG restarts after a true-residual check above rtol */
  int32_t fallback_flags;/* bit l: level l kept gamma although use_learned asked for the network
                            (stability check or cost judge rejected its weights) */
  double setup_ms;       /* wall time of the last imsmg_setup on this context */
  double factor_ms;      /* wall time of the last imsmg_factor_patches */
} imsmg_info;

/* Fills opt with the defaults (FP64, V(1,1), max_iter 500, check_every 4, graph on, compress on). */
void imsmg_default_options(imsmg_options *opt);

/* Creates a context on HIP device `device`.  stream: a hipStream_t to order
 * work on, or NULL for a library-owned stream. */
int imsmg_create(imsmg_ctx **out, int device, void *stream);

/* Copies the hierarchy to the device.  A[nlevels], R[nlevels] (R[0] ignored;
 * R[l] is n_{l-1} x n_l and maps level l to level l-1), P[nlevels] (P[0]
 * ignored), L[nlevels]; E may be NULL (then opt->gamma must be > 0). */
int imsmg_setup(imsmg_ctx *ctx, int nlevels, const imsmg_csr *A, const imsmg_csr *R, const imsmg_patches *P,
                const imsmg_lattice *L, const imsmg_elements *E, const imsmg_options *opt);

/* Optional per-block damping weights of level l (host array, nblocks, > 0).
 * Replaces gamma on that level; blocks added by the factorization (DOFs left
 * without a block) take the level's gamma.  Call before imsmg_factor_patches. */
int imsmg_set_patch_weights(imsmg_ctx *ctx, int level, const double *omega);

/* Factorizes every block on the device (FP64 Jacobi eigensolver with the
 * removal rule), forms the smoother, the damping and the coarsest inverse.
 * With opt.use_learned, every level l >= 1 without given weights then takes
 * omega_j = gamma_l exp(clip(o_j, -3, 3)) from the damping network on the
 * block features; the weights are kept only if a 60-step power iteration
 * finds lambda_max(S_omega A_l) < 2 (1 - 0.05) (the stability condition
 * eq:stabilityMulti keeps I - S A a contraction).  On a first failure all
 * weights of the level are scaled by 1.8 / lambda_max and checked again; on a
 * second the level falls back to gamma_l (imsmg_get_patch_weights reports
 * which).  With use_learned = 1 the uniform smoother then judges the cost:
 * PCG on the probe b = A v (v_i = 1 + sin(0.7 i + 0.3) / 2 + cos(1.9 i) / 4,
 * x0 = 0, rtol 1e-8) runs once with gamma on every level and once with the
 * kept network weights; unless the network needs fewer iterations, every
 * level returns to gamma (learned_status -2). */
int imsmg_factor_patches(imsmg_ctx *ctx);

/* ---- several right-hand sides with the same matrix (nrhs = 1 .. 16) ----
 * B, X, R, Z: device, compact numbering of the finest level, column-major
 * n x nrhs (column k at offset k * n).  Internally the columns are
 * interleaved on the lattice (4, 8 or 16 wide, unused columns zero) so that
 * every stencil row, block row and transfer coefficient is read once for all
 * columns. */

/* Z = B R column by column (one V-cycle). */
int imsmg_vcycle_multi(imsmg_ctx *ctx, int nrhs, const double *R_dev, double *Z_dev);

/* nrhs independent PCG solves A x_k = b_k sharing every kernel launch; CG
 * scalars, stopping test (||r_k|| <= rtol min(||r_k,0||, ||b_k||)),
 * true-residual restarts (as imsmg_pcg_solve; columns already below rtol stay
 * converged) and iteration counts are per column (a converged column stops
 * moving while the others continue); the call returns when every column has
 * converged or on the first error.  infos: nrhs entries (may be NULL);
 * solve_ms is the wall time of the call.  Returns IMSMG_ERR_NOT_CONVERGED
 * when some column ends above rtol (that column's info.status says so, the
 * others' are 0), IMSMG_ERR_NAN / IMSMG_ERR_NOT_SPD for the whole call. */
int imsmg_pcg_solve_multi(imsmg_ctx *ctx, int nrhs, const double *B_dev, double *X_dev, double rtol,
                          imsmg_info *infos);

/* ---- batched problems.  A fresh context becomes a batch context holding
 * nprob independent problems; each gets its own device context and stream
 * (created on the batch context's device), the per-problem arguments are
 * those of imsmg_setup (E may be NULL, or E[p] NULL per problem).  The
 * library owns the children: imsmg_destroy(ctx) destroys them.  Errors name
 * the problem.  imsmg_factor_patches(ctx) factorizes every problem. */
int imsmg_setup_batched(imsmg_ctx *ctx, int nprob, const int *nlevels, const imsmg_csr *const *A,
                        const imsmg_csr *const *R, const imsmg_patches *const *P, const imsmg_lattice *const *L,
                        const imsmg_elements *const *E, const imsmg_options *opt);
/* The context of problem p of a batch (owned by the batch; for per-problem
 * queries such as imsmg_get_level_stats). */
int imsmg_batch_problem(imsmg_ctx *ctx, int p, imsmg_ctx **child);
/* nrhs systems per problem: B_dev[p], X_dev[p] are device arrays n_p x nrhs
 * (column k at offset k n_p) as in imsmg_pcg_solve_multi; infos (may be NULL)
 * holds nprob * nrhs entries, problem-major.  nthreads host threads (<= 0: 4)
 * each take the next unsolved problem and drive its multi-column solve on the
 * problem's stream, so the problems' latency-bound V-cycles overlap on the
 * device.  Results do not depend on nthreads (no state is shared).  Returns
 * IMSMG_OK or the first error. */
int imsmg_pcg_solve_batched(imsmg_ctx *ctx, int nrhs, const double *const *B_dev, double *const *X_dev, double rtol,
                            imsmg_info *infos, int nthreads);

/* ---- per-block damping (an extension: the paper uses one factor per level,
 * see the discussion after eq:applyCS).  "Final blocks" are the blocks after
 * factorization: the input blocks in input order (members removed by the
 * removal rule dropped, possibly empty) followed by singletons for DOFs left
 * in no block; imsmg_get_patches lists them. */

/* Copies the damping network's 5313 FP32 parameters (host) to the device:
 * W1 (64 x 16, row-major), b1 (64), W2 (64 x 64, row-major), b2 (64),
 * w3 (64), b3 (1); o = w3 . relu(W2 relu(W1 x + b1) + b2) + b3. */
int imsmg_load_mlp(imsmg_ctx *ctx, const float *params, int64_t nparams);

/* Features of the final blocks of level l >= 1 after imsmg_factor_patches
 * (host, nblocks x 16 row-major; feat may be NULL to query nblocks).  Needs
 * the element arrays with elem and eta.  For final block j with input block
 * B (the block itself for added singletons), support S = union of the
 * active elements of B's members, K = (2p+1)^d, E = (p+1)^d, p = reach:
 *   0 |j| / K            1 |B| / K            2 |S| / E
 *   3 sum_S eta / E      4 log10(max(min_S eta, 1e-16)) / 16
 *   5 mean over cut elements of S (eta < 1 - 1e-12) of log10(max(eta, 1e-16)) / 16 (0 if none)
 *   6 max_S N_K / E      7 mean_S N_K / E
 *   8 log10(lambda_max / lambda_min) / 16 of the final block (0 below size 2)
 *   9 log10(max(lambda_min / max diag, 1e-30)) / 16 of the input block
 *  10 (|B| - |j|) / K (0 for added singletons)
 *  11 fraction of j's functions with a cut element in their support
 *  12-14 offset per axis of the eta-weighted mean element index of S from its
 *        unweighted mean, / (p + 1) (0 on unused axes)
 *  15 fraction of the level's active elements that are cut (eta < 1 - 1e-12) */
int imsmg_get_patch_features(imsmg_ctx *ctx, int level, int32_t *nblocks, float *feat);

/* Current weight of every final block of level l (host, may be NULL),
 * learned_status 1 = network weights accepted, -1 = rejected by the stability
 * check (gamma used), -2 = rejected by the iteration judge (gamma used),
 * 0 = gamma or given weights; lambda_max = the stability
 * check's estimate (0 if it did not run).  Pointers other than nblocks may be NULL. */
int imsmg_get_patch_weights(imsmg_ctx *ctx, int level, int32_t *nblocks, double *omega, int32_t *learned_status,
                            double *lambda_max);

/* Replaces the weights of the final blocks of level l (host, nblocks, > 0)
 * of a factorized hierarchy without refactorizing (no stability check). */
int imsmg_set_block_weights(imsmg_ctx *ctx, int level, const double *omega);

/* Power-iteration estimate (iters steps, Rayleigh quotient in the A inner
 * product, increasing towards the limit) of lambda_max(S A_l), level l >= 1. */
int imsmg_lambda_max(imsmg_ctx *ctx, int level, int iters, double *lambda_max);

/* Two-grid objective of a factorized TWO-level hierarchy (level 1 smoothed,
 * level 0 solved exactly), with the current weights of level 1:
 *   E = (I - S A)(I - R^T A_0^{-1} R A)(I - S A)   (eq:eigenMulti, one smoothing step each side),
 *   J = tr((E^k Z)^T A E^k Z) / tr(Z^T A Z)   (energy norm, in which E is self-adjoint),
 * Z: host, n_1 x m column-major (compact level-1 numbering).  grad (host,
 * nblocks final blocks of level 1, may be NULL) receives dJ/domega_j by the
 * adjoint recursion.  FP64 throughout. */
int imsmg_two_grid_objective(imsmg_ctx *ctx, int m, const double *Z, int k, double *J, double *grad);

/* Stand-alone network kernels (device pointers, ordered on `stream`, a
 * hipStream_t or NULL; asynchronous).  X: n x 16 row-major FP32.
 *   forward:   out[i] = o(X_i)
 *   loss_grad: loss = mean_i (o(X_i) - t_i)^2 and its gradient (5313), with a
 *              caller-owned device workspace of imsmg_mlp_workspace_bytes(n) bytes
 *              (sums in a fixed order: deterministic)
 *   adam:      one Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected; step >= 1)
 * Return IMSMG_ERR_INVALID_ARG on bad arguments, IMSMG_ERR_HIP on a launch error. */
int64_t imsmg_mlp_workspace_bytes(int n);
int imsmg_mlp_forward(void *stream, const float *params, const float *X, int n, float *out);
int imsmg_mlp_loss_grad(void *stream, const float *params, const float *X, const float *t, int n, void *work,
                        float *loss, float *grad);
int imsmg_mlp_adam(void *stream, float *params, const float *grad, float *m, float *v, int step, float lr);

/* For callers that cannot allocate device memory (work under HIP graph
 * capture, tight training or serving loops, harnesses that forbid hipMalloc):
 * imsmg_mlp_loss_grad without the caller's workspace.  The workspace is a
 * static device array inside the library, 9.4 MiB per GPU for at most
 * IMSMG_NOALLOC_MAX_SAMPLES samples, held by every GPU the library runs on
 * until the process ends; its device address is looked up once per device on
 * the first call.  Same kernels, same arithmetic and summation order as
 * imsmg_mlp_loss_grad (results are bitwise equal).  The call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine).  All calls
 * on one GPU share that array: calls that overlap on one GPU (two streams, two
 * threads) race and must be serialized by the caller.  Nothing needs clearing
 * between calls (each call writes every workspace word it reads).
 * Errors: IMSMG_ERR_INVALID_ARG for n < 1, n > IMSMG_NOALLOC_MAX_SAMPLES or a
 * null pointer; IMSMG_ERR_HIP when the device or the array's address cannot
 * be obtained or the launch fails. */
#define IMSMG_NOALLOC_MAX_SAMPLES 8192
int imsmg_mlp_loss_grad_noalloc(void *stream, const float *params, const float *X, const float *t, int n,
                                float *loss, float *grad);

/* Post-removal blocks of level l: sizes first (ptr may be NULL to query). */
int imsmg_get_patches(imsmg_ctx *ctx, int level, int32_t *nblocks, int64_t *nnz, int32_t *ptr, int32_t *idx);
/* Colours of the post-removal blocks of level l (multiplicative Schwarz,
 * smoothers subsection): ncolours = number of colours, colour[nblocks] (may
 * be NULL to query); the order of imsmg_get_patches.  Defined on every
 * smoothed level (the additive smoother ignores them). */
int imsmg_get_patch_colours(imsmg_ctx *ctx, int level, int32_t *ncolours, int32_t *colour);
/* Damping factor of level l (1 / max_K N_K or the uniform override). */
int imsmg_get_gamma(imsmg_ctx *ctx, int level, double *gamma);

/* z = B r: one V-cycle of Algorithm alg:MGV on the finest level (x = 0, nu_pre
 * smoothing steps, residual, restriction, recursion, prolongation, nu_post
 * smoothing steps; direct solve on level 0).  r_dev, z_dev: caller-owned
 * device arrays of n_{L} FP64 (compact numbering of the finest level); r is
 * only read.  Errors: IMSMG_ERR_STATE before imsmg_factor_patches,
 * IMSMG_ERR_INVALID_ARG for a null pointer, IMSMG_ERR_HIP. */
int imsmg_vcycle(imsmg_ctx *ctx, const double *r_dev, double *z_dev);

/* Times one V-cycle as imsmg_vcycle runs it (residual staged once, then reps
 * cycles, each between two HIP events on the context's stream; with
 * opt.use_graph the cycle is one captured graph): median and mean in ms over
 * the reps (1 .. 100000).  The V-cycle throughput of the solve is
 * n_L / median.  Errors: IMSMG_ERR_STATE before imsmg_factor_patches,
 * IMSMG_ERR_INVALID_ARG for bad arguments or opt.timing != 0. */
int imsmg_vcycle_time(imsmg_ctx *ctx, const double *r_dev, int reps, double *median_ms, double *mean_ms);

/* CG preconditioned by the V-cycle (the paragraph after Algorithm alg:MGV).
 * b_dev: right-hand side, x_dev: x0 on entry and the solution on return, both
 * caller-owned device arrays of n_{L} FP64 (compact numbering of the finest
 * level).  Iterates until ||r_k|| <= rtol min(||r_0||, ||b||) (2-norm,
 * recursive residual; the two norms agree for x0 = 0), then recomputes
 * ||b - A x|| / ||b|| in FP64 and restarts CG from x (fresh direction) while
 * that is above rtol, at most three times (the first start's threshold and
 * iteration count are kept).  beta: opt.flexible_cg.  The iterations run as
 * captured graphs of opt.check_every iterations (opt.use_graph) with every CG
 * scalar on the device.  info (may be NULL): status, iterations, both
 * residuals, wall time.
 * Errors: IMSMG_ERR_STATE before imsmg_factor_patches; IMSMG_ERR_INVALID_ARG
 * for null vectors or rtol <= 0; IMSMG_ERR_NOT_SPD when p.Ap <= 0;
 * IMSMG_ERR_NOT_CONVERGED when the true relative residual is still above
 * rtol at the end (restarts used up or opt.max_iter iterations reached; x
 * holds the last iterate, info is filled); IMSMG_ERR_NAN; IMSMG_ERR_HIP. */
int imsmg_pcg_solve(imsmg_ctx *ctx, const double *b_dev, double *x_dev, double rtol, imsmg_info *info);

/* Multigrid as a standalone solver (the paragraph after Algorithm alg:MGV:
 * the cycle applied iteratively, x <- x + B (b - A x), B the factorized
 * cycle of the options: V or W, the configured smoothers and precision).
 * fmg != 0: the iteration starts from a full multigrid pass (nested
 * iteration, the FMG cycle named in the same paragraph): b restricted to
 * every level (r_{l-1} = R_l r_l), the coarsest level solved directly, every
 * finer level started from the prolongated coarser solution and improved by
 * one cycle of that level; the x passed in is then ignored.  fmg == 0: x
 * holds the start.  b_dev, x_dev: device, n of the finest level.  Stops when
 * ||b - A x|| <= rtol ||b|| (2-norm, FP64 operator) or after max_cycles
 * cycles (max_cycles = 0 with fmg: the FMG pass alone); x holds the last
 * iterate.  info->iterations = cycles after the start, rel_res =
 * true_rel_res = the final relative residual.  The residual norm is read on
 * the host after every cycle (one stream synchronization per cycle); the
 * first call with fmg != 0 allocates two vectors per level, which the context
 * keeps until imsmg_destroy.  Errors: STATE before factorization,
 * INVALID_ARG (null vector, rtol <= 0, max_cycles < 0), NOT_CONVERGED (rtol
 * not reached; x holds the last iterate, info is filled), NAN, HIP. */
int imsmg_mg_solve(imsmg_ctx *ctx, const double *b_dev, double *x_dev, double rtol, int max_cycles, int fmg,
                   imsmg_info *info);

/* Kernel-level entry points (device, compact vectors of the level). */
int imsmg_apply_operator(imsmg_ctx *ctx, int level, const double *x, double *y);   /* y = A_l x */
int imsmg_apply_smoother(imsmg_ctx *ctx, int level, const double *r, double *y);   /* y = S_l r */
int imsmg_apply_restriction(imsmg_ctx *ctx, int level, const double *rf, double *rc); /* rc = R_l rf */
int imsmg_apply_prolongation(imsmg_ctx *ctx, int level, const double *xc, double *xf); /* xf += R_l^T xc */
int imsmg_coarse_solve(imsmg_ctx *ctx, const double *r, double *x);               /* x = A_0^{-1} r */

/* Storage statistics of level l (after imsmg_factor_patches). */
typedef struct {
  int32_t n;             /* active rows */
  int32_t stencil;       /* K = (2 reach + 1)^dim slots per row */
  int32_t stored_rows;   /* rows keeping their own values; the others read the uniform stencil */
  int32_t general_rows;  /* rows in general (non-singleton or shared) Schwarz blocks */
  int64_t sg_nnz;        /* entries of the assembled general smoother on those rows */
  int64_t lattice;       /* padded lattice size of the level's vectors */
  int32_t value_bytes;   /* 8 (FP64) or 4 (FP32 V-cycle operators) */
  int32_t general_lanes; /* lanes per row of the general-row smoother (2, 4 or 8) */
  int32_t patch_gemm;    /* 1: the multi-right-hand-side smoother applies this level's general
                            blocks as patch GEMMs (options.block_gemm > 0, blocks <= 16) */
  int32_t bf16_blocks;   /* of those, the blocks with cond(A_j) <= 16, which take BF16 operands
                            when options.block_gemm == 2 (the others stay FP64) */
} imsmg_level_stats;
int imsmg_get_level_stats(imsmg_ctx *ctx, int level, imsmg_level_stats *stats);

/* Accumulated time of the finest-level residual kernel since the last reset
 * (requires opt.timing; the timed kernel is the finest level's fused residual +
 * trivial-row smoothing step): total milliseconds and number of launches
 * (opt.timing launches per timed step). */
int imsmg_kernel_time(imsmg_ctx *ctx, double *total_ms, int64_t *launches, int reset);

const char *imsmg_last_error(imsmg_ctx *ctx);
int imsmg_destroy(imsmg_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
