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
  IMSMG_ERR_NOT_SPD = -4,      /* block / coarse factorization or CG breakdown (p.Ap <= 0) */
  IMSMG_ERR_NOT_CONVERGED = -5,/* max_iter reached; x holds the last iterate */
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
 * idx[ptr[j] .. ptr[j+1]), sorted compact indices. */
typedef struct {
  int32_t nblocks;
  const int32_t *ptr;
  const int32_t *idx;
} imsmg_patches;

/* Element incidence of one level (host arrays, optional): for every active
 * element e the compact indices of the active functions non-zero on it,
 * eidx[eptr[e] .. eptr[e+1]).  Used for N_K in gamma = 1 / max_K N_K. */
typedef struct {
  int32_t nelements;
  const int32_t *eptr;
  const int32_t *eidx;
} imsmg_elements;

/* Function lattice of one level. */
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
  int32_t timing;      /* record HIP events around the finest-level residual kernel */
  double gamma;        /* > 0: uniform damping on all levels; <= 0: 1 / max_K N_K per level */
  int32_t compress;    /* 1: rows equal to the level's interior stencil (1e-14 relative) read that
                          stencil instead of their own values (default 1) */
} imsmg_options;

typedef struct {
  int32_t status;        /* IMSMG_OK or an error code */
  int32_t iterations;
  double rel_res;        /* ||r_k|| / ||r_0|| (recursive residual) */
  double true_rel_res;   /* ||b - A x|| / ||b|| recomputed at the end */
  double solve_ms;       /* wall time of the call */
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
 * removal rule), forms the smoother, the damping and the coarsest inverse. */
int imsmg_factor_patches(imsmg_ctx *ctx);

/* Post-removal blocks of level l: sizes first (ptr may be NULL to query). */
int imsmg_get_patches(imsmg_ctx *ctx, int level, int32_t *nblocks, int64_t *nnz, int32_t *ptr, int32_t *idx);
/* Damping factor of level l (1 / max_K N_K or the uniform override). */
int imsmg_get_gamma(imsmg_ctx *ctx, int level, double *gamma);

/* z = B r for the finest level (one V-cycle).  r, z: device, compact, FP64. */
int imsmg_vcycle(imsmg_ctx *ctx, const double *r_dev, double *z_dev);

/* Preconditioned CG from x (device; in: x0, out: solution) until
 * ||r_k|| <= rtol ||r_0|| and ||b - A x|| <= rtol ||b||. */
int imsmg_pcg_solve(imsmg_ctx *ctx, const double *b_dev, double *x_dev, double rtol, imsmg_info *info);

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
  int32_t reserved;
} imsmg_level_stats;
int imsmg_get_level_stats(imsmg_ctx *ctx, int level, imsmg_level_stats *stats);

/* Accumulated time of the finest-level residual kernel since the last reset
 * (requires opt.timing; the timed kernel is the finest level's fused residual +
 * trivial-row smoothing step): total milliseconds and number of launches. */
int imsmg_kernel_time(imsmg_ctx *ctx, double *total_ms, int64_t *launches, int reset);

const char *imsmg_last_error(imsmg_ctx *ctx);
int imsmg_destroy(imsmg_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
