/*
 * imsmg_gen.h - native generator of immersed multigrid problems (host C++).
 *
 * Builds, for a synthetic workload, everything the solver library's setup
 * call consumes:
 *   - the fine system A x = b with A_ij = a_h(phi_i, phi_j), b_i = b_h(phi_i)
 *     (eq:systemMulti): the scalar analogue of eq:weakMulti / eq:operatorsMulti,
 *     or linear elasticity itself (penalty Dirichlet, constant body load),
 *     integrated with the cut-cell procedure of Figure 1 (bisection to a
 *     maximum depth, triangulation, Gauss rules on the clipped subcells and on
 *     the approximate boundary);
 *   - the nested hierarchy: two-scale restrictions R_l with
 *     Phi_{l-1} = R_l Phi_l (eq:coarsening) and Galerkin operators
 *     A_{l-1} = R_l A_l R_l^T (Remark rem:gridParamCorr);
 *   - the Schwarz blocks by encapsulating supports on every level above the
 *     coarsest (smoothers subsection; Lagrange: vertex functions only).
 *
 * Conventions: level 0 is the coarsest, level nlevels-1 the finest.  On every
 * level the active functions are numbered in ascending lattice index (x
 * fastest); CSR columns are sorted; the CSR pattern is structural (two active
 * functions sharing an active element), explicit zeros included.  All arrays
 * returned by the getters are copied into caller-owned buffers sized by the
 * matching *_info call.
 *
 * Errors: every call returns 0 on success and a negative code otherwise
 * (-1 invalid argument, -2 out of memory); imsmg_gen_last_error() gives text.
 * The problem object is not thread-safe; one object per thread.
 */
#ifndef IMSMG_GEN_H
#define IMSMG_GEN_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { IMSMG_GEN_BSPLINE = 0, IMSMG_GEN_LAGRANGE = 1 };
enum { IMSMG_GEN_BOX_DIRICHLET = 0, IMSMG_GEN_PENALTY = 1, IMSMG_GEN_NEUMANN = 2 };
enum { IMSMG_GEN_RHS_ONE = 0, IMSMG_GEN_RHS_MANUFACTURED = 1, IMSMG_GEN_RHS_ZERO = 2 };
enum { IMSMG_GEN_GEOM_NONE = 0, IMSMG_GEN_GEOM_DISCS = 1, IMSMG_GEN_GEOM_GYROID = 2, IMSMG_GEN_GEOM_STAR = 3,
       IMSMG_GEN_GEOM_APPLE = 4, IMSMG_GEN_GEOM_SLAB = 5 };
/* physics: scalar Poisson, or linear elasticity (eq:weakMulti / eq:operatorsMulti) with dim
 * displacement components */
enum { IMSMG_GEN_POISSON = 0, IMSMG_GEN_ELASTICITY = 1 };
/* part of the immersed boundary that carries the penalty Dirichlet condition: all of it, or the
 * apple's bite (boundary points where the bite's level set is the smaller of the two) */
enum { IMSMG_GEN_DIRICHLET_ALL = 0, IMSMG_GEN_DIRICHLET_BITE = 1 };

typedef struct {
  int32_t dim;          /* 2 or 3 */
  int32_t degree;       /* p >= 1 */
  int32_t n;            /* elements per axis on the finest level (divisible by 2^(levels-1)) */
  int32_t depth;        /* bisection depth of cut elements on the finest level */
  int32_t levels;       /* >= 1 */
  int32_t basis;        /* IMSMG_GEN_BSPLINE / IMSMG_GEN_LAGRANGE */
  int32_t bc;           /* IMSMG_GEN_BOX_DIRICHLET / _PENALTY / _NEUMANN */
  int32_t rhs;          /* IMSMG_GEN_RHS_* */
  int32_t geometry;     /* IMSMG_GEN_GEOM_* */
  int32_t ndiscs;       /* discs: rows (cx, cy, r) in `discs` */
  const double *discs;
  double phase[3];      /* gyroid phase shift */
  double gyroid_level;  /* gyroid keeps {g < level} */
  double box_lo, box_hi;
  double penalty_factor;/* beta = penalty_factor / h_finest */
  int32_t q_cell, q_simplex, q_bnd; /* Gauss points per axis; 0 = defaults */
  int32_t nthreads;     /* 0 = OpenMP default */
  int32_t with_mass;    /* also assemble the fine mass matrix */
  int32_t physics;      /* IMSMG_GEN_POISSON / IMSMG_GEN_ELASTICITY */
  int32_t dirichlet_part; /* IMSMG_GEN_DIRICHLET_* (bc = PENALTY) */
  double lame_lambda, lame_mu; /* elasticity: Lame parameters */
  double force[3];      /* elasticity: constant body load */
  double plane_x;       /* slab: Omega = {x < plane_x} */
} imsmg_gen_spec;

typedef struct imsmg_gen_problem imsmg_gen_problem;

typedef struct {
  int32_t n_active;      /* active functions (rows) */
  int64_t nnz;           /* CSR entries of A_l */
  int32_t lattice[3];    /* functions per axis (unused axes = 1) */
  int32_t n_elements;    /* elements per axis on this level */
  int32_t nblocks;       /* Schwarz blocks (0 on the coarsest level) */
  int64_t block_nnz;     /* total block entries */
  int64_t r_nnz;         /* entries of R_l (maps this level to level-1; 0 on level 0) */
  int32_t n_cut;         /* active elements that are cut */
  int32_t n_active_elements;
  int64_t elem_nnz;      /* entries of the element -> active function incidence */
  double eta_min;        /* smallest volume fraction of an active element */
  int32_t ncomp;         /* components per function: 1 (Poisson) or dim (elasticity) */
} imsmg_gen_level_info;

int imsmg_gen_build(const imsmg_gen_spec *spec, imsmg_gen_problem **out);
int imsmg_gen_level_info_get(const imsmg_gen_problem *p, int level, imsmg_gen_level_info *info);
/* dof_to_lattice[n_active]; rowptr[n_active+1], col[nnz], val[nnz] (any may be NULL) */
int imsmg_gen_get_operator(const imsmg_gen_problem *p, int level, int32_t *dof_to_lattice,
                           int32_t *rowptr, int32_t *col, double *val);
/* Elasticity: the values of the operator's component block (ci, cj) (rows: component ci of the
 * active functions, columns: component cj) on the scalar pattern of imsmg_gen_get_operator;
 * the vector operator is [A_(ci,cj)] with DOF c n_active + i (component-major).  Poisson:
 * only (0, 0), equal to the operator's values. */
int imsmg_gen_get_operator_block(const imsmg_gen_problem *p, int level, int ci, int cj, double *val);
/* R_l: n_active(level-1) x n_active(level), rowptr[n_{l-1}+1], col/val[r_nnz] */
int imsmg_gen_get_restriction(const imsmg_gen_problem *p, int level, int32_t *rowptr, int32_t *col,
                              double *val);
/* 1D two-scale matrix of R_l (dense, row-major): rows = functions per axis of
 * level l-1, cols = functions per axis of level l (level >= 1) */
int imsmg_gen_get_two_scale(const imsmg_gen_problem *p, int level, double *R1);
/* blocks: ptr[nblocks+1], idx[block_nnz] (sorted compact indices), assoc[nblocks] */
int imsmg_gen_get_blocks(const imsmg_gen_problem *p, int level, int32_t *ptr, int32_t *idx, int32_t *assoc);
/* Colours for the multiplicative smoother (smoothers subsection: blocks of one
 * colour share no element).  kind 0: one per Schwarz block (nblocks; B-splines
 * (p+1)^d colours from the associated function's lattice position mod p+1,
 * Lagrange vertex blocks 2^d colours from the vertex position mod 2); kind 1:
 * one per active function (n_active) for one-function blocks (Gauss-Seidel,
 * (p+1)^d colours). */
int imsmg_gen_get_block_colours(const imsmg_gen_problem *p, int level, int kind, int32_t *colour);
/* The same colour rule on given lattice positions (no problem object):
 * colour[j] = sum_a ((m_a / stride) mod q) q^a for the function at
 * dof_to_lattice[j] (x fastest over nf1 functions per axis); q = p + 1,
 * stride 1 for B-splines and one-function blocks, q = 2, stride p for
 * Lagrange vertex blocks. */
int imsmg_gen_lattice_colours(int n, const int32_t *dof_to_lattice, int nf1, int dim, int q, int stride,
                              int32_t *colour);
/* active elements in ascending element index: eptr[n_active_elements+1],
 * eidx[elem_nnz] = compact indices of the active functions non-zero on the
 * element (x offset fastest), elem[n_active_elements] = element index */
int imsmg_gen_get_elements(const imsmg_gen_problem *p, int level, int32_t *eptr, int32_t *eidx, int32_t *elem);
/* fine right-hand side b[ncomp n_active(fine)] (component-major for elasticity) */
int imsmg_gen_get_rhs(const imsmg_gen_problem *p, double *b);
/* fine mass matrix values on the fine pattern (requires with_mass) */
int imsmg_gen_get_mass(const imsmg_gen_problem *p, double *val);
/* volume fraction |K cap Omega_h|/|K| per element of a level (n_elements^dim, x fastest; 0 = inactive) */
int imsmg_gen_get_volume_fractions(const imsmg_gen_problem *p, int level, double *eta);
double imsmg_gen_setup_seconds(const imsmg_gen_problem *p);
const char *imsmg_gen_last_error(void);
void imsmg_gen_free(imsmg_gen_problem *p);

#ifdef __cplusplus
}
#endif
#endif
