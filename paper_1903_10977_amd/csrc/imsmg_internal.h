// Internal declarations of the HIP solver library (gfx950 / MI355X).
//
// Data layout on every level (see the library header for the public view):
//   * vectors live on the padded function lattice of the level (x fastest),
//     with a zero guard band on both sides so that every stencil offset of
//     every active row stays in bounds; inactive lattice entries stay 0;
//   * the operator is "lattice-ELL": K = (2 reach + 1)^d slots per active row,
//     slot s <-> fixed lattice offset off[s], values stored slot-major
//     (val[s * n + i]) so that consecutive rows read consecutive addresses; no
//     column indices are stored;
//   * restriction / prolongation are ELL with explicit lattice columns;
//   * additive Schwarz: rows whose only block is their own singleton are
//     "trivial" (x_i += c_i r_i); other blocks keep packed column-major FP64
//     inverses, a task list (one entry per block row) and a deterministic
//     gather map row -> task entries.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#define IMSMG_MAX_SLOTS 343  // (2*3+1)^3
#define IMSMG_MAX_BLOCK 60   // largest Schwarz block factorized in LDS (2 x 60^2 FP64 < 64 KiB)

namespace imsmg {

struct Offsets {
  int32_t off[IMSMG_MAX_SLOTS];
};

// Scalars of the CG iteration, kept on the device.
struct CGState {
  double rz;       // r . z of the current iterate
  double rz_old;   // previous r . z
  double beta;
  double pq;
  double alpha;
  double rr;       // ||r||^2
  double r0sq;     // ||r_0||^2
  double tol2;     // (rtol * ||r_0||)^2
  double bb;       // ||b||^2
  double aux;      // scratch scalar (true residual)
  int32_t done;    // 1: converged or stopped
  int32_t iters;
  int32_t status;  // 0 ok, IMSMG_ERR_NOT_SPD on p.q <= 0, IMSMG_ERR_NAN on NaN
  int32_t first;   // 1 before the first direction is formed
};


// --------------------------------------------------------------- launchers
// lattice-ELL residual / product: y = b - A x  (b may be null -> y = A x; sign=-1 gives -Ax)
void launch_ell_residual(hipStream_t s, int n, int K, const Offsets &off, const int32_t *row_lat,
                         const double *val, const double *x, const double *b, double *y, const int32_t *done);
void launch_ell_residual_f32(hipStream_t s, int n, int K, const Offsets &off, const int32_t *row_lat,
                             const float *val, const double *x, const double *b, double *y, const int32_t *done);
// ELL gather: y[lat_row[i]] (+)= sum_s v[s*n+i] x[col[s*n+i]]
void launch_ell_gather(hipStream_t s, int n, int w, const int32_t *row_lat, const int32_t *col, const double *v,
                       const double *x, double *y, int accumulate, const int32_t *done);
// index-free tensor transfer: y[row_lat[i]] (+)= sum over the band product of xin
void launch_tensor_transfer(hipStream_t s, int dim, int n, const int32_t *row_lat, int ox, int oy,
                            const int32_t *start, const int32_t *len, const double *coef, int W, int ix, int iy,
                            const double *xin, double *y, int accumulate, const int32_t *done);
// Schwarz phase 1: y[t] = w_j * sum_b inv_j[a + n_j b] r[blat[start_j + b]]
void launch_schwarz_blocks(hipStream_t s, int ntask, const int32_t *task_block, const int32_t *bstart,
                           const int32_t *bsize, const int64_t *binv_off, const int32_t *blat, const double *binv,
                           const double *bw, const double *r, double *y, const int32_t *done);
// Schwarz phase 2: x[lat_i] = (acc ? x : 0) + c_i r[lat_i] + sum_{t in g(i)} y[t]
void launch_schwarz_gather(hipStream_t s, int n, const int32_t *row_lat, const double *c, const int32_t *gptr,
                           const int32_t *gidx, const double *y, const double *r, double *x, int accumulate,
                           const int32_t *done);
// dense coarse solve x[lat_i] = sum_j Ainv[i n + j] r[lat_j]
void launch_dense_gemv(hipStream_t s, int n, const int32_t *row_lat, const double *Ainv, const double *r, double *x,
                       const int32_t *done);
// compact <-> padded lattice
void launch_scatter(hipStream_t s, int n, const int32_t *row_lat, const double *src, double *dst);
void launch_gather(hipStream_t s, int n, const int32_t *row_lat, const double *src, double *dst);
void launch_fill(hipStream_t s, size_t n, double v, double *dst);

// CG kernels (fine level, padded vectors, active rows only)
void launch_cg_init(hipStream_t s, int n, int K, const Offsets &off, const int32_t *row_lat, const double *val,
                    const double *x, const double *b, double *r, double *part, CGState *st, double rtol);
void launch_cg_dot_rz(hipStream_t s, int n, const int32_t *row_lat, const double *r, const double *z, double *part,
                      CGState *st);
void launch_cg_direction(hipStream_t s, int n, const int32_t *row_lat, const double *z, double *p, CGState *st);
void launch_cg_spmv_pq(hipStream_t s, int n, int K, const Offsets &off, const int32_t *row_lat, const double *val,
                       const double *p, double *q, double *part, CGState *st);
void launch_cg_update(hipStream_t s, int n, const int32_t *row_lat, const double *p, const double *q, double *x,
                      double *r, double *part, CGState *st, int max_iter);
void launch_cg_true_residual(hipStream_t s, int n, int K, const Offsets &off, const int32_t *row_lat,
                             const double *val, const double *x, const double *b, double *tmp, double *part,
                             CGState *st);
int reduction_blocks(int n);

// factorization
int launch_block_factor_geom(hipStream_t s, int nblocks, int maxn, const int32_t *bstart, const int32_t *bsize,
                             const int32_t *blat, const int32_t *brow, int n, int dim, int nx, int ny, int reach,
                             const double *val, double *inv_out, const int64_t *inv_off, uint8_t *keep_out,
                             double *lam_out, int32_t *info_out, double ratio);
void launch_gauss_jordan_step(hipStream_t s, int n, int k, double *A, double *colk, double *rowk,
                              int32_t *bad_pivot);
void launch_dense_from_ell(hipStream_t s, int n, int K, const Offsets &off, const int32_t *row_lat,
                           const int32_t *lat2c, const double *val, double *dense);
void launch_count_nk(hipStream_t s, int nel, const int32_t *eptr, const int32_t *eidx, const int32_t *fptr,
                     const int32_t *fblk, int32_t *nk, int32_t *overflow);
void launch_diag_coef(hipStream_t s, int n, int K, int center_slot, const int32_t *trivial_block, const double *val,
                      const double *bw, double *c);

}  // namespace imsmg

#define HIP_CHECK_RET(expr)                                                                  \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess) {                                                                  \
      throw imsmg::HipFailure(std::string(#expr) + ": " + hipGetErrorString(_e));            \
    }                                                                                        \
  } while (0)

namespace imsmg {
struct HipFailure {
  std::string msg;
  explicit HipFailure(std::string m) : msg(std::move(m)) {}
};
}  // namespace imsmg
