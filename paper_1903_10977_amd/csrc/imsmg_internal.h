// Internal declarations of the HIP solver library (gfx950 / MI355X).
//
// Data layout on every level (the public view is in include/imsmg.h):
//   * vectors live on the padded function lattice of the level (x fastest),
//     with a zero guard band on both sides so that every stencil offset of
//     every active row stays in bounds; inactive lattice entries stay 0;
//   * the operator is a compressed lattice-ELL: K = (2 reach + 1)^d slots per
//     active row, slot s <-> fixed lattice offset off[s], no column indices;
//     rows equal (to 1e-14 relative) to the level's uniform interior stencil
//     read that stencil from the kernel arguments, the other rows keep their
//     own values slot-major (val[s * nv + g]);
//   * restriction / prolongation are index-free tensor products of the 1D
//     two-scale matrix (or ELL with explicit lattice columns);
//   * additive Schwarz: trivial rows (own singleton block only) get
//     x_i += c_i r_i inside the residual kernel; general rows apply rows of
//     omega_j A_j^{-1} (stored contiguously, FP64) to the block residuals.
#pragma once
#include <stdexcept>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "imsmg.h"

#define IMSMG_MAX_SLOTS 125  // (2*2+1)^3: 3D up to reach 2, 2D up to reach 5
#define IMSMG_MAX_BLOCK 60   // largest Schwarz block factorized in LDS (2 x 60^2 FP64 < 64 KiB)

namespace imsmg {

constexpr int kTileRows = 256;  // rows (= threads) per workgroup of the stencil kernels
// lattice box of a stencil workgroup: 32 x 8 points in 2D, 16 x 4 x 4 in 3D
constexpr int kTile2X = 32, kTile2Y = 8;
constexpr int kTile3X = 16, kTile3Y = 4, kTile3Z = 4;

constexpr uint32_t kMetaIndex = 0x3fffffffu;    // low 30 bits: compressed-value index, all ones = uniform
constexpr uint32_t kMetaGeneral = 0x40000000u;  // row belongs to a general Schwarz block

struct Offsets {
  int32_t off[IMSMG_MAX_SLOTS];
};

// Operator of a general sparse level (no function lattice): CSR with sorted
// columns; vectors of such a level are indexed by row.
template <typename V>
struct CsrView {
  const int32_t *ptr;
  const int32_t *col;
  const V *val;
};

template <typename V>
struct OpView {
  Offsets off;
  const V *ref;            // uniform interior stencil (K values)
  const double *refd;      // the same K values widened to FP64 (tiled kernels: no per-tap conversion)
  const V *val;            // stored rows, slot-major
  int nv;                  // number of stored rows (numbered tile by tile)
  const int32_t *sloc;     // lattice point of every stored row within its tile box (tx + TX (ty + TY tz))
  const int32_t *tile_g0;  // first stored row of every lattice tile (ntiles + 1 entries)
  const int32_t *lat2row;  // lattice point -> row (-1: inactive)
  int sx, sy, sz;          // lattice shape (sz = 1 in 2D)
  int ntx, nty, ntiles;    // lattice tiles along x, along y, in total
  int stream;              // 1: stored values read with the non-temporal hint (see stream_load)
};

// Streamed operator values: where a level holds more than kStreamValues
// stored values (they are read once per launch and, with the level's other
// data, exceed the last-level cache), 16-byte loads with the non-temporal
// hint keep them from evicting the x windows that neighbouring tiles share.
// Smaller levels stay cache-resident between launches and use ordinary loads.
// Measured (FP64 V-cycle): the 128^3 gyroid 0.590 ms with ordinary loads,
// 0.564 ms streaming its two finest levels; the 1024^2 discs (7.8M values on
// the finest level) 0.319 ms with ordinary loads, 0.363 ms streaming; the
// count, not the bytes, decides (FP32 values: the same levels stream best).
constexpr size_t kStreamValues = size_t(8) << 20;
typedef double nt_double2 __attribute__((ext_vector_type(2)));
typedef float nt_float4 __attribute__((ext_vector_type(4)));
// NT is a compile-time choice: a run-time test per load splits the unrolled
// load sequences and serializes them (measured 4.7x slower).
template <bool NT>
__device__ __forceinline__ double2 stream_load(const double2 *p) {
  if constexpr (!NT) {
    return *p;
  } else {
    const nt_double2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_double2 *>(p));
    return make_double2(v.x, v.y);
  }
}
template <bool NT>
__device__ __forceinline__ float4 stream_load(const float4 *p) {
  if constexpr (!NT) {
    return *p;
  } else {
    const nt_float4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_float4 *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
  }
}

// Vector operators (linear elasticity, ncomp displacement components): the
// ncomp x ncomp component blocks A_(c,e) of a level, each a compressed
// lattice-ELL operator on the scalar lattice, for the tiled vector kernels
// (vec_row.h).  Vectors hold the components as consecutive padded scalar
// arrays: component e of lattice point L at x[e * cstride + L].
constexpr int kMaxComp = 3;

template <typename V>
struct VecOps {
  // block b = c * ncomp + e
  const double *refd[kMaxComp * kMaxComp];
  const V *val[kMaxComp * kMaxComp];
  const int32_t *sloc[kMaxComp * kMaxComp];
  const int32_t *tile_g0[kMaxComp * kMaxComp];
  const uint32_t *meta[kMaxComp * kMaxComp];  // per scalar row: stored index or kMetaIndex
  int nv[kMaxComp * kMaxComp];
  const int32_t *lat2row;  // lattice point -> scalar row (-1: inactive)
  int sx, sy, sz, ntx, nty, ntiles;
  int ncomp, ns;           // components, scalar rows
  int64_t cstride;         // component stride of the level's vectors
};

// Stored-row values: the K slots of a row in groups of 16 bytes (G = 2 FP64 or
// 4 FP32 values), group-major over the stored rows: value (g, s) sits at
// ((s / G) nv + g) G + s % G.  A lane reads one group of its row with one
// 16-byte load and consecutive lanes read consecutive groups (a wavefront's
// load is one contiguous kilobyte), so a row costs ceil(K / G) vector loads
// instead of K.  Padding slots of the last group hold zeros.
template <typename V>
struct SlotGroup {
  static constexpr int G = 16 / int(sizeof(V));
};
template <typename V>
__host__ __device__ __forceinline__ size_t stored_at(size_t nv, size_t g, int s) {
  constexpr int G = SlotGroup<V>::G;
  return (size_t(s / G) * nv + g) * G + size_t(s % G);
}
inline size_t stored_size(int K, size_t nv, int G) { return size_t((K + G - 1) / G) * nv * size_t(G); }

// bands of 1D two-scale matrices up to this length take the unrolled
// transfer paths (B-splines of degree <= 3)
constexpr int kBandMax = 5;

// Prolongation x_f += R^T x_c applied inside a smoothing step's staging:
// R^T is the tensor product of one 1D matrix given by bands (per fine 1D
// index: first coarse index, length, and coefficients with stride kBandMax,
// zero past the length; W <= kBandMax is the longest band);
// org holds, per lattice tile along x, then y, then z, the first coarse index
// of the coarse window the tile's x window needs.
struct ProlongView {
  const double *xc;
  const int32_t *start;
  const int32_t *len;
  const double *coef;
  int W;
  int cs;  // coarse functions per axis
  const int32_t *org;
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
  double rz_mix;   // r_{k+1} . z_k (flexible CG)
  int32_t done;    // 1: converged or stopped
  int32_t iters;
  int32_t status;  // 0 ok, IMSMG_ERR_NOT_SPD on p.q <= 0, IMSMG_ERR_NAN on NaN
  int32_t first;   // 1 before the first direction is formed
};

// Scalars of the multi-right-hand-side CG (up to kMaxRhs columns).
constexpr int kMaxRhs = 16;
struct MState {
  double rz[kMaxRhs], rz_old[kMaxRhs], beta[kMaxRhs], alpha[kMaxRhs], rr[kMaxRhs], r0sq[kMaxRhs];
  double tol2[kMaxRhs], bb[kMaxRhs], aux[kMaxRhs];
  int32_t cdone[kMaxRhs];  // column converged
  int32_t iters[kMaxRhs];
  int32_t done;            // every column converged, or stopped
  int32_t status;
  int32_t first;
  int32_t pad;
};

// The lattice kernels read the stored values and the reference stencil of an
// OpView; a level without them (a general sparse level, or the FP32 view of
// an FP64 setup) must never reach those kernels.
template <typename V>
inline void require_lattice_op(const OpView<V> &op) {
  if (!op.val || !op.ref) throw std::invalid_argument("lattice kernel launched without a lattice operator");
}

// --------------------------------------------------------------- level kernels
void launch_residual(hipStream_t s, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                     const uint32_t *meta, const double *x, const double *b, double *y, const int32_t *done);
void launch_residual(hipStream_t s, int n, int K, const OpView<float> &op, const int32_t *row_lat,
                     const uint32_t *meta, const double *x, const double *b, double *y, const int32_t *done);
// pv != nullptr: the step starts from xa + R^T xc (prolongation of the coarse
// correction applied while the x window is staged; tiled K, tensor transfers)
void launch_residual_smooth(hipStream_t s, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                            const uint32_t *meta, const double *c, const double *xa, const double *r, double *rh,
                            double *xb, const int32_t *done, const ProlongView *pv = nullptr);
void launch_residual_smooth(hipStream_t s, int n, int K, const OpView<float> &op, const int32_t *row_lat,
                            const uint32_t *meta, const double *c, const double *xa, const double *r, double *rh,
                            double *xb, const int32_t *done, const ProlongView *pv = nullptr);
// general sparse levels (CSR operator, ln lanes per row: 4, 8 or 16):
// y = b - A x (b == nullptr: y = A x) and the smoothing step with the same
// contract as launch_residual_smooth (no fused prolongation)
void launch_csr_residual(hipStream_t s, int n, int ln, const CsrView<double> &A, const uint32_t *meta,
                         const double *x, const double *b, double *y, const int32_t *done);
void launch_csr_residual(hipStream_t s, int n, int ln, const CsrView<float> &A, const uint32_t *meta,
                         const double *x, const double *b, double *y, const int32_t *done);
void launch_csr_residual_smooth(hipStream_t s, int n, int ln, const CsrView<double> &A, const uint32_t *meta,
                                const double *c, const double *xa, const double *r, double *rh, double *xb,
                                const int32_t *done);
void launch_csr_residual_smooth(hipStream_t s, int n, int ln, const CsrView<float> &A, const uint32_t *meta,
                                const double *c, const double *xa, const double *r, double *rh, double *xb,
                                const int32_t *done);
// general Schwarz rows: x[grow_lat[t]] += sum_k S[t,k] r[scol[k]]  (S_G in CSR, lattice columns)
// vector levels: y = b - A x (b == nullptr: y = A x) and the smoothing step
// (rh = r - A xa on general rows, xb = xa + c (r - A xa)), per component;
// flags: per vector row, the general-block bit; c: per vector row
void launch_vresidual(hipStream_t s, int K, const VecOps<double> &ops, const uint32_t *flags, const double *x,
                      const double *b, double *y, const int32_t *done);
void launch_vresidual(hipStream_t s, int K, const VecOps<float> &ops, const uint32_t *flags, const double *x,
                      const double *b, double *y, const int32_t *done);
void launch_vresidual_smooth(hipStream_t s, int K, const VecOps<double> &ops, const uint32_t *flags, const double *c,
                             const double *xa, const double *r, double *rh, double *xb, const int32_t *done);
void launch_vresidual_smooth(hipStream_t s, int K, const VecOps<float> &ops, const uint32_t *flags, const double *c,
                             const double *xa, const double *r, double *rh, double *xb, const int32_t *done);
void launch_smooth_general(hipStream_t s, int ng, const int32_t *grow_lat, const int32_t *sptr,
                           const int32_t *scol, const double *sval, const double *r, double *x, const int32_t *done,
                           int lanes = 4);  // lanes per row: 2, 4 or 8
// S_G = sum_j omega_j P_j A_j^{-1} P_j^T on the general rows, accumulated entry by entry in
// ascending block order into the CSR pattern (epos: CSR slot of every (entry, member) pair)
void launch_assemble_sg(hipStream_t s, int ng, const int32_t *gptr, const int64_t *ent_off, const int32_t *ent_n,
                        const int64_t *ent_pos, const int32_t *epos, const double *winv, double *sval);
void launch_diag_scale(hipStream_t s, int n, const int32_t *row_lat, const double *c, const double *r, double *x,
                       const int32_t *done);
void launch_ell_gather(hipStream_t s, int n, int w, const int32_t *row_lat, const int32_t *col, const double *v,
                       const double *x, double *y, int accumulate, const double *cinit, double *xinit,
                       const int32_t *done);
void launch_tensor_transfer(hipStream_t s, int dim, int n, const int32_t *row_lat, int ox, int oy,
                            const int32_t *start, const int32_t *len, const double *coef, int W, int ix, int iy,
                            const double *xin, double *y, int accumulate, const double *cinit, double *xinit,
                            const int32_t *done);
void launch_dense_gemv(hipStream_t s, int n, const int32_t *row_lat, const double *Ainv, const double *r, double *x,
                       const int32_t *done);
void launch_scatter(hipStream_t s, int n, const int32_t *row_lat, const double *src, double *dst);
// multiplicative Schwarz: one colour's rows (residual of the current x; in-place
// update of one-function blocks with cf != 0, residual into rh for the others);
// stored rows read the colour-ordered value copy (vidx: its entry, -1 = the
// reference stencil), built by launch_ms_pack from the level's operator values
void launch_ms_colour(hipStream_t s, int m, const int32_t *rows, const double *cf, const int32_t *vidx,
                      const double *vals, int K, const OpView<double> &op, const int32_t *row_lat, const double *r,
                      double *x, double *rh, const int32_t *done, int stream);
void launch_ms_colour(hipStream_t s, int m, const int32_t *rows, const double *cf, const int32_t *vidx,
                      const float *vals, int K, const OpView<float> &op, const int32_t *row_lat, const double *r,
                      double *x, double *rh, const int32_t *done, int stream);
// vector levels: vidx holds ncomp entries per list entry (block (c, e) of the row)
void launch_vms_colour(hipStream_t s, int m, const int32_t *rows, const double *cf, const int32_t *vidx,
                       const double *vals, int K, const VecOps<double> &ops, const int32_t *row_lat, const double *r,
                       double *x, double *rh, const int32_t *done, int stream);
void launch_vms_colour(hipStream_t s, int m, const int32_t *rows, const double *cf, const int32_t *vidx,
                       const float *vals, int K, const VecOps<float> &ops, const int32_t *row_lat, const double *r,
                       double *x, double *rh, const int32_t *done, int stream);
// general sparse levels: the colour step on CSR rows (ln lanes per row)
void launch_csr_ms_colour(hipStream_t s, int m, int ln, const int32_t *rows, const double *cf,
                          const CsrView<double> &A, const double *r, double *x, double *rh, const int32_t *done);
void launch_csr_ms_colour(hipStream_t s, int m, int ln, const int32_t *rows, const double *cf,
                          const CsrView<float> &A, const double *r, double *x, double *rh, const int32_t *done);
void launch_ms_pack(hipStream_t s, int ne, int K, int KP, const int32_t *g, const double *val, int nv, double *out);
void launch_ms_pack(hipStream_t s, int ne, int K, int KP, const int32_t *g, const float *val, int nv, float *out);
// active rows of a level vector: op 0: y = 0, 1: y = x, 2: y += x
void launch_rows_op(hipStream_t s, int n, const int32_t *row_lat, const double *x, double *y, int op,
                    const int32_t *done);
void launch_gather(hipStream_t s, int n, const int32_t *row_lat, const double *src, double *dst);

// --------------------------------------------------------------- CG kernels
// (finest level, padded vectors, active rows only, operator in FP64)
void launch_cg_init(hipStream_t s, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                    const uint32_t *meta, const double *x, const double *b, double *r, double *part, CGState *st,
                    double rtol, int restart);
// r . z and beta (flexible: Polak-Ribiere form with the r_{k+1} . z_k of the last update)
// CG on a vector finest level: init (r = b - A x, ||r||^2, ||b||^2), q = A p
// with p.q, and ||b - A x||^2, partials over all (tile, component) workgroups
void launch_vcg_init(hipStream_t s, int K, const VecOps<double> &ops, const uint32_t *flags, const double *x,
                     const double *b, double *r, double *part, CGState *st, double rtol, int restart);
void launch_vcg_spmv_pq(hipStream_t s, int K, const VecOps<double> &ops, const uint32_t *flags, const double *p,
                        double *q, double *part, CGState *st);
void launch_vcg_true_residual(hipStream_t s, int K, const VecOps<double> &ops, const uint32_t *flags,
                              const double *x, const double *b, double *part, CGState *st);
void launch_cg_dot_rz(hipStream_t s, int n, const int32_t *row_lat, const double *r, const double *z, double *part,
                      CGState *st, int flexible);
void launch_cg_direction(hipStream_t s, int n, const int32_t *row_lat, const double *z, double *p, CGState *st);
void launch_cg_spmv_pq(hipStream_t s, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                       const uint32_t *meta, const double *p, double *q, double *part, CGState *st);
// x += alpha p, r -= alpha q, ||r||^2; also zs = c * r (first smoothing step of the next V-cycle);
// zk != nullptr (flexible CG): also r_{k+1} . z_k (part must hold two partial arrays)
void launch_cg_update(hipStream_t s, int n, const int32_t *row_lat, const double *p, const double *q, double *x,
                      double *r, const double *c, double *zs, const double *zk, double *part, CGState *st,
                      int max_iter);
void launch_cg_true_residual(hipStream_t s, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                             const uint32_t *meta, const double *x, const double *b, double *part, CGState *st);
int reduction_blocks(int n);
// CG on a general sparse finest level (CSR operator, ln lanes per row);
// partial sums per workgroup as the lattice forms (csr_part_blocks of them)
int csr_part_blocks(int n, int ln);
void launch_csr_cg_init(hipStream_t s, int n, int ln, const CsrView<double> &A, const double *x, const double *b,
                        double *r, double *part, CGState *st, double rtol, int restart);
void launch_csr_cg_spmv_pq(hipStream_t s, int n, int ln, const CsrView<double> &A, const double *p, double *q,
                           double *part, CGState *st);
void launch_csr_cg_true_residual(hipStream_t s, int n, int ln, const CsrView<double> &A, const double *x,
                                 const double *b, double *part, CGState *st);

// --------------------------------------------------------------- multi-RHS (R = 4, 8, 16 interleaved columns)
bool multi_supported(int R);
int multi_blocks(int R, int n);
size_t multi_part_size(int R, int n, int ntiles);  // partial-sum workspace (doubles)
void launch_m_residual(hipStream_t s, int R, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                       const uint32_t *meta, const double *x, const double *b, double *y, const int32_t *done);
void launch_m_residual(hipStream_t s, int R, int n, int K, const OpView<float> &op, const int32_t *row_lat,
                       const uint32_t *meta, const double *x, const double *b, double *y, const int32_t *done);
void launch_m_residual_smooth(hipStream_t s, int R, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                              const uint32_t *meta, const double *c, const double *xa, const double *r, double *rh,
                              double *xb, const int32_t *done);
void launch_m_residual_smooth(hipStream_t s, int R, int n, int K, const OpView<float> &op, const int32_t *row_lat,
                              const uint32_t *meta, const double *c, const double *xa, const double *r, double *rh,
                              double *xb, const int32_t *done);
void launch_m_smooth_general(hipStream_t s, int R, int ng, const int32_t *grow_lat, const int32_t *sptr,
                             const int32_t *scol, const double *sval, const double *r, double *x, const int32_t *done);
void launch_m_diag_scale(hipStream_t s, int R, int n, const int32_t *row_lat, const double *c, const double *r,
                         double *x, const int32_t *done);
// general blocks of <= 16 functions as patch GEMMs on the matrix cores: Y_q =
// W_q R_q (bf16 != 0: BF16 operands with FP32 accumulation on the blocks
// flagged in lp, FP64 on the others), then per general row x += sum of its
// blocks' Y rows (ascending block order)
constexpr double kBf16Kappa = 16.0;  // blocks with cond(A_j) up to this take BF16
void launch_m_block_gemm(hipStream_t s, int bf16, int nb, int R, const int32_t *blat, const double *W,
                         const uint16_t *Wb, const int32_t *lp, const double *r, double *Y, const int32_t *done);
void launch_m_block_gather(hipStream_t s, int R, int ng, const int32_t *grow_lat, const int32_t *yp,
                           const int32_t *ypos, const double *Y, double *x, const int32_t *done);
void launch_pack_blocks(hipStream_t s, int nb, const int64_t *g_off, const int32_t *g_sz, const double *inv,
                        double *W, uint16_t *Wb);
void launch_m_tensor_transfer(hipStream_t s, int R, int dim, int n, const int32_t *row_lat, int ox, int oy,
                              const int32_t *start, const int32_t *len, const double *coef, int W, int ix, int iy,
                              const double *xin, double *y, int accumulate, const double *cinit, double *xinit,
                              const int32_t *done);
void launch_m_ell_gather(hipStream_t s, int R, int n, int w, const int32_t *row_lat, const int32_t *col,
                         const double *v, const double *x, double *y, int accumulate, const double *cinit,
                         double *xinit, const int32_t *done);
void launch_m_dense_gemm(hipStream_t s, int R, int n, const int32_t *row_lat, const double *Ainv, const double *r,
                         double *x, const int32_t *done);
void launch_m_scatter(hipStream_t s, int R, int n, int ncols, const int32_t *row_lat, const double *src, double *dst);
void launch_m_gather(hipStream_t s, int R, int n, int ncols, const int32_t *row_lat, const double *src, double *dst);
void launch_mcg_init(hipStream_t s, int R, int ncols, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                     const uint32_t *meta, const double *x, const double *b, double *r, double *part, MState *st,
                     double rtol, int restart, int keep_mask);
void launch_mcg_dot_rz(hipStream_t s, int R, int n, const int32_t *row_lat, const double *r, const double *z,
                       double *part, MState *st);
void launch_mcg_direction(hipStream_t s, int R, int n, const int32_t *row_lat, const double *z, double *p,
                          MState *st);
void launch_mcg_spmv_pq(hipStream_t s, int R, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                        const uint32_t *meta, const double *p, double *q, double *part, MState *st);
void launch_mcg_update(hipStream_t s, int R, int n, const int32_t *row_lat, const double *p, const double *q,
                       double *x, double *r, const double *c, double *zs, double *part, MState *st, int max_iter);
void launch_mcg_true_residual(hipStream_t s, int R, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                              const uint32_t *meta, const double *x, const double *b, double *part, MState *st);

// --------------------------------------------------------------- per-block damping
constexpr int kMlpInputs = 16, kMlpHidden = 64;
// largest sample count of the allocation-free loss/gradient entry point
constexpr int kNoAllocMaxSamples = IMSMG_NOALLOC_MAX_SAMPLES;
constexpr int kMlpParams = kMlpInputs * kMlpHidden + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden + kMlpHidden + 1;
constexpr double kMlpOutClip = 3.0;  // omega_j = gamma exp(clip(o_j, -3, 3))
size_t mlp_workspace_bytes(int n);
// allocation-free loss/gradient: the static device workspace (per device)
size_t mlp_noalloc_scratch_bytes();
int mlp_noalloc_scratch(hipStream_t s, void **out);
void launch_mlp_forward(hipStream_t s, int n, const float *params, const float *X, float *out);
void launch_mlp_loss_grad(hipStream_t s, int n, const float *params, const float *X, const float *t, void *work,
                          float *loss, float *grad);
void launch_mlp_adam(hipStream_t s, float *theta, const float *g, float *m, float *v, int step, float lr);
void launch_block_bilinear(hipStream_t s, int nb, const int32_t *bptr, const int32_t *blat, const int64_t *boff,
                           const double *bdiag, const double *wfold, const double *inv, const double *u,
                           const double *v, double coef, double *out);
int dot_blocks(int n);
void launch_dot_partial(hipStream_t s, int n, const int32_t *row_lat, const double *a, const double *b, double *part);
void launch_scale_copy(hipStream_t s, int n, const int32_t *row_lat, double alpha, const double *x, double *y);
void launch_sub_from(hipStream_t s, int n, const int32_t *row_lat, const double *x, double *y);

// --------------------------------------------------------------- factorization
int launch_block_factor_geom(hipStream_t s, int nblocks, int maxn, const int32_t *bstart, const int32_t *bsize,
                             const int32_t *blat, const int32_t *brow, int n, int dim, int nx, int ny, int reach,
                             const double *val, double *inv_out, const int64_t *inv_off, uint8_t *keep_out,
                             double *lam_out, int32_t *info_out, double ratio);
// the same factorization gathering A_j from a CSR operator (general sparse
// levels: brow are the members' rows, columns sorted)
int launch_block_factor_csr(hipStream_t s, int nblocks, int maxn, const int32_t *bstart, const int32_t *bsize,
                            const int32_t *brow, const CsrView<double> &A, double *inv_out, const int64_t *inv_off,
                            uint8_t *keep_out, double *lam_out, int32_t *info_out, double ratio);
void launch_gauss_jordan_step(hipStream_t s, int n, int k, double *A, double *colk, double *rowk,
                              int32_t *bad_pivot);
void launch_dense_from_ell(hipStream_t s, int n, int K, const Offsets &off, const int32_t *row_lat,
                           const int32_t *lat2c, const double *val, double *dense);
void launch_count_nk(hipStream_t s, int nel, const int32_t *eptr, const int32_t *eidx, const int32_t *fptr,
                     const int32_t *fblk, int32_t *nk, int32_t *overflow);
void launch_diag_coef(hipStream_t s, int n, int K, int center_slot, const int32_t *trivial_block, const double *val,
                      const double *bw, double *c);
void launch_scale_blocks(hipStream_t s, int nblocks, const int64_t *off, const int32_t *size, const double *w,
                         double *inv);

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
