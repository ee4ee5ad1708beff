// Per-level kernels of the V-cycle (Algorithm alg:MGV).
//
// Operator storage ("compressed lattice-ELL"): on a uniform tensor grid every
// row whose support lies inside the physical domain carries the same stencil.
// Such rows read their K values from a reference stencil passed as a kernel
// argument; the other rows (cut region, box boundary) keep their own values,
// slot-major over the compressed rows (val[s * nv + g]) so that consecutive
// rows still read consecutive addresses.  Per row one 32-bit word `meta`
// holds the compressed-value index (or kUniform) and the flag "row belongs to
// a general Schwarz block".
//
// Additive Schwarz (smoothers subsection) is split by rows:
//   * trivial rows (their only block is their own singleton):
//       x_i += c_i (r - A x)_i,  c_i = omega_j / A_ii, fused into the residual
//       kernel (ping-pong x buffers, because neighbours read the old x);
//   * general rows: x_i += sum over the blocks j holding i of row a_ij of
//       (omega_j A_j^{-1}) times the block's residual, one thread per row, no
//       atomics and a fixed summation order (deterministic).
//
// All row kernels map one thread to one active row; workgroups are renumbered
// so that each of the 8 XCDs walks one contiguous chunk of rows and keeps the
// neighbouring lattice lines of the input vector in its own L2.  The stencil
// kernels stage the workgroup's window of the input vector in LDS (op_row.h).
#include <stdexcept>

#include "imsmg_internal.h"
#include "csr_row.h"
#include "op_row.h"
#include "vec_row.h"

namespace imsmg {

constexpr int kRowBlock = 256;
static_assert(kRowBlock == kTileRows, "stencil kernels: one lattice point or row per thread");

__device__ __forceinline__ int xcd_block(int b, int nb) {
  // hardware dispatches workgroup b to XCD (b % 8); give XCD k a contiguous
  // range of logical blocks (a bijection of [0, nb))
  const int per = (nb + 7) / 8;
  const int xcd = b % 8;
  const int k = b / 8;
  const int full = nb % 8 == 0 ? 8 : nb % 8;
  if (xcd < full) return xcd * per + k;
  return full * per + (xcd - full) * (per - 1) + k;
}

static inline int grid_for(int n) { return (n + kRowBlock - 1) / kRowBlock; }

// epilogue of the residual: y = b - A x (b == nullptr: y = A x)
struct ResidualEpi {
  const double *__restrict__ b;
  double *__restrict__ y;
  struct Pre {
    double b;
  };
  __device__ Pre pre(int, int L) const { return {b ? b[L] : 0.0}; }
  __device__ double2 post(int, int L, unsigned, double ax, double, const Pre &p) const {
    y[L] = b ? p.b - ax : ax;
    return make_double2(0.0, 0.0);
  }
};

// epilogue of the smoothing step (trivial rows): rh = r - A xa on general
// rows, xb = xa + c (r - A xa)
struct SmoothEpi {
  const double *__restrict__ r;
  const double *__restrict__ c;
  double *__restrict__ rh;
  double *__restrict__ xb;
  struct Pre {
    double r, c;
  };
  __device__ Pre pre(int i, int L) const { return {r[L], c[i]}; }
  __device__ double2 post(int, int L, unsigned m, double ax, double xc, const Pre &p) const {
    const double res = p.r - ax;
    if (m & kMetaGeneral) rh[L] = res;
    xb[L] = xc + p.c * res;
    return make_double2(0.0, 0.0);
  }
};

// y = b - A x   (b == nullptr: y = A x)
template <int K, typename V, bool NT>
__global__ __launch_bounds__(kRowBlock, kTileBlocksPerCU) void k_residual(int n, int Kdyn, OpView<V> op, const int32_t *__restrict__ row_lat,
                                                        const uint32_t *__restrict__ meta,
                                                        const double *__restrict__ x, const double *__restrict__ b,
                                                        double *__restrict__ y, const int32_t *__restrict__ done) {
  __shared__ double tile[StencilShape<K>::LDS_DOUBLES];
  tile_rows<K, V, ResidualEpi, false, NT>(n, xcd_block(blockIdx.x, gridDim.x), op, row_lat, meta, x, tile, Kdyn,
                                          ResidualEpi{b, y}, done);
}

// smoothing step, trivial rows:  rh = r - A xa  (stored for general rows only),
// xb = xa + c * rh   (c = 0 on general rows, which the general kernel completes);
// PRO: xa + R^T xc in place of xa (the prolongation of the coarse correction)
template <int K, typename V, bool PRO, bool NT>
__global__ __launch_bounds__(kRowBlock, kTileBlocksPerCU) void k_residual_smooth(int n, int Kdyn, OpView<V> op,
                                                               const int32_t *__restrict__ row_lat,
                                                               const uint32_t *__restrict__ meta,
                                                               const double *__restrict__ c,
                                                               const double *__restrict__ xa,
                                                               const double *__restrict__ r, double *__restrict__ rh,
                                                               double *__restrict__ xb,
                                                               const int32_t *__restrict__ done, ProlongView pv) {
  __shared__ double tile[StencilShape<K>::LDS_DOUBLES + (PRO ? ProShape<K>::LDS_EXTRA : 0)];
  tile_rows<K, V, SmoothEpi, PRO, NT>(n, xcd_block(blockIdx.x, gridDim.x), op, row_lat, meta, xa, tile, Kdyn,
                                      SmoothEpi{r, c, rh, xb}, done, &pv);
}

template <typename V>
static void dispatch_residual(hipStream_t s, int n, int K, const OpView<V> &op, const int32_t *row_lat,
                              const uint32_t *meta, const double *x, const double *b, double *y, const int32_t *done) {
  if (n <= 0) return;
  require_lattice_op(op);
  dim3 g(stencil_grid(K, n, op)), t(kRowBlock);
#define IMSMG_R(KK)                                                                  \
  if (op.stream)                                                                     \
    k_residual<KK, V, true><<<g, t, 0, s>>>(n, K, op, row_lat, meta, x, b, y, done);  \
  else                                                                               \
    k_residual<KK, V, false><<<g, t, 0, s>>>(n, K, op, row_lat, meta, x, b, y, done);
  switch (K) {
    case 9: IMSMG_R(9) break;
    case 25: IMSMG_R(25) break;
    case 49: IMSMG_R(49) break;
    case 27: IMSMG_R(27) break;
    case 125: IMSMG_R(125) break;
    default: k_residual<0, V, false><<<g, t, 0, s>>>(n, K, op, row_lat, meta, x, b, y, done); break;
  }
#undef IMSMG_R
}

template <typename V>
static void dispatch_residual_smooth(hipStream_t s, int n, int K, const OpView<V> &op, const int32_t *row_lat,
                                     const uint32_t *meta, const double *c, const double *xa, const double *r,
                                     double *rh, double *xb, const int32_t *done, const ProlongView *pv) {
  if (n <= 0) return;
  require_lattice_op(op);
  dim3 g(stencil_grid(K, n, op)), t(kRowBlock);
  const ProlongView p = pv ? *pv : ProlongView{};
#define IMSMG_RS(KK)                                                                                         \
  if (pv)                                                                                                    \
    k_residual_smooth<KK, V, true, false><<<g, t, 0, s>>>(n, K, op, row_lat, meta, c, xa, r, rh, xb, done, p); \
  else if (op.stream)                                                                                        \
    k_residual_smooth<KK, V, false, true><<<g, t, 0, s>>>(n, K, op, row_lat, meta, c, xa, r, rh, xb, done, p); \
  else                                                                                                       \
    k_residual_smooth<KK, V, false, false><<<g, t, 0, s>>>(n, K, op, row_lat, meta, c, xa, r, rh, xb, done, p);
#define IMSMG_RS3(KK)                                                                                        \
  if (pv) throw std::invalid_argument("fused prolongation: 2D lattices only");                               \
  if (op.stream)                                                                                             \
    k_residual_smooth<KK, V, false, true><<<g, t, 0, s>>>(n, K, op, row_lat, meta, c, xa, r, rh, xb, done, p); \
  else                                                                                                       \
    k_residual_smooth<KK, V, false, false><<<g, t, 0, s>>>(n, K, op, row_lat, meta, c, xa, r, rh, xb, done, p);
  switch (K) {
    case 9: IMSMG_RS(9) break;
    case 25: IMSMG_RS(25) break;
    case 49: IMSMG_RS(49) break;
    case 27: IMSMG_RS3(27) break;
    case 125: IMSMG_RS3(125) break;
    default:
      if (pv) throw std::invalid_argument("fused prolongation needs a tiled stencil");
      k_residual_smooth<0, V, false, false><<<g, t, 0, s>>>(n, K, op, row_lat, meta, c, xa, r, rh, xb, done, p);
      break;
  }
#undef IMSMG_RS
#undef IMSMG_RS3
}

void launch_residual(hipStream_t s, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                     const uint32_t *meta, const double *x, const double *b, double *y, const int32_t *done) {
  dispatch_residual<double>(s, n, K, op, row_lat, meta, x, b, y, done);
}
void launch_residual(hipStream_t s, int n, int K, const OpView<float> &op, const int32_t *row_lat,
                     const uint32_t *meta, const double *x, const double *b, double *y, const int32_t *done) {
  dispatch_residual<float>(s, n, K, op, row_lat, meta, x, b, y, done);
}
void launch_residual_smooth(hipStream_t s, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                            const uint32_t *meta, const double *c, const double *xa, const double *r, double *rh,
                            double *xb, const int32_t *done, const ProlongView *pv) {
  dispatch_residual_smooth<double>(s, n, K, op, row_lat, meta, c, xa, r, rh, xb, done, pv);
}
void launch_residual_smooth(hipStream_t s, int n, int K, const OpView<float> &op, const int32_t *row_lat,
                            const uint32_t *meta, const double *c, const double *xa, const double *r, double *rh,
                            double *xb, const int32_t *done, const ProlongView *pv) {
  dispatch_residual_smooth<float>(s, n, K, op, row_lat, meta, c, xa, r, rh, xb, done, pv);
}

// General sparse levels (csr_row.h): LN lanes per CSR row, the lattice
// kernels' epilogues at row positions.
template <int LN, typename V>
__global__ __launch_bounds__(kRowBlock) void k_csr_residual(int n, CsrView<V> A, const uint32_t *__restrict__ meta,
                                                            const double *__restrict__ x,
                                                            const double *__restrict__ b, double *__restrict__ y,
                                                            const int32_t *__restrict__ done) {
  csr_rows<LN, V, ResidualEpi>(n, A, meta, x, ResidualEpi{b, y}, done);
}

template <int LN, typename V>
__global__ __launch_bounds__(kRowBlock) void k_csr_residual_smooth(int n, CsrView<V> A,
                                                                   const uint32_t *__restrict__ meta,
                                                                   const double *__restrict__ c,
                                                                   const double *__restrict__ xa,
                                                                   const double *__restrict__ r,
                                                                   double *__restrict__ rh, double *__restrict__ xb,
                                                                   const int32_t *__restrict__ done) {
  csr_rows<LN, V, SmoothEpi>(n, A, meta, xa, SmoothEpi{r, c, rh, xb}, done);
}

#define IMSMG_CSR_LN(LN_, KERNEL, ...)                                         \
  switch (LN_) {                                                               \
    case 4: KERNEL<4, V><<<csr_grid(n, 4), kRowBlock, 0, s>>>(__VA_ARGS__); break;   \
    case 8: KERNEL<8, V><<<csr_grid(n, 8), kRowBlock, 0, s>>>(__VA_ARGS__); break;   \
    case 16: KERNEL<16, V><<<csr_grid(n, 16), kRowBlock, 0, s>>>(__VA_ARGS__); break; \
    default: throw std::invalid_argument("CSR rows: 4, 8 or 16 lanes per row");      \
  }

template <typename V>
static void csr_residual(hipStream_t s, int n, int ln, const CsrView<V> &A, const uint32_t *meta, const double *x,
                         const double *b, double *y, const int32_t *done) {
  if (n > 0) IMSMG_CSR_LN(ln, k_csr_residual, n, A, meta, x, b, y, done)
}
template <typename V>
static void csr_residual_smooth(hipStream_t s, int n, int ln, const CsrView<V> &A, const uint32_t *meta,
                                const double *c, const double *xa, const double *r, double *rh, double *xb,
                                const int32_t *done) {
  if (n > 0) IMSMG_CSR_LN(ln, k_csr_residual_smooth, n, A, meta, c, xa, r, rh, xb, done)
}
#undef IMSMG_CSR_LN

void launch_csr_residual(hipStream_t s, int n, int ln, const CsrView<double> &A, const uint32_t *meta,
                         const double *x, const double *b, double *y, const int32_t *done) {
  csr_residual<double>(s, n, ln, A, meta, x, b, y, done);
}
void launch_csr_residual(hipStream_t s, int n, int ln, const CsrView<float> &A, const uint32_t *meta,
                         const double *x, const double *b, double *y, const int32_t *done) {
  csr_residual<float>(s, n, ln, A, meta, x, b, y, done);
}
void launch_csr_residual_smooth(hipStream_t s, int n, int ln, const CsrView<double> &A, const uint32_t *meta,
                                const double *c, const double *xa, const double *r, double *rh, double *xb,
                                const int32_t *done) {
  csr_residual_smooth<double>(s, n, ln, A, meta, c, xa, r, rh, xb, done);
}
void launch_csr_residual_smooth(hipStream_t s, int n, int ln, const CsrView<float> &A, const uint32_t *meta,
                                const double *c, const double *xa, const double *r, double *rh, double *xb,
                                const int32_t *done) {
  csr_residual_smooth<float>(s, n, ln, A, meta, c, xa, r, rh, xb, done);
}

// Vector levels (vec_row.h): one workgroup per (lattice tile, output
// component); the epilogues are the scalar ones on component c's vectors.
template <int K, typename V>
__global__ __launch_bounds__(kRowBlock, kTileBlocksPerCU) void k_vresidual(VecOps<V> ops,
                                                         const uint32_t *__restrict__ flags,
                                                         const double *__restrict__ x, const double *__restrict__ b,
                                                         double *__restrict__ y, const int32_t *__restrict__ done) {
  __shared__ double tile[VecShape<K>::LDS_DOUBLES];
  const int c = blockIdx.y;
  const int64_t o = c * ops.cstride;
  vtile_rows<K, V>(xcd_block(blockIdx.x, gridDim.x), c, ops, flags, x, tile, ResidualEpi{b ? b + o : nullptr, y + o},
                   done);
}

template <int K, typename V>
__global__ __launch_bounds__(kRowBlock, kTileBlocksPerCU) void k_vresidual_smooth(
    VecOps<V> ops, const uint32_t *__restrict__ flags, const double *__restrict__ cd, const double *__restrict__ xa,
    const double *__restrict__ r, double *__restrict__ rh, double *__restrict__ xb, const int32_t *__restrict__ done) {
  __shared__ double tile[VecShape<K>::LDS_DOUBLES];
  const int c = blockIdx.y;
  const int64_t o = c * ops.cstride;
  vtile_rows<K, V>(xcd_block(blockIdx.x, gridDim.x), c, ops, flags, xa, tile,
                   SmoothEpi{r + o, cd + size_t(c) * ops.ns, rh + o, xb + o}, done);
}

template <typename V>
static void dispatch_vresidual(hipStream_t s, int K, const VecOps<V> &ops, const uint32_t *flags, const double *x,
                               const double *b, double *y, const int32_t *done) {
  if (ops.ns <= 0) return;
  dim3 g(ops.ntiles, ops.ncomp), t(kRowBlock);
  if (K == 125)
    k_vresidual<125, V><<<g, t, 0, s>>>(ops, flags, x, b, y, done);
  else if (K == 27)
    k_vresidual<27, V><<<g, t, 0, s>>>(ops, flags, x, b, y, done);
  else
    throw std::invalid_argument("vector operators: 3D tiled stencils (K = 27 or 125)");
}

template <typename V>
static void dispatch_vresidual_smooth(hipStream_t s, int K, const VecOps<V> &ops, const uint32_t *flags,
                                      const double *c, const double *xa, const double *r, double *rh, double *xb,
                                      const int32_t *done) {
  if (ops.ns <= 0) return;
  dim3 g(ops.ntiles, ops.ncomp), t(kRowBlock);
  if (K == 125)
    k_vresidual_smooth<125, V><<<g, t, 0, s>>>(ops, flags, c, xa, r, rh, xb, done);
  else if (K == 27)
    k_vresidual_smooth<27, V><<<g, t, 0, s>>>(ops, flags, c, xa, r, rh, xb, done);
  else
    throw std::invalid_argument("vector operators: 3D tiled stencils (K = 27 or 125)");
}

void launch_vresidual(hipStream_t s, int K, const VecOps<double> &ops, const uint32_t *flags, const double *x,
                      const double *b, double *y, const int32_t *done) {
  dispatch_vresidual<double>(s, K, ops, flags, x, b, y, done);
}
void launch_vresidual(hipStream_t s, int K, const VecOps<float> &ops, const uint32_t *flags, const double *x,
                      const double *b, double *y, const int32_t *done) {
  dispatch_vresidual<float>(s, K, ops, flags, x, b, y, done);
}
void launch_vresidual_smooth(hipStream_t s, int K, const VecOps<double> &ops, const uint32_t *flags, const double *c,
                             const double *xa, const double *r, double *rh, double *xb, const int32_t *done) {
  dispatch_vresidual_smooth<double>(s, K, ops, flags, c, xa, r, rh, xb, done);
}
void launch_vresidual_smooth(hipStream_t s, int K, const VecOps<float> &ops, const uint32_t *flags, const double *c,
                             const double *xa, const double *r, double *rh, double *xb, const int32_t *done) {
  dispatch_vresidual_smooth<float>(s, K, ops, flags, c, xa, r, rh, xb, done);
}

// General Schwarz rows: x[L_t] += sum_k S_G[t,k] r[col_k].  S_G is the sum of
// omega_j P_j A_j^{-1} P_j^T over the general blocks, restricted to the rows
// that belong to one, assembled once at factorization; applying it is a CSR
// product with lattice column positions (deterministic, no atomics).  LANES
// lanes share a row (entries k0 + lane, k0 + lane + LANES, ...: coalesced
// index and value loads, LANES times the rows' parallelism), then add their
// sums in a fixed shuffle order; LANES (2, 4, 8) is chosen per level.
template <int LANES>
__global__ __launch_bounds__(kRowBlock) void k_smooth_general(int ng, const int32_t *__restrict__ grow_lat,
                                                              const int32_t *__restrict__ sptr,
                                                              const int32_t *__restrict__ scol,
                                                              const double *__restrict__ sval,
                                                              const double *__restrict__ r, double *__restrict__ x,
                                                              const int32_t *__restrict__ done) {
  if (done && *done) return;
  const int gt = xcd_block(blockIdx.x, gridDim.x) * kRowBlock + threadIdx.x;
  const int t = gt / LANES, sub = gt % LANES;
  if (t >= ng) return;  // all lanes of a row leave together
  const int k0 = sptr[t], k1 = sptr[t + 1];
  const int L = grow_lat[t];
  // the row's own x, fetched with the row bounds (only this row writes it)
  const double x0 = sub == 0 ? x[L] : 0.0;
  double acc = 0.0;
  // chunks of 4 entries per lane with guarded, fixed trip counts: the index,
  // value and r loads of a chunk issue together
  for (int kb = k0 + sub; kb < k1; kb += 4 * LANES) {
    int c[4];
    double v[4], rv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = kb + q * LANES;
      const bool in = k < k1;
      c[q] = scol[in ? k : kb];
      v[q] = in ? sval[k] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) rv[q] = r[c[q]];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc += v[q] * rv[q];
  }
#pragma unroll
  for (int o = 1; o < LANES; o <<= 1) acc += __shfl_xor(acc, o, LANES);
  if (sub == 0) x[L] = x0 + acc;
}

void launch_smooth_general(hipStream_t s, int ng, const int32_t *grow_lat, const int32_t *sptr,
                           const int32_t *scol, const double *sval, const double *r, double *x, const int32_t *done,
                           int lanes) {
  if (ng <= 0) return;
  switch (lanes) {
    case 2:
      k_smooth_general<2><<<grid_for(ng * 2), kRowBlock, 0, s>>>(ng, grow_lat, sptr, scol, sval, r, x, done);
      break;
    case 8:
      k_smooth_general<8><<<grid_for(ng * 8), kRowBlock, 0, s>>>(ng, grow_lat, sptr, scol, sval, r, x, done);
      break;
    default:
      k_smooth_general<4><<<grid_for(ng * 4), kRowBlock, 0, s>>>(ng, grow_lat, sptr, scol, sval, r, x, done);
      break;
  }
}

// one thread per general row: adds row a of every block holding the row into
// the row's CSR slots, blocks in ascending order (fixed summation order)
__global__ void k_assemble_sg(int ng, const int32_t *__restrict__ gptr, const int64_t *__restrict__ ent_off,
                              const int32_t *__restrict__ ent_n, const int64_t *__restrict__ ent_pos,
                              const int32_t *__restrict__ epos, const double *__restrict__ winv,
                              double *__restrict__ sval) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ng) return;
  for (int e = gptr[t]; e < gptr[t + 1]; ++e) {
    const double *w = winv + ent_off[e];
    const int32_t *pos = epos + ent_pos[e];
    for (int b = 0; b < ent_n[e]; ++b) sval[pos[b]] += w[b];
  }
}

void launch_assemble_sg(hipStream_t s, int ng, const int32_t *gptr, const int64_t *ent_off, const int32_t *ent_n,
                        const int64_t *ent_pos, const int32_t *epos, const double *winv, double *sval) {
  if (ng > 0) k_assemble_sg<<<(ng + 255) / 256, 256, 0, s>>>(ng, gptr, ent_off, ent_n, ent_pos, epos, winv, sval);
}

// x[L_i] = c_i r[L_i]  (trivial part of the first smoothing step from x = 0)
__global__ __launch_bounds__(kRowBlock) void k_diag_scale(int n, const int32_t *__restrict__ row_lat,
                                                          const double *__restrict__ c, const double *__restrict__ r,
                                                          double *__restrict__ x, const int32_t *__restrict__ done) {
  if (done && *done) return;
  const int i = xcd_block(blockIdx.x, gridDim.x) * kRowBlock + threadIdx.x;
  if (i >= n) return;
  const int L = row_lat[i];
  x[L] = c[i] * r[L];
}

void launch_diag_scale(hipStream_t s, int n, const int32_t *row_lat, const double *c, const double *r, double *x,
                       const int32_t *done) {
  if (n > 0) k_diag_scale<<<grid_for(n), kRowBlock, 0, s>>>(n, row_lat, c, r, x, done);
}

// ELL gather (transfer through stored CSR): y[lat_row[i]] (+)= sum_s v[s n + i] x[col[s n + i]];
// optionally also xinit[lat] = cinit[i] * result (first smoothing step of the level)
__global__ __launch_bounds__(kRowBlock) void k_ell_gather(int n, int w, const int32_t *__restrict__ row_lat,
                                                          const int32_t *__restrict__ col,
                                                          const double *__restrict__ v, const double *__restrict__ x,
                                                          double *__restrict__ y, int accumulate,
                                                          const double *__restrict__ cinit,
                                                          double *__restrict__ xinit,
                                                          const int32_t *__restrict__ done) {
  if (done && *done) return;
  const int i = xcd_block(blockIdx.x, gridDim.x) * kRowBlock + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
#pragma unroll 8
  for (int s = 0; s < w; ++s) acc += v[size_t(s) * n + i] * x[col[size_t(s) * n + i]];
  const int L = row_lat[i];
  const double out = accumulate ? y[L] + acc : acc;
  y[L] = out;
  if (xinit) xinit[L] = cinit[i] * out;
}

void launch_ell_gather(hipStream_t s, int n, int w, const int32_t *row_lat, const int32_t *col, const double *v,
                       const double *x, double *y, int accumulate, const double *cinit, double *xinit,
                       const int32_t *done) {
  if (n <= 0) return;
  k_ell_gather<<<grid_for(n), kRowBlock, 0, s>>>(n, w, row_lat, col, v, x, y, accumulate, cinit, xinit, done);
}

// Index-free transfers R_l = tensor product of one 1D two-scale matrix
// (eq:coarsening on the tensor grid), restricted to active functions.  The
// vectors are zero at inactive lattice points, so the full tensor stencil can
// be applied without a mask.  Band: per 1D index, start of the band in the
// other level's 1D numbering, band length, and the band coefficients
// (stride W).
struct Band {
  const int32_t *start;
  const int32_t *len;
  const double *coef;
  int W;
};

// DIM = 3, WB > 0: every band has at most WB entries (WB = the band width,
// 2 .. 4 in practice), the row's loads unrolled slice by slice
template <int DIM, int WB = 0>
__global__ __launch_bounds__(kRowBlock) void k_tensor_transfer(int n, const int32_t *__restrict__ row_lat,
                                                               int ox, int oy, Band band, int ix_, int iy_,
                                                               const double *__restrict__ xin,
                                                               double *__restrict__ y, int accumulate,
                                                               const double *__restrict__ cinit,
                                                               double *__restrict__ xinit,
                                                               const int32_t *__restrict__ done) {
  // rows: this level (lattice ox x oy x .), inputs: other level (lattice ix_ x iy_ x .)
  if (done && *done) return;
  const int i = xcd_block(blockIdx.x, gridDim.x) * kRowBlock + threadIdx.x;
  if (i >= n) return;
  const int L = row_lat[i];
  const int mx = L % ox;
  const int my = (L / ox) % oy;
  const int mz = DIM == 3 ? L / (ox * oy) : 0;
  const int sx = band.start[mx], nx = band.len[mx];
  const int sy = band.start[my], ny = band.len[my];
  const double *cx = band.coef + size_t(mx) * band.W;
  const double *cy = band.coef + size_t(my) * band.W;
  double acc = 0.0;
  if (DIM == 2 && band.W <= kBandMax) {
    // fixed trip counts with guards: every coefficient and input load of the
    // row issues before the first wait
    double cxv[kBandMax], cyv[kBandMax];
#pragma unroll
    for (int a = 0; a < kBandMax; ++a) {
      cxv[a] = a < nx ? cx[a] : 0.0;
      cyv[a] = a < ny ? cy[a] : 0.0;
    }
    double in[kBandMax][kBandMax];
#pragma unroll
    for (int b = 0; b < kBandMax; ++b)
#pragma unroll
      for (int a = 0; a < kBandMax; ++a)
        in[b][a] = (a < nx && b < ny) ? xin[size_t(sy + b) * ix_ + sx + a] : 0.0;
#pragma unroll
    for (int b = 0; b < kBandMax; ++b) {
      double t = 0.0;
#pragma unroll
      for (int a = 0; a < kBandMax; ++a) t += cxv[a] * in[b][a];
      acc += cyv[b] * t;
    }
  } else if (DIM == 2) {
    for (int b = 0; b < ny; ++b) {
      const double *row = xin + size_t(sy + b) * ix_ + sx;
      double t = 0.0;
      for (int a = 0; a < nx; ++a) t += cx[a] * row[a];
      acc += cy[b] * t;
    }
  } else if (DIM == 3 && WB > 0) {
    // fixed trip counts with guards: per z slice, every input load of the
    // slice issues before the first wait (the loop form chains up to
    // (p+2)^3 dependent loads per row)
    constexpr int B = WB > 0 ? WB : 1;
    const int sz = band.start[mz], nz = band.len[mz];
    const double *cz = band.coef + size_t(mz) * band.W;
    double cxv[B], cyv[B], czv[B];
#pragma unroll
    for (int a = 0; a < B; ++a) {
      cxv[a] = a < nx ? cx[a] : 0.0;
      cyv[a] = a < ny ? cy[a] : 0.0;
      czv[a] = a < nz ? cz[a] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < B; ++c) {
      double in[B][B];
#pragma unroll
      for (int b = 0; b < B; ++b)
#pragma unroll
        for (int a = 0; a < B; ++a) {
          in[b][a] = 0.0;
          if (a < nx && b < ny && c < nz) in[b][a] = xin[(size_t(sz + c) * iy_ + (sy + b)) * ix_ + sx + a];
        }
      double tz = 0.0;
#pragma unroll
      for (int b = 0; b < B; ++b) {
        double t = 0.0;
#pragma unroll
        for (int a = 0; a < B; ++a) t += cxv[a] * in[b][a];
        tz += cyv[b] * t;
      }
      acc += czv[c] * tz;
    }
  } else {
    const int sz = band.start[mz], nz = band.len[mz];
    const double *cz = band.coef + size_t(mz) * band.W;
    for (int c = 0; c < nz; ++c) {
      double tz = 0.0;
      for (int b = 0; b < ny; ++b) {
        const double *row = xin + (size_t(sz + c) * iy_ + (sy + b)) * ix_ + sx;
        double t = 0.0;
        for (int a = 0; a < nx; ++a) t += cx[a] * row[a];
        tz += cy[b] * t;
      }
      acc += cz[c] * tz;
    }
  }
  const double out = accumulate ? y[L] + acc : acc;
  y[L] = out;
  if (xinit) xinit[L] = cinit[i] * out;
}

void launch_tensor_transfer(hipStream_t s, int dim, int n, const int32_t *row_lat, int ox, int oy,
                            const int32_t *start, const int32_t *len, const double *coef, int W, int ix, int iy,
                            const double *xin, double *y, int accumulate, const double *cinit, double *xinit,
                            const int32_t *done) {
  if (n <= 0) return;
  Band b{start, len, coef, W};
  if (dim == 2)
    k_tensor_transfer<2><<<grid_for(n), kRowBlock, 0, s>>>(n, row_lat, ox, oy, b, ix, iy, xin, y, accumulate, cinit,
                                                           xinit, done);
  else if (W == 2)
    k_tensor_transfer<3, 2><<<grid_for(n), kRowBlock, 0, s>>>(n, row_lat, ox, oy, b, ix, iy, xin, y, accumulate,
                                                              cinit, xinit, done);
  else if (W == 3)
    k_tensor_transfer<3, 3><<<grid_for(n), kRowBlock, 0, s>>>(n, row_lat, ox, oy, b, ix, iy, xin, y, accumulate,
                                                              cinit, xinit, done);
  else if (W == 4)
    k_tensor_transfer<3, 4><<<grid_for(n), kRowBlock, 0, s>>>(n, row_lat, ox, oy, b, ix, iy, xin, y, accumulate,
                                                              cinit, xinit, done);
  else
    k_tensor_transfer<3><<<grid_for(n), kRowBlock, 0, s>>>(n, row_lat, ox, oy, b, ix, iy, xin, y, accumulate, cinit,
                                                           xinit, done);
}

// Dense coarsest solve: r gathered into LDS, one wavefront per output row.
// Large coarsest levels: 16 rows per workgroup share one gathered copy of r
// (with 4 rows per workgroup the gathers of r moved a quarter as many bytes
// as A^-1 itself); small ones keep 4 rows per workgroup, so that enough
// workgroups run.
constexpr int kGemvThreads = 1024;
__global__ __launch_bounds__(kGemvThreads) void k_dense_gemv(int n, const int32_t *__restrict__ row_lat,
                                                             const double *__restrict__ Ainv,
                                                             const double *__restrict__ r, double *__restrict__ x,
                                                             const int32_t *__restrict__ done) {
  if (done && *done) return;
  extern __shared__ double rs[];
  // gather r in batches of 8 per thread: indices first, then values, so that
  // the loads of a batch are in flight together
  const int nt = blockDim.x;
  for (int j0 = threadIdx.x; j0 < n; j0 += 4 * nt) {
    // unconditional loads at clamped positions: no wait between them
    int idx[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) idx[q] = row_lat[min(j0 + q * nt, n - 1)];
    double val[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) val[q] = r[idx[q]];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (j0 + q * nt < n) rs[j0 + q * nt] = val[q];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int rows_per_block = nt / 64;
  const int i = blockIdx.x * rows_per_block + wave;
  if (i >= n) return;
  const double *row = Ainv + size_t(i) * n;
  double acc = 0.0;
#pragma unroll 8
  for (int j = lane; j < n; j += 64) acc += row[j] * rs[j];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if (lane == 0) x[row_lat[i]] = acc;
}

void launch_dense_gemv(hipStream_t s, int n, const int32_t *row_lat, const double *Ainv, const double *r, double *x,
                       const int32_t *done) {
  if (n <= 0) return;
  const int nt = n >= 2048 ? kGemvThreads : 256;
  const int rpb = nt / 64;
  k_dense_gemv<<<(n + rpb - 1) / rpb, nt, size_t(n) * sizeof(double), s>>>(n, row_lat, Ainv, r, x, done);
}

__global__ void k_scatter(int n, const int32_t *__restrict__ row_lat, const double *__restrict__ src,
                          double *__restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[row_lat[i]] = src[i];
}
__global__ void k_gather(int n, const int32_t *__restrict__ row_lat, const double *__restrict__ src,
                         double *__restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[row_lat[i]];
}

void launch_scatter(hipStream_t s, int n, const int32_t *row_lat, const double *src, double *dst) {
  if (n > 0) k_scatter<<<grid_for(n), kRowBlock, 0, s>>>(n, row_lat, src, dst);
}
void launch_gather(hipStream_t s, int n, const int32_t *row_lat, const double *src, double *dst) {
  if (n > 0) k_gather<<<grid_for(n), kRowBlock, 0, s>>>(n, row_lat, src, dst);
}

}  // namespace imsmg
