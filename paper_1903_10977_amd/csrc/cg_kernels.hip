// Conjugate-gradient kernels on the finest level (the paragraph after
// Algorithm alg:MGV: the symmetric V-cycle preconditions CG).
//
// Every dot product is reduced deterministically in two kernels: each
// workgroup of the streaming kernel writes one partial sum (fixed thread
// order, fixed LDS tree), then a one-workgroup finalize kernel adds the
// partials in index order and derives the CG scalars on the device, so no
// host round trip is needed inside an iteration.  The kernel boundary orders
// the partial stores; no device-scope fence (an L2 write-back on a multi-XCD
// part) is issued per workgroup.  Once the `done` flag is set, every kernel
// returns at once.
#include <stdexcept>

#include "csr_row.h"
#include "imsmg_internal.h"
#include "op_row.h"
#include "vec_row.h"

namespace imsmg {

constexpr int kRedThreads = 256;
static_assert(kRedThreads == kTileRows, "stencil kernels: one lattice point or row per thread");
constexpr int kFinThreads = 1024;

int reduction_blocks(int n) { return n < 1 ? 1 : (n + kRedThreads - 1) / kRedThreads; }

__device__ __forceinline__ int xcd_block_cg(int b, int nb) {
  const int per = (nb + 7) / 8;
  const int xcd = b % 8;
  const int k = b / 8;
  const int full = nb % 8 == 0 ? 8 : nb % 8;
  if (xcd < full) return xcd * per + k;
  return full * per + (xcd - full) * (per - 1) + k;
}

// workgroup sum in a fixed order: a lane-shuffle tree per wavefront, then the
// NT / 64 wavefront sums in index order (one barrier instead of log2 NT)
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *lds) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) r += lds[w];
  __syncthreads();
  return r;
}

// ordered sum of part[0 .. m) by one workgroup
__device__ __forceinline__ double sum_partials(const double *__restrict__ part, int m, double *lds) {
  double v = 0.0;
  // chunks of 4 per thread, loads issued together, added in index order
  for (int b0 = threadIdx.x; b0 < m; b0 += 4 * kFinThreads) {
    double w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = b0 + q * kFinThreads < m ? part[b0 + q * kFinThreads] : 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) v += w[q];
  }
  return block_sum<kFinThreads>(v, lds);
}

// r = b - A x, accumulating (||r||^2, ||b||^2)
struct InitEpi {
  const double *__restrict__ b;
  double *__restrict__ r;
  struct Pre {
    double b;
  };
  __device__ Pre pre(int, int L) const { return {b[L]}; }
  __device__ double2 post(int, int L, unsigned, double ax, double, const Pre &p) const {
    const double ri = p.b - ax;
    r[L] = ri;
    return make_double2(ri * ri, p.b * p.b);
  }
};

// q = A p, accumulating p . q
struct SpmvEpi {
  double *__restrict__ q;
  struct Pre {};
  __device__ Pre pre(int, int) const { return {}; }
  __device__ double2 post(int, int L, unsigned, double ax, double pc, const Pre &) const {
    q[L] = ax;
    return make_double2(pc * ax, 0.0);
  }
};

// accumulates ||b - A x||^2
struct TrueResEpi {
  const double *__restrict__ b;
  struct Pre {
    double b;
  };
  __device__ Pre pre(int, int L) const { return {b[L]}; }
  __device__ double2 post(int, int, unsigned, double ax, double, const Pre &p) const {
    const double ri = p.b - ax;
    return make_double2(ri * ri, 0.0);
  }
};

// r = b - A x; partials of ||r||^2 (part[0..g)) and ||b||^2 (part[g..2g))
template <int K, bool NT>
__global__ __launch_bounds__(kRedThreads, kTileBlocksPerCU) void k_cg_init(int n, int Kdyn, OpView<double> op,
                                                         const int32_t *__restrict__ row_lat,
                                                         const uint32_t *__restrict__ meta,
                                                         const double *__restrict__ x,
                                                         const double *__restrict__ b, double *__restrict__ r,
                                                         double *__restrict__ part) {
  __shared__ double lds[kRedThreads];
  __shared__ double tile[StencilShape<K>::LDS_DOUBLES];
  const int blk = xcd_block_cg(blockIdx.x, gridDim.x);
  const double2 s = tile_rows<K, double, InitEpi, false, NT>(n, blk, op, row_lat, meta, x, tile, Kdyn, InitEpi{b, r});
  double rr = s.x, bb = s.y;
  rr = block_sum<kRedThreads>(rr, lds);
  bb = block_sum<kRedThreads>(bb, lds);
  if (threadIdx.x == 0) {
    part[blk] = rr;
    part[gridDim.x + blk] = bb;
  }
}

// Stopping threshold ||r_k|| <= rtol min(||r_0||, ||b||) (equal for x_0 = 0;
// with a start x_0 whose residual exceeds ||b|| the threshold still aims at
// the true relative residual ||b - A x|| / ||b||).  restart != 0: CG
// restarted from the current iterate; the threshold and the iteration count of
// the first start are kept.
__global__ __launch_bounds__(kFinThreads) void k_cg_init_fin(int m, const double *__restrict__ part, CGState *st,
                                                             double rtol, int restart) {
  __shared__ double lds[kFinThreads];
  const double rr = sum_partials(part, m, lds);
  const double bb = sum_partials(part + m, m, lds);
  if (threadIdx.x == 0) {
    if (!restart) {
      st->r0sq = rr;
      st->tol2 = rtol * rtol * (rr < bb ? rr : bb);
      st->iters = 0;
    }
    st->rr = rr;
    st->bb = bb;
    st->first = 1;
    st->status = 0;
    st->beta = 0.0;
    st->done = (rr == 0.0) ? 1 : 0;
    if (!(rr == rr) || !(bb == bb)) {
      st->status = -6;
      st->done = 1;
    }
  }
}

__global__ __launch_bounds__(kRedThreads) void k_cg_dot_rz(int n, const int32_t *__restrict__ row_lat,
                                                           const double *__restrict__ r,
                                                           const double *__restrict__ z, double *__restrict__ part,
                                                           const CGState *st) {
  if (st->done) return;
  __shared__ double lds[kRedThreads];
  const int blk = xcd_block_cg(blockIdx.x, gridDim.x);
  const int i = blk * kRedThreads + threadIdx.x;
  // unconditional loads at a clamped row (n >= 1), then a select
  const int L = row_lat[min(i, n - 1)];
  const double rz = r[L] * z[L];
  double acc = i < n ? rz : 0.0;
  acc = block_sum<kRedThreads>(acc, lds);
  if (threadIdx.x == 0) part[blk] = acc;
}

// beta: Hestenes-Stiefel r_{k+1}.z_{k+1} / r_k.z_k, or (flexible) the
// Polak-Ribiere form (r_{k+1}.z_{k+1} - r_{k+1}.z_k) / r_k.z_k, whose second
// term the update kernel reduced while z_k was still in place; both agree
// in exact arithmetic when the preconditioner is one fixed SPD operator
__global__ __launch_bounds__(kFinThreads) void k_cg_rz_fin(int m, const double *__restrict__ part, CGState *st,
                                                           int flexible) {
  if (st->done) return;
  __shared__ double lds[kFinThreads];
  const double tot = sum_partials(part, m, lds);
  if (threadIdx.x == 0) {
    st->rz_old = st->rz;
    st->rz = tot;
    st->beta = st->first ? 0.0 : (flexible ? tot - st->rz_mix : tot) / st->rz_old;
    if (!(tot == tot)) {
      st->status = -6;
      st->done = 1;
    }
  }
}

__global__ __launch_bounds__(kRedThreads) void k_cg_direction(int n, const int32_t *__restrict__ row_lat,
                                                              const double *__restrict__ z, double *__restrict__ p,
                                                              const CGState *st) {
  if (st->done) return;
  const double beta = st->beta;
  const bool first = st->first != 0;
  const int i = xcd_block_cg(blockIdx.x, gridDim.x) * kRedThreads + threadIdx.x;
  if (i >= n) return;
  const int L = row_lat[i];
  p[L] = first ? z[L] : z[L] + beta * p[L];
}

template <int K, bool NT>
__global__ __launch_bounds__(kRedThreads, kTileBlocksPerCU) void k_cg_spmv_pq(int n, int Kdyn, OpView<double> op,
                                                            const int32_t *__restrict__ row_lat,
                                                            const uint32_t *__restrict__ meta,
                                                            const double *__restrict__ p, double *__restrict__ q,
                                                            double *__restrict__ part, const CGState *st) {
  __shared__ double lds[kRedThreads];
  __shared__ double tile[StencilShape<K>::LDS_DOUBLES];
  const int blk = xcd_block_cg(blockIdx.x, gridDim.x);
  double acc = tile_rows<K, double, SpmvEpi, false, NT>(n, blk, op, row_lat, meta, p, tile, Kdyn, SpmvEpi{q}, &st->done).x;
  if (st->done) return;  // uniform: the flag does not change during the kernel
  acc = block_sum<kRedThreads>(acc, lds);
  if (threadIdx.x == 0) part[blk] = acc;
}

__global__ __launch_bounds__(kFinThreads) void k_cg_pq_fin(int m, const double *__restrict__ part, CGState *st) {
  if (st->done) return;
  __shared__ double lds[kFinThreads];
  const double tot = sum_partials(part, m, lds);
  if (threadIdx.x == 0) {
    st->pq = tot;
    st->first = 0;
    if (!(tot > 0.0)) {
      st->status = (tot == tot) ? -4 : -6;
      st->done = 1;
      st->alpha = 0.0;
    } else {
      st->alpha = st->rz / tot;
    }
  }
}

// FLEX: also the partials of r_{k+1} . z_k into part[gridDim.x + blk]; zs
// may be the buffer holding z_k (then each lane reads its z_k before it
// writes zs at the same index), so neither pointer is restrict-qualified
template <bool FLEX>
__global__ __launch_bounds__(kRedThreads) void k_cg_update(int n, const int32_t *__restrict__ row_lat,
                                                           const double *__restrict__ p,
                                                           const double *__restrict__ q, double *__restrict__ x,
                                                           double *__restrict__ r, const double *__restrict__ c,
                                                           double *zs, const double *zk, double *__restrict__ part,
                                                           const CGState *st) {
  if (st->done) return;
  __shared__ double lds[kRedThreads];
  const double alpha = st->alpha;
  const int blk = xcd_block_cg(blockIdx.x, gridDim.x);
  const int i = blk * kRedThreads + threadIdx.x;
  double acc = 0.0, mix = 0.0;
  if (i < n) {
    const int L = row_lat[i];
    x[L] += alpha * p[L];
    const double ri = r[L] - alpha * q[L];
    r[L] = ri;
    if (FLEX) mix = ri * zk[L];
    zs[L] = c[i] * ri;
    acc = ri * ri;
  }
  acc = block_sum<kRedThreads>(acc, lds);
  if (threadIdx.x == 0) part[blk] = acc;
  if (FLEX) {
    mix = block_sum<kRedThreads>(mix, lds);
    if (threadIdx.x == 0) part[gridDim.x + blk] = mix;
  }
}

__global__ __launch_bounds__(kFinThreads) void k_cg_update_fin(int m, const double *__restrict__ part, CGState *st,
                                                               int max_iter, int flexible) {
  if (st->done) return;
  __shared__ double lds[kFinThreads];
  const double tot = sum_partials(part, m, lds);
  const double mix = flexible ? sum_partials(part + m, m, lds) : 0.0;
  if (threadIdx.x == 0) {
    st->rz_mix = mix;
    st->rr = tot;
    st->iters += 1;
    if (!(tot == tot)) {
      st->status = -6;
      st->done = 1;
    } else if (tot <= st->tol2) {
      st->done = 1;
    } else if (st->iters >= max_iter) {
      st->status = -5;
      st->done = 1;
    }
  }
}

// partials of ||b - A x||^2
template <int K, bool NT>
__global__ __launch_bounds__(kRedThreads, kTileBlocksPerCU) void k_cg_true_residual(int n, int Kdyn, OpView<double> op,
                                                                  const int32_t *__restrict__ row_lat,
                                                                  const uint32_t *__restrict__ meta,
                                                                  const double *__restrict__ x,
                                                                  const double *__restrict__ b,
                                                                  double *__restrict__ part) {
  __shared__ double lds[kRedThreads];
  __shared__ double tile[StencilShape<K>::LDS_DOUBLES];
  const int blk = xcd_block_cg(blockIdx.x, gridDim.x);
  double acc = tile_rows<K, double, TrueResEpi, false, NT>(n, blk, op, row_lat, meta, x, tile, Kdyn, TrueResEpi{b}).x;
  acc = block_sum<kRedThreads>(acc, lds);
  if (threadIdx.x == 0) part[blk] = acc;
}

__global__ __launch_bounds__(kFinThreads) void k_cg_aux_fin(int m, const double *__restrict__ part, CGState *st) {
  __shared__ double lds[kFinThreads];
  const double tot = sum_partials(part, m, lds);
  if (threadIdx.x == 0) st->aux = tot;
}

// Vector finest level: one workgroup per (lattice tile, component), partial
// sums at blockIdx.y * gridDim.x + tile (the finalize adds them in index order).
template <int K>
__global__ __launch_bounds__(kRedThreads, kTileBlocksPerCU) void k_vcg_init(VecOps<double> ops,
                                                          const uint32_t *__restrict__ flags,
                                                          const double *__restrict__ x,
                                                          const double *__restrict__ b, double *__restrict__ r,
                                                          double *__restrict__ part) {
  __shared__ double lds[kRedThreads];
  __shared__ double tile[VecShape<K>::LDS_DOUBLES];
  const int blk = xcd_block_cg(blockIdx.x, gridDim.x);
  const int c = blockIdx.y;
  const int64_t o = c * ops.cstride;
  const double2 sm = vtile_rows<K, double>(blk, c, ops, flags, x, tile, InitEpi{b + o, r + o}, nullptr);
  const double rr = block_sum<kRedThreads>(sm.x, lds);
  const double bb = block_sum<kRedThreads>(sm.y, lds);
  const int f = c * gridDim.x + blk, m = gridDim.x * gridDim.y;
  if (threadIdx.x == 0) {
    part[f] = rr;
    part[m + f] = bb;
  }
}

template <int K>
__global__ __launch_bounds__(kRedThreads, kTileBlocksPerCU) void k_vcg_spmv_pq(VecOps<double> ops,
                                                             const uint32_t *__restrict__ flags,
                                                             const double *__restrict__ p, double *__restrict__ q,
                                                             double *__restrict__ part, const CGState *st) {
  __shared__ double lds[kRedThreads];
  __shared__ double tile[VecShape<K>::LDS_DOUBLES];
  const int blk = xcd_block_cg(blockIdx.x, gridDim.x);
  const int c = blockIdx.y;
  const int64_t o = c * ops.cstride;
  double acc = vtile_rows<K, double>(blk, c, ops, flags, p, tile, SpmvEpi{q + o}, &st->done).x;
  if (st->done) return;
  acc = block_sum<kRedThreads>(acc, lds);
  if (threadIdx.x == 0) part[c * gridDim.x + blk] = acc;
}

template <int K>
__global__ __launch_bounds__(kRedThreads, kTileBlocksPerCU) void k_vcg_true_residual(VecOps<double> ops,
                                                                   const uint32_t *__restrict__ flags,
                                                                   const double *__restrict__ x,
                                                                   const double *__restrict__ b,
                                                                   double *__restrict__ part) {
  __shared__ double lds[kRedThreads];
  __shared__ double tile[VecShape<K>::LDS_DOUBLES];
  const int blk = xcd_block_cg(blockIdx.x, gridDim.x);
  const int c = blockIdx.y;
  const int64_t o = c * ops.cstride;
  double acc = vtile_rows<K, double>(blk, c, ops, flags, x, tile, TrueResEpi{b + o}, nullptr).x;
  acc = block_sum<kRedThreads>(acc, lds);
  if (threadIdx.x == 0) part[c * gridDim.x + blk] = acc;
}

// General sparse finest level (csr_row.h): LN lanes per CSR row, partial
// sums per workgroup in workgroup order.
template <int LN>
__global__ __launch_bounds__(kRedThreads) void k_csr_cg_init(int n, CsrView<double> A, const double *__restrict__ x,
                                                             const double *__restrict__ b, double *__restrict__ r,
                                                             double *__restrict__ part) {
  __shared__ double lds[kRedThreads];
  const double2 s = csr_rows<LN, double, InitEpi>(n, A, nullptr, x, InitEpi{b, r});
  const double rr = block_sum<kRedThreads>(s.x, lds);
  const double bb = block_sum<kRedThreads>(s.y, lds);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = rr;
    part[gridDim.x + blockIdx.x] = bb;
  }
}

template <int LN>
__global__ __launch_bounds__(kRedThreads) void k_csr_cg_spmv_pq(int n, CsrView<double> A,
                                                                const double *__restrict__ p, double *__restrict__ q,
                                                                double *__restrict__ part, const CGState *st) {
  __shared__ double lds[kRedThreads];
  if (st->done) return;  // uniform: the flag does not change during the kernel
  const double acc = block_sum<kRedThreads>(csr_rows<LN, double, SpmvEpi>(n, A, nullptr, p, SpmvEpi{q}).x, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

template <int LN>
__global__ __launch_bounds__(kRedThreads) void k_csr_cg_true_residual(int n, CsrView<double> A,
                                                                      const double *__restrict__ x,
                                                                      const double *__restrict__ b,
                                                                      double *__restrict__ part) {
  __shared__ double lds[kRedThreads];
  const double acc = block_sum<kRedThreads>(csr_rows<LN, double, TrueResEpi>(n, A, nullptr, x, TrueResEpi{b}).x, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

int csr_part_blocks(int n, int ln) { return csr_grid(n, ln); }

#define IMSMG_CSR_CG(KERNEL, ...)                                                      \
  switch (ln) {                                                                        \
    case 4: KERNEL<4><<<g, kRedThreads, 0, s>>>(__VA_ARGS__); break;                   \
    case 8: KERNEL<8><<<g, kRedThreads, 0, s>>>(__VA_ARGS__); break;                   \
    case 16: KERNEL<16><<<g, kRedThreads, 0, s>>>(__VA_ARGS__); break;                 \
    default: throw std::invalid_argument("CSR rows: 4, 8 or 16 lanes per row");       \
  }

void launch_csr_cg_init(hipStream_t s, int n, int ln, const CsrView<double> &A, const double *x, const double *b,
                        double *r, double *part, CGState *st, double rtol, int restart) {
  const int g = csr_grid(n, ln);
  IMSMG_CSR_CG(k_csr_cg_init, n, A, x, b, r, part)
  k_cg_init_fin<<<1, kFinThreads, 0, s>>>(g, part, st, rtol, restart);
}

void launch_csr_cg_spmv_pq(hipStream_t s, int n, int ln, const CsrView<double> &A, const double *p, double *q,
                           double *part, CGState *st) {
  const int g = csr_grid(n, ln);
  IMSMG_CSR_CG(k_csr_cg_spmv_pq, n, A, p, q, part, st)
  k_cg_pq_fin<<<1, kFinThreads, 0, s>>>(g, part, st);
}

void launch_csr_cg_true_residual(hipStream_t s, int n, int ln, const CsrView<double> &A, const double *x,
                                 const double *b, double *part, CGState *st) {
  const int g = csr_grid(n, ln);
  IMSMG_CSR_CG(k_csr_cg_true_residual, n, A, x, b, part)
  k_cg_aux_fin<<<1, kFinThreads, 0, s>>>(g, part, st);
}
#undef IMSMG_CSR_CG

#define IMSMG_DISPATCH_V(K, KERNEL, ...)                                                 \
  do {                                                                                   \
    const dim3 g2(ops.ntiles, ops.ncomp);                                                \
    if (K == 125)                                                                        \
      KERNEL<125><<<g2, kRedThreads, 0, s>>>(__VA_ARGS__);                               \
    else if (K == 27)                                                                    \
      KERNEL<27><<<g2, kRedThreads, 0, s>>>(__VA_ARGS__);                                \
    else                                                                                 \
      throw std::invalid_argument("vector operators: 3D tiled stencils (K = 27 or 125)"); \
  } while (0)

void launch_vcg_init(hipStream_t s, int K, const VecOps<double> &ops, const uint32_t *flags, const double *x,
                     const double *b, double *r, double *part, CGState *st, double rtol, int restart) {
  IMSMG_DISPATCH_V(K, k_vcg_init, ops, flags, x, b, r, part);
  k_cg_init_fin<<<1, kFinThreads, 0, s>>>(ops.ntiles * ops.ncomp, part, st, rtol, restart);
}

void launch_vcg_spmv_pq(hipStream_t s, int K, const VecOps<double> &ops, const uint32_t *flags, const double *p,
                        double *q, double *part, CGState *st) {
  IMSMG_DISPATCH_V(K, k_vcg_spmv_pq, ops, flags, p, q, part, st);
  k_cg_pq_fin<<<1, kFinThreads, 0, s>>>(ops.ntiles * ops.ncomp, part, st);
}

void launch_vcg_true_residual(hipStream_t s, int K, const VecOps<double> &ops, const uint32_t *flags,
                              const double *x, const double *b, double *part, CGState *st) {
  IMSMG_DISPATCH_V(K, k_vcg_true_residual, ops, flags, x, b, part);
  k_cg_aux_fin<<<1, kFinThreads, 0, s>>>(ops.ntiles * ops.ncomp, part, st);
}
#undef IMSMG_DISPATCH_V

#define IMSMG_DISPATCH_KN(KK, KERNEL, ...)                                               \
  if (op.stream)                                                                         \
    KERNEL<KK, true><<<g, kRedThreads, 0, s>>>(__VA_ARGS__);                             \
  else                                                                                   \
    KERNEL<KK, false><<<g, kRedThreads, 0, s>>>(__VA_ARGS__);
#define IMSMG_DISPATCH_K(K, KERNEL, ...)                                                 \
  switch (K) {                                                                           \
    case 9: IMSMG_DISPATCH_KN(9, KERNEL, __VA_ARGS__) break;                             \
    case 25: IMSMG_DISPATCH_KN(25, KERNEL, __VA_ARGS__) break;                           \
    case 49: IMSMG_DISPATCH_KN(49, KERNEL, __VA_ARGS__) break;                           \
    case 27: IMSMG_DISPATCH_KN(27, KERNEL, __VA_ARGS__) break;                           \
    case 125: IMSMG_DISPATCH_KN(125, KERNEL, __VA_ARGS__) break;                         \
    default: KERNEL<0, false><<<g, kRedThreads, 0, s>>>(__VA_ARGS__); break;            \
  }

void launch_cg_init(hipStream_t s, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                    const uint32_t *meta, const double *x, const double *b, double *r, double *part, CGState *st,
                    double rtol, int restart) {
  require_lattice_op(op);
  const int g = stencil_grid(K, n, op);
  IMSMG_DISPATCH_K(K, k_cg_init, n, K, op, row_lat, meta, x, b, r, part);
  k_cg_init_fin<<<1, kFinThreads, 0, s>>>(g, part, st, rtol, restart);
}

void launch_cg_dot_rz(hipStream_t s, int n, const int32_t *row_lat, const double *r, const double *z, double *part,
                      CGState *st, int flexible) {
  const int g = reduction_blocks(n);
  k_cg_dot_rz<<<g, kRedThreads, 0, s>>>(n, row_lat, r, z, part, st);
  k_cg_rz_fin<<<1, kFinThreads, 0, s>>>(g, part, st, flexible);
}

void launch_cg_direction(hipStream_t s, int n, const int32_t *row_lat, const double *z, double *p, CGState *st) {
  k_cg_direction<<<reduction_blocks(n), kRedThreads, 0, s>>>(n, row_lat, z, p, st);
}

void launch_cg_spmv_pq(hipStream_t s, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                       const uint32_t *meta, const double *p, double *q, double *part, CGState *st) {
  require_lattice_op(op);
  const int g = stencil_grid(K, n, op);
  IMSMG_DISPATCH_K(K, k_cg_spmv_pq, n, K, op, row_lat, meta, p, q, part, st);
  k_cg_pq_fin<<<1, kFinThreads, 0, s>>>(g, part, st);
}

void launch_cg_update(hipStream_t s, int n, const int32_t *row_lat, const double *p, const double *q, double *x,
                      double *r, const double *c, double *zs, const double *zk, double *part, CGState *st,
                      int max_iter) {
  const int g = reduction_blocks(n);
  if (zk)
    k_cg_update<true><<<g, kRedThreads, 0, s>>>(n, row_lat, p, q, x, r, c, zs, zk, part, st);
  else
    k_cg_update<false><<<g, kRedThreads, 0, s>>>(n, row_lat, p, q, x, r, c, zs, nullptr, part, st);
  k_cg_update_fin<<<1, kFinThreads, 0, s>>>(g, part, st, max_iter, zk != nullptr);
}

void launch_cg_true_residual(hipStream_t s, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                             const uint32_t *meta, const double *x, const double *b, double *part, CGState *st) {
  require_lattice_op(op);
  const int g = stencil_grid(K, n, op);
  IMSMG_DISPATCH_K(K, k_cg_true_residual, n, K, op, row_lat, meta, x, b, part);
  k_cg_aux_fin<<<1, kFinThreads, 0, s>>>(g, part, st);
}

}  // namespace imsmg
