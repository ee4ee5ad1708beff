// Conjugate-gradient kernels on the finest level (the paragraph after
// Algorithm alg:MGV: the symmetric V-cycle preconditions CG).
//
// Every dot product is reduced deterministically: each workgroup writes one
// partial sum (fixed thread order, fixed LDS tree), the last workgroup to
// finish (atomic ticket) adds the partials in index order and derives the CG
// scalars on the device, so no host round trip is needed inside an iteration.
// The ticket is reset by that last workgroup, which keeps the kernels
// replayable from a captured graph without any memset node.
// Once the `done` flag is set, every kernel returns at once.
#include "imsmg_internal.h"

namespace imsmg {

constexpr int kRedThreads = 256;
constexpr int kRedMaxBlocks = 2048;

int reduction_blocks(int n) {
  int b = (n + kRedThreads - 1) / kRedThreads;
  return b < 1 ? 1 : (b > kRedMaxBlocks ? kRedMaxBlocks : b);
}

__device__ __forceinline__ double block_sum(double v, double *lds) {
  lds[threadIdx.x] = v;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
    __syncthreads();
  }
  double r = lds[0];
  __syncthreads();
  return r;
}

// Writes this block's partial; returns true in exactly one (the last) block,
// where `total` then holds the ordered sum of all partials.
__device__ __forceinline__ bool finish_reduction(double mine, double *part, uint32_t *ticket, double *lds,
                                                 double &total) {
  __shared__ bool last;
  double bs = block_sum(mine, lds);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = bs;
    __threadfence();
    uint32_t t = atomicAdd(ticket, 1u);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  double v = 0.0;
  for (int b = threadIdx.x; b < int(gridDim.x); b += kRedThreads) v += part[b];
  total = block_sum(v, lds);
  if (threadIdx.x == 0) *ticket = 0u;
  return true;
}

template <int K>
__device__ __forceinline__ double ell_row(int i, int n, const Offsets &off, int L, const double *__restrict__ val,
                                          const double *__restrict__ x, int Kdyn) {
  double acc = 0.0;
  if (K > 0) {
#pragma unroll
    for (int s = 0; s < K; ++s) acc += val[size_t(s) * n + i] * x[L + off.off[s]];
  } else {
    for (int s = 0; s < Kdyn; ++s) acc += val[size_t(s) * n + i] * x[L + off.off[s]];
  }
  return acc;
}

// r = b - A x, ||r0||^2, ||b||^2 (two partial arrays: part and part + gridDim)
template <int K>
__global__ __launch_bounds__(kRedThreads) void k_cg_init(int n, int Kdyn, Offsets off,
                                                         const int32_t *__restrict__ row_lat,
                                                         const double *__restrict__ val, const double *__restrict__ x,
                                                         const double *__restrict__ b, double *__restrict__ r,
                                                         double *__restrict__ part, CGState *st, double rtol) {
  __shared__ double lds[kRedThreads];
  double rr = 0.0, bb = 0.0;
  for (int i = blockIdx.x * kRedThreads + threadIdx.x; i < n; i += gridDim.x * kRedThreads) {
    const int L = row_lat[i];
    const double bi = b[L];
    const double ri = bi - ell_row<K>(i, n, off, L, val, x, Kdyn);
    r[L] = ri;
    rr += ri * ri;
    bb += bi * bi;
  }
  double tot_rr;
  // pack both sums: first reduce bb into the second half of the partials
  double bsum = block_sum(bb, lds);
  if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = bsum;
  if (finish_reduction(rr, part, &st->ticket[T_RESID], lds, tot_rr)) {
    double v = 0.0;
    for (int q = threadIdx.x; q < int(gridDim.x); q += kRedThreads) v += part[gridDim.x + q];
    double tot_bb = block_sum(v, lds);
    if (threadIdx.x == 0) {
      st->r0sq = tot_rr;
      st->rr = tot_rr;
      st->bb = tot_bb;
      st->tol2 = rtol * rtol * tot_rr;
      st->iters = 0;
      st->first = 1;
      st->status = 0;
      st->beta = 0.0;
      st->done = (tot_rr == 0.0) ? 1 : 0;
      if (!(tot_rr == tot_rr) || !(tot_bb == tot_bb)) {
        st->status = -6;
        st->done = 1;
      }
    }
  }
}

__global__ __launch_bounds__(kRedThreads) void k_cg_dot_rz(int n, const int32_t *__restrict__ row_lat,
                                                           const double *__restrict__ r,
                                                           const double *__restrict__ z, double *__restrict__ part,
                                                           CGState *st) {
  if (st->done) return;
  __shared__ double lds[kRedThreads];
  double acc = 0.0;
  for (int i = blockIdx.x * kRedThreads + threadIdx.x; i < n; i += gridDim.x * kRedThreads) {
    const int L = row_lat[i];
    acc += r[L] * z[L];
  }
  double tot;
  if (finish_reduction(acc, part, &st->ticket[T_DOT_RZ], lds, tot)) {
    if (threadIdx.x == 0) {
      st->rz_old = st->rz;
      st->rz = tot;
      st->beta = st->first ? 0.0 : tot / st->rz_old;
      if (!(tot == tot)) {
        st->status = -6;
        st->done = 1;
      }
    }
  }
}

__global__ __launch_bounds__(kRedThreads) void k_cg_direction(int n, const int32_t *__restrict__ row_lat,
                                                              const double *__restrict__ z, double *__restrict__ p,
                                                              CGState *st) {
  if (st->done) return;
  const double beta = st->beta;
  const bool first = st->first != 0;
  const int i = blockIdx.x * kRedThreads + threadIdx.x;
  if (i >= n) return;
  const int L = row_lat[i];
  p[L] = first ? z[L] : z[L] + beta * p[L];
}

template <int K>
__global__ __launch_bounds__(kRedThreads) void k_cg_spmv_pq(int n, int Kdyn, Offsets off,
                                                            const int32_t *__restrict__ row_lat,
                                                            const double *__restrict__ val,
                                                            const double *__restrict__ p, double *__restrict__ q,
                                                            double *__restrict__ part, CGState *st) {
  if (st->done) return;
  __shared__ double lds[kRedThreads];
  double acc = 0.0;
  for (int i = blockIdx.x * kRedThreads + threadIdx.x; i < n; i += gridDim.x * kRedThreads) {
    const int L = row_lat[i];
    const double qi = ell_row<K>(i, n, off, L, val, p, Kdyn);
    q[L] = qi;
    acc += p[L] * qi;
  }
  double tot;
  if (finish_reduction(acc, part, &st->ticket[T_SPMV_PQ], lds, tot)) {
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
}

__global__ __launch_bounds__(kRedThreads) void k_cg_update(int n, const int32_t *__restrict__ row_lat,
                                                           const double *__restrict__ p,
                                                           const double *__restrict__ q, double *__restrict__ x,
                                                           double *__restrict__ r, double *__restrict__ part,
                                                           CGState *st, int max_iter) {
  if (st->done) return;
  __shared__ double lds[kRedThreads];
  const double alpha = st->alpha;
  double acc = 0.0;
  for (int i = blockIdx.x * kRedThreads + threadIdx.x; i < n; i += gridDim.x * kRedThreads) {
    const int L = row_lat[i];
    x[L] += alpha * p[L];
    const double ri = r[L] - alpha * q[L];
    r[L] = ri;
    acc += ri * ri;
  }
  double tot;
  if (finish_reduction(acc, part, &st->ticket[T_UPDATE], lds, tot)) {
    if (threadIdx.x == 0) {
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
}

// ||b - A x||^2 into st->aux (x, b padded; tmp unused scratch kept for symmetry)
template <int K>
__global__ __launch_bounds__(kRedThreads) void k_cg_true_residual(int n, int Kdyn, Offsets off,
                                                                  const int32_t *__restrict__ row_lat,
                                                                  const double *__restrict__ val,
                                                                  const double *__restrict__ x,
                                                                  const double *__restrict__ b,
                                                                  double *__restrict__ part, CGState *st) {
  __shared__ double lds[kRedThreads];
  double acc = 0.0;
  for (int i = blockIdx.x * kRedThreads + threadIdx.x; i < n; i += gridDim.x * kRedThreads) {
    const int L = row_lat[i];
    const double ri = b[L] - ell_row<K>(i, n, off, L, val, x, Kdyn);
    acc += ri * ri;
  }
  double tot;
  if (finish_reduction(acc, part, &st->ticket[T_DOT], lds, tot)) {
    if (threadIdx.x == 0) st->aux = tot;
  }
}

#define IMSMG_DISPATCH_K(K, KERNEL, ...)                                        \
  switch (K) {                                                                  \
    case 9: KERNEL<9><<<g, kRedThreads, 0, s>>>(__VA_ARGS__); break;            \
    case 25: KERNEL<25><<<g, kRedThreads, 0, s>>>(__VA_ARGS__); break;          \
    case 49: KERNEL<49><<<g, kRedThreads, 0, s>>>(__VA_ARGS__); break;          \
    case 27: KERNEL<27><<<g, kRedThreads, 0, s>>>(__VA_ARGS__); break;          \
    case 125: KERNEL<125><<<g, kRedThreads, 0, s>>>(__VA_ARGS__); break;        \
    default: KERNEL<0><<<g, kRedThreads, 0, s>>>(__VA_ARGS__); break;           \
  }

void launch_cg_init(hipStream_t s, int n, int K, const Offsets &off, const int32_t *row_lat, const double *val,
                    const double *x, const double *b, double *r, double *part, CGState *st, double rtol) {
  const int g = reduction_blocks(n);
  IMSMG_DISPATCH_K(K, k_cg_init, n, K, off, row_lat, val, x, b, r, part, st, rtol);
}

void launch_cg_dot_rz(hipStream_t s, int n, const int32_t *row_lat, const double *r, const double *z, double *part,
                      CGState *st) {
  k_cg_dot_rz<<<reduction_blocks(n), kRedThreads, 0, s>>>(n, row_lat, r, z, part, st);
}

void launch_cg_direction(hipStream_t s, int n, const int32_t *row_lat, const double *z, double *p, CGState *st) {
  k_cg_direction<<<(n + kRedThreads - 1) / kRedThreads, kRedThreads, 0, s>>>(n, row_lat, z, p, st);
}

void launch_cg_spmv_pq(hipStream_t s, int n, int K, const Offsets &off, const int32_t *row_lat, const double *val,
                       const double *p, double *q, double *part, CGState *st) {
  const int g = reduction_blocks(n);
  IMSMG_DISPATCH_K(K, k_cg_spmv_pq, n, K, off, row_lat, val, p, q, part, st);
}

void launch_cg_update(hipStream_t s, int n, const int32_t *row_lat, const double *p, const double *q, double *x,
                      double *r, double *part, CGState *st, int max_iter) {
  k_cg_update<<<reduction_blocks(n), kRedThreads, 0, s>>>(n, row_lat, p, q, x, r, part, st, max_iter);
}

void launch_cg_true_residual(hipStream_t s, int n, int K, const Offsets &off, const int32_t *row_lat,
                             const double *val, const double *x, const double *b, double *tmp, double *part,
                             CGState *st) {
  (void)tmp;
  const int g = reduction_blocks(n);
  IMSMG_DISPATCH_K(K, k_cg_true_residual, n, K, off, row_lat, val, x, b, part, st);
}

}  // namespace imsmg
