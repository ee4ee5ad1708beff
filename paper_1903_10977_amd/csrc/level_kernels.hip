// Per-level kernels of the V-cycle (Algorithm alg:MGV): lattice-ELL residual,
// additive Schwarz smoother (two phases), restriction / prolongation, dense
// coarsest solve, compact <-> lattice scatter and gather.
//
// All row kernels map one thread to one active row; consecutive threads
// handle consecutive active rows, whose lattice positions are increasing, so
// the slot-major value streams are fully coalesced and the stencil gathers of
// the input vector hit the same cache lines across a wavefront.  Workgroups
// are renumbered so that each of the 8 XCDs walks one contiguous chunk of rows
// and keeps the neighbouring lattice lines of the input vector in its own L2.
#include "imsmg_internal.h"

namespace imsmg {

constexpr int kRowBlock = 256;

__device__ __forceinline__ int xcd_block(int b, int nb) {
  // hardware dispatches workgroup b to XCD (b % 8); give XCD k the
  // contiguous range [k * ceil(nb/8), ...) of logical blocks
  const int per = (nb + 7) / 8;
  const int xcd = b % 8;
  const int k = b / 8;
  const int full = nb % 8 == 0 ? 8 : nb % 8;  // XCDs that receive `per` blocks
  // blocks b with xcd < full get index xcd*per + k; others are shifted
  if (xcd < full) return xcd * per + k;
  return full * per + (xcd - full) * (per - 1) + k;
}

static inline int grid_for(int n) { return (n + kRowBlock - 1) / kRowBlock; }

template <int K, typename V>
__global__ __launch_bounds__(kRowBlock) void k_ell_residual(int n, Offsets off, const int32_t *__restrict__ row_lat,
                                                             const V *__restrict__ val, const double *__restrict__ x,
                                                             const double *__restrict__ b, double *__restrict__ y,
                                                             const int32_t *__restrict__ done) {
  if (*done) return;
  const int i = xcd_block(blockIdx.x, gridDim.x) * kRowBlock + threadIdx.x;
  if (i >= n) return;
  const int L = row_lat[i];
  double acc = 0.0;
#pragma unroll
  for (int s = 0; s < K; ++s) acc += double(val[size_t(s) * n + i]) * x[L + off.off[s]];
  y[L] = b ? b[L] - acc : acc;
}

template <typename V>
__global__ __launch_bounds__(kRowBlock) void k_ell_residual_any(int n, int K, Offsets off,
                                                                 const int32_t *__restrict__ row_lat,
                                                                 const V *__restrict__ val,
                                                                 const double *__restrict__ x,
                                                                 const double *__restrict__ b, double *__restrict__ y,
                                                                 const int32_t *__restrict__ done) {
  if (*done) return;
  const int i = xcd_block(blockIdx.x, gridDim.x) * kRowBlock + threadIdx.x;
  if (i >= n) return;
  const int L = row_lat[i];
  double acc = 0.0;
  for (int s = 0; s < K; ++s) acc += double(val[size_t(s) * n + i]) * x[L + off.off[s]];
  y[L] = b ? b[L] - acc : acc;
}

template <typename V>
static void ell_residual(hipStream_t s, int n, int K, const Offsets &off, const int32_t *row_lat, const V *val,
                         const double *x, const double *b, double *y, const int32_t *done) {
  if (n <= 0) return;
  dim3 g(grid_for(n)), t(kRowBlock);
  switch (K) {
    case 9: k_ell_residual<9, V><<<g, t, 0, s>>>(n, off, row_lat, val, x, b, y, done); break;
    case 25: k_ell_residual<25, V><<<g, t, 0, s>>>(n, off, row_lat, val, x, b, y, done); break;
    case 49: k_ell_residual<49, V><<<g, t, 0, s>>>(n, off, row_lat, val, x, b, y, done); break;
    case 27: k_ell_residual<27, V><<<g, t, 0, s>>>(n, off, row_lat, val, x, b, y, done); break;
    case 125: k_ell_residual<125, V><<<g, t, 0, s>>>(n, off, row_lat, val, x, b, y, done); break;
    default: k_ell_residual_any<V><<<g, t, 0, s>>>(n, K, off, row_lat, val, x, b, y, done); break;
  }
}

void launch_ell_residual(hipStream_t s, int n, int K, const Offsets &off, const int32_t *row_lat, const double *val,
                         const double *x, const double *b, double *y, const int32_t *done) {
  ell_residual<double>(s, n, K, off, row_lat, val, x, b, y, done);
}
void launch_ell_residual_f32(hipStream_t s, int n, int K, const Offsets &off, const int32_t *row_lat,
                             const float *val, const double *x, const double *b, double *y, const int32_t *done) {
  ell_residual<float>(s, n, K, off, row_lat, val, x, b, y, done);
}

// y[lat_row[i]] (+)= sum_s v[s n + i] x[col[s n + i]]   (restriction / prolongation)
__global__ __launch_bounds__(kRowBlock) void k_ell_gather(int n, int w, const int32_t *__restrict__ row_lat,
                                                          const int32_t *__restrict__ col,
                                                          const double *__restrict__ v, const double *__restrict__ x,
                                                          double *__restrict__ y, int accumulate,
                                                          const int32_t *__restrict__ done) {
  if (*done) return;
  const int i = xcd_block(blockIdx.x, gridDim.x) * kRowBlock + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
#pragma unroll 8
  for (int s = 0; s < w; ++s) acc += v[size_t(s) * n + i] * x[col[size_t(s) * n + i]];
  const int L = row_lat[i];
  y[L] = accumulate ? y[L] + acc : acc;
}

void launch_ell_gather(hipStream_t s, int n, int w, const int32_t *row_lat, const int32_t *col, const double *v,
                       const double *x, double *y, int accumulate, const int32_t *done) {
  if (n <= 0) return;
  k_ell_gather<<<grid_for(n), kRowBlock, 0, s>>>(n, w, row_lat, col, v, x, y, accumulate, done);
}

// Index-free transfers R_l = tensor product of one 1D two-scale matrix
// (eq:coarsening on the tensor grid), restricted to active functions.  The
// vectors are zero at inactive lattice points, so the full tensor stencil can
// be applied without a mask.  tab: per 1D index, start of the band in the
// other level's 1D numbering, band length, and the band coefficients
// (stride W).
struct Band {
  const int32_t *start;
  const int32_t *len;
  const double *coef;
  int W;
};

template <int DIM>
__global__ __launch_bounds__(kRowBlock) void k_tensor_transfer(int n, const int32_t *__restrict__ row_lat,
                                                               int ox, int oy, Band band, int ix_, int iy_,
                                                               const double *__restrict__ xin,
                                                               double *__restrict__ y, int accumulate,
                                                               const int32_t *__restrict__ done) {
  // rows: this level (lattice ox x oy x .), inputs: other level (lattice ix_ x iy_ x .)
  if (*done) return;
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
  if (DIM == 2) {
    for (int b = 0; b < ny; ++b) {
      const double *row = xin + size_t(sy + b) * ix_ + sx;
      double t = 0.0;
      for (int a = 0; a < nx; ++a) t += cx[a] * row[a];
      acc += cy[b] * t;
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
  y[L] = accumulate ? y[L] + acc : acc;
}

void launch_tensor_transfer(hipStream_t s, int dim, int n, const int32_t *row_lat, int ox, int oy,
                            const int32_t *start, const int32_t *len, const double *coef, int W, int ix, int iy,
                            const double *xin, double *y, int accumulate, const int32_t *done) {
  if (n <= 0) return;
  Band b{start, len, coef, W};
  if (dim == 2)
    k_tensor_transfer<2><<<grid_for(n), kRowBlock, 0, s>>>(n, row_lat, ox, oy, b, ix, iy, xin, y, accumulate, done);
  else
    k_tensor_transfer<3><<<grid_for(n), kRowBlock, 0, s>>>(n, row_lat, ox, oy, b, ix, iy, xin, y, accumulate, done);
}

// Schwarz phase 1: one thread per block row.  The inverse is stored column
// major per block, so the threads of one block read consecutive addresses.
__global__ __launch_bounds__(kRowBlock) void k_schwarz_blocks(
    int ntask, const int32_t *__restrict__ task_block, const int32_t *__restrict__ bstart,
    const int32_t *__restrict__ bsize, const int64_t *__restrict__ binv_off, const int32_t *__restrict__ blat,
    const double *__restrict__ binv, const double *__restrict__ bw, const double *__restrict__ r,
    double *__restrict__ y, const int32_t *__restrict__ done) {
  if (*done) return;
  const int t = blockIdx.x * kRowBlock + threadIdx.x;
  if (t >= ntask) return;
  const int j = task_block[t];
  const int st = bstart[j];
  const int nj = bsize[j];
  const int a = t - st;
  const double *inv = binv + binv_off[j];
  double acc = 0.0;
#pragma unroll 4
  for (int b = 0; b < nj; ++b) acc += inv[a + size_t(nj) * b] * r[blat[st + b]];
  y[t] = bw[j] * acc;
}

void launch_schwarz_blocks(hipStream_t s, int ntask, const int32_t *task_block, const int32_t *bstart,
                           const int32_t *bsize, const int64_t *binv_off, const int32_t *blat, const double *binv,
                           const double *bw, const double *r, double *y, const int32_t *done) {
  if (ntask <= 0) return;
  k_schwarz_blocks<<<grid_for(ntask), kRowBlock, 0, s>>>(ntask, task_block, bstart, bsize, binv_off, blat, binv,
                                                         bw, r, y, done);
}

// Schwarz phase 2: deterministic gather of the block contributions per row.
__global__ __launch_bounds__(kRowBlock) void k_schwarz_gather(int n, const int32_t *__restrict__ row_lat,
                                                              const double *__restrict__ c,
                                                              const int32_t *__restrict__ gptr,
                                                              const int32_t *__restrict__ gidx,
                                                              const double *__restrict__ y,
                                                              const double *__restrict__ r, double *__restrict__ x,
                                                              int accumulate, const int32_t *__restrict__ done) {
  if (*done) return;
  const int i = xcd_block(blockIdx.x, gridDim.x) * kRowBlock + threadIdx.x;
  if (i >= n) return;
  const int L = row_lat[i];
  double v = c[i] * r[L];
  const int g0 = gptr[i], g1 = gptr[i + 1];
  for (int g = g0; g < g1; ++g) v += y[gidx[g]];
  x[L] = accumulate ? x[L] + v : v;
}

void launch_schwarz_gather(hipStream_t s, int n, const int32_t *row_lat, const double *c, const int32_t *gptr,
                           const int32_t *gidx, const double *y, const double *r, double *x, int accumulate,
                           const int32_t *done) {
  if (n <= 0) return;
  k_schwarz_gather<<<grid_for(n), kRowBlock, 0, s>>>(n, row_lat, c, gptr, gidx, y, r, x, accumulate, done);
}

// Dense coarsest solve: r gathered into LDS, one wavefront per output row.
constexpr int kGemvThreads = 256;
constexpr int kGemvMaxN = 8192;
__global__ __launch_bounds__(kGemvThreads) void k_dense_gemv(int n, const int32_t *__restrict__ row_lat,
                                                             const double *__restrict__ Ainv,
                                                             const double *__restrict__ r, double *__restrict__ x,
                                                             const int32_t *__restrict__ done) {
  if (*done) return;
  extern __shared__ double rs[];
  for (int j = threadIdx.x; j < n; j += kGemvThreads) rs[j] = r[row_lat[j]];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int rows_per_block = kGemvThreads / 64;
  const int i = blockIdx.x * rows_per_block + wave;
  if (i >= n) return;
  const double *row = Ainv + size_t(i) * n;
  double acc = 0.0;
  for (int j = lane; j < n; j += 64) acc += row[j] * rs[j];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if (lane == 0) x[row_lat[i]] = acc;
}

void launch_dense_gemv(hipStream_t s, int n, const int32_t *row_lat, const double *Ainv, const double *r, double *x,
                       const int32_t *done) {
  if (n <= 0) return;
  const int rpb = kGemvThreads / 64;
  k_dense_gemv<<<(n + rpb - 1) / rpb, kGemvThreads, size_t(n) * sizeof(double), s>>>(n, row_lat, Ainv, r, x, done);
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
__global__ void k_fill(size_t n, double v, double *__restrict__ dst) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = v;
}

void launch_scatter(hipStream_t s, int n, const int32_t *row_lat, const double *src, double *dst) {
  if (n > 0) k_scatter<<<grid_for(n), kRowBlock, 0, s>>>(n, row_lat, src, dst);
}
void launch_gather(hipStream_t s, int n, const int32_t *row_lat, const double *src, double *dst) {
  if (n > 0) k_gather<<<grid_for(n), kRowBlock, 0, s>>>(n, row_lat, src, dst);
}
void launch_fill(hipStream_t s, size_t n, double v, double *dst) {
  if (n > 0) k_fill<<<dim3(unsigned((n + kRowBlock - 1) / kRowBlock)), kRowBlock, 0, s>>>(n, v, dst);
}

}  // namespace imsmg
