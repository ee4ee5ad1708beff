// Multi-right-hand-side form of the V-cycle and of CG: R systems with the
// same matrix solved together (R = 4, 8 or 16 columns).
//
// Layout: every level vector holds the R columns interleaved on the padded
// function lattice, v[L * R + col], so that the R values of one lattice point
// are one contiguous 8R-byte segment.  One thread per (row, column): the R
// lanes of a row share the row's lattice position, meta word and stencil
// coefficients (broadcast loads) and read the neighbours' R values with
// contiguous, coalesced loads.  The matrix bytes per row are thereby read
// once for R solves.
//
// CG keeps separate scalars per column (MState); a column that has converged
// stops moving (its alpha and beta are zero) while the others continue.
// Reductions are deterministic: per workgroup and column one partial sum
// (fixed LDS tree over the workgroup's rows), then one workgroup adds the
// partials of each column in index order.
#include "imsmg_internal.h"
#include "op_row.h"

namespace imsmg {

namespace {
constexpr int kMT = 256;   // threads per workgroup
constexpr int kMFin = 1024;

__device__ __forceinline__ int xcd_map(int b, int nb) {
  const int per = (nb + 7) / 8;
  const int xcd = b % 8;
  const int k = b / 8;
  const int full = nb % 8 == 0 ? 8 : nb % 8;
  if (xcd < full) return xcd * per + k;
  return full * per + (xcd - full) * (per - 1) + k;
}

// (A x)_{L, col} with per-lane coefficient select (reference or stored row)
template <int K, int R, typename V>
__device__ __forceinline__ double mrow(unsigned meta, const OpView<V> &op, const double *__restrict__ x, int L,
                                       int col, int Kdyn) {
  const unsigned g = meta & kMetaIndex;
  const bool uni = g == kMetaIndex;
  const size_t nv = size_t(op.nv);
  double acc = 0.0;
  if (K > 0) {
#pragma unroll
    for (int s = 0; s < K; ++s)
      acc += double(uni ? op.ref[s] : op.val[stored_at<V>(nv, g, s)]) * x[size_t(L + op.off.off[s]) * R + col];
  } else {
    for (int s = 0; s < Kdyn; ++s)
      acc += double(uni ? op.ref[s] : op.val[stored_at<V>(nv, g, s)]) * x[size_t(L + op.off.off[s]) * R + col];
  }
  return acc;
}

// per-column sum over the workgroup's rows (lds: kMT doubles); result valid in
// threads 0 .. R-1 (column = thread index)
template <int R>
__device__ __forceinline__ double col_sum(double v, double *lds) {
  lds[threadIdx.x] = v;
  __syncthreads();
  for (int s = kMT / 2; s >= R; s >>= 1) {
    if (threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
    __syncthreads();
  }
  return lds[threadIdx.x];
}

// per-column sums of part[b * R + col] over b < m for all R columns at once
// (R a power of two <= 16): thread t adds column t % R over b = t / R,
// t / R + kMFin / R, ... in that order, then a fixed tree over the kMFin / R
// threads of each column (strides are multiples of R).  The sums are left in
// lds[0 .. R); every thread of the workgroup must call it.
__device__ __forceinline__ void sum_cols(const double *__restrict__ part, int m, int R, double *lds) {
  const int col = threadIdx.x % R, lane = threadIdx.x / R, lanes = kMFin / R;
  double v = 0.0;
  for (int b = lane; b < m; b += lanes) v += part[size_t(b) * R + col];
  lds[threadIdx.x] = v;
  __syncthreads();
  for (int s = kMFin / 2; s >= R; s >>= 1) {
    if (threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
    __syncthreads();
  }
}
}  // namespace

// ------------------------------------------------------------------ level kernels
template <int K, int R, typename V>
__global__ __launch_bounds__(kMT) void k_m_residual(int n, int Kdyn, OpView<V> op, const int32_t *__restrict__ row_lat,
                                                    const uint32_t *__restrict__ meta, const double *__restrict__ x,
                                                    const double *__restrict__ b, double *__restrict__ y,
                                                    const int32_t *__restrict__ done) {
  if (done && *done) return;
  const int t = xcd_map(blockIdx.x, gridDim.x) * kMT + threadIdx.x;
  const int i = t / R, col = t % R;
  if (i >= n) return;
  const int L = row_lat[i];
  const double ax = mrow<K, R, V>(meta[i], op, x, L, col, Kdyn);
  const size_t o = size_t(L) * R + col;
  y[o] = b ? b[o] - ax : ax;
}

template <int K, int R, typename V>
__global__ __launch_bounds__(kMT) void k_m_residual_smooth(int n, int Kdyn, OpView<V> op,
                                                           const int32_t *__restrict__ row_lat,
                                                           const uint32_t *__restrict__ meta,
                                                           const double *__restrict__ c,
                                                           const double *__restrict__ xa,
                                                           const double *__restrict__ r, double *__restrict__ rh,
                                                           double *__restrict__ xb, const int32_t *__restrict__ done) {
  if (done && *done) return;
  const int t = xcd_map(blockIdx.x, gridDim.x) * kMT + threadIdx.x;
  const int i = t / R, col = t % R;
  if (i >= n) return;
  const int L = row_lat[i];
  const unsigned m = meta[i];
  const double ax = mrow<K, R, V>(m, op, xa, L, col, Kdyn);
  const size_t o = size_t(L) * R + col;
  const double res = r[o] - ax;
  if (m & kMetaGeneral) rh[o] = res;
  xb[o] = xa[o] + c[i] * res;
}

// Lattice-tiled forms of the two kernels above for tiled stencils (the
// single-column tiles: one lattice point per thread, x window in LDS), four
// interleaved columns per workgroup: workgroup = (tile, column group), the
// window holds the group's four columns of every window point (32 bytes,
// contiguous in the interleaved layout), and each lane applies its row to
// the four columns.  Same slot order and arithmetic as mrow: bitwise the
// results of the untiled kernels.  SMOOTH: rh = r - A xa (general rows), xb
// = xa + c (r - A xa); RESIDUAL: y = b - A x (b == nullptr: y = A x); SPMV
// (the multi-column CG): y = q = A p and, per column, the tile's partial sum
// of p . q into part[tile * R + column].
constexpr int kMCols = 4;
enum MTileMode { RESIDUAL = 0, SMOOTH = 1, SPMV = 2 };
template <int K, typename V, int MODE>
__global__ __launch_bounds__(kTileRows) void k_m_tile(int R, OpView<V> op, const uint32_t *__restrict__ meta,
                                                      const double *__restrict__ c, const double *__restrict__ x,
                                                      const double *__restrict__ b, double *__restrict__ y,
                                                      double *__restrict__ xb, const int32_t *__restrict__ done,
                                                      double *__restrict__ part) {
  using SS = StencilShape<K>;
  constexpr int NC = kMCols;
  __shared__ double win[SS::WINDOW * NC];
  __shared__ double xch[kTileRows * NC];
  const int ngrp = R / NC;
  const int bid = xcd_map(blockIdx.x, gridDim.x);
  const int blk = bid / ngrp, col0 = (bid % ngrp) * NC;
  const TileBox tb = tile_box<K>(blk, op.ntx, op.nty);
  const int tx = threadIdx.x % SS::TX;
  const int ty = (threadIdx.x / SS::TX) % SS::TY;
  const int tz = threadIdx.x / (SS::TX * SS::TY);
  const int gx = tb.x0 + tx, gy = tb.y0 + ty, gz = tb.z0 + tz;
  const bool inbox = gx < op.sx && gy < op.sy && gz < op.sz;
  const int L = inbox ? gx + op.sx * (gy + op.sy * gz) : 0;
  const int i0 = op.lat2row[L];
  const int i = inbox ? i0 : -1;
  // load (1): the window's four columns (unconditional loads at lattice point
  // 0 outside the lattice, so that the wait for the row index excludes them)
  constexpr int PER = (SS::WINDOW + kTileRows - 1) / kTileRows;
  double w[PER][NC];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * kTileRows;
    const int wx = e % SS::WX, wy = (e / SS::WX) % SS::WY, wz = e / (SS::WX * SS::WY);
    const int ex = tb.x0 - SS::P + wx, ey = tb.y0 - SS::P + wy, ez = tb.z0 - (SS::DIM == 3 ? SS::P : 0) + wz;
    const bool in = e < SS::WINDOW && ex >= 0 && ex < op.sx && ey >= 0 && ey < op.sy && ez >= 0 && ez < op.sz;
    const double2 *src = reinterpret_cast<const double2 *>(x + size_t(in ? ex + op.sx * (ey + op.sy * ez) : 0) * R + col0);
#pragma unroll
    for (int k = 0; k < NC / 2; ++k) {
      const double2 u = src[k];
      w[q][2 * k] = in ? u.x : 0.0;
      w[q][2 * k + 1] = in ? u.y : 0.0;
    }
  }
  const int g = op.tile_g0[blk] + threadIdx.x;
  const bool act2 = g < op.tile_g0[blk + 1];
  // load (2): the row's meta and epilogue inputs, the stored rows' owners
  unsigned m = 0u;
  double bv[NC] = {}, ci = 0.0;
  if (i >= 0) {
    m = meta[i];
    if (b) {
      const double2 *bs = reinterpret_cast<const double2 *>(b + size_t(L) * R + col0);
#pragma unroll
      for (int k = 0; k < NC / 2; ++k) {
        const double2 u = bs[k];
        bv[2 * k] = u.x;
        bv[2 * k + 1] = u.y;
      }
    }
    if (MODE == SMOOTH) ci = c[i];
  }
  const int own2 = act2 ? op.sloc[g] : 0;
  if (done && *done) return;  // uniform
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * kTileRows;
    if (e < SS::WINDOW) {
#pragma unroll
      for (int k = 0; k < NC; ++k) win[e * NC + k] = w[q][k];
    }
  }
  __syncthreads();
  const int tl = tile_local<K>(threadIdx.x);
  double ax[NC] = {};
  // phase 1: rows on the reference stencil
  if (i >= 0 && (m & kMetaIndex) == kMetaIndex) {
    const ConstPtr<double> ref = (ConstPtr<double>)op.refd;
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const int dx = s % SS::W, dy = (s / SS::W) % SS::W, dz = s / (SS::W * SS::W);
      const double *t = win + (tl + (dz * SS::WY + dy) * SS::WX + dx) * NC;
      const double a = ref[s];
#pragma unroll
      for (int k = 0; k < NC; ++k) ax[k] += a * t[k];
    }
  }
  // phase 2: the tile's stored rows on the first lanes, results to the owners
  if (act2) {
    const int t2 = tile_local<K>(own2);
    double a2[NC] = {};
    stored_row_slots_nt<K, V, false>(op.val, size_t(op.nv), g, [&](int s, double a) {
      const int dx = s % SS::W, dy = (s / SS::W) % SS::W, dz = s / (SS::W * SS::W);
      const double *t = win + (t2 + (dz * SS::WY + dy) * SS::WX + dx) * NC;
#pragma unroll
      for (int k = 0; k < NC; ++k) a2[k] += a * t[k];
    });
#pragma unroll
    for (int k = 0; k < NC; ++k) xch[own2 * NC + k] = a2[k];
  }
  __syncthreads();
  const double *xc = win + (tl + ((SS::DIM == 3 ? SS::P : 0) * SS::WY + SS::P) * SS::WX + SS::P) * NC;
  if constexpr (MODE == SPMV) {
    // q = A p; per column the workgroup's p . q in a fixed order (shuffle
    // tree per wavefront, then the four wavefronts in index order)
    double pq[NC] = {};
    if (i >= 0) {
      if ((m & kMetaIndex) != kMetaIndex)
#pragma unroll
        for (int k = 0; k < NC; ++k) ax[k] = xch[threadIdx.x * NC + k];
      const size_t o = size_t(L) * R + col0;
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        y[o + k] = ax[k];
        pq[k] = xc[k] * ax[k];
      }
    }
    __syncthreads();  // xch is reused for the wavefront sums
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      double v = pq[k];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if ((threadIdx.x & 63) == 0) xch[(threadIdx.x >> 6) * NC + k] = v;
    }
    __syncthreads();
    if (threadIdx.x < NC) {
      double t = 0.0;
#pragma unroll
      for (int wv = 0; wv < kTileRows / 64; ++wv) t += xch[wv * NC + threadIdx.x];
      part[size_t(blk) * R + col0 + threadIdx.x] = t;
    }
    return;
  }
  if (i < 0) return;
  if ((m & kMetaIndex) != kMetaIndex)
#pragma unroll
    for (int k = 0; k < NC; ++k) ax[k] = xch[threadIdx.x * NC + k];
  const size_t o = size_t(L) * R + col0;
  if constexpr (MODE == SMOOTH) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const double res = bv[k] - ax[k];
      if (m & kMetaGeneral) y[o + k] = res;
      xb[o + k] = xc[k] + ci * res;
    }
  } else {
#pragma unroll
    for (int k = 0; k < NC; ++k) y[o + k] = b ? bv[k] - ax[k] : ax[k];
  }
}

template <int R>
__global__ __launch_bounds__(kMT) void k_m_smooth_general(int ng, const int32_t *__restrict__ grow_lat,
                                                          const int32_t *__restrict__ sptr,
                                                          const int32_t *__restrict__ scol,
                                                          const double *__restrict__ sval,
                                                          const double *__restrict__ r, double *__restrict__ x,
                                                          const int32_t *__restrict__ done) {
  if (done && *done) return;
  const int t = xcd_map(blockIdx.x, gridDim.x) * kMT + threadIdx.x;
  const int i = t / R, col = t % R;
  if (i >= ng) return;
  const int k0 = sptr[i], k1 = sptr[i + 1];
  double acc = 0.0;
  // chunks of 8 with guarded, fixed trip counts (see the single-column kernel)
  for (int kb = k0; kb < k1; kb += 8) {
    int c[8];
    double v[8], rv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const bool in = kb + q < k1;
      c[q] = scol[in ? kb + q : kb];
      v[q] = in ? sval[kb + q] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) rv[q] = r[size_t(c[q]) * R + col];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc += v[q] * rv[q];
  }
  x[size_t(grow_lat[i]) * R + col] += acc;
}

template <int R>
__global__ __launch_bounds__(kMT) void k_m_diag_scale(int n, const int32_t *__restrict__ row_lat,
                                                      const double *__restrict__ c, const double *__restrict__ r,
                                                      double *__restrict__ x, const int32_t *__restrict__ done) {
  if (done && *done) return;
  const int t = xcd_map(blockIdx.x, gridDim.x) * kMT + threadIdx.x;
  const int i = t / R, col = t % R;
  if (i >= n) return;
  const size_t o = size_t(row_lat[i]) * R + col;
  x[o] = c[i] * r[o];
}

struct MBand {
  const int32_t *start;
  const int32_t *len;
  const double *coef;
  int W;
};
constexpr int kMBandMax = 5;

template <int DIM, int R>
__global__ __launch_bounds__(kMT) void k_m_tensor_transfer(int n, const int32_t *__restrict__ row_lat, int ox, int oy,
                                                           MBand band, int ix_, int iy_,
                                                           const double *__restrict__ xin, double *__restrict__ y,
                                                           int accumulate, const double *__restrict__ cinit,
                                                           double *__restrict__ xinit,
                                                           const int32_t *__restrict__ done) {
  if (done && *done) return;
  const int t = xcd_map(blockIdx.x, gridDim.x) * kMT + threadIdx.x;
  const int i = t / R, col = t % R;
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
  if (DIM == 2 && band.W <= kMBandMax) {
    // fixed trip counts with guards: all loads of the row issue before the first wait
    double cxv[kMBandMax], cyv[kMBandMax], in[kMBandMax][kMBandMax];
#pragma unroll
    for (int a = 0; a < kMBandMax; ++a) {
      cxv[a] = a < nx ? cx[a] : 0.0;
      cyv[a] = a < ny ? cy[a] : 0.0;
    }
#pragma unroll
    for (int b = 0; b < kMBandMax; ++b)
#pragma unroll
      for (int a = 0; a < kMBandMax; ++a)
        in[b][a] = (a < nx && b < ny) ? xin[(size_t(sy + b) * ix_ + sx + a) * R + col] : 0.0;
#pragma unroll
    for (int b = 0; b < kMBandMax; ++b) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < kMBandMax; ++a) s += cxv[a] * in[b][a];
      acc += cyv[b] * s;
    }
  } else if (DIM == 2) {
    for (int b = 0; b < ny; ++b) {
      const size_t row = size_t(sy + b) * ix_ + sx;
      double s = 0.0;
      for (int a = 0; a < nx; ++a) s += cx[a] * xin[(row + a) * R + col];
      acc += cy[b] * s;
    }
  } else {
    const int sz = band.start[mz], nz = band.len[mz];
    const double *cz = band.coef + size_t(mz) * band.W;
    for (int c3 = 0; c3 < nz; ++c3) {
      double tz = 0.0;
      for (int b = 0; b < ny; ++b) {
        const size_t row = (size_t(sz + c3) * iy_ + (sy + b)) * ix_ + sx;
        double s = 0.0;
        for (int a = 0; a < nx; ++a) s += cx[a] * xin[(row + a) * R + col];
        tz += cy[b] * s;
      }
      acc += cz[c3] * tz;
    }
  }
  const size_t o = size_t(L) * R + col;
  const double out = accumulate ? y[o] + acc : acc;
  y[o] = out;
  if (xinit) xinit[o] = cinit[i] * out;
}

// 2D tensor transfer with bands up to kMBandMax, four interleaved columns
// per thread: the row's band starts, lengths and coefficients are loaded
// once for the four columns, the inputs as 32-byte vectors; per column the
// same arithmetic as k_m_tensor_transfer (bitwise the same results).
template <int R>
__global__ __launch_bounds__(kMT) void k_m_tensor_transfer4(int n, const int32_t *__restrict__ row_lat, int ox,
                                                            MBand band, int ix_, const double *__restrict__ xin,
                                                            double *__restrict__ y, int accumulate,
                                                            const double *__restrict__ cinit,
                                                            double *__restrict__ xinit,
                                                            const int32_t *__restrict__ done) {
  if (done && *done) return;
  constexpr int NG = R / 4;
  const int t = xcd_map(blockIdx.x, gridDim.x) * kMT + threadIdx.x;
  const int i = t / NG, col0 = (t % NG) * 4;
  if (i >= n) return;
  const int L = row_lat[i];
  const int mx = L % ox;
  const int my = L / ox;
  const int sx = band.start[mx], nx = band.len[mx];
  const int sy = band.start[my], ny = band.len[my];
  const double *cx = band.coef + size_t(mx) * band.W;
  const double *cy = band.coef + size_t(my) * band.W;
  double cxv[kMBandMax], cyv[kMBandMax];
#pragma unroll
  for (int a = 0; a < kMBandMax; ++a) {
    cxv[a] = a < nx ? cx[a] : 0.0;
    cyv[a] = a < ny ? cy[a] : 0.0;
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int b = 0; b < kMBandMax; ++b) {
    double in[kMBandMax][4];
#pragma unroll
    for (int a = 0; a < kMBandMax; ++a) {
      if (a < nx && b < ny) {
        const double *src = xin + (size_t(sy + b) * ix_ + sx + a) * R + col0;
        const double2 u0 = *reinterpret_cast<const double2 *>(src);
        const double2 u1 = *reinterpret_cast<const double2 *>(src + 2);
        in[a][0] = u0.x;
        in[a][1] = u0.y;
        in[a][2] = u1.x;
        in[a][3] = u1.y;
      } else {
        in[a][0] = in[a][1] = in[a][2] = in[a][3] = 0.0;
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double sum = 0.0;
#pragma unroll
      for (int a = 0; a < kMBandMax; ++a) sum += cxv[a] * in[a][k];
      acc[k] += cyv[b] * sum;
    }
  }
  const size_t o = size_t(L) * R + col0;
  const double ci = xinit ? cinit[i] : 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double out = accumulate ? y[o + k] + acc[k] : acc[k];
    y[o + k] = out;
    if (xinit) xinit[o + k] = ci * out;
  }
}

template <int R>
__global__ __launch_bounds__(kMT) void k_m_ell_gather(int n, int w, const int32_t *__restrict__ row_lat,
                                                      const int32_t *__restrict__ colidx,
                                                      const double *__restrict__ v, const double *__restrict__ x,
                                                      double *__restrict__ y, int accumulate,
                                                      const double *__restrict__ cinit, double *__restrict__ xinit,
                                                      const int32_t *__restrict__ done) {
  if (done && *done) return;
  const int t = xcd_map(blockIdx.x, gridDim.x) * kMT + threadIdx.x;
  const int i = t / R, col = t % R;
  if (i >= n) return;
  double acc = 0.0;
  for (int s = 0; s < w; ++s) acc += v[size_t(s) * n + i] * x[size_t(colidx[size_t(s) * n + i]) * R + col];
  const size_t o = size_t(row_lat[i]) * R + col;
  const double out = accumulate ? y[o] + acc : acc;
  y[o] = out;
  if (xinit) xinit[o] = cinit[i] * out;
}

// coarsest level: X = A^{-1} Rhs for R columns, one wavefront per row; the
// right-hand sides are staged through LDS in chunks of kGChunk rows
// (kGChunk x R doubles).
constexpr int kGChunk = 128;
static_assert(kGChunk % 64 == 0, "chunks keep each lane's ascending j sequence");
constexpr int kGemmThreads = 1024;  // 16 rows per workgroup: each staged chunk serves 16 rows
template <int R>
__global__ __launch_bounds__(kGemmThreads) void k_m_dense_gemm(int n, const int32_t *__restrict__ row_lat,
                                                      const double *__restrict__ Ainv, const double *__restrict__ r,
                                                      double *__restrict__ x, const int32_t *__restrict__ done) {
  // one wavefront per row of A^{-1}: lane l adds the entries j = l, l + 64,
  // ... in ascending order for all R columns, then a shuffle tree per column
  // (per column the order of the single-column product); the right-hand
  // sides are staged per chunk in LDS, column-major, so that the lanes of a
  // wavefront read consecutive doubles
  if (done && *done) return;
  __shared__ double rs[R * kGChunk];
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (kGemmThreads / 64) + (threadIdx.x >> 6);
  const double *row = Ainv + size_t(i < n ? i : 0) * n;
  double acc[R];
#pragma unroll
  for (int c = 0; c < R; ++c) acc[c] = 0.0;
  for (int j0 = 0; j0 < n; j0 += kGChunk) {
    const int m = min(kGChunk, n - j0);
    for (int e = threadIdx.x; e < m * R; e += kGemmThreads) rs[(e % R) * kGChunk + e / R] = r[size_t(row_lat[j0 + e / R]) * R + (e % R)];
    __syncthreads();
    if (i < n) {
      for (int j = lane; j < m; j += 64) {
        const double a = row[j0 + j];
#pragma unroll
        for (int c = 0; c < R; ++c) acc[c] += a * rs[c * kGChunk + j];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < R; ++c)
    for (int o = 32; o > 0; o >>= 1) acc[c] += __shfl_down(acc[c], o, 64);
  if (i < n && lane == 0) {
#pragma unroll
    for (int c = 0; c < R; ++c) x[size_t(row_lat[i]) * R + c] = acc[c];
  }
}

// user layout (column-major n x ncols, ld = n) <-> interleaved padded lattice
template <int R>
__global__ void k_m_scatter(int n, int ncols, const int32_t *__restrict__ row_lat, const double *__restrict__ src,
                            double *__restrict__ dst) {
  const int t = blockIdx.x * kMT + threadIdx.x;
  const int i = t / R, col = t % R;
  if (i >= n) return;
  dst[size_t(row_lat[i]) * R + col] = col < ncols ? src[size_t(col) * n + i] : 0.0;
}
template <int R>
__global__ void k_m_gather(int n, int ncols, const int32_t *__restrict__ row_lat, const double *__restrict__ src,
                           double *__restrict__ dst) {
  const int t = blockIdx.x * kMT + threadIdx.x;
  const int i = t / R, col = t % R;
  if (i >= n || col >= ncols) return;
  dst[size_t(col) * n + i] = src[size_t(row_lat[i]) * R + col];
}

// ------------------------------------------------------------------ CG kernels
// (finest level, FP64 operator)
template <int K, int R>
__global__ __launch_bounds__(kMT) void k_mcg_init(int n, int Kdyn, OpView<double> op,
                                                  const int32_t *__restrict__ row_lat,
                                                  const uint32_t *__restrict__ meta, const double *__restrict__ x,
                                                  const double *__restrict__ b, double *__restrict__ r,
                                                  double *__restrict__ part) {
  __shared__ double lds[kMT];
  const int blk = xcd_map(blockIdx.x, gridDim.x);
  const int t = blk * kMT + threadIdx.x;
  const int i = t / R, col = t % R;
  double rr = 0.0, bb = 0.0;
  if (i < n) {
    const int L = row_lat[i];
    const size_t o = size_t(L) * R + col;
    const double bi = b[o];
    const double ri = bi - mrow<K, R, double>(meta[i], op, x, L, col, Kdyn);
    r[o] = ri;
    rr = ri * ri;
    bb = bi * bi;
  }
  rr = col_sum<R>(rr, lds);
  if (threadIdx.x < R) part[size_t(blk) * R + threadIdx.x] = rr;
  __syncthreads();
  bb = col_sum<R>(bb, lds);
  if (threadIdx.x < R) part[(size_t(gridDim.x) + blk) * R + threadIdx.x] = bb;
}

template <int R>
__global__ __launch_bounds__(kMT) void k_mcg_dot(int n, const int32_t *__restrict__ row_lat,
                                                 const double *__restrict__ a, const double *__restrict__ b,
                                                 double *__restrict__ part, const MState *st) {
  if (st->done) return;
  __shared__ double lds[kMT];
  const int blk = xcd_map(blockIdx.x, gridDim.x);
  const int t = blk * kMT + threadIdx.x;
  const int i = t / R, col = t % R;
  double acc = 0.0;
  if (i < n) {
    const size_t o = size_t(row_lat[i]) * R + col;
    acc = a[o] * b[o];
  }
  acc = col_sum<R>(acc, lds);
  if (threadIdx.x < R) part[size_t(blk) * R + threadIdx.x] = acc;
}

template <int R>
__global__ __launch_bounds__(kMT) void k_mcg_direction(int n, const int32_t *__restrict__ row_lat,
                                                       const double *__restrict__ z, double *__restrict__ p,
                                                       const MState *st) {
  if (st->done) return;
  const int t = xcd_map(blockIdx.x, gridDim.x) * kMT + threadIdx.x;
  const int i = t / R, col = t % R;
  if (i >= n) return;
  const size_t o = size_t(row_lat[i]) * R + col;
  const double beta = st->beta[col];
  p[o] = st->first ? z[o] : z[o] + beta * p[o];
}

template <int K, int R>
__global__ __launch_bounds__(kMT) void k_mcg_spmv_pq(int n, int Kdyn, OpView<double> op,
                                                     const int32_t *__restrict__ row_lat,
                                                     const uint32_t *__restrict__ meta, const double *__restrict__ p,
                                                     double *__restrict__ q, double *__restrict__ part,
                                                     const MState *st) {
  if (st->done) return;
  __shared__ double lds[kMT];
  const int blk = xcd_map(blockIdx.x, gridDim.x);
  const int t = blk * kMT + threadIdx.x;
  const int i = t / R, col = t % R;
  double acc = 0.0;
  if (i < n) {
    const int L = row_lat[i];
    const size_t o = size_t(L) * R + col;
    const double qi = mrow<K, R, double>(meta[i], op, p, L, col, Kdyn);
    q[o] = qi;
    acc = p[o] * qi;
  }
  acc = col_sum<R>(acc, lds);
  if (threadIdx.x < R) part[size_t(blk) * R + threadIdx.x] = acc;
}

template <int R>
__global__ __launch_bounds__(kMT) void k_mcg_update(int n, const int32_t *__restrict__ row_lat,
                                                    const double *__restrict__ p, const double *__restrict__ q,
                                                    double *__restrict__ x, double *__restrict__ r,
                                                    const double *__restrict__ c, double *__restrict__ zs,
                                                    double *__restrict__ part, const MState *st) {
  if (st->done) return;
  __shared__ double lds[kMT];
  const int blk = xcd_map(blockIdx.x, gridDim.x);
  const int t = blk * kMT + threadIdx.x;
  const int i = t / R, col = t % R;
  double acc = 0.0;
  if (i < n) {
    const size_t o = size_t(row_lat[i]) * R + col;
    const double alpha = st->alpha[col];
    x[o] += alpha * p[o];
    const double ri = r[o] - alpha * q[o];
    r[o] = ri;
    zs[o] = c[i] * ri;
    acc = ri * ri;
  }
  acc = col_sum<R>(acc, lds);
  if (threadIdx.x < R) part[size_t(blk) * R + threadIdx.x] = acc;
}

template <int K, int R>
__global__ __launch_bounds__(kMT) void k_mcg_true_residual(int n, int Kdyn, OpView<double> op,
                                                           const int32_t *__restrict__ row_lat,
                                                           const uint32_t *__restrict__ meta,
                                                           const double *__restrict__ x,
                                                           const double *__restrict__ b, double *__restrict__ part) {
  __shared__ double lds[kMT];
  const int blk = xcd_map(blockIdx.x, gridDim.x);
  const int t = blk * kMT + threadIdx.x;
  const int i = t / R, col = t % R;
  double acc = 0.0;
  if (i < n) {
    const int L = row_lat[i];
    const double ri = b[size_t(L) * R + col] - mrow<K, R, double>(meta[i], op, x, L, col, Kdyn);
    acc = ri * ri;
  }
  acc = col_sum<R>(acc, lds);
  if (threadIdx.x < R) part[size_t(blk) * R + threadIdx.x] = acc;
}

// ---- first stage of the partial sums: workgroup b adds the partials of a
// contiguous range of source workgroups for all R columns (coalesced reads,
// fixed order) -> out[b * R + col]
constexpr int kStage = 256;  // second-stage partials per column
__global__ __launch_bounds__(kMT) void k_mcg_stage(int m, int R, const double *__restrict__ part,
                                                   double *__restrict__ out) {
  __shared__ double lds[kMT];
  const int per = (m + kStage - 1) / kStage;
  const int b0 = blockIdx.x * per, b1 = min(m, b0 + per);
  const int col = threadIdx.x % R, lane = threadIdx.x / R, lanes = kMT / R;
  double v = 0.0;
  for (int b = b0 + lane; b < b1; b += lanes) v += part[size_t(b) * R + col];
  lds[threadIdx.x] = v;
  __syncthreads();
  for (int s = kMT / 2; s >= R; s >>= 1) {
    if (threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < R) out[size_t(blockIdx.x) * R + threadIdx.x] = lds[threadIdx.x];
}

// ---- finalize kernels (one workgroup; all columns reduced together, then
// thread 0 updates the per-column state in column order)
// restart != 0: CG restarted from the current iterate; the stopping threshold
// and the iteration counts of the first start are kept, and the columns in
// keep_mask (bit col) stay converged
__global__ __launch_bounds__(kMFin) void k_mcg_init_fin(int m, int R, int ncols, const double *__restrict__ part,
                                                        MState *st, double rtol, int restart, int keep_mask) {
  __shared__ double lds[kMFin];
  __shared__ double rrs[16];
  sum_cols(part, m, R, lds);
  if (threadIdx.x < R) rrs[threadIdx.x] = lds[threadIdx.x];
  __syncthreads();
  sum_cols(part + size_t(m) * R, m, R, lds);
  int all = 1;
  // a NaN of an earlier solve must not stop this one: the status is this call's
  if (threadIdx.x == 0) st->status = 0;
  for (int col = 0; col < R; ++col) {
    if (threadIdx.x == 0) {
      const double rr = rrs[col], bb = lds[col];
      if (!restart) {
        st->r0sq[col] = rr;
        st->tol2[col] = rtol * rtol * (rr < bb ? rr : bb);
        st->iters[col] = 0;
      }
      st->rr[col] = rr;
      st->bb[col] = bb;
      st->beta[col] = 0.0;
      st->alpha[col] = 0.0;
      st->rz[col] = 0.0;
      const int d = (col >= ncols || rr == 0.0 || (restart && ((keep_mask >> col) & 1))) ? 1 : 0;
      st->cdone[col] = d;
      all &= d;
      if (!(rr == rr) || !(bb == bb)) st->status = -6;
    }
  }
  if (threadIdx.x == 0) {
    st->first = 1;
    st->done = (all || st->status != 0) ? 1 : 0;
  }
}

__global__ __launch_bounds__(kMFin) void k_mcg_rz_fin(int m, int R, const double *__restrict__ part, MState *st) {
  if (st->done) return;
  __shared__ double lds[kMFin];
  sum_cols(part, m, R, lds);
  for (int col = 0; col < R; ++col) {
    if (threadIdx.x == 0) {
      const double tot = lds[col];
      if (st->cdone[col]) {
        st->beta[col] = 0.0;
      } else {
        st->rz_old[col] = st->rz[col];
        st->rz[col] = tot;
        st->beta[col] = st->first ? 0.0 : tot / st->rz_old[col];
        if (!(tot == tot)) {
          st->status = -6;
          st->done = 1;
        }
      }
    }
  }
}

__global__ __launch_bounds__(kMFin) void k_mcg_pq_fin(int m, int R, const double *__restrict__ part, MState *st) {
  if (st->done) return;
  __shared__ double lds[kMFin];
  sum_cols(part, m, R, lds);
  for (int col = 0; col < R; ++col) {
    if (threadIdx.x == 0) {
      const double tot = lds[col];
      if (st->cdone[col]) {
        st->alpha[col] = 0.0;
      } else if (!(tot > 0.0)) {
        st->status = (tot == tot) ? -4 : -6;
        st->done = 1;
        st->alpha[col] = 0.0;
      } else {
        st->alpha[col] = st->rz[col] / tot;
      }
    }
  }
  if (threadIdx.x == 0) st->first = 0;
}

__global__ __launch_bounds__(kMFin) void k_mcg_update_fin(int m, int R, const double *__restrict__ part, MState *st,
                                                          int max_iter) {
  if (st->done) return;
  __shared__ double lds[kMFin];
  sum_cols(part, m, R, lds);
  int all = 1;
  for (int col = 0; col < R; ++col) {
    if (threadIdx.x == 0) {
      const double tot = lds[col];
      if (!st->cdone[col]) {
        st->rr[col] = tot;
        st->iters[col] += 1;
        if (!(tot == tot)) {
          st->status = -6;
        } else if (tot <= st->tol2[col]) {
          st->cdone[col] = 1;
        } else if (st->iters[col] >= max_iter) {
          st->status = -5;
        }
      }
      all &= st->cdone[col];
    }
  }
  if (threadIdx.x == 0 && (all || st->status != 0)) st->done = 1;
}

__global__ __launch_bounds__(kMFin) void k_mcg_aux_fin(int m, int R, const double *__restrict__ part, MState *st) {
  __shared__ double lds[kMFin];
  sum_cols(part, m, R, lds);
  if (threadIdx.x == 0)
    for (int col = 0; col < R; ++col) st->aux[col] = lds[col];
}

// ------------------------------------------------------------------ launchers
#define MR_DISPATCH(R, BODY)                 \
  switch (R) {                               \
    case 4: { constexpr int RR = 4; BODY; } break;  \
    case 8: { constexpr int RR = 8; BODY; } break;  \
    case 16: { constexpr int RR = 16; BODY; } break; \
    default: break;                          \
  }
#define MK_DISPATCH(K, BODY)                         \
  switch (K) {                                       \
    case 9: { constexpr int KK = 9; BODY; } break;   \
    case 25: { constexpr int KK = 25; BODY; } break; \
    case 49: { constexpr int KK = 49; BODY; } break; \
    case 27: { constexpr int KK = 27; BODY; } break; \
    case 125: { constexpr int KK = 125; BODY; } break; \
    default: { constexpr int KK = 0; BODY; } break;  \
  }

bool multi_supported(int R) { return R == 4 || R == 8 || R == 16; }

int multi_blocks(int R, int n) { return std::max(1, (n * R + kMT - 1) / kMT); }
// partial-sum workspace (doubles): two first-level arrays and the second stage
size_t multi_part_size(int R, int n, int ntiles) {
  return size_t(2) * std::max(multi_blocks(R, n), ntiles) * R + size_t(2) * kStage * R;
}

#define MT_DISPATCH(K, BODY)                           \
  switch (K) {                                         \
    case 9: { constexpr int KK = 9; BODY; } break;     \
    case 25: { constexpr int KK = 25; BODY; } break;   \
    case 49: { constexpr int KK = 49; BODY; } break;   \
    case 27: { constexpr int KK = 27; BODY; } break;   \
    case 125: { constexpr int KK = 125; BODY; } break; \
    default: break;                                    \
  }
static bool m_tiled(int K, int R) {
  return (K == 9 || K == 25 || K == 49 || K == 27 || K == 125) && R % kMCols == 0;
}

template <typename V>
static void m_residual_impl(hipStream_t s, int R, int n, int K, const OpView<V> &op, const int32_t *row_lat,
                            const uint32_t *meta, const double *x, const double *b, double *y, const int32_t *done) {
  if (n <= 0) return;
  if (m_tiled(K, R) && op.ntiles > 0) {
    const int gt = op.ntiles * (R / kMCols);
    MT_DISPATCH(K, (k_m_tile<KK, V, RESIDUAL><<<gt, kTileRows, 0, s>>>(R, op, meta, nullptr, x, b, y, nullptr, done,
                                                                      nullptr)))
    return;
  }
  const int g = multi_blocks(R, n);
  MR_DISPATCH(R, MK_DISPATCH(K, (k_m_residual<KK, RR, V><<<g, kMT, 0, s>>>(n, K, op, row_lat, meta, x, b, y, done))))
}
void launch_m_residual(hipStream_t s, int R, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                       const uint32_t *meta, const double *x, const double *b, double *y, const int32_t *done) {
  m_residual_impl<double>(s, R, n, K, op, row_lat, meta, x, b, y, done);
}
void launch_m_residual(hipStream_t s, int R, int n, int K, const OpView<float> &op, const int32_t *row_lat,
                       const uint32_t *meta, const double *x, const double *b, double *y, const int32_t *done) {
  m_residual_impl<float>(s, R, n, K, op, row_lat, meta, x, b, y, done);
}

template <typename V>
static void m_residual_smooth_impl(hipStream_t s, int R, int n, int K, const OpView<V> &op, const int32_t *row_lat,
                                   const uint32_t *meta, const double *c, const double *xa, const double *r,
                                   double *rh, double *xb, const int32_t *done) {
  if (n <= 0) return;
  if (m_tiled(K, R) && op.ntiles > 0) {
    const int gt = op.ntiles * (R / kMCols);
    MT_DISPATCH(K, (k_m_tile<KK, V, SMOOTH><<<gt, kTileRows, 0, s>>>(R, op, meta, c, xa, r, rh, xb, done, nullptr)))
    return;
  }
  const int g = multi_blocks(R, n);
  MR_DISPATCH(R, MK_DISPATCH(K, (k_m_residual_smooth<KK, RR, V><<<g, kMT, 0, s>>>(n, K, op, row_lat, meta, c, xa, r,
                                                                                   rh, xb, done))))
}
void launch_m_residual_smooth(hipStream_t s, int R, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                              const uint32_t *meta, const double *c, const double *xa, const double *r, double *rh,
                              double *xb, const int32_t *done) {
  m_residual_smooth_impl<double>(s, R, n, K, op, row_lat, meta, c, xa, r, rh, xb, done);
}
void launch_m_residual_smooth(hipStream_t s, int R, int n, int K, const OpView<float> &op, const int32_t *row_lat,
                              const uint32_t *meta, const double *c, const double *xa, const double *r, double *rh,
                              double *xb, const int32_t *done) {
  m_residual_smooth_impl<float>(s, R, n, K, op, row_lat, meta, c, xa, r, rh, xb, done);
}

void launch_m_smooth_general(hipStream_t s, int R, int ng, const int32_t *grow_lat, const int32_t *sptr,
                             const int32_t *scol, const double *sval, const double *r, double *x,
                             const int32_t *done) {
  if (ng <= 0) return;
  const int g = multi_blocks(R, ng);
  MR_DISPATCH(R, (k_m_smooth_general<RR><<<g, kMT, 0, s>>>(ng, grow_lat, sptr, scol, sval, r, x, done)))
}

// ---------------------------------------------------------- patch GEMMs
// General Schwarz blocks of up to 16 functions applied as dense products on
// the matrix cores, one wavefront per block: Y_q = W_q R_q with W_q =
// omega_q A_q^{-1} (16 x 16, zero-padded, row-major) and R_q = the block
// members' residual rows (member k x right-hand-side column n, 16 columns,
// columns >= R and members past the block size zero).  FP64 operands: four
// v_mfma_f64_16x16x4 steps (exact FP64 products); BF16 operands with FP32
// accumulation: one v_mfma_f32_16x16x16_bf16.  Lane layouts (checked on the
// device): FP64 A[lane % 16][k], B[k][lane % 16] with k = 4 step + lane / 16,
// D[lane / 16 + 4 q][lane % 16]; BF16 A[lane % 16][4 (lane / 16) + q],
// B[4 (lane / 16) + q][lane % 16], D[4 (lane / 16) + q][lane % 16].
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float f) {  // round to nearest even (finite inputs)
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return short(u >> 16);
}

constexpr int kGemmWaves = 4;  // blocks (wavefronts) per workgroup

// BF16 = true: blocks flagged in lp (well conditioned) take BF16 operands,
// the others FP64 (a wavefront-uniform choice per block)
template <bool BF16>
__global__ __launch_bounds__(64 * kGemmWaves) void k_m_block_gemm(int nb, int R, const int32_t *__restrict__ blat,
                                                                   const double *__restrict__ W,
                                                                   const uint16_t *__restrict__ Wb,
                                                                   const int32_t *__restrict__ lp,
                                                                   const double *__restrict__ r,
                                                                   double *__restrict__ Y,
                                                                   const int32_t *__restrict__ done) {
  if (done && *done) return;
  const int q = blockIdx.x * kGemmWaves + threadIdx.x / 64;
  if (q >= nb) return;  // whole wavefronts
  const int lane = threadIdx.x % 64;
  const int n = lane % 16;
  if (BF16 && lp[q]) {
    bf16x4 a, b;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = 4 * (lane / 16) + t;
      a[t] = short(Wb[size_t(q) * 256 + n * 16 + k]);  // A[m = lane % 16][k]
      const int L = blat[q * 16 + k];
      const double v = (L >= 0 && n < R) ? r[size_t(L) * R + n] : 0.0;
      b[t] = bf16_bits(float(v));
    }
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
#pragma unroll
    for (int t = 0; t < 4; ++t) Y[size_t(q) * 256 + (4 * (lane / 16) + t) * 16 + n] = double(c[t]);
  } else {
    f64x4 c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int k = 4 * st + lane / 16;
      const double a = W[size_t(q) * 256 + n * 16 + k];  // A[m = lane % 16][k]
      const int L = blat[q * 16 + k];
      const double b = (L >= 0 && n < R) ? r[size_t(L) * R + n] : 0.0;
      c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) Y[size_t(q) * 256 + (lane / 16 + 4 * t) * 16 + n] = c[t];
  }
}

// x[row] += sum over the row's blocks (ascending block order) of Y[block][row's
// member position][column]; one thread per (general row, column)
template <int R>
__global__ __launch_bounds__(kMT) void k_m_block_gather(int ng, const int32_t *__restrict__ grow_lat,
                                                        const int32_t *__restrict__ yp,
                                                        const int32_t *__restrict__ ypos,
                                                        const double *__restrict__ Y, double *__restrict__ x,
                                                        const int32_t *__restrict__ done) {
  if (done && *done) return;
  const int gt = blockIdx.x * kMT + threadIdx.x;
  const int t = gt / R, col = gt % R;
  if (t >= ng) return;
  double acc = 0.0;
  for (int k = yp[t]; k < yp[t + 1]; ++k) acc += Y[size_t(ypos[k]) + col];
  x[size_t(grow_lat[t]) * R + col] += acc;
}

// W (FP64, 16 x 16 zero-padded per block) and its BF16 copy from the packed
// block inverses (size g_sz[q] at g_off[q], row-major)
__global__ void k_pack_blocks(int nb, const int64_t *__restrict__ g_off, const int32_t *__restrict__ g_sz,
                              const double *__restrict__ inv, double *__restrict__ W, uint16_t *__restrict__ Wb) {
  const int gt = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = gt / 256, e = gt % 256;
  if (q >= nb) return;
  const int m = e / 16, k = e % 16, sz = g_sz[q];
  const double v = (m < sz && k < sz) ? inv[g_off[q] + int64_t(m) * sz + k] : 0.0;
  W[gt] = v;
  Wb[gt] = uint16_t(bf16_bits(float(v)));
}

void launch_m_block_gemm(hipStream_t s, int bf16, int nb, int R, const int32_t *blat, const double *W,
                         const uint16_t *Wb, const int32_t *lp, const double *r, double *Y, const int32_t *done) {
  if (nb <= 0) return;
  const int g = (nb + kGemmWaves - 1) / kGemmWaves;
  if (bf16)
    k_m_block_gemm<true><<<g, 64 * kGemmWaves, 0, s>>>(nb, R, blat, W, Wb, lp, r, Y, done);
  else
    k_m_block_gemm<false><<<g, 64 * kGemmWaves, 0, s>>>(nb, R, blat, W, Wb, lp, r, Y, done);
}

void launch_m_block_gather(hipStream_t s, int R, int ng, const int32_t *grow_lat, const int32_t *yp,
                           const int32_t *ypos, const double *Y, double *x, const int32_t *done) {
  if (ng <= 0) return;
  const int g = multi_blocks(R, ng);
  MR_DISPATCH(R, (k_m_block_gather<RR><<<g, kMT, 0, s>>>(ng, grow_lat, yp, ypos, Y, x, done)))
}

void launch_pack_blocks(hipStream_t s, int nb, const int64_t *g_off, const int32_t *g_sz, const double *inv,
                        double *W, uint16_t *Wb) {
  if (nb <= 0) return;
  k_pack_blocks<<<(nb * 256 + 255) / 256, 256, 0, s>>>(nb, g_off, g_sz, inv, W, Wb);
}

void launch_m_diag_scale(hipStream_t s, int R, int n, const int32_t *row_lat, const double *c, const double *r,
                         double *x, const int32_t *done) {
  if (n <= 0) return;
  const int g = multi_blocks(R, n);
  MR_DISPATCH(R, (k_m_diag_scale<RR><<<g, kMT, 0, s>>>(n, row_lat, c, r, x, done)))
}

void launch_m_tensor_transfer(hipStream_t s, int R, int dim, int n, const int32_t *row_lat, int ox, int oy,
                              const int32_t *start, const int32_t *len, const double *coef, int W, int ix, int iy,
                              const double *xin, double *y, int accumulate, const double *cinit, double *xinit,
                              const int32_t *done) {
  if (n <= 0) return;
  const int g = multi_blocks(R, n);
  MBand b{start, len, coef, W};
  if (dim == 2 && W <= kMBandMax && R % 4 == 0) {
    const int g4 = std::max(1, (n * (R / 4) + kMT - 1) / kMT);
    MR_DISPATCH(R, (k_m_tensor_transfer4<RR><<<g4, kMT, 0, s>>>(n, row_lat, ox, b, ix, xin, y, accumulate, cinit,
                                                                 xinit, done)))
  } else if (dim == 2) {
    MR_DISPATCH(R, (k_m_tensor_transfer<2, RR><<<g, kMT, 0, s>>>(n, row_lat, ox, oy, b, ix, iy, xin, y, accumulate,
                                                                  cinit, xinit, done)))
  } else {
    MR_DISPATCH(R, (k_m_tensor_transfer<3, RR><<<g, kMT, 0, s>>>(n, row_lat, ox, oy, b, ix, iy, xin, y, accumulate,
                                                                  cinit, xinit, done)))
  }
}

void launch_m_ell_gather(hipStream_t s, int R, int n, int w, const int32_t *row_lat, const int32_t *col,
                         const double *v, const double *x, double *y, int accumulate, const double *cinit,
                         double *xinit, const int32_t *done) {
  if (n <= 0) return;
  const int g = multi_blocks(R, n);
  MR_DISPATCH(R, (k_m_ell_gather<RR><<<g, kMT, 0, s>>>(n, w, row_lat, col, v, x, y, accumulate, cinit, xinit, done)))
}

void launch_m_dense_gemm(hipStream_t s, int R, int n, const int32_t *row_lat, const double *Ainv, const double *r,
                         double *x, const int32_t *done) {
  if (n <= 0) return;
  const int g = (n + kGemmThreads / 64 - 1) / (kGemmThreads / 64);  // one wavefront per row
  MR_DISPATCH(R, (k_m_dense_gemm<RR><<<g, kGemmThreads, 0, s>>>(n, row_lat, Ainv, r, x, done)))
}

void launch_m_scatter(hipStream_t s, int R, int n, int ncols, const int32_t *row_lat, const double *src,
                      double *dst) {
  if (n <= 0) return;
  const int g = multi_blocks(R, n);
  MR_DISPATCH(R, (k_m_scatter<RR><<<g, kMT, 0, s>>>(n, ncols, row_lat, src, dst)))
}
void launch_m_gather(hipStream_t s, int R, int n, int ncols, const int32_t *row_lat, const double *src,
                     double *dst) {
  if (n <= 0) return;
  const int g = multi_blocks(R, n);
  MR_DISPATCH(R, (k_m_gather<RR><<<g, kMT, 0, s>>>(n, ncols, row_lat, src, dst)))
}

void launch_mcg_init(hipStream_t s, int R, int ncols, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                     const uint32_t *meta, const double *x, const double *b, double *r, double *part, MState *st,
                     double rtol, int restart, int keep_mask) {
  const int g = multi_blocks(R, n);
  MR_DISPATCH(R, MK_DISPATCH(K, (k_mcg_init<KK, RR><<<g, kMT, 0, s>>>(n, K, op, row_lat, meta, x, b, r, part))))
  double *p2 = part + size_t(2) * g * R;
  k_mcg_stage<<<kStage, kMT, 0, s>>>(g, R, part, p2);
  k_mcg_stage<<<kStage, kMT, 0, s>>>(g, R, part + size_t(g) * R, p2 + size_t(kStage) * R);
  k_mcg_init_fin<<<1, kMFin, 0, s>>>(kStage, R, ncols, p2, st, rtol, restart, keep_mask);
}
void launch_mcg_dot_rz(hipStream_t s, int R, int n, const int32_t *row_lat, const double *r, const double *z,
                       double *part, MState *st) {
  const int g = multi_blocks(R, n);
  MR_DISPATCH(R, (k_mcg_dot<RR><<<g, kMT, 0, s>>>(n, row_lat, r, z, part, st)))
  double *p2 = part + size_t(2) * g * R;
  k_mcg_stage<<<kStage, kMT, 0, s>>>(g, R, part, p2);
  k_mcg_rz_fin<<<1, kMFin, 0, s>>>(kStage, R, p2, st);
}
void launch_mcg_direction(hipStream_t s, int R, int n, const int32_t *row_lat, const double *z, double *p,
                          MState *st) {
  const int g = multi_blocks(R, n);
  MR_DISPATCH(R, (k_mcg_direction<RR><<<g, kMT, 0, s>>>(n, row_lat, z, p, st)))
}
void launch_mcg_spmv_pq(hipStream_t s, int R, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                        const uint32_t *meta, const double *p, double *q, double *part, MState *st) {
  int g = multi_blocks(R, n);
  if (m_tiled(K, R) && op.ntiles > 0) {
    g = op.ntiles;  // one partial row per tile
    const int gt = op.ntiles * (R / kMCols);
    MT_DISPATCH(K, (k_m_tile<KK, double, SPMV><<<gt, kTileRows, 0, s>>>(R, op, meta, nullptr, p, nullptr, q, nullptr,
                                                                       &st->done, part)))
  } else {
    MR_DISPATCH(R, MK_DISPATCH(K, (k_mcg_spmv_pq<KK, RR><<<g, kMT, 0, s>>>(n, K, op, row_lat, meta, p, q, part, st))))
  }
  double *p2 = part + size_t(2) * g * R;
  k_mcg_stage<<<kStage, kMT, 0, s>>>(g, R, part, p2);
  k_mcg_pq_fin<<<1, kMFin, 0, s>>>(kStage, R, p2, st);
}
void launch_mcg_update(hipStream_t s, int R, int n, const int32_t *row_lat, const double *p, const double *q,
                       double *x, double *r, const double *c, double *zs, double *part, MState *st, int max_iter) {
  const int g = multi_blocks(R, n);
  MR_DISPATCH(R, (k_mcg_update<RR><<<g, kMT, 0, s>>>(n, row_lat, p, q, x, r, c, zs, part, st)))
  double *p2 = part + size_t(2) * g * R;
  k_mcg_stage<<<kStage, kMT, 0, s>>>(g, R, part, p2);
  k_mcg_update_fin<<<1, kMFin, 0, s>>>(kStage, R, p2, st, max_iter);
}
void launch_mcg_true_residual(hipStream_t s, int R, int n, int K, const OpView<double> &op, const int32_t *row_lat,
                              const uint32_t *meta, const double *x, const double *b, double *part, MState *st) {
  const int g = multi_blocks(R, n);
  MR_DISPATCH(R, MK_DISPATCH(K, (k_mcg_true_residual<KK, RR><<<g, kMT, 0, s>>>(n, K, op, row_lat, meta, x, b, part))))
  double *p2 = part + size_t(2) * g * R;
  k_mcg_stage<<<kStage, kMT, 0, s>>>(g, R, part, p2);
  k_mcg_aux_fin<<<1, kMFin, 0, s>>>(kStage, R, p2, st);
}

}  // namespace imsmg
