// Multiplicative Schwarz with colouring (smoothers subsection,
// eq:multiplicativeSchwarz1 and its coloured form): the blocks of one colour
// share no element, so within a colour every block sees the same residual and
// no block's update changes another's residual; the residual is refreshed once
// per colour.  One colour of a sweep is two launches:
//   k_ms_colour      on the rows the colour's blocks touch: the residual
//                    r - A x of the current x; one-function blocks update x
//                    in place (x_L += cf (r - A x)_L, cf = w_j / A_ii), rows of
//                    larger blocks store their residual in rh;
//   smooth_general   x += S_c rh with S_c the colour's larger blocks w_j A_j^-1
//                    (CSR, lattice columns; one block per row, since blocks of
//                    one colour share no function).
// Race freedom: a thread reads x only at the stencil neighbours of its row;
// the rows written in place belong to one-function blocks of this colour, and
// no other row of the colour shares an element with them (the colouring's
// invariant), so no thread reads a value another thread of the launch writes.
#include <stdexcept>

#include "csr_row.h"
#include "op_row.h"

namespace imsmg {

namespace {
constexpr int kMsBlock = 256;
}

// LANES lanes share a row (16 for scalar rows), then add their partial sums
// in a fixed shuffle order: a colour holds a small fraction of the level's
// rows, so one lane per row would leave most of the chip idle and each lane
// with a long chain of gathers.  Stored rows read their values from the colour-ordered copy vals
// (entry e: KP values, slots in order, zero padded) in 16-byte slot groups
// q = lane, lane + LANES, ...: the LANES lanes of a row read LANES x 16
// contiguous bytes per step.  Rows on the level's reference stencil (vidx < 0)
// read its coefficients.
template <int K, typename V, int LANES, bool NT>
__global__ __launch_bounds__(kMsBlock) void k_ms_colour(int m, const int32_t *__restrict__ rows,
                                                        const double *__restrict__ cf,
                                                        const int32_t *__restrict__ vidx,
                                                        const V *__restrict__ vals, OpView<V> op,
                                                        const int32_t *__restrict__ row_lat,
                                                        const double *__restrict__ r, double *x,
                                                        double *__restrict__ rh, const int32_t *__restrict__ done) {
  if (done && *done) return;
  constexpr int G = SlotGroup<V>::G;
  constexpr int NG = (K + G - 1) / G;
  constexpr int W = StencilShape<K>::W, P = StencilShape<K>::P, DIM = StencilShape<K>::DIM;
  const int tid = blockIdx.x * kMsBlock + threadIdx.x;
  const int t = tid / LANES, lane = tid % LANES;
  const bool ok = t < m;
  double part = 0.0;
  int L = 0;
  // lattice offset of slot s (x fastest, reach P per axis)
  auto off = [&](int s) {
    const int dx = s % W - P, dy = (s / W) % W - P, dz = DIM == 3 ? s / (W * W) - P : 0;
    return dx + op.sx * (dy + op.sy * dz);
  };
  if (ok) {
    // row_lat == nullptr: rows holds the lattice positions themselves (one
    // dependent load less at the head of every lane's chain)
    L = row_lat ? row_lat[rows[t]] : rows[t];
    const int e = vidx[t];
    if (e < 0) {
      for (int s = lane; s < K; s += LANES) part += op.refd[s] * x[L + off(s)];
    } else {
      const V *__restrict__ rowv = vals + size_t(e) * (NG * G);
      for (int q = lane; q < NG; q += LANES) {
        if constexpr (G == 2) {
          const double2 v = stream_load<NT>(reinterpret_cast<const double2 *>(rowv) + q);
          part += v.x * x[L + off(2 * q)];
          if (2 * q + 1 < K) part += v.y * x[L + off(2 * q + 1)];
        } else {
          const float4 v = stream_load<NT>(reinterpret_cast<const float4 *>(rowv) + q);
          part += double(v.x) * x[L + off(4 * q)];
          if (4 * q + 1 < K) part += double(v.y) * x[L + off(4 * q + 1)];
          if (4 * q + 2 < K) part += double(v.z) * x[L + off(4 * q + 2)];
          if (4 * q + 3 < K) part += double(v.w) * x[L + off(4 * q + 3)];
        }
      }
    }
  }
#pragma unroll
  for (int o = LANES / 2; o > 0; o >>= 1) part += __shfl_xor(part, o, LANES);
  if (ok && lane == 0) {
    const double res = r[L] - part;
    const double c = cf[t];
    if (c != 0.0)
      x[L] += c * res;
    else
      rh[L] = res;
  }
}

// Vector levels: row i of component c = i / ns sums its ncomp block rows
// A_(c,e) x_e, block by block (e = 0, 1, ..), each from the block's
// reference stencil (vidx[t ncomp + e] < 0) or from its entry of the
// colour-ordered copy; then the same update as the scalar kernel.
template <int K, typename V, int LANES, bool NT>
__global__ __launch_bounds__(kMsBlock) void k_vms_colour(int m, const int32_t *__restrict__ rows,
                                                         const double *__restrict__ cf,
                                                         const int32_t *__restrict__ vidx,
                                                         const V *__restrict__ vals, VecOps<V> ops,
                                                         const int32_t *__restrict__ row_lat,
                                                         const double *__restrict__ r, double *x,
                                                         double *__restrict__ rh, const int32_t *__restrict__ done) {
  if (done && *done) return;
  constexpr int G = SlotGroup<V>::G;
  constexpr int NG = (K + G - 1) / G;
  constexpr int W = StencilShape<K>::W, P = StencilShape<K>::P;
  const int tid = blockIdx.x * kMsBlock + threadIdx.x;
  const int t = tid / LANES, lane = tid % LANES;
  const bool ok = t < m;
  double part = 0.0;
  int L = 0;
  auto off = [&](int s) {
    const int dx = s % W - P, dy = (s / W) % W - P, dz = s / (W * W) - P;
    return dx + ops.sx * (dy + ops.sy * dz);
  };
  if (ok) {
    const int i = rows[t];
    const int c = i / ops.ns;
    L = row_lat[i];
    const int64_t Ls = L - c * ops.cstride;
    for (int e = 0; e < ops.ncomp; ++e) {
      const double *xe = x + (e * ops.cstride + Ls);
      const int ve = vidx[size_t(t) * ops.ncomp + e];
      if (ve < 0) {
        const double *__restrict__ ref = ops.refd[c * ops.ncomp + e];
        for (int s = lane; s < K; s += LANES) part += ref[s] * xe[off(s)];
      } else {
        const V *__restrict__ rowv = vals + size_t(ve) * (NG * G);
        for (int q = lane; q < NG; q += LANES) {
          if constexpr (G == 2) {
            const double2 v = stream_load<NT>(reinterpret_cast<const double2 *>(rowv) + q);
            part += v.x * xe[off(2 * q)];
            if (2 * q + 1 < K) part += v.y * xe[off(2 * q + 1)];
          } else {
            const float4 v = stream_load<NT>(reinterpret_cast<const float4 *>(rowv) + q);
            part += double(v.x) * xe[off(4 * q)];
            if (4 * q + 1 < K) part += double(v.y) * xe[off(4 * q + 1)];
            if (4 * q + 2 < K) part += double(v.z) * xe[off(4 * q + 2)];
            if (4 * q + 3 < K) part += double(v.w) * xe[off(4 * q + 3)];
          }
        }
      }
    }
  }
#pragma unroll
  for (int o = LANES / 2; o > 0; o >>= 1) part += __shfl_xor(part, o, LANES);
  if (ok && lane == 0) {
    const double res = r[L] - part;
    const double cc = cf[t];
    if (cc != 0.0)
      x[L] += cc * res;
    else
      rh[L] = res;
  }
}

template <typename V>
static void dispatch_vms_colour(hipStream_t s, int m, const int32_t *rows, const double *cf, const int32_t *vidx,
                                const V *vals, int K, const VecOps<V> &ops, const int32_t *row_lat,
                                const double *r, double *x, double *rh, const int32_t *done, int stream) {
  if (m <= 0) return;
  // a vector row is ncomp block rows: 32 lanes per row keep each lane's chain
  // of dependent gathers short (one block per 16 lanes would need 48)
  constexpr int LN = 32;
  dim3 g((size_t(m) * LN + kMsBlock - 1) / kMsBlock), t(kMsBlock);
#define IMSMG_VMS(KK)                                                                                   \
  if (stream)                                                                                           \
    k_vms_colour<KK, V, LN, true><<<g, t, 0, s>>>(m, rows, cf, vidx, vals, ops, row_lat, r, x, rh, done);  \
  else                                                                                                  \
    k_vms_colour<KK, V, LN, false><<<g, t, 0, s>>>(m, rows, cf, vidx, vals, ops, row_lat, r, x, rh, done);
  if (K == 125) {
    IMSMG_VMS(125)
  } else if (K == 27) {
    IMSMG_VMS(27)
  } else
    throw std::invalid_argument("vector multiplicative smoother: 3D stencils of 27 or 125 slots");
#undef IMSMG_VMS
}

void launch_vms_colour(hipStream_t s, int m, const int32_t *rows, const double *cf, const int32_t *vidx,
                       const double *vals, int K, const VecOps<double> &ops, const int32_t *row_lat, const double *r,
                       double *x, double *rh, const int32_t *done, int stream) {
  dispatch_vms_colour<double>(s, m, rows, cf, vidx, vals, K, ops, row_lat, r, x, rh, done, stream);
}
void launch_vms_colour(hipStream_t s, int m, const int32_t *rows, const double *cf, const int32_t *vidx,
                       const float *vals, int K, const VecOps<float> &ops, const int32_t *row_lat, const double *r,
                       double *x, double *rh, const int32_t *done, int stream) {
  dispatch_vms_colour<float>(s, m, rows, cf, vidx, vals, K, ops, row_lat, r, x, rh, done, stream);
}

template <typename V>
static void dispatch_ms_colour(hipStream_t s, int m, const int32_t *rows, const double *cf, const int32_t *vidx,
                               const V *vals, int K, const OpView<V> &op, const int32_t *row_lat, const double *r,
                               double *x, double *rh, const int32_t *done, int stream) {
  if (m <= 0) return;
  constexpr int LN = 16;
  dim3 g((size_t(m) * LN + kMsBlock - 1) / kMsBlock), t(kMsBlock);
#define IMSMG_MS(KK)                                                                                  \
  if (stream)                                                                                         \
    k_ms_colour<KK, V, LN, true><<<g, t, 0, s>>>(m, rows, cf, vidx, vals, op, row_lat, r, x, rh, done);  \
  else                                                                                                \
    k_ms_colour<KK, V, LN, false><<<g, t, 0, s>>>(m, rows, cf, vidx, vals, op, row_lat, r, x, rh, done);
  switch (K) {
    case 9: IMSMG_MS(9) break;
    case 25: IMSMG_MS(25) break;
    case 49: IMSMG_MS(49) break;
    case 27: IMSMG_MS(27) break;
    case 125: IMSMG_MS(125) break;
    default: throw std::invalid_argument("multiplicative smoother: stencils of 9, 25, 49, 27 or 125 slots");
  }
#undef IMSMG_MS
}

// The colour-ordered copy of the stored rows' values: entry e takes stored
// row g[e] of the level's operator (slot groups of SlotGroup<V>) as KP
// consecutive values, zero padded.
template <typename V>
__global__ void k_ms_pack(int ne, int K, int KP, const int32_t *__restrict__ g, const V *__restrict__ val, int nv,
                          V *__restrict__ out) {
  const int64_t id = int64_t(blockIdx.x) * kMsBlock + threadIdx.x;
  if (id >= int64_t(ne) * KP) return;
  const int e = int(id / KP), s = int(id % KP);
  out[id] = s < K ? val[stored_at<V>(size_t(nv), size_t(g[e]), s)] : V(0);
}

void launch_ms_colour(hipStream_t s, int m, const int32_t *rows, const double *cf, const int32_t *vidx,
                      const double *vals, int K, const OpView<double> &op, const int32_t *row_lat, const double *r,
                      double *x, double *rh, const int32_t *done, int stream) {
  dispatch_ms_colour<double>(s, m, rows, cf, vidx, vals, K, op, row_lat, r, x, rh, done, stream);
}
void launch_ms_colour(hipStream_t s, int m, const int32_t *rows, const double *cf, const int32_t *vidx,
                      const float *vals, int K, const OpView<float> &op, const int32_t *row_lat, const double *r,
                      double *x, double *rh, const int32_t *done, int stream) {
  dispatch_ms_colour<float>(s, m, rows, cf, vidx, vals, K, op, row_lat, r, x, rh, done, stream);
}
// General sparse levels: the same colour step on CSR rows (LN lanes per row,
// fixed-order lane sums as csr_rows); the race argument above holds because
// A couples two functions only where they share an element.
template <int LN, typename V>
__global__ __launch_bounds__(kMsBlock) void k_csr_ms_colour(int m, const int32_t *__restrict__ rows,
                                                            const double *__restrict__ cf, CsrView<V> A,
                                                            const double *__restrict__ r, double *x,
                                                            double *__restrict__ rh,
                                                            const int32_t *__restrict__ done) {
  if (done && *done) return;
  const int t = blockIdx.x * (kMsBlock / LN) + int(threadIdx.x) / LN;
  const int lane = int(threadIdx.x) % LN;
  const bool ok = t < m;
  double part = 0.0;
  int i = 0;
  if (ok) {
    i = rows[t];
    for (int k = A.ptr[i] + lane; k < A.ptr[i + 1]; k += LN) part += double(A.val[k]) * x[A.col[k]];
  }
#pragma unroll
  for (int o = LN / 2; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
  if (ok && lane == 0) {
    const double res = r[i] - part;
    const double c = cf[t];
    if (c != 0.0)
      x[i] += c * res;
    else
      rh[i] = res;
  }
}

template <typename V>
static void csr_ms_colour(hipStream_t s, int m, int ln, const int32_t *rows, const double *cf, const CsrView<V> &A,
                          const double *r, double *x, double *rh, const int32_t *done) {
  if (m <= 0) return;
  switch (ln) {
    case 4: k_csr_ms_colour<4, V><<<csr_grid(m, 4), kMsBlock, 0, s>>>(m, rows, cf, A, r, x, rh, done); break;
    case 8: k_csr_ms_colour<8, V><<<csr_grid(m, 8), kMsBlock, 0, s>>>(m, rows, cf, A, r, x, rh, done); break;
    case 16: k_csr_ms_colour<16, V><<<csr_grid(m, 16), kMsBlock, 0, s>>>(m, rows, cf, A, r, x, rh, done); break;
    default: throw std::invalid_argument("CSR rows: 4, 8 or 16 lanes per row");
  }
}

void launch_csr_ms_colour(hipStream_t s, int m, int ln, const int32_t *rows, const double *cf,
                          const CsrView<double> &A, const double *r, double *x, double *rh, const int32_t *done) {
  csr_ms_colour<double>(s, m, ln, rows, cf, A, r, x, rh, done);
}
void launch_csr_ms_colour(hipStream_t s, int m, int ln, const int32_t *rows, const double *cf,
                          const CsrView<float> &A, const double *r, double *x, double *rh, const int32_t *done) {
  csr_ms_colour<float>(s, m, ln, rows, cf, A, r, x, rh, done);
}

void launch_ms_pack(hipStream_t s, int ne, int K, int KP, const int32_t *g, const double *val, int nv, double *out) {
  if (ne > 0)
    k_ms_pack<double><<<(int64_t(ne) * KP + kMsBlock - 1) / kMsBlock, kMsBlock, 0, s>>>(ne, K, KP, g, val, nv, out);
}
void launch_ms_pack(hipStream_t s, int ne, int K, int KP, const int32_t *g, const float *val, int nv, float *out) {
  if (ne > 0)
    k_ms_pack<float><<<(int64_t(ne) * KP + kMsBlock - 1) / kMsBlock, kMsBlock, 0, s>>>(ne, K, KP, g, val, nv, out);
}

// Row-wise vector operations on a level's padded lattice vectors (active
// rows only; the inactive lattice points stay zero): y = 0, y = x, y += x.
__global__ __launch_bounds__(kMsBlock) void k_rows_op(int n, const int32_t *__restrict__ row_lat,
                                                      const double *__restrict__ x, double *__restrict__ y, int op,
                                                      const int32_t *__restrict__ done) {
  if (done && *done) return;
  const int i = blockIdx.x * kMsBlock + threadIdx.x;
  if (i >= n) return;
  const int L = row_lat[i];
  if (op == 0)
    y[L] = 0.0;
  else if (op == 1)
    y[L] = x[L];
  else
    y[L] += x[L];
}

void launch_rows_op(hipStream_t s, int n, const int32_t *row_lat, const double *x, double *y, int op,
                    const int32_t *done) {
  if (n > 0) k_rows_op<<<(n + kMsBlock - 1) / kMsBlock, kMsBlock, 0, s>>>(n, row_lat, x, y, op, done);
}

}  // namespace imsmg
