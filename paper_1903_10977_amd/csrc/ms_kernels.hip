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
#include "op_row.h"

namespace imsmg {

namespace {
constexpr int kMsBlock = 256;
}

// LANES lanes share a row (slots lane, lane + LANES, ...), then add their
// partial sums in a fixed shuffle order: a colour holds a small fraction of
// the level's rows, so one lane per row would leave most of the chip idle and
// each lane with a long chain of gathers.
template <int K, typename V, int LANES>
__global__ __launch_bounds__(kMsBlock) void k_ms_colour(int m, const int32_t *__restrict__ rows,
                                                        const double *__restrict__ cf, OpView<V> op,
                                                        const int32_t *__restrict__ row_lat,
                                                        const uint32_t *__restrict__ meta,
                                                        const double *__restrict__ r, double *x,
                                                        double *__restrict__ rh, const int32_t *__restrict__ done,
                                                        int Kdyn) {
  if (done && *done) return;
  const int tid = blockIdx.x * kMsBlock + threadIdx.x;
  const int t = tid / LANES, lane = tid % LANES;
  const bool ok = t < m;
  double part = 0.0;
  int L = 0;
  if (ok) {
    const int i = rows[t];
    L = row_lat[i];
    const unsigned g = meta[i] & kMetaIndex;
    const bool uni = g == kMetaIndex;
    const size_t nv = size_t(op.nv);
    const int KK = K > 0 ? K : Kdyn;
#pragma unroll
    for (int s = lane; s < (K > 0 ? K : IMSMG_MAX_SLOTS); s += LANES) {
      if (K == 0 && s >= KK) break;
      const double a = double(uni ? op.ref[s] : op.val[stored_at<V>(nv, g, s)]);
      part += a * x[L + op.off.off[s]];
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

template <typename V>
static void dispatch_ms_colour(hipStream_t s, int m, const int32_t *rows, const double *cf, int K,
                               const OpView<V> &op, const int32_t *row_lat, const uint32_t *meta, const double *r,
                               double *x, double *rh, const int32_t *done) {
  if (m <= 0) return;
  constexpr int LN = 8;
  dim3 g((size_t(m) * LN + kMsBlock - 1) / kMsBlock), t(kMsBlock);
  switch (K) {
    case 9: k_ms_colour<9, V, LN><<<g, t, 0, s>>>(m, rows, cf, op, row_lat, meta, r, x, rh, done, K); break;
    case 25: k_ms_colour<25, V, LN><<<g, t, 0, s>>>(m, rows, cf, op, row_lat, meta, r, x, rh, done, K); break;
    case 49: k_ms_colour<49, V, LN><<<g, t, 0, s>>>(m, rows, cf, op, row_lat, meta, r, x, rh, done, K); break;
    case 27: k_ms_colour<27, V, LN><<<g, t, 0, s>>>(m, rows, cf, op, row_lat, meta, r, x, rh, done, K); break;
    case 125: k_ms_colour<125, V, LN><<<g, t, 0, s>>>(m, rows, cf, op, row_lat, meta, r, x, rh, done, K); break;
    default: k_ms_colour<0, V, LN><<<g, t, 0, s>>>(m, rows, cf, op, row_lat, meta, r, x, rh, done, K); break;
  }
}

void launch_ms_colour(hipStream_t s, int m, const int32_t *rows, const double *cf, int K, const OpView<double> &op,
                      const int32_t *row_lat, const uint32_t *meta, const double *r, double *x, double *rh,
                      const int32_t *done) {
  dispatch_ms_colour<double>(s, m, rows, cf, K, op, row_lat, meta, r, x, rh, done);
}
void launch_ms_colour(hipStream_t s, int m, const int32_t *rows, const double *cf, int K, const OpView<float> &op,
                      const int32_t *row_lat, const uint32_t *meta, const double *r, double *x, double *rh,
                      const int32_t *done) {
  dispatch_ms_colour<float>(s, m, rows, cf, K, op, row_lat, meta, r, x, rh, done);
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
