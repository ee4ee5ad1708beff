// Rows of the compressed lattice-ELL operator: sum_s a_s x[L + off_s].
//
// Two cooperating mechanisms keep the per-row memory instructions low (the
// stencil kernels are bound by vector address processing, not by HBM: the
// level's matrix and vectors stay resident in the Infinity Cache between the
// V-cycle's sweeps):
//   * LDS tile: a workgroup of consecutive active rows spans the lattice
//     range [Lmin, Lmax]; for every stencil line (fixed dy, dz) the x window
//     [Lmin - p + line_off, Lmax + p + line_off] is loaded once, coalesced,
//     into LDS and the K gathers of a row become LDS reads;
//   * wave-uniform stencil: when every row of a wavefront uses the level's
//     reference stencil, its K coefficients are wave-uniform (scalar loads);
//     otherwise each lane selects its own (pointer, stride): the reference
//     stencil (stride 1) or its stored slot-major values (stride nv).
// Shared by the level and CG kernels.
#pragma once
#include "imsmg_internal.h"

namespace imsmg {

constexpr int kTileRows = 256;  // rows per workgroup of the stencil kernels
constexpr int kTileSpan = 640;  // largest lattice span staged in LDS (else global gathers)

template <int K>
struct StencilShape {
  static constexpr int W = K == 9 ? 3 : K == 25 ? 5 : K == 49 ? 7 : K == 27 ? 3 : K == 125 ? 5 : 0;
  static constexpr int P = (W - 1) / 2;
  static constexpr int LINES = W > 0 ? K / W : 0;
  static constexpr int STRIDE = kTileSpan + 2 * P;
  // LDS tiling for the 2D stencils and the 27-point 3D stencil (the 125-point
  // tile would need 25 lines and throttle occupancy)
  static constexpr bool TILED = W > 0 && K != 125;
  static constexpr int LDS_DOUBLES = TILED ? LINES * STRIDE : 1;
};

// Per-lane (pointer, stride) row: global gathers.
template <int K, typename V>
__device__ __forceinline__ double op_row(unsigned meta, const OpView<V> &op, const double *__restrict__ x, int L,
                                         int Kdyn) {
  const unsigned g = meta & kMetaIndex;
  const bool uni = g == kMetaIndex;
  const V *__restrict__ v = uni ? op.ref : op.val + g;
  const size_t st = uni ? 1 : size_t(op.nv);
  double acc = 0.0;
  if (K > 0) {
#pragma unroll
    for (int s = 0; s < K; ++s) acc += double(v[s * st]) * x[L + op.off.off[s]];
  } else {
    for (int s = 0; s < Kdyn; ++s) acc += double(v[s * st]) * x[L + op.off.off[s]];
  }
  return acc;
}

// Stage the x window of the workgroup's rows [first, first + kTileRows) into
// LDS.  Returns the workgroup's Lmin, or -1 when the span exceeds the tile
// (then the rows use global gathers).  All threads of the workgroup call it.
template <int K>
__device__ __forceinline__ int stage_tile(const int32_t *__restrict__ row_lat, int first, int n,
                                          const Offsets &off, const double *__restrict__ x, double *lds) {
  using SS = StencilShape<K>;
  __shared__ int s_lo, s_hi;
  if (threadIdx.x == 0) {
    const int last = min(first + kTileRows, n) - 1;
    s_lo = row_lat[first];
    s_hi = row_lat[last];
  }
  __syncthreads();
  const int lo = s_lo, hi = s_hi;
  const int span = hi - lo + 1 + 2 * SS::P;
  if (hi - lo + 1 > kTileSpan) return -1;
#pragma unroll
  for (int j = 0; j < SS::LINES; ++j) {
    const double *src = x + (lo - SS::P + off.off[j * SS::W + SS::P]);
    for (int t = threadIdx.x; t < span; t += kTileRows) lds[j * SS::STRIDE + t] = src[t];
  }
  __syncthreads();
  return lo;
}

// One row from the LDS tile (lo = the workgroup's Lmin).
template <int K, typename V>
__device__ __forceinline__ double op_row_tile(unsigned meta, const OpView<V> &op, const double *lds, int L, int lo,
                                              bool wave_uniform) {
  using SS = StencilShape<K>;
  const int c0 = L - lo;  // column of dx = -p
  double acc = 0.0;
  if (wave_uniform) {
    const V *__restrict__ ref = op.ref;
#pragma unroll
    for (int s = 0; s < K; ++s) acc += double(ref[s]) * lds[(s / SS::W) * SS::STRIDE + c0 + (s % SS::W)];
  } else {
    const unsigned g = meta & kMetaIndex;
    const bool uni = g == kMetaIndex;
    const V *__restrict__ v = uni ? op.ref : op.val + g;
    const size_t st = uni ? 1 : size_t(op.nv);
#pragma unroll
    for (int s = 0; s < K; ++s) acc += double(v[s * st]) * lds[(s / SS::W) * SS::STRIDE + c0 + (s % SS::W)];
  }
  return acc;
}

// A x for row i of a workgroup staged with stage_tile (lo >= 0) or by
// global gathers (lo < 0).  `active` = this thread owns a row.
template <int K, typename V>
__device__ __forceinline__ double op_apply(bool active, unsigned meta, const OpView<V> &op,
                                           const double *__restrict__ x, int L, int lo, const double *lds, int Kdyn) {
  if constexpr (StencilShape<K>::TILED) {
    if (lo >= 0) {
      const bool wu = __all(!active || (meta & kMetaIndex) == kMetaIndex);
      return active ? op_row_tile<K, V>(meta, op, lds, L, lo, wu) : 0.0;
    }
  }
  return active ? op_row<K, V>(meta, op, x, L, Kdyn) : 0.0;
}

}  // namespace imsmg
