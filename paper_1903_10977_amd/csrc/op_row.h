// Rows of the compressed lattice-ELL operator: (A x)_L = sum_s a_s x[L + off_s].
//
// The stencil kernels are limited by vector address processing rather than by
// HBM (the level's matrix and vectors stay resident in the Infinity Cache
// between the V-cycle's sweeps), so these helpers minimise the vector memory
// instructions per row:
//   * LDS tile: the kTileRows consecutive active rows of a workgroup span the
//     lattice range [lo, hi] (rows are numbered in lattice order); for every
//     stencil line (fixed dy, dz) the x window [lo - p, hi + p], shifted by
//     the line's offset, is loaded once and coalesced into LDS, and the K
//     gathers of a row become LDS reads;
//   * two phases per tile: (1) every row whose values equal the reference
//     stencil takes its K coefficients from scalar loads (wave-uniform
//     addresses); (2) the tile's stored rows, numbered consecutively, are
//     packed onto the first lanes, so that their slot-major values are read
//     with fully coalesced, fully active vector loads.
// Workgroups whose span exceeds kTileSpan (large holes of the domain), the
// 125-point 3D stencil and generic K gather per lane from global memory.
// Shared by the level and CG kernels.
#pragma once
#include "imsmg_internal.h"

namespace imsmg {

constexpr int kTileSpan = 512;  // largest lattice span of a workgroup staged in LDS
// register cap of the tiled kernels: 4 resident workgroups per CU (16 waves);
// the 49-point tile (7 x 518 doubles) would allow 5 in 160 KiB of LDS, but the
// tighter register budget that needs spills in the FP64 kernels
constexpr int kTileBlocksPerCU = 4;

template <int K>
struct StencilShape {
  static constexpr int W = K == 9 ? 3 : K == 25 ? 5 : K == 49 ? 7 : K == 27 ? 3 : K == 125 ? 5 : 0;
  static constexpr int P = W > 0 ? (W - 1) / 2 : 0;
  static constexpr int LINES = W > 0 ? K / W : 0;
  static constexpr int STRIDE = kTileSpan + 2 * P;
  static constexpr bool TILED = W > 0 && K != 125;  // 125 points: 25 lines would throttle occupancy
  static constexpr int LDS_DOUBLES = TILED ? LINES * STRIDE : 1;
};

// Read-only device memory read with a wave-uniform address through the
// constant address space, so that it is fetched by scalar loads.
template <typename V>
using ConstPtr = const __attribute__((address_space(4))) V *;

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

constexpr int kTileDone = -2;  // tile_stage: the convergence flag is set, nothing to do

// Stages the x window of the workgroup's rows [first, min(first + kTileRows, n))
// into LDS and returns lo = row_lat[first], -1 when the operator is not tiled
// or the span exceeds kTileSpan, or kTileDone when *done is set (read
// together with the tile bounds, so that the flag adds no latency of its
// own).  Every thread of the workgroup must call it (it synchronizes); first < n.
template <int K>
__device__ __forceinline__ int tile_stage(const int32_t *__restrict__ row_lat, int first, int n, const Offsets &off,
                                          const double *__restrict__ x, double *lds, const int32_t *done) {
  using SS = StencilShape<K>;
  if constexpr (!SS::TILED) {
    return (done && *done) ? kTileDone : -1;
  } else {
    const int lo = row_lat[first];
    const int hi = row_lat[min(first + kTileRows, n) - 1];
    if (done && *done) return kTileDone;
    if (hi - lo + 1 > kTileSpan) return -1;
    const int span = hi - lo + 1 + 2 * SS::P;
    // all loads of the window first, then all LDS writes: the thread waits for
    // its loads once instead of once per element
    constexpr int PER = (SS::STRIDE + kTileRows - 1) / kTileRows;
    double v[SS::LINES][PER];
#pragma unroll
    for (int j = 0; j < SS::LINES; ++j) {
      const double *__restrict__ src = x + (lo - SS::P + off.off[j * SS::W + SS::P]);
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int t = threadIdx.x + q * kTileRows;
        v[j][q] = t < span ? src[t] : 0.0;
      }
    }
#pragma unroll
    for (int j = 0; j < SS::LINES; ++j)
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int t = threadIdx.x + q * kTileRows;
        if (t < span) lds[j * SS::STRIDE + t] = v[j][q];
      }
    __syncthreads();
    return lo;
  }
}

// tile entry of slot s for the row whose dx = -p column on line 0 is t
template <int K>
__device__ __forceinline__ double tile_at(const double *t, int s) {
  using SS = StencilShape<K>;
  return t[(s / SS::W) * SS::STRIDE + s % SS::W];
}

template <int K>
__device__ __forceinline__ double tile_center(const double *t) {
  using SS = StencilShape<K>;
  return t[(SS::LINES / 2) * SS::STRIDE + SS::P];
}

// Applies the operator to every row of a workgroup tile and hands each row
// exactly once to the epilogue: epi.post(i, L, meta, (A x)_L, x_L, pre) with
// pre = epi.pre(i, L) fetched before the tile is staged (so that its loads
// overlap the staging); post returns a pair of partial sums that tile_rows
// adds up per thread.  With done != nullptr nothing is computed or stored
// once *done is set.  Every thread of the workgroup must call it; first =
// the tile's first row (< n).
template <int K, typename V, typename Epi>
__device__ __forceinline__ double2 tile_rows(int n, int first, const OpView<V> &op,
                                             const int32_t *__restrict__ row_lat, const uint32_t *__restrict__ meta,
                                             const double *__restrict__ x, double *lds, int Kdyn, const Epi &epi,
                                             const int32_t *done = nullptr) {
  using Pre = typename Epi::Pre;
  double2 acc = make_double2(0.0, 0.0);
  const int i = first + threadIdx.x;
  const bool act = i < n;
  int L = 0;
  unsigned m = 0u;
  Pre p1{};
  if (act) {
    L = row_lat[i];
    m = meta[i];
    p1 = epi.pre(i, L);
  }
  if constexpr (StencilShape<K>::TILED) {
    // the tile's stored rows (phase 2), fetched before staging as well
    const int tile = first / kTileRows;
    const int g = op.tile_g0[tile] + threadIdx.x;
    const bool act2 = g < op.tile_g0[tile + 1];
    int i2 = 0, L2 = 0;
    unsigned m2 = 0u;
    Pre p2{};
    if (act2) {
      i2 = op.srow[g];
      L2 = op.slat[g];
      m2 = meta[i2];
      p2 = epi.pre(i2, L2);
    }
    const int lo = tile_stage<K>(row_lat, first, n, op.off, x, lds, done);
    if (lo == kTileDone) return acc;
    if (lo >= 0) {
      // phase 1: rows on the reference stencil
      if (act && (m & kMetaIndex) == kMetaIndex) {
        const double *t = lds + (L - lo);
        const ConstPtr<V> ref = (ConstPtr<V>)op.ref;
        double ax = 0.0;
#pragma unroll
        for (int s = 0; s < K; ++s) ax += double(ref[s]) * tile_at<K>(t, s);
        const double2 c = epi.post(i, L, m, ax, tile_center<K>(t), p1);
        acc.x += c.x;
        acc.y += c.y;
      }
      // phase 2: the tile's stored rows, packed onto the first lanes
      if (act2) {
        const double *t = lds + (L2 - lo);
        const V *__restrict__ v = op.val + g;
        const size_t nv = size_t(op.nv);
        double ax = 0.0;
#pragma unroll
        for (int s = 0; s < K; ++s) ax += double(v[s * nv]) * tile_at<K>(t, s);
        const double2 c = epi.post(i2, L2, m2, ax, tile_center<K>(t), p2);
        acc.x += c.x;
        acc.y += c.y;
      }
      return acc;
    }
  }
  if constexpr (!StencilShape<K>::TILED) {
    if (done && *done) return acc;
  }
  if (act) {
    const double2 c = epi.post(i, L, m, op_row<K, V>(m, op, x, L, Kdyn), x[L], p1);
    acc.x += c.x;
    acc.y += c.y;
  }
  return acc;
}

}  // namespace imsmg
