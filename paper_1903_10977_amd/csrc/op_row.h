// Rows of the compressed lattice-ELL operator: (A x)_L = sum_s a_s x[L + off_s].
//
// The stencil kernels are limited by the vector memory instructions they
// issue and by the dependent round trips of a workgroup rather than by HBM
// bytes (traffic measures close to the algorithmic bytes), so these helpers
// minimise both:
//   * lattice tiles: a workgroup owns a box of the level's lattice (32 x 8
//     points in 2D, 16 x 4 x 4 in 3D: one lattice point per thread); the x
//     window of the box widened by the stencil reach p on every side is
//     loaded once, coalesced along x, into LDS, and the K gathers of a row
//     become LDS reads (2.1 staged values per point for the 49-point 2D
//     stencil, 5 for the 125-point 3D stencil);
//   * two phases per tile: (1) every row whose values equal the reference
//     stencil takes its K coefficients from scalar loads (wave-uniform
//     addresses); (2) the tile's stored rows, numbered consecutively tile by
//     tile, are packed onto the first lanes, so that their slot-major values
//     are read with fully coalesced, fully active vector loads.
// Generic K gathers per lane from global memory (one row per thread).
// Shared by the level and CG kernels.
#pragma once
#include "imsmg_internal.h"

namespace imsmg {

// register cap of the tiled kernels: 4 resident workgroups per CU (16 waves);
// a tighter budget spills in the FP64 kernels
constexpr int kTileBlocksPerCU = 4;

template <int K>
struct StencilShape {
  static constexpr int W = K == 9 ? 3 : K == 25 ? 5 : K == 49 ? 7 : K == 27 ? 3 : K == 125 ? 5 : 0;
  static constexpr int P = W > 0 ? (W - 1) / 2 : 0;
  static constexpr int DIM = (K == 27 || K == 125) ? 3 : 2;
  static constexpr bool TILED = W > 0;
  // lattice box of a workgroup (TX * TY * TZ == kTileRows) and its window
  static constexpr int TX = DIM == 2 ? kTile2X : kTile3X;
  static constexpr int TY = DIM == 2 ? kTile2Y : kTile3Y;
  static constexpr int TZ = DIM == 2 ? 1 : kTile3Z;
  static constexpr int WX = TX + 2 * P;
  static constexpr int WY = TY + 2 * P;
  static constexpr int WZ = DIM == 2 ? 1 : TZ + 2 * P;
  static constexpr int LDS_DOUBLES = TILED ? WX * WY * WZ : 1;
  static_assert(!TILED || TX * TY * TZ == kTileRows, "one lattice point per thread");
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

// Lattice box of tile b (x fastest over the tile grid).
struct TileBox {
  int x0, y0, z0;
};

template <int K>
__device__ __forceinline__ TileBox tile_box(int b, int ntx, int nty) {
  using SS = StencilShape<K>;
  const int bx = b % ntx;
  const int r = b / ntx;
  return {bx * SS::TX, (r % nty) * SS::TY, (r / nty) * SS::TZ};
}

// Stages the x window of the tile box into LDS: window point (wx, wy, wz) is
// lattice point (x0 - p + wx, y0 - p + wy, z0 - p + wz), 0 outside the
// lattice (such points only meet zero coefficients).  All loads of a thread
// are issued before its LDS writes, so that it waits for them once.  Every
// thread of the workgroup must call it (it synchronizes).
template <int K, typename V>
__device__ __forceinline__ void tile_stage(const TileBox &tb, const OpView<V> &op, const double *__restrict__ x,
                                           double *lds) {
  using SS = StencilShape<K>;
  constexpr int N = SS::WX * SS::WY * SS::WZ;
  constexpr int PER = (N + kTileRows - 1) / kTileRows;
  double v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * kTileRows;
    const int wx = e % SS::WX;
    const int wy = (e / SS::WX) % SS::WY;
    const int wz = e / (SS::WX * SS::WY);
    const int gx = tb.x0 - SS::P + wx;
    const int gy = tb.y0 - SS::P + wy;
    const int gz = tb.z0 - (SS::DIM == 3 ? SS::P : 0) + wz;
    const bool in = e < N && gx >= 0 && gx < op.sx && gy >= 0 && gy < op.sy && gz >= 0 && gz < op.sz;
    v[q] = in ? x[gx + op.sx * (gy + op.sy * gz)] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * kTileRows;
    if (e < N) lds[e] = v[q];
  }
  __syncthreads();
}

// window entry of slot s for the row whose window corner (dx = dy = dz = -p)
// is t
template <int K>
__device__ __forceinline__ double tile_at(const double *t, int s) {
  using SS = StencilShape<K>;
  const int dx = s % SS::W, dy = (s / SS::W) % SS::W, dz = s / (SS::W * SS::W);
  return t[(dz * SS::WY + dy) * SS::WX + dx];
}

template <int K>
__device__ __forceinline__ double tile_center(const double *t) {
  using SS = StencilShape<K>;
  return t[((SS::DIM == 3 ? SS::P : 0) * SS::WY + SS::P) * SS::WX + SS::P];
}

// window corner offset of the lattice point at box-local (tx, ty, tz)
template <int K>
__device__ __forceinline__ int tile_local(int tx, int ty, int tz) {
  using SS = StencilShape<K>;
  return (tz * SS::WY + ty) * SS::WX + tx;
}

// Grid of a stencil kernel over a level: one workgroup per lattice tile when
// K is tiled, else one per kTileRows rows.
template <typename V>
inline int stencil_grid(int K, int n, const OpView<V> &op) {
  const bool tiled = K == 9 || K == 25 || K == 49 || K == 27 || K == 125;
  return tiled ? op.ntiles : (n + kTileRows - 1) / kTileRows;
}

// Applies the operator to every row of workgroup blk and hands each row
// exactly once to the epilogue: epi.post(i, L, meta, (A x)_L, x_L, pre) with
// pre = epi.pre(i, L) fetched before the tile is staged (so that its loads
// overlap the staging); post returns a pair of partial sums that tile_rows
// adds up per thread.  Tiled K: blk is a lattice tile; otherwise rows
// [blk * kTileRows, ...).  With done != nullptr nothing is computed or stored
// once *done is set.  Every thread of the workgroup must call it.
template <int K, typename V, typename Epi>
__device__ __forceinline__ double2 tile_rows(int n, int blk, const OpView<V> &op,
                                             const int32_t *__restrict__ row_lat, const uint32_t *__restrict__ meta,
                                             const double *__restrict__ x, double *lds, int Kdyn, const Epi &epi,
                                             const int32_t *done = nullptr) {
  using Pre = typename Epi::Pre;
  using SS = StencilShape<K>;
  double2 acc = make_double2(0.0, 0.0);
  if constexpr (SS::TILED) {
    const TileBox tb = tile_box<K>(blk, op.ntx, op.nty);
    const int tx = threadIdx.x % SS::TX;
    const int ty = (threadIdx.x / SS::TX) % SS::TY;
    const int tz = threadIdx.x / (SS::TX * SS::TY);
    const int gx = tb.x0 + tx, gy = tb.y0 + ty, gz = tb.z0 + tz;
    const bool inbox = gx < op.sx && gy < op.sy && gz < op.sz;
    const int L = inbox ? gx + op.sx * (gy + op.sy * gz) : 0;
    int i = -1;
    unsigned m = 0u;
    Pre p1{};
    if (inbox) {
      i = op.lat2row[L];
      if (i >= 0) {
        m = meta[i];
        p1 = epi.pre(i, L);
      }
    }
    const bool act = i >= 0;
    // the tile's stored rows (phase 2), fetched before staging as well
    const int g = op.tile_g0[blk] + threadIdx.x;
    const bool act2 = g < op.tile_g0[blk + 1];
    int i2 = 0, L2 = 0, o2 = 0;
    unsigned m2 = 0u;
    Pre p2{};
    if (act2) {
      i2 = op.srow[g];
      L2 = op.slat[g];
      o2 = op.sloc[g];
      m2 = meta[i2];
      p2 = epi.pre(i2, L2);
    }
    if (done && *done) return acc;
    if (!op.tile_any[blk]) return acc;  // no active row in the box (uniform)
    tile_stage<K>(tb, op, x, lds);
    // phase 1: rows on the reference stencil
    if (act && (m & kMetaIndex) == kMetaIndex) {
      const double *t = lds + tile_local<K>(tx, ty, tz);
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
      const double *t = lds + o2;
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
  } else {
    if (done && *done) return acc;
    const int i = blk * kTileRows + threadIdx.x;
    if (i < n) {
      const int L = row_lat[i];
      const unsigned m = meta[i];
      const Pre p1 = epi.pre(i, L);
      const double2 c = epi.post(i, L, m, op_row<K, V>(m, op, x, L, Kdyn), x[L], p1);
      acc.x += c.x;
      acc.y += c.y;
    }
    return acc;
  }
}

}  // namespace imsmg
