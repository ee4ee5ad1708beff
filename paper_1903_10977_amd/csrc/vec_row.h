// Rows of a vector operator (linear elasticity: eq:weakMulti with d
// displacement components) on the lattice tiles of op_row.h.
//
// A vector level stores its operator as ncomp x ncomp component blocks
// A_(c,e), each a compressed lattice-ELL operator on the scalar lattice
// (reference stencil + stored rows in slot groups), and its vectors as ncomp
// consecutive padded scalar arrays (component e at x + e * cstride).  A
// workgroup owns one lattice tile and one output component c (blockIdx.y):
// for e = 0 .. ncomp-1 it stages the tile's window of component e in LDS and
// adds the tile's rows of A_(c,e) x_e (reference rows from scalar loads,
// stored rows on packed lanes, as in tile_rows), in the fixed order e = 0, 1,
// .. ; the epilogue then sees (A x)_(c,L) once per row, like a scalar row.
#pragma once
#include "op_row.h"

namespace imsmg {

// The x window of tile box tb for one component (zeros outside the lattice).
template <int K>
__device__ __forceinline__ void vtile_load(const TileBox &tb, int sx, int sy, int sz, const double *__restrict__ x,
                                           TileRegs<K> &w) {
  using SS = StencilShape<K>;
#pragma unroll
  for (int q = 0; q < TileRegs<K>::PER; ++q) {
    const int e = threadIdx.x + q * kTileRows;
    const int wx = e % SS::WX;
    const int wy = (e / SS::WX) % SS::WY;
    const int wz = e / (SS::WX * SS::WY);
    const int gx = tb.x0 - SS::P + wx;
    const int gy = tb.y0 - SS::P + wy;
    const int gz = tb.z0 - (SS::DIM == 3 ? SS::P : 0) + wz;
    const bool in = e < SS::WINDOW && gx >= 0 && gx < sx && gy >= 0 && gy < sy && gz >= 0 && gz < sz;
    const double t = x[in ? gx + sx * (gy + sy * gz) : 0];
    w.v[q] = in ? t : 0.0;
  }
}

// Applies output component c's block row to every row of tile blk and hands
// each row once to epi.post(i, L, flags[c ns + i], (A x)_(c,L), x_(c,L), pre);
// epi's vectors are those of component c (the caller offsets them).  The
// windows of all components are loaded together at the start (one round of
// global loads), then staged in LDS one after the other (one window and one
// set of exchange slots in LDS, as the scalar tiles, so the occupancy stays
// that of the scalar kernels); a row adds its block results in the order
// e = 0, 1, ...  Every thread of the workgroup must call it; tiled K only;
// lds holds VecShape<K>::LDS_DOUBLES doubles.
template <int K>
struct VecShape {
  static constexpr int LDS_DOUBLES = StencilShape<K>::WINDOW + kTileRows;
};

template <int K, typename V, typename Epi>
__device__ __forceinline__ double2 vtile_rows(int blk, int c, const VecOps<V> &ops, const uint32_t *__restrict__ flags,
                                              const double *__restrict__ x, double *lds, const Epi &epi,
                                              const int32_t *done) {
  static_assert(StencilShape<K>::TILED, "vector operators need a tiled stencil");
  using Pre = typename Epi::Pre;
  using SS = StencilShape<K>;
  double2 acc = make_double2(0.0, 0.0);
  const int nc = ops.ncomp;
  const TileBox tb = tile_box<K>(blk, ops.ntx, ops.nty);
  const int tx = threadIdx.x % SS::TX;
  const int ty = (threadIdx.x / SS::TX) % SS::TY;
  const int tz = threadIdx.x / (SS::TX * SS::TY);
  const int gx = tb.x0 + tx, gy = tb.y0 + ty, gz = tb.z0 + tz;
  const bool inbox = gx < ops.sx && gy < ops.sy && gz < ops.sz;
  const int L = inbox ? gx + ops.sx * (gy + ops.sy * gz) : 0;
  const int i0 = ops.lat2row[L];
  const int i = inbox ? i0 : -1;
  TileRegs<K> w[kMaxComp];
#pragma unroll
  for (int e = 0; e < kMaxComp; ++e)
    if (e < nc) vtile_load<K>(tb, ops.sx, ops.sy, ops.sz, x + e * ops.cstride, w[e]);
  Pre p1{};
  unsigned mf = 0u;
  if (i >= 0) {
    p1 = epi.pre(i, L);
    mf = flags[size_t(c) * ops.ns + i];
  }
  if (done && *done) return acc;
  double *xch = lds + SS::WINDOW;
  const double *t = lds + tile_local<K>(threadIdx.x);
  double ax = 0.0, xc = 0.0;
#pragma unroll
  for (int e = 0; e < kMaxComp; ++e) {
    if (e >= nc) break;
    const int b = c * nc + e;
    const int g = ops.tile_g0[b][blk] + threadIdx.x;
    const bool act2 = g < ops.tile_g0[b][blk + 1];
    const int own2 = act2 ? ops.sloc[b][g] : 0;
    const unsigned m = i >= 0 ? ops.meta[b][i] : 0u;
    if (e > 0) __syncthreads();  // the previous component's window and exchange are consumed
    tile_store<K>(w[e], lds);
    __syncthreads();
    double a1 = 0.0;
    if (i >= 0 && (m & kMetaIndex) == kMetaIndex) {
      const ConstPtr<double> ref = (ConstPtr<double>)ops.refd[b];
#pragma unroll
      for (int s = 0; s < K; ++s) a1 += ref[s] * tile_at<K>(t, s);
    }
    if (act2) {
      const double *t2 = lds + tile_local<K>(own2);
      double a2 = 0.0;
      // vector levels stream their values (nine blocks per point: the
      // elasticity operators far exceed the caches on every level that counts)
      stored_row_slots_nt<K, V, true>(ops.val[b], size_t(ops.nv[b]), g,
                                      [&](int s, double v) { a2 += v * tile_at<K>(t2, s); });
      xch[own2] = a2;
    }
    __syncthreads();
    if (i >= 0) {
      ax += (m & kMetaIndex) == kMetaIndex ? a1 : xch[threadIdx.x];
      if (e == c) xc = tile_center<K>(t);
    }
  }
  if (i >= 0) {
    const double2 r = epi.post(i, L, mf, ax, xc, p1);
    acc.x += r.x;
    acc.y += r.y;
  }
  return acc;
}

}  // namespace imsmg
