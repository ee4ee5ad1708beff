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
//     are read with fully coalesced, fully active vector loads; their
//     results go back to the rows' own lanes through LDS.
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
  static constexpr int WINDOW = WX * WY * WZ;
  // x window, then one exchange slot per lattice point of the box
  static constexpr int LDS_DOUBLES = TILED ? WINDOW + kTileRows : 1;
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
  const size_t nv = size_t(op.nv);
  double acc = 0.0;
  if (K > 0) {
#pragma unroll
    for (int s = 0; s < K; ++s)
      acc += double(uni ? op.ref[s] : op.val[stored_at<V>(nv, g, s)]) * x[L + op.off.off[s]];
  } else {
    for (int s = 0; s < Kdyn; ++s)
      acc += double(uni ? op.ref[s] : op.val[stored_at<V>(nv, g, s)]) * x[L + op.off.off[s]];
  }
  return acc;
}

// The K values of stored row g in slot order, one 16-byte load per slot
// group (SlotGroup): f(s, a_s) for s = 0 .. K-1; NT: non-temporal loads.
template <int K, typename V, bool NT, typename F>
__device__ __forceinline__ void stored_row_slots_nt(const V *__restrict__ val, size_t nv, int g, F &&f) {
  constexpr int G = SlotGroup<V>::G;
  constexpr int NG = (K + G - 1) / G;
  if constexpr (G == 2) {
    const double2 *__restrict__ p = reinterpret_cast<const double2 *>(val) + g;
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      const double2 v = stream_load<NT>(p + q * nv);
      f(2 * q, v.x);
      if (2 * q + 1 < K) f(2 * q + 1, v.y);
    }
  } else {
    const float4 *__restrict__ p = reinterpret_cast<const float4 *>(val) + g;
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      const float4 v = stream_load<NT>(p + q * nv);
      f(4 * q, double(v.x));
      if (4 * q + 1 < K) f(4 * q + 1, double(v.y));
      if (4 * q + 2 < K) f(4 * q + 2, double(v.z));
      if (4 * q + 3 < K) f(4 * q + 3, double(v.w));
    }
  }
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

// The x window of the tile box: window point (wx, wy, wz) is lattice point
// (x0 - p + wx, y0 - p + wy, z0 - p + wz), 0 outside the lattice (such points
// only meet zero coefficients).  tile_load issues every load of a thread
// (they depend on the box only), tile_store writes them to LDS once they have
// arrived (the caller synchronizes).
template <int K>
struct TileRegs {
  static constexpr int PER = StencilShape<K>::TILED ? (StencilShape<K>::WINDOW + kTileRows - 1) / kTileRows : 1;
  double v[PER];
};

template <int K, typename V>
__device__ __forceinline__ void tile_load(const TileBox &tb, const OpView<V> &op, const double *__restrict__ x,
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
    const bool in = e < SS::WINDOW && gx >= 0 && gx < op.sx && gy >= 0 && gy < op.sy && gz >= 0 && gz < op.sz;
    // unconditional load (lattice point 0 outside the box), so that the
    // loads stay countable and a later wait for an older load need not
    // include them
    const double t = x[in ? gx + op.sx * (gy + op.sy * gz) : 0];
    w.v[q] = in ? t : 0.0;
  }
}

template <int K>
__device__ __forceinline__ void tile_store(const TileRegs<K> &w, double *lds) {
#pragma unroll
  for (int q = 0; q < TileRegs<K>::PER; ++q) {
    const int e = threadIdx.x + q * kTileRows;
    if (e < StencilShape<K>::WINDOW) lds[e] = w.v[q];
  }
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

// window corner offset of the box's lattice point t (= tx + TX (ty + TY tz),
// the thread that owns it)
template <int K>
__device__ __forceinline__ int tile_local(int t) {
  using SS = StencilShape<K>;
  const int tx = t % SS::TX, ty = (t / SS::TX) % SS::TY, tz = t / (SS::TX * SS::TY);
  return (tz * SS::WY + ty) * SS::WX + tx;
}

// Coarse window of a tile for the fused prolongation (2D): the coarse points
// the two-scale bands of the x window reach (at most W / 2 + kBandMax + 1
// per axis, checked on the host), per window index along x and y the band
// (local first index, length, kBandMax coefficients), and the x-pass sums
// (one per coarse row of the window and window column).
template <int K>
struct ProShape {
  using SS = StencilShape<K>;
  static constexpr int CWX = SS::WX / 2 + kBandMax + 1;
  static constexpr int CWY = SS::WY / 2 + kBandMax + 1;
  static constexpr int CWN = CWX * CWY;
  static constexpr int NB = SS::WX + SS::WY;  // band rows
  static constexpr int NT = CWY * SS::WX;     // x-pass sums
  static constexpr int PERC = (CWN + kTileRows - 1) / kTileRows;
  static constexpr int PERT = (NT + kTileRows - 1) / kTileRows;
  // LDS (doubles) after the x window and the exchange slots: coarse window,
  // band coefficients, band first index and length (two ints per double),
  // x-pass sums
  static constexpr int LDS_EXTRA = CWN + NB * kBandMax + NB + NT;
};

// Grid of a stencil kernel over a level: one workgroup per lattice tile when
// K is tiled, else one per kTileRows rows.
template <typename V>
inline int stencil_grid(int K, int n, const OpView<V> &op) {
  const bool tiled = K == 9 || K == 25 || K == 49 || K == 27 || K == 125;
  return tiled ? op.ntiles : (n + kTileRows - 1) / kTileRows;
}

// Applies the operator to every row of workgroup blk and hands each row
// exactly once to the epilogue (NT: the stored values with non-temporal
// loads, for levels whose values far exceed the caches; OpView::stream): epi.post(i, L, meta, (A x)_L, x_L, pre) with
// pre = epi.pre(i, L) fetched before the tile is staged (so that its loads
// overlap the staging); post returns a pair of partial sums that tile_rows
// adds up per thread.  Tiled K: blk is a lattice tile; otherwise rows
// [blk * kTileRows, ...).  With done != nullptr nothing is computed or stored
// once *done is set.  Every thread of the workgroup must call it.
//
// Tiled, the dependent memory steps are: (1) the x window (it depends on
// the box only), the lane's row index and the tile's stored-row range;
// (2) the lane's meta and epilogue loads, the stored rows' owners.  A stored
// row's A x is computed on a packed lane and handed to the lane owning the row
// through LDS, so that every epilogue runs on its own lane's data.
//
// PRO: the rows see x + R^T xc (pv): the band rows of the window and the
// coarse window origins join load (1), the coarse window load (2); the
// corrections are added to the window registers before they go to LDS, in
// the order of the transfer kernel (bitwise the same x + R^T xc).
template <int K, typename V, typename Epi, bool PRO = false, bool NT = false>
__device__ __forceinline__ double2 tile_rows(int n, int blk, const OpView<V> &op,
                                             const int32_t *__restrict__ row_lat, const uint32_t *__restrict__ meta,
                                             const double *__restrict__ x, double *lds, int Kdyn, const Epi &epi,
                                             const int32_t *done = nullptr, const ProlongView *pv = nullptr) {
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
    // the row index first: the wait for it (loads complete in issue order)
    // then does not include the window
    const int i0 = op.lat2row[L];  // L = 0 outside the box: a valid address
    const int i = inbox ? i0 : -1;
    TileRegs<K> w;
    tile_load<K>(tb, op, x, w);
    using PS = ProShape<K>;
    // PRO, load (1): this lane's band row (lanes < NB) and the coarse origins
    int bsx = 0, bln = 0;
    double bcf[kBandMax];
    int co[2] = {0, 0};
    if constexpr (PRO) {
      static_assert(SS::DIM == 2, "fused prolongation: 2D lattices");
      co[0] = pv->org[blk % op.ntx];
      co[1] = pv->org[op.ntx + (blk / op.ntx) % op.nty];
      const int e = threadIdx.x;
      const int ax = e < SS::WX ? 0 : 1;
      const int f = (ax == 0 ? tb.x0 + e : tb.y0 + e - SS::WX) - SS::P;
      const int sa = ax == 0 ? op.sx : op.sy;
      const bool ok = e < PS::NB && f >= 0 && f < sa;
      const int fc = ok ? f : 0;  // unconditional loads
      const int st = pv->start[fc], ln = pv->len[fc];
#pragma unroll
      for (int a = 0; a < kBandMax; ++a) {
        const double cv = pv->coef[fc * kBandMax + a];  // stride kBandMax, zero-padded
        bcf[a] = ok ? cv : 0.0;
      }
      bsx = (ok && ln > 0) ? st : 0;
      bln = ok ? ln : 0;
    }
    const int g = op.tile_g0[blk] + threadIdx.x;
    const bool act2 = g < op.tile_g0[blk + 1];
    unsigned m = 0u;
    Pre p1{};
    if (i >= 0) {
      m = meta[i];
      p1 = epi.pre(i, L);
    }
    const int own2 = act2 ? op.sloc[g] : 0;
    if (done && *done) return acc;
    double *xch = lds + SS::WINDOW;
    if constexpr (PRO) {
      // load (2): the coarse window
      double cwv[PS::PERC];
#pragma unroll
      for (int q = 0; q < PS::PERC; ++q) {
        const int e = threadIdx.x + q * kTileRows;
        const int cx = co[0] + e % PS::CWX;
        const int cy = co[1] + e / PS::CWX;
        const bool in = e < PS::CWN && cx < pv->cs && cy < pv->cs;
        const double t = pv->xc[in ? cx + size_t(pv->cs) * cy : 0];
        cwv[q] = in ? t : 0.0;
      }
      double *cw = xch + kTileRows;
      double *bc = cw + PS::CWN;
      int *bi = reinterpret_cast<int *>(bc + PS::NB * kBandMax);
      double *tx1 = bc + PS::NB * kBandMax + PS::NB;
      if (threadIdx.x < PS::NB) {
        const int ax = threadIdx.x < SS::WX ? 0 : 1;
#pragma unroll
        for (int a = 0; a < kBandMax; ++a) bc[threadIdx.x * kBandMax + a] = bcf[a];
        bi[2 * threadIdx.x] = max(bsx - co[ax], 0);  // length-0 bands: 0 (zero coefficients)
        bi[2 * threadIdx.x + 1] = bln;
      }
#pragma unroll
      for (int q = 0; q < PS::PERC; ++q) {
        const int e = threadIdx.x + q * kTileRows;
        if (e < PS::CWN) cw[e] = cwv[q];
      }
      __syncthreads();
      // R^T xc separably, in the transfer kernel's order: per coarse row and
      // window column t = sum_a cx[a] xc[row][sx + a], then per window point
      // sum_b cy[b] t[sy + b].  Entries past a band's length have zero
      // coefficients; their (clamped, finite) inputs add exact zeros.
      const int W = pv->W;
#pragma unroll
      for (int q = 0; q < PS::PERT; ++q) {
        const int e = threadIdx.x + q * kTileRows;
        if (e < PS::NT) {
          const int wx = e % SS::WX, cyl = e / SS::WX;
          const double *cxv = bc + wx * kBandMax;
          const double *row = cw + cyl * PS::CWX;
          const int sxl = bi[2 * wx];
          double t = 0.0;
          for (int a = 0; a < W; ++a) t += cxv[a] * row[min(sxl + a, PS::CWX - 1)];
          tx1[e] = t;
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < TileRegs<K>::PER; ++q) {
        const int e = threadIdx.x + q * kTileRows;
        const int wx = e % SS::WX, wy = e / SS::WX;
        const int gx2 = tb.x0 - SS::P + wx, gy2 = tb.y0 - SS::P + wy;
        const bool in = e < SS::WINDOW && gx2 >= 0 && gx2 < op.sx && gy2 >= 0 && gy2 < op.sy;
        if (!in) continue;
        const int ry = SS::WX + wy;
        const double *cyv = bc + ry * kBandMax;
        const int syl = bi[2 * ry];
        double corr = 0.0;
        for (int b = 0; b < W; ++b) corr += cyv[b] * tx1[min(syl + b, PS::CWY - 1) * SS::WX + wx];
        w.v[q] = w.v[q] + corr;
      }
    }
    tile_store<K>(w, lds);
    __syncthreads();
    const double *t = lds + tile_local<K>(threadIdx.x);
    double ax = 0.0;
    // phase 1: rows on the reference stencil
    if (i >= 0 && (m & kMetaIndex) == kMetaIndex) {
      const ConstPtr<double> ref = (ConstPtr<double>)op.refd;
#pragma unroll
      for (int s = 0; s < K; ++s) ax += ref[s] * tile_at<K>(t, s);
    }
    // phase 2: the tile's stored rows, packed onto the first lanes
    if (act2) {
      const double *t2 = lds + tile_local<K>(own2);
      double a2 = 0.0;
      stored_row_slots_nt<K, V, NT>(op.val, size_t(op.nv), g, [&](int s, double a) { a2 += a * tile_at<K>(t2, s); });
      xch[own2] = a2;
    }
    __syncthreads();
    if (i >= 0) {
      if ((m & kMetaIndex) != kMetaIndex) ax = xch[threadIdx.x];
      const double2 c = epi.post(i, L, m, ax, tile_center<K>(t), p1);
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
