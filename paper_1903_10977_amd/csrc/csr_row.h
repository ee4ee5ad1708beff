// Rows of a general sparse level: locally refined (truncated hierarchical
// B-spline) levels have no function lattice and no common stencil, so their
// operator is kept as CSR and a row's product reads its own column indices.
//
// LN consecutive lanes share one row: lane t adds the entries t, t + LN, ...
// of the row in order, then a butterfly of lane exchanges forms the sum
// (every lane ends with the same value; each partial sum is formed from the
// same operands in the same order on every run, so the result is
// deterministic).  The row's first lane hands (A x)_i to the epilogue, in
// the form the lattice kernels use: epi.post(i, i, meta[i] (0 without meta),
// (A x)_i, x_i, epi.pre(i, i)) (vectors of general levels are indexed by row).
#pragma once
#include "imsmg_internal.h"

namespace imsmg {

template <int LN, typename V, typename Epi>
__device__ __forceinline__ double2 csr_rows(int n, const CsrView<V> &A, const uint32_t *__restrict__ meta,
                                            const double *__restrict__ x, const Epi &epi,
                                            const int32_t *done = nullptr) {
  static_assert(LN == 4 || LN == 8 || LN == 16, "lanes per row");
  double2 acc = make_double2(0.0, 0.0);
  if (done && *done) return acc;  // uniform over the workgroup
  const int i = blockIdx.x * (int(blockDim.x) / LN) + int(threadIdx.x) / LN;
  const int lane = int(threadIdx.x) % LN;
  const bool live = i < n;
  typename Epi::Pre pre{};
  double ax = 0.0;
  if (live) {
    if (lane == 0) pre = epi.pre(i, i);
    const int beg = A.ptr[i], end = A.ptr[i + 1];
    for (int k = beg + lane; k < end; k += LN) ax += double(A.val[k]) * x[A.col[k]];
  }
#pragma unroll
  for (int o = LN / 2; o > 0; o >>= 1) ax += __shfl_xor(ax, o, 64);
  if (live && lane == 0) acc = epi.post(i, i, meta ? meta[i] : 0u, ax, x[i], pre);
  return acc;
}

// workgroups of a CSR launch with LN lanes per row (256 threads)
inline int csr_grid(int n, int LN) { return n < 1 ? 1 : (n + 256 / LN - 1) / (256 / LN); }

}  // namespace imsmg
