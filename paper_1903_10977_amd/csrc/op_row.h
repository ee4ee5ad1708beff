// One row of the compressed lattice-ELL operator: sum_s a_s x[L + off_s],
// a_s from the reference stencil (uniform rows) or from the row's own
// slot-major values.  Shared by the level and CG kernels.
#pragma once
#include "imsmg_internal.h"

namespace imsmg {

template <int K, typename V>
__device__ __forceinline__ double op_row(unsigned meta, const OpView<V> &op, const double *__restrict__ x, int L,
                                         int Kdyn) {
  double acc = 0.0;
  const unsigned g = meta & kMetaIndex;
  if (K > 0) {
    if (g == kMetaIndex) {
#pragma unroll
      for (int s = 0; s < K; ++s) acc += double(op.ref.v[s]) * x[L + op.off.off[s]];
    } else {
      const V *__restrict__ v = op.val + g;
#pragma unroll
      for (int s = 0; s < K; ++s) acc += double(v[size_t(s) * op.nv]) * x[L + op.off.off[s]];
    }
  } else {
    if (g == kMetaIndex) {
      for (int s = 0; s < Kdyn; ++s) acc += double(op.ref.v[s]) * x[L + op.off.off[s]];
    } else {
      const V *__restrict__ v = op.val + g;
      for (int s = 0; s < Kdyn; ++s) acc += double(v[size_t(s) * op.nv]) * x[L + op.off.off[s]];
    }
  }
  return acc;
}

}  // namespace imsmg
