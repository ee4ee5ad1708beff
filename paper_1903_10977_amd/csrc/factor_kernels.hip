// Setup-time kernels: Schwarz block factorization, coarsest-level inverse,
// N_K counts for the damping gamma = 1 / max_K N_K (eq:applyCS).
//
// Block factorization (smoothers subsection, additive Schwarz and the remark
// on eigenvalues of the order of machine precision): one workgroup per block
// gathers A_j = P_j^T A P_j from the lattice-ELL operator (or, on general
// sparse levels, from the CSR operator) into LDS and runs a
// cyclic two-sided Jacobi eigensolver with the round-robin parallel ordering
// (n/2 disjoint rotations per step, rows then columns, eigenvectors
// accumulated alongside).  Jacobi with the relative off-diagonal test keeps
// small eigenvalues accurate relative to the diagonal scale, which is what
// the removal decision needs.  While the smallest eigenvalue is below
// ratio x (largest diagonal entry), the function with the largest |v_i| in
// that eigenvector (lowest index on ties) leaves the block and the block is
// re-factorized.  The kept block's inverse V diag(1/lambda) V^T is written
// column-major.
#include "imsmg_internal.h"

namespace imsmg {

constexpr int kFacThreads = 256;

struct LatticeGeom {
  int dim, nx, ny, reach, W;
};

__device__ __forceinline__ int slot_of(const LatticeGeom &g, int la, int lb) {
  // lattice offset lb - la as a stencil slot, -1 when outside the stencil
  int ax = la % g.nx, ay = (la / g.nx) % g.ny, az = la / (g.nx * g.ny);
  int bx = lb % g.nx, by = (lb / g.nx) % g.ny, bz = lb / (g.nx * g.ny);
  int dx = bx - ax, dy = by - ay, dz = bz - az;
  if (dx < -g.reach || dx > g.reach || dy < -g.reach || dy > g.reach) return -1;
  if (g.dim == 3) {
    if (dz < -g.reach || dz > g.reach) return -1;
    return ((dz + g.reach) * g.W + (dy + g.reach)) * g.W + (dx + g.reach);
  }
  return (dy + g.reach) * g.W + (dx + g.reach);
}

// A_ab of a block from the lattice-ELL operator (members' rows and lattice
// points) or from a CSR operator (members' rows; binary search in the row)
struct LatticeGather {
  LatticeGeom geom;
  const double *__restrict__ val;
  int n;
  __device__ double operator()(int ra, int la, int, int lb) const {
    const int s = slot_of(geom, la, lb);
    return s >= 0 ? val[size_t(s) * n + ra] : 0.0;
  }
};

struct CsrGather {
  CsrView<double> A;
  __device__ double operator()(int ra, int, int rb, int) const {
    int lo = A.ptr[ra], hi = A.ptr[ra + 1];
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (A.col[mid] < rb) lo = mid + 1;
      else hi = mid;
    }
    return (lo < A.ptr[ra + 1] && A.col[lo] == rb) ? A.val[lo] : 0.0;
  }
};

template <typename Gather>
__global__ __launch_bounds__(kFacThreads) void k_block_factor(
    int nblocks, const int32_t *__restrict__ bstart, const int32_t *__restrict__ bsize,
    const int32_t *__restrict__ blat, const int32_t *__restrict__ brow, Gather gather,
    double *__restrict__ inv_out, const int64_t *__restrict__ inv_off,
    uint8_t *__restrict__ keep_out, double *__restrict__ lam_out, int32_t *__restrict__ info_out, double ratio,
    int maxn) {
  const int j = blockIdx.x;
  if (j >= nblocks) return;
  extern __shared__ double smem[];
  const int nj = bsize[j];
  const int st = bstart[j];
  double *A = smem;                       // maxn * maxn
  double *V = A + size_t(maxn) * maxn;    // maxn * maxn
  double *cs = V + size_t(maxn) * maxn;   // maxn/2 + 1
  double *sn = cs + (maxn / 2 + 1);
  __shared__ int keep_idx[IMSMG_MAX_BLOCK];
  __shared__ int nk;
  __shared__ int rotated;
  __shared__ int removed_local;
  __shared__ double dmax_s;
  const int tid = threadIdx.x;

  if (tid == 0) nk = nj;
  for (int a = tid; a < nj; a += kFacThreads) {
    keep_idx[a] = a;
    keep_out[st + a] = 1;
  }
  __syncthreads();

  for (int round = 0; round <= nj; ++round) {
    const int m = nk;
    if (m == 0) break;
    // gather A_j for the kept indices
    for (int e = tid; e < m * m; e += kFacThreads) {
      const int a = e % m, b = e / m;
      const int ra = brow[st + keep_idx[a]], rb = brow[st + keep_idx[b]];
      const int la = blat[st + keep_idx[a]], lb = blat[st + keep_idx[b]];
      A[a * maxn + b] = gather(ra, la, rb, lb);
      V[a * maxn + b] = (a == b) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
      double dm = 0.0;
      for (int a = 0; a < m; ++a) dm = fmax(dm, A[a * maxn + a]);
      dmax_s = dm;
    }
    const int me = (m + 1) & ~1;  // even size with a dummy index when m is odd
    for (int sweep = 0; sweep < 40; ++sweep) {
      if (tid == 0) rotated = 0;
      __syncthreads();
      for (int step = 0; step < me - 1; ++step) {
        // pair t: (p, q) by the circle method, index me-1 fixed
        for (int t = tid; t < me / 2; t += kFacThreads) {
          int p, q;
          if (t == 0) {
            p = step % (me - 1);
            q = me - 1;
          } else {
            p = (step + t) % (me - 1);
            q = (step - t + (me - 1)) % (me - 1);
          }
          double c = 1.0, s = 0.0;
          if (p < m && q < m) {
            const double app = A[p * maxn + p], aqq = A[q * maxn + q], apq = A[p * maxn + q];
            if (fabs(apq) > 1e-18 * sqrt(fabs(app * aqq)) && apq != 0.0) {
              const double theta = (aqq - app) / (2.0 * apq);
              const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
              c = 1.0 / sqrt(tt * tt + 1.0);
              s = tt * c;
              rotated = 1;
            }
          }
          cs[t] = c;
          sn[t] = s;
        }
        __syncthreads();
        // rows p, q:  A <- J^T A
        for (int e = tid; e < (me / 2) * m; e += kFacThreads) {
          const int t = e / m, k = e % m;
          int p, q;
          if (t == 0) { p = step % (me - 1); q = me - 1; }
          else { p = (step + t) % (me - 1); q = (step - t + (me - 1)) % (me - 1); }
          if (p >= m || q >= m) continue;
          const double c = cs[t], s = sn[t];
          if (s == 0.0) continue;
          const double a1 = A[p * maxn + k], a2 = A[q * maxn + k];
          A[p * maxn + k] = c * a1 - s * a2;
          A[q * maxn + k] = s * a1 + c * a2;
        }
        __syncthreads();
        // columns p, q:  A <- A J,  V <- V J
        for (int e = tid; e < (me / 2) * m; e += kFacThreads) {
          const int t = e / m, k = e % m;
          int p, q;
          if (t == 0) { p = step % (me - 1); q = me - 1; }
          else { p = (step + t) % (me - 1); q = (step - t + (me - 1)) % (me - 1); }
          if (p >= m || q >= m) continue;
          const double c = cs[t], s = sn[t];
          if (s == 0.0) continue;
          const double a1 = A[k * maxn + p], a2 = A[k * maxn + q];
          A[k * maxn + p] = c * a1 - s * a2;
          A[k * maxn + q] = s * a1 + c * a2;
          const double v1 = V[k * maxn + p], v2 = V[k * maxn + q];
          V[k * maxn + p] = c * v1 - s * v2;
          V[k * maxn + q] = s * v1 + c * v2;
        }
        __syncthreads();
      }
      if (!rotated) break;
      __syncthreads();
    }
    // removal test on the smallest eigenvalue
    if (tid == 0) {
      int kmin = 0;
      double lmin = A[0], lmax = A[0];
      for (int a = 1; a < m; ++a) {
        const double l = A[a * maxn + a];
        if (l < lmin) { lmin = l; kmin = a; }
        if (l > lmax) lmax = l;
      }
      removed_local = -1;
      if (lmin < ratio * dmax_s) {
        int imax = 0;
        double vmax = -1.0;
        for (int a = 0; a < m; ++a) {
          const double v = fabs(V[a * maxn + kmin]);
          if (v > vmax) { vmax = v; imax = a; }
        }
        removed_local = imax;
      }
      // [input block lambda_min, input block max diag, final lambda_min, final lambda_max]
      if (round == 0) {
        lam_out[4 * j] = lmin;
        lam_out[4 * j + 1] = dmax_s;
      }
      lam_out[4 * j + 2] = lmin;
      lam_out[4 * j + 3] = lmax;
    }
    __syncthreads();
    if (removed_local < 0) break;
    if (tid == 0) {
      keep_out[st + keep_idx[removed_local]] = 0;
      for (int a = removed_local; a < m - 1; ++a) keep_idx[a] = keep_idx[a + 1];
      nk = m - 1;
    }
    __syncthreads();
  }
  const int m = nk;
  // inverse V diag(1/lambda) V^T, column-major, into inv_out
  double *out = inv_out + inv_off[j];
  for (int e = tid; e < m * m; e += kFacThreads) {
    const int a = e % m, b = e / m;  // out[a + m b]
    double acc = 0.0;
    for (int k = 0; k < m; ++k) acc += V[a * maxn + k] * V[b * maxn + k] / A[k * maxn + k];
    out[a + size_t(m) * b] = acc;
  }
  if (tid == 0) info_out[j] = m;
}

// launcher with the lattice geometry (used by the API)
int launch_block_factor_geom(hipStream_t s, int nblocks, int maxn, const int32_t *bstart, const int32_t *bsize,
                             const int32_t *blat, const int32_t *brow, int n, int dim, int nx, int ny, int reach,
                             const double *val, double *inv_out, const int64_t *inv_off, uint8_t *keep_out,
                             double *lam_out, int32_t *info_out, double ratio) {
  if (nblocks <= 0) return 0;
  if (maxn > IMSMG_MAX_BLOCK) return -1;
  const LatticeGather g{LatticeGeom{dim, nx, ny, reach, 2 * reach + 1}, val, n};
  const size_t shmem = (size_t(2) * maxn * maxn + 2 * (maxn / 2 + 1)) * sizeof(double);
  k_block_factor<<<nblocks, kFacThreads, shmem, s>>>(nblocks, bstart, bsize, blat, brow, g, inv_out, inv_off,
                                                     keep_out, lam_out, info_out, ratio, maxn);
  return 0;
}

int launch_block_factor_csr(hipStream_t s, int nblocks, int maxn, const int32_t *bstart, const int32_t *bsize,
                            const int32_t *brow, const CsrView<double> &A, double *inv_out, const int64_t *inv_off,
                            uint8_t *keep_out, double *lam_out, int32_t *info_out, double ratio) {
  if (nblocks <= 0) return 0;
  if (maxn > IMSMG_MAX_BLOCK) return -1;
  const size_t shmem = (size_t(2) * maxn * maxn + 2 * (maxn / 2 + 1)) * sizeof(double);
  k_block_factor<<<nblocks, kFacThreads, shmem, s>>>(nblocks, bstart, bsize, brow, brow, CsrGather{A}, inv_out,
                                                     inv_off, keep_out, lam_out, info_out, ratio, maxn);
  return 0;
}

// -------- coarsest level: dense matrix from ELL, Gauss-Jordan inversion
__global__ void k_dense_from_ell(int n, int K, Offsets off, const int32_t *__restrict__ row_lat,
                                 const int32_t *__restrict__ lat2c, const double *__restrict__ val,
                                 double *__restrict__ dense) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int L = row_lat[i];
  for (int s = 0; s < K; ++s) {
    const double v = val[size_t(s) * n + i];
    if (v == 0.0) continue;
    const int c = lat2c[L + off.off[s]];
    if (c >= 0) dense[size_t(i) * n + c] = v;
  }
}

void launch_dense_from_ell(hipStream_t s, int n, int K, const Offsets &off, const int32_t *row_lat,
                           const int32_t *lat2c, const double *val, double *dense) {
  if (n > 0) k_dense_from_ell<<<(n + 255) / 256, 256, 0, s>>>(n, K, off, row_lat, lat2c, val, dense);
}

__global__ void k_gj_copy(int n, int k, const double *__restrict__ A, double *__restrict__ colk,
                          double *__restrict__ rowk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  colk[i] = A[size_t(i) * n + k];
  rowk[i] = A[size_t(k) * n + i];
}

__global__ void k_gj_update(int n, int k, double *__restrict__ A, const double *__restrict__ colk,
                            const double *__restrict__ rowk, int32_t *__restrict__ bad_pivot) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= n) return;
  const double piv = rowk[k];
  // Gauss-Jordan pivots of an SPD matrix are the positive Schur-complement diagonals
  if (i == k && j == k && !(piv > 0.0 && piv < INFINITY)) *bad_pivot = 1;
  double v;
  if (i == k && j == k) v = 1.0 / piv;
  else if (i == k) v = rowk[j] / piv;
  else if (j == k) v = -colk[i] / piv;
  else v = A[size_t(i) * n + j] - colk[i] * rowk[j] / piv;
  A[size_t(i) * n + j] = v;
}

void launch_gauss_jordan_step(hipStream_t s, int n, int k, double *A, double *colk, double *rowk,
                              int32_t *bad_pivot) {
  k_gj_copy<<<(n + 255) / 256, 256, 0, s>>>(n, k, A, colk, rowk);
  dim3 g((n + 255) / 256, n);
  k_gj_update<<<g, 256, 0, s>>>(n, k, A, colk, rowk, bad_pivot);
}

// -------- N_K: number of blocks holding a function non-zero on element K
__global__ void k_count_nk(int nel, const int32_t *__restrict__ eptr, const int32_t *__restrict__ eidx,
                           const int32_t *__restrict__ fptr, const int32_t *__restrict__ fblk, int32_t *__restrict__ nk,
                           int32_t *__restrict__ overflow) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nel) return;
  constexpr int kCap = 128;
  int seen[kCap];
  int cnt = 0;
  for (int a = eptr[e]; a < eptr[e + 1]; ++a) {
    const int f = eidx[a];
    for (int t = fptr[f]; t < fptr[f + 1]; ++t) {
      const int b = fblk[t];
      bool dup = false;
      for (int u = 0; u < cnt; ++u)
        if (seen[u] == b) { dup = true; break; }
      if (dup) continue;
      if (cnt == kCap) { atomicOr(overflow, 1); nk[e] = cnt; return; }
      seen[cnt++] = b;
    }
  }
  nk[e] = cnt;
}

void launch_count_nk(hipStream_t s, int nel, const int32_t *eptr, const int32_t *eidx, const int32_t *fptr,
                     const int32_t *fblk, int32_t *nk, int32_t *overflow) {
  if (nel > 0) k_count_nk<<<(nel + 127) / 128, 128, 0, s>>>(nel, eptr, eidx, fptr, fblk, nk, overflow);
}

// inv_j *= w_j (the damping weight is folded into the stored inverse)
__global__ void k_scale_blocks(int nblocks, const int64_t *__restrict__ off, const int32_t *__restrict__ size,
                               const double *__restrict__ w, double *__restrict__ inv) {
  const int j = blockIdx.x;
  if (j >= nblocks) return;
  const int m = size[j];
  double *p = inv + off[j];
  const double wj = w[j];
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) p[e] *= wj;
}

void launch_scale_blocks(hipStream_t s, int nblocks, const int64_t *off, const int32_t *size, const double *w,
                         double *inv) {
  if (nblocks > 0) k_scale_blocks<<<nblocks, 64, 0, s>>>(nblocks, off, size, w, inv);
}

// c_i = w_j / A_ii for rows whose only block is their own singleton
__global__ void k_diag_coef(int n, int center, const int32_t *__restrict__ trivial_block,
                            const double *__restrict__ val, const double *__restrict__ bw, double *__restrict__ c) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = trivial_block[i];
  c[i] = j >= 0 ? bw[j] / val[size_t(center) * n + i] : 0.0;
}

void launch_diag_coef(hipStream_t s, int n, int K, int center_slot, const int32_t *trivial_block, const double *val,
                      const double *bw, double *c) {
  (void)K;
  if (n > 0) k_diag_coef<<<(n + 255) / 256, 256, 0, s>>>(n, center_slot, trivial_block, val, bw, c);
}

}  // namespace imsmg
