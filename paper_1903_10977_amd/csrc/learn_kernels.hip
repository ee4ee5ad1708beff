// Kernels of the per-block damping: the damping network (inference, loss
// gradient by backpropagation, Adam), block bilinear forms for the gradient of
// the two-grid objective, and a plain dot product for the stability check.
//
// The paper uses one damping factor per level (the discussion after
// eq:applyCS); per-block weights omega_j are an extension whose network is
//   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), o = w3 . h2 + b3,
// 16 -> 64 -> 64 -> 1, FP32, parameters flat: W1 (64 x 16 row-major), b1,
// W2 (64 x 64 row-major), b2, w3, b3 (5313 floats).
#include <mutex>

#include "imsmg_internal.h"

namespace imsmg {

namespace {
constexpr int kNF = kMlpInputs, kNH = kMlpHidden, kNP = kMlpParams;
constexpr int oW1 = 0, oB1 = oW1 + kNH * kNF, oW2 = oB1 + kNH, oB2 = oW2 + kNH * kNH, oW3 = oB2 + kNH,
              oB3 = oW3 + kNH;
static_assert(oB3 + 1 == kNP, "parameter layout");
constexpr int kMlpThreads = 128;
constexpr int kChunk = 256;  // samples per gradient partial

__device__ __forceinline__ void load_params(const float *__restrict__ params, float *P) {
  for (int k = threadIdx.x; k < kNP; k += blockDim.x) P[k] = params[k];
  __syncthreads();
}
}  // namespace

// o_i for every sample (X row-major, n x 16)
__global__ __launch_bounds__(kMlpThreads) void k_mlp_forward(int n, const float *__restrict__ params,
                                                             const float *__restrict__ X, float *__restrict__ out) {
  __shared__ float P[kNP];
  load_params(params, P);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float x[kNF], h1[kNH];
  for (int f = 0; f < kNF; ++f) x[f] = X[size_t(i) * kNF + f];
  for (int h = 0; h < kNH; ++h) {
    float a = P[oB1 + h];
    for (int f = 0; f < kNF; ++f) a += P[oW1 + h * kNF + f] * x[f];
    h1[h] = fmaxf(a, 0.0f);
  }
  float o = P[oB3];
  for (int k = 0; k < kNH; ++k) {
    float a = P[oB2 + k];
    for (int h = 0; h < kNH; ++h) a += P[oW2 + k * kNH + h] * h1[h];
    if (a > 0.0f) o += P[oW3 + k] * a;
  }
  out[i] = o;
}

// per sample: forward, error e = o - t, and the backpropagated signals of the
// mean squared error L = mean(e^2):  dL/do = 2 e / n,  da2 = dL/do w3 [a2 > 0],
// da1 = (W2^T da2) [a1 > 0].  Stored feature-major (index [unit * n + sample]).
__global__ __launch_bounds__(kMlpThreads) void k_mlp_backprop(int n, const float *__restrict__ params,
                                                              const float *__restrict__ X,
                                                              const float *__restrict__ t, float *__restrict__ H1,
                                                              float *__restrict__ H2, float *__restrict__ DA1,
                                                              float *__restrict__ DA2, float *__restrict__ DO,
                                                              float *__restrict__ E2) {
  __shared__ float P[kNP];
  load_params(params, P);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float x[kNF], h1[kNH], dh1[kNH];
  for (int f = 0; f < kNF; ++f) x[f] = X[size_t(i) * kNF + f];
  for (int h = 0; h < kNH; ++h) {
    float a = P[oB1 + h];
    for (int f = 0; f < kNF; ++f) a += P[oW1 + h * kNF + f] * x[f];
    h1[h] = fmaxf(a, 0.0f);
    H1[size_t(h) * n + i] = h1[h];
    dh1[h] = 0.0f;
  }
  float o = P[oB3];
  for (int k = 0; k < kNH; ++k) {
    float a = P[oB2 + k];
    for (int h = 0; h < kNH; ++h) a += P[oW2 + k * kNH + h] * h1[h];
    const float h2 = fmaxf(a, 0.0f);
    H2[size_t(k) * n + i] = h2;
    o += P[oW3 + k] * h2;
  }
  const float e = o - t[i];
  const float dout = 2.0f * e / float(n);
  DO[i] = dout;
  E2[i] = e * e;
  for (int k = 0; k < kNH; ++k) {
    const float h2 = H2[size_t(k) * n + i];
    const float d = h2 > 0.0f ? dout * P[oW3 + k] : 0.0f;
    DA2[size_t(k) * n + i] = d;
    if (d != 0.0f)
      for (int h = 0; h < kNH; ++h) dh1[h] += d * P[oW2 + k * kNH + h];
  }
  for (int h = 0; h < kNH; ++h) DA1[size_t(h) * n + i] = h1[h] > 0.0f ? dh1[h] : 0.0f;
}

// partial parameter gradients over one chunk of samples (fixed order), plus
// the chunk's sum of squared errors in slot kNP
__global__ __launch_bounds__(256) void k_mlp_grad_partial(int n, const float *__restrict__ X,
                                                          const float *__restrict__ H1, const float *__restrict__ H2,
                                                          const float *__restrict__ DA1,
                                                          const float *__restrict__ DA2,
                                                          const float *__restrict__ DO,
                                                          const float *__restrict__ E2, double *__restrict__ part) {
  const int c = blockIdx.x;
  const int s0 = c * kChunk, s1 = min(n, s0 + kChunk);
  for (int p = threadIdx.x; p <= kNP; p += blockDim.x) {
    double acc = 0.0;
    if (p < oB1) {
      const int h = p / kNF, f = p % kNF;
      for (int s = s0; s < s1; ++s) acc += double(DA1[size_t(h) * n + s]) * X[size_t(s) * kNF + f];
    } else if (p < oW2) {
      const int h = p - oB1;
      for (int s = s0; s < s1; ++s) acc += DA1[size_t(h) * n + s];
    } else if (p < oB2) {
      const int k = (p - oW2) / kNH, h = (p - oW2) % kNH;
      for (int s = s0; s < s1; ++s) acc += double(DA2[size_t(k) * n + s]) * H1[size_t(h) * n + s];
    } else if (p < oW3) {
      const int k = p - oB2;
      for (int s = s0; s < s1; ++s) acc += DA2[size_t(k) * n + s];
    } else if (p < oB3) {
      const int k = p - oW3;
      for (int s = s0; s < s1; ++s) acc += double(DO[s]) * H2[size_t(k) * n + s];
    } else if (p == oB3) {
      for (int s = s0; s < s1; ++s) acc += DO[s];
    } else {
      for (int s = s0; s < s1; ++s) acc += E2[s];
    }
    part[size_t(c) * (kNP + 1) + p] = acc;
  }
}

__global__ void k_mlp_grad_final(int n, int chunks, const double *__restrict__ part, float *__restrict__ grad,
                                 float *__restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kNP) return;
  double acc = 0.0;
  for (int c = 0; c < chunks; ++c) acc += part[size_t(c) * (kNP + 1) + p];
  if (p < kNP) grad[p] = float(acc);
  else *loss = float(acc / n);
}

__global__ void k_mlp_adam(float *__restrict__ theta, const float *__restrict__ g, float *__restrict__ m,
                           float *__restrict__ v, float lr, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNP) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mi = b1 * m[p] + (1.0f - b1) * g[p];
  const float vi = b2 * v[p] + (1.0f - b2) * g[p] * g[p];
  m[p] = mi;
  v[p] = vi;
  theta[p] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

size_t mlp_workspace_bytes(int n) {
  const int chunks = (n + kChunk - 1) / kChunk;
  return size_t(n) * (4 * kNH + 2) * sizeof(float) + size_t(std::max(chunks, 1)) * (kNP + 1) * sizeof(double) + 256;
}

void launch_mlp_forward(hipStream_t s, int n, const float *params, const float *X, float *out) {
  if (n > 0) k_mlp_forward<<<(n + kMlpThreads - 1) / kMlpThreads, kMlpThreads, 0, s>>>(n, params, X, out);
}

void launch_mlp_loss_grad(hipStream_t s, int n, const float *params, const float *X, const float *t, void *work,
                          float *loss, float *grad) {
  const int chunks = (n + kChunk - 1) / kChunk;
  double *part = reinterpret_cast<double *>(work);
  float *H1 = reinterpret_cast<float *>(part + size_t(std::max(chunks, 1)) * (kNP + 1));
  float *H2 = H1 + size_t(n) * kNH, *DA1 = H2 + size_t(n) * kNH, *DA2 = DA1 + size_t(n) * kNH;
  float *DO = DA2 + size_t(n) * kNH, *E2 = DO + n;
  k_mlp_backprop<<<(n + kMlpThreads - 1) / kMlpThreads, kMlpThreads, 0, s>>>(n, params, X, t, H1, H2, DA1, DA2, DO,
                                                                            E2);
  k_mlp_grad_partial<<<chunks, 256, 0, s>>>(n, X, H1, H2, DA1, DA2, DO, E2, part);
  k_mlp_grad_final<<<(kNP + 1 + 255) / 256, 256, 0, s>>>(n, chunks, part, grad, loss);
}

// Workspace of the allocation-free loss/gradient entry point: a file-scope
// device array sized for kNoAllocMaxSamples samples (every GPU the library
// runs on holds its own copy until the process ends).  Every word the three
// kernels read is written earlier in the same call (activations by
// k_mlp_backprop, partials by k_mlp_grad_partial), so nothing is cleared; two
// calls that overlap on one GPU share the array and race.
constexpr size_t kNoAllocScratchBytes =
    size_t(kNoAllocMaxSamples) * (4 * kNH + 2) * sizeof(float) +
    size_t((kNoAllocMaxSamples + kChunk - 1) / kChunk) * (kNP + 1) * sizeof(double) + 256;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

size_t mlp_noalloc_scratch_bytes() { return kNoAllocScratchBytes; }

// Device address of `scratch` on the device of stream s (the current device
// for the null stream), looked up once per device with that device current.
// In host code the array's name is only a host-side stand-in: kernels get
// this address, never the name.
int mlp_noalloc_scratch(hipStream_t s, void **out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void *ptrs[kMaxDevices] = {};
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return IMSMG_ERR_HIP;
  int dev = cur;
  if (s) {
    hipDevice_t d = 0;
    if (hipStreamGetDevice(s, &d) != hipSuccess) return IMSMG_ERR_HIP;
    dev = d;
  }
  if (dev < 0 || dev >= kMaxDevices) return IMSMG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(mu);
  if (!ptrs[dev]) {
    if (dev != cur && hipSetDevice(dev) != hipSuccess) return IMSMG_ERR_HIP;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (dev != cur) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) return IMSMG_ERR_HIP;
    ptrs[dev] = p;
  }
  *out = ptrs[dev];
  return IMSMG_OK;
}

void launch_mlp_adam(hipStream_t s, float *theta, const float *g, float *m, float *v, int step, float lr) {
  const float c1 = 1.0f - powf(0.9f, float(step)), c2 = 1.0f - powf(0.999f, float(step));
  k_mlp_adam<<<(kNP + 255) / 256, 256, 0, s>>>(theta, g, m, v, lr, c1, c2);
}

// out[j] += coef * u_j^T A_j^{-1} v_j for every final block j: members' lattice
// positions blat[bptr[j] .. bptr[j+1]); factorized or general blocks read the
// stored inverse (column-major, scaled by the weight wfold[j], which is
// divided out); singletons without a stored inverse use bdiag[j] = 1 / A_ii
__global__ void k_block_bilinear(int nb, const int32_t *__restrict__ bptr, const int32_t *__restrict__ blat,
                                 const int64_t *__restrict__ boff, const double *__restrict__ bdiag,
                                 const double *__restrict__ wfold, const double *__restrict__ inv,
                                 const double *__restrict__ u, const double *__restrict__ v, double coef,
                                 double *__restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nb) return;
  const int p0 = bptr[j], m = bptr[j + 1] - p0;
  double acc = 0.0;
  if (m == 0) {
    acc = 0.0;
  } else if (boff[j] < 0) {
    const int L = blat[p0];
    acc = u[L] * bdiag[j] * v[L];
  } else {
    const double *A = inv + boff[j];
    for (int b = 0; b < m; ++b) {
      double col = 0.0;
      for (int a = 0; a < m; ++a) col += u[blat[p0 + a]] * A[a + size_t(m) * b];
      acc += col * v[blat[p0 + b]];
    }
    acc /= wfold[j];
  }
  out[j] += coef * acc;
}

void launch_block_bilinear(hipStream_t s, int nb, const int32_t *bptr, const int32_t *blat, const int64_t *boff,
                           const double *bdiag, const double *wfold, const double *inv, const double *u,
                           const double *v, double coef, double *out) {
  if (nb > 0) k_block_bilinear<<<(nb + 255) / 256, 256, 0, s>>>(nb, bptr, blat, boff, bdiag, wfold, inv, u, v, coef, out);
}

// partial sums of a[L] b[L] over the active rows, one per workgroup
__global__ __launch_bounds__(256) void k_dot_partial(int n, const int32_t *__restrict__ row_lat,
                                                     const double *__restrict__ a, const double *__restrict__ b,
                                                     double *__restrict__ part) {
  __shared__ double sm[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const int L = row_lat[i];
    v = a[L] * b[L];
  }
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sm[threadIdx.x] += sm[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

int dot_blocks(int n) { return std::max(1, (n + 255) / 256); }

void launch_dot_partial(hipStream_t s, int n, const int32_t *row_lat, const double *a, const double *b,
                        double *part) {
  k_dot_partial<<<dot_blocks(n), 256, 0, s>>>(n, row_lat, a, b, part);
}

// y[L] = alpha x[L] for the active rows
__global__ void k_scale_copy(int n, const int32_t *__restrict__ row_lat, double alpha, const double *__restrict__ x,
                             double *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int L = row_lat[i];
  y[L] = alpha * x[L];
}

void launch_scale_copy(hipStream_t s, int n, const int32_t *row_lat, double alpha, const double *x, double *y) {
  if (n > 0) k_scale_copy<<<(n + 255) / 256, 256, 0, s>>>(n, row_lat, alpha, x, y);
}

// y[L] = x[L] - y[L]   (y := x - y on the active rows)
__global__ void k_sub_from(int n, const int32_t *__restrict__ row_lat, const double *__restrict__ x,
                           double *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int L = row_lat[i];
  y[L] = x[L] - y[L];
}

void launch_sub_from(hipStream_t s, int n, const int32_t *row_lat, const double *x, double *y) {
  if (n > 0) k_sub_from<<<(n + 255) / 256, 256, 0, s>>>(n, row_lat, x, y);
}

}  // namespace imsmg
