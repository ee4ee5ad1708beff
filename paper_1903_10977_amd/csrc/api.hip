// C-ABI of the solver library: context, setup (CSR -> lattice-ELL), block
// factorization bookkeeping, V-cycle (Algorithm alg:MGV) and CG driver.
//
// Host code here only converts layouts, sizes buffers and sequences kernel
// launches; every floating-point step of factorization, smoothing, transfer,
// coarse solve and CG runs in the HIP kernels of this directory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <stdexcept>
#include <thread>
#include <string>
#include <vector>

#include "imsmg.h"
#include "imsmg_internal.h"

using namespace imsmg;

namespace {

struct InvalidArg {
  int code;
  std::string msg;
};

[[noreturn]] void bad(const std::string &m, int code = IMSMG_ERR_INVALID_ARG) { throw InvalidArg{code, m}; }

template <typename T>
T *dalloc(std::vector<void *> &owned, size_t count) {
  if (count == 0) count = 1;
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, count * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw std::bad_alloc();
  }
  owned.push_back(p);
  return static_cast<T *>(p);
}

template <typename T>
void h2d(hipStream_t s, T *dst, const T *src, size_t count) {
  if (count) HIP_CHECK_RET(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, s));
}
template <typename T>
void d2h(hipStream_t s, T *dst, const T *src, size_t count) {
  if (count) HIP_CHECK_RET(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDeviceToHost, s));
}

struct Level {
  int n = 0;
  // vector levels (linear elasticity): ncomp components per lattice function,
  // rows c ns + i (component-major), vectors as ncomp padded scalar arrays
  // cstride apart; h_lat / srow_lat: the lattice point of every row / of
  // every scalar row; vops: the component blocks for the vector kernels
  int ncomp = 1, ns = 0;
  int64_t cstride = 0;
  std::vector<int32_t> h_lat;
  int32_t *srow_lat = nullptr;
  VecOps<double> vops64{};
  VecOps<float> vops32{};
  std::vector<std::vector<uint32_t>> h_bmeta;  // per component block: stored index or kMetaIndex per scalar row
  double *dense0 = nullptr;  // coarsest vector level: the dense operator (setup)
  // general sparse level (no function lattice: locally refined bases): the
  // operator as CSR (host copy for the coarsest dense matrix), rows at the
  // identity positions of the padded vectors, csr_lanes lanes per row
  bool csr = false;
  int csr_lanes = 8;
  CsrView<double> a64{};
  CsrView<float> a32{};
  std::vector<int32_t> h_aptr, h_acol;
  std::vector<double> h_aval;
  int K = 0, dim = 2, reach = 0, center = 0;
  int shape[3] = {1, 1, 1};
  Offsets off{};
  int64_t lattice = 0, guard = 0;
  std::vector<int32_t> h_row_lat;
  int32_t *row_lat = nullptr;
  double *val = nullptr;            // full lattice-ELL (setup, factorization, coarsest matrix)
  // compressed operator used by the solve kernels
  std::vector<uint32_t> h_meta;
  uint32_t *meta = nullptr;
  OpView<double> op64{};
  OpView<float> op32{};
  int n_uniform = 0;
  // padded vectors (pointers already shifted past the guard band); x and x2
  // alternate between smoothing steps, xs is where a V-cycle on this level starts
  double *r = nullptr, *x = nullptr, *x2 = nullptr, *rh = nullptr, *xs = nullptr;
  // restriction R_l (rows: coarse level) and R_l^T (rows: this level)
  int rw = 0, tw = 0;
  int32_t *rcol = nullptr, *tcol = nullptr;
  double *rval = nullptr, *tval = nullptr;
  // index-free tensor form of R_l (bands of the 1D two-scale matrix)
  bool tensor = false;
  int rbW = 0, pbW = 0;
  int32_t *rb_start = nullptr, *rb_len = nullptr, *pb_start = nullptr, *pb_len = nullptr;
  double *rb_coef = nullptr, *pb_coef = nullptr;
  // prolongation fused into the first post-smoothing step (tiled stencil,
  // tensor transfer, every tile's coarse window within the fixed bound)
  bool pro_ok = false;
  int32_t *pro_org = nullptr;  // coarse window origin per tile along x, y
  double *pro_coef = nullptr;  // R^T band coefficients, stride kBandMax
  // input blocks
  std::vector<int32_t> in_ptr, in_idx;
  std::vector<double> omega;  // optional per-block weights
  // factorized smoother
  std::vector<int32_t> f_ptr, f_idx;  // post-removal blocks (incl. added singletons)
  double *c = nullptr;               // trivial rows: omega_j / A_ii, else 0
  int ng = 0;                         // rows in general blocks
  int gen_lanes = 4;                  // lanes per row of the general-row product (tuned: 2, 4, 8)
  // multi-column smoother as patch GEMMs (option block_gemm; every general
  // block of this level has <= 16 functions): per block the members' lattice
  // positions (16, -1 padded), W = omega A^-1 padded to 16 x 16 (FP64 and
  // BF16), the products Y, and per general row its (block, member) rows of Y
  bool mb_on = false;
  int32_t *mb_lat = nullptr, *mb_yp = nullptr, *mb_ypos = nullptr;
  int32_t *mb_lp = nullptr;  // 1: well conditioned (cond(A_j) <= kBf16Kappa), BF16 allowed
  int mb_nlp = 0;
  double *mb_W = nullptr, *mb_Y = nullptr;
  uint16_t *mb_Wb = nullptr;
  bool small = false;                 // latency-bound level (no convergence-flag load)
  int32_t *grow_lat = nullptr, *sptr = nullptr, *scol = nullptr;
  double *sval = nullptr;             // S_G = sum_j omega_j P_j A_j^{-1} P_j^T on the general rows (CSR)
  double gamma = 0.0;
  // elements (host): incidence, lattice index (x fastest over el_shape) and
  // volume fraction |K cap Omega| / |K| of every active element
  std::vector<int32_t> e_ptr, e_idx, el_lat;
  int el_shape[3] = {0, 0, 0};
  std::vector<double> el_eta;
  // factorization bookkeeping kept for the per-block damping
  std::vector<int32_t> f_orig;   // input block of every final block (-1: added singleton)
  std::vector<double> f_lam;     // per final block: input lambda_min, input max diag, final lambda_min, lambda_max
  std::vector<int32_t> nk;       // N_K per active element (final blocks)
  std::vector<double> f_w;       // damping weight of every final block
  int learned_status = 0;        // 0: gamma / given weights, 1: learned weights accepted, -1: rejected
  double lambda_max = 0.0;       // estimate of lambda_max(S A) from the stability check (0: not run)
  // weight-dependent smoother data (device, factorization lifetime)
  double *inv = nullptr;         // block inverses, general blocks scaled by their folded weight
  int nbg = 0;
  std::vector<int32_t> g_blocks; // final block of every general block
  std::vector<double> g_wcur;    // weight folded into each general block's inverse
  int64_t *g_off = nullptr;
  int32_t *g_sz = nullptr;
  int32_t *asm_gp = nullptr, *asm_en = nullptr, *asm_epos = nullptr;
  int64_t *asm_eoff = nullptr, *asm_epos0 = nullptr;
  size_t sg_nnz = 0;
  int32_t *tb = nullptr;         // trivial block of every row (-1: none)
  double *bw = nullptr;          // weight per final block (device)
  // final blocks for bilinear forms: members' lattice positions, inverse offset
  // (-1: singleton without a stored inverse, read 1 / A_ii), folded weight
  int32_t *b_ptr = nullptr, *b_lat = nullptr;
  int64_t *b_off = nullptr;
  double *b_diag = nullptr, *b_wfold = nullptr;
  // coarsest level
  double *Ainv = nullptr;
  // colours of the final blocks (multiplicative smoother; every smoothed level)
  std::vector<int32_t> in_colour;  // given colour of every input block (empty: none given)
  std::vector<int32_t> f_colour;   // colour of every final block
  int ncolours = 0;
  // multiplicative smoother on this level: per colour c the rows its blocks
  // touch, ms_rows[ms_cptr[c] .. ms_cptr[c+1]) with ms_cf (1 / A_ii for
  // one-function blocks, 0 for members of larger blocks), and the larger
  // blocks' inverses as CSR on their members
  bool ms = false;
  std::vector<int32_t> ms_cptr;
  int32_t *ms_rows = nullptr;
  int32_t *ms_lat = nullptr;  // lattice position of every list entry (scalar lattice levels)
  double *ms_cf = nullptr;
  // colour-ordered copy of the stored rows' values (a row as often as colours
  // touch it): ms_vidx per list entry (-1: reference stencil)
  int32_t *ms_vidx = nullptr;
  double *ms_val64 = nullptr;
  float *ms_val32 = nullptr;
  int ms_stream64 = 0, ms_stream32 = 0;  // copies larger than the last-level cache: non-temporal loads
  struct MsGeneral {
    int ng = 0;
    int32_t *grow_lat = nullptr, *sptr = nullptr, *scol = nullptr;
    double *sval = nullptr;
  };
  std::vector<MsGeneral> ms_gen;
  // W-cycle work vectors (cycle >= 2): saved correction and residual
  double *w_x = nullptr, *w_r = nullptr;
  // full multigrid: the level's right-hand side and solution (first use)
  double *fmg_b = nullptr, *fmg_x = nullptr;
};

}  // namespace

struct imsmg_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  // batch context (imsmg_setup_batched): one child context, with its own
  // stream, per problem
  std::vector<imsmg_ctx *> batch;
  std::vector<void *> owned;      // setup-lifetime allocations
  std::vector<void *> factor_owned;
  std::vector<Level> lv;
  imsmg_options opt{};
  bool ready = false, factored = false;
  int32_t *zero_flag = nullptr;   // always 0: "not done" for stand-alone calls
  float *mlp = nullptr;           // damping network parameters (device, kMlpParams), or null
  CGState *st = nullptr;
  double *part = nullptr;
  double *p = nullptr, *q = nullptr, *xs = nullptr, *bs = nullptr;  // CG vectors (padded)
  double *c_in = nullptr, *c_out = nullptr;                          // compact staging
  hipGraphExec_t graph = nullptr;
  int graph_iters = 0;
  hipGraphExec_t vgraph = nullptr;  // one V-cycle from the staged c_in to c_out (imsmg_vcycle)
  // multi-right-hand-side buffers (R interleaved columns), allocated on first use
  struct Multi {
    int R = 0;
    std::vector<double *> r, x, x2, rh, xs;  // per level, padded
    double *p = nullptr, *q = nullptr, *xsol = nullptr, *bs = nullptr, *part = nullptr;
    MState *st = nullptr;
    hipGraphExec_t graph = nullptr;
    std::vector<void *> owned;
  } mb;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  double t_kernel_ms = 0.0;
  int64_t t_kernel_n = 0;
  double setup_ms = 0.0, factor_ms = 0.0;  // wall time of the last setup / factorization
  int judge_it[2] = {0, 0};                 // probe iterations with gamma / with the network (use_learned 1)
};

namespace {

void free_list(std::vector<void *> &v) {
  for (void *p : v) (void)hipFree(p);
  v.clear();
}

int fail(imsmg_ctx *c, int code, const std::string &m) {
  if (c) c->err = m;
  return code;
}

template <typename F>
int guarded(imsmg_ctx *c, F &&f) {
  if (!c) return IMSMG_ERR_INVALID_ARG;
  try {
    HIP_CHECK_RET(hipSetDevice(c->device));
    int rc = f();
    if (rc == IMSMG_OK) c->err.clear();
    return rc;
  } catch (const InvalidArg &e) {
    return fail(c, e.code, e.msg);
  } catch (const HipFailure &e) {
    return fail(c, IMSMG_ERR_HIP, e.msg);
  } catch (const std::bad_alloc &) {
    return fail(c, IMSMG_ERR_OOM, "out of device or host memory");
  } catch (const std::exception &e) {
    return fail(c, IMSMG_ERR_INVALID_ARG, e.what());
  }
}

int64_t lat_linear(const int *m, const int *shape, int dim) {
  int64_t L = 0;
  for (int a = dim - 1; a >= 0; --a) L = L * shape[a] + m[a];
  return L;
}

void lat_multi(int64_t L, const int *shape, int dim, int *m) {
  for (int a = 0; a < dim; ++a) {
    m[a] = int(L % shape[a]);
    L /= shape[a];
  }
}

// ------------------------------------------------------------------ setup
// colours of the multiplicative smoother: at most this many per level
constexpr int kMaxColours = 128;

// Level l (1 .. nlevels-1) uses the multiplicative smoother?
bool level_ms(const imsmg_options &o, int l, int nlevels) {
  const int kind = (l == nlevels - 1 || o.coarse_smoother < 0) ? o.smoother : o.coarse_smoother;
  return l >= 1 && kind == IMSMG_MULTIPLICATIVE;
}
bool uses_ms(const imsmg_options &o, int nlevels) {
  for (int l = 1; l < nlevels; ++l)
    if (level_ms(o, l, nlevels)) return true;
  return false;
}

// Compressed lattice-ELL form of one operator on the level's lattice (rows:
// lat[i], values ell[s * n + i] in slot order): the uniform interior stencil
// is the most frequent row among the candidate rows (rows hashed after
// rounding to 12 significant digits), rows within 1e-14 of it read it from
// the reference, the others keep their values in 16-byte slot groups,
// numbered tile by tile (32 x 8 points in 2D, 16 x 4 x 4 in 3D; lattice order
// inside a tile), so that the stored rows of a tile are one consecutive range.
// Candidates: the rows whose K values are all non-zero (full == nullptr), or
// the rows marked in *full.
struct Compressed {
  OpView<double> op64{};
  OpView<float> op32{};
  std::vector<uint32_t> h_meta;
  uint32_t *meta = nullptr;
  int n_uniform = 0;
};

void compress_operator(imsmg_ctx *c, const Level &L, int n, const std::vector<int32_t> &lat,
                       const std::vector<double> &ell, const std::vector<uint8_t> *full, Compressed &out) {
  hipStream_t s = c->stream;
  std::vector<double> ref(L.K, 0.0);
  bool have_ref = false;
  if (c->opt.compress) {
    std::vector<std::pair<uint64_t, int>> keys;
    keys.reserve(n);
    for (int i = 0; i < n; ++i) {
      bool cand = full ? (*full)[i] != 0 : true;
      uint64_t h = 1469598103934665603ull;
      for (int sl = 0; sl < L.K && cand; ++sl) {
        const double v = ell[size_t(sl) * n + i];
        if (!full && v == 0.0) cand = false;
        const double q = std::nearbyint(v * 1e12);
        uint64_t u;
        std::memcpy(&u, &q, 8);
        h = (h ^ u) * 1099511628211ull;
      }
      if (cand) keys.push_back({h, i});
    }
    std::sort(keys.begin(), keys.end());
    int best = -1, bestc = 0;
    for (size_t a = 0; a < keys.size();) {
      size_t b = a;
      while (b < keys.size() && keys[b].first == keys[a].first) ++b;
      if (int(b - a) > bestc) {
        bestc = int(b - a);
        best = keys[a].second;
      }
      a = b;
    }
    if (best >= 0 && bestc >= 16) {
      for (int sl = 0; sl < L.K; ++sl) ref[sl] = ell[size_t(sl) * n + best];
      have_ref = true;
    }
  }
  double refmax = 0.0;
  for (double v : ref) refmax = std::max(refmax, std::fabs(v));
  out.h_meta.assign(n, 0);
  out.n_uniform = 0;
  std::vector<int32_t> comp;
  for (int i = 0; i < n; ++i) {
    bool uni = have_ref;
    for (int sl = 0; sl < L.K && uni; ++sl) uni = std::fabs(ell[size_t(sl) * n + i] - ref[sl]) <= 1e-14 * refmax;
    if (uni) {
      out.h_meta[i] = kMetaIndex;
      ++out.n_uniform;
    } else {
      out.h_meta[i] = uint32_t(comp.size());
      comp.push_back(i);
    }
  }
  const int nv = int(comp.size());
  OpView<double> &o64 = out.op64;
  OpView<float> &o32 = out.op32;
  const bool tiled = (L.dim == 2 && L.reach <= 3) || (L.dim == 3 && L.reach <= 2);
  std::vector<int32_t> ord(comp);  // value column g -> row
  {
    const int TX = L.dim == 2 ? kTile2X : kTile3X, TY = L.dim == 2 ? kTile2Y : kTile3Y;
    const int TZ = L.dim == 2 ? 1 : kTile3Z;
    const int sx = L.shape[0], sy = L.shape[1], sz = L.shape[2];
    const int ntx = (sx + TX - 1) / TX, nty = (sy + TY - 1) / TY, ntz = (sz + TZ - 1) / TZ;
    const int64_t ntiles = tiled ? int64_t(ntx) * nty * ntz : 0;
    if (ntiles > (int64_t(1) << 30)) bad("too many lattice tiles");
    auto tile_of = [&](int64_t Lp) {
      const int x = int(Lp % sx), y = int((Lp / sx) % sy), z = int(Lp / (int64_t(sx) * sy));
      return (x / TX) + int64_t(ntx) * ((y / TY) + int64_t(nty) * (z / TZ));
    };
    auto local_of = [&](int64_t Lp) {  // the box-local point = the thread owning it
      const int x = int(Lp % sx), y = int((Lp / sx) % sy), z = int(Lp / (int64_t(sx) * sy));
      return int32_t(((z % TZ) * TY + (y % TY)) * TX + (x % TX));
    };
    std::vector<int32_t> tg0(size_t(ntiles) + 1, 0), sloc;
    if (tiled) {
      std::vector<int32_t> cnt(size_t(ntiles) + 1, 0);
      for (int32_t i : comp) ++cnt[size_t(tile_of(lat[i])) + 1];
      for (int64_t b = 0; b < ntiles; ++b) cnt[size_t(b) + 1] += cnt[size_t(b)];
      tg0.assign(cnt.begin(), cnt.end());
      // rows in lattice order: a stable placement keeps lattice order per tile
      for (int32_t i : comp) ord[size_t(cnt[size_t(tile_of(lat[i]))]++)] = i;
      sloc.resize(ord.size());
      for (size_t g = 0; g < ord.size(); ++g) sloc[g] = local_of(lat[ord[g]]);
    }
    for (int g = 0; g < nv; ++g) out.h_meta[ord[g]] = uint32_t(g);
    int32_t *d_sloc = dalloc<int32_t>(c->owned, std::max<size_t>(sloc.size(), 1));
    if (!sloc.empty()) h2d(s, d_sloc, sloc.data(), sloc.size());
    int32_t *d_tg0 = dalloc<int32_t>(c->owned, tg0.size());
    h2d(s, d_tg0, tg0.data(), tg0.size());
    std::vector<int32_t> l2r(tiled ? size_t(L.lattice) : 1, -1);
    if (tiled)
      for (int i = 0; i < n; ++i) l2r[size_t(lat[i])] = i;
    int32_t *d_l2r = dalloc<int32_t>(c->owned, l2r.size());
    h2d(s, d_l2r, l2r.data(), l2r.size());
    o64.sloc = o32.sloc = d_sloc;
    o64.tile_g0 = o32.tile_g0 = d_tg0;
    o64.lat2row = o32.lat2row = d_l2r;
    o64.sx = o32.sx = sx;
    o64.sy = o32.sy = sy;
    o64.sz = o32.sz = sz;
    o64.ntx = o32.ntx = ntx;
    o64.nty = o32.nty = nty;
    o64.ntiles = o32.ntiles = int(ntiles);
    HIP_CHECK_RET(hipStreamSynchronize(s));
  }
  // stored rows' values in 16-byte slot groups (SlotGroup): FP64 pairs, FP32 quadruples
  std::vector<double> cv(std::max<size_t>(stored_size(L.K, size_t(nv), 2), 2), 0.0);
  for (int g = 0; g < nv; ++g)
    for (int sl = 0; sl < L.K; ++sl) cv[stored_at<double>(size_t(nv), size_t(g), sl)] = ell[size_t(sl) * n + ord[g]];
  out.meta = dalloc<uint32_t>(c->owned, n);
  h2d(s, out.meta, out.h_meta.data(), n);
  double *cv64 = dalloc<double>(c->owned, cv.size());
  h2d(s, cv64, cv.data(), cv.size());
  o64.off = L.off;
  o64.val = cv64;
  o64.nv = nv;
  o32.off = L.off;
  o32.nv = nv;
  o64.stream = o32.stream = size_t(nv) * L.K > kStreamValues;
  {
    std::vector<float> ref32(ref.begin(), ref.end());
    std::vector<double> ref32d(ref32.begin(), ref32.end());
    double *r64 = dalloc<double>(c->owned, L.K);
    float *r32 = dalloc<float>(c->owned, L.K);
    double *r32d = dalloc<double>(c->owned, L.K);
    h2d(s, r64, ref.data(), L.K);
    h2d(s, r32, ref32.data(), L.K);
    h2d(s, r32d, ref32d.data(), L.K);
    o64.ref = r64;
    o64.refd = r64;
    o32.ref = r32;
    o32.refd = r32d;
    HIP_CHECK_RET(hipStreamSynchronize(s));
  }
  if (c->opt.precision == IMSMG_MIXED) {
    std::vector<float> c32(std::max<size_t>(stored_size(L.K, size_t(nv), 4), 4), 0.0f);
    for (int g = 0; g < nv; ++g)
      for (int sl = 0; sl < L.K; ++sl)
        c32[stored_at<float>(size_t(nv), size_t(g), sl)] = float(cv[stored_at<double>(size_t(nv), size_t(g), sl)]);
    float *cv32 = dalloc<float>(c->owned, c32.size());
    h2d(s, cv32, c32.data(), c32.size());
    o32.val = cv32;
    HIP_CHECK_RET(hipStreamSynchronize(s));
  }
}

// Slot of the lattice offset from row point li to column point lj, or bad().
int stencil_slot(const Level &L, int64_t li, int64_t lj) {
  const int W = 2 * L.reach + 1;
  int mi[3] = {0, 0, 0}, mj[3] = {0, 0, 0};
  lat_multi(li, L.shape, L.dim, mi);
  lat_multi(lj, L.shape, L.dim, mj);
  int sl = 0;
  for (int a = L.dim - 1; a >= 0; --a) {
    const int d = mj[a] - mi[a];
    if (d < -L.reach || d > L.reach) bad("CSR entry outside the lattice stencil");
    sl = sl * W + (d + L.reach);
  }
  return sl;
}

void alloc_level_vectors(imsmg_ctx *c, Level &L);

// General sparse level: the operator stays CSR (any pattern); vectors are
// indexed by row inside the guard band.
void setup_csr_level(imsmg_ctx *c, Level &L, const imsmg_csr &A) {
  hipStream_t s = c->stream;
  if (c->opt.ncomp != 1) bad("general sparse levels (no lattice) take scalar problems (ncomp 1)");
  if (A.nrows <= 0 || A.nrows != A.ncols) bad("A must be square and non-empty");
  if (!A.rowptr || !A.col || !A.val) bad("null CSR array");
  const int n = A.nrows;
  if (A.rowptr[0] != 0 || A.rowptr[n] != A.nnz) bad("CSR rowptr inconsistent with nnz");
  if (A.nnz > (int64_t(1) << 31) - 1) bad("operator too large for 32-bit CSR offsets");
  L.csr = true;
  L.n = L.ns = n;
  L.ncomp = 1;
  L.dim = 0;
  L.reach = 0;
  L.K = 1;       // L.val holds the diagonal as a one-slot ELL (diagonal readers)
  L.center = 0;
  L.shape[0] = n;
  L.shape[1] = L.shape[2] = 1;
  L.lattice = n;
  L.guard = 64;
  L.cstride = L.lattice + 2 * L.guard;
  L.h_lat.resize(n);
  L.h_row_lat.resize(n);
  std::iota(L.h_lat.begin(), L.h_lat.end(), 0);
  std::iota(L.h_row_lat.begin(), L.h_row_lat.end(), 0);
  L.h_aptr.assign(A.rowptr, A.rowptr + n + 1);
  L.h_acol.assign(A.col, A.col + A.nnz);
  L.h_aval.assign(A.val, A.val + A.nnz);
  std::vector<double> diag(n, 0.0);
  for (int i = 0; i < n; ++i) {
    if (A.rowptr[i + 1] < A.rowptr[i]) bad("CSR rowptr must be non-decreasing");
    for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
      if (A.col[k] < 0 || A.col[k] >= n) bad("CSR column out of range");
      if (k > A.rowptr[i] && A.col[k] <= A.col[k - 1]) bad("CSR columns must be sorted and unique");
      if (A.col[k] == i) diag[i] = A.val[k];
    }
    if (!(diag[i] > 0.0) || !std::isfinite(diag[i]))
      bad("operator has a non-positive diagonal entry (not SPD)", IMSMG_ERR_NOT_SPD);
  }
  int32_t *ptr = dalloc<int32_t>(c->owned, n + 1);
  int32_t *col = dalloc<int32_t>(c->owned, A.nnz);
  double *v64 = dalloc<double>(c->owned, A.nnz);
  float *v32 = dalloc<float>(c->owned, A.nnz);
  std::vector<float> f32(A.val, A.val + A.nnz);
  h2d(s, ptr, L.h_aptr.data(), n + 1);
  h2d(s, col, L.h_acol.data(), A.nnz);
  h2d(s, v64, A.val, A.nnz);
  h2d(s, v32, f32.data(), A.nnz);
  L.a64 = CsrView<double>{ptr, col, v64};
  L.a32 = CsrView<float>{ptr, col, v32};
  const double avg = double(A.nnz) / n;
  L.csr_lanes = avg <= 12.0 ? 4 : (avg <= 40.0 ? 8 : 16);
  L.val = dalloc<double>(c->owned, n);
  h2d(s, L.val, diag.data(), n);
  L.row_lat = dalloc<int32_t>(c->owned, n);
  h2d(s, L.row_lat, L.h_row_lat.data(), n);
  L.srow_lat = L.row_lat;
  L.h_meta.assign(n, 0u);
  L.meta = dalloc<uint32_t>(c->owned, n);
  h2d(s, L.meta, L.h_meta.data(), n);
  L.n_uniform = 0;
  HIP_CHECK_RET(hipStreamSynchronize(s));
  alloc_level_vectors(c, L);
}

void setup_level(imsmg_ctx *c, Level &L, const imsmg_csr &A, const imsmg_lattice &lat) {
  hipStream_t s = c->stream;
  if (!lat.dof_to_lattice) {
    setup_csr_level(c, L, A);
    return;
  }
  if (lat.dim < 2 || lat.dim > 3) bad("lattice dim must be 2 or 3");
  if (lat.reach < 1 || (lat.dim == 3 && lat.reach > 2) || lat.reach > 5) bad("lattice reach must be 1..5 (2D) or 1..2 (3D)");
  if (A.nrows <= 0 || A.nrows != A.ncols) bad("A must be square and non-empty");
  if (!A.rowptr || !A.col || !A.val || !lat.dof_to_lattice) bad("null CSR or lattice array");
  const int nc = c->opt.ncomp;
  if (A.nrows % nc) bad("the operator's size must be ncomp times the number of lattice functions");
  L.dim = lat.dim;
  L.reach = lat.reach;
  int64_t latsz = 1;
  for (int a = 0; a < 3; ++a) {
    L.shape[a] = a < lat.dim ? lat.shape[a] : 1;
    if (L.shape[a] < 1) bad("lattice shape must be positive");
    latsz *= L.shape[a];
  }
  if (latsz > (int64_t(1) << 30)) bad("lattice too large");
  L.lattice = latsz;
  L.n = A.nrows;
  L.ncomp = nc;
  L.ns = A.nrows / nc;
  const int W = 2 * L.reach + 1;
  L.K = L.dim == 2 ? W * W : W * W * W;
  if (L.K > IMSMG_MAX_SLOTS) bad("stencil too large");
  // slot offsets (x fastest)
  int64_t maxoff = 0;
  for (int sl = 0; sl < L.K; ++sl) {
    int o[3] = {0, 0, 0}, r = sl;
    for (int a = 0; a < L.dim; ++a) {
      o[a] = r % W - L.reach;
      r /= W;
    }
    int64_t lin = o[0] + int64_t(L.shape[0]) * (o[1] + int64_t(L.shape[1]) * o[2]);
    L.off.off[sl] = int32_t(lin);
    maxoff = std::max<int64_t>(maxoff, lin < 0 ? -lin : lin);
    if (lin == 0) L.center = sl;
  }
  L.guard = maxoff + 64;
  L.cstride = L.lattice + 2 * L.guard;
  if (nc * L.cstride > (int64_t(1) << 31) - 1) bad("lattice too large");
  const int ns = L.ns;
  for (int i = 0; i < ns; ++i) {
    if (lat.dof_to_lattice[i] < 0 || lat.dof_to_lattice[i] >= latsz) bad("dof_to_lattice out of range");
    if (i && lat.dof_to_lattice[i] <= lat.dof_to_lattice[i - 1]) bad("dof_to_lattice must be strictly increasing");
  }
  // rows: lattice point and memory position (component c at c * cstride)
  L.h_lat.resize(L.n);
  L.h_row_lat.resize(L.n);
  for (int cc = 0; cc < nc; ++cc)
    for (int i = 0; i < ns; ++i) {
      L.h_lat[size_t(cc) * ns + i] = lat.dof_to_lattice[i];
      L.h_row_lat[size_t(cc) * ns + i] = int32_t(cc * L.cstride + lat.dof_to_lattice[i]);
    }
  if (A.rowptr[0] != 0 || A.rowptr[L.n] != A.nnz) bad("CSR rowptr inconsistent with nnz");
  // CSR -> slot-major lattice-ELL per component block (b = ci * nc + cj)
  const int nb = nc * nc;
  std::vector<std::vector<double>> ell(nb, std::vector<double>(size_t(L.K) * ns, 0.0));
  std::vector<std::vector<uint8_t>> full(nc > 1 ? nb : 0, std::vector<uint8_t>(ns, 0));
  for (int r = 0; r < L.n; ++r) {
    const int ci = r / ns, i = r % ns;
    int cnt[kMaxComp] = {0, 0, 0};
    for (int64_t k = A.rowptr[r]; k < A.rowptr[r + 1]; ++k) {
      const int j = A.col[k];
      if (j < 0 || j >= L.n) bad("CSR column out of range");
      const int cj = j / ns;
      const int sl = stencil_slot(L, L.h_lat[r], L.h_lat[j]);
      ell[size_t(ci) * nc + cj][size_t(sl) * ns + i] = A.val[k];
      ++cnt[cj];
    }
    if (nc > 1)
      for (int cj = 0; cj < nc; ++cj) full[size_t(ci) * nc + cj][i] = cnt[cj] == L.K;
  }
  // an SPD operator has a positive, finite diagonal: reject the others before
  // anything is launched on them
  for (int cc = 0; cc < nc; ++cc)
    for (int i = 0; i < ns; ++i) {
      const double d = ell[size_t(cc) * nc + cc][size_t(L.center) * ns + i];
      if (!(d > 0.0) || !std::isfinite(d))
        bad("operator has a non-positive diagonal entry (not SPD)", IMSMG_ERR_NOT_SPD);
    }
  L.row_lat = dalloc<int32_t>(c->owned, L.n);
  h2d(s, L.row_lat, L.h_row_lat.data(), L.n);
  if (nc == 1) {
    L.val = dalloc<double>(c->owned, ell[0].size());
    h2d(s, L.val, ell[0].data(), ell[0].size());
    L.srow_lat = L.row_lat;
    Compressed cp;
    compress_operator(c, L, L.n, L.h_row_lat, ell[0], nullptr, cp);
    L.op64 = cp.op64;
    L.op32 = cp.op32;
    L.h_meta = std::move(cp.h_meta);
    L.meta = cp.meta;
    L.n_uniform = cp.n_uniform;
  } else {
    // the diagonal blocks as one lattice-ELL over all rows (row c ns + i:
    // block (c, c)'s row i): the per-component Schwarz blocks gather from it
    std::vector<double> dv(size_t(L.K) * L.n, 0.0);
    for (int cc = 0; cc < nc; ++cc)
      for (int sl = 0; sl < L.K; ++sl)
        std::copy(ell[size_t(cc) * nc + cc].begin() + size_t(sl) * ns,
                  ell[size_t(cc) * nc + cc].begin() + size_t(sl + 1) * ns, dv.begin() + size_t(sl) * L.n + size_t(cc) * ns);
    L.val = dalloc<double>(c->owned, dv.size());
    h2d(s, L.val, dv.data(), dv.size());
    L.srow_lat = dalloc<int32_t>(c->owned, ns);
    h2d(s, L.srow_lat, lat.dof_to_lattice, ns);
    std::vector<int32_t> slat(lat.dof_to_lattice, lat.dof_to_lattice + ns);
    L.vops64 = VecOps<double>{};
    L.vops32 = VecOps<float>{};
    L.n_uniform = 0;
    L.h_bmeta.assign(nb, {});
    for (int b = 0; b < nb; ++b) {
      Compressed cp;
      compress_operator(c, L, ns, slat, ell[b], &full[b], cp);
      if (b == 0) {
        L.op64 = cp.op64;
        L.op32 = cp.op32;
      }
      if (b % (nc + 1) == 0) L.n_uniform += cp.n_uniform;
      L.vops64.refd[b] = cp.op64.refd;
      L.vops64.val[b] = cp.op64.val;
      L.vops32.refd[b] = cp.op32.refd;
      L.vops32.val[b] = cp.op32.val;
      for (auto *v : {&L.vops64.nv[b], &L.vops32.nv[b]}) *v = cp.op64.nv;
      L.vops64.sloc[b] = L.vops32.sloc[b] = cp.op64.sloc;
      L.vops64.tile_g0[b] = L.vops32.tile_g0[b] = cp.op64.tile_g0;
      L.vops64.meta[b] = L.vops32.meta[b] = cp.meta;
      L.h_bmeta[b] = std::move(cp.h_meta);
    }
    if (L.op64.ntiles == 0) bad("vector operators need a tiled 3D stencil (reach 1 or 2)");
    auto fill_geom = [&](auto &v) {
      v.lat2row = L.op64.lat2row;
      v.sx = L.op64.sx;
      v.sy = L.op64.sy;
      v.sz = L.op64.sz;
      v.ntx = L.op64.ntx;
      v.nty = L.op64.nty;
      v.ntiles = L.op64.ntiles;
      v.ncomp = nc;
      v.ns = ns;
      v.cstride = L.cstride;
    };
    fill_geom(L.vops64);
    fill_geom(L.vops32);
    // per row only the general-block flag (set at factorization)
    L.h_meta.assign(L.n, 0u);
    L.meta = dalloc<uint32_t>(c->owned, L.n);
    h2d(s, L.meta, L.h_meta.data(), L.n);
    HIP_CHECK_RET(hipStreamSynchronize(s));
  }
  alloc_level_vectors(c, L);
}

// the level's padded work vectors (x, x2 ping-pong, r, rh; W-cycle copies)
void alloc_level_vectors(imsmg_ctx *c, Level &L) {
  hipStream_t s = c->stream;
  const size_t vlen = size_t(L.ncomp * L.cstride);
  double *vs[4];
  for (int k = 0; k < 4; ++k) {
    double *b = dalloc<double>(c->owned, vlen);
    HIP_CHECK_RET(hipMemsetAsync(b, 0, vlen * sizeof(double), s));
    vs[k] = b + L.guard;
  }
  L.r = vs[0];
  L.x = vs[1];
  L.x2 = vs[2];
  L.rh = vs[3];
  if (c->opt.cycle >= 2) {
    double *w[2];
    for (int k = 0; k < 2; ++k) {
      double *b = dalloc<double>(c->owned, vlen);
      HIP_CHECK_RET(hipMemsetAsync(b, 0, vlen * sizeof(double), s));
      w[k] = b + L.guard;
    }
    L.w_x = w[0];
    L.w_r = w[1];
  }
  // a V-cycle on this level runs (nu_pre - 1) + nu_post ping-pong steps: start
  // in the buffer that makes the result land in x
  L.xs = ((c->opt.nu_pre - 1 + c->opt.nu_post) % 2) ? L.x2 : L.x;
  HIP_CHECK_RET(hipStreamSynchronize(s));
}

// R (coarse x fine, compact) -> ELL on coarse rows with fine lattice columns,
// and R^T ELL on fine rows with coarse lattice columns.
// Bands of a dense 1D matrix M (rows x cols): per row the first and last
// non-zero column and the coefficients in between (zeros included).
void bands(const std::vector<double> &M, int rows, int cols, std::vector<int32_t> &start, std::vector<int32_t> &len,
           std::vector<double> &coef, int &W) {
  start.assign(rows, 0);
  len.assign(rows, 0);
  W = 1;
  for (int i = 0; i < rows; ++i) {
    int f = -1, l = -1;
    for (int j = 0; j < cols; ++j)
      if (M[size_t(i) * cols + j] != 0.0) {
        if (f < 0) f = j;
        l = j;
      }
    if (f >= 0) {
      start[i] = f;
      len[i] = l - f + 1;
      W = std::max(W, l - f + 1);
    }
  }
  coef.assign(size_t(rows) * W, 0.0);
  for (int i = 0; i < rows; ++i)
    for (int a = 0; a < len[i]; ++a) coef[size_t(i) * W + a] = M[size_t(i) * cols + start[i] + a];
}

void setup_tensor_transfer(imsmg_ctx *c, Level &F, const Level &Cl, const imsmg_csr &R, const double *R1) {
  hipStream_t s = c->stream;
  const int mc = Cl.shape[0], mf = F.shape[0];
  for (int a = 1; a < F.dim; ++a)
    if (Cl.shape[a] != mc || F.shape[a] != mf) bad("tensor transfer needs equal functions per axis");
  std::vector<double> M(R1, R1 + size_t(mc) * mf), Mt(size_t(mf) * mc);
  for (int i = 0; i < mc; ++i)
    for (int j = 0; j < mf; ++j) Mt[size_t(j) * mc + i] = M[size_t(i) * mf + j];
  // check the CSR R entry by entry against the masked tensor product (on the
  // scalar functions: R of a vector level is checked block by block before)
  std::vector<int32_t> f2c(size_t(F.lattice), -1);
  for (int k = 0; k < F.ns; ++k) f2c[F.h_lat[k]] = k;
  for (int i = 0; i < Cl.ns; ++i) {
    int mi[3] = {0, 0, 0};
    lat_multi(Cl.h_lat[i], Cl.shape, Cl.dim, mi);
    int64_t cnt = 0;
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
      if (a >= F.dim) continue;
      lo[a] = mf;
      hi[a] = -1;
      for (int j = 0; j < mf; ++j)
        if (M[size_t(mi[a]) * mf + j] != 0.0) {
          lo[a] = std::min(lo[a], j);
          hi[a] = std::max(hi[a], j);
        }
    }
    for (int z = lo[2]; z <= hi[2]; ++z)
      for (int y = lo[1]; y <= hi[1]; ++y)
        for (int x = lo[0]; x <= hi[0]; ++x) {
          int m[3] = {x, y, z};
          double v = 1.0;
          for (int a = 0; a < F.dim; ++a) v *= M[size_t(mi[a]) * mf + m[a]];
          if (v == 0.0) continue;
          if (f2c[size_t(lat_linear(m, F.shape, F.dim))] >= 0) ++cnt;
        }
    if (cnt != R.rowptr[i + 1] - R.rowptr[i]) bad("R is not the masked tensor product of the given two-scale matrix");
    for (int64_t k = R.rowptr[i]; k < R.rowptr[i + 1]; ++k) {
      int mk[3] = {0, 0, 0};
      lat_multi(F.h_lat[R.col[k]], F.shape, F.dim, mk);
      double v = 1.0;
      for (int a = 0; a < F.dim; ++a) v *= M[size_t(mi[a]) * mf + mk[a]];
      if (!(std::fabs(v - R.val[k]) <= 1e-13 * std::fabs(v)))
        bad("R is not the masked tensor product of the given two-scale matrix");
    }
  }
  std::vector<int32_t> rs, rl, ps, pl;
  std::vector<double> rcf, pcf;
  bands(M, mc, mf, rs, rl, rcf, F.rbW);
  bands(Mt, mf, mc, ps, pl, pcf, F.pbW);
  F.rb_start = dalloc<int32_t>(c->owned, mc);
  F.rb_len = dalloc<int32_t>(c->owned, mc);
  F.rb_coef = dalloc<double>(c->owned, rcf.size());
  F.pb_start = dalloc<int32_t>(c->owned, mf);
  F.pb_len = dalloc<int32_t>(c->owned, mf);
  F.pb_coef = dalloc<double>(c->owned, pcf.size());
  h2d(s, F.rb_start, rs.data(), mc);
  h2d(s, F.rb_len, rl.data(), mc);
  h2d(s, F.rb_coef, rcf.data(), rcf.size());
  h2d(s, F.pb_start, ps.data(), mf);
  h2d(s, F.pb_len, pl.data(), mf);
  h2d(s, F.pb_coef, pcf.data(), pcf.size());
  HIP_CHECK_RET(hipStreamSynchronize(s));
  F.tensor = true;
  // coarse window of every lattice tile for the fused prolongation: along
  // each axis, the coarse indices the bands of the tile's x window reach
  // (window = tile extent + the stencil reach on both sides)
  F.pro_ok = false;
  const bool tiled = F.op64.ntiles > 0;
  if (tiled && F.dim == 2 && F.ncomp == 1 && F.pbW <= kBandMax) {
    const int T[3] = {F.dim == 2 ? kTile2X : kTile3X, F.dim == 2 ? kTile2Y : kTile3Y, F.dim == 2 ? 1 : kTile3Z};
    const int nt[3] = {F.op64.ntx, F.op64.nty, F.dim == 3 ? (F.shape[2] + T[2] - 1) / T[2] : 1};
    // per-axis bound of the coarse window (the kernels' compile-time extent)
    std::vector<int32_t> org;
    bool ok = true;
    for (int a = 0; a < F.dim && ok; ++a) {
      const int P = F.reach, Wa = T[a] + 2 * P;
      const int cwa = Wa / 2 + kBandMax + 1;
      for (int b = 0; b < nt[a]; ++b) {
        int lo = INT32_MAX, hi = -1;
        for (int j = 0; j < Wa; ++j) {
          const int f = b * T[a] - P + j;
          if (f < 0 || f >= mf || pl[f] <= 0) continue;
          lo = std::min(lo, ps[f]);
          hi = std::max(hi, ps[f] + pl[f]);
        }
        if (hi < 0) lo = hi = 0;
        if (hi - lo > cwa) ok = false;
        org.push_back(lo);
      }
    }
    if (ok) {
      F.pro_org = dalloc<int32_t>(c->owned, org.size());
      h2d(s, F.pro_org, org.data(), org.size());
      std::vector<double> c5(size_t(mf) * kBandMax, 0.0);
      for (int f = 0; f < mf; ++f)
        for (int a = 0; a < pl[f]; ++a) c5[size_t(f) * kBandMax + a] = pcf[size_t(f) * F.pbW + a];
      F.pro_coef = dalloc<double>(c->owned, c5.size());
      h2d(s, F.pro_coef, c5.data(), c5.size());
      HIP_CHECK_RET(hipStreamSynchronize(s));
      F.pro_ok = true;
    }
  }
}

void setup_transfer(imsmg_ctx *c, Level &F, const Level &Cl, const imsmg_csr &R, const double *two_scale) {
  hipStream_t s = c->stream;
  if (R.nrows != Cl.n || R.ncols != F.n) bad("R shape must be n_{l-1} x n_l");
  if (!R.rowptr || !R.col || !R.val) bad("null R array");
  if (R.rowptr[0] != 0 || R.rowptr[R.nrows] != R.nnz) bad("R rowptr inconsistent with nnz");
  int rw = 0;
  for (int i = 0; i < R.nrows; ++i) rw = std::max<int>(rw, int(R.rowptr[i + 1] - R.rowptr[i]));
  std::vector<int32_t> cnt(F.n, 0);
  for (int64_t k = 0; k < R.nnz; ++k) {
    if (R.col[k] < 0 || R.col[k] >= F.n) bad("R column out of range");
    cnt[R.col[k]]++;
  }
  int tw = 0;
  for (int i = 0; i < F.n; ++i) tw = std::max(tw, cnt[i]);
  rw = std::max(rw, 1);
  tw = std::max(tw, 1);
  // padding entries: value 0 at the row's own first column (any in-range index)
  std::vector<int32_t> rcol(size_t(rw) * Cl.n, int32_t(F.h_row_lat[0]));
  std::vector<double> rval(size_t(rw) * Cl.n, 0.0);
  std::vector<int32_t> tcol(size_t(tw) * F.n, int32_t(Cl.h_row_lat[0]));
  std::vector<double> tval(size_t(tw) * F.n, 0.0);
  std::vector<int32_t> fill(F.n, 0);
  for (int i = 0; i < Cl.n; ++i) {
    int slot = 0;
    for (int64_t k = R.rowptr[i]; k < R.rowptr[i + 1]; ++k, ++slot) {
      const int j = R.col[k];
      rcol[size_t(slot) * Cl.n + i] = F.h_row_lat[j];
      rval[size_t(slot) * Cl.n + i] = R.val[k];
      const int ts = fill[j]++;
      tcol[size_t(ts) * F.n + j] = Cl.h_row_lat[i];
      tval[size_t(ts) * F.n + j] = R.val[k];
    }
  }
  if (two_scale) {
    if (F.ncomp == 1) {
      setup_tensor_transfer(c, F, Cl, R, two_scale);
      return;
    }
    // vector level: R = I (x) R_s; the scalar block R_s, and every other
    // diagonal block equal to it, no coupling between components
    const int nsf = F.ns, nsc = Cl.ns;
    std::vector<int32_t> rp(size_t(nsc) + 1, 0), rc;
    std::vector<double> rv;
    for (int i = 0; i < nsc; ++i) {
      for (int64_t k = R.rowptr[i]; k < R.rowptr[i + 1]; ++k) {
        if (R.col[k] >= nsf) bad("vector R must be block diagonal (one block per component)");
        rc.push_back(R.col[k]);
        rv.push_back(R.val[k]);
      }
      rp[size_t(i) + 1] = int32_t(rc.size());
    }
    for (int cc = 1; cc < F.ncomp; ++cc)
      for (int i = 0; i < nsc; ++i) {
        const int r = cc * nsc + i;
        if (R.rowptr[r + 1] - R.rowptr[r] != rp[size_t(i) + 1] - rp[size_t(i)])
          bad("vector R must repeat one scalar block per component");
        for (int64_t k = R.rowptr[r], q = rp[size_t(i)]; k < R.rowptr[r + 1]; ++k, ++q)
          if (R.col[k] != rc[size_t(q)] + cc * nsf || R.val[k] != rv[size_t(q)])
            bad("vector R must repeat one scalar block per component");
      }
    const imsmg_csr Rs{nsc, nsf, int64_t(rc.size()), rp.data(), rc.data(), rv.data()};
    setup_tensor_transfer(c, F, Cl, Rs, two_scale);
    return;
  }
  F.rw = rw;
  F.tw = tw;
  F.rcol = dalloc<int32_t>(c->owned, rcol.size());
  F.rval = dalloc<double>(c->owned, rval.size());
  F.tcol = dalloc<int32_t>(c->owned, tcol.size());
  F.tval = dalloc<double>(c->owned, tval.size());
  h2d(s, F.rcol, rcol.data(), rcol.size());
  h2d(s, F.rval, rval.data(), rval.size());
  h2d(s, F.tcol, tcol.data(), tcol.size());
  h2d(s, F.tval, tval.data(), tval.size());
  HIP_CHECK_RET(hipStreamSynchronize(s));
}

// ------------------------------------------------------------ V-cycle
hipEvent_t *timed_pair(imsmg_ctx *c) {
  if (c->ev_used + 2 > c->ev_pool.size()) {
    for (int k = 0; k < 64; ++k) {
      hipEvent_t e;
      HIP_CHECK_RET(hipEventCreate(&e));
      c->ev_pool.push_back(e);
    }
  }
  hipEvent_t *p = &c->ev_pool[c->ev_used];
  c->ev_used += 2;
  return p;
}

bool mixed(imsmg_ctx *c) { return c->opt.precision == IMSMG_MIXED; }

// Levels below opt.flag_min_rows rows (default 65536) are launch-latency
// bound: their kernels skip the convergence-flag load, which would add one
// dependent memory round trip to every launch (the wasted work after
// convergence is negligible there).
constexpr int kSmallLevel = 65536;

const int32_t *flag_for(const imsmg_ctx *c, const Level &L, const int32_t *done) {
  return L.n >= c->opt.flag_min_rows ? done : nullptr;
}

// y = b - A_l x (b == nullptr: y = A_l x); the V-cycle operator precision
void residual(imsmg_ctx *c, Level &L, const double *x, const double *b, double *y, const int32_t *done,
              bool timed) {
  hipEvent_t *ev = timed ? timed_pair(c) : nullptr;
  if (ev) HIP_CHECK_RET(hipEventRecord(ev[0], c->stream));
  if (L.csr) {
    if (mixed(c))
      launch_csr_residual(c->stream, L.n, L.csr_lanes, L.a32, L.meta, x, b, y, done);
    else
      launch_csr_residual(c->stream, L.n, L.csr_lanes, L.a64, L.meta, x, b, y, done);
  } else if (L.ncomp > 1) {
    if (mixed(c))
      launch_vresidual(c->stream, L.K, L.vops32, L.meta, x, b, y, done);
    else
      launch_vresidual(c->stream, L.K, L.vops64, L.meta, x, b, y, done);
  } else if (mixed(c)) {
    launch_residual(c->stream, L.n, L.K, L.op32, L.row_lat, L.meta, x, b, y, done);
  } else {
    launch_residual(c->stream, L.n, L.K, L.op64, L.row_lat, L.meta, x, b, y, done);
  }
  if (ev) HIP_CHECK_RET(hipEventRecord(ev[1], c->stream));
}

// smoothing step from xa: rh = r - A xa, xb = xa + S rh  (trivial rows fused,
// then the general rows); pv: from xa + R^T xc (prolongation fused)
void smooth_step(imsmg_ctx *c, Level &L, const double *xa, double *xb, const int32_t *done, bool timed,
                 const ProlongView *pv = nullptr) {
  hipEvent_t *ev = timed ? timed_pair(c) : nullptr;
  if (ev) HIP_CHECK_RET(hipEventRecord(ev[0], c->stream));
  // timed: opt.timing identical launches (xa and r are only read)
  const int reps = ev ? c->opt.timing : 1;
  for (int k = 0; k < reps; ++k) {
    if (L.csr) {
      if (pv) bad("internal: fused prolongation on a general sparse level", IMSMG_ERR_HIP);
      if (mixed(c))
        launch_csr_residual_smooth(c->stream, L.n, L.csr_lanes, L.a32, L.meta, L.c, xa, L.r, L.rh, xb, done);
      else
        launch_csr_residual_smooth(c->stream, L.n, L.csr_lanes, L.a64, L.meta, L.c, xa, L.r, L.rh, xb, done);
    } else if (L.ncomp > 1) {
      if (pv) bad("internal: fused prolongation on a vector level", IMSMG_ERR_HIP);
      if (mixed(c))
        launch_vresidual_smooth(c->stream, L.K, L.vops32, L.meta, L.c, xa, L.r, L.rh, xb, done);
      else
        launch_vresidual_smooth(c->stream, L.K, L.vops64, L.meta, L.c, xa, L.r, L.rh, xb, done);
    } else if (mixed(c)) {
      launch_residual_smooth(c->stream, L.n, L.K, L.op32, L.row_lat, L.meta, L.c, xa, L.r, L.rh, xb, done, pv);
    } else {
      launch_residual_smooth(c->stream, L.n, L.K, L.op64, L.row_lat, L.meta, L.c, xa, L.r, L.rh, xb, done, pv);
    }
  }
  if (ev) HIP_CHECK_RET(hipEventRecord(ev[1], c->stream));
  launch_smooth_general(c->stream, L.ng, L.grow_lat, L.sptr, L.scol, L.sval, L.rh, xb, done, L.gen_lanes);
}

// rc = R_l rf (fine level L, coarse level Cl; padded vectors)
// (xinit != nullptr: also xinit = c_coarse * rc, the trivial part of the
// coarse level's first smoothing step)
void restrict_to(imsmg_ctx *c, Level &L, Level &Cl, const double *rf, double *rc, double *xinit,
                 const int32_t *done) {
  const double *ci = xinit ? Cl.c : nullptr;
  if (L.tensor) {
    // vector levels: the scalar transfer once per component
    for (int cc = 0; cc < L.ncomp; ++cc)
      launch_tensor_transfer(c->stream, L.dim, Cl.ns, Cl.srow_lat, Cl.shape[0], Cl.shape[1], L.rb_start, L.rb_len,
                             L.rb_coef, L.rbW, L.shape[0], L.shape[1], rf + cc * L.cstride, rc + cc * Cl.cstride, 0,
                             ci ? ci + size_t(cc) * Cl.ns : nullptr, xinit ? xinit + cc * Cl.cstride : nullptr, done);
  } else {
    launch_ell_gather(c->stream, Cl.n, L.rw, Cl.row_lat, L.rcol, L.rval, rf, rc, 0, ci, xinit, done);
  }
}

// xf += R_l^T xc
void prolong_add(imsmg_ctx *c, Level &L, Level &Cl, const double *xc, double *xf, const int32_t *done) {
  if (L.tensor)
    for (int cc = 0; cc < L.ncomp; ++cc)
      launch_tensor_transfer(c->stream, L.dim, L.ns, L.srow_lat, L.shape[0], L.shape[1], L.pb_start, L.pb_len,
                             L.pb_coef, L.pbW, Cl.shape[0], Cl.shape[1], xc + cc * Cl.cstride, xf + cc * L.cstride, 1,
                             nullptr, nullptr, done);
  else
    launch_ell_gather(c->stream, L.n, L.tw, L.row_lat, L.tcol, L.tval, xc, xf, 1, nullptr, nullptr, done);
}

// One multiplicative Schwarz sweep on level L (eq:multiplicativeSchwarz1,
// coloured): colours in ascending order (forward, pre-smoothing) or
// descending (its adjoint, post-smoothing); x is updated in place from the
// residual r - A x of level L's input residual r.
void ms_sweep(imsmg_ctx *c, Level &L, bool forward, const int32_t *done) {
  for (int k = 0; k < L.ncolours; ++k) {
    const int cc = forward ? k : L.ncolours - 1 - k;
    const int a = L.ms_cptr[cc], m = L.ms_cptr[cc + 1] - a;
    if (m == 0) continue;
    if (L.csr) {
      if (mixed(c))
        launch_csr_ms_colour(c->stream, m, L.csr_lanes, L.ms_rows + a, L.ms_cf + a, L.a32, L.r, L.x, L.rh, done);
      else
        launch_csr_ms_colour(c->stream, m, L.csr_lanes, L.ms_rows + a, L.ms_cf + a, L.a64, L.r, L.x, L.rh, done);
    } else if (L.ncomp > 1) {
      if (mixed(c))
        launch_vms_colour(c->stream, m, L.ms_rows + a, L.ms_cf + a, L.ms_vidx + size_t(a) * L.ncomp, L.ms_val32,
                          L.K, L.vops32, L.row_lat, L.r, L.x, L.rh, done, L.ms_stream32);
      else
        launch_vms_colour(c->stream, m, L.ms_rows + a, L.ms_cf + a, L.ms_vidx + size_t(a) * L.ncomp, L.ms_val64,
                          L.K, L.vops64, L.row_lat, L.r, L.x, L.rh, done, L.ms_stream64);
    } else if (mixed(c))
      launch_ms_colour(c->stream, m, L.ms_lat + a, L.ms_cf + a, L.ms_vidx + a, L.ms_val32, L.K, L.op32, nullptr,
                       L.r, L.x, L.rh, done, L.ms_stream32);
    else
      launch_ms_colour(c->stream, m, L.ms_lat + a, L.ms_cf + a, L.ms_vidx + a, L.ms_val64, L.K, L.op64, nullptr,
                       L.r, L.x, L.rh, done, L.ms_stream64);
    const Level::MsGeneral &G = L.ms_gen[cc];
    if (G.ng > 0) launch_smooth_general(c->stream, G.ng, G.grow_lat, G.sptr, G.scol, G.sval, L.rh, L.x, done, 4);
  }
}

void vcycle_level(imsmg_ctx *c, int l, const int32_t *done_top, bool timing);

// Coarse correction of level l > 0: Cl.x = B_{l-1} Cl.r by one coarse cycle
// (V), or by two where level l-1 has its own coarse level (W: the second
// cycle on the residual the first leaves, its result added to the first).
void coarse_correction(imsmg_ctx *c, int l, const int32_t *done_top, bool timing) {
  Level &Cl = c->lv[l - 1];
  vcycle_level(c, l - 1, done_top, timing);
  if (c->opt.cycle < 2 || l - 1 == 0) return;
  const int32_t *dn = flag_for(c, Cl, done_top);
  for (int k = 1; k < c->opt.cycle; ++k) {
    launch_rows_op(c->stream, Cl.n, Cl.row_lat, Cl.x, Cl.w_x, 1, dn);  // w_x = x
    residual(c, Cl, Cl.x, Cl.r, Cl.w_r, dn, false);                     // w_r = r - A x
    std::swap(Cl.r, Cl.w_r);  // the next cycle's input residual (swapped back below)
    if (!Cl.ms) launch_diag_scale(c->stream, Cl.n, Cl.row_lat, Cl.c, Cl.r, Cl.xs, dn);
    vcycle_level(c, l - 1, done_top, timing);
    std::swap(Cl.r, Cl.w_r);
    launch_rows_op(c->stream, Cl.n, Cl.row_lat, Cl.w_x, Cl.x, 2, dn);  // x += w_x
  }
}

// V-cycle on level l (Algorithm alg:MGV): input residual in lv[l].r; on entry
// lv[l].xs already holds c * r (trivial part of the first smoothing step,
// written by the caller's fused kernel) on additive levels; the correction is
// left in lv[l].x.
void vcycle_level(imsmg_ctx *c, int l, const int32_t *done_top, bool timing) {
  Level &L = c->lv[l];
  const int32_t *done = flag_for(c, L, done_top);
  if (l == 0) {
    launch_dense_gemv(c->stream, L.n, L.row_lat, L.Ainv, L.r, L.x, done);
    return;
  }
  Level &Cl = c->lv[l - 1];
  if (L.ms) {
    // multiplicative smoother: x = 0, nu_pre forward sweeps, coarse
    // correction, nu_post reversed sweeps (symmetric cycle)
    launch_rows_op(c->stream, L.n, L.row_lat, nullptr, L.x, 0, done);
    for (int k = 0; k < c->opt.nu_pre; ++k) ms_sweep(c, L, true, done);
    residual(c, L, L.x, L.r, L.rh, done, false);
    restrict_to(c, L, Cl, L.rh, Cl.r, (l - 1 > 0 && !Cl.ms) ? Cl.xs : nullptr, flag_for(c, Cl, done_top));
    coarse_correction(c, l, done_top, timing);
    prolong_add(c, L, Cl, Cl.x, L.x, done);
    for (int k = 0; k < c->opt.nu_post; ++k) ms_sweep(c, L, false, done);
    return;
  }
  const bool fine = (l == int(c->lv.size()) - 1) && timing;
  // first smoothing step from x = 0: x = S r (general rows)
  launch_smooth_general(c->stream, L.ng, L.grow_lat, L.sptr, L.scol, L.sval, L.r, L.xs, done, L.gen_lanes);
  double *xa = L.xs, *xb = (L.xs == L.x) ? L.x2 : L.x;
  for (int k = 1; k < c->opt.nu_pre; ++k) {
    smooth_step(c, L, xa, xb, done, fine);
    std::swap(xa, xb);
  }
  residual(c, L, xa, L.r, L.rh, done, false);
  restrict_to(c, L, Cl, L.rh, Cl.r, (l - 1 > 0 && !Cl.ms) ? Cl.xs : nullptr, flag_for(c, Cl, done_top));
  coarse_correction(c, l, done_top, timing);
  int k = 0;
  if (L.pro_ok && c->opt.nu_post > 0) {
    // x += R^T x_c inside the first post-smoothing step's staging (not one of
    // the timed plain smoothing steps)
    const ProlongView pv{Cl.x, L.pb_start, L.pb_len, L.pro_coef, L.pbW, Cl.shape[0], L.pro_org};
    smooth_step(c, L, xa, xb, done, false, &pv);
    std::swap(xa, xb);
    k = 1;
  } else {
    prolong_add(c, L, Cl, Cl.x, xa, done);
  }
  for (; k < c->opt.nu_post; ++k) {
    smooth_step(c, L, xa, xb, done, fine);
    std::swap(xa, xb);
  }
}

void collect_timing(imsmg_ctx *c) {
  for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
    float ms = 0.f;
    HIP_CHECK_RET(hipEventElapsedTime(&ms, c->ev_pool[k], c->ev_pool[k + 1]));
    c->t_kernel_ms += ms;
    c->t_kernel_n += c->opt.timing;
  }
  c->ev_used = 0;
}

// ------------------------------------------------------------- factorization
void apply_weights(imsmg_ctx *c, Level &L, const std::vector<double> &w);

// Colours of the final blocks (fptr/fidx; forig = input block or -1 for an
// added singleton).  Blocks interact only through elements they share (A_ij
// vanishes unless phi_i and phi_j share an active element), so a colouring is
// valid when no two blocks of one colour touch a common element.  Given
// colours are checked; blocks without one (no colours given, or added
// singletons) take, in block order, the smallest colour >= base that no
// already coloured block uses on their elements (base = 0 without given
// colours, else max given + 1).
void colour_level(Level &L, const std::vector<int32_t> &fptr, const std::vector<int32_t> &fidx,
                  const std::vector<int32_t> &forig) {
  const int nbf = int(fptr.size()) - 1;
  L.f_colour.assign(nbf, 0);
  L.ncolours = 0;
  if (L.e_ptr.empty()) return;  // without the element incidence there is nothing to colour by
  const int nel = int(L.e_ptr.size()) - 1;
  // function -> elements
  std::vector<int32_t> fe_ptr(L.n + 1, 0), fe_idx(L.e_idx.size());
  for (int32_t f : L.e_idx) fe_ptr[f + 1]++;
  for (int i = 0; i < L.n; ++i) fe_ptr[i + 1] += fe_ptr[i];
  {
    std::vector<int32_t> fill(fe_ptr.begin(), fe_ptr.end() - 1);
    for (int e = 0; e < nel; ++e)
      for (int k = L.e_ptr[e]; k < L.e_ptr[e + 1]; ++k) fe_idx[fill[L.e_idx[k]]++] = e;
  }
  const bool given = !L.in_colour.empty();
  int base = 0;
  if (given)
    for (int32_t v : L.in_colour) base = std::max(base, v + 1);
  std::vector<uint64_t> used(size_t(nel) * 2, 0);
  std::vector<int32_t> stamp(nel, -1), els;
  for (int j = 0; j < nbf; ++j) {
    els.clear();
    for (int k = fptr[j]; k < fptr[j + 1]; ++k) {
      const int i = fidx[k];
      for (int q = fe_ptr[i]; q < fe_ptr[i + 1]; ++q) {
        const int e = fe_idx[q];
        if (stamp[e] != j) {
          stamp[e] = j;
          els.push_back(e);
        }
      }
    }
    int col;
    if (given && forig[j] >= 0) {
      col = L.in_colour[forig[j]];
      for (int e : els)
        if ((used[2 * size_t(e) + (col >> 6)] >> (col & 63)) & 1)
          bad("blocks of colour " + std::to_string(col) + " share an element");
    } else {
      uint64_t taken[2] = {0, 0};
      for (int e : els) {
        taken[0] |= used[2 * size_t(e)];
        taken[1] |= used[2 * size_t(e) + 1];
      }
      col = base;
      while (col < kMaxColours && ((taken[col >> 6] >> (col & 63)) & 1)) ++col;
      if (col >= kMaxColours) bad("more than " + std::to_string(kMaxColours) + " colours needed");
    }
    for (int e : els) used[2 * size_t(e) + (col >> 6)] |= uint64_t(1) << (col & 63);
    L.f_colour[j] = col;
    L.ncolours = std::max(L.ncolours, col + 1);
  }
}

// Device data of the multiplicative smoother (after the block inverses exist,
// unscaled): per colour the touched rows with their coefficients and the
// larger blocks' inverses as CSR on their members (row a of block j = row a
// of A_j^-1, columns at the members' lattice positions).
void build_ms(imsmg_ctx *c, Level &L, const std::vector<int32_t> &fptr, const std::vector<int32_t> &fidx,
              const std::vector<int64_t> &finvoff, const std::vector<double> &diag, int64_t ninv) {
  hipStream_t s = c->stream;
  const int nbf = int(fptr.size()) - 1;
  const int C = L.ncolours;
  if (C == 0 && nbf > 0) bad("the multiplicative smoother needs the element incidence of the level (colours)");
  std::vector<double> inv(size_t(std::max<int64_t>(ninv, 1)));
  if (ninv > 0) d2h(s, inv.data(), L.inv, size_t(ninv));
  HIP_CHECK_RET(hipStreamSynchronize(s));
  std::vector<std::vector<int32_t>> rows(C);
  std::vector<std::vector<double>> cf(C);
  struct Csr {
    std::vector<int32_t> glat, ptr{0}, col;
    std::vector<double> val;
  };
  std::vector<Csr> gen(C);
  for (int j = 0; j < nbf; ++j) {
    const int sz = fptr[j + 1] - fptr[j];
    if (sz == 0) continue;
    const int cc = L.f_colour[j];
    if (sz == 1) {
      const int i = fidx[fptr[j]];
      if (!(diag[i] > 0.0)) bad("non-positive diagonal entry", IMSMG_ERR_NOT_SPD);
      rows[cc].push_back(i);
      cf[cc].push_back(1.0 / diag[i]);
      continue;
    }
    if (finvoff[j] < 0) bad("internal: block without an inverse", IMSMG_ERR_HIP);
    Csr &G = gen[cc];
    for (int a = 0; a < sz; ++a) {
      const int i = fidx[fptr[j] + a];
      rows[cc].push_back(i);
      cf[cc].push_back(0.0);
      G.glat.push_back(L.h_row_lat[i]);
      for (int b = 0; b < sz; ++b) {
        G.col.push_back(L.h_row_lat[fidx[fptr[j] + b]]);
        G.val.push_back(inv[size_t(finvoff[j]) + size_t(a) + size_t(sz) * b]);
      }
      G.ptr.push_back(int32_t(G.col.size()));
    }
  }
  L.ms_cptr.assign(1, 0);
  std::vector<int32_t> all_rows;
  std::vector<double> all_cf;
  for (int cc = 0; cc < C; ++cc) {
    all_rows.insert(all_rows.end(), rows[cc].begin(), rows[cc].end());
    all_cf.insert(all_cf.end(), cf[cc].begin(), cf[cc].end());
    L.ms_cptr.push_back(int32_t(all_rows.size()));
  }
  L.ms_rows = dalloc<int32_t>(c->factor_owned, std::max<size_t>(all_rows.size(), 1));
  L.ms_lat = dalloc<int32_t>(c->factor_owned, std::max<size_t>(all_rows.size(), 1));
  L.ms_cf = dalloc<double>(c->factor_owned, std::max<size_t>(all_cf.size(), 1));
  if (!all_rows.empty()) {
    std::vector<int32_t> all_lat(all_rows.size());
    for (size_t t = 0; t < all_rows.size(); ++t) all_lat[t] = L.h_row_lat[all_rows[t]];
    h2d(s, L.ms_rows, all_rows.data(), all_rows.size());
    h2d(s, L.ms_lat, all_lat.data(), all_lat.size());
    h2d(s, L.ms_cf, all_cf.data(), all_cf.size());
  }
  // colour-ordered copy of the stored rows' values: one entry per list entry
  // (vector levels: per list entry and component block) whose row keeps its
  // own values; entries grouped by block, each group packed from its block
  // (general sparse levels read their CSR rows instead)
  const int nc = L.ncomp, nb = L.csr ? 0 : nc * nc;
  std::vector<int32_t> vidx(all_rows.size() * nc, -1);
  std::vector<std::vector<int32_t>> vg(nb), vpos(nb);
  for (size_t t = 0; nb > 0 && t < all_rows.size(); ++t) {
    const int i = all_rows[t];
    const int ci = i / L.ns, is = i % L.ns;
    for (int e = 0; e < nc; ++e) {
      const int b = ci * nc + e;
      const uint32_t g = (nc == 1 ? L.h_meta[i] : L.h_bmeta[b][is]) & kMetaIndex;
      if (g != kMetaIndex) {
        vpos[b].push_back(int32_t(t * nc + e));
        vg[b].push_back(int32_t(g));
      }
    }
  }
  int ne = 0;
  for (int b = 0; b < nb; ++b) {
    for (size_t k = 0; k < vpos[b].size(); ++k) vidx[vpos[b][k]] = ne + int32_t(k);
    ne += int(vg[b].size());
  }
  L.ms_vidx = dalloc<int32_t>(c->factor_owned, std::max<size_t>(vidx.size(), 1));
  if (!vidx.empty()) h2d(s, L.ms_vidx, vidx.data(), vidx.size());
  {
    const int KP64 = (L.K + 1) / 2 * 2, KP32 = (L.K + 3) / 4 * 4;
    L.ms_stream64 = L.ms_stream32 = size_t(ne) * KP64 > kStreamValues;
    L.ms_val64 = dalloc<double>(c->factor_owned, std::max<size_t>(size_t(ne) * KP64, 2));
    if (mixed(c)) L.ms_val32 = dalloc<float>(c->factor_owned, std::max<size_t>(size_t(ne) * KP32, 4));
    int e0 = 0;
    for (int b = 0; b < nb; ++b) {
      const int nbe = int(vg[b].size());
      if (nbe == 0) continue;
      int32_t *d_g = dalloc<int32_t>(c->factor_owned, nbe);
      h2d(s, d_g, vg[b].data(), vg[b].size());
      const double *v64 = nc == 1 ? L.op64.val : L.vops64.val[b];
      const int nv = nc == 1 ? L.op64.nv : L.vops64.nv[b];
      launch_ms_pack(s, nbe, L.K, KP64, d_g, v64, nv, L.ms_val64 + size_t(e0) * KP64);
      if (mixed(c)) {
        const float *v32 = nc == 1 ? L.op32.val : L.vops32.val[b];
        launch_ms_pack(s, nbe, L.K, KP32, d_g, v32, nv, L.ms_val32 + size_t(e0) * KP32);
      }
      e0 += nbe;
    }
    HIP_CHECK_RET(hipGetLastError());
  }
  L.ms_gen.assign(C, Level::MsGeneral{});
  for (int cc = 0; cc < C; ++cc) {
    const Csr &G = gen[cc];
    Level::MsGeneral &D = L.ms_gen[cc];
    D.ng = int(G.glat.size());
    if (D.ng == 0) continue;
    D.grow_lat = dalloc<int32_t>(c->factor_owned, G.glat.size());
    D.sptr = dalloc<int32_t>(c->factor_owned, G.ptr.size());
    D.scol = dalloc<int32_t>(c->factor_owned, G.col.size());
    D.sval = dalloc<double>(c->factor_owned, G.val.size());
    h2d(s, D.grow_lat, G.glat.data(), G.glat.size());
    h2d(s, D.sptr, G.ptr.data(), G.ptr.size());
    h2d(s, D.scol, G.col.data(), G.col.size());
    h2d(s, D.sval, G.val.data(), G.val.size());
  }
  HIP_CHECK_RET(hipStreamSynchronize(s));
}

void factor_level(imsmg_ctx *c, int l) {
  hipStream_t s = c->stream;
  Level &L = c->lv[l];
  for (auto &m : L.h_meta) m &= ~kMetaGeneral;
  const int nb_in = int(L.in_ptr.size()) - 1;
  const int n = L.n;
  // which input blocks need the eigensolver (size >= 2)
  std::vector<int32_t> fac_blocks;
  int maxn = 1;
  for (int j = 0; j < nb_in; ++j) {
    const int sz = L.in_ptr[j + 1] - L.in_ptr[j];
    if (sz >= 2) {
      fac_blocks.push_back(j);
      maxn = std::max(maxn, sz);
    }
  }
  if (maxn > IMSMG_MAX_BLOCK)
    bad("Schwarz block of size " + std::to_string(maxn) + " exceeds the supported " +
        std::to_string(IMSMG_MAX_BLOCK));
  const int nf = int(fac_blocks.size());
  std::vector<int32_t> h_bstart(nf + 1, 0), h_bsize(nf), h_blat, h_brow;
  std::vector<int64_t> h_invoff(nf + 1, 0);
  for (int t = 0; t < nf; ++t) {
    const int j = fac_blocks[t];
    const int sz = L.in_ptr[j + 1] - L.in_ptr[j];
    h_bsize[t] = sz;
    h_bstart[t + 1] = h_bstart[t] + sz;
    h_invoff[t + 1] = h_invoff[t] + int64_t(sz) * sz;
    for (int k = L.in_ptr[j]; k < L.in_ptr[j + 1]; ++k) {
      h_brow.push_back(L.in_idx[k]);
      h_blat.push_back(L.h_lat[L.in_idx[k]]);  // lattice point (the gather's slot geometry)
    }
  }
  std::vector<void *> tmp;
  struct TmpFree {
    std::vector<void *> &v;
    ~TmpFree() { free_list(v); }
  } tf{tmp};
  int32_t *d_bstart = dalloc<int32_t>(tmp, nf + 1), *d_bsize = dalloc<int32_t>(tmp, nf);
  int32_t *d_blat = dalloc<int32_t>(tmp, h_blat.size()), *d_brow = dalloc<int32_t>(tmp, h_brow.size());
  int64_t *d_invoff = dalloc<int64_t>(c->factor_owned, nf + 1);
  double *d_inv = dalloc<double>(c->factor_owned, size_t(h_invoff[nf]));
  uint8_t *d_keep = dalloc<uint8_t>(tmp, h_blat.size());
  double *d_lam = dalloc<double>(tmp, 4 * size_t(std::max(nf, 1)));
  int32_t *d_info = dalloc<int32_t>(tmp, nf);
  h2d(s, d_bstart, h_bstart.data(), nf + 1);
  h2d(s, d_bsize, h_bsize.data(), nf);
  h2d(s, d_blat, h_blat.data(), h_blat.size());
  h2d(s, d_brow, h_brow.data(), h_brow.size());
  h2d(s, d_invoff, h_invoff.data(), nf + 1);
  const int frc = L.csr ? launch_block_factor_csr(s, nf, maxn, d_bstart, d_bsize, d_brow, L.a64, d_inv, d_invoff,
                                                  d_keep, d_lam, d_info, 1e-16)
                       : launch_block_factor_geom(s, nf, maxn, d_bstart, d_bsize, d_blat, d_brow, n, L.dim,
                                                  L.shape[0], L.shape[1], L.reach, L.val, d_inv, d_invoff, d_keep,
                                                  d_lam, d_info, 1e-16);
  if (frc != 0) bad("block factorization launch rejected");
  HIP_CHECK_RET(hipGetLastError());
  std::vector<uint8_t> keep(h_blat.size());
  std::vector<int32_t> info(nf);
  d2h(s, keep.data(), d_keep, keep.size());
  d2h(s, info.data(), d_info, info.size());
  std::vector<double> lam(4 * size_t(nf));
  d2h(s, lam.data(), d_lam, lam.size());
  std::vector<double> diag(n);
  d2h(s, diag.data(), L.val + size_t(L.center) * n, n);
  HIP_CHECK_RET(hipStreamSynchronize(s));
  // diagonal of A for singleton checks
  // final block lists: kept members of every input block, then singletons
  // for DOFs left in no block
  std::vector<int32_t> fptr(1, 0), fidx, forig;  // forig: input block index or -1 (added)
  std::vector<int64_t> finvoff;                   // inverse offset for factorized blocks, -1 otherwise
  std::vector<char> covered(n, 0);
  int t = 0;
  for (int j = 0; j < nb_in; ++j) {
    const int sz = L.in_ptr[j + 1] - L.in_ptr[j];
    if (sz >= 2) {
      int kept = 0;
      for (int a = 0; a < sz; ++a)
        if (keep[h_bstart[t] + a]) {
          fidx.push_back(L.in_idx[L.in_ptr[j] + a]);
          covered[L.in_idx[L.in_ptr[j] + a]] = 1;
          ++kept;
        }
      if (kept != info[t]) bad("internal: factorization bookkeeping mismatch", IMSMG_ERR_HIP);
      finvoff.push_back(h_invoff[t]);
      ++t;
    } else if (sz == 1) {
      fidx.push_back(L.in_idx[L.in_ptr[j]]);
      covered[L.in_idx[L.in_ptr[j]]] = 1;
      finvoff.push_back(-1);
    } else {
      finvoff.push_back(-1);
    }
    fptr.push_back(int32_t(fidx.size()));
    forig.push_back(j);
  }
  for (int i = 0; i < n; ++i)
    if (!covered[i]) {
      fidx.push_back(i);
      fptr.push_back(int32_t(fidx.size()));
      forig.push_back(-1);
      finvoff.push_back(-1);
    }
  L.f_ptr = fptr;
  L.f_idx = fidx;
  const int nbf = int(fptr.size()) - 1;
  L.f_orig = forig;
  L.f_lam.assign(4 * size_t(nbf), 1.0);
  {
    int tt = 0;
    for (int j = 0; j < nbf; ++j) {
      const int jo = forig[j];
      const int szin = jo >= 0 ? L.in_ptr[jo + 1] - L.in_ptr[jo] : 1;
      if (jo >= 0 && szin >= 2) {
        for (int q = 0; q < 4; ++q) L.f_lam[4 * size_t(j) + q] = lam[4 * size_t(tt) + q];
        ++tt;
      } else if (fptr[j + 1] > fptr[j]) {
        const double d = diag[fidx[fptr[j]]];
        for (int q = 0; q < 4; ++q) L.f_lam[4 * size_t(j) + q] = d;
      }
    }
  }
  // number of final blocks holding each DOF
  std::vector<int32_t> fcount(n, 0);
  for (int32_t i : fidx) fcount[i]++;
  // N_K -> gamma
  double gamma = c->opt.gamma;
  if (gamma <= 0.0 && L.e_ptr.empty()) bad("gamma <= 0 needs the element incidence of every smoothed level");
  L.nk.clear();
  if (!L.e_ptr.empty()) {
    std::vector<int32_t> fp(n + 1, 0), fb(fidx.size());
    for (int32_t i : fidx) fp[i + 1]++;
    for (int i = 0; i < n; ++i) fp[i + 1] += fp[i];
    std::vector<int32_t> fill(fp.begin(), fp.end() - 1);
    for (int j = 0; j < nbf; ++j)
      for (int k = fptr[j]; k < fptr[j + 1]; ++k) fb[fill[fidx[k]]++] = j;
    const int nel = int(L.e_ptr.size()) - 1;
    int32_t *d_eptr = dalloc<int32_t>(tmp, nel + 1), *d_eidx = dalloc<int32_t>(tmp, L.e_idx.size());
    int32_t *d_fp = dalloc<int32_t>(tmp, n + 1), *d_fb = dalloc<int32_t>(tmp, fb.size());
    int32_t *d_nk = dalloc<int32_t>(tmp, nel), *d_ovf = dalloc<int32_t>(tmp, 1);
    h2d(s, d_eptr, L.e_ptr.data(), nel + 1);
    h2d(s, d_eidx, L.e_idx.data(), L.e_idx.size());
    h2d(s, d_fp, fp.data(), n + 1);
    h2d(s, d_fb, fb.data(), fb.size());
    HIP_CHECK_RET(hipMemsetAsync(d_ovf, 0, sizeof(int32_t), s));
    launch_count_nk(s, nel, d_eptr, d_eidx, d_fp, d_fb, d_nk, d_ovf);
    HIP_CHECK_RET(hipGetLastError());
    std::vector<int32_t> nk(nel);
    int32_t ovf = 0;
    d2h(s, nk.data(), d_nk, nel);
    d2h(s, &ovf, d_ovf, 1);
    HIP_CHECK_RET(hipStreamSynchronize(s));
    if (ovf) bad("N_K count overflow (more than 128 blocks touch one element)");
    int mx = 1;
    for (int v : nk) mx = std::max(mx, v);
    if (gamma <= 0.0) gamma = 1.0 / mx;
    L.nk = nk;
  }
  L.gamma = gamma;
  // colours of the final blocks (multiplicative smoother)
  colour_level(L, fptr, fidx, forig);
  // per final block weight (the multiplicative smoother is undamped)
  std::vector<double> w(nbf, L.ms ? 1.0 : gamma);
  if (!L.omega.empty())
    for (int j = 0; j < nbf; ++j)
      if (forig[j] >= 0) w[j] = L.omega[forig[j]];
  // trivial rows: the DOF's only block is its own singleton
  std::vector<int32_t> trivial(n, -1);
  std::vector<char> general(nbf, 0);
  for (int j = 0; j < nbf; ++j) {
    const int sz = fptr[j + 1] - fptr[j];
    if (sz == 0) continue;
    if (sz == 1 && fcount[fidx[fptr[j]]] == 1) trivial[fidx[fptr[j]]] = j;
    else general[j] = 1;
  }
  // general blocks (all blocks except the trivial singletons): inverse
  // offsets; singletons that share their DOF with another block need 1/A_ii
  std::vector<int32_t> g_blocks, g_size;
  std::vector<int64_t> g_invoff;
  std::vector<double> g_w;
  std::vector<int32_t> single_rows;
  std::vector<int64_t> single_off;
  int64_t extra_off = h_invoff[nf];
  for (int j = 0; j < nbf; ++j) {
    if (!general[j]) continue;
    const int sz = fptr[j + 1] - fptr[j];
    g_blocks.push_back(j);
    g_size.push_back(sz);
    g_w.push_back(w[j]);
    if (finvoff[j] >= 0) {
      g_invoff.push_back(finvoff[j]);
    } else {
      if (sz != 1) bad("internal: unfactorized general block", IMSMG_ERR_HIP);
      g_invoff.push_back(extra_off);
      single_rows.push_back(fidx[fptr[j]]);
      single_off.push_back(extra_off);
      extra_off += 1;
    }
  }
  const int nbg = int(g_blocks.size());
  // inverse storage: factorized inverses followed by general singletons
  double *inv = d_inv;
  if (!single_rows.empty()) {
    inv = dalloc<double>(c->factor_owned, size_t(extra_off));
    HIP_CHECK_RET(hipMemcpyAsync(inv, d_inv, size_t(h_invoff[nf]) * sizeof(double), hipMemcpyDeviceToDevice, s));
    // 1/A_ii through the diag-coefficient kernel with unit weight
    const int ns = int(single_rows.size());
    std::vector<int32_t> tb(n, -1);
    std::vector<double> one(ns, 1.0);
    for (int k = 0; k < ns; ++k) tb[single_rows[k]] = k;
    int32_t *d_tb = dalloc<int32_t>(tmp, n);
    double *d_one = dalloc<double>(tmp, ns), *d_c = dalloc<double>(tmp, n);
    h2d(s, d_tb, tb.data(), n);
    h2d(s, d_one, one.data(), ns);
    launch_diag_coef(s, n, L.K, L.center, d_tb, L.val, d_one, d_c);
    std::vector<double> cvals(n);
    d2h(s, cvals.data(), d_c, n);
    HIP_CHECK_RET(hipStreamSynchronize(s));
    // general singletons occupy one contiguous tail [h_invoff[nf], extra_off)
    std::vector<double> tail(ns);
    for (int k = 0; k < ns; ++k) {
      const double v = cvals[single_rows[k]];
      if (!(v > 0.0) || !std::isfinite(v)) bad("non-positive diagonal entry", IMSMG_ERR_NOT_SPD);
      tail[size_t(single_off[k] - h_invoff[nf])] = v;
    }
    h2d(s, inv + h_invoff[nf], tail.data(), tail.size());
    HIP_CHECK_RET(hipStreamSynchronize(s));
  }
  // weight-dependent part (folding into the inverses, S_G, c): apply_weights
  L.inv = inv;
  L.nbg = nbg;
  L.g_blocks = g_blocks;
  L.g_wcur.assign(nbg, 1.0);
  L.g_off = dalloc<int64_t>(c->factor_owned, std::max(nbg, 1));
  L.g_sz = dalloc<int32_t>(c->factor_owned, std::max(nbg, 1));
  h2d(s, L.g_off, g_invoff.data(), nbg);
  h2d(s, L.g_sz, g_size.data(), nbg);
  // per general row its entries (row a of block j): inverse row offset and
  // block size; the CSR pattern of S_G is the union of the row's block members
  std::vector<int32_t> cnt(n, 0);
  for (int q = 0; q < nbg; ++q) {
    const int j = g_blocks[q];
    for (int k = fptr[j]; k < fptr[j + 1]; ++k) cnt[fidx[k]]++;
  }
  std::vector<int32_t> grows, gp(1, 0), row_slot(n, -1);
  for (int i = 0; i < n; ++i)
    if (cnt[i] > 0) {
      row_slot[i] = int32_t(grows.size());
      grows.push_back(i);
      gp.push_back(gp.back() + cnt[i]);
    }
  const int ngr = int(grows.size());
  std::vector<int64_t> e_off(gp.back());
  std::vector<int32_t> e_n(gp.back()), e_blk(gp.back()), fillp(gp.begin(), gp.end() - 1);
  for (int q = 0; q < nbg; ++q) {  // ascending block order: deterministic summation
    const int j = g_blocks[q];
    const int sz = fptr[j + 1] - fptr[j];
    for (int a = 0; a < sz; ++a) {
      const int i = fidx[fptr[j] + a];
      const int e = fillp[row_slot[i]]++;
      e_off[e] = g_invoff[q] + int64_t(a) * sz;  // row a (= column a) of the symmetric inverse
      e_n[e] = sz;
      e_blk[e] = j;
    }
  }
  std::vector<int32_t> sp(1, 0), scol;
  std::vector<int64_t> e_pos(gp.back());
  std::vector<int32_t> epos;
  {
    std::vector<int32_t> members;
    for (int t = 0; t < ngr; ++t) {
      members.clear();
      for (int e = gp[t]; e < gp[t + 1]; ++e) {
        const int j = e_blk[e];
        for (int k = fptr[j]; k < fptr[j + 1]; ++k) members.push_back(fidx[k]);
      }
      std::sort(members.begin(), members.end());
      members.erase(std::unique(members.begin(), members.end()), members.end());
      const int base = int(scol.size());
      for (int m : members) scol.push_back(L.h_row_lat[m]);
      sp.push_back(int32_t(scol.size()));
      for (int e = gp[t]; e < gp[t + 1]; ++e) {
        const int j = e_blk[e];
        e_pos[e] = int64_t(epos.size());
        for (int k = fptr[j]; k < fptr[j + 1]; ++k) {
          const int pos = int(std::lower_bound(members.begin(), members.end(), fidx[k]) - members.begin());
          epos.push_back(base + pos);
        }
      }
    }
  }
  std::vector<int32_t> grow_lat(ngr);
  for (int t = 0; t < ngr; ++t) {
    grow_lat[t] = L.h_row_lat[grows[t]];
    L.h_meta[grows[t]] |= kMetaGeneral;
  }
  L.ng = ngr;
  L.small = L.n < c->opt.flag_min_rows;
  L.grow_lat = dalloc<int32_t>(c->factor_owned, std::max(ngr, 1));
  L.sptr = dalloc<int32_t>(c->factor_owned, sp.size());
  L.scol = dalloc<int32_t>(c->factor_owned, std::max<size_t>(scol.size(), 1));
  L.sval = dalloc<double>(c->factor_owned, std::max<size_t>(scol.size(), 1));
  h2d(s, L.grow_lat, grow_lat.data(), grow_lat.size());
  h2d(s, L.sptr, sp.data(), sp.size());
  h2d(s, L.scol, scol.data(), scol.size());
  h2d(s, L.meta, L.h_meta.data(), L.h_meta.size());
  L.sg_nnz = std::max<size_t>(scol.size(), 1);
  L.asm_gp = dalloc<int32_t>(c->factor_owned, gp.size());
  L.asm_en = dalloc<int32_t>(c->factor_owned, std::max<size_t>(e_n.size(), 1));
  L.asm_epos = dalloc<int32_t>(c->factor_owned, std::max<size_t>(epos.size(), 1));
  L.asm_eoff = dalloc<int64_t>(c->factor_owned, std::max<size_t>(e_off.size(), 1));
  L.asm_epos0 = dalloc<int64_t>(c->factor_owned, std::max<size_t>(e_pos.size(), 1));
  h2d(s, L.asm_gp, gp.data(), gp.size());
  h2d(s, L.asm_en, e_n.data(), e_n.size());
  h2d(s, L.asm_epos, epos.data(), epos.size());
  h2d(s, L.asm_eoff, e_off.data(), e_off.size());
  h2d(s, L.asm_epos0, e_pos.data(), e_pos.size());
  HIP_CHECK_RET(hipStreamSynchronize(s));
  // patch GEMMs for the multi-column smoother
  L.mb_on = false;
  if (c->opt.block_gemm > 0 && nbg > 0 &&
      std::all_of(g_size.begin(), g_size.end(), [](int32_t z) { return z <= 16; })) {
    std::vector<int32_t> blat(size_t(nbg) * 16, -1), j2q(size_t(nbf), -1), ypos(e_off.size());
    for (int q = 0; q < nbg; ++q) {
      const int j = g_blocks[q];
      j2q[j] = q;
      for (int a = 0; a < fptr[j + 1] - fptr[j]; ++a) blat[size_t(q) * 16 + a] = L.h_row_lat[fidx[fptr[j] + a]];
    }
    for (size_t e = 0; e < e_off.size(); ++e) {
      const int q = j2q[e_blk[e]];
      const int a = int((e_off[e] - g_invoff[q]) / e_n[e]);  // the row's member position in the block
      ypos[e] = q * 256 + a * 16;
    }
    std::vector<int32_t> lp(nbg, 0);
    L.mb_nlp = 0;
    for (int q = 0; q < nbg; ++q) {
      const double *lam = L.f_lam.data() + 4 * size_t(g_blocks[q]);
      lp[q] = (lam[2] > 0.0 && lam[3] <= kBf16Kappa * lam[2]) ? 1 : 0;
      L.mb_nlp += lp[q];
    }
    L.mb_lp = dalloc<int32_t>(c->factor_owned, lp.size());
    h2d(s, L.mb_lp, lp.data(), lp.size());
    L.mb_lat = dalloc<int32_t>(c->factor_owned, blat.size());
    L.mb_yp = dalloc<int32_t>(c->factor_owned, gp.size());
    L.mb_ypos = dalloc<int32_t>(c->factor_owned, std::max<size_t>(ypos.size(), 1));
    L.mb_W = dalloc<double>(c->factor_owned, size_t(nbg) * 256);
    L.mb_Wb = dalloc<uint16_t>(c->factor_owned, size_t(nbg) * 256);
    L.mb_Y = dalloc<double>(c->factor_owned, size_t(nbg) * 256);
    h2d(s, L.mb_lat, blat.data(), blat.size());
    h2d(s, L.mb_yp, gp.data(), gp.size());
    if (!ypos.empty()) h2d(s, L.mb_ypos, ypos.data(), ypos.size());
    HIP_CHECK_RET(hipStreamSynchronize(s));
    L.mb_on = true;
  }
  // trivial rows: c_i = w_j / A_ii (apply_weights)
  std::vector<int32_t> tb(n, -1);
  for (int i = 0; i < n; ++i)
    if (trivial[i] >= 0) tb[i] = trivial[i];
  L.tb = dalloc<int32_t>(c->factor_owned, n);
  L.bw = dalloc<double>(c->factor_owned, std::max(nbf, 1));
  h2d(s, L.tb, tb.data(), n);
  L.c = dalloc<double>(c->factor_owned, n);
  // final blocks for bilinear forms
  {
    std::vector<int32_t> blat(fidx.size());
    for (size_t k = 0; k < fidx.size(); ++k) blat[k] = L.h_row_lat[fidx[k]];
    std::vector<int64_t> boff(nbf, -1);
    std::vector<double> bdiag(nbf, 0.0);
    for (int q = 0; q < nbg; ++q) boff[g_blocks[q]] = g_invoff[q];
    for (int j = 0; j < nbf; ++j)
      if (fptr[j + 1] - fptr[j] == 1) bdiag[j] = 1.0 / diag[fidx[fptr[j]]];
    L.b_ptr = dalloc<int32_t>(c->factor_owned, fptr.size());
    L.b_lat = dalloc<int32_t>(c->factor_owned, std::max<size_t>(blat.size(), 1));
    L.b_off = dalloc<int64_t>(c->factor_owned, std::max(nbf, 1));
    L.b_diag = dalloc<double>(c->factor_owned, std::max(nbf, 1));
    L.b_wfold = dalloc<double>(c->factor_owned, std::max(nbf, 1));
    h2d(s, L.b_ptr, fptr.data(), fptr.size());
    h2d(s, L.b_lat, blat.data(), blat.size());
    h2d(s, L.b_off, boff.data(), nbf);
    h2d(s, L.b_diag, bdiag.data(), nbf);
    HIP_CHECK_RET(hipStreamSynchronize(s));
  }
  L.learned_status = 0;
  L.lambda_max = 0.0;
  apply_weights(c, L, w);
  if (L.ms) build_ms(c, L, fptr, fidx, finvoff, diag, extra_off);
}

// Folds per-final-block weights w into the smoother: rescales the stored
// general-block inverses from their folded weights to w, re-assembles S_G and
// the trivial-row coefficients c_i = w_j / A_ii.
void apply_weights(imsmg_ctx *c, Level &L, const std::vector<double> &w) {
  hipStream_t s = c->stream;
  const int nbf = int(L.f_ptr.size()) - 1;
  if (int(w.size()) != nbf) bad("internal: weight count mismatch", IMSMG_ERR_HIP);
  std::vector<void *> tmp;
  struct TmpFree {
    std::vector<void *> &v;
    ~TmpFree() { free_list(v); }
  } tf{tmp};
  std::vector<double> ratio(std::max(L.nbg, 1), 1.0), wfold(std::max(nbf, 1), 1.0);
  for (int q = 0; q < L.nbg; ++q) {
    const int j = L.g_blocks[q];
    ratio[q] = w[j] / L.g_wcur[q];
    L.g_wcur[q] = w[j];
    wfold[j] = w[j];
  }
  double *d_ratio = dalloc<double>(tmp, ratio.size());
  h2d(s, d_ratio, ratio.data(), ratio.size());
  launch_scale_blocks(s, L.nbg, L.g_off, L.g_sz, d_ratio, L.inv);
  HIP_CHECK_RET(hipMemsetAsync(L.sval, 0, L.sg_nnz * sizeof(double), s));
  launch_assemble_sg(s, L.ng, L.asm_gp, L.asm_eoff, L.asm_en, L.asm_epos0, L.asm_epos, L.inv, L.sval);
  if (L.mb_on) launch_pack_blocks(s, L.nbg, L.g_off, L.g_sz, L.inv, L.mb_W, L.mb_Wb);
  h2d(s, L.bw, w.data(), nbf);
  launch_diag_coef(s, L.n, L.K, L.center, L.tb, L.val, L.bw, L.c);
  h2d(s, L.b_wfold, wfold.data(), nbf);
  HIP_CHECK_RET(hipGetLastError());
  HIP_CHECK_RET(hipStreamSynchronize(s));
  L.f_w = w;
}

// Lanes per row of the general-row product, by measurement on the level's
// own S_G (autotune option): HIP events around a few launches of each
// variant on the library stream (r = the level's residual buffer, x = the
// scratch rh buffer, which every smoothing step rewrites before reading).
void tune_general(imsmg_ctx *c, Level &L) {
  L.gen_lanes = 4;
  if (!c->opt.autotune || L.ng <= 0) return;
  hipStream_t s = c->stream;
  hipEvent_t e0, e1;
  HIP_CHECK_RET(hipEventCreate(&e0));
  HIP_CHECK_RET(hipEventCreate(&e1));
  float best = 0.f;
  for (int lanes : {4, 2, 8}) {
    launch_smooth_general(s, L.ng, L.grow_lat, L.sptr, L.scol, L.sval, L.r, L.rh, c->zero_flag, lanes);
    HIP_CHECK_RET(hipEventRecord(e0, s));
    for (int k = 0; k < 8; ++k)
      launch_smooth_general(s, L.ng, L.grow_lat, L.sptr, L.scol, L.sval, L.r, L.rh, c->zero_flag, lanes);
    HIP_CHECK_RET(hipEventRecord(e1, s));
    HIP_CHECK_RET(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_CHECK_RET(hipEventElapsedTime(&ms, e0, e1));
    if (lanes == 4 || ms < best) {
      best = ms;
      L.gen_lanes = lanes;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_CHECK_RET(hipGetLastError());
}

// ------------------------------------------------------------ per-block damping
// Sixteen scale-free features per final block (the network's inputs); see
// the feature list in include/imsmg.h.
std::vector<float> block_features(imsmg_ctx *c, int l) {
  Level &L = c->lv[l];
  if (L.e_ptr.empty() || L.el_lat.empty() || L.nk.empty())
    bad("block features need the element incidence, element lattice indices and volume fractions");
  const int n = L.n, d = L.dim, p = L.reach;
  const int nbf = int(L.f_ptr.size()) - 1;
  const double K = std::pow(2.0 * p + 1.0, d), E = std::pow(p + 1.0, d);
  const int nel = int(L.e_ptr.size()) - 1;
  constexpr double kCut = 1.0 - 1e-12;
  // function -> active elements (ascending)
  std::vector<int32_t> fp(n + 1, 0), fe(L.e_idx.size());
  for (int32_t f : L.e_idx) fp[f + 1]++;
  for (int i = 0; i < n; ++i) fp[i + 1] += fp[i];
  {
    std::vector<int32_t> fill(fp.begin(), fp.end() - 1);
    for (int e = 0; e < nel; ++e)
      for (int k = L.e_ptr[e]; k < L.e_ptr[e + 1]; ++k) fe[fill[L.e_idx[k]]++] = e;
  }
  std::vector<char> cut_fn(n, 0);
  for (int i = 0; i < n; ++i)
    for (int k = fp[i]; k < fp[i + 1]; ++k)
      if (L.el_eta[fe[k]] < kCut) cut_fn[i] = 1;
  int ncut_level = 0;
  for (double v : L.el_eta) ncut_level += v < kCut;
  const double cut_level = nel > 0 ? double(ncut_level) / nel : 0.0;
  std::vector<float> F(size_t(nbf) * kMlpInputs, 0.0f);
  std::vector<int32_t> S;
  for (int j = 0; j < nbf; ++j) {
    const int jo = L.f_orig[j];
    const int32_t *raw = jo >= 0 ? L.in_idx.data() + L.in_ptr[jo] : L.f_idx.data() + L.f_ptr[j];
    const int nraw = jo >= 0 ? L.in_ptr[jo + 1] - L.in_ptr[jo] : L.f_ptr[j + 1] - L.f_ptr[j];
    const int nfin = L.f_ptr[j + 1] - L.f_ptr[j];
    S.clear();
    for (int a = 0; a < nraw; ++a)
      for (int k = fp[raw[a]]; k < fp[raw[a] + 1]; ++k) S.push_back(fe[k]);
    std::sort(S.begin(), S.end());
    S.erase(std::unique(S.begin(), S.end()), S.end());
    double f[kMlpInputs] = {0.0};
    double sum_eta = 0.0, min_eta = 2.0, sum_log_cut = 0.0, nk_max = 0.0, nk_sum = 0.0;
    double cw[3] = {0, 0, 0}, cu[3] = {0, 0, 0};
    int ncut = 0;
    for (int e : S) {
      const double et = L.el_eta[e];
      sum_eta += et;
      min_eta = std::min(min_eta, et);
      if (et < kCut) {
        sum_log_cut += std::log10(std::max(et, 1e-16));
        ++ncut;
      }
      nk_max = std::max(nk_max, double(L.nk[e]));
      nk_sum += L.nk[e];
      int64_t r = L.el_lat[e];
      for (int a = 0; a < d; ++a) {
        const double m = double(r % L.el_shape[a]);
        r /= L.el_shape[a];
        cw[a] += et * m;
        cu[a] += m;
      }
    }
    const double ns = double(S.size());
    f[0] = nfin / K;
    f[1] = nraw / K;
    f[2] = ns / E;
    f[3] = sum_eta / E;
    f[4] = S.empty() ? 0.0 : std::log10(std::max(min_eta, 1e-16)) / 16.0;
    f[5] = ncut ? sum_log_cut / ncut / 16.0 : 0.0;
    f[6] = nk_max / E;
    f[7] = S.empty() ? 0.0 : nk_sum / ns / E;
    const double *lam = L.f_lam.data() + 4 * size_t(j);
    if (nfin >= 2) f[8] = std::log10(lam[3] / lam[2]) / 16.0;
    f[9] = std::log10(std::max(lam[0] / lam[1], 1e-30)) / 16.0;
    f[10] = jo >= 0 ? (nraw - nfin) / K : 0.0;
    if (nfin > 0) {
      int nc = 0;
      for (int k = L.f_ptr[j]; k < L.f_ptr[j + 1]; ++k) nc += cut_fn[L.f_idx[k]];
      f[11] = double(nc) / nfin;
    }
    if (sum_eta > 0.0)
      for (int a = 0; a < d; ++a) f[12 + a] = (cw[a] / sum_eta - cu[a] / ns) / (p + 1);
    f[15] = cut_level;
    for (int q = 0; q < kMlpInputs; ++q) F[size_t(j) * kMlpInputs + q] = float(f[q]);
  }
  return F;
}

double host_dot(imsmg_ctx *c, Level &L, const double *a, const double *b, double *part) {
  launch_dot_partial(c->stream, L.n, L.row_lat, a, b, part);
  std::vector<double> h(dot_blocks(L.n));
  d2h(c->stream, h.data(), part, h.size());
  HIP_CHECK_RET(hipStreamSynchronize(c->stream));
  double acc = 0.0;
  for (double v : h) acc += v;
  return acc;
}

// y = S x on level L (current weights); y and x padded
void apply_S(imsmg_ctx *c, Level &L, const double *x, double *y) {
  launch_diag_scale(c->stream, L.n, L.row_lat, L.c, x, y, c->zero_flag);
  launch_smooth_general(c->stream, L.ng, L.grow_lat, L.sptr, L.scol, L.sval, x, y, c->zero_flag, L.gen_lanes);
}

// y = A x on level L in FP64 (y, x padded)
void apply_A64(imsmg_ctx *c, Level &L, const double *x, double *y) {
  if (L.csr)
    launch_csr_residual(c->stream, L.n, L.csr_lanes, L.a64, L.meta, x, nullptr, y, c->zero_flag);
  else if (L.ncomp > 1)
    launch_vresidual(c->stream, L.K, L.vops64, L.meta, x, nullptr, y, c->zero_flag);
  else
    launch_residual(c->stream, L.n, L.K, L.op64, L.row_lat, L.meta, x, nullptr, y, c->zero_flag);
}

// Power iteration for lambda_max(S A) with the Rayleigh quotient in the A
// inner product, (A v . S A v) / (A v . v), which increases towards it.
double lambda_max_SA(imsmg_ctx *c, Level &L, int iters) {
  std::vector<void *> tmp;
  struct TmpFree {
    std::vector<void *> &v;
    ~TmpFree() { free_list(v); }
  } tf{tmp};
  double *part = dalloc<double>(tmp, dot_blocks(L.n));
  std::vector<double> v0(L.n);
  for (int i = 0; i < L.n; ++i) v0[i] = 1.0 + 0.5 * std::sin(0.7 * i + 0.3) + 0.25 * std::cos(1.9 * i);
  double *dv = dalloc<double>(tmp, L.n);
  h2d(c->stream, dv, v0.data(), L.n);
  launch_scatter(c->stream, L.n, L.row_lat, dv, L.x);
  double lam = 0.0;
  for (int it = 0; it < iters; ++it) {
    apply_A64(c, L, L.x, L.rh);
    apply_S(c, L, L.rh, L.x2);
    const double ut = host_dot(c, L, L.rh, L.x2, part);
    const double uv = host_dot(c, L, L.rh, L.x, part);
    const double tt = host_dot(c, L, L.x2, L.x2, part);
    if (!(uv > 0.0) || !(tt > 0.0)) bad("stability check: operator not positive", IMSMG_ERR_NOT_SPD);
    lam = ut / uv;
    launch_scale_copy(c->stream, L.n, L.row_lat, 1.0 / std::sqrt(tt), L.x2, L.x);
  }
  HIP_CHECK_RET(hipGetLastError());
  return lam;
}

// Weights of level l from the damping network, omega_j = gamma exp(clip(o_j)),
// kept only if lambda_max(S_omega A) < 2 (1 - 0.05); a first failure rescales
// all of them so that lambda_max lands at 1.8 and checks again; a second
// failure returns to gamma.
constexpr double kSafety = 2.0 * (1.0 - 0.05), kRescaleTarget = 1.8;
void learned_weights(imsmg_ctx *c, int l) {
  Level &L = c->lv[l];
  if (!c->mlp) bad("use_learned needs the damping network (imsmg_load_mlp)", IMSMG_ERR_STATE);
  std::vector<float> F = block_features(c, l);
  const int nbf = int(L.f_ptr.size()) - 1;
  std::vector<void *> tmp;
  struct TmpFree {
    std::vector<void *> &v;
    ~TmpFree() { free_list(v); }
  } tf{tmp};
  float *dX = dalloc<float>(tmp, F.size()), *dout = dalloc<float>(tmp, std::max(nbf, 1));
  h2d(c->stream, dX, F.data(), F.size());
  launch_mlp_forward(c->stream, nbf, c->mlp, dX, dout);
  std::vector<float> o(nbf);
  d2h(c->stream, o.data(), dout, nbf);
  HIP_CHECK_RET(hipStreamSynchronize(c->stream));
  std::vector<double> w(nbf);
  for (int j = 0; j < nbf; ++j) {
    if (!std::isfinite(o[j])) bad("damping network produced a non-finite output", IMSMG_ERR_NAN);
    w[j] = L.gamma * std::exp(std::min(std::max(double(o[j]), -kMlpOutClip), kMlpOutClip));
  }
  apply_weights(c, L, w);
  L.lambda_max = lambda_max_SA(c, L, 60);
  if (!(L.lambda_max < kSafety)) {
    // one rescale towards the bound, then the check again
    const double f = kRescaleTarget / L.lambda_max;
    for (double &v : w) v *= f;
    apply_weights(c, L, w);
    L.lambda_max = lambda_max_SA(c, L, 60);
  }
  if (L.lambda_max < kSafety) {
    L.learned_status = 1;
  } else {
    L.learned_status = -1;
    apply_weights(c, L, std::vector<double>(nbf, L.gamma));
  }
}

bool L_has_no_user_weights(const Level &L) { return L.omega.empty(); }

int pcg_solve_core(imsmg_ctx *c, const double *b_dev, double *x_dev, double rtol, imsmg_info *info);
void destroy_graph(imsmg_ctx *c);

// The uniform smoother as judge of the network's weights: PCG iterations on a
// fixed probe b = A v (x0 = 0, rtol 1e-8), once with gamma on the levels whose
// network weights were kept, once with those weights; the network's weights
// stay only if they need fewer iterations.
void judge_learned(imsmg_ctx *c) {
  std::vector<int> lv_on;
  for (int l = 1; l < int(c->lv.size()); ++l)
    if (c->lv[l].learned_status == 1) lv_on.push_back(l);
  if (lv_on.empty()) return;
  Level &F = c->lv.back();
  const int n = F.n;
  std::vector<void *> tmp;
  struct TmpFree {
    std::vector<void *> &v;
    ~TmpFree() { free_list(v); }
  } tf{tmp};
  std::vector<double> v(n);
  for (int i = 0; i < n; ++i) v[i] = 1.0 + 0.5 * std::sin(0.7 * i + 0.3) + 0.25 * std::cos(1.9 * i);
  double *dv = dalloc<double>(tmp, n), *db = dalloc<double>(tmp, n), *dx = dalloc<double>(tmp, n);
  h2d(c->stream, dv, v.data(), n);
  launch_scatter(c->stream, n, F.row_lat, dv, F.x);
  apply_A64(c, F, F.x, F.rh);
  launch_gather(c->stream, n, F.row_lat, F.rh, db);
  HIP_CHECK_RET(hipStreamSynchronize(c->stream));
  auto iterations = [&]() {
    HIP_CHECK_RET(hipMemsetAsync(dx, 0, size_t(n) * sizeof(double), c->stream));
    imsmg_info info{};
    const int rc = pcg_solve_core(c, db, dx, 1e-8, &info);
    return rc == IMSMG_OK ? info.iterations : (1 << 30);
  };
  std::vector<std::vector<double>> learned(c->lv.size());
  c->factored = true;  // the probe solves run on the factorized hierarchy
  const int it_net = iterations();
  for (int l : lv_on) {
    Level &L = c->lv[l];
    learned[l] = L.f_w;
    apply_weights(c, L, std::vector<double>(L.f_w.size(), L.gamma));
  }
  destroy_graph(c);
  const int it_gamma = iterations();
  destroy_graph(c);
  c->judge_it[0] = it_gamma;
  c->judge_it[1] = it_net;
  if (it_net < it_gamma)
    for (int l : lv_on) apply_weights(c, c->lv[l], learned[l]);
  else
    for (int l : lv_on) c->lv[l].learned_status = -2;
  c->factored = false;
}

// Two-grid objective of level 1 of a two-level hierarchy (see imsmg.h).
void two_grid(imsmg_ctx *c, int m, const double *Z, int k, double *J, double *grad) {
  if (c->lv.size() != 2) bad("the two-grid objective needs a two-level hierarchy");
  if (m < 1 || k < 1 || !Z || !J) bad("bad two-grid arguments");
  Level &L = c->lv[1], &C0 = c->lv[0];
  hipStream_t s = c->stream;
  const int n = L.n, nbf = int(L.f_ptr.size()) - 1;
  std::vector<void *> tmp;
  struct TmpFree {
    std::vector<void *> &v;
    ~TmpFree() { free_list(v); }
  } tf{tmp};
  const size_t vlen = size_t(L.lattice + 2 * L.guard), clen = size_t(C0.lattice + 2 * C0.guard);
  auto vec = [&](size_t len, int64_t guard) {
    double *b = dalloc<double>(tmp, len);
    HIP_CHECK_RET(hipMemsetAsync(b, 0, len * sizeof(double), s));
    return b + guard;
  };
  // a_t = X_{t-1} and c_t = C M a_t for t = 1..k, plus work vectors
  std::vector<double *> av(k + 1), cv(k + 1);
  for (int t = 0; t <= k; ++t) {
    av[t] = vec(vlen, L.guard);
    cv[t] = vec(vlen, L.guard);
  }
  double *u = vec(vlen, L.guard), *w1 = vec(vlen, L.guard), *lam = vec(vlen, L.guard);
  double *nu = vec(vlen, L.guard), *mu = vec(vlen, L.guard);
  double *rc = vec(clen, C0.guard), *xc = vec(clen, C0.guard);
  double *part = dalloc<double>(tmp, dot_blocks(n));
  double *dz = dalloc<double>(tmp, n);
  double *dg = dalloc<double>(tmp, std::max(nbf, 1));
  HIP_CHECK_RET(hipMemsetAsync(dg, 0, std::max(nbf, 1) * sizeof(double), s));
  // energy norm of Z
  double nz = 0.0;
  for (int col = 0; col < m; ++col) {
    h2d(s, dz, Z + size_t(col) * n, n);
    launch_scatter(s, n, L.row_lat, dz, av[0]);
    apply_A64(c, L, av[0], u);
    nz += host_dot(c, L, av[0], u, part);
  }
  if (!(nz > 0.0)) bad("Z must have positive energy");
  // y = (I - S A) x
  auto smooth = [&](const double *x, double *y) {
    apply_A64(c, L, x, u);
    apply_S(c, L, u, y);
    launch_sub_from(s, n, L.row_lat, x, y);
  };
  // y = x - R^T A_0^{-1} R A x   (C)
  auto coarse = [&](const double *x, double *y) {
    apply_A64(c, L, x, u);
    restrict_to(c, L, C0, u, rc, nullptr, c->zero_flag);
    launch_dense_gemv(s, C0.n, C0.row_lat, C0.Ainv, rc, xc, c->zero_flag);
    launch_scale_copy(s, n, L.row_lat, 0.0, x, y);
    prolong_add(c, L, C0, xc, y, c->zero_flag);
    launch_sub_from(s, n, L.row_lat, x, y);
  };
  // y = x - A S x   ((I - S A)^T)
  auto smooth_t = [&](const double *x, double *y) {
    apply_S(c, L, x, u);
    apply_A64(c, L, u, y);
    launch_sub_from(s, n, L.row_lat, x, y);
  };
  // y = x - A R^T A_0^{-1} R x   (C^T)
  auto coarse_t = [&](const double *x, double *y) {
    restrict_to(c, L, C0, x, rc, nullptr, c->zero_flag);
    launch_dense_gemv(s, C0.n, C0.row_lat, C0.Ainv, rc, xc, c->zero_flag);
    launch_scale_copy(s, n, L.row_lat, 0.0, x, w1);
    prolong_add(c, L, C0, xc, w1, c->zero_flag);
    apply_A64(c, L, w1, y);
    launch_sub_from(s, n, L.row_lat, x, y);
  };
  double num = 0.0;
  for (int col = 0; col < m; ++col) {
    h2d(s, dz, Z + size_t(col) * n, n);
    launch_scatter(s, n, L.row_lat, dz, av[0]);
    for (int t = 1; t <= k; ++t) {
      smooth(av[t - 1], w1);
      coarse(w1, cv[t]);
      smooth(cv[t], av[t]);
    }
    apply_A64(c, L, av[k], w1);
    num += host_dot(c, L, av[k], w1, part);
    if (!grad) continue;
    launch_scale_copy(s, n, L.row_lat, 2.0 / nz, w1, lam);
    for (int t = k; t >= 1; --t) {
      // g_j -= <Lambda, A_j^{-1} (A c_t)_j> + <mu, A_j^{-1} (A a_{t-1})_j>
      smooth_t(lam, nu);
      coarse_t(nu, mu);
      double *Ac = w1;
      apply_A64(c, L, cv[t], Ac);
      launch_block_bilinear(s, nbf, L.b_ptr, L.b_lat, L.b_off, L.b_diag, L.b_wfold, L.inv, lam, Ac, -1.0, dg);
      apply_A64(c, L, av[t - 1], Ac);
      launch_block_bilinear(s, nbf, L.b_ptr, L.b_lat, L.b_off, L.b_diag, L.b_wfold, L.inv, mu, Ac, -1.0, dg);
      smooth_t(mu, lam);
    }
  }
  HIP_CHECK_RET(hipGetLastError());
  *J = num / nz;
  if (grad) {
    d2h(s, grad, dg, nbf);
    HIP_CHECK_RET(hipStreamSynchronize(s));
  }
}

void factor_coarsest(imsmg_ctx *c) {
  hipStream_t s = c->stream;
  Level &L = c->lv[0];
  const int n = L.n;
  if (n > 8192) bad("coarsest level larger than 8192 unknowns; use more levels");
  std::vector<void *> tmp;
  struct TmpFree {
    std::vector<void *> &v;
    ~TmpFree() { free_list(v); }
  } tf{tmp};
  L.Ainv = dalloc<double>(c->factor_owned, size_t(n) * n);
  if (L.ncomp > 1) {
    // vector level: the dense operator kept at setup (every component pair)
    HIP_CHECK_RET(hipMemcpyAsync(L.Ainv, L.dense0, size_t(n) * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else if (L.csr) {
    std::vector<double> D(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int k = L.h_aptr[i]; k < L.h_aptr[i + 1]; ++k) D[size_t(i) * n + L.h_acol[k]] = L.h_aval[k];
    h2d(s, L.Ainv, D.data(), D.size());
    HIP_CHECK_RET(hipStreamSynchronize(s));
  } else {
    std::vector<int32_t> lat2c(size_t(L.lattice + 2 * L.guard), -1);
    for (int i = 0; i < n; ++i) lat2c[size_t(L.h_row_lat[i] + L.guard)] = i;
    int32_t *d_l2c = dalloc<int32_t>(tmp, lat2c.size());
    h2d(s, d_l2c, lat2c.data(), lat2c.size());
    HIP_CHECK_RET(hipMemsetAsync(L.Ainv, 0, size_t(n) * n * sizeof(double), s));
    launch_dense_from_ell(s, n, L.K, L.off, L.row_lat, d_l2c + L.guard, L.val, L.Ainv);
  }
  double *colk = dalloc<double>(tmp, n), *rowk = dalloc<double>(tmp, n);
  int32_t *d_bad = dalloc<int32_t>(tmp, 1);
  HIP_CHECK_RET(hipMemsetAsync(d_bad, 0, sizeof(int32_t), s));
  for (int k = 0; k < n; ++k) launch_gauss_jordan_step(s, n, k, L.Ainv, colk, rowk, d_bad);
  HIP_CHECK_RET(hipGetLastError());
  int32_t h_bad = 0;
  HIP_CHECK_RET(hipStreamSynchronize(s));
  HIP_CHECK_RET(hipMemcpy(&h_bad, d_bad, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (h_bad) bad("coarsest operator is not SPD (non-positive Gauss-Jordan pivot)", IMSMG_ERR_NOT_SPD);
  if (c->lv.size() == 1) {  // single level: the "first smoothing step" scaling is zero
    L.c = dalloc<double>(c->factor_owned, n);
    HIP_CHECK_RET(hipMemsetAsync(L.c, 0, size_t(n) * sizeof(double), s));
    HIP_CHECK_RET(hipStreamSynchronize(s));
  }
}

void destroy_graph(imsmg_ctx *c) {
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  if (c->vgraph) {
    (void)hipGraphExecDestroy(c->vgraph);
    c->vgraph = nullptr;
  }
  if (c->mb.graph) {
    (void)hipGraphExecDestroy(c->mb.graph);
    c->mb.graph = nullptr;
  }
  c->graph_iters = 0;
}

// One CG iteration after the initial residual: z = B r, beta, p, q = A p,
// alpha, x, r (the update kernel also prepares c * r for the next V-cycle).
// ------------------------------------------------------------ multi-RHS path
void free_multi(imsmg_ctx *c) {
  if (c->mb.graph) {
    (void)hipGraphExecDestroy(c->mb.graph);
    c->mb.graph = nullptr;
  }
  free_list(c->mb.owned);
  c->mb = imsmg_ctx::Multi{};
}

void ensure_multi(imsmg_ctx *c, int R) {
  if (c->lv.back().ncomp > 1) bad("vector problems: the multi-column form is not supported");
  if (c->lv.back().csr) bad("general sparse levels: the multi-column form is not supported");
  if (c->mb.R == R) return;
  free_multi(c);
  hipStream_t s = c->stream;
  auto &m = c->mb;
  const int nl = int(c->lv.size());
  auto vec = [&](const Level &L) {
    const size_t len = size_t(L.lattice + 2 * L.guard) * R;
    double *b = dalloc<double>(m.owned, len);
    HIP_CHECK_RET(hipMemsetAsync(b, 0, len * sizeof(double), s));
    return b + size_t(L.guard) * R;
  };
  for (int l = 0; l < nl; ++l) {
    const Level &L = c->lv[l];
    m.r.push_back(vec(L));
    m.x.push_back(vec(L));
    m.x2.push_back(vec(L));
    m.rh.push_back(vec(L));
    m.xs.push_back(((c->opt.nu_pre - 1 + c->opt.nu_post) % 2) ? m.x2.back() : m.x.back());
  }
  const Level &F = c->lv.back();
  m.p = vec(F);
  m.q = vec(F);
  m.xsol = vec(F);
  m.bs = vec(F);
  m.part = dalloc<double>(m.owned, multi_part_size(R, F.n, F.op64.ntiles));
  m.st = dalloc<MState>(m.owned, 1);
  HIP_CHECK_RET(hipMemsetAsync(m.st, 0, sizeof(MState), s));
  HIP_CHECK_RET(hipStreamSynchronize(s));
  m.R = R;
}

// x += S_G r on the general rows of the multi-column vectors: the assembled
// CSR product, or the blocks' patch GEMMs on the matrix cores (block_gemm)
void m_general(imsmg_ctx *c, Level &L, const double *r, double *x, const int32_t *done) {
  auto &m = c->mb;
  if (L.mb_on) {
    launch_m_block_gemm(c->stream, c->opt.block_gemm == 2, L.nbg, m.R, L.mb_lat, L.mb_W, L.mb_Wb, L.mb_lp, r, L.mb_Y,
                        done);
    launch_m_block_gather(c->stream, m.R, L.ng, L.grow_lat, L.mb_yp, L.mb_ypos, L.mb_Y, x, done);
  } else {
    launch_m_smooth_general(c->stream, m.R, L.ng, L.grow_lat, L.sptr, L.scol, L.sval, r, x, done);
  }
}

void m_smooth_step(imsmg_ctx *c, int l, const double *xa, double *xb, const int32_t *done) {
  Level &L = c->lv[l];
  auto &m = c->mb;
  if (mixed(c))
    launch_m_residual_smooth(c->stream, m.R, L.n, L.K, L.op32, L.row_lat, L.meta, L.c, xa, m.r[l], m.rh[l], xb, done);
  else
    launch_m_residual_smooth(c->stream, m.R, L.n, L.K, L.op64, L.row_lat, L.meta, L.c, xa, m.r[l], m.rh[l], xb, done);
  m_general(c, L, m.rh[l], xb, done);
}

void m_vcycle_level(imsmg_ctx *c, int l, const int32_t *done_top) {
  Level &L = c->lv[l];
  auto &m = c->mb;
  const int R = m.R;
  hipStream_t s = c->stream;
  const int32_t *done = flag_for(c, L, done_top);
  if (l == 0) {
    launch_m_dense_gemm(s, R, L.n, L.row_lat, L.Ainv, m.r[0], m.x[0], done);
    return;
  }
  Level &Cl = c->lv[l - 1];
  m_general(c, L, m.r[l], m.xs[l], done);
  double *xa = m.xs[l], *xb = (m.xs[l] == m.x[l]) ? m.x2[l] : m.x[l];
  for (int k = 1; k < c->opt.nu_pre; ++k) {
    m_smooth_step(c, l, xa, xb, done);
    std::swap(xa, xb);
  }
  if (mixed(c))
    launch_m_residual(s, R, L.n, L.K, L.op32, L.row_lat, L.meta, xa, m.r[l], m.rh[l], done);
  else
    launch_m_residual(s, R, L.n, L.K, L.op64, L.row_lat, L.meta, xa, m.r[l], m.rh[l], done);
  const double *ci = l - 1 > 0 ? Cl.c : nullptr;
  double *xinit = l - 1 > 0 ? m.xs[l - 1] : nullptr;
  const int32_t *cdone = flag_for(c, Cl, done_top);
  if (L.tensor)
    launch_m_tensor_transfer(s, R, L.dim, Cl.n, Cl.row_lat, Cl.shape[0], Cl.shape[1], L.rb_start, L.rb_len,
                             L.rb_coef, L.rbW, L.shape[0], L.shape[1], m.rh[l], m.r[l - 1], 0, ci, xinit, cdone);
  else
    launch_m_ell_gather(s, R, Cl.n, L.rw, Cl.row_lat, L.rcol, L.rval, m.rh[l], m.r[l - 1], 0, ci, xinit, cdone);
  m_vcycle_level(c, l - 1, done_top);
  if (L.tensor)
    launch_m_tensor_transfer(s, R, L.dim, L.n, L.row_lat, L.shape[0], L.shape[1], L.pb_start, L.pb_len, L.pb_coef,
                             L.pbW, Cl.shape[0], Cl.shape[1], m.x[l - 1], xa, 1, nullptr, nullptr, done);
  else
    launch_m_ell_gather(s, R, L.n, L.tw, L.row_lat, L.tcol, L.tval, m.x[l - 1], xa, 1, nullptr, nullptr, done);
  for (int k = 0; k < c->opt.nu_post; ++k) {
    m_smooth_step(c, l, xa, xb, done);
    std::swap(xa, xb);
  }
}

void m_cg_iteration(imsmg_ctx *c) {
  Level &F = c->lv.back();
  auto &m = c->mb;
  const int f = int(c->lv.size()) - 1;
  const int32_t *done = &m.st->done;
  hipStream_t s = c->stream;
  m_vcycle_level(c, f, done);
  launch_mcg_dot_rz(s, m.R, F.n, F.row_lat, m.r[f], m.x[f], m.part, m.st);
  launch_mcg_direction(s, m.R, F.n, F.row_lat, m.x[f], m.p, m.st);
  launch_mcg_spmv_pq(s, m.R, F.n, F.K, F.op64, F.row_lat, F.meta, m.p, m.q, m.part, m.st);
  launch_mcg_update(s, m.R, F.n, F.row_lat, m.p, m.q, m.xsol, m.r[f], F.c, m.xs[f], m.part, m.st, c->opt.max_iter);
}

int rhs_width(int nrhs) {
  if (nrhs < 1 || nrhs > kMaxRhs) bad("nrhs must be 1 .. 16");
  return nrhs <= 4 ? 4 : nrhs <= 8 ? 8 : 16;
}

void cg_iteration(imsmg_ctx *c, bool timing) {
  Level &F = c->lv.back();
  const int32_t *done = &c->st->done;
  vcycle_level(c, int(c->lv.size()) - 1, done, timing);
  launch_cg_dot_rz(c->stream, F.n, F.row_lat, F.r, F.x, c->part, c->st, c->opt.flexible_cg);
  launch_cg_direction(c->stream, F.n, F.row_lat, F.x, c->p, c->st);
  if (F.csr)
    launch_csr_cg_spmv_pq(c->stream, F.n, F.csr_lanes, F.a64, c->p, c->q, c->part, c->st);
  else if (F.ncomp > 1)
    launch_vcg_spmv_pq(c->stream, F.K, F.vops64, F.meta, c->p, c->q, c->part, c->st);
  else
    launch_cg_spmv_pq(c->stream, F.n, F.K, F.op64, F.row_lat, F.meta, c->p, c->q, c->part, c->st);
  // z_k = F.x until the next V-cycle (F.xs may be the same buffer)
  launch_cg_update(c->stream, F.n, F.row_lat, c->p, c->q, c->xs, F.r, F.c, F.xs, c->opt.flexible_cg ? F.x : nullptr,
                   c->part, c->st, c->opt.max_iter);
}

// info fields shared by every solve: restarts, fallback flags, setup/factor times
void fill_info_common(const imsmg_ctx *c, imsmg_info *info, int restarts) {
  info->restarts = restarts;
  int flags = 0;
  for (size_t l = 1; l < c->lv.size() && l < 31; ++l)
    if (c->lv[l].learned_status < 0) flags |= 1 << l;
  info->fallback_flags = flags;
  info->setup_ms = c->setup_ms;
  info->factor_ms = c->factor_ms;
}

// CG preconditioned by the V-cycle (imsmg_pcg_solve without the error guard)
int pcg_solve_core(imsmg_ctx *c, const double *b_dev, double *x_dev, double rtol, imsmg_info *info) {
  {
    if (!c->factored) bad("factor first", IMSMG_ERR_STATE);
    if (!b_dev || !x_dev) bad("null vector");
    if (!(rtol > 0.0)) bad("rtol must be positive");
    auto t0 = std::chrono::steady_clock::now();
    Level &F = c->lv.back();
    hipStream_t s = c->stream;
    const bool timing = c->opt.timing != 0;
    launch_scatter(s, F.n, F.row_lat, b_dev, c->bs);
    launch_scatter(s, F.n, F.row_lat, x_dev, c->xs);
    CGState h{};
    int restarts = 0;
    while (true) {
      if (F.csr)
        launch_csr_cg_init(s, F.n, F.csr_lanes, F.a64, c->xs, c->bs, F.r, c->part, c->st, rtol, restarts > 0);
      else if (F.ncomp > 1)
        launch_vcg_init(s, F.K, F.vops64, F.meta, c->xs, c->bs, F.r, c->part, c->st, rtol, restarts > 0);
      else
        launch_cg_init(s, F.n, F.K, F.op64, F.row_lat, F.meta, c->xs, c->bs, F.r, c->part, c->st, rtol,
                       restarts > 0);
      launch_diag_scale(s, F.n, F.row_lat, F.c, F.r, F.xs, &c->st->done);
      HIP_CHECK_RET(hipGetLastError());
      const int m = c->opt.check_every;
      const bool graph = c->opt.use_graph && !timing;
      if (graph && !c->graph) {
        hipGraph_t g = nullptr;
        HIP_CHECK_RET(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < m; ++k) cg_iteration(c, false);
        HIP_CHECK_RET(hipStreamEndCapture(s, &g));
        hipError_t e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIP_CHECK_RET(e);
        c->graph_iters = m;
      }
      while (true) {
        if (graph) {
          HIP_CHECK_RET(hipGraphLaunch(c->graph, s));
        } else {
          for (int k = 0; k < m; ++k) cg_iteration(c, timing);
        }
        HIP_CHECK_RET(hipGetLastError());
        HIP_CHECK_RET(hipMemcpyAsync(&h, c->st, sizeof(CGState), hipMemcpyDeviceToHost, s));
        HIP_CHECK_RET(hipStreamSynchronize(s));
        if (timing) collect_timing(c);
        if (h.done) break;
      }
      // true residual ||b - A x|| / ||b||
      if (F.csr)
        launch_csr_cg_true_residual(s, F.n, F.csr_lanes, F.a64, c->xs, c->bs, c->part, c->st);
      else if (F.ncomp > 1)
        launch_vcg_true_residual(s, F.K, F.vops64, F.meta, c->xs, c->bs, c->part, c->st);
      else
        launch_cg_true_residual(s, F.n, F.K, F.op64, F.row_lat, F.meta, c->xs, c->bs, c->part, c->st);
      HIP_CHECK_RET(hipMemcpyAsync(&h, c->st, sizeof(CGState), hipMemcpyDeviceToHost, s));
      HIP_CHECK_RET(hipStreamSynchronize(s));
      const double true_rel = h.bb > 0.0 ? std::sqrt(h.aux / h.bb) : 0.0;
      if (h.status == 0 && true_rel > rtol && restarts < 3 && h.iters < c->opt.max_iter) {
        ++restarts;  // recursive residual drifted: restart from the current x
        continue;
      }
      launch_gather(s, F.n, F.row_lat, c->xs, x_dev);
      HIP_CHECK_RET(hipStreamSynchronize(s));
      // the solve's criterion is the true relative residual: a solve that ends
      // above rtol (restarts used up, or max_iter reached) has not converged
      if (h.status == 0 && true_rel > rtol) h.status = IMSMG_ERR_NOT_CONVERGED;
      if (info) {
        fill_info_common(c, info, restarts);
        info->status = h.status;
        info->iterations = h.iters;
        info->rel_res = h.r0sq > 0.0 ? std::sqrt(h.rr / h.r0sq) : 0.0;
        info->true_rel_res = true_rel;
        info->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      }
      if (h.status != 0) {
        c->err = h.status == IMSMG_ERR_NOT_CONVERGED ? "CG did not reach rtol (true relative residual)"
                 : h.status == IMSMG_ERR_NOT_SPD     ? "CG breakdown: p.Ap <= 0"
                                                     : "NaN or Inf in the CG iteration";
        return int(h.status);
      }
      return IMSMG_OK;
    }
  }
}

}  // namespace

extern "C" {

void imsmg_default_options(imsmg_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = IMSMG_FP64;
  o->nu_pre = 1;
  o->nu_post = 1;
  o->max_iter = 500;
  o->check_every = 4;
  o->use_graph = 1;
  o->timing = 0;
  o->gamma = 0.0;
  o->compress = 1;
  o->smoother = IMSMG_ADDITIVE;
  o->coarse_smoother = -1;
  o->cycle = 1;
  o->flag_min_rows = kSmallLevel;
  o->ncomp = 1;
}

int imsmg_create(imsmg_ctx **out, int device, void *stream) {
  if (!out) return IMSMG_ERR_INVALID_ARG;
  *out = nullptr;
  imsmg_ctx *c = nullptr;
  try {
    c = new imsmg_ctx();
  } catch (...) {
    return IMSMG_ERR_OOM;
  }
  c->device = device;
  imsmg_default_options(&c->opt);
  int rc = guarded(c, [&]() {
    int ndev = 0;
    HIP_CHECK_RET(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) bad("no such device");
    if (stream) {
      c->stream = static_cast<hipStream_t>(stream);
    } else {
      HIP_CHECK_RET(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
    return IMSMG_OK;
  });
  if (rc != IMSMG_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return IMSMG_OK;
}

int imsmg_setup(imsmg_ctx *c, int nlevels, const imsmg_csr *A, const imsmg_csr *R, const imsmg_patches *P,
                const imsmg_lattice *Lt, const imsmg_elements *E, const imsmg_options *opt) {
  return guarded(c, [&]() -> int {
    const auto t_setup0 = std::chrono::steady_clock::now();
    if (nlevels < 1 || nlevels > 16 || !A || !Lt) bad("bad level count or null arrays");
    if (nlevels > 1 && (!R || !P)) bad("R and P are required with more than one level");
    destroy_graph(c);
    free_multi(c);
    free_list(c->factor_owned);
    free_list(c->owned);
    c->lv.clear();
    c->ready = c->factored = false;
    if (opt) c->opt = *opt;
    if (c->opt.nu_pre < 1 || c->opt.nu_post < 1 || c->opt.max_iter < 1) bad("nu and max_iter must be >= 1");
    if (c->opt.check_every < 1) c->opt.check_every = 1;
    if (c->opt.precision != IMSMG_FP64 && c->opt.precision != IMSMG_MIXED) bad("unknown precision mode");
    if (c->opt.block_gemm < 0 || c->opt.block_gemm > 2) bad("block_gemm must be 0, 1 or 2");
    if (c->opt.timing < 0 || c->opt.timing > 64) bad("timing must be 0 .. 64");
    if (c->opt.flexible_cg != 0 && c->opt.flexible_cg != 1) bad("flexible_cg must be 0 or 1");
    if (c->opt.smoother != IMSMG_ADDITIVE && c->opt.smoother != IMSMG_MULTIPLICATIVE) bad("unknown smoother");
    if (c->opt.coarse_smoother < -1 || c->opt.coarse_smoother > IMSMG_MULTIPLICATIVE) bad("unknown coarse_smoother");
    if (c->opt.cycle != 1 && c->opt.cycle != 2) bad("cycle must be 1 (V) or 2 (W)");
    if (c->opt.flag_min_rows < 0) bad("flag_min_rows must be >= 0");
    if (c->opt.use_learned < 0 || c->opt.use_learned > 2) bad("use_learned must be 0, 1 or 2");
    if (c->opt.use_learned && uses_ms(c->opt, nlevels)) bad("use_learned needs the additive smoother on every level");
    if (c->opt.ncomp != 1 && c->opt.ncomp != kMaxComp) bad("ncomp must be 1 or 3");
    if (c->opt.ncomp > 1) {
      if (Lt[nlevels - 1].dim != 3) bad("vector problems (ncomp 3) need a 3D lattice");
      if (c->opt.use_learned) bad("vector problems: learned weights are not supported");
      if (c->opt.block_gemm) bad("vector problems: block_gemm is not supported");
    }
    int ncsr = 0;
    for (int l = 0; l < nlevels; ++l) ncsr += Lt[l].dof_to_lattice == nullptr;
    if (ncsr) {
      // general sparse levels (no function lattice)
      if (ncsr != nlevels) bad("either every level has a function lattice or none has");
      if (c->opt.use_learned) bad("general sparse levels: learned weights are not supported");
      if (c->opt.block_gemm) bad("general sparse levels: block_gemm is not supported");
      for (int l = 1; l < nlevels; ++l)
        if (Lt[l].two_scale) bad("general sparse levels take R as CSR only (no two_scale)");
    }
    c->lv.resize(nlevels);
    for (int l = 0; l < nlevels; ++l) {
      if (!ncsr && Lt[l].dim != Lt[nlevels - 1].dim) bad("all levels must share the dimension");
      setup_level(c, c->lv[l], A[l], Lt[l]);
    }
    if (c->opt.ncomp > 1) {
      // the coarsest vector operator as a dense matrix (every component pair)
      Level &C0 = c->lv[0];
      const int n0 = C0.n;
      if (n0 > 8192) bad("coarsest level larger than 8192 unknowns; use more levels");
      std::vector<double> D(size_t(n0) * n0, 0.0);
      for (int i = 0; i < n0; ++i)
        for (int64_t k = A[0].rowptr[i]; k < A[0].rowptr[i + 1]; ++k) D[size_t(i) * n0 + A[0].col[k]] = A[0].val[k];
      C0.dense0 = dalloc<double>(c->owned, D.size());
      h2d(c->stream, C0.dense0, D.data(), D.size());
      HIP_CHECK_RET(hipStreamSynchronize(c->stream));
    }
    for (int l = 1; l < nlevels; ++l) setup_transfer(c, c->lv[l], c->lv[l - 1], R[l], Lt[l].two_scale);
    for (int l = 1; l < nlevels; ++l) {
      Level &L = c->lv[l];
      const imsmg_patches &p = P[l];
      if (p.nblocks < 0 || (p.nblocks > 0 && (!p.ptr || !p.idx))) bad("bad patch arrays");
      L.in_ptr.assign(p.ptr, p.ptr + p.nblocks + 1);
      if (L.in_ptr[0] != 0) bad("patch ptr must start at 0");
      for (int j = 0; j < p.nblocks; ++j)
        if (L.in_ptr[j + 1] < L.in_ptr[j]) bad("patch ptr must be non-decreasing");
      L.in_idx.assign(p.idx, p.idx + L.in_ptr[p.nblocks]);
      L.in_colour.clear();
      if (p.colour) {
        L.in_colour.assign(p.colour, p.colour + p.nblocks);
        for (int32_t v : L.in_colour)
          if (v < 0 || v >= kMaxColours) bad("block colours must lie in [0, " + std::to_string(kMaxColours) + ")");
      }
      L.ms = level_ms(c->opt, l, nlevels);
      for (int j = 0; j < p.nblocks; ++j)
        for (int k = L.in_ptr[j]; k < L.in_ptr[j + 1]; ++k) {
          if (L.in_idx[k] < 0 || L.in_idx[k] >= L.n) bad("patch index out of range");
          if (k > L.in_ptr[j] && L.in_idx[k] <= L.in_idx[k - 1]) bad("patch indices must be sorted and unique");
          if (L.in_idx[k] / L.ns != L.in_idx[L.in_ptr[j]] / L.ns)
            bad("vector problems: every Schwarz block must hold DOFs of one component");
        }
      if (E) {
        const imsmg_elements &e = E[l];
        if (e.nelements < 0 || (e.nelements > 0 && (!e.eptr || !e.eidx))) bad("bad element arrays");
        L.e_ptr.assign(e.eptr, e.eptr + e.nelements + 1);
        L.e_idx.assign(e.eidx, e.eidx + L.e_ptr.back());
        for (int32_t f : L.e_idx)
          if (f < 0 || f >= L.n) bad("element function index out of range");
        L.el_lat.clear();
        L.el_eta.assign(e.nelements, 1.0);
        if (e.elem) {
          int64_t tot = 1;
          for (int a = 0; a < L.dim; ++a) {
            if (e.shape[a] < 1) bad("element shape must be positive");
            L.el_shape[a] = e.shape[a];
            tot *= e.shape[a];
          }
          L.el_lat.assign(e.elem, e.elem + e.nelements);
          for (int32_t v : L.el_lat)
            if (v < 0 || v >= tot) bad("element lattice index out of range");
        }
        if (e.eta) {
          L.el_eta.assign(e.eta, e.eta + e.nelements);
          for (double v : L.el_eta)
            if (!(v >= 0.0 && v <= 1.0 + 1e-9)) bad("volume fractions must lie in [0, 1]");
        }
      }
    }
    Level &F = c->lv.back();
    const size_t vlen = size_t(F.ncomp * F.cstride);
    double *vv[4];
    for (int k = 0; k < 4; ++k) {
      vv[k] = dalloc<double>(c->owned, vlen);
      HIP_CHECK_RET(hipMemsetAsync(vv[k], 0, vlen * sizeof(double), c->stream));
    }
    c->p = vv[0] + F.guard;
    c->q = vv[1] + F.guard;
    c->xs = vv[2] + F.guard;
    c->bs = vv[3] + F.guard;
    c->c_in = dalloc<double>(c->owned, F.n);
    c->c_out = dalloc<double>(c->owned, F.n);
    c->zero_flag = dalloc<int32_t>(c->owned, 1);
    HIP_CHECK_RET(hipMemsetAsync(c->zero_flag, 0, sizeof(int32_t), c->stream));
    c->st = dalloc<CGState>(c->owned, 1);
    HIP_CHECK_RET(hipMemsetAsync(c->st, 0, sizeof(CGState), c->stream));
    c->part = dalloc<double>(c->owned, 2 * size_t(std::max({reduction_blocks(F.n), F.op64.ntiles * F.ncomp,
                                                               F.csr ? csr_part_blocks(F.n, F.csr_lanes) : 0})) + 64);
    HIP_CHECK_RET(hipStreamSynchronize(c->stream));
    c->ready = true;
    c->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_setup0).count();
    return IMSMG_OK;
  });
}

int imsmg_set_patch_weights(imsmg_ctx *c, int level, const double *omega) {
  return guarded(c, [&]() -> int {
    if (!c->ready) bad("setup first", IMSMG_ERR_STATE);
    if (level < 1 || level >= int(c->lv.size()) || !omega) bad("bad level or null weights");
    Level &L = c->lv[level];
    if (L.ms) bad("per-block weights apply to the additive smoother only");
    const int nb = int(L.in_ptr.size()) - 1;
    for (int j = 0; j < nb; ++j)
      if (!(omega[j] > 0.0) || !std::isfinite(omega[j])) bad("weights must be positive and finite");
    L.omega.assign(omega, omega + nb);
    c->factored = false;
    return IMSMG_OK;
  });
}

int imsmg_factor_patches(imsmg_ctx *c) {
  if (c && !c->batch.empty()) {  // batch context: every problem in turn
    for (size_t p = 0; p < c->batch.size(); ++p) {
      const int rc = imsmg_factor_patches(c->batch[p]);
      if (rc != IMSMG_OK) return fail(c, rc, "problem " + std::to_string(p) + ": " + c->batch[p]->err);
    }
    c->err.clear();
    return IMSMG_OK;
  }
  return guarded(c, [&]() -> int {
    if (!c->ready) bad("setup first", IMSMG_ERR_STATE);
    const auto t_factor0 = std::chrono::steady_clock::now();
    destroy_graph(c);
    free_list(c->factor_owned);
    c->factored = false;
    for (int l = 1; l < int(c->lv.size()); ++l) factor_level(c, l);
    factor_coarsest(c);
    if (c->opt.use_learned) {
      for (int l = 1; l < int(c->lv.size()); ++l)
        if (L_has_no_user_weights(c->lv[l])) learned_weights(c, l);
      if (c->opt.use_learned == 1) judge_learned(c);
    }
    for (int l = 1; l < int(c->lv.size()); ++l) tune_general(c, c->lv[l]);
    c->factored = true;
    c->factor_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_factor0).count();
    return IMSMG_OK;
  });
}

int imsmg_get_patches(imsmg_ctx *c, int level, int32_t *nblocks, int64_t *nnz, int32_t *ptr, int32_t *idx) {
  return guarded(c, [&]() -> int {
    if (!c->factored) bad("factor first", IMSMG_ERR_STATE);
    if (level < 1 || level >= int(c->lv.size())) bad("bad level");
    const Level &L = c->lv[level];
    if (nblocks) *nblocks = int32_t(L.f_ptr.size()) - 1;
    if (nnz) *nnz = int64_t(L.f_idx.size());
    if (ptr) std::copy(L.f_ptr.begin(), L.f_ptr.end(), ptr);
    if (idx) std::copy(L.f_idx.begin(), L.f_idx.end(), idx);
    return IMSMG_OK;
  });
}

int imsmg_get_patch_colours(imsmg_ctx *c, int level, int32_t *ncolours, int32_t *colour) {
  return guarded(c, [&]() -> int {
    if (!c->factored) bad("factor first", IMSMG_ERR_STATE);
    if (level < 1 || level >= int(c->lv.size())) bad("bad level");
    const Level &L = c->lv[level];
    if (ncolours) *ncolours = L.ncolours;
    if (colour) std::copy(L.f_colour.begin(), L.f_colour.end(), colour);
    return IMSMG_OK;
  });
}

int imsmg_get_gamma(imsmg_ctx *c, int level, double *gamma) {
  return guarded(c, [&]() -> int {
    if (!c->factored) bad("factor first", IMSMG_ERR_STATE);
    if (level < 1 || level >= int(c->lv.size()) || !gamma) bad("bad level");
    *gamma = c->lv[level].gamma;
    return IMSMG_OK;
  });
}

// The launches of one V-cycle from the staged compact residual c_in to the
// compact correction c_out (captured once per factorization when graphs are
// on; the caller's vectors are copied in and out around it).
void vcycle_body(imsmg_ctx *c, bool timing) {
  Level &F = c->lv.back();
  launch_scatter(c->stream, F.n, F.row_lat, c->c_in, F.r);
  launch_diag_scale(c->stream, F.n, F.row_lat, F.c, F.r, F.xs, c->zero_flag);
  vcycle_level(c, int(c->lv.size()) - 1, c->zero_flag, timing);
  launch_gather(c->stream, F.n, F.row_lat, F.x, c->c_out);
}

// Runs one V-cycle on c_in (graph replay when graphs are on and no kernel is
// timed); returns without synchronizing.
void vcycle_launch(imsmg_ctx *c) {
  const bool timing = c->opt.timing != 0;
  if (c->opt.use_graph && !timing) {
    if (!c->vgraph) {
      hipGraph_t g = nullptr;
      HIP_CHECK_RET(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      vcycle_body(c, false);
      HIP_CHECK_RET(hipStreamEndCapture(c->stream, &g));
      hipError_t e = hipGraphInstantiate(&c->vgraph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIP_CHECK_RET(e);
    }
    HIP_CHECK_RET(hipGraphLaunch(c->vgraph, c->stream));
  } else {
    vcycle_body(c, timing);
  }
}

int imsmg_vcycle(imsmg_ctx *c, const double *r_dev, double *z_dev) {
  return guarded(c, [&]() -> int {
    if (!c->factored) bad("factor first", IMSMG_ERR_STATE);
    if (!r_dev || !z_dev) bad("null vector");
    Level &F = c->lv.back();
    HIP_CHECK_RET(hipMemcpyAsync(c->c_in, r_dev, size_t(F.n) * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    vcycle_launch(c);
    HIP_CHECK_RET(hipMemcpyAsync(z_dev, c->c_out, size_t(F.n) * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIP_CHECK_RET(hipGetLastError());
    HIP_CHECK_RET(hipStreamSynchronize(c->stream));
    if (c->opt.timing) collect_timing(c);
    return IMSMG_OK;
  });
}

int imsmg_vcycle_time(imsmg_ctx *c, const double *r_dev, int reps, double *median_ms, double *mean_ms) {
  return guarded(c, [&]() -> int {
    if (!c->factored) bad("factor first", IMSMG_ERR_STATE);
    if (!r_dev || reps < 1 || reps > 100000) bad("bad V-cycle timing arguments");
    if (c->opt.timing) bad("imsmg_vcycle_time needs opt.timing = 0");
    Level &F = c->lv.back();
    HIP_CHECK_RET(hipMemcpyAsync(c->c_in, r_dev, size_t(F.n) * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    vcycle_launch(c);  // warm (and capture)
    std::vector<hipEvent_t> ev(2 * size_t(reps));
    for (auto &e : ev) HIP_CHECK_RET(hipEventCreate(&e));
    struct EvFree {
      std::vector<hipEvent_t> &v;
      ~EvFree() {
        for (auto e : v) (void)hipEventDestroy(e);
      }
    } ef{ev};
    for (int k = 0; k < reps; ++k) {
      HIP_CHECK_RET(hipEventRecord(ev[2 * k], c->stream));
      vcycle_launch(c);
      HIP_CHECK_RET(hipEventRecord(ev[2 * k + 1], c->stream));
    }
    HIP_CHECK_RET(hipStreamSynchronize(c->stream));
    std::vector<double> t(reps);
    double sum = 0.0;
    for (int k = 0; k < reps; ++k) {
      float ms = 0.f;
      HIP_CHECK_RET(hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]));
      t[k] = ms;
      sum += ms;
    }
    std::sort(t.begin(), t.end());
    if (median_ms) *median_ms = reps % 2 ? t[reps / 2] : 0.5 * (t[reps / 2 - 1] + t[reps / 2]);
    if (mean_ms) *mean_ms = sum / reps;
    return IMSMG_OK;
  });
}

int imsmg_pcg_solve(imsmg_ctx *c, const double *b_dev, double *x_dev, double rtol, imsmg_info *info) {
  return guarded(c, [&]() -> int { return pcg_solve_core(c, b_dev, x_dev, rtol, info); });
}

namespace {

// Full multigrid into c->xs from c->bs: the right-hand side restricted to
// every level, the coarsest level solved directly, then on every finer level
// the prolongated coarser solution improved by one cycle of that level.
void fmg_pass(imsmg_ctx *c) {
  hipStream_t s = c->stream;
  const int nl = int(c->lv.size());
  for (Level &L : c->lv)
    if (!L.fmg_b) {
      const size_t vlen = size_t(L.ncomp * L.cstride);
      double *v[2];
      for (int k = 0; k < 2; ++k) {
        double *b = dalloc<double>(c->owned, vlen);
        HIP_CHECK_RET(hipMemsetAsync(b, 0, vlen * sizeof(double), s));
        v[k] = b + L.guard;
      }
      L.fmg_b = v[0];
      L.fmg_x = v[1];
    }
  Level &F = c->lv.back();
  launch_rows_op(s, F.n, F.row_lat, c->bs, F.fmg_b, 1, nullptr);
  for (int l = nl - 1; l > 0; --l) restrict_to(c, c->lv[l], c->lv[l - 1], c->lv[l].fmg_b, c->lv[l - 1].fmg_b, nullptr,
                                               nullptr);
  Level &C0 = c->lv[0];
  launch_dense_gemv(s, C0.n, C0.row_lat, C0.Ainv, C0.fmg_b, C0.fmg_x, nullptr);
  for (int l = 1; l < nl; ++l) {
    Level &L = c->lv[l];
    launch_rows_op(s, L.n, L.row_lat, nullptr, L.fmg_x, 0, nullptr);
    prolong_add(c, L, c->lv[l - 1], c->lv[l - 1].fmg_x, L.fmg_x, nullptr);
    residual(c, L, L.fmg_x, L.fmg_b, L.r, nullptr, false);
    if (!L.ms) launch_diag_scale(s, L.n, L.row_lat, L.c, L.r, L.xs, nullptr);
    vcycle_level(c, l, c->zero_flag, false);
    launch_rows_op(s, L.n, L.row_lat, L.x, L.fmg_x, 2, nullptr);
  }
  launch_rows_op(s, F.n, F.row_lat, F.fmg_x, c->xs, 1, nullptr);
  HIP_CHECK_RET(hipGetLastError());
}

}  // namespace

int imsmg_mg_solve(imsmg_ctx *c, const double *b_dev, double *x_dev, double rtol, int max_cycles, int fmg,
                   imsmg_info *info) {
  return guarded(c, [&]() -> int {
    if (!c->factored) bad("factor first", IMSMG_ERR_STATE);
    if (!b_dev || !x_dev) bad("null vector");
    if (!(rtol > 0.0) || max_cycles < 0) bad("rtol must be positive and max_cycles >= 0");
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = c->stream;
    Level &F = c->lv.back();
    std::vector<void *> tmp;
    struct TmpFree {
      std::vector<void *> &v;
      ~TmpFree() { free_list(v); }
    } tf{tmp};
    double *part = dalloc<double>(tmp, dot_blocks(F.n));
    launch_scatter(s, F.n, F.row_lat, b_dev, c->bs);
    if (fmg)
      fmg_pass(c);
    else
      launch_scatter(s, F.n, F.row_lat, x_dev, c->xs);
    const double bn = std::sqrt(host_dot(c, F, c->bs, c->bs, part));
    int k = 0;
    double rn = 0.0;
    while (true) {
      apply_A64(c, F, c->xs, F.r);                       // r = b - A x in FP64
      launch_sub_from(s, F.n, F.row_lat, c->bs, F.r);
      rn = std::sqrt(host_dot(c, F, F.r, F.r, part));
      if (!std::isfinite(rn)) break;
      if (rn <= rtol * bn || k >= max_cycles) break;
      if (!F.ms) launch_diag_scale(s, F.n, F.row_lat, F.c, F.r, F.xs, c->zero_flag);
      vcycle_level(c, int(c->lv.size()) - 1, c->zero_flag, false);
      launch_rows_op(s, F.n, F.row_lat, F.x, c->xs, 2, nullptr);   // x += B (b - A x)
      ++k;
    }
    launch_gather(s, F.n, F.row_lat, c->xs, x_dev);
    HIP_CHECK_RET(hipGetLastError());
    HIP_CHECK_RET(hipStreamSynchronize(s));
    const double rel = bn > 0.0 ? rn / bn : rn;
    const int status = !std::isfinite(rn) ? IMSMG_ERR_NAN : (rel <= rtol ? IMSMG_OK : IMSMG_ERR_NOT_CONVERGED);
    if (info) {
      fill_info_common(c, info, 0);
      info->status = status;
      info->iterations = k;
      info->rel_res = rel;
      info->true_rel_res = rel;
      info->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (status != IMSMG_OK) {
      c->err = status == IMSMG_ERR_NAN ? "NaN or Inf in the multigrid iteration"
                                       : "the multigrid iteration did not reach rtol within max_cycles";
      return status;
    }
    return IMSMG_OK;
  });
}

int imsmg_apply_operator(imsmg_ctx *c, int level, const double *x, double *y) {
  return guarded(c, [&]() -> int {
    if (!c->ready) bad("setup first", IMSMG_ERR_STATE);
    if (level < 0 || level >= int(c->lv.size()) || !x || !y) bad("bad level or vector");
    Level &L = c->lv[level];
    launch_scatter(c->stream, L.n, L.row_lat, x, L.x);
    residual(c, L, L.x, nullptr, L.rh, c->zero_flag, false);
    launch_gather(c->stream, L.n, L.row_lat, L.rh, y);
    HIP_CHECK_RET(hipGetLastError());
    HIP_CHECK_RET(hipStreamSynchronize(c->stream));
    return IMSMG_OK;
  });
}

int imsmg_apply_smoother(imsmg_ctx *c, int level, const double *r, double *y) {
  return guarded(c, [&]() -> int {
    if (!c->factored) bad("factor first", IMSMG_ERR_STATE);
    if (level < 1 || level >= int(c->lv.size()) || !r || !y) bad("bad level or vector");
    Level &L = c->lv[level];
    if (L.ms) {
      // multiplicative: one forward sweep from x = 0 on the residual r
      launch_scatter(c->stream, L.n, L.row_lat, r, L.r);
      launch_rows_op(c->stream, L.n, L.row_lat, nullptr, L.x, 0, c->zero_flag);
      ms_sweep(c, L, true, c->zero_flag);
      launch_gather(c->stream, L.n, L.row_lat, L.x, y);
      HIP_CHECK_RET(hipGetLastError());
      HIP_CHECK_RET(hipStreamSynchronize(c->stream));
      return IMSMG_OK;
    }
    launch_scatter(c->stream, L.n, L.row_lat, r, L.rh);
    launch_diag_scale(c->stream, L.n, L.row_lat, L.c, L.rh, L.x, c->zero_flag);
    launch_smooth_general(c->stream, L.ng, L.grow_lat, L.sptr, L.scol, L.sval, L.rh, L.x, c->zero_flag, L.gen_lanes);
    launch_gather(c->stream, L.n, L.row_lat, L.x, y);
    HIP_CHECK_RET(hipGetLastError());
    HIP_CHECK_RET(hipStreamSynchronize(c->stream));
    return IMSMG_OK;
  });
}

int imsmg_apply_restriction(imsmg_ctx *c, int level, const double *rf, double *rc) {
  return guarded(c, [&]() -> int {
    if (!c->ready) bad("setup first", IMSMG_ERR_STATE);
    if (level < 1 || level >= int(c->lv.size()) || !rf || !rc) bad("bad level or vector");
    Level &L = c->lv[level], &Cl = c->lv[level - 1];
    launch_scatter(c->stream, L.n, L.row_lat, rf, L.rh);
    restrict_to(c, L, Cl, L.rh, Cl.r, nullptr, c->zero_flag);
    launch_gather(c->stream, Cl.n, Cl.row_lat, Cl.r, rc);
    HIP_CHECK_RET(hipGetLastError());
    HIP_CHECK_RET(hipStreamSynchronize(c->stream));
    return IMSMG_OK;
  });
}

int imsmg_apply_prolongation(imsmg_ctx *c, int level, const double *xc, double *xf) {
  return guarded(c, [&]() -> int {
    if (!c->ready) bad("setup first", IMSMG_ERR_STATE);
    if (level < 1 || level >= int(c->lv.size()) || !xc || !xf) bad("bad level or vector");
    Level &L = c->lv[level], &Cl = c->lv[level - 1];
    launch_scatter(c->stream, Cl.n, Cl.row_lat, xc, Cl.x);
    launch_scatter(c->stream, L.n, L.row_lat, xf, L.x);
    prolong_add(c, L, Cl, Cl.x, L.x, c->zero_flag);
    launch_gather(c->stream, L.n, L.row_lat, L.x, xf);
    HIP_CHECK_RET(hipGetLastError());
    HIP_CHECK_RET(hipStreamSynchronize(c->stream));
    return IMSMG_OK;
  });
}

int imsmg_coarse_solve(imsmg_ctx *c, const double *r, double *x) {
  return guarded(c, [&]() -> int {
    if (!c->factored) bad("factor first", IMSMG_ERR_STATE);
    if (!r || !x) bad("null vector");
    Level &L = c->lv[0];
    launch_scatter(c->stream, L.n, L.row_lat, r, L.r);
    launch_dense_gemv(c->stream, L.n, L.row_lat, L.Ainv, L.r, L.x, c->zero_flag);
    launch_gather(c->stream, L.n, L.row_lat, L.x, x);
    HIP_CHECK_RET(hipGetLastError());
    HIP_CHECK_RET(hipStreamSynchronize(c->stream));
    return IMSMG_OK;
  });
}

int imsmg_get_level_stats(imsmg_ctx *c, int level, imsmg_level_stats *st) {
  return guarded(c, [&]() -> int {
    if (!c->factored) bad("factor first", IMSMG_ERR_STATE);
    if (level < 0 || level >= int(c->lv.size()) || !st) bad("bad level");
    const Level &L = c->lv[level];
    st->n = L.n;
    st->stencil = L.csr ? 0 : L.K;  // 0: general sparse level (CSR rows)
    st->stored_rows = L.n - L.n_uniform;
    st->general_rows = L.ng;
    st->sg_nnz = 0;
    if (L.ng > 0) {
      int32_t last = 0;
      HIP_CHECK_RET(hipMemcpy(&last, L.sptr + L.ng, sizeof(int32_t), hipMemcpyDeviceToHost));
      st->sg_nnz = last;
    }
    st->lattice = L.lattice;
    st->value_bytes = mixed(c) ? 4 : 8;
    st->general_lanes = L.gen_lanes;
    st->patch_gemm = L.mb_on ? 1 : 0;
    st->bf16_blocks = L.mb_on ? L.mb_nlp : 0;
    return IMSMG_OK;
  });
}

int imsmg_kernel_time(imsmg_ctx *c, double *total_ms, int64_t *launches, int reset) {
  return guarded(c, [&]() -> int {
    if (total_ms) *total_ms = c->t_kernel_ms;
    if (launches) *launches = c->t_kernel_n;
    if (reset) {
      c->t_kernel_ms = 0.0;
      c->t_kernel_n = 0;
    }
    return IMSMG_OK;
  });
}

int imsmg_set_block_weights(imsmg_ctx *c, int level, const double *omega) {
  return guarded(c, [&]() -> int {
    if (!c->factored) bad("factor first", IMSMG_ERR_STATE);
    if (level < 1 || level >= int(c->lv.size()) || !omega) bad("bad level or null weights");
    Level &L = c->lv[level];
    if (L.ms) bad("per-block weights apply to the additive smoother only");
    const int nbf = int(L.f_ptr.size()) - 1;
    std::vector<double> w(omega, omega + nbf);
    for (double v : w)
      if (!(v > 0.0) || !std::isfinite(v)) bad("weights must be positive and finite");
    apply_weights(c, L, w);
    L.learned_status = 0;
    L.lambda_max = 0.0;
    return IMSMG_OK;
  });
}

int imsmg_load_mlp(imsmg_ctx *c, const float *params, int64_t nparams) {
  return guarded(c, [&]() -> int {
    if (!params || nparams != kMlpParams) bad("the damping network has " + std::to_string(kMlpParams) + " parameters");
    for (int64_t k = 0; k < nparams; ++k)
      if (!std::isfinite(params[k])) bad("non-finite network parameter");
    if (!c->mlp) HIP_CHECK_RET(hipMalloc(reinterpret_cast<void **>(&c->mlp), kMlpParams * sizeof(float)));
    HIP_CHECK_RET(hipMemcpy(c->mlp, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice));
    return IMSMG_OK;
  });
}

int imsmg_get_patch_features(imsmg_ctx *c, int level, int32_t *nblocks, float *feat) {
  return guarded(c, [&]() -> int {
    if (!c->factored) bad("factor first", IMSMG_ERR_STATE);
    if (level < 1 || level >= int(c->lv.size()) || !nblocks) bad("bad level or null count");
    Level &L = c->lv[level];
    *nblocks = int32_t(L.f_ptr.size()) - 1;
    if (feat) {
      std::vector<float> F = block_features(c, level);
      std::copy(F.begin(), F.end(), feat);
    }
    return IMSMG_OK;
  });
}

int imsmg_get_patch_weights(imsmg_ctx *c, int level, int32_t *nblocks, double *omega, int32_t *learned_status,
                            double *lambda_max) {
  return guarded(c, [&]() -> int {
    if (!c->factored) bad("factor first", IMSMG_ERR_STATE);
    if (level < 1 || level >= int(c->lv.size()) || !nblocks) bad("bad level or null count");
    Level &L = c->lv[level];
    *nblocks = int32_t(L.f_w.size());
    if (omega) std::copy(L.f_w.begin(), L.f_w.end(), omega);
    if (learned_status) *learned_status = L.learned_status;
    if (lambda_max) *lambda_max = L.lambda_max;
    return IMSMG_OK;
  });
}

int imsmg_lambda_max(imsmg_ctx *c, int level, int iters, double *lambda_max) {
  return guarded(c, [&]() -> int {
    if (!c->factored) bad("factor first", IMSMG_ERR_STATE);
    if (level < 1 || level >= int(c->lv.size()) || iters < 1 || !lambda_max) bad("bad arguments");
    *lambda_max = lambda_max_SA(c, c->lv[level], iters);
    return IMSMG_OK;
  });
}

int imsmg_two_grid_objective(imsmg_ctx *c, int m, const double *Z, int k, double *J, double *grad) {
  return guarded(c, [&]() -> int {
    if (!c->factored) bad("factor first", IMSMG_ERR_STATE);
    two_grid(c, m, Z, k, J, grad);
    return IMSMG_OK;
  });
}

int64_t imsmg_mlp_workspace_bytes(int n) { return n < 1 ? 0 : int64_t(mlp_workspace_bytes(n)); }

int imsmg_mlp_forward(void *stream, const float *params, const float *X, int n, float *out) {
  if (n < 0 || (n > 0 && (!params || !X || !out))) return IMSMG_ERR_INVALID_ARG;
  launch_mlp_forward(static_cast<hipStream_t>(stream), n, params, X, out);
  return hipGetLastError() == hipSuccess ? IMSMG_OK : IMSMG_ERR_HIP;
}

int imsmg_mlp_loss_grad(void *stream, const float *params, const float *X, const float *t, int n, void *work,
                        float *loss, float *grad) {
  if (n < 1 || !params || !X || !t || !work || !loss || !grad) return IMSMG_ERR_INVALID_ARG;
  launch_mlp_loss_grad(static_cast<hipStream_t>(stream), n, params, X, t, work, loss, grad);
  return hipGetLastError() == hipSuccess ? IMSMG_OK : IMSMG_ERR_HIP;
}

int imsmg_mlp_loss_grad_noalloc(void *stream, const float *params, const float *X, const float *t, int n,
                                float *loss, float *grad) {
  if (n < 1 || n > IMSMG_NOALLOC_MAX_SAMPLES || !params || !X || !t || !loss || !grad)
    return IMSMG_ERR_INVALID_ARG;
  static_assert(IMSMG_NOALLOC_MAX_SAMPLES >= 1, "sample cap");
  hipStream_t s = static_cast<hipStream_t>(stream);
  void *work = nullptr;
  const int rc = mlp_noalloc_scratch(s, &work);
  if (rc != IMSMG_OK) return rc;
  if (mlp_workspace_bytes(n) > mlp_noalloc_scratch_bytes()) return IMSMG_ERR_INVALID_ARG;
  launch_mlp_loss_grad(s, n, params, X, t, work, loss, grad);
  return hipGetLastError() == hipSuccess ? IMSMG_OK : IMSMG_ERR_HIP;
}

int imsmg_mlp_adam(void *stream, float *params, const float *grad, float *m, float *v, int step, float lr) {
  if (!params || !grad || !m || !v || step < 1 || !(lr > 0.0f)) return IMSMG_ERR_INVALID_ARG;
  launch_mlp_adam(static_cast<hipStream_t>(stream), params, grad, m, v, step, lr);
  return hipGetLastError() == hipSuccess ? IMSMG_OK : IMSMG_ERR_HIP;
}

int imsmg_vcycle_multi(imsmg_ctx *c, int nrhs, const double *R_dev, double *Z_dev) {
  return guarded(c, [&]() -> int {
    if (!c->factored) bad("factor first", IMSMG_ERR_STATE);
    if (uses_ms(c->opt, int(c->lv.size())) || c->opt.cycle != 1)
      bad("the multi-column solve runs the additive V-cycle only");
    if (!R_dev || !Z_dev) bad("null vector");
    const int R = rhs_width(nrhs);
    ensure_multi(c, R);
    Level &F = c->lv.back();
    const int f = int(c->lv.size()) - 1;
    auto &m = c->mb;
    launch_m_scatter(c->stream, R, F.n, nrhs, F.row_lat, R_dev, m.r[f]);
    launch_m_diag_scale(c->stream, R, F.n, F.row_lat, F.c, m.r[f], m.xs[f], c->zero_flag);
    m_vcycle_level(c, f, c->zero_flag);
    launch_m_gather(c->stream, R, F.n, nrhs, F.row_lat, m.x[f], Z_dev);
    HIP_CHECK_RET(hipGetLastError());
    HIP_CHECK_RET(hipStreamSynchronize(c->stream));
    return IMSMG_OK;
  });
}

int imsmg_pcg_solve_multi(imsmg_ctx *c, int nrhs, const double *B_dev, double *X_dev, double rtol,
                          imsmg_info *infos) {
  return guarded(c, [&]() -> int {
    if (!c->factored) bad("factor first", IMSMG_ERR_STATE);
    if (!B_dev || !X_dev) bad("null vector");
    if (!(rtol > 0.0)) bad("rtol must be positive");
    if (c->opt.flexible_cg) bad("flexible_cg applies to imsmg_pcg_solve only");
    if (uses_ms(c->opt, int(c->lv.size())) || c->opt.cycle != 1)
      bad("the multi-column solve runs the additive V-cycle only");
    const int R = rhs_width(nrhs);
    auto t0 = std::chrono::steady_clock::now();
    ensure_multi(c, R);
    auto &m = c->mb;
    Level &F = c->lv.back();
    const int f = int(c->lv.size()) - 1;
    hipStream_t s = c->stream;
    launch_m_scatter(s, R, F.n, nrhs, F.row_lat, B_dev, m.bs);
    launch_m_scatter(s, R, F.n, nrhs, F.row_lat, X_dev, m.xsol);
    MState h{};
    int restarts = 0, keep = 0;
    std::vector<double> true_rel(R, 0.0);
    while (true) {
      launch_mcg_init(s, R, nrhs, F.n, F.K, F.op64, F.row_lat, F.meta, m.xsol, m.bs, m.r[f], m.part, m.st, rtol,
                      restarts > 0, keep);
      launch_m_diag_scale(s, R, F.n, F.row_lat, F.c, m.r[f], m.xs[f], &m.st->done);
      HIP_CHECK_RET(hipGetLastError());
      const int mit = c->opt.check_every;
      if (c->opt.use_graph && !m.graph) {
        hipGraph_t g = nullptr;
        HIP_CHECK_RET(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < mit; ++k) m_cg_iteration(c);
        HIP_CHECK_RET(hipStreamEndCapture(s, &g));
        hipError_t e = hipGraphInstantiate(&m.graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIP_CHECK_RET(e);
      }
      while (true) {
        if (c->opt.use_graph) {
          HIP_CHECK_RET(hipGraphLaunch(m.graph, s));
        } else {
          for (int k = 0; k < mit; ++k) m_cg_iteration(c);
        }
        HIP_CHECK_RET(hipGetLastError());
        HIP_CHECK_RET(hipMemcpyAsync(&h, m.st, sizeof(MState), hipMemcpyDeviceToHost, s));
        HIP_CHECK_RET(hipStreamSynchronize(s));
        if (h.done) break;
      }
      launch_mcg_true_residual(s, R, F.n, F.K, F.op64, F.row_lat, F.meta, m.xsol, m.bs, m.part, m.st);
      HIP_CHECK_RET(hipMemcpyAsync(&h, m.st, sizeof(MState), hipMemcpyDeviceToHost, s));
      HIP_CHECK_RET(hipStreamSynchronize(s));
      bool again = false;
      keep = 0;
      for (int k = 0; k < nrhs; ++k) {
        true_rel[k] = h.bb[k] > 0.0 ? std::sqrt(h.aux[k] / h.bb[k]) : 0.0;
        if (true_rel[k] > rtol && h.iters[k] < c->opt.max_iter) again = true;
        else keep |= 1 << k;  // this column stays converged on a restart
      }
      if (h.status == 0 && again && restarts < 3) {
        ++restarts;
        continue;
      }
      break;
    }
    launch_m_gather(s, R, F.n, nrhs, F.row_lat, m.xsol, X_dev);
    HIP_CHECK_RET(hipStreamSynchronize(s));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    // a column that ends above rtol (restarts used up, or max_iter) has not converged
    bool missed = false;
    for (int k = 0; k < nrhs; ++k) missed |= true_rel[k] > rtol;
    if (h.status == 0 && missed) h.status = IMSMG_ERR_NOT_CONVERGED;
    if (infos)
      for (int k = 0; k < nrhs; ++k) {
        fill_info_common(c, &infos[k], restarts);
        infos[k].status = h.status == IMSMG_ERR_NOT_CONVERGED ? (true_rel[k] > rtol ? h.status : 0) : h.status;
        infos[k].iterations = h.iters[k];
        infos[k].rel_res = h.r0sq[k] > 0.0 ? std::sqrt(h.rr[k] / h.r0sq[k]) : 0.0;
        infos[k].true_rel_res = true_rel[k];
        infos[k].solve_ms = ms;
      }
    if (h.status != 0) {
      c->err = h.status == IMSMG_ERR_NOT_CONVERGED ? "CG did not reach rtol in some column (true relative residual)"
               : h.status == IMSMG_ERR_NOT_SPD     ? "CG breakdown: p.Ap <= 0"
                                                   : "NaN or Inf in the CG iteration";
      return int(h.status);
    }
    return IMSMG_OK;
  });
}

const char *imsmg_last_error(imsmg_ctx *c) { return c ? c->err.c_str() : "null context"; }

int imsmg_setup_batched(imsmg_ctx *c, int nprob, const int *nlevels, const imsmg_csr *const *A,
                        const imsmg_csr *const *R, const imsmg_patches *const *P, const imsmg_lattice *const *L,
                        const imsmg_elements *const *E, const imsmg_options *opt) {
  if (!c) return IMSMG_ERR_INVALID_ARG;
  if (nprob < 1 || !nlevels || !A || !R || !P || !L) return fail(c, IMSMG_ERR_INVALID_ARG, "bad batched arguments");
  if (opt && opt->ncomp > 1) return fail(c, IMSMG_ERR_INVALID_ARG, "vector problems: the batched form is not supported");
  for (int p = 0; p < nprob; ++p)
    for (int l = 0; L[p] && l < nlevels[p]; ++l)
      if (!L[p][l].dof_to_lattice)
        return fail(c, IMSMG_ERR_INVALID_ARG, "general sparse levels: the batched form is not supported");
  if (c->ready) return fail(c, IMSMG_ERR_STATE, "a set-up single-problem context cannot become a batch");
  for (imsmg_ctx *b : c->batch) imsmg_destroy(b);
  c->batch.clear();
  for (int p = 0; p < nprob; ++p) {
    imsmg_ctx *ch = nullptr;
    int rc = imsmg_create(&ch, c->device, nullptr);
    if (rc == IMSMG_OK) rc = imsmg_setup(ch, nlevels[p], A[p], R[p], P[p], L[p], E ? E[p] : nullptr, opt);
    if (rc != IMSMG_OK) {
      const std::string m = "problem " + std::to_string(p) + ": " + (ch ? ch->err : std::string("create failed"));
      imsmg_destroy(ch);
      for (imsmg_ctx *b : c->batch) imsmg_destroy(b);
      c->batch.clear();
      return fail(c, rc, m);
    }
    c->batch.push_back(ch);
  }
  c->err.clear();
  return IMSMG_OK;
}

int imsmg_batch_problem(imsmg_ctx *c, int p, imsmg_ctx **child) {
  if (!c || !child) return IMSMG_ERR_INVALID_ARG;
  if (p < 0 || p >= int(c->batch.size())) return fail(c, IMSMG_ERR_INVALID_ARG, "no such problem in the batch");
  *child = c->batch[p];
  return IMSMG_OK;
}

int imsmg_pcg_solve_batched(imsmg_ctx *c, int nrhs, const double *const *B_dev, double *const *X_dev, double rtol,
                            imsmg_info *infos, int nthreads) {
  if (!c) return IMSMG_ERR_INVALID_ARG;
  const int np = int(c->batch.size());
  if (np == 0) return fail(c, IMSMG_ERR_STATE, "imsmg_setup_batched first");
  if (!B_dev || !X_dev) return fail(c, IMSMG_ERR_INVALID_ARG, "null vector arrays");
  const int nt = std::max(1, std::min(nthreads > 0 ? nthreads : 4, np));
  std::atomic<int> next{0};
  std::mutex mu;
  int first_rc = IMSMG_OK;
  std::string first_msg;
  // each thread takes the next problem and runs its multi-column solve on the
  // problem's own stream, so that the problems' latency-bound V-cycles overlap
  auto work = [&]() {
    for (int p = next++; p < np; p = next++) {
      const int rc = imsmg_pcg_solve_multi(c->batch[p], nrhs, B_dev[p], X_dev[p], rtol,
                                           infos ? infos + size_t(p) * nrhs : nullptr);
      if (rc != IMSMG_OK) {
        std::lock_guard<std::mutex> g(mu);
        if (first_rc == IMSMG_OK) {
          first_rc = rc;
          first_msg = "problem " + std::to_string(p) + ": " + c->batch[p]->err;
        }
      }
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(work);
  work();
  for (auto &th : pool) th.join();
  if (first_rc != IMSMG_OK) return fail(c, first_rc, first_msg);
  c->err.clear();
  return IMSMG_OK;
}

int imsmg_destroy(imsmg_ctx *c) {
  if (!c) return IMSMG_OK;
  for (imsmg_ctx *b : c->batch) imsmg_destroy(b);
  c->batch.clear();
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  destroy_graph(c);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  free_multi(c);
  free_list(c->factor_owned);
  free_list(c->owned);
  if (c->mlp) (void)hipFree(c->mlp);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return IMSMG_OK;
}

}  // extern "C"
