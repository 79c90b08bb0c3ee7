// C ABI and the host-side LOBPCG driver (Algorithm 1) of the partitioner
// (Algorithm 2).  Everything is ordered on the handle's stream; the only
// per-iteration host/device exchange is one small status read.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>

#include "kernels.h"

using namespace sphx;

namespace {

const char *kStatusText[] = {
    "ok", "invalid argument", "malformed CSR graph", "graph not symmetric",
    "bad weight", "self-loop", "Rayleigh-Ritz breakdown", "HIP error",
    "workspace too small or allocation failed"};

int bytes_of(int dtype) { return dtype == SPHX_F32 ? 4 : 8; }

// Workspace: the caller's if large enough, else an owned (cached) one.
int get_workspace(sphx_handle *h, size_t need, char **out) {
  if (h->ws_user && h->ws_user_bytes >= need) {
    *out = static_cast<char *>(h->ws_user);
    return SPHX_OK;
  }
  if (h->ws_own_bytes < need) {
    if (h->ws_own) (void)hipFree(h->ws_own);
    h->ws_own = nullptr;
    h->ws_own_bytes = 0;
    if (hipMalloc(&h->ws_own, need) != hipSuccess)
      return set_err(h, SPHX_E_WORKSPACE, "workspace allocation failed");
    h->ws_own_bytes = need;
  }
  *out = static_cast<char *>(h->ws_own);
  return SPHX_OK;
}

// Device scratch of sphx_quality_noalloc: a fixed array in the library's
// code object, so that entry point never allocates.  Each GPU holds its own
// copy; its address on a device is resolved once (hipGetSymbolAddress, with
// that device current) when the first handle on that device is created, and
// only that address is passed to kernels or copies.
constexpr size_t kNoAllocScratchBytes = size_t(1) << 20;
constexpr int kNoAllocMaxK = 65536;
constexpr int kNoAllocMaxDevices = 64;
static __device__ __align__(256) unsigned char noalloc_scratch[kNoAllocScratchBytes];

std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kNoAllocMaxDevices] = {};

// With `device` current: resolve this device's copy of noalloc_scratch.
int resolve_noalloc_scratch(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return SPHX_OK;   // entry point refuses
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return SPHX_OK;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)) != hipSuccess || !p)
    return SPHX_E_HIP;
  g_noalloc_ptr[device] = p;
  return SPHX_OK;
}

void *noalloc_scratch_ptr(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  return g_noalloc_ptr[device];
}

constexpr int kDegBlocksMax = 1024;
constexpr int kRqBlocks = 256;

// Workspace layout of a solve (also used for sizing with count_only).
template <typename T>
struct SolveWs {
  double *d64, *dinv, *sq, *rsq;
  T *X, *LX, *R, *B1, *B2, *LH, *P, *LP;
  double *X64, *LX64;
  double *norm_partials, *gram_partials, *gram_out, *Y, *theta;
  DevStatus *status;
  double *rq_partials, *rq_sums, *res_sums;
  void *norm_scratch;
  double *deg_scratch;
  int *flags;
  void *split_scratch, *quality_scratch;
  void *poly_scratch;   // Lanczos basis of the GMRES polynomial (or null)
  double *poly_b, *poly_tmp;
  char *ord_scratch;    // degree-ordered copy of the graph (or null)
  T *V;        // eigenvectors when the caller passes none (partition)
  int32_t *part;
  SpmmPlan plan;
  size_t plan_off;
};

template <typename T>
void layout(Arena &a, SolveWs<T> &w, int64_t n, int m, int K, size_t plan_b,
            bool want_split, int poly_degree, size_t ord_b) {
  w.d64 = a.take<double>(n);
  w.dinv = a.take<double>(n);
  w.sq = a.take<double>(n);
  w.rsq = a.take<double>(n);
  const size_t blk = (size_t)n * padded_ld(m, sizeof(T));
  w.X = a.take<T>(blk);
  w.LX = a.take<T>(blk);
  w.R = a.take<T>(blk);
  w.B1 = a.take<T>(blk);
  w.B2 = a.take<T>(blk);
  w.LH = a.take<T>(blk);
  w.P = a.take<T>(blk);
  w.LP = a.take<T>(blk);
  if (std::is_same_v<T, float>) {
    w.X64 = a.take<double>(blk);
    w.LX64 = a.take<double>(blk);
  } else {
    w.X64 = w.LX64 = nullptr;
  }
  w.norm_partials = a.take<double>((size_t)kMaxNormBlocks * 2 * kMaxNev);
  w.gram_partials = a.take<double>(gram_partial_doubles(kGramBlocks));
  w.gram_out = a.take<double>(2 * kMaxW * kMaxW);
  w.Y = a.take<double>(kMaxW * kMaxNev);
  w.theta = a.take<double>(kMaxNev);
  w.status = a.take<DevStatus>(1);
  w.rq_partials = a.take<double>((size_t)kRqBlocks * 2 * kMaxNev);
  w.rq_sums = a.take<double>(2 * kMaxNev);
  w.res_sums = a.take<double>(2 * kMaxNev);
  w.norm_scratch = a.take<char>(normalize_scratch_bytes());
  w.deg_scratch = a.take<double>(4 * kDegBlocksMax);
  w.flags = a.take<int>(64);
  if (want_split) {
    w.split_scratch = a.take<char>(split_scratch_bytes(n, K));
    w.quality_scratch = a.take<char>(quality_scratch_bytes(K));
    w.V = a.take<T>((size_t)n * m);
    w.part = a.take<int32_t>(n);
  } else {
    w.split_scratch = w.quality_scratch = nullptr;
    w.V = nullptr;
    w.part = nullptr;
  }
  if (poly_degree > 0) {
    w.poly_scratch = a.take<char>(poly_scratch_bytes(n, poly_degree));
    w.poly_b = a.take<double>(n);
    w.poly_tmp = a.take<double>(n);
  } else {
    w.poly_scratch = nullptr;
    w.poly_b = w.poly_tmp = nullptr;
  }
  w.ord_scratch = ord_b ? a.take<char>(ord_b) : nullptr;
  w.plan_off = a.off;
  a.off += plan_b;
}

// dst row i (m values) = src row idx[i]
template <typename T>
__global__ void k_gather_rows(const T *__restrict__ src, int lds, const int32_t *__restrict__ idx,
                              T *dst, int ldd, int64_t n, int m) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / m;
    const int c = (int)(e - i * m);
    dst[i * ldd + c] = src[(int64_t)idx[i] * lds + c];
  }
}

bool valid_options(const sphx_options *o) {
  if (!o) return false;
  if (o->problem != SPHX_COMBINATORIAL && o->problem != SPHX_GENERALIZED &&
      o->problem != SPHX_NORMALIZED)
    return false;
  if (o->precond < SPHX_PRECOND_NONE || o->precond > SPHX_PRECOND_GMRES) return false;
  if (o->precond == SPHX_PRECOND_CHEBYSHEV && (o->cheb_degree < 1 || !(o->cheb_ratio > 1.0)))
    return false;
  if (o->precond == SPHX_PRECOND_GMRES && (o->cheb_degree < 1 || o->cheb_degree + 1 > kMaxW))
    return false;
  if (o->precision != SPHX_FP64 && o->precision != SPHX_MIXED) return false;
  if (!(o->tol > 0.0) || o->max_iter < 0) return false;
  if (o->init < SPHX_INIT_RANDOM || o->init > SPHX_INIT_USER) return false;
  if (o->drop_tol < 0.0) return false;
  if (o->reorder != 0 && o->reorder != 1) return false;
  return true;
}

ColMap identity_map(int m) {
  ColMap c;
  c.count = m;
  for (int i = 0; i < kMaxNev; ++i) c.col[i] = i < m ? i : 0;
  return c;
}

// sq = sqrt(d), rsq = 1 / sqrt(d): the congruence between L_N and (L_C, D)
__global__ void k_sqrt_pair(const double *d, double *sq, double *rsq, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double r = sqrt(d[i]);
    sq[i] = r;
    rsq[i] = 1.0 / r;
  }
}

__global__ void k_inverse(const double *d, double *dinv, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dinv[i] = 1.0 / d[i];
}

// out[i, c] = scale * dinv[i] * in[i, c]
template <typename T>
__global__ void k_scale_rows(const T *in, const double *dinv, double scale, T *out, int64_t n,
                             int m) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * m;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = T(scale * dinv[e / m] * double(in[e]));
}

template <typename T>
__global__ void k_jacobi(const T *R, const double *d, T *H, int64_t n, int m) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * m;
       e += (int64_t)gridDim.x * blockDim.x)
    H[e] = T(double(R[e]) / d[e / m]);
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  bool on = false;
  void start(hipStream_t s) {
    if (!a) { (void)hipEventCreate(&a); (void)hipEventCreate(&b); }
    (void)hipEventRecord(a, s);
    on = true;
  }
  double stop(hipStream_t s) {
    if (!on) return 0.0;
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    return ms;
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Chebyshev step coefficients (Chebyshev iteration for L h = r on [lo, hi]).
struct ChebCoef {
  double c, e;
  std::vector<double> alpha, beta;
};
ChebCoef cheb_coef(int degree, double lo, double hi) {
  ChebCoef k;
  k.c = 0.5 * (hi + lo);
  k.e = 0.5 * (hi - lo);
  double sigma = k.c / k.e;
  double rho_prev = 1.0 / sigma;
  for (int s = 0; s < degree; ++s) {
    double rho = 1.0 / (2.0 * sigma - rho_prev);
    k.alpha.push_back(rho * rho_prev);
    k.beta.push_back(2.0 * rho / k.e);
    rho_prev = rho;
  }
  return k;
}

// Algorithmic bytes of one Laplacian product over G columns of s-byte
// values: index arrays once, `vec_passes` block passes (the gathered source
// counted once), `row_doubles` FP64 per-row values.
// Algorithmic bytes of one product over the caller's int32 CSR (int16 column
// offsets, when the plan has them, are read in half the index bytes).
double spmm_bytes(const sphx_graph *g, const SpmmPlan &plan, int G, int s, int vec_passes,
                  int row_doubles) {
  double b = (g->rp64 ? 8.0 : 4.0) * double(g->n + 1) + 4.0 * double(g->nnz);
  if (g->wdt == SPHX_F32) b += 4.0 * double(g->nnz);
  if (g->wdt == SPHX_F64) b += 8.0 * double(g->nnz);
  if (plan.binned) b += 4.0 * double(g->n);
  return b + double(vec_passes) * double(g->n) * G * s + 8.0 * row_doubles * double(g->n);
}

// Rc[i, q] = R[i, act[q]] for q < na, 0 for na <= q < lda; with X1 also
// X1[i, q] = scale * dinv[i] * Rc[i, q] (the first Chebyshev iterate)
template <typename T>
__global__ void k_compact_cols(const T *R, int ld, ColMap act, int lda, const double *dinv,
                               double scale, T *Rc, T *X1, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * lda;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / lda;
    const int q = (int)(e - i * lda);
    const T v = q < act.count ? R[i * ld + act.col[q]] : T(0);
    Rc[e] = v;
    if (X1) X1[e] = T(scale * dinv[i] * double(v));
  }
}

// H[i, act[q]] = Hc[i, q] for q < na (other columns of H are left as they are)
template <typename T>
__global__ void k_expand_cols(const T *Hc, int lda, ColMap act, T *H, int ld, int64_t n) {
  const int na = act.count;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * na;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / na;
    const int q = (int)(e - i * na);
    H[i * ld + act.col[q]] = Hc[i * lda + q];
  }
}

// Row width of the compacted Chebyshev block for na active columns: even,
// so that FP32 rows are whole 8-byte vectors and FP64 rows 16-byte ones.
inline int compact_ld(int na) { return (na + 1) / 2 * 2; }

// H[:, cm] = p(L) R[:, cm]: returns the buffer holding the result (n x ld,
// the columns of cm).  With `spare` (an n x ld buffer whose contents may be
// destroyed, e.g. R itself) and fewer active columns than the padded width,
// the iteration runs on a compacted block of the active columns only.
template <typename T>
int cheb_apply(sphx_handle *h, sphx_graph *g, const SpmmPlan &plan, int m, int ld,
               const ColMap &cm, const T *R, T *B1, T *B2, T *spare, const ChebCoef &k,
               const double *dinv, hipStream_t s, T **result, int64_t *calls,
               int64_t *pcalls) {
  const int rd = dinv ? 1 : 0;
  const double b3 = spmm_bytes(g, plan, cm.count, sizeof(T), 3, rd);
  const double b4 = spmm_bytes(g, plan, cm.count, sizeof(T), 4, rd);
  const int64_t n = g->n;
  const int na = cm.count;
  const int lda = compact_ld(na);
  const bool compact = spare && lda < ld;
  const int wd = compact ? lda : ld;     // row width of the iteration buffers
  const int mm = compact ? na : m;
  auto launch = [&](const T *src, EpiChebP<T> e, double bytes) -> int {
    // padded rows (the solver's blocks) take the vector-row kernels; the
    // column-lane kernels serve unpadded caller blocks
    int st;
    if (compact || ld != m || (m * (int)sizeof(T)) % 16 == 0) {
      LaunchEvents ev;
      const bool timed = h->plog.begin_stamped(PH_PRECOND, bytes, &ev.start, &ev.stop);
      st = vspmm_cheb<T>(g, plan, src, wd, mm, e, s, timed ? &ev : nullptr);
    } else {
      int id = h->plog.begin(PH_PRECOND, bytes, s);
      st = spmm_cheb<T>(g, plan, src, m, cm, e, s);
      h->plog.end(id, s);
    }
    ++*calls;
    ++*pcalls;
    return st;
  };
  const T *rhs = R;
  auto epi = [&](const T *prev, double prev_scale, T *out, double src_scale, int st) {
    EpiChebP<T> e;
    e.prev = prev;
    e.R = rhs;
    e.OUT = out;
    e.ld = wd;
    e.src_scale = src_scale;
    e.prev_scale = prev_scale;
    e.alpha = k.alpha[st];
    e.beta = k.beta[st];
    e.dinv = dinv;
    return e;
  };
  // h1 = rhs / c: rhs = r (combinatorial), read from R with a scale; or
  // rhs = D^-1 r (generalized), materialised first.  `slot` is the buffer
  // that step 2 overwrites (it holds h1, or is free).
  const T *h1 = R;
  double h1_scale = 1.0 / k.c;
  T *it1 = B1, *slot = B2;
  if (compact) {
    // Rc -> B2 (the right-hand side of every step), h1 -> B1 if it must be
    // materialised; R is free once this kernel is done, so the iterates use
    // B1 and spare
    hipLaunchKernelGGL(k_compact_cols<T>, dim3(grid_for(n * lda, 256, 4096)), dim3(256), 0, s,
                       R, ld, cm, lda, dinv, 1.0 / k.c, B2, dinv ? B1 : (T *)nullptr, n);
    rhs = B2;
    if (dinv) {
      h1 = B1;
      h1_scale = 1.0;
      it1 = spare;
      slot = B1;
    } else {
      h1 = B2;
      it1 = B1;
      slot = spare;
    }
  } else if (dinv) {
    hipLaunchKernelGGL(k_scale_rows<T>, dim3(grid_for(n * ld, 256, 4096)), dim3(256), 0, s, R,
                       dinv, 1.0 / k.c, B2, n, ld);
    h1 = B2;
    h1_scale = 1.0;
  }
  SPHX_TRY(launch(h1, epi(nullptr, 1.0, it1, h1_scale, 0), b3));
  T *cur = it1, *other = slot;
  const int deg = (int)k.alpha.size();
  if (deg >= 2) {
    // step 2: the previous iterate is h1 (scaled, possibly in `slot`, which
    // is then overwritten in place by h3)
    SPHX_TRY(launch(it1, epi(h1, h1_scale, slot, 1.0, 1), b4));
    cur = slot;
    other = it1;
    // later steps overwrite the older iterate in place (each element is read
    // and written by the same lane only)
    for (int st = 2; st < deg; ++st) {
      SPHX_TRY(launch(cur, epi(other, 1.0, other, 1.0, st), b4));
      std::swap(cur, other);
    }
  }
  if (compact) {
    // back to the padded layout, in B2 (the compacted right-hand side is done)
    hipLaunchKernelGGL(k_expand_cols<T>, dim3(grid_for(n * na, 256, 4096)), dim3(256), 0, s,
                       (const T *)cur, lda, cm, B2, ld, n);
    cur = B2;
  }
  *result = cur;
  return SPHX_OK;
}

// H[:, cm] = p(L) R[:, cm] for the GMRES polynomial with the given roots
// (Leja order; nroots = degree + 1), on the compacted block of the active
// columns (`spare` and B1, B2 are n x ld buffers; `spare` may be R itself,
// which is read before it is overwritten).  Returns the buffer holding the
// result in the padded layout.
template <typename T>
int poly_apply(sphx_handle *h, sphx_graph *g, const SpmmPlan &plan, int m, int ld,
               const ColMap &cm, const T *R, T *B1, T *B2, T *spare, const double *roots,
               int nroots, const double *dinv, hipStream_t s, T **result, int64_t *calls,
               int64_t *pcalls) {
  const int64_t n = g->n;
  const int na = cm.count;
  const int lda = compact_ld(na);
  const int rd = dinv ? 1 : 0;
  const double b3 = spmm_bytes(g, plan, na, sizeof(T), 3, rd);
  const double b4 = spmm_bytes(g, plan, na, sizeof(T), 4, rd);
  const int k = nroots - 1;             // Laplacian products
  // P_1 = s R (compacted) -> B2; Y -> B1; P_2, P_3, ... alternate spare / B2
  hipLaunchKernelGGL(k_compact_cols<T>, dim3(grid_for(n * lda, 256, 4096)), dim3(256), 0, s,
                     R, ld, cm, lda, (const double *)nullptr, 1.0, B2, (T *)nullptr, n);
  if (dinv)
    hipLaunchKernelGGL(k_scale_rows<T>, dim3(grid_for(n * lda, 256, 4096)), dim3(256), 0, s,
                       (const T *)B2, dinv, 1.0, B2, n, lda);
  T *Y = B1;
  if (k == 0) {
    // degree 0: Y = P_1 / theta_1
    hipLaunchKernelGGL(k_scale_rows<T>, dim3(grid_for(n * lda, 256, 4096)), dim3(256), 0, s,
                       (const T *)B2, (const double *)nullptr, 1.0 / roots[0], Y, n, lda);
  }
  T *Pa = B2, *Pb = spare;
  for (int i = 0; i < k; ++i) {
    EpiPolyP<T> e;
    e.Yin = i == 0 ? nullptr : Y;
    e.Yout = Y;
    e.Pout = Pb;
    e.ld = lda;
    e.inv_t = 1.0 / roots[i];
    e.inv_t_next = 1.0 / roots[i + 1];
    e.dinv = dinv;
    e.last = i == k - 1 ? 1 : 0;
    const double bytes = (i == 0 || i == k - 1) ? b3 : b4;
    LaunchEvents ev;
    const bool timed = h->plog.begin_stamped(PH_PRECOND, bytes, &ev.start, &ev.stop);
    int st = vspmm_poly<T>(g, plan, Pa, lda, na, e, s, timed ? &ev : nullptr);
    ++*calls;
    ++*pcalls;
    SPHX_TRY(st);
    std::swap(Pa, Pb);
  }
  // back to the padded layout (B2 or spare is free: expand into the one
  // that does not hold Y)
  T *dst = (Y == B2) ? spare : B2;
  hipLaunchKernelGGL(k_expand_cols<T>, dim3(grid_for(n * na, 256, 4096)), dim3(256), 0, s,
                     (const T *)Y, lda, cm, dst, ld, n);
  *result = dst;
  return SPHX_OK;
}

// The LOBPCG solve (Algorithm 1) in precision T; fills eigvals / vecs.
template <typename T>
int solve(sphx_handle *h, sphx_graph *g, int m, const sphx_options &o, const void *X0,
          double *eigvals, T *vecs_out, sphx_stats *stats, SolveWs<T> &w, char *wsbase,
          bool *hit_max, bool *stalled, int *iterations) {
  hipStream_t s = h->stream;
  const int64_t n = g->n;
  int64_t calls = 0, pcalls = 0, pcols = 0;
  Timer tall;
  tall.start(s);
  PhaseLog &pl = h->plog;
  // ---- setup: degrees, classification, row bins
  int tid = pl.begin(PH_SETUP, 0.0, s);
  DegreeStats ds;
  SPHX_TRY(compute_degrees(g, w.d64, nullptr, w.deg_scratch, &ds, h->pinned_small, s));
  // graphs with rows of more than kUnbinnedMaxDeg neighbours run on a copy in
  // degree order (frequently gathered rows share cache lines); blocks live
  // in that order and are mapped at the start and the end of the solve
  sphx_graph gq;
  sphx_graph *G = g;
  int32_t *operm = nullptr, *oinv = nullptr;
  const bool reorder = o.reorder && ds.max_deg > kUnbinnedMaxDeg && w.ord_scratch;
  if (reorder) {
    SPHX_TRY(build_degree_order(g, w.ord_scratch, &gq, &operm, &oinv, s));
    G = &gq;
    SPHX_TRY(compute_degrees(G, w.d64, nullptr, w.deg_scratch, &ds, h->pinned_small, s));
  }
  // the normalized problem runs as the generalized pencil in x = D^-1/2 y
  const bool norm = o.problem == SPHX_NORMALIZED;
  const bool gen = o.problem != SPHX_COMBINATORIAL;
  if ((gen || o.precond == SPHX_PRECOND_JACOBI) && !(ds.min_wdeg > 0.0))
    return set_err(h, SPHX_E_INVALID_ARG,
                   "isolated vertex: the generalized and normalized problems and Jacobi "
                   "need all degrees > 0");
  if (norm)
    hipLaunchKernelGGL(k_sqrt_pair, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, w.d64, w.sq,
                       w.rsq, n);
  Arena pa;
  pa.base = wsbase + w.plan_off;
  pa.cap = plan_bytes(G);
  SPHX_TRY(build_plan(G, pa, &w.plan, ds, h->pinned_small, s));
  pl.end(tid, s);
  const int vs = sizeof(T);
  const int ld = padded_ld(m, sizeof(T));   // 16-byte rows for the vector kernels
  const double *bdiag = gen ? w.d64 : nullptr;
  const double *dinv = nullptr;
  ChebCoef ck;
  // Gershgorin bound of the operator (B^-1 L for the generalized pencil)
  const double l_norm = gen ? 2.0 : 2.0 * ds.max_wdeg;
  if (o.precond == SPHX_PRECOND_CHEBYSHEV) ck = cheb_coef(o.cheb_degree, l_norm / o.cheb_ratio, l_norm);
  if ((o.precond == SPHX_PRECOND_CHEBYSHEV || o.precond == SPHX_PRECOND_GMRES) && gen) {
    hipLaunchKernelGGL(k_inverse, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, w.d64, w.dinv,
                       n);
    dinv = w.dinv;
  }
  // GMRES polynomial: roots from a seeded start vector (in y for the
  // normalized problem, mapped to x = D^-1/2 y)
  double roots[kMaxW];
  int nroots = 0;
  if (o.precond == SPHX_PRECOND_GMRES) {
    launch_init_random<double>(reorder ? w.poly_tmp : w.poly_b, n, 1, 1,
                               o.seed ^ 0x9e3779b97f4a7c15ull, s);
    if (reorder)
      hipLaunchKernelGGL(k_gather_rows<double>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s,
                         (const double *)w.poly_tmp, 1, (const int32_t *)operm, w.poly_b, 1,
                         n, 1);
    if (norm)
      hipLaunchKernelGGL(k_scale_rows<double>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s,
                         (const double *)w.poly_b, (const double *)w.rsq, 1.0, w.poly_b, n, 1);
    std::string err;
    int id = pl.begin(PH_SETUP, 0.0, s);
    int r = poly_roots(G, w.plan, gen, w.d64, dinv, w.poly_b, o.cheb_degree, roots, &nroots,
                       w.poly_scratch, h->pinned_small, s, &err);
    pl.end(id, s);
    if (r != SPHX_OK) return set_err(h, r, err);
  }
  if (stats) {
    stats->max_degree = ds.max_deg;
    stats->avg_degree = n ? double(ds.sum_deg) / double(n) : 0.0;
    stats->graph_regular = (ds.max_deg * n <= 10 * ds.sum_deg) ? 1 : 0;
  }
  const double drop = o.drop_tol > 0 ? o.drop_tol
                                     : (std::is_same_v<T, float> ? 1e-10 : 1e-14);
  const ColMap idm = identity_map(m);
  DevStatus *hs = h->pinned_status;
  // ---- initial block and Rayleigh-Ritz
  T *Xi = reorder ? w.B2 : w.X;   // the initial block in the caller's order
  if (o.init == SPHX_INIT_USER) {
    SPHX_HIP(h, hipMemsetAsync(Xi, 0, sizeof(T) * n * ld, s));
    launch_copy_cols<T>(static_cast<const T *>(X0), m, Xi, ld, n, m, s);
  } else if (o.init == SPHX_INIT_PIECEWISE)
    launch_init_piecewise<T>(Xi, n, m, ld, s);
  else
    launch_init_random<T>(Xi, n, m, ld, o.seed, s);
  if (reorder) {
    SPHX_HIP(h, hipMemsetAsync(w.X, 0, sizeof(T) * n * ld, s));
    hipLaunchKernelGGL(k_gather_rows<T>, dim3(grid_for((int64_t)n * m, 256, 4096)), dim3(256),
                       0, s, (const T *)Xi, ld, (const int32_t *)operm, w.X, ld, n, m);
  }
  if (norm)   // the initial block is given in y; x = D^-1/2 y
    hipLaunchKernelGGL(k_scale_rows<T>, dim3(grid_for((int64_t)n * ld, 256, 4096)), dim3(256),
                       0, s, (const T *)w.X, (const double *)w.rsq, 1.0, w.X, n, ld);
  tid = pl.begin(PH_SPMM, spmm_bytes(G, w.plan, m, vs, 2, 0), s);
  SPHX_TRY(vspmm_store<T>(G, w.plan, w.X, ld, m, EpiStoreP<T>{w.LX, ld}, s));
  pl.end(tid, s);
  ++calls;
  GramArgs ga{n, m, ld, idm, 0, 0, bdiag};
  ga.act.count = 0;
  tid = pl.begin(PH_GRAM, 0.0, s);
  SPHX_TRY(gram<T>(w.X, w.LX, nullptr, nullptr, nullptr, nullptr, ga, w.gram_partials,
                   kGramBlocks, w.gram_out, s));
  pl.end(tid, s);
  tid = pl.begin(PH_RR, 0.0, s);
  launch_rr(w.gram_out, RRArgs{m, m, m, drop}, w.Y, w.theta, w.status, s);
  pl.end(tid, s);
  UpdateArgs ua{n, m, ld, idm, 0, 0};
  ua.act.count = 0;
  tid = pl.begin(PH_UPDATE, 0.0, s);
  SPHX_TRY(launch_update<T>(w.X, nullptr, w.P, nullptr, nullptr, w.Y, ua, s));
  pl.end(tid, s);
  const bool jac = o.precond == SPHX_PRECOND_JACOBI;
  auto residual = [&]() -> int {
    int nb = 0;
    EpiResidualP<T> er{w.LX, jac ? w.B1 : w.R, ld, w.theta, w.d64, gen ? 1 : 0, jac ? 1 : 0};
    int id = pl.begin(PH_SPMM, spmm_bytes(G, w.plan, m, vs, 3, 1), s);
    SPHX_TRY(vspmm_residual<T>(G, w.plan, w.X, ld, m, er, w.norm_partials, &nb, s));
    pl.end(id, s);
    ++calls;
    id = pl.begin(PH_OTHER, 0.0, s);
    launch_finalize(w.norm_partials, nb, m, w.theta, o.tol, o.locking, w.status, s);
    pl.end(id, s);
    SPHX_HIP(h, hipMemcpyAsync(hs, w.status, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    SPHX_HIP(h, hipStreamSynchronize(s));
    return SPHX_OK;
  };
  SPHX_TRY(residual());
  if (hs->breakdown)
    return set_err(h, SPHX_E_BREAKDOWN, "initial block is rank deficient");
  // ---- iterations
  int it = 0, restarts = 0;
  bool have_p = false;
  // FP32 stagnation watch (see sphx_options.promote_window)
  const int window = o.promote_window == 0 ? 100 : o.promote_window;
  const bool watch = std::is_same_v<T, float> && o.promote_window >= 0 && stalled;
  auto worst_active = [&]() {
    double r = 0.0;
    for (int q = 0; q < hs->nact; ++q) r = std::max(r, hs->rho[hs->act[q]]);
    return r;
  };
  int ref_nact = hs->nact, ref_it = 0;
  double ref_rho = worst_active();
  if (stalled) *stalled = false;
  while (hs->nact > 0 && it < o.max_iter) {
    ColMap act;
    act.count = hs->nact;
    for (int q = 0; q < kMaxNev; ++q) act.col[q] = q < hs->nact ? hs->act[q] : 0;
    T *H = w.B1;
    pcols += act.count;
    if (o.precond == SPHX_PRECOND_CHEBYSHEV) {
      SPHX_TRY(cheb_apply<T>(h, G, w.plan, m, ld, act, w.R, w.B1, w.B2, w.R, ck, dinv, s, &H,
                             &calls, &pcalls));
    } else if (o.precond == SPHX_PRECOND_GMRES) {
      SPHX_TRY(poly_apply<T>(h, G, w.plan, m, ld, act, w.R, w.B1, w.B2, w.R, roots, nroots,
                             dinv, s, &H, &calls, &pcalls));
    } else if (o.precond == SPHX_PRECOND_NONE) {
      H = w.R;
    }
    tid = pl.begin(PH_SPMM, spmm_bytes(G, w.plan, act.count, vs, 2, 0), s);
    SPHX_TRY(vspmm_store<T>(G, w.plan, H, ld, m, EpiStoreP<T>{w.LH, ld}, s));
    pl.end(tid, s);
    ++calls;
    GramArgs gb{n, m, ld, act, 1, have_p ? 1 : 0, bdiag};
    tid = pl.begin(PH_GRAM, 0.0, s);
    SPHX_TRY(gram<T>(w.X, w.LX, H, w.LH, w.P, w.LP, gb, w.gram_partials, kGramBlocks,
                     w.gram_out, s));
    pl.end(tid, s);
    const int na = act.count;
    const int wdt = m + na + (have_p ? na : 0);
    tid = pl.begin(PH_RR, 0.0, s);
    launch_rr(w.gram_out, RRArgs{m, wdt, have_p ? m + na : wdt, drop}, w.Y, w.theta,
              w.status, s);
    pl.end(tid, s);
    UpdateArgs ub{n, m, ld, act, 1, have_p ? 1 : 0};
    tid = pl.begin(PH_UPDATE, 0.0, s);
    // L P is carried along as L H y + L P z, except in FP32 near its rounding
    // floor, where it is formed by a product: the combination keeps the
    // absolute rounding of the stored FP32 products of earlier steps while P
    // shrinks, and once P is rescaled in the Rayleigh-Ritz step that error
    // dominates its projected entries (converged columns then diverged near
    // the tolerance).  Near the floor: 2^-24 ||L|| / theta_1 (the relative
    // residual of a rounded eigenvector at most, theta_1 the smallest
    // non-trivial Ritz value) above a tenth of the tolerance.
    bool lp_product = false;
    if constexpr (std::is_same_v<T, float>) {
      const double th1 = hs->theta[m > 1 ? 1 : 0];
      lp_product = !(th1 > 0.0) || 0x1p-24 * l_norm / th1 > 0.1 * o.tol;
    }
    SPHX_TRY(launch_update<T>(w.X, H, w.P, w.LH, lp_product ? nullptr : w.LP, w.Y, ub, s));
    pl.end(tid, s);
    if (lp_product) {
      tid = pl.begin(PH_SPMM, spmm_bytes(G, w.plan, m, vs, 2, 0), s);
      SPHX_TRY(vspmm_store<T>(G, w.plan, w.P, ld, m, EpiStoreP<T>{w.LP, ld}, s));
      pl.end(tid, s);
      ++calls;
    }
    have_p = true;
    // Jacobi writes the next H into B1, which held this iteration's H (consumed
    // by the update above); Chebyshev and no preconditioner write R.
    SPHX_TRY(residual());
    ++it;
    restarts += hs->restarted;
    if (hs->breakdown)
      return set_err(h, SPHX_E_BREAKDOWN,
                     "Rayleigh-Ritz basis rank deficient even without the P block");
    if (watch && hs->nact > 0) {
      const double wr = worst_active();
      if (hs->nact < ref_nact || wr < 0.7 * ref_rho) {
        ref_nact = hs->nact;
        ref_rho = wr;
        ref_it = it;
      } else if (it - ref_it >= window) {
        *stalled = true;
        break;
      }
    }
  }
  *hit_max = hs->nact > 0 && !(stalled && *stalled);
  if (iterations) *iterations = it;
  // ---- final FP64 residual check and normalisation
  double *X64 = reinterpret_cast<double *>(w.X);
  double *LX64 = reinterpret_cast<double *>(w.LX);
  if constexpr (std::is_same_v<T, float>) {
    launch_convert<float, double>(w.X, w.X64, n * ld, s);
    X64 = w.X64;
    LX64 = w.LX64;
    SPHX_TRY(vspmm_store<double>(G, w.plan, X64, ld, m, EpiStoreP<double>{LX64, ld}, s));
    ++calls;
  }
  int rb = (int)grid_for(n, 256 / ld, kRqBlocks);
  launch_rq_partials<double>(X64, LX64, n, m, ld, bdiag, w.rq_partials, rb, s);
  launch_sum_partials(w.rq_partials, rb, m, w.rq_sums, s);
  double sums[2 * kMaxNev];
  SPHX_HIP(h, hipMemcpyAsync(sums, w.rq_sums, sizeof(sums), hipMemcpyDeviceToHost, s));
  SPHX_HIP(h, hipStreamSynchronize(s));
  double th[kMaxNev];
  for (int c = 0; c < m; ++c) th[c] = sums[kMaxNev + c] > 0 ? sums[c] / sums[kMaxNev + c] : 0;
  SPHX_HIP(h, hipMemcpyAsync(w.theta, th, sizeof(double) * m, hipMemcpyHostToDevice, s));
  launch_res_partials<double>(X64, LX64, n, m, ld, bdiag, w.theta, w.rq_partials, rb, s);
  launch_sum_partials(w.rq_partials, rb, m, w.res_sums, s);
  double rs[2 * kMaxNev];
  SPHX_HIP(h, hipMemcpyAsync(rs, w.res_sums, sizeof(rs), hipMemcpyDeviceToHost, s));
  SPHX_HIP(h, hipStreamSynchronize(s));
  // ascending order of the Rayleigh quotients
  std::vector<int> perm(m);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return th[a] < th[b]; });
  double floor_th = m > 1 ? th[perm[1]] : th[perm[0]];
  double scale[kMaxNev];
  int nconv = 0;
  for (int q = 0; q < m; ++q) {
    int c = perm[q];
    eigvals[q] = th[c];
    double sc = std::max(th[c], floor_th);
    if (!(sc > 0)) sc = 1.0;
    double rho = rs[kMaxNev + c] > 0 ? std::sqrt(rs[c]) / (sc * std::sqrt(rs[kMaxNev + c]))
                                     : INFINITY;
    if (stats && q < 32) stats->rho[q] = rho;
    if (rho <= o.tol) ++nconv;
    scale[q] = rs[kMaxNev + c] > 0 ? 1.0 / std::sqrt(rs[kMaxNev + c]) : 1.0;
  }
  T *vo = reorder ? w.B2 : vecs_out;   // n x m in the solver's row order
  for (int q = 0; q < m; ++q)
    launch_copy_cols<T>(w.X + perm[q], ld, vo + q, m, n, 1, s);
  if (norm)   // y = D^1/2 x; ||y||_2 = ||x||_D, so the same scale normalises y
    hipLaunchKernelGGL(k_scale_rows<T>, dim3(grid_for((int64_t)n * m, 256, 4096)), dim3(256),
                       0, s, (const T *)vo, (const double *)w.sq, 1.0, vo, n, m);
  if (reorder)
    hipLaunchKernelGGL(k_gather_rows<T>, dim3(grid_for((int64_t)n * m, 256, 4096)), dim3(256),
                       0, s, (const T *)vo, m, (const int32_t *)oinv, vecs_out, m, n, m);
  SPHX_TRY(normalize_columns<T>(vecs_out, n, m, scale, w.norm_scratch, s));
  if (stats) {
    stats->iterations = it;
    stats->converged = nconv;
    stats->restarts = restarts;
    stats->spmm_calls = calls;
    stats->precond_calls = pcalls;
    stats->precond_cols = pcols;
    stats->col_index_bytes = w.plan.dcol ? 2 : 4;
    stats->ms_total = tall.stop(s);
  } else {
    SPHX_HIP(h, hipStreamSynchronize(s));
  }
  return SPHX_OK;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

const char *sphx_status_string(int status) {
  if (status == SPHX_NOT_CONVERGED) return "not converged (max_iter reached)";
  if (status <= 0 && status >= -8) return kStatusText[-status];
  return "unknown status";
}

int sphx_create(sphx_handle **out, int device, void *stream) {
  if (!out) return SPHX_E_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return SPHX_E_INVALID_ARG;
  auto *h = new sphx_handle();
  h->device = device;
  h->stream = static_cast<hipStream_t>(stream);
  if (hipSetDevice(device) != hipSuccess ||
      hipHostMalloc((void **)&h->pinned_status, sizeof(DevStatus)) != hipSuccess ||
      hipHostMalloc(&h->pinned_small, kPinnedSmallBytes) != hipSuccess ||
      hipMalloc((void **)&h->flags_dev, 256) != hipSuccess ||
      resolve_noalloc_scratch(device) != SPHX_OK) {
    if (h->pinned_status) (void)hipHostFree(h->pinned_status);
    if (h->pinned_small) (void)hipHostFree(h->pinned_small);
    if (h->flags_dev) (void)hipFree(h->flags_dev);
    delete h;
    return SPHX_E_HIP;
  }
  *out = h;
  return SPHX_OK;
}

int sphx_destroy(sphx_handle *h) {
  if (!h) return SPHX_E_INVALID_ARG;
  (void)hipSetDevice(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  if (h->ws_own) (void)hipFree(h->ws_own);
  if (h->flags_dev) (void)hipFree(h->flags_dev);
  if (h->pinned_status) (void)hipHostFree(h->pinned_status);
  if (h->pinned_small) (void)hipHostFree(h->pinned_small);
  delete h;
  return SPHX_OK;
}

int sphx_set_stream(sphx_handle *h, void *stream) {
  if (!h) return SPHX_E_INVALID_ARG;
  h->stream = static_cast<hipStream_t>(stream);
  return SPHX_OK;
}

const char *sphx_last_error(const sphx_handle *h) { return h ? h->err.c_str() : ""; }

int sphx_set_timing(sphx_handle *h, int on) {
  if (!h) return SPHX_E_INVALID_ARG;
  h->timing = on ? 1 : 0;
  return SPHX_OK;
}

int sphx_num_eigenvectors(int K) {
  if (K < 1) return -1;
  int d = 0;
  while (K) { ++d; K >>= 1; }
  return d;
}

void sphx_options_default(sphx_options *o, int regular, int precond) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precond = precond;
  const bool poly = precond == SPHX_PRECOND_CHEBYSHEV || precond == SPHX_PRECOND_GMRES;
  o->problem = regular ? SPHX_COMBINATORIAL : (poly ? SPHX_NORMALIZED : SPHX_GENERALIZED);
  o->tol = regular ? 1e-3 : 1e-2;
  o->init = regular ? SPHX_INIT_RANDOM : SPHX_INIT_PIECEWISE;
  o->cheb_degree = 25;
  o->cheb_ratio = 1000.0;
  o->precision = SPHX_FP64;
  o->max_iter = 10000;
  o->seed = 0x5eed;
  o->locking = 1;
  o->drop_tol = 0.0;
  o->promote_window = 0;
  o->reorder = 1;
}

int sphx_graph_create(sphx_handle *h, int64_t n, int64_t nnz, const void *row_ptr,
                      int row_ptr_is_64, const int32_t *col, const void *w, int w_dtype,
                      const int32_t *vwgt, uint32_t flags, sphx_graph **out) {
  if (!h || !out) return SPHX_E_INVALID_ARG;
  *out = nullptr;
  if (n < 1 || n >= (int64_t(1) << 31) || nnz < 0 || !row_ptr || (nnz > 0 && !col))
    return set_err(h, SPHX_E_INVALID_ARG, "bad sizes or null pointers");
  if (!row_ptr_is_64 && nnz >= (int64_t(1) << 31))
    return set_err(h, SPHX_E_INVALID_ARG, "nnz needs an int64 row_ptr");
  if (w_dtype != SPHX_UNIT && w_dtype != SPHX_F32 && w_dtype != SPHX_F64)
    return set_err(h, SPHX_E_INVALID_ARG, "bad weight dtype");
  if ((w_dtype == SPHX_UNIT) != (w == nullptr))
    return set_err(h, SPHX_E_INVALID_ARG, "weights pointer and dtype disagree");
  if (hipSetDevice(h->device) != hipSuccess) return SPHX_E_HIP;
  auto *g = new sphx_graph();
  g->h = h;
  g->n = n;
  g->nnz = nnz;
  g->rowptr = row_ptr;
  g->rp64 = row_ptr_is_64 ? 1 : 0;
  g->col = col;
  g->w = w;
  g->wdt = w_dtype;
  g->vwgt = vwgt;
  if (!(flags & SPHX_SKIP_VALIDATE)) {
    // the flags live in the handle's own 256 device bytes (no allocation)
    int st = validate_graph(g, h->stream, h->flags_dev, static_cast<int *>(h->pinned_small));
    if (st != SPHX_OK) {
      delete g;
      return st;
    }
  }
  *out = g;
  return SPHX_OK;
}

int sphx_graph_destroy(sphx_graph *g) {
  if (!g) return SPHX_E_INVALID_ARG;
  delete g;
  return SPHX_OK;
}

int sphx_graph_info(sphx_handle *h, sphx_graph *g, int *is_regular, int64_t *max_degree,
                    double *avg_degree) {
  if (!h || !g) return SPHX_E_INVALID_ARG;
  size_t need = align_up(sizeof(double) * g->n, 256) + 4 * kDegBlocksMax * sizeof(double) + 512;
  char *ws = nullptr;
  SPHX_TRY(get_workspace(h, need, &ws));
  DegreeStats ds;
  SPHX_TRY(compute_degrees(g, reinterpret_cast<double *>(ws), nullptr,
                           ws + align_up(sizeof(double) * g->n, 256), &ds, h->pinned_small,
                           h->stream));
  if (is_regular) *is_regular = (ds.max_deg * g->n <= 10 * ds.sum_deg) ? 1 : 0;
  if (max_degree) *max_degree = ds.max_deg;
  if (avg_degree) *avg_degree = double(ds.sum_deg) / double(g->n);
  return SPHX_OK;
}

static int poly_degree_of(const sphx_options *o) {
  return o->precond == SPHX_PRECOND_GMRES ? o->cheb_degree : 0;
}

// Bytes of the FP32 solve's layout; a MIXED solve keeps, after it, room for
// an FP64 continuation (its own layout plus the n x nev initial and result
// blocks), laid out from this offset.
static size_t fp32_layout_bytes(sphx_graph *g, int nev, int K, bool split, int poly_degree,
                                size_t ord_b) {
  Arena a;
  a.count_only = true;
  SolveWs<float> w;
  layout(a, w, g->n, nev, K, plan_bytes(g), split, poly_degree, ord_b);
  return align_up(a.off, 256);
}

// room for the degree-ordered copy of the graph: while the degrees are not
// known yet, whenever the option asks for it
static size_t ord_bytes_of(sphx_graph *g, const sphx_options *o) {
  const bool may = o->reorder && (!g->stats_valid || g->max_deg > kUnbinnedMaxDeg);
  return may ? degree_order_bytes(g) : 0;
}

static size_t solve_bytes(sphx_graph *g, int nev, int precision, int K, bool split,
                          int poly_degree, size_t ord_b) {
  Arena a;
  a.count_only = true;
  size_t pb = plan_bytes(g);
  SolveWs<double> w;
  if (precision == SPHX_MIXED) {
    a.off = fp32_layout_bytes(g, nev, K, split, poly_degree, ord_b);
    layout(a, w, g->n, nev, K, pb, false, poly_degree, ord_b);
    (void)a.take<double>((size_t)g->n * nev * 2);
  } else {
    layout(a, w, g->n, nev, K, pb, split, poly_degree, ord_b);
  }
  return a.off + 4096;
}

int sphx_workspace_size(sphx_handle *h, sphx_graph *g, int nev, const sphx_options *opt,
                        size_t *bytes) {
  if (!h || !g || !opt || !bytes || nev < 1 || nev > kMaxNev) return SPHX_E_INVALID_ARG;
  // the largest K with floor(log2 K) + 1 = nev: the split and quality scratch
  // grow with K, so this bounds every partition into d = nev coordinates
  int K = (1 << nev) - 1;
  size_t a = solve_bytes(g, nev, opt->precision, K, true, poly_degree_of(opt),
                         ord_bytes_of(g, opt));
  size_t b = adjoint_scratch_bytes(g->n, nev) + plan_bytes(g) + sizeof(double) * 2 * g->n +
             4096;
  *bytes = std::max(a, b);
  return SPHX_OK;
}

int sphx_set_workspace(sphx_handle *h, void *ptr, size_t bytes) {
  if (!h) return SPHX_E_INVALID_ARG;
  h->ws_user = ptr;
  h->ws_user_bytes = ptr ? bytes : 0;
  return SPHX_OK;
}

int sphx_workspace_owned(const sphx_handle *h, size_t *bytes) {
  if (!h || !bytes) return SPHX_E_INVALID_ARG;
  *bytes = h->ws_own_bytes;
  return SPHX_OK;
}

int sphx_workspace_release(sphx_handle *h) {
  if (!h) return SPHX_E_INVALID_ARG;
  if (h->ws_own) {
    if (hipSetDevice(h->device) != hipSuccess) return SPHX_E_HIP;
    if (h->stream) SPHX_HIP(h, hipStreamSynchronize(h->stream));
    else SPHX_HIP(h, hipDeviceSynchronize());
    SPHX_HIP(h, hipFree(h->ws_own));
  }
  h->ws_own = nullptr;
  h->ws_own_bytes = 0;
  return SPHX_OK;
}

int sphx_laplacian_apply(sphx_handle *h, sphx_graph *g, int problem, int m, int dtype,
                         const void *X, void *Y) {
  if (!h || !g || !X || !Y || m < 1 || m > kMaxNev ||
      (dtype != SPHX_F32 && dtype != SPHX_F64) ||
      (problem != SPHX_COMBINATORIAL && problem != SPHX_GENERALIZED &&
       problem != SPHX_NORMALIZED))
    return SPHX_E_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return SPHX_E_HIP;
  hipStream_t s = h->stream;
  const bool norm = problem == SPHX_NORMALIZED;
  const size_t blk = (size_t)g->n * m * bytes_of(dtype);
  char *ws = nullptr;
  size_t need = plan_bytes(g) + 3 * align_up(sizeof(double) * g->n, 256) +
                align_up(4 * kDegBlocksMax * sizeof(double), 256) +
                (norm ? align_up(blk, 256) : 0) + 1024;
  SPHX_TRY(get_workspace(h, need, &ws));
  Arena a;
  a.base = ws;
  double *d64 = a.take<double>(g->n);
  double *sq = a.take<double>(g->n);
  double *rsq = a.take<double>(g->n);
  double *degs = a.take<double>(4 * kDegBlocksMax);
  char *tmp = norm ? a.take<char>(blk) : nullptr;
  DegreeStats ds;
  SPHX_TRY(compute_degrees(g, d64, nullptr, degs, &ds, h->pinned_small, s));
  SpmmPlan plan;
  SPHX_TRY(build_plan(g, a, &plan, ds, h->pinned_small, s));
  const int64_t n = g->n;
  const void *src = X;
  if (norm) {
    // L_N X = D^-1/2 (L_C (D^-1/2 X))
    if (!(ds.min_wdeg > 0)) return set_err(h, SPHX_E_INVALID_ARG, "isolated vertex");
    hipLaunchKernelGGL(k_sqrt_pair, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, d64, sq, rsq,
                       n);
    if (dtype == SPHX_F32)
      hipLaunchKernelGGL(k_scale_rows<float>, dim3(grid_for(n * m, 256, 4096)), dim3(256), 0, s,
                         (const float *)X, (const double *)rsq, 1.0, (float *)tmp, n, m);
    else
      hipLaunchKernelGGL(k_scale_rows<double>, dim3(grid_for(n * m, 256, 4096)), dim3(256), 0,
                         s, (const double *)X, (const double *)rsq, 1.0, (double *)tmp, n, m);
    src = tmp;
  }
  ColMap cm = identity_map(m);
  // rows that are whole 16-byte vectors take the vector-row kernels
  const bool vec = (m * bytes_of(dtype)) % 16 == 0 && ((uintptr_t)src % 16) == 0 &&
                   ((uintptr_t)Y % 16) == 0;
  int r;
  if (dtype == SPHX_F32)
    r = vec ? vspmm_store<float>(g, plan, (const float *)src, m, m,
                                 EpiStoreP<float>{(float *)Y, m}, s)
            : spmm_store<float>(g, plan, (const float *)src, m, cm,
                                EpiStoreP<float>{(float *)Y, m}, s);
  else
    r = vec ? vspmm_store<double>(g, plan, (const double *)src, m, m,
                                  EpiStoreP<double>{(double *)Y, m}, s)
            : spmm_store<double>(g, plan, (const double *)src, m, cm,
                                 EpiStoreP<double>{(double *)Y, m}, s);
  if (r != SPHX_OK || !norm) return r;
  if (dtype == SPHX_F32)
    hipLaunchKernelGGL(k_scale_rows<float>, dim3(grid_for(n * m, 256, 4096)), dim3(256), 0, s,
                       (const float *)Y, (const double *)rsq, 1.0, (float *)Y, n, m);
  else
    hipLaunchKernelGGL(k_scale_rows<double>, dim3(grid_for(n * m, 256, 4096)), dim3(256), 0, s,
                       (const double *)Y, (const double *)rsq, 1.0, (double *)Y, n, m);
  SPHX_HIP(h, hipGetLastError());
  return SPHX_OK;
}

int sphx_precond_apply(sphx_handle *h, sphx_graph *g, const sphx_options *o, int m,
                       int dtype, const void *R, void *H) {
  if (!h || !g || !valid_options(o) || !R || !H || m < 1 || m > kMaxNev ||
      (dtype != SPHX_F32 && dtype != SPHX_F64))
    return SPHX_E_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return SPHX_E_HIP;
  hipStream_t s = h->stream;
  size_t blk = (size_t)g->n * m * bytes_of(dtype);
  size_t need = plan_bytes(g) + 4 * align_up(sizeof(double) * g->n, 256) +
                3 * align_up(blk, 256) + 4 * kDegBlocksMax * sizeof(double) + 4096;
  char *ws = nullptr;
  SPHX_TRY(get_workspace(h, need, &ws));
  Arena a;
  a.base = ws;
  double *d64 = a.take<double>(g->n);
  double *dinv = a.take<double>(g->n);
  double *sq = a.take<double>(g->n);
  double *rsq = a.take<double>(g->n);
  char *b0 = a.take<char>(blk);
  double *degs = a.take<double>(4 * kDegBlocksMax);
  char *b1 = a.take<char>(blk);
  char *b2 = a.take<char>(blk);
  DegreeStats ds;
  SPHX_TRY(compute_degrees(g, d64, nullptr, degs, &ds, h->pinned_small, s));
  SpmmPlan plan;
  SPHX_TRY(build_plan(g, a, &plan, ds, h->pinned_small, s));
  const int64_t n = g->n;
  const bool norm = o->problem == SPHX_NORMALIZED;
  if (o->precond == SPHX_PRECOND_NONE || (norm && o->precond == SPHX_PRECOND_JACOBI)) {
    // diag(L_N) = I: Jacobi is the identity for the normalized problem
    SPHX_HIP(h, hipMemcpyAsync(H, R, blk, hipMemcpyDeviceToDevice, s));
  } else if (o->precond == SPHX_PRECOND_JACOBI) {
    if (!(ds.min_wdeg > 0)) return set_err(h, SPHX_E_INVALID_ARG, "isolated vertex");
    if (dtype == SPHX_F32)
      hipLaunchKernelGGL(k_jacobi<float>, dim3(grid_for(n * m, 256, 4096)), dim3(256), 0, s,
                         (const float *)R, d64, (float *)H, n, m);
    else
      hipLaunchKernelGGL(k_jacobi<double>, dim3(grid_for(n * m, 256, 4096)), dim3(256), 0, s,
                         (const double *)R, d64, (double *)H, n, m);
  } else if (o->precond == SPHX_PRECOND_GMRES) {
    return set_err(h, SPHX_E_INVALID_ARG,
                   "the GMRES polynomial is applied with sphx_poly_apply (roots from "
                   "sphx_poly_roots)");
  } else {
    const bool gen = o->problem != SPHX_COMBINATORIAL;
    if (gen && !(ds.min_wdeg > 0)) return set_err(h, SPHX_E_INVALID_ARG, "isolated vertex");
    if (norm) {
      // p(L_N) r = D^1/2 [p(D^-1 L_C) D^-1] (D^1/2 r): the generalized iteration
      // on D^1/2 r, scaled by D^1/2 at the end
      hipLaunchKernelGGL(k_sqrt_pair, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, d64, sq,
                         rsq, n);
      if (dtype == SPHX_F32)
        hipLaunchKernelGGL(k_scale_rows<float>, dim3(grid_for(n * m, 256, 4096)), dim3(256), 0,
                           s, (const float *)R, (const double *)sq, 1.0, (float *)b0, n, m);
      else
        hipLaunchKernelGGL(k_scale_rows<double>, dim3(grid_for(n * m, 256, 4096)), dim3(256),
                           0, s, (const double *)R, (const double *)sq, 1.0, (double *)b0, n, m);
      R = b0;
    }
    double hi = gen ? 2.0 : 2.0 * ds.max_wdeg;
    ChebCoef ck = cheb_coef(o->cheb_degree, hi / o->cheb_ratio, hi);
    const double *dv = nullptr;
    if (gen) {
      hipLaunchKernelGGL(k_inverse, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, d64, dinv, n);
      dv = dinv;
    }
    ColMap cm = identity_map(m);
    int64_t calls = 0, pcalls = 0;
    h->plog.reset();
    h->plog.on = false;
    const double *post = norm ? sq : nullptr;
    if (dtype == SPHX_F32) {
      float *res = nullptr;
      SPHX_TRY(cheb_apply<float>(h, g, plan, m, m, cm, (const float *)R, (float *)b1,
                                 (float *)b2, nullptr, ck, dv, s, &res, &calls, &pcalls));
      if (post)
        hipLaunchKernelGGL(k_scale_rows<float>, dim3(grid_for(n * m, 256, 4096)), dim3(256), 0,
                           s, (const float *)res, post, 1.0, (float *)H, n, m);
      else
        SPHX_HIP(h, hipMemcpyAsync(H, res, blk, hipMemcpyDeviceToDevice, s));
    } else {
      double *res = nullptr;
      SPHX_TRY(cheb_apply<double>(h, g, plan, m, m, cm, (const double *)R, (double *)b1,
                                  (double *)b2, nullptr, ck, dv, s, &res, &calls, &pcalls));
      if (post)
        hipLaunchKernelGGL(k_scale_rows<double>, dim3(grid_for(n * m, 256, 4096)), dim3(256),
                           0, s, (const double *)res, post, 1.0, (double *)H, n, m);
      else
        SPHX_HIP(h, hipMemcpyAsync(H, res, blk, hipMemcpyDeviceToDevice, s));
    }
  }
  SPHX_HIP(h, hipGetLastError());
  return SPHX_OK;
}

int sphx_poly_roots(sphx_handle *h, sphx_graph *g, int problem, int degree, const double *b,
                    double *roots, int *nroots) {
  if (!h || !g || !b || !roots || !nroots || degree < 1 || degree + 1 > kMaxW ||
      (problem != SPHX_COMBINATORIAL && problem != SPHX_GENERALIZED &&
       problem != SPHX_NORMALIZED))
    return SPHX_E_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return SPHX_E_HIP;
  hipStream_t s = h->stream;
  const int64_t n = g->n;
  size_t need = plan_bytes(g) + 5 * align_up(sizeof(double) * n, 256) +
                align_up(4 * kDegBlocksMax * sizeof(double), 256) +
                poly_scratch_bytes(n, degree) + 4096;
  char *ws = nullptr;
  SPHX_TRY(get_workspace(h, need, &ws));
  Arena a;
  a.base = ws;
  double *d64 = a.take<double>(n);
  double *dinv = a.take<double>(n);
  double *sq = a.take<double>(n);
  double *rsq = a.take<double>(n);
  double *bx = a.take<double>(n);
  double *degs = a.take<double>(4 * kDegBlocksMax);
  char *scr = a.take<char>(poly_scratch_bytes(n, degree));
  DegreeStats ds;
  SPHX_TRY(compute_degrees(g, d64, nullptr, degs, &ds, h->pinned_small, s));
  SpmmPlan plan;
  SPHX_TRY(build_plan(g, a, &plan, ds, h->pinned_small, s));
  const bool gen = problem != SPHX_COMBINATORIAL;
  if (gen && !(ds.min_wdeg > 0)) return set_err(h, SPHX_E_INVALID_ARG, "isolated vertex");
  hipLaunchKernelGGL(k_inverse, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, d64, dinv, n);
  const double *bb = b;
  if (problem == SPHX_NORMALIZED) {   // b is given in y; x = D^-1/2 y
    hipLaunchKernelGGL(k_sqrt_pair, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, d64, sq, rsq,
                       n);
    hipLaunchKernelGGL(k_scale_rows<double>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, b,
                       (const double *)rsq, 1.0, bx, n, 1);
    bb = bx;
  }
  std::string err;
  int r = poly_roots(g, plan, gen, d64, gen ? dinv : nullptr, bb, degree, roots, nroots, scr,
                     h->pinned_small, s, &err);
  if (r != SPHX_OK) return set_err(h, r, err);
  return SPHX_OK;
}

int sphx_poly_apply(sphx_handle *h, sphx_graph *g, int problem, int nroots,
                    const double *roots, int m, int dtype, const void *R, void *H) {
  if (!h || !g || !roots || !R || !H || nroots < 1 || nroots > kMaxW || m < 1 ||
      m > kMaxNev || (dtype != SPHX_F32 && dtype != SPHX_F64) ||
      (problem != SPHX_COMBINATORIAL && problem != SPHX_GENERALIZED &&
       problem != SPHX_NORMALIZED))
    return SPHX_E_INVALID_ARG;
  for (int i = 0; i < nroots; ++i)
    if (!(roots[i] != 0.0) || !std::isfinite(roots[i]))
      return set_err(h, SPHX_E_INVALID_ARG, "polynomial roots must be finite and non-zero");
  if (hipSetDevice(h->device) != hipSuccess) return SPHX_E_HIP;
  hipStream_t s = h->stream;
  const int64_t n = g->n;
  const int es = bytes_of(dtype);
  const int wd = std::max(m, compact_ld(m));   // widest row the buffers must hold
  const size_t blk = (size_t)n * wd * es;
  size_t need = plan_bytes(g) + 4 * align_up(sizeof(double) * n, 256) +
                align_up(4 * kDegBlocksMax * sizeof(double), 256) + 4 * align_up(blk, 256) +
                4096;
  char *ws = nullptr;
  SPHX_TRY(get_workspace(h, need, &ws));
  Arena a;
  a.base = ws;
  double *d64 = a.take<double>(n);
  double *dinv = a.take<double>(n);
  double *sq = a.take<double>(n);
  double *rsq = a.take<double>(n);
  double *degs = a.take<double>(4 * kDegBlocksMax);
  char *b0 = a.take<char>(blk);
  char *b1 = a.take<char>(blk);
  char *b2 = a.take<char>(blk);
  char *b3 = a.take<char>(blk);
  DegreeStats ds;
  SPHX_TRY(compute_degrees(g, d64, nullptr, degs, &ds, h->pinned_small, s));
  SpmmPlan plan;
  SPHX_TRY(build_plan(g, a, &plan, ds, h->pinned_small, s));
  const bool gen = problem != SPHX_COMBINATORIAL;
  const bool norm = problem == SPHX_NORMALIZED;
  if (gen && !(ds.min_wdeg > 0)) return set_err(h, SPHX_E_INVALID_ARG, "isolated vertex");
  hipLaunchKernelGGL(k_inverse, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, d64, dinv, n);
  if (norm)
    hipLaunchKernelGGL(k_sqrt_pair, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, d64, sq, rsq,
                       n);
  ColMap cm = identity_map(m);
  int64_t calls = 0, pcalls = 0;
  h->plog.reset();
  h->plog.on = false;
  auto go = [&](auto tag) -> int {
    using T = decltype(tag);
    const T *src = static_cast<const T *>(R);
    if (norm) {   // p(L_N) r = D^1/2 [p(D^-1 L) D^-1] (D^1/2 r)
      hipLaunchKernelGGL(k_scale_rows<T>, dim3(grid_for(n * m, 256, 4096)), dim3(256), 0, s,
                         src, (const double *)sq, 1.0, (T *)b0, n, m);
      src = (const T *)b0;
    }
    T *res = nullptr;
    SPHX_TRY(poly_apply<T>(h, g, plan, m, m, cm, src, (T *)b1, (T *)b2, (T *)b3, roots, nroots,
                           gen ? dinv : nullptr, s, &res, &calls, &pcalls));
    if (norm)
      hipLaunchKernelGGL(k_scale_rows<T>, dim3(grid_for(n * m, 256, 4096)), dim3(256), 0, s,
                         (const T *)res, (const double *)sq, 1.0, (T *)H, n, m);
    else
      SPHX_HIP(h, hipMemcpyAsync(H, res, sizeof(T) * n * m, hipMemcpyDeviceToDevice, s));
    return SPHX_OK;
  };
  SPHX_TRY(dtype == SPHX_F32 ? go(float{}) : go(double{}));
  SPHX_HIP(h, hipGetLastError());
  return SPHX_OK;
}

static int eigensolve_impl(sphx_handle *h, sphx_graph *g, int nev, const sphx_options *o,
                           const void *X0, double *eigvals, void *eigvecs, int K,
                           int32_t *part, double *cut, double *imbalance,
                           sphx_stats *stats) {
  if (!h || !g || !valid_options(o) || !eigvals) return SPHX_E_INVALID_ARG;
  if (nev < 1 || nev > kMaxNev || nev >= g->n)
    return set_err(h, SPHX_E_INVALID_ARG, "need 1 <= nev <= 16 and nev < n");
  if (o->init == SPHX_INIT_USER && !X0)
    return set_err(h, SPHX_E_INVALID_ARG, "SPHX_INIT_USER needs X0");
  if (hipSetDevice(h->device) != hipSuccess) return SPHX_E_HIP;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  h->plog.reset();
  h->plog.on = h->timing && stats;
  const bool split = part != nullptr;
  char *ws = nullptr;
  const size_t ord_b = ord_bytes_of(g, o);
  SPHX_TRY(get_workspace(h,
                         solve_bytes(g, nev, o->precision, std::max(K, 1), split,
                                     poly_degree_of(o), ord_b),
                         &ws));
  bool hit_max = false;
  int st;
  auto run = [&](auto tag) -> int {
    using T = decltype(tag);
    Arena a;
    a.base = ws;
    SolveWs<T> w;
    layout(a, w, g->n, nev, std::max(K, 1), plan_bytes(g), split, poly_degree_of(o), ord_b);
    const size_t used = align_up(a.off, 256);   // the FP64 continuation starts here
    T *vecs = eigvecs ? static_cast<T *>(eigvecs) : w.V;
    if (!vecs) return set_err(h, SPHX_E_INVALID_ARG, "eigvecs is NULL");
    bool stalled = false;
    int its = 0;
    SPHX_TRY(solve<T>(h, g, nev, *o, X0, eigvals, vecs, stats, w, ws, &hit_max, &stalled,
                      &its));
    if constexpr (std::is_same_v<T, float>) {
      if (stalled) {
        // continue in FP64 from the current vectors (their normalised form,
        // in y for the normalized problem, is exactly an initial block)
        Arena a64;
        a64.base = ws + used;
        SolveWs<double> w64;
        layout(a64, w64, g->n, nev, std::max(K, 1), plan_bytes(g), false,
               poly_degree_of(o), ord_b);
        double *x0 = a64.take<double>((size_t)g->n * nev);
        double *v64 = a64.take<double>((size_t)g->n * nev);
        launch_convert<float, double>(vecs, x0, (int64_t)g->n * nev, h->stream);
        sphx_options o64 = *o;
        o64.precision = SPHX_FP64;
        o64.init = SPHX_INIT_USER;
        o64.drop_tol = 0.0;
        o64.max_iter = std::max(1, o->max_iter - its);   // one budget for both parts
        sphx_stats s64;
        std::memset(&s64, 0, sizeof(s64));
        SPHX_TRY(solve<double>(h, g, nev, o64, x0, eigvals, v64, stats ? &s64 : nullptr, w64,
                               (char *)a64.base, &hit_max, nullptr, nullptr));
        launch_convert<double, float>(v64, vecs, (int64_t)g->n * nev, h->stream);
        if (stats) {
          stats->iterations += s64.iterations;
          stats->converged = s64.converged;
          stats->restarts += s64.restarts;
          for (int q = 0; q < 32; ++q) stats->rho[q] = s64.rho[q];
          stats->spmm_calls += s64.spmm_calls;
          stats->precond_calls += s64.precond_calls;
          stats->precond_cols += s64.precond_cols;
          stats->ms_total += s64.ms_total;
          stats->promoted = 1;
        }
      }
    }
    if (split) {
      Timer ts;
      if (stats) ts.start(h->stream);
      std::string err;
      int id = h->plog.begin(PH_SPLIT, 0.0, h->stream);
      int r = split_mj<T>(g, vecs + 1, nev, nev - 1, K, part, w.split_scratch,
                            h->pinned_small, h->stream, &err);
      h->plog.end(id, h->stream);
      if (r != SPHX_OK) return set_err(h, r, err);
      id = h->plog.begin(PH_QUALITY, 0.0, h->stream);
      r = quality(g, part, K, cut, imbalance, nullptr, w.quality_scratch, h->pinned_small,
                  h->stream, &err);
      h->plog.end(id, h->stream);
      if (r != SPHX_OK) return set_err(h, r, err);
      if (stats) stats->ms_total += ts.stop(h->stream);
    }
    return SPHX_OK;
  };
  st = o->precision == SPHX_MIXED ? run(float{}) : run(double{});
  if (st < 0) return st;
  if (stats && h->plog.on) {
    (void)hipStreamSynchronize(h->stream);
    double ms[PH_COUNT] = {0}, gb[PH_COUNT] = {0};
    for (auto &r : h->plog.recs) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) ms[r.phase] += t;
      gb[r.phase] += r.bytes * 1e-9;
    }
    stats->ms_setup = ms[PH_SETUP];
    stats->ms_spmm = ms[PH_SPMM];
    stats->ms_precond = ms[PH_PRECOND];
    stats->ms_gram = ms[PH_GRAM];
    stats->ms_rr = ms[PH_RR];
    stats->ms_update = ms[PH_UPDATE];
    stats->ms_split = ms[PH_SPLIT];
    stats->ms_quality = ms[PH_QUALITY];
    stats->gb_spmm = gb[PH_SPMM];
    stats->gb_precond = gb[PH_PRECOND];
  }
  if (hit_max)
    return set_err(h, SPHX_NOT_CONVERGED,
                   "max_iter reached before every relative residual met tol");
  return SPHX_OK;
}

int sphx_eigensolve(sphx_handle *h, sphx_graph *g, int nev, const sphx_options *o,
                    const void *X0, double *eigvals, void *eigvecs, sphx_stats *stats) {
  if (!eigvecs) return SPHX_E_INVALID_ARG;
  return eigensolve_impl(h, g, nev, o, X0, eigvals, eigvecs, 1, nullptr, nullptr, nullptr,
                         stats);
}

int sphx_partition(sphx_handle *h, sphx_graph *g, int K, const sphx_options *o,
                   const void *X0, double *eigvals, void *eigvecs, int32_t *part,
                   double *cut, double *imbalance, sphx_stats *stats) {
  if (!h || !g || !part) return SPHX_E_INVALID_ARG;
  if (K < 2 || K > g->n)
    return set_err(h, SPHX_E_INVALID_ARG, "need 2 <= K <= n");
  int d = sphx_num_eigenvectors(K);
  if (d > kMaxNev) return set_err(h, SPHX_E_INVALID_ARG, "K too large (d > 16)");
  return eigensolve_impl(h, g, d, o, X0, eigvals, eigvecs, K, part, cut, imbalance, stats);
}

int sphx_split(sphx_handle *h, sphx_graph *g, const void *coords, int ld, int ncoord,
               int dtype, int K, int32_t *part) {
  if (!h || !g || !coords || !part || ncoord < 1 || ld < ncoord ||
      (dtype != SPHX_F32 && dtype != SPHX_F64))
    return SPHX_E_INVALID_ARG;
  if (K < 1 || K > (1 << 30) || K > g->n)
    return set_err(h, SPHX_E_INVALID_ARG, "need 1 <= K <= n");
  if (hipSetDevice(h->device) != hipSuccess) return SPHX_E_HIP;
  char *ws = nullptr;
  SPHX_TRY(get_workspace(h, split_scratch_bytes(g->n, K), &ws));
  std::string err;
  int r = dtype == SPHX_F32
              ? split_mj<float>(g, (const float *)coords, ld, ncoord, K, part, ws,
                                  h->pinned_small, h->stream, &err)
              : split_mj<double>(g, (const double *)coords, ld, ncoord, K, part, ws,
                                   h->pinned_small, h->stream, &err);
  if (r != SPHX_OK) return set_err(h, r, err);
  return SPHX_OK;
}

int sphx_quality(sphx_handle *h, sphx_graph *g, const int32_t *part, int K, double *cut,
                 double *cut2x, double *imbalance, int64_t *part_weights) {
  if (!h || !g || !part || K < 1) return SPHX_E_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return SPHX_E_HIP;
  char *ws = nullptr;
  SPHX_TRY(get_workspace(h, quality_scratch_bytes(K), &ws));
  // the exact cut's fixed-point exponent needs the weight range (the
  // quality scratch holds the range pass's block partials)
  SPHX_TRY(weight_range(g, ws, h->pinned_small, h->stream));
  std::string err;
  double c = 0.0;
  int r = quality(g, part, K, &c, imbalance, part_weights, ws, h->pinned_small, h->stream, &err);
  if (r != SPHX_OK) return set_err(h, r, err);
  if (cut) *cut = c;
  if (cut2x) *cut2x = 2.0 * c;
  return SPHX_OK;
}

int sphx_quality_noalloc(sphx_handle *h, sphx_graph *g, const int32_t *part, int K,
                         double *cut, double *cut2x, double *imbalance,
                         int64_t *part_weights) {
  if (!h || !g || !part || K < 1) return SPHX_E_INVALID_ARG;
  if (K > kNoAllocMaxK || quality_scratch_bytes(K) > kNoAllocScratchBytes)
    return set_err(h, SPHX_E_WORKSPACE,
                   "sphx_quality_noalloc: K above its fixed scratch limit of 65536 parts");
  if (hipSetDevice(h->device) != hipSuccess) return SPHX_E_HIP;
  char *ws = static_cast<char *>(noalloc_scratch_ptr(h->device));
  if (!ws) return set_err(h, SPHX_E_HIP, "sphx_quality_noalloc: device scratch not resolved");
  SPHX_TRY(weight_range(g, ws, h->pinned_small, h->stream));
  std::string err;
  double c = 0.0;
  int r = quality(g, part, K, &c, imbalance, part_weights, ws, h->pinned_small, h->stream, &err);
  if (r != SPHX_OK) return set_err(h, r, err);
  if (cut) *cut = c;
  if (cut2x) *cut2x = 2.0 * c;
  return SPHX_OK;
}

int sphx_refine(sphx_handle *h, sphx_graph *g, int K, int32_t *part, double eps,
                int max_passes, double *cut, double *imbalance, int *passes,
                int64_t *moves) {
  if (!h || !g || !part || K < 1 || max_passes < 0 || !(eps >= 0.0) || !std::isfinite(eps))
    return SPHX_E_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return SPHX_E_HIP;
  char *ws = nullptr;
  SPHX_TRY(get_workspace(h, refine_scratch_bytes(g->n, K), &ws));
  // fixed-point exponent of the exact gains and cuts: the weight range
  SPHX_TRY(weight_range(g, ws, h->pinned_small, h->stream));
  std::string err;
  int r = refine(g, part, K, eps, max_passes, cut, imbalance, passes, moves, ws,
                 h->pinned_small, h->stream, &err);
  if (r != SPHX_OK) return set_err(h, r, err);
  return SPHX_OK;
}

int sphx_block_gram(sphx_handle *h, int64_t n, int m, int dtype, const void *X,
                    const void *LX, const void *H, const void *LH, const void *P,
                    const void *LP, int nact, const int32_t *act, int use_h, int use_p,
                    const double *bdiag, double *GA, double *GB) {
  if (!h || n < 1 || m < 1 || m > kMaxNev || nact < 0 || nact > m || !X || !LX || !GA ||
      !GB || (dtype != SPHX_F32 && dtype != SPHX_F64) || (nact > 0 && !act))
    return SPHX_E_INVALID_ARG;
  if ((use_h && (!H || !LH)) || (use_p && (!P || !LP))) return SPHX_E_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return SPHX_E_HIP;
  char *ws = nullptr;
  size_t need = sizeof(double) * (gram_partial_doubles(kGramBlocks) + 2 * kMaxW * kMaxW) + 1024;
  SPHX_TRY(get_workspace(h, need, &ws));
  double *parts = reinterpret_cast<double *>(ws);
  double *out = parts + gram_partial_doubles(kGramBlocks);
  GramArgs a{n, m, m, identity_map(m), use_h, use_p, bdiag};
  a.act.count = nact;
  for (int q = 0; q < nact; ++q) {
    if (act[q] < 0 || act[q] >= m) return SPHX_E_INVALID_ARG;
    a.act.col[q] = act[q];
  }
  int st = dtype == SPHX_F32
               ? gram<float>((const float *)X, (const float *)LX, (const float *)H,
                             (const float *)LH, (const float *)P, (const float *)LP, a, parts,
                             kGramBlocks, out, h->stream)
               : gram<double>((const double *)X, (const double *)LX, (const double *)H,
                              (const double *)LH, (const double *)P, (const double *)LP, a,
                              parts, kGramBlocks, out, h->stream);
  if (st != SPHX_OK) return set_err(h, st, "gram launch failed");
  std::vector<double> host(2 * kMaxW * kMaxW);
  SPHX_HIP(h, hipMemcpyAsync(host.data(), out, sizeof(double) * host.size(),
                             hipMemcpyDeviceToHost, h->stream));
  SPHX_HIP(h, hipStreamSynchronize(h->stream));
  const int w = m + (nact > 0 ? nact * ((use_h ? 1 : 0) + (use_p ? 1 : 0)) : 0);
  for (int i = 0; i < w; ++i)
    for (int j = 0; j < w; ++j) {
      int lo = std::min(i, j), hi = std::max(i, j);
      GA[i * w + j] = host[lo * kMaxW + hi];
      GB[i * w + j] = host[kMaxW * kMaxW + lo * kMaxW + hi];
    }
  return SPHX_OK;
}

int sphx_rayleigh_ritz(sphx_handle *h, int m, int w, int p_begin, double drop_tol,
                       const double *GA, const double *GB, double *Y, double *theta,
                       int *kept, int *breakdown) {
  if (!h || m < 1 || m > kMaxNev || w < m || w > kMaxW || p_begin < m || p_begin > w ||
      !GA || !GB || !Y || !theta || !(drop_tol > 0))
    return SPHX_E_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return SPHX_E_HIP;
  char *ws = nullptr;
  size_t need = sizeof(double) * (2 * kMaxW * kMaxW + kMaxW * kMaxNev + kMaxNev) +
                sizeof(DevStatus) + 2048;
  SPHX_TRY(get_workspace(h, need, &ws));
  Arena a;
  a.base = ws;
  double *g = a.take<double>(2 * kMaxW * kMaxW);
  double *Yd = a.take<double>(kMaxW * kMaxNev);
  double *th = a.take<double>(kMaxNev);
  DevStatus *st = a.take<DevStatus>(1);
  std::vector<double> host(2 * kMaxW * kMaxW, 0.0);
  for (int i = 0; i < w; ++i)
    for (int j = i; j < w; ++j) {
      host[i * kMaxW + j] = GA[i * w + j];
      host[kMaxW * kMaxW + i * kMaxW + j] = GB[i * w + j];
    }
  SPHX_HIP(h, hipMemcpyAsync(g, host.data(), sizeof(double) * host.size(),
                             hipMemcpyHostToDevice, h->stream));
  launch_rr(g, RRArgs{m, w, p_begin, drop_tol}, Yd, th, st, h->stream);
  SPHX_HIP(h, hipGetLastError());
  std::vector<double> yh(kMaxW * kMaxNev);
  DevStatus sh;
  SPHX_HIP(h, hipMemcpyAsync(yh.data(), Yd, sizeof(double) * yh.size(), hipMemcpyDeviceToHost,
                             h->stream));
  SPHX_HIP(h, hipMemcpyAsync(theta, th, sizeof(double) * m, hipMemcpyDeviceToHost, h->stream));
  SPHX_HIP(h, hipMemcpyAsync(&sh, st, sizeof(DevStatus), hipMemcpyDeviceToHost, h->stream));
  SPHX_HIP(h, hipStreamSynchronize(h->stream));
  for (int i = 0; i < w; ++i)
    for (int c = 0; c < m; ++c) Y[i * m + c] = yh[i * kMaxNev + c];
  if (kept) *kept = sh.kept;
  if (breakdown) *breakdown = sh.breakdown;
  return SPHX_OK;
}

int sphx_eig_backward(sphx_handle *h, sphx_graph *g, int problem, int nev,
                      const double *eigvals, const void *eigvecs, const double *g_vals,
                      const void *g_vecs, double cg_tol, int cg_max_iter, void *grad_w) {
  if (!h || !g || !eigvals || !eigvecs || !grad_w || nev < 1 || nev > kMaxNev ||
      nev >= g->n || !(cg_tol > 0) || cg_max_iter < 1 ||
      (problem != SPHX_COMBINATORIAL && problem != SPHX_GENERALIZED &&
       problem != SPHX_NORMALIZED))
    return SPHX_E_INVALID_ARG;
  if (g->wdt == SPHX_F32)
    return set_err(h, SPHX_E_INVALID_ARG, "the adjoint needs F64 (or unit) edge weights");
  if (hipSetDevice(h->device) != hipSuccess) return SPHX_E_HIP;
  size_t need = adjoint_scratch_bytes(g->n, nev) + plan_bytes(g) +
                align_up(sizeof(double) * g->n, 256) + 4 * kDegBlocksMax * sizeof(double) +
                4096;
  char *ws = nullptr;
  SPHX_TRY(get_workspace(h, need, &ws));
  Arena a;
  a.base = ws;
  double *d64 = a.take<double>(g->n);
  double *degs = a.take<double>(4 * kDegBlocksMax);
  DegreeStats ds;
  SPHX_TRY(compute_degrees(g, d64, nullptr, degs, &ds, h->pinned_small, h->stream));
  SpmmPlan plan;
  SPHX_TRY(build_plan(g, a, &plan, ds, h->pinned_small, h->stream));
  if (problem != SPHX_COMBINATORIAL && !(ds.min_wdeg > 0))
    return set_err(h, SPHX_E_INVALID_ARG, "isolated vertex");
  char *scratch = a.take<char>(adjoint_scratch_bytes(g->n, nev));
  std::string err;
  h->last_cg_iters = 0;
  h->last_cg_relres = 0.0;
  int r = eig_backward(g, plan, problem, nev, eigvals, (const double *)eigvecs, g_vals,
                       (const double *)g_vecs, cg_tol, cg_max_iter, d64, (double *)grad_w,
                       scratch, h->pinned_small, h->stream, &err, &h->last_cg_iters,
                       &h->last_cg_relres);
  if (r < 0) return set_err(h, r, err);
  if (r == SPHX_NOT_CONVERGED)
    return set_err(h, r, err.empty() ? "adjoint CG reached cg_max_iter" : err);
  return r;
}

int sphx_backward_info(const sphx_handle *h, int *cg_iterations, double *cg_rel_residual) {
  if (!h) return SPHX_E_INVALID_ARG;
  if (cg_iterations) *cg_iterations = h->last_cg_iters;
  if (cg_rel_residual) *cg_rel_residual = h->last_cg_relres;
  return SPHX_OK;
}

}  // extern "C"
