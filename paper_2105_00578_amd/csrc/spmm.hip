// Laplacian block product Y = L_C X for a CSR graph (Eq. 2 with weights),
// summed per row in difference form y_i = sum_j w_ij (x_i - x_j).
//
// Layout: X and Y are row-major n x ld blocks.  The kernels use a
// column-lane mapping: a group of G lanes serves one row, lane c owning
// column cm.col[c], so the G values of a gathered neighbour row are read by G
// adjacent lanes from one contiguous segment.  Rows are split by degree:
//   rows of the lower degree classes: one lane group per row, 64/G rows per
//     wave;
//   rows of the highest class below the hubs: one wavefront per row, its
//     64/G groups striding over the neighbours, combined with cross-lane
//     shuffles in a fixed order;
//   hub rows (deg > kHubDeg): kHubChunk-entry chunks, one wavefront each,
//     partial sums combined per row in a second kernel (fixed order).
// All sums are in a fixed order, so results are bitwise reproducible.
//
// Epilogues fused into the product:
//   Store     y = acc
//   Residual  LX = acc; r = acc - b_i theta_c x_i (b_i = d_i for the
//             generalized problem, else 1); writes r or the Jacobi step
//             r / d_i (Sec. 5.1); accumulates ||r||^2_{B^-1} and ||x||^2_B per
//             column in FP64 (per-block partials).
//   Cheb      one step of the Chebyshev iteration for L h = r (Sec. 5.2):
//             out = xs + alpha (xs - prev) + beta s_i (r - L xs), xs = scale x,
//             s_i = 1 or 1/d_i (generalized).
#include "kernels.h"

namespace sphx {
namespace {

template <typename IdxT, typename WT>
struct Csr {
  const IdxT *rp;
  const int32_t *col;
  const WT *w;
};

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c) {
  if constexpr (std::is_same_v<T, float>) return fmaf(a, b, c);
  else return fma(a, b, c);
}

// Sum over entries k0, k0+step, ... < k1 of w_k (xi - x_{col[k]}[col]).
template <typename T, typename IdxT, typename WT>
__device__ __forceinline__ T row_acc(const Csr<IdxT, WT> &A, int64_t k0,
                                     int64_t k1, int step, const T *__restrict__ X,
                                     int ldx, int col, T xi) {
  T acc0 = T(0), acc1 = T(0);
  int64_t k = k0;
  // two independent gathers in flight per iteration
  for (; k + step < k1; k += 2 * step) {
    int j0 = A.col[k];
    int j1 = A.col[k + step];
    T x0 = X[(int64_t)j0 * ldx + col];
    T x1 = X[(int64_t)j1 * ldx + col];
    if constexpr (std::is_same_v<WT, Unit>) {
      acc0 += xi - x0;
      acc1 += xi - x1;
    } else {
      acc0 = fma_t(T(A.w[k]), xi - x0, acc0);
      acc1 = fma_t(T(A.w[k + step]), xi - x1, acc1);
    }
  }
  if (k < k1) {
    int j0 = A.col[k];
    T x0 = X[(int64_t)j0 * ldx + col];
    if constexpr (std::is_same_v<WT, Unit>) acc0 += xi - x0;
    else acc0 = fma_t(T(A.w[k]), xi - x0, acc0);
  }
  return acc0 + acc1;
}

// ------------------------------------------------------------- epilogues
template <typename T>
struct EpiStore {
  EpiStoreP<T> p;
  static constexpr bool kNorms = false;
  __device__ void operator()(int64_t i, int c, int col, T xi, T acc, double &,
                             double &) const {
    p.Y[i * p.ldy + col] = acc;
  }
};

template <typename T>
struct EpiResidual {
  EpiResidualP<T> p;
  static constexpr bool kNorms = true;
  __device__ void operator()(int64_t i, int c, int col, T xi, T acc, double &n1,
                             double &n2) const {
    int64_t o = i * p.ld + col;
    p.LX[o] = acc;
    double di = p.d64 ? p.d64[i] : 1.0;
    double b = p.generalized ? di : 1.0;
    double x = double(xi);
    double r = double(acc) - b * p.theta[col] * x;
    p.OUT[o] = T(p.jacobi ? r / di : r);
    n1 += r * r / b;
    n2 += b * x * x;
  }
};

template <typename T>
struct EpiCheb {
  EpiChebP<T> p;
  static constexpr bool kNorms = false;
  __device__ void operator()(int64_t i, int c, int col, T xi, T acc, double &,
                             double &) const {
    int64_t o = i * p.ld + col;
    double xs = p.src_scale * double(xi);
    double pv = p.prev ? p.prev_scale * double(p.prev[o]) : 0.0;
    double si = p.dinv ? p.dinv[i] : 1.0;
    double res = double(p.R[o]) - p.src_scale * double(acc);
    p.OUT[o] = T(xs + p.alpha * (xs - pv) + p.beta * si * res);
  }
};

// Per-column block sums of (v1, v2) in a fixed order, stored sum-major:
// partials[q * kMaxNormBlocks + slot], q = column (v1) or kMaxNev + column
// (v2).  Every thread of the block must call this.  c < 0 marks a lane
// without a column.
__device__ void block_colsum(int c, double v1, double v2, int G, double *partials,
                             int slot) {
  __shared__ double s1[256], s2[256];
  __shared__ int sc[256];
  int t = threadIdx.x;
  s1[t] = v1;
  s2[t] = v2;
  sc[t] = c;
  __syncthreads();
  if (t < G) {
    double a = 0.0, b = 0.0;
    for (int u = 0; u < (int)blockDim.x; ++u)
      if (sc[u] == t) {
        a += s1[u];
        b += s2[u];
      }
    partials[(int64_t)t * kMaxNormBlocks + slot] = a;
    partials[(int64_t)(kMaxNev + t) * kMaxNormBlocks + slot] = b;
  }
}

// ---------------------------------------------------------------- kernels
template <typename T, typename IdxT, typename WT, typename Epi>
__global__ __launch_bounds__(256) void k_spmm_group(
    Csr<IdxT, WT> A, const int32_t *__restrict__ rows, int64_t nrows,
    const T *__restrict__ X, int ldx, ColMap cm, Epi epi, double *partials,
    int slot0) {
  const int G = cm.count;
  const int gpw = kWave / G;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int g = lane / G;
  const int c = lane - g * G;
  const bool ok = g < gpw;
  const int col = ok ? cm.col[c] : 0;
  double n1 = 0.0, n2 = 0.0;
  const int64_t per_block = (int64_t)(blockDim.x / kWave) * gpw;
  if (ok) {
    for (int64_t r = (int64_t)blockIdx.x * per_block + wave * gpw + g; r < nrows;
         r += (int64_t)gridDim.x * per_block) {
      int64_t i = rows ? rows[r] : r;
      T xi = X[i * ldx + col];
      T acc = row_acc<T>(A, (int64_t)A.rp[i], (int64_t)A.rp[i + 1], 1, X, ldx, col, xi);
      epi(i, c, col, xi, acc, n1, n2);
    }
  }
  if constexpr (Epi::kNorms)
    block_colsum(ok ? c : -1, n1, n2, G, partials, slot0 + (int)blockIdx.x);
}

// Sum lane values of all groups for column c (result valid in lanes < G).
template <typename T>
__device__ __forceinline__ T group_reduce(T v, int G, int lane) {
  const int ng = kWave / G;
  const int c = lane % G;
  T tot = T(0);
  for (int q = 0; q < ng; ++q) {
    T o = __shfl(v, q * G + c);
    tot += o;
  }
  return tot;
}

template <typename T, typename IdxT, typename WT, typename Epi>
__global__ __launch_bounds__(256) void k_spmm_wave(
    Csr<IdxT, WT> A, const int32_t *__restrict__ rows, int64_t nrows,
    const T *__restrict__ X, int ldx, ColMap cm, Epi epi, double *partials,
    int slot0) {
  const int G = cm.count;
  const int ng = kWave / G;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int g = lane / G;
  const int c = lane % G;
  const bool ok = g < ng;
  const int col = cm.col[c];
  const int wpb = blockDim.x / kWave;
  double n1 = 0.0, n2 = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * wpb + wave; r < nrows;
       r += (int64_t)gridDim.x * wpb) {
    int64_t i = rows[r];
    T xi = X[i * ldx + col];
    T acc = T(0);
    if (ok)
      acc = row_acc<T>(A, (int64_t)A.rp[i] + g, (int64_t)A.rp[i + 1], ng, X, ldx, col, xi);
    T tot = group_reduce(acc, G, lane);
    if (lane < G) epi(i, c, col, xi, tot, n1, n2);
  }
  if constexpr (Epi::kNorms)
    block_colsum(lane < G ? c : -1, n1, n2, G, partials, slot0 + (int)blockIdx.x);
}

template <typename T, typename IdxT, typename WT>
__global__ __launch_bounds__(256) void k_spmm_hub_partial(
    Csr<IdxT, WT> A, const int32_t *__restrict__ hub_rows,
    const int32_t *__restrict__ hub_chunk_begin, int64_t n_hub,
    const int64_t *__restrict__ k0s, const int64_t *__restrict__ k1s,
    int64_t n_chunks, const T *__restrict__ X, int ldx, ColMap cm, double *out) {
  const int G = cm.count;
  const int ng = kWave / G;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int g = lane / G;
  const int c = lane % G;
  const int col = cm.col[c];
  const int wpb = blockDim.x / kWave;
  for (int64_t q = (int64_t)blockIdx.x * wpb + wave; q < n_chunks;
       q += (int64_t)gridDim.x * wpb) {
    // hub row owning chunk q: last h with hub_chunk_begin[h] <= q
    int64_t lo = 0, hi = n_hub - 1;
    while (lo < hi) {
      int64_t mid = (lo + hi + 1) / 2;
      if (hub_chunk_begin[mid] <= q) lo = mid; else hi = mid - 1;
    }
    int64_t i = hub_rows[lo];
    T xi = X[i * ldx + col];
    T acc = T(0);
    if (g < ng) acc = row_acc<T>(A, k0s[q] + g, k1s[q], ng, X, ldx, col, xi);
    T tot = group_reduce(acc, G, lane);
    if (lane < G) out[q * kMaxNev + c] = double(tot);
  }
}

template <typename T, typename Epi>
__global__ __launch_bounds__(256) void k_spmm_hub_combine(
    const int32_t *__restrict__ hub_rows, const int32_t *__restrict__ hub_chunk_begin,
    int64_t n_hub, const double *__restrict__ part, const T *__restrict__ X,
    int ldx, ColMap cm, Epi epi, double *partials, int slot0) {
  const int G = cm.count;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int wpb = blockDim.x / kWave;
  double n1 = 0.0, n2 = 0.0;
  const int c = lane;
  for (int64_t h = (int64_t)blockIdx.x * wpb + wave; h < n_hub;
       h += (int64_t)gridDim.x * wpb) {
    if (c < G) {
      int64_t i = hub_rows[h];
      int col = cm.col[c];
      T xi = X[i * ldx + col];
      T tot = T(0);
      for (int64_t q = hub_chunk_begin[h]; q < hub_chunk_begin[h + 1]; ++q)
        tot += T(part[q * kMaxNev + c]);
      epi(i, c, col, xi, tot, n1, n2);
    }
  }
  if constexpr (Epi::kNorms)
    block_colsum(c < G ? c : -1, n1, n2, G, partials, slot0 + (int)blockIdx.x);
}

// --------------------------------------------------------------- dispatch
constexpr int kGroupBlocks = 2048;
constexpr int kWaveBlocks = 1024;
constexpr int kHubBlocks = 64;

template <typename T, typename IdxT, typename WT, typename Epi>
void run_all(const Csr<IdxT, WT> &A, int64_t n, const SpmmPlan &plan,
             const T *X, int ldx, const ColMap &cm, const Epi &epi,
             double *partials, int *nparts, hipStream_t s) {
  const int G = cm.count;
  const int gpw = kWave / G;
  int used = 0;
  auto slot = [&](int blocks) {
    int b = used;
    used += blocks;
    return b;
  };
  if (!plan.binned) {
    unsigned gb = grid_for(n, 4 * gpw, kGroupBlocks);
    hipLaunchKernelGGL((k_spmm_group<T, IdxT, WT, Epi>), dim3(gb), dim3(256), 0, s,
                       A, (const int32_t *)nullptr, n, X, ldx, cm, epi, partials, slot(gb));
  } else {
    // rows of the first kNumBins - 1 classes: one lane group per row; the
    // last class: one wavefront per row
    for (int c = 0; c < kNumBins - 1; ++c) {
      if (plan.nrows[c] == 0) continue;
      unsigned gb = grid_for(plan.nrows[c], 4 * gpw, kGroupBlocks);
      hipLaunchKernelGGL((k_spmm_group<T, IdxT, WT, Epi>), dim3(gb), dim3(256), 0, s,
                         A, plan.rows[c], plan.nrows[c], X, ldx, cm, epi, partials, slot(gb));
    }
    if (plan.nrows[kNumBins - 1] > 0) {
      unsigned gb = grid_for(plan.nrows[kNumBins - 1], 4, kWaveBlocks);
      hipLaunchKernelGGL((k_spmm_wave<T, IdxT, WT, Epi>), dim3(gb), dim3(256), 0, s,
                         A, plan.rows[kNumBins - 1], plan.nrows[kNumBins - 1], X, ldx, cm, epi,
                         partials, slot(gb));
    }
    if (plan.n_hub > 0) {
      unsigned gb = grid_for(plan.n_chunks, 4, kWaveBlocks);
      hipLaunchKernelGGL((k_spmm_hub_partial<T, IdxT, WT>), dim3(gb), dim3(256), 0, s,
                         A, plan.hub_rows, plan.hub_chunk_begin, plan.n_hub,
                         plan.chunk_k0, plan.chunk_k1, plan.n_chunks, X, ldx, cm,
                         plan.hub_partial);
      unsigned gc = grid_for(plan.n_hub, 4, kHubBlocks);
      hipLaunchKernelGGL((k_spmm_hub_combine<T, Epi>), dim3(gc), dim3(256), 0, s,
                         plan.hub_rows, plan.hub_chunk_begin, plan.n_hub,
                         (const double *)plan.hub_partial, X, ldx, cm, epi, partials, slot(gc));
    }
  }
  if (nparts) *nparts = used;
}

template <typename T, typename Epi>
int dispatch(sphx_graph *g, const SpmmPlan &plan, const T *X, int ldx,
             const ColMap &cm, const Epi &epi, double *partials, int *nparts,
             hipStream_t s) {
  if (cm.count < 1 || cm.count > kMaxNev) return SPHX_E_INVALID_ARG;
  auto go = [&](auto idx_tag, auto w_tag) {
    using IdxT = decltype(idx_tag);
    using WT = decltype(w_tag);
    Csr<IdxT, WT> A{static_cast<const IdxT *>(g->rowptr), g->col,
                    static_cast<const WT *>(g->w)};
    run_all<T>(A, g->n, plan, X, ldx, cm, epi, partials, nparts, s);
  };
  if (g->rp64) {
    if (g->wdt == SPHX_UNIT) go(int64_t{}, Unit{});
    else if (g->wdt == SPHX_F32) go(int64_t{}, float{});
    else go(int64_t{}, double{});
  } else {
    if (g->wdt == SPHX_UNIT) go(int32_t{}, Unit{});
    else if (g->wdt == SPHX_F32) go(int32_t{}, float{});
    else go(int32_t{}, double{});
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPHX_OK : SPHX_E_HIP;
}

}  // namespace

template <typename T>
int spmm_store(sphx_graph *g, const SpmmPlan &plan, const T *X, int ldx,
               const ColMap &cm, EpiStoreP<T> epi, hipStream_t s) {
  return dispatch(g, plan, X, ldx, cm, EpiStore<T>{epi}, nullptr, nullptr, s);
}

template <typename T>
int spmm_residual(sphx_graph *g, const SpmmPlan &plan, const T *X, int ldx,
                  const ColMap &cm, EpiResidualP<T> epi, double *norm_partials,
                  int *n_norm_blocks, hipStream_t s) {
  return dispatch(g, plan, X, ldx, cm, EpiResidual<T>{epi}, norm_partials,
                  n_norm_blocks, s);
}

template <typename T>
int spmm_cheb(sphx_graph *g, const SpmmPlan &plan, const T *X, int ldx,
              const ColMap &cm, EpiChebP<T> epi, hipStream_t s) {
  return dispatch(g, plan, X, ldx, cm, EpiCheb<T>{epi}, nullptr, nullptr, s);
}

template int spmm_store<float>(sphx_graph *, const SpmmPlan &, const float *, int,
                               const ColMap &, EpiStoreP<float>, hipStream_t);
template int spmm_store<double>(sphx_graph *, const SpmmPlan &, const double *, int,
                                const ColMap &, EpiStoreP<double>, hipStream_t);
template int spmm_residual<float>(sphx_graph *, const SpmmPlan &, const float *, int,
                                  const ColMap &, EpiResidualP<float>, double *, int *,
                                  hipStream_t);
template int spmm_residual<double>(sphx_graph *, const SpmmPlan &, const double *, int,
                                   const ColMap &, EpiResidualP<double>, double *, int *,
                                   hipStream_t);
template int spmm_cheb<float>(sphx_graph *, const SpmmPlan &, const float *, int,
                              const ColMap &, EpiChebP<float>, hipStream_t);
template int spmm_cheb<double>(sphx_graph *, const SpmmPlan &, const double *, int,
                               const ColMap &, EpiChebP<double>, hipStream_t);

}  // namespace sphx
