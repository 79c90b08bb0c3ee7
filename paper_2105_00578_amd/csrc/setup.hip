// Graph validation, degrees and the degree-binned row plan of the Laplacian
// product.  Degrees are the diagonal of L_C (Eq. 2, weighted); the regular /
// irregular classification is max degree / average degree <= 10 (Sec. 6.1).
#include <algorithm>

#include "fixed.h"
#include "kernels.h"

namespace sphx {
namespace {

enum : int {
  F_BAD_GRAPH = 1,
  F_SELF_LOOP = 2,
  F_NOT_SYM = 4,
  F_BAD_WEIGHT = 8,
};

// One wavefront per row; lanes stride over the row's entries.
template <typename IdxT, typename WT>
__global__ __launch_bounds__(256) void k_validate(int64_t n, int64_t nnz,
                                                  const IdxT *rp, const int32_t *col,
                                                  const WT *w, const int32_t *vwgt,
                                                  int *flags) {
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x / 64;
  int f = 0;
  for (int64_t i = (int64_t)blockIdx.x * wpb + threadIdx.x / 64; i < n;
       i += (int64_t)gridDim.x * wpb) {
    int64_t b = rp[i], e = rp[i + 1];
    if (lane == 0) {
      if (e < b || b < 0 || e > nnz) f |= F_BAD_GRAPH;
      if (i == 0 && b != 0) f |= F_BAD_GRAPH;
      if (i == n - 1 && e != nnz) f |= F_BAD_GRAPH;
      if (vwgt && vwgt[i] < 1) f |= F_BAD_WEIGHT;
    }
    if (e < b || b < 0 || e > nnz) continue;
    for (int64_t k = b + lane; k < e; k += 64) {
      int64_t j = col[k];
      if (j < 0 || j >= n) { f |= F_BAD_GRAPH; continue; }
      if (j == i) f |= F_SELF_LOOP;
      if (k > b && col[k - 1] >= col[k]) f |= F_BAD_GRAPH;
      if constexpr (!std::is_same_v<WT, Unit>) {
        WT wk = w[k];
        if (!(wk > WT(0)) || !(wk < WT(INFINITY))) f |= F_BAD_WEIGHT;
      }
      // symmetric partner (i in row j), binary search over row j, whose
      // bounds are checked first (a malformed row_ptr must not send the
      // search outside col[0..nnz))
      int64_t lo = rp[j], hi = rp[j + 1] - 1;
      if (lo < 0 || hi + 1 < lo || hi + 1 > nnz) { f |= F_BAD_GRAPH; continue; }
      bool found = false;
      int64_t kk = -1;
      while (lo <= hi) {
        int64_t mid = (lo + hi) >> 1;
        int64_t cm = col[mid];
        if (cm == i) { found = true; kk = mid; break; }
        if (cm < i) lo = mid + 1; else hi = mid - 1;
      }
      if (!found) f |= F_NOT_SYM;
      else if constexpr (!std::is_same_v<WT, Unit>) {
        if (!(w[kk] == w[k])) f |= F_NOT_SYM;
      }
    }
  }
  if (f) atomicOr(flags, f);
}

// Degrees: one wavefront per row.  The weighted degree is the exact sum of
// the row's weights rounded once to FP64 (128-bit fixed point, see fixed.h),
// so it does not depend on any summation order.  Each lane sums a strided
// part of the row; lane 0 adds the 64 lane sums from LDS.  The row loop is
// uniform over the block (rows r0 + wave), so the barriers are reached by
// every wave.  Block statistics -> stats[block][4]: max pattern deg, min
// pattern deg, max wdeg, min wdeg.
template <typename IdxT, typename WT>
__global__ __launch_bounds__(256) void k_degrees(int64_t n, const IdxT *rp,
                                                 const WT *w, int e0, double *d64,
                                                 float *d32, double *stats) {
  __shared__ unsigned long long plo[256], phi[256];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wpb = blockDim.x / 64;
  double mx = 0.0, mn = 1e300, wmx = 0.0, wmn = 1e300;
  for (int64_t r0 = (int64_t)blockIdx.x * wpb; r0 < n; r0 += (int64_t)gridDim.x * wpb) {
    const int64_t i = r0 + wave;
    U128 acc{0, 0};
    int64_t b = 0, e = 0;
    if (i < n) {
      b = rp[i];
      e = rp[i + 1];
      if constexpr (!std::is_same_v<WT, Unit>) {
        for (int64_t k = b + lane; k < e; k += 64) {
          unsigned long long lo, hi;
          fixed_of(w[k], e0, lo, hi);
          add128(acc, lo, hi);
        }
      }
    }
    plo[threadIdx.x] = acc.lo;
    phi[threadIdx.x] = acc.hi;
    __syncthreads();
    if (lane == 0 && i < n) {
      double s;
      if constexpr (std::is_same_v<WT, Unit>) {
        s = double(e - b);
      } else {
        U128 tot{0, 0};
        for (int q = 0; q < 64; ++q) add128(tot, plo[wave * 64 + q], phi[wave * 64 + q]);
        s = fixed_to_double(tot, e0);
      }
      d64[i] = s;
      if (d32) d32[i] = float(s);
      double deg = double(e - b);
      mx = fmax(mx, deg);
      mn = fmin(mn, deg);
      wmx = fmax(wmx, s);
      wmn = fmin(wmn, s);
    }
    __syncthreads();
  }
  __shared__ double sh[4][256];
  sh[0][threadIdx.x] = mx;
  sh[1][threadIdx.x] = mn;
  sh[2][threadIdx.x] = wmx;
  sh[3][threadIdx.x] = wmn;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int t = 1; t < (int)blockDim.x; ++t) {
      mx = fmax(mx, sh[0][t]);
      mn = fmin(mn, sh[1][t]);
      wmx = fmax(wmx, sh[2][t]);
      wmn = fmin(wmn, sh[3][t]);
    }
    stats[blockIdx.x * 4 + 0] = mx;
    stats[blockIdx.x * 4 + 1] = mn;
    stats[blockIdx.x * 4 + 2] = wmx;
    stats[blockIdx.x * 4 + 3] = wmn;
  }
}

// Unit weights: the degree is the row length; one thread per row.
template <typename IdxT>
__global__ __launch_bounds__(256) void k_degrees_unit(int64_t n, const IdxT *rp, double *d64,
                                                      float *d32, double *stats) {
  double mx = 0.0, mn = 1e300;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = double(rp[i + 1] - rp[i]);
    d64[i] = s;
    if (d32) d32[i] = float(s);
    mx = fmax(mx, s);
    mn = fmin(mn, s);
  }
  __shared__ double sh[2][256];
  sh[0][threadIdx.x] = mx;
  sh[1][threadIdx.x] = mn;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int t = 1; t < (int)blockDim.x; ++t) {
      mx = fmax(mx, sh[0][t]);
      mn = fmin(mn, sh[1][t]);
    }
    stats[blockIdx.x * 4 + 0] = mx;
    stats[blockIdx.x * 4 + 1] = mn;
    stats[blockIdx.x * 4 + 2] = mx;
    stats[blockIdx.x * 4 + 3] = mn;
  }
}

// edge-weight range (for the exact cut), block partials
template <typename WT>
__global__ __launch_bounds__(256) void k_wrange(int64_t nnz, const WT *w, double *stats) {
  double mx = 0.0, mn = 1e300;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * blockDim.x) {
    double v = double(w[k]);
    mx = fmax(mx, v);
    mn = fmin(mn, v);
  }
  __shared__ double s0[256], s1[256];
  s0[threadIdx.x] = mx;
  s1[threadIdx.x] = mn;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int t = 1; t < (int)blockDim.x; ++t) {
      mx = fmax(mx, s0[t]);
      mn = fmin(mn, s1[t]);
    }
    stats[blockIdx.x * 2] = mx;
    stats[blockIdx.x * 2 + 1] = mn;
  }
}

// Deterministic row binning into kNumBins + 1 classes (the last = hubs).
constexpr int kBinRows = 1024;   // rows per block
constexpr int kNumCls = kNumBins + 1;

template <typename IdxT>
__device__ __forceinline__ int row_class(const IdxT *rp, int64_t i) {
  const int64_t d = rp[i + 1] - rp[i];
  int c = 0;
  while (c < kNumBins && d > bin_max_deg(c)) ++c;
  return c;
}

template <typename IdxT>
__global__ __launch_bounds__(256) void k_bin_count(int64_t n, const IdxT *rp, int *counts) {
  __shared__ int c[kNumCls];
  if (threadIdx.x < kNumCls) c[threadIdx.x] = 0;
  __syncthreads();
  int64_t r0 = (int64_t)blockIdx.x * kBinRows;
  for (int t = threadIdx.x; t < kBinRows; t += blockDim.x) {
    int64_t i = r0 + t;
    if (i < n) atomicAdd(&c[row_class(rp, i)], 1);
  }
  __syncthreads();
  if (threadIdx.x < kNumCls) counts[blockIdx.x * kNumCls + threadIdx.x] = c[threadIdx.x];
}

// Exclusive scan of the per-block counts into positions of one packed list
// (class 0 rows first, then class 1, ...); totals[c] = rows of class c.
__global__ void k_bin_scan(int nblocks, int *counts, int *totals) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int tot[kNumCls] = {};
    for (int b = 0; b < nblocks; ++b)
      for (int c = 0; c < kNumCls; ++c) tot[c] += counts[b * kNumCls + c];
    int base = 0;
    int acc[kNumCls];
    for (int c = 0; c < kNumCls; ++c) {
      acc[c] = base;
      base += tot[c];
      totals[c] = tot[c];
    }
    for (int b = 0; b < nblocks; ++b)
      for (int c = 0; c < kNumCls; ++c) {
        int v = counts[b * kNumCls + c];
        counts[b * kNumCls + c] = acc[c];
        acc[c] += v;
      }
  }
}

template <typename IdxT>
__global__ __launch_bounds__(256) void k_bin_scatter(int64_t n, const IdxT *rp,
                                                     const int *offsets, int32_t *packed) {
  // each thread owns kBinRows/256 consecutive rows; ranks via a block scan
  __shared__ int cnt[kNumCls][256];
  const int per = kBinRows / 256;
  int64_t r0 = (int64_t)blockIdx.x * kBinRows + (int64_t)threadIdx.x * per;
  int local[kNumCls] = {};
  for (int t = 0; t < per; ++t) {
    int64_t i = r0 + t;
    if (i < n) local[row_class(rp, i)]++;
  }
  for (int c = 0; c < kNumCls; ++c) cnt[c][threadIdx.x] = local[c];
  __syncthreads();
  if (threadIdx.x < kNumCls) {
    int c = threadIdx.x, acc = 0;
    for (int t = 0; t < 256; ++t) {
      int v = cnt[c][t];
      cnt[c][t] = acc;
      acc += v;
    }
  }
  __syncthreads();
  int pos[kNumCls];
  for (int c = 0; c < kNumCls; ++c) pos[c] = offsets[blockIdx.x * kNumCls + c] + cnt[c][threadIdx.x];
  for (int t = 0; t < per; ++t) {
    int64_t i = r0 + t;
    if (i < n) {
      int c = row_class(rp, i);
      packed[pos[c]++] = (int32_t)i;
    }
  }
}

template <typename F>
void with_types(sphx_graph *g, F &&f) {
  if (g->rp64) {
    if (g->wdt == SPHX_UNIT) f(int64_t{}, Unit{});
    else if (g->wdt == SPHX_F32) f(int64_t{}, float{});
    else f(int64_t{}, double{});
  } else {
    if (g->wdt == SPHX_UNIT) f(int32_t{}, Unit{});
    else if (g->wdt == SPHX_F32) f(int32_t{}, float{});
    else f(int32_t{}, double{});
  }
}

}  // namespace

int validate_graph(sphx_graph *g, hipStream_t s, int32_t *flags_dev, int *flags_host) {
  SPHX_HIP(g->h, hipMemsetAsync(flags_dev, 0, sizeof(int), s));
  unsigned gb = grid_for(g->n, 4, 1 << 16);
  with_types(g, [&](auto it, auto wt) {
    using IdxT = decltype(it);
    using WT = decltype(wt);
    hipLaunchKernelGGL((k_validate<IdxT, WT>), dim3(gb), dim3(256), 0, s, g->n, g->nnz,
                       (const IdxT *)g->rowptr, g->col, (const WT *)g->w, g->vwgt,
                       (int *)flags_dev);
  });
  SPHX_HIP(g->h, hipGetLastError());
  SPHX_HIP(g->h, hipMemcpyAsync(flags_host, flags_dev, sizeof(int), hipMemcpyDeviceToHost, s));
  SPHX_HIP(g->h, hipStreamSynchronize(s));
  int f = *flags_host;
  if (f & F_BAD_GRAPH) return set_err(g->h, SPHX_E_BAD_GRAPH,
      "CSR arrays malformed: row_ptr not monotone / not [0..nnz], column out of range, "
      "or columns not strictly increasing within a row");
  if (f & F_SELF_LOOP) return set_err(g->h, SPHX_E_SELF_LOOP, "graph has a self-loop");
  if (f & F_BAD_WEIGHT) return set_err(g->h, SPHX_E_BAD_WEIGHT,
      "edge weight not finite and > 0, or vertex weight < 1");
  if (f & F_NOT_SYM) return set_err(g->h, SPHX_E_NOT_SYMMETRIC,
      "pattern or weights not symmetric");
  return SPHX_OK;
}

constexpr int kDegBlocks = 1024;

int weight_range(sphx_graph *g, void *scratch, void *pinned, hipStream_t s) {
  if (g->wdt == SPHX_UNIT || g->wrange_valid) return SPHX_OK;
  double *stats = static_cast<double *>(scratch);
  double *host = static_cast<double *>(pinned);
  const unsigned gw = grid_for(g->nnz, 256, kWrangeBlocks);
  if (g->wdt == SPHX_F32)
    hipLaunchKernelGGL((k_wrange<float>), dim3(gw), dim3(256), 0, s, g->nnz,
                       (const float *)g->w, stats);
  else
    hipLaunchKernelGGL((k_wrange<double>), dim3(gw), dim3(256), 0, s, g->nnz,
                       (const double *)g->w, stats);
  SPHX_HIP(g->h, hipGetLastError());
  SPHX_HIP(g->h, hipMemcpyAsync(host, stats, sizeof(double) * 2 * gw,
                                hipMemcpyDeviceToHost, s));
  SPHX_HIP(g->h, hipStreamSynchronize(s));
  double a = 0, b = 1e300;
  for (unsigned q = 0; q < gw; ++q) {
    a = std::max(a, host[q * 2]);
    b = std::min(b, host[q * 2 + 1]);
  }
  int ea, eb;
  std::frexp(a, &ea);
  std::frexp(b, &eb);
  if (g->nnz > 0 && ea - eb > 40)
    return set_err(g->h, SPHX_E_BAD_WEIGHT,
                   "edge weights span more than a factor 2^40 (exact sums unsupported)");
  g->wmax = a;
  g->wmin = b;
  g->wrange_valid = 1;
  return SPHX_OK;
}

int compute_degrees(sphx_graph *g, double *d64, float *d32, void *scratch,
                    DegreeStats *out, void *pinned, hipStream_t s) {
  double *stats = static_cast<double *>(scratch);
  double *host = static_cast<double *>(pinned);
  // edge-weight range: e0 of the exact degree sums and of the exact cut
  SPHX_TRY(weight_range(g, scratch, pinned, s));
  int e0 = 0;
  if (g->wdt == SPHX_F32) e0 = fixed_exponent<float>(g->wmin);
  if (g->wdt == SPHX_F64) e0 = fixed_exponent<double>(g->wmin);
  unsigned gb = grid_for(g->n, 4, kDegBlocks);
  if (g->wdt == SPHX_UNIT) {
    gb = grid_for(g->n, 256, kDegBlocks);
    if (g->rp64)
      hipLaunchKernelGGL((k_degrees_unit<int64_t>), dim3(gb), dim3(256), 0, s, g->n,
                         (const int64_t *)g->rowptr, d64, d32, stats);
    else
      hipLaunchKernelGGL((k_degrees_unit<int32_t>), dim3(gb), dim3(256), 0, s, g->n,
                         (const int32_t *)g->rowptr, d64, d32, stats);
  } else {
    with_types(g, [&](auto it, auto wt) {
      using IdxT = decltype(it);
      using WT = decltype(wt);
      hipLaunchKernelGGL((k_degrees<IdxT, WT>), dim3(gb), dim3(256), 0, s, g->n,
                         (const IdxT *)g->rowptr, (const WT *)g->w, e0, d64, d32, stats);
    });
  }
  SPHX_HIP(g->h, hipGetLastError());
  SPHX_HIP(g->h, hipMemcpyAsync(host, stats, sizeof(double) * 4 * gb,
                                hipMemcpyDeviceToHost, s));
  SPHX_HIP(g->h, hipStreamSynchronize(s));
  double mx = 0, mn = 1e300, wmx = 0, wmn = 1e300;
  for (unsigned b = 0; b < gb; ++b) {
    mx = std::max(mx, host[b * 4 + 0]);
    mn = std::min(mn, host[b * 4 + 1]);
    wmx = std::max(wmx, host[b * 4 + 2]);
    wmn = std::min(wmn, host[b * 4 + 3]);
  }
  out->max_deg = (int64_t)mx;
  out->min_deg = (int64_t)mn;
  out->sum_deg = g->nnz;
  out->max_wdeg = wmx;
  out->min_wdeg = wmn;
  g->max_deg = out->max_deg;
  g->sum_deg = out->sum_deg;
  g->max_wdeg = wmx;
  g->stats_valid = 1;
  return SPHX_OK;
}

namespace {

// Column offsets from the row as int16, one thread per row; *overflow is
// set when some offset does not fit (the offsets are then not used).
__global__ __launch_bounds__(256) void k_delta16(int64_t n, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ col, int16_t *d,
                                                 int *overflow) {
  int f = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    for (int64_t k = rp[i]; k < (int64_t)rp[i + 1]; ++k) {
      const int64_t o = (int64_t)col[k] - i;
      const bool fits = o >= -32767 && o <= 32767;
      d[k] = (int16_t)(fits ? o : 0);
      f |= fits ? 0 : 1;
    }
  }
  if (f) atomicOr(overflow, 1);
}

__global__ void k_fill_int(int *x, int cnt, int v) {
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) x[i] = v;
}

}  // namespace

namespace {

// ---- degree order: rows by floor(log2 degree), descending, ties in
// increasing id (a stable bucket sort), so that the frequently gathered rows
// of high degree share cache lines
constexpr int kOrdCls = 32;
constexpr int kOrdRows = 1024;   // rows per counting block

template <typename IdxT>
__device__ __forceinline__ int ord_class(const IdxT *rp, int64_t i) {
  const int64_t d = (int64_t)rp[i + 1] - (int64_t)rp[i];
  int lg = 0;
  for (int64_t x = d; x > 1; x >>= 1) ++lg;
  return kOrdCls - 1 - min(lg, kOrdCls - 1);
}

template <typename IdxT>
__global__ __launch_bounds__(256) void k_ord_count(int64_t n, const IdxT *rp, int *counts) {
  __shared__ int c[kOrdCls];
  if (threadIdx.x < kOrdCls) c[threadIdx.x] = 0;
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * kOrdRows;
  for (int t = threadIdx.x; t < kOrdRows; t += blockDim.x) {
    const int64_t i = r0 + t;
    if (i < n) atomicAdd(&c[ord_class(rp, i)], 1);
  }
  __syncthreads();
  if (threadIdx.x < kOrdCls) counts[blockIdx.x * kOrdCls + threadIdx.x] = c[threadIdx.x];
}

// counts[b][c] -> start of block b's class-c rows in the new order (class 0
// first): one thread per class scans the blocks, then thread 0 adds the
// class offsets
__global__ __launch_bounds__(64) void k_ord_scan(int nblocks, int *counts) {
  __shared__ long long tot[kOrdCls];
  const int c = threadIdx.x;
  if (c < kOrdCls) {
    long long acc = 0;
    for (int b = 0; b < nblocks; ++b) {
      const int v = counts[b * kOrdCls + c];
      counts[b * kOrdCls + c] = (int)acc;
      acc += v;
    }
    tot[c] = acc;
  }
  __syncthreads();
  if (c < kOrdCls) {
    long long base = 0;
    for (int q = 0; q < c; ++q) base += tot[q];
    for (int b = 0; b < nblocks; ++b) counts[b * kOrdCls + c] += (int)base;
  }
}

// perm[new] = old
template <typename IdxT>
__global__ __launch_bounds__(256) void k_ord_scatter(int64_t n, const IdxT *rp,
                                                     const int *offsets, int32_t *perm) {
  __shared__ int cnt[kOrdCls][256];
  const int per = kOrdRows / 256;
  const int64_t r0 = (int64_t)blockIdx.x * kOrdRows + (int64_t)threadIdx.x * per;
  int local[kOrdCls];
  for (int c = 0; c < kOrdCls; ++c) local[c] = 0;
  for (int t = 0; t < per; ++t) {
    const int64_t i = r0 + t;
    if (i < n) local[ord_class(rp, i)]++;
  }
  for (int c = 0; c < kOrdCls; ++c) cnt[c][threadIdx.x] = local[c];
  __syncthreads();
  if (threadIdx.x < kOrdCls) {
    const int c = threadIdx.x;
    int acc = 0;
    for (int t = 0; t < 256; ++t) {
      const int v = cnt[c][t];
      cnt[c][t] = acc;
      acc += v;
    }
  }
  __syncthreads();
  int pos[kOrdCls];
  for (int c = 0; c < kOrdCls; ++c)
    pos[c] = offsets[blockIdx.x * kOrdCls + c] + cnt[c][threadIdx.x];
  for (int t = 0; t < per; ++t) {
    const int64_t i = r0 + t;
    if (i < n) perm[pos[ord_class(rp, i)]++] = (int32_t)i;
  }
}

template <typename IdxT>
__global__ __launch_bounds__(256) void k_ord_degrees(int64_t n, const IdxT *rp,
                                                     const int32_t *perm, int32_t *inv,
                                                     long long *deg_new) {
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * 256) {
    const int64_t o = perm[p];
    inv[o] = (int32_t)p;
    deg_new[p] = (long long)rp[o + 1] - (long long)rp[o];
  }
}

// exclusive scan of deg_new into the new row pointers: block sums, a scan of
// the block sums (one block), then each block's local scan plus its offset
constexpr int kScanRows = 1024;

__global__ __launch_bounds__(256) void k_scan_sums(int64_t n, const long long *x,
                                                   long long *bsum) {
  __shared__ long long sh[4];
  const int64_t r0 = (int64_t)blockIdx.x * kScanRows;
  long long acc = 0;
  for (int t = threadIdx.x; t < kScanRows; t += 256) {
    const int64_t i = r0 + t;
    if (i < n) acc += x[i];
  }
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) bsum[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ __launch_bounds__(64) void k_scan_bsums(int nb, long long *bsum) {
  if (threadIdx.x == 0) {
    long long acc = 0;
    for (int b = 0; b < nb; ++b) {
      const long long v = bsum[b];
      bsum[b] = acc;
      acc += v;
    }
  }
}

template <typename IdxT>
__global__ __launch_bounds__(256) void k_scan_rows(int64_t n, const long long *x,
                                                   const long long *bsum, IdxT *out) {
  __shared__ long long sh[kScanRows];
  const int64_t r0 = (int64_t)blockIdx.x * kScanRows;
  for (int t = threadIdx.x; t < kScanRows; t += 256) {
    const int64_t i = r0 + t;
    sh[t] = i < n ? x[i] : 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long acc = bsum[blockIdx.x];
    for (int t = 0; t < kScanRows; ++t) {
      const long long v = sh[t];
      sh[t] = acc;
      acc += v;
    }
    if (r0 + kScanRows >= n) out[n] = (IdxT)acc;   // the last block writes the total
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kScanRows; t += 256) {
    const int64_t i = r0 + t;
    if (i < n) out[i] = (IdxT)sh[t];
  }
}

// new row p = old row perm[p], columns renamed by inv: one wavefront per row
template <typename IdxT, typename WT>
__global__ __launch_bounds__(256) void k_ord_rows(int64_t n, const IdxT *rp, const int32_t *col,
                                                  const WT *w, const int32_t *perm,
                                                  const int32_t *inv, const IdxT *rp_new,
                                                  int32_t *col_new, WT *w_new) {
  const int lane = threadIdx.x & 63;
  for (int64_t p = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6; p < n;
       p += ((int64_t)gridDim.x * 256) >> 6) {
    const int64_t o = perm[p];
    const int64_t k0 = rp[o], d = (int64_t)rp[o + 1] - k0, q0 = rp_new[p];
    for (int64_t k = lane; k < d; k += 64) {
      col_new[q0 + k] = inv[col[k0 + k]];
      if constexpr (!std::is_same_v<WT, Unit>) w_new[q0 + k] = w[k0 + k];
    }
  }
}

}  // namespace

size_t degree_order_bytes(const sphx_graph *g) {
  const int64_t n = g->n;
  const int64_t nb = ceil_div(n, kOrdRows);
  const size_t ib = g->rp64 ? 8 : 4;
  const size_t wb = g->wdt == SPHX_F64 ? 8 : (g->wdt == SPHX_F32 ? 4 : 0);
  size_t b = 0;
  b += align_up(sizeof(int32_t) * n, 256) * 2;                 // perm, inv
  b += align_up(ib * (n + 1), 256);                            // row pointers
  b += align_up(sizeof(int32_t) * g->nnz, 256);                // columns
  b += align_up(wb * g->nnz, 256);                             // weights
  b += align_up(sizeof(long long) * n, 256);                   // new degrees
  b += align_up(sizeof(int) * nb * kOrdCls, 256);              // class counts
  b += align_up(sizeof(long long) * ceil_div(n, kScanRows), 256);
  return b + 1024;
}

int build_degree_order(sphx_graph *g, void *scratch, sphx_graph *out, int32_t **perm_out,
                       int32_t **inv_out, hipStream_t s) {
  const int64_t n = g->n;
  const int64_t nb = ceil_div(n, kOrdRows);
  const size_t wb = g->wdt == SPHX_F64 ? 8 : (g->wdt == SPHX_F32 ? 4 : 0);
  Arena a;
  a.base = static_cast<char *>(scratch);
  int32_t *perm = a.take<int32_t>(n);
  int32_t *inv = a.take<int32_t>(n);
  char *rpn = a.take<char>((g->rp64 ? 8 : 4) * (n + 1));
  int32_t *coln = a.take<int32_t>(g->nnz);
  char *wn = a.take<char>(wb * g->nnz);
  long long *degn = a.take<long long>(n);
  int *counts = a.take<int>(nb * kOrdCls);
  long long *bsum = a.take<long long>(ceil_div(n, kScanRows));
  const unsigned gs = (unsigned)ceil_div(n, kScanRows);
  auto go = [&](auto idx_tag, auto w_tag) {
    using IdxT = decltype(idx_tag);
    using WT = decltype(w_tag);
    const IdxT *rp = static_cast<const IdxT *>(g->rowptr);
    hipLaunchKernelGGL((k_ord_count<IdxT>), dim3((unsigned)nb), dim3(256), 0, s, n, rp, counts);
    hipLaunchKernelGGL(k_ord_scan, dim3(1), dim3(64), 0, s, (int)nb, counts);
    hipLaunchKernelGGL((k_ord_scatter<IdxT>), dim3((unsigned)nb), dim3(256), 0, s, n, rp,
                       (const int *)counts, perm);
    hipLaunchKernelGGL((k_ord_degrees<IdxT>), dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, n,
                       rp, (const int32_t *)perm, inv, degn);
    hipLaunchKernelGGL(k_scan_sums, dim3(gs), dim3(256), 0, s, n, (const long long *)degn, bsum);
    hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(64), 0, s, (int)gs, bsum);
    hipLaunchKernelGGL((k_scan_rows<IdxT>), dim3(gs), dim3(256), 0, s, n,
                       (const long long *)degn, (const long long *)bsum, (IdxT *)rpn);
    hipLaunchKernelGGL((k_ord_rows<IdxT, WT>), dim3(grid_for(n, 4, 8192)), dim3(256), 0, s, n,
                       rp, g->col, static_cast<const WT *>(g->w), (const int32_t *)perm,
                       (const int32_t *)inv, (const IdxT *)rpn, coln, (WT *)wn);
  };
  with_types(g, go);
  SPHX_HIP(g->h, hipGetLastError());
  *out = *g;
  out->rowptr = rpn;
  out->col = coln;
  out->w = wb ? wn : nullptr;
  out->vwgt = nullptr;
  out->stats_valid = 0;
  *perm_out = perm;
  *inv_out = inv;
  return SPHX_OK;
}

// the int16 column offsets are kept for unit-weight graphs with 32-bit row
// pointers that are (or may be, before their degrees are known) unbinned
static bool may_compress(const sphx_graph *g) {
  return g->wdt == SPHX_UNIT && !g->rp64 && (!g->stats_valid || g->max_deg <= kUnbinnedMaxDeg);
}

size_t plan_bytes(sphx_graph *g) {
  int64_t n = g->n;
  int64_t nb = ceil_div(n, kBinRows);
  int64_t max_hub = g->nnz / kHubDeg + 1;
  int64_t max_chunks = g->nnz / kHubChunk + max_hub + 1;
  size_t b = 0;
  b += align_up(sizeof(int32_t) * n, 256);              // packed class lists
  b += align_up(sizeof(int32_t) * (max_hub + 1), 256);  // hub chunk begin
  b += align_up(sizeof(int64_t) * max_chunks, 256) * 2; // chunk ranges
  b += align_up(sizeof(double) * max_chunks * kMaxNev, 256);
  b += align_up(sizeof(int) * (nb * kNumCls + kNumCls), 256);
  if (may_compress(g)) b += align_up(sizeof(int16_t) * g->nnz, 256) + 256;
  return b + 4096;
}

int build_plan(sphx_graph *g, Arena &ws, SpmmPlan *plan, const DegreeStats &st,
               void *pinned, hipStream_t s) {
  *plan = SpmmPlan{};
  int64_t n = g->n;
  int64_t nb = ceil_div(n, kBinRows);
  int64_t max_hub = g->nnz / kHubDeg + 1;
  int64_t max_chunks = g->nnz / kHubChunk + max_hub + 1;
  int32_t *packed = ws.take<int32_t>(n);
  int32_t *hcb = ws.take<int32_t>(max_hub + 1);
  int64_t *k0 = ws.take<int64_t>(max_chunks);
  int64_t *k1 = ws.take<int64_t>(max_chunks);
  double *hp = ws.take<double>(max_chunks * kMaxNev);
  int *counts = ws.take<int>(nb * kNumCls + kNumCls);
  if (st.max_deg <= kUnbinnedMaxDeg) {   // natural order, one group size
    plan->group = st.max_deg <= bin_max_deg(0) ? bin_group(0) : bin_group(1);
    if (may_compress(g) && g->nnz > 0) {
      int16_t *d = ws.take<int16_t>(g->nnz);
      int *flag = ws.take<int>(4);
      hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, flag, 4, 0);
      hipLaunchKernelGGL(k_delta16, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, n,
                         (const int32_t *)g->rowptr, g->col, d, flag);
      SPHX_HIP(g->h, hipGetLastError());
      int *hf = static_cast<int *>(pinned);
      SPHX_HIP(g->h, hipMemcpyAsync(hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
      SPHX_HIP(g->h, hipStreamSynchronize(s));
      if (hf[0] == 0) plan->dcol = d;
    }
    return SPHX_OK;
  }
  plan->binned = true;
  int *totals = counts + nb * kNumCls;
  if (g->rp64) {
    hipLaunchKernelGGL((k_bin_count<int64_t>), dim3(nb), dim3(256), 0, s, n,
                       (const int64_t *)g->rowptr, counts);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1), 0, s, (int)nb, counts, totals);
    hipLaunchKernelGGL((k_bin_scatter<int64_t>), dim3(nb), dim3(256), 0, s, n,
                       (const int64_t *)g->rowptr, counts, packed);
  } else {
    hipLaunchKernelGGL((k_bin_count<int32_t>), dim3(nb), dim3(256), 0, s, n,
                       (const int32_t *)g->rowptr, counts);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1), 0, s, (int)nb, counts, totals);
    hipLaunchKernelGGL((k_bin_scatter<int32_t>), dim3(nb), dim3(256), 0, s, n,
                       (const int32_t *)g->rowptr, counts, packed);
  }
  SPHX_HIP(g->h, hipGetLastError());
  int *th = static_cast<int *>(pinned);
  SPHX_HIP(g->h, hipMemcpyAsync(th, totals, sizeof(int) * kNumCls, hipMemcpyDeviceToHost, s));
  SPHX_HIP(g->h, hipStreamSynchronize(s));
  int64_t base = 0;
  for (int c = 0; c < kNumBins; ++c) {
    plan->rows[c] = packed + base;
    plan->nrows[c] = th[c];
    base += th[c];
  }
  const int32_t *l2 = packed + base;
  plan->hub_rows = l2;
  plan->n_hub = th[kNumBins];
  plan->hub_chunk_begin = hcb;
  plan->chunk_k0 = k0;
  plan->chunk_k1 = k1;
  plan->hub_partial = hp;
  if (plan->n_hub > 0) {
    // chunk table on the host (hub rows are few)
    int64_t nh = plan->n_hub;
    std::vector<int32_t> rows(nh);
    SPHX_HIP(g->h, hipMemcpyAsync(rows.data(), l2, sizeof(int32_t) * nh,
                                  hipMemcpyDeviceToHost, s));
    std::vector<int64_t> rb(nh), re(nh);
    SPHX_HIP(g->h, hipStreamSynchronize(s));
    size_t esz = g->rp64 ? 8 : 4;
    for (int64_t q = 0; q < nh; ++q) {
      int64_t i = rows[q];
      int64_t pair[2] = {0, 0};
      if (g->rp64) {
        SPHX_HIP(g->h, hipMemcpy(pair, (const char *)g->rowptr + esz * i, 16,
                                 hipMemcpyDeviceToHost));
      } else {
        int32_t p32[2];
        SPHX_HIP(g->h, hipMemcpy(p32, (const char *)g->rowptr + esz * i, 8,
                                 hipMemcpyDeviceToHost));
        pair[0] = p32[0];
        pair[1] = p32[1];
      }
      rb[q] = pair[0];
      re[q] = pair[1];
    }
    std::vector<int32_t> begin(nh + 1);
    std::vector<int64_t> c0, c1;
    for (int64_t q = 0; q < nh; ++q) {
      begin[q] = (int32_t)c0.size();
      for (int64_t k = rb[q]; k < re[q]; k += kHubChunk) {
        c0.push_back(k);
        c1.push_back(std::min<int64_t>(k + kHubChunk, re[q]));
      }
    }
    begin[nh] = (int32_t)c0.size();
    plan->n_chunks = (int64_t)c0.size();
    SPHX_HIP(g->h, hipMemcpyAsync(hcb, begin.data(), sizeof(int32_t) * (nh + 1),
                                  hipMemcpyHostToDevice, s));
    SPHX_HIP(g->h, hipMemcpyAsync(k0, c0.data(), sizeof(int64_t) * c0.size(),
                                  hipMemcpyHostToDevice, s));
    SPHX_HIP(g->h, hipMemcpyAsync(k1, c1.data(), sizeof(int64_t) * c1.size(),
                                  hipMemcpyHostToDevice, s));
    SPHX_HIP(g->h, hipStreamSynchronize(s));
  }
  return SPHX_OK;
}

}  // namespace sphx
