// Partition quality (Sec. 3.1): cutsize of Eq. 1, part weights W_k and the
// imbalance max_k W_k / W_avg.
//
// Exactness: unit weights are counted in int64.  Float edge weights are
// summed exactly in 128-bit fixed point: with e0 the exponent of the last
// mantissa bit of the smallest weight, every weight is an integer multiple of
// 2^e0, so the cut is an exact integer times 2^e0, rounded once at the end.
#include <cmath>

#include "fixed.h"
#include "kernels.h"

namespace sphx {
namespace {

// Each block takes contiguous chunks of kCutChunk CSR entries; thread t
// reads entries k0 + t + 256 q, so every load is coalesced.  The row of an
// entry (the largest i with row_ptr[i] <= k) is found by binary search over
// the chunk's rows, whose row_ptr values are staged in LDS when they fit.
// Each thread accumulates an exact partial.
constexpr int kCutChunk = 256 * 16;
constexpr int kCutRows = 4096;

template <typename IdxT, typename WT>
__global__ __launch_bounds__(256) void k_cut(int64_t n, int64_t nnz, const IdxT *rp,
                                             const int32_t *col, const WT *w,
                                             const int32_t *part, int e0,
                                             unsigned long long *out) {
  __shared__ int64_t srp[kCutRows + 1];
  __shared__ int64_t bounds[2];
  U128 acc{0, 0};
  const int tid = threadIdx.x;
  auto row_of = [&](int64_t k, int64_t lo, int64_t hi, bool lds) {
    // largest i in [lo, hi] with row_ptr[i] <= k (row_ptr[lo] <= k holds)
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      const int64_t v = lds ? srp[mid - bounds[0]] : (int64_t)rp[mid];
      if (v <= k) lo = mid;
      else hi = mid - 1;
    }
    return lo;
  };
  for (int64_t c = blockIdx.x; c * kCutChunk < nnz; c += gridDim.x) {
    const int64_t k0 = c * kCutChunk;
    const int64_t k1 = min(nnz, k0 + kCutChunk);
    if (tid == 0) {
      bounds[0] = row_of(k0, 0, n - 1, false);
      bounds[1] = row_of(k1 - 1, bounds[0], n - 1, false);
    }
    __syncthreads();
    const int64_t r0 = bounds[0], r1 = bounds[1];
    const bool lds = r1 - r0 + 1 <= kCutRows;
    if (lds)
      for (int64_t i = tid; i <= r1 - r0; i += 256) srp[i] = (int64_t)rp[r0 + i];
    __syncthreads();
    for (int64_t k = k0 + tid; k < k1; k += 256) {
      const int64_t i = row_of(k, r0, r1, lds);
      const int64_t j = col[k];
      if (j <= i || part[j] == part[i]) continue;
      if constexpr (std::is_same_v<WT, Unit>) add128(acc, 1ull, 0ull);
      else {
        unsigned long long l, h;
        fixed_of(w[k], e0, l, h);
        add128(acc, l, h);
      }
    }
    __syncthreads();   // srp and bounds are rewritten for the next chunk
  }
  __shared__ unsigned long long slo[256], shi[256];
  slo[tid] = acc.lo;
  shi[tid] = acc.hi;
  __syncthreads();
  if (tid == 0) {
    U128 t{0, 0};
    for (int u = 0; u < (int)blockDim.x; ++u) add128(t, slo[u], shi[u]);
    out[2 * blockIdx.x] = t.lo;
    out[2 * blockIdx.x + 1] = t.hi;
  }
}

// Part weights: integer sums, so the order of the additions does not matter.
// Up to kLdsParts parts are counted in LDS first (no global contention).
constexpr int kLdsParts = 4096;

__global__ __launch_bounds__(256) void k_part_weights(int64_t n, const int32_t *part,
                                                      const int32_t *vwgt, int K,
                                                      unsigned long long *pw, int *bad) {
  __shared__ unsigned long long h[kLdsParts];
  const bool lds = K <= kLdsParts;
  if (lds) {
    for (int k = threadIdx.x; k < K; k += blockDim.x) h[k] = 0;
    __syncthreads();
  }
  int f = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int p = part[i];
    if (p < 0 || p >= K) { f = 1; continue; }
    unsigned long long wt = (unsigned long long)(vwgt ? vwgt[i] : 1);
    if (lds) atomicAdd(&h[p], wt);
    else atomicAdd(&pw[p], wt);
  }
  if (f) atomicOr(bad, 1);
  if (lds) {
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x)
      if (h[k]) atomicAdd(&pw[k], h[k]);
  }
}

constexpr int kCutBlocks = 1024;

// Clears n 64-bit words (a kernel rather than a memset node, so that the
// clearing is an ordinary launch on the stream).
__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

double u128_to_double(unsigned __int128 v) {
  if (v == 0) return 0.0;
  int nb = 0;
  for (unsigned __int128 t = v; t; t >>= 1) ++nb;
  if (nb <= 53) return (double)(unsigned long long)v;
  int sh = nb - 53;
  unsigned __int128 top = v >> sh;
  unsigned __int128 rem = v - (top << sh);
  unsigned __int128 half = (unsigned __int128)1 << (sh - 1);
  if (rem > half || (rem == half && (top & 1))) top += 1;   // nearest, ties to even
  return std::ldexp((double)(unsigned long long)top, sh);
}

}  // namespace

size_t quality_scratch_bytes(int K) {
  return align_up(sizeof(unsigned long long) * 2 * kCutBlocks, 256) +
         align_up(sizeof(unsigned long long) * (size_t)(K > 0 ? K : 1), 256) + 1024;
}

int quality(sphx_graph *g, const int32_t *part, int K, double *cut, double *imbalance,
            int64_t *part_weights, void *scratch, void *pinned, hipStream_t s,
            std::string *err, unsigned __int128 *cut_fixed) {
  Arena a;
  a.base = static_cast<char *>(scratch);
  unsigned long long *cp = a.take<unsigned long long>(2 * kCutBlocks);
  unsigned long long *pw = a.take<unsigned long long>(K);
  // the bad-part flag shares the zeroed region: one 64-bit word after pw
  unsigned long long *bad = a.take<unsigned long long>(1);
  // the weight range (and its e0) is known from the degree pass
  int e0 = 0;
  if (g->wdt == SPHX_F32) e0 = fixed_exponent<float>(g->wmin);
  if (g->wdt == SPHX_F64) e0 = fixed_exponent<double>(g->wmin);
  const int64_t nz = (int64_t)(reinterpret_cast<char *>(bad + 1) -
                               reinterpret_cast<char *>(pw)) / 8;
  hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(nz, 256, 1024)), dim3(256), 0, s, pw, nz);
  hipLaunchKernelGGL(k_part_weights, dim3(grid_for(g->n, 256 * 16, 1024)), dim3(256), 0, s,
                     g->n, part, g->vwgt, K, pw, reinterpret_cast<int *>(bad));
  const unsigned nb = grid_for(g->nnz, kCutChunk, kCutBlocks);
  auto go = [&](auto it, auto wt) {
    using IdxT = decltype(it);
    using WT = decltype(wt);
    hipLaunchKernelGGL((k_cut<IdxT, WT>), dim3(nb), dim3(256), 0, s, g->n, g->nnz,
                       (const IdxT *)g->rowptr, g->col, (const WT *)g->w, part, e0, cp);
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
  if (hipGetLastError() != hipSuccess) {
    *err = "quality kernel launch failed";
    return SPHX_E_HIP;
  }
  // results come back through the pinned host buffer (kQualityPinnedWords
  // 64-bit words): the cut partials and flag first, then the part weights in
  // chunks, so no host memory is allocated here
  unsigned long long *hb = static_cast<unsigned long long *>(pinned);
  if (hipMemcpyAsync(hb, cp, sizeof(unsigned long long) * 2 * nb, hipMemcpyDeviceToHost,
                     s) != hipSuccess ||
      hipMemcpyAsync(hb + 2 * kCutBlocks, bad, sizeof(unsigned long long),
                     hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    *err = "quality: copy failed";
    return SPHX_E_HIP;
  }
  if (hb[2 * kCutBlocks]) {
    *err = "part id out of range [0, K)";
    return SPHX_E_INVALID_ARG;
  }
  unsigned __int128 tot = 0;
  for (unsigned b = 0; b < nb; ++b)
    tot += ((unsigned __int128)hb[2 * b + 1] << 64) + hb[2 * b];
  if (cut_fixed) *cut_fixed = tot;
  double c = u128_to_double(tot);
  if (g->wdt != SPHX_UNIT) c = std::ldexp(c, e0);
  if (cut) *cut = c;
  unsigned long long mx = 0, sum = 0;
  for (int k0 = 0; k0 < K; k0 += kQualityPinnedWords) {
    const int cnt = std::min(K - k0, kQualityPinnedWords);
    if (hipMemcpyAsync(hb, pw + k0, sizeof(unsigned long long) * cnt, hipMemcpyDeviceToHost,
                       s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      *err = "quality: copy failed";
      return SPHX_E_HIP;
    }
    for (int k = 0; k < cnt; ++k) {
      mx = std::max(mx, hb[k]);
      sum += hb[k];
      if (part_weights) part_weights[k0 + k] = (int64_t)hb[k];
    }
  }
  if (imbalance) *imbalance = sum ? (double)(mx * (unsigned long long)K) / (double)sum : 1.0;
  return SPHX_OK;
}

}  // namespace sphx
