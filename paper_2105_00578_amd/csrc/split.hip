// Coordinate split of the spectral embedding into K parts (Algorithm 2, the
// multi-jagged split of Sec. 4).
//
// One level per prime factor p of K, largest first; level l splits every
// current section into p children along coordinate l mod ncoord.  The
// members of a section are ordered by the composite key (value, vertex id),
// value mapped to an order-preserving unsigned integer with -0 == +0, so every
// key is unique.  Cut j (1 <= j < p) of a section of weight W follows the
// prefix whose weight C minimises |p C - j W|, the shorter prefix on ties
// (for p = 2: |2 W_lo - W|); children are the members between consecutive
// cuts and part ids are the mixed-radix digits, most significant first.
//
// A cut is found without sorting: for every (section, cut) target a radix
// select over the bytes of the composite key (most significant first) finds
// the first member e* whose inclusive prefix weight C reaches j W / p; e*
// itself is included iff that brings |p C - j W| strictly down.  Integer
// vertex weights make every histogram exact, so the result does not depend
// on the order of the atomic additions.
#include <algorithm>
#include <vector>

#include "kernels.h"

namespace sphx {
namespace {

template <typename T> struct Ord;
template <> struct Ord<float> {
  using K = uint32_t;
  __device__ static K map(float v, bool &nan) {
    if (v != v) { nan = true; return 0; }
    if (v == 0.0f) v = 0.0f;                      // -0 -> +0
    uint32_t u = __float_as_uint(v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  }
};
template <> struct Ord<double> {
  using K = uint64_t;
  __device__ static K map(double v, bool &nan) {
    if (v != v) { nan = true; return 0; }
    if (v == 0.0) v = 0.0;
    uint64_t u = (uint64_t)__double_as_longlong(v);
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
  }
};

template <typename T>
__global__ void k_keys(const T *coords, int ld, int c, int64_t n, typename Ord<T>::K *keys,
                       int *flag) {
  bool nan = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    keys[i] = Ord<T>::map(coords[i * ld + c], nan);
  if (nan) atomicOr(flag, 1);
}

// byte d of the composite key (ord, id), most significant first
template <typename K>
__device__ __forceinline__ int digit(K ord, uint32_t id, int d) {
  constexpr int OB = sizeof(K);
  if (d < OB) return (int)((ord >> (8 * (OB - 1 - d))) & 0xFF);
  return (int)((id >> (8 * (3 - (d - OB)))) & 0xFF);
}

// do the first d bytes of (ord, id) equal those of the prefix (pord, pid)?
// (prefix bytes beyond d are zero)
template <typename K>
__device__ __forceinline__ bool prefix_match(K ord, uint32_t id, K pord, uint32_t pid, int d) {
  constexpr int OB = sizeof(K);
  if (d == 0) return true;
  if (d < OB) {
    K mask = ~K(0) << (8 * (OB - d));
    return (ord & mask) == pord;
  }
  if (ord != pord) return false;
  int dd = d - OB;
  if (dd == 0) return true;
  uint32_t mask = dd >= 4 ? ~0u : (~0u << (8 * (4 - dd)));
  return (id & mask) == pid;
}

// Up to 32 targets count in LDS first (16 or 32 rows of 256 bins), more in
// global memory.
constexpr int kLdsTargets = 32;

// Histogram of byte d over the members of every target's section whose first
// d key bytes match the target's prefix.  Target t = s * (p - 1) + j - 1.
// LT: targets held in LDS (0: global atomics).
template <typename K, int LT>
__global__ __launch_bounds__(256) void k_hist(int64_t n, const K *__restrict__ keys,
                                              const int32_t *__restrict__ part,
                                              const int32_t *__restrict__ vwgt, int d, int p,
                                              int ntgt, const K *__restrict__ pord,
                                              const uint32_t *__restrict__ pid,
                                              unsigned long long *hist) {
  constexpr bool kLds = LT > 0;
  __shared__ unsigned long long h[kLds ? LT * 256 : 1];
  if constexpr (kLds) {
    for (int e = threadIdx.x; e < ntgt * 256; e += blockDim.x) h[e] = 0;
    __syncthreads();
  }
  const int pm = p - 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int s = part[i];
    const K o = keys[i];
    const uint32_t id = (uint32_t)i;
    const unsigned long long wt = vwgt ? (unsigned long long)vwgt[i] : 1ull;
    const int b = digit(o, id, d);
    for (int j = 0; j < pm; ++j) {
      const int t = s * pm + j;
      if (!prefix_match(o, id, pord[t], pid[t], d)) continue;
      if constexpr (kLds) atomicAdd(&h[t * 256 + b], wt);
      else atomicAdd(&hist[(int64_t)t * 256 + b], wt);
    }
  }
  if constexpr (kLds) {
    __syncthreads();
    for (int e = threadIdx.x; e < ntgt * 256; e += blockDim.x)
      if (h[e]) atomicAdd(&hist[e], h[e]);
  }
}

// One wavefront per target: choose byte d (the first bucket where p * C
// reaches j * W), clear the histogram row.  Lane l holds buckets 4l .. 4l+3;
// the weight before a lane's buckets is an exclusive scan over the lanes, and
// the lowest lane with a qualifying bucket holds the choice.
template <typename K>
__global__ __launch_bounds__(256) void k_select(int ntgt, int p, int d, int nd,
                                                unsigned long long *hist, K *pord,
                                                uint32_t *pid, long long *base,
                                                const long long *W, long long *wstar) {
  constexpr int OB = sizeof(K);
  const int lane = threadIdx.x & 63;
  const int t = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (t >= ntgt) return;   // wave-uniform
  const int s = t / (p - 1);
  const long long jW = (long long)(t % (p - 1) + 1) * W[s];
  unsigned long long *row = hist + (int64_t)t * 256 + 4 * lane;
  long long v[4], local = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    v[u] = (long long)row[u];
    row[u] = 0;
    local += v[u];
  }
  long long incl = local;
  for (int off = 1; off < 64; off <<= 1) {
    const long long y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  long long cum = base[t] + (incl - local);
  int pick = -1;
  long long hb = 0, at = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if (pick < 0) {
      if (v[u] > 0 && (long long)p * (cum + v[u]) >= jW) {
        pick = 4 * lane + u;
        hb = v[u];
        at = cum;
      } else {
        cum += v[u];
      }
    }
  }
  const unsigned long long mask = __ballot(pick >= 0);
  if (mask == 0ull) return;   // empty section
  const int first = __ffsll((long long)mask) - 1;
  const int chosen = __shfl(pick, first);
  hb = __shfl(hb, first);
  at = __shfl(at, first);
  if (lane == 0) {
    base[t] = at;
    if (d < OB) pord[t] |= (K)chosen << (8 * (OB - 1 - d));
    else pid[t] |= (uint32_t)chosen << (8 * (3 - (d - OB)));
    if (d == nd - 1) wstar[t] = hb;
  }
}

// Per target: include e* or not; lo[t] = weight of the prefix before the cut.
__global__ void k_finish_targets(int ntgt, int p, const long long *base, const long long *W,
                                 const long long *wstar, int *incl, long long *lo) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntgt) return;
  const int s = t / (p - 1);
  const long long Ws = W[s], b = base[t], ws = wstar[t];
  const long long jW = (long long)(t % (p - 1) + 1) * Ws;
  int inc = 0;
  if (Ws > 0) inc = ((long long)p * (b + ws) - jW) < (jW - (long long)p * b) ? 1 : 0;
  incl[t] = inc;
  lo[t] = Ws > 0 ? b + (inc ? ws : 0) : 0;
}

// Per section: the weights of its p children.
__global__ void k_finish_sections(int nsec, int p, const long long *lo, const long long *W,
                                  long long *Wnext) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsec) return;
  long long prev = 0;
  for (int c = 0; c < p; ++c) {
    const long long cur = c < p - 1 ? lo[s * (p - 1) + c] : W[s];
    Wnext[(int64_t)s * p + c] = cur - prev;
    prev = cur;
  }
}

// child = number of cuts of the member's section that it lies after
template <typename K>
__global__ void k_assign(int64_t n, const K *keys, int32_t *part, int p, const K *pord,
                         const uint32_t *pid, const int *incl, const long long *W) {
  const int pm = p - 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int s = part[i];
    const K o = keys[i];
    const uint32_t id = (uint32_t)i;
    int child = 0;
    if (W[s] != 0)
      for (int j = 0; j < pm; ++j) {
        const int t = s * pm + j;
        const K po = pord[t];
        const uint32_t pi = pid[t];
        bool low;
        if (o != po) low = o < po;
        else if (id != pi) low = id < pi;
        else low = incl[t] != 0;
        child += low ? 0 : 1;
      }
    part[i] = s * p + child;
  }
}

template <typename K>
__global__ void k_reset(int nsec, K *pord, uint32_t *pid, long long *base) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nsec) { pord[s] = 0; pid[s] = 0; base[s] = 0; }
}

__global__ void k_wsum(int64_t n, const int32_t *vwgt, long long *out) {
  long long acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += vwgt ? vwgt[i] : 1;
  atomicAdd((unsigned long long *)out, (unsigned long long)acc);
}

}  // namespace

size_t split_scratch_bytes(int64_t n, int K) {
  // targets of a level (nsec * (p - 1)), sections and children all fit in K
  int64_t ns = K < 1 ? 1 : K;
  size_t b = 0;
  b += align_up(sizeof(uint64_t) * n, 256);                 // keys
  b += align_up(sizeof(unsigned long long) * ns * 256, 256); // hist (one row per target)
  b += align_up(sizeof(uint64_t) * ns, 256);                // pord
  b += align_up(sizeof(uint32_t) * ns, 256);                // pid
  b += align_up(sizeof(long long) * ns, 256) * 4;           // base, wstar, W, lo
  b += align_up(sizeof(long long) * ns, 256);               // Wnext
  b += align_up(sizeof(int) * ns, 256);                     // incl
  b += 1024;
  return b;
}

std::vector<int> section_counts(int K) {
  std::vector<int> f;
  int k = K;
  for (int q = 2; (int64_t)q * q <= k; ++q)
    while (k % q == 0) {
      f.push_back(q);
      k /= q;
    }
  if (k > 1) f.push_back(k);
  std::sort(f.begin(), f.end(), [](int a, int b) { return a > b; });
  return f;
}

template <typename T>
int split_mj(sphx_graph *g, const T *coords, int ld, int ncoord, int K, int32_t *part,
             void *scratch, void *pinned, hipStream_t s, std::string *err) {
  using KT = typename Ord<T>::K;
  const int64_t n = g->n;
  const std::vector<int> counts = section_counts(K);
  Arena a;
  a.base = static_cast<char *>(scratch);
  a.cap = split_scratch_bytes(n, K);
  KT *keys = a.take<KT>(n);
  unsigned long long *hist = a.take<unsigned long long>((size_t)K * 256);
  KT *pord = a.take<KT>(K);
  uint32_t *pid = a.take<uint32_t>(K);
  long long *base = a.take<long long>(K);
  long long *wstar = a.take<long long>(K);
  long long *W = a.take<long long>(K);
  long long *lo = a.take<long long>(K);
  long long *Wnext = a.take<long long>(K);
  int *incl = a.take<int>(K);
  int *flag = a.take<int>(4);
  bool ok = hipMemsetAsync(part, 0, sizeof(int32_t) * n, s) == hipSuccess;
  ok &= hipMemsetAsync(hist, 0, sizeof(unsigned long long) * (size_t)K * 256, s) == hipSuccess;
  ok &= hipMemsetAsync(W, 0, sizeof(long long) * K, s) == hipSuccess;
  ok &= hipMemsetAsync(flag, 0, sizeof(int) * 4, s) == hipSuccess;
  hipLaunchKernelGGL(k_wsum, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, n, g->vwgt, W);
  const int nd = (int)sizeof(KT) + 4;
  const unsigned gn = grid_for(n, 256, 4096);
  int nsec = 1;
  for (size_t l = 0; l < counts.size(); ++l) {
    const int p = counts[l];
    const int ntgt = nsec * (p - 1);
    const int c = (int)(l % (size_t)ncoord);
    const unsigned gt = grid_for(ntgt, 256, 1 << 16);
    const unsigned gw = (unsigned)ceil_div(ntgt, 4);   // one wavefront per target
    hipLaunchKernelGGL((k_keys<T>), dim3(gn), dim3(256), 0, s, coords, ld, c, n, keys, flag);
    hipLaunchKernelGGL((k_reset<KT>), dim3(gt), dim3(256), 0, s, ntgt, pord, pid, base);
    for (int d = 0; d < nd; ++d) {
      if (ntgt <= 16)
        hipLaunchKernelGGL((k_hist<KT, 16>), dim3(gn), dim3(256), 0, s, n, keys, part,
                           g->vwgt, d, p, ntgt, pord, pid, hist);
      else if (ntgt <= kLdsTargets)
        hipLaunchKernelGGL((k_hist<KT, kLdsTargets>), dim3(gn), dim3(256), 0, s, n, keys, part,
                           g->vwgt, d, p, ntgt, pord, pid, hist);
      else
        hipLaunchKernelGGL((k_hist<KT, 0>), dim3(gn), dim3(256), 0, s, n, keys, part,
                           g->vwgt, d, p, ntgt, pord, pid, hist);
      hipLaunchKernelGGL((k_select<KT>), dim3(gw), dim3(256), 0, s, ntgt, p, d, nd, hist, pord,
                         pid, base, W, wstar);
    }
    hipLaunchKernelGGL(k_finish_targets, dim3(gt), dim3(256), 0, s, ntgt, p, base, W, wstar,
                       incl, lo);
    hipLaunchKernelGGL(k_finish_sections, dim3(grid_for(nsec, 256, 1 << 16)), dim3(256), 0, s,
                       nsec, p, lo, W, Wnext);
    hipLaunchKernelGGL((k_assign<KT>), dim3(gn), dim3(256), 0, s, n, keys, part, p, pord, pid,
                       incl, W);
    nsec *= p;
    ok &= hipMemcpyAsync(W, Wnext, sizeof(long long) * nsec, hipMemcpyDeviceToDevice, s) ==
          hipSuccess;
  }
  if (!ok || hipGetLastError() != hipSuccess) {
    *err = "split kernel launch failed";
    return SPHX_E_HIP;
  }
  int *fh = static_cast<int *>(pinned);
  if (hipMemcpyAsync(fh, flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    *err = "split: stream error";
    return SPHX_E_HIP;
  }
  if (*fh) {
    *err = "NaN coordinate";
    return SPHX_E_INVALID_ARG;
  }
  return SPHX_OK;
}

template int split_mj<float>(sphx_graph *, const float *, int, int, int, int32_t *, void *,
                             void *, hipStream_t, std::string *);
template int split_mj<double>(sphx_graph *, const double *, int, int, int, int32_t *, void *,
                              void *, hipStream_t, std::string *);

}  // namespace sphx
