// Coordinate split of the spectral embedding into K = 2^L parts (Algorithm 2,
// the multi-jagged split specialised to bisections, Sec. 4).
//
// Level l bisects every current section along coordinate l mod ncoord.  The
// members of a section are ordered by the composite key (value, vertex id),
// value mapped to an order-preserving unsigned integer with -0 == +0, so every
// key is unique.  The lower child receives the prefix whose weight W_lo
// minimises |2 W_lo - W|, the shorter prefix on ties.
//
// The prefix end is found without sorting: for every section a radix select
// over the bytes of the composite key (most significant first) finds the
// first member e* whose inclusive prefix weight reaches W/2; e* itself goes
// low iff that brings |2 W_lo - W| strictly down.  Integer vertex weights
// make every histogram exact, so the result does not depend on the order of
// the atomic additions.
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

constexpr int kLdsSections = 16;

template <typename K, bool kLds>
__global__ __launch_bounds__(256) void k_hist(int64_t n, const K *__restrict__ keys,
                                              const int32_t *__restrict__ part,
                                              const int32_t *__restrict__ vwgt, int d,
                                              int nsec, const K *__restrict__ pord,
                                              const uint32_t *__restrict__ pid,
                                              unsigned long long *hist) {
  __shared__ unsigned long long h[kLds ? kLdsSections * 256 : 1];
  if constexpr (kLds) {
    for (int e = threadIdx.x; e < nsec * 256; e += blockDim.x) h[e] = 0;
    __syncthreads();
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int s = part[i];
    K o = keys[i];
    uint32_t id = (uint32_t)i;
    if (!prefix_match(o, id, pord[s], pid[s], d)) continue;
    unsigned long long wt = vwgt ? (unsigned long long)vwgt[i] : 1ull;
    int b = digit(o, id, d);
    if constexpr (kLds) atomicAdd(&h[s * 256 + b], wt);
    else atomicAdd(&hist[(int64_t)s * 256 + b], wt);
  }
  if constexpr (kLds) {
    __syncthreads();
    for (int e = threadIdx.x; e < nsec * 256; e += blockDim.x)
      if (h[e]) atomicAdd(&hist[e], h[e]);
  }
}

// One thread per section: choose byte d, clear the histogram row.
template <typename K>
__global__ void k_select(int nsec, int d, int nd, unsigned long long *hist, K *pord,
                         uint32_t *pid, long long *base, const long long *W,
                         long long *wstar) {
  constexpr int OB = sizeof(K);
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsec) return;
  long long Ws = W[s];
  long long cum = base[s];
  int chosen = -1;
  long long hb = 0;
  for (int b = 0; b < 256; ++b) {
    long long v = (long long)hist[(int64_t)s * 256 + b];
    hist[(int64_t)s * 256 + b] = 0;
    if (chosen < 0) {
      if (v > 0 && 2 * (cum + v) >= Ws) { chosen = b; hb = v; }
      else cum += v;
    }
  }
  if (chosen < 0) return;   // empty section
  base[s] = cum;
  if (d < OB) pord[s] |= (K)chosen << (8 * (OB - 1 - d));
  else pid[s] |= (uint32_t)chosen << (8 * (3 - (d - OB)));
  if (d == nd - 1) wstar[s] = hb;
}

__global__ void k_finish_level(int nsec, const long long *base, const long long *W,
                               const long long *wstar, int *incl, long long *Wnext) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsec) return;
  long long Ws = W[s], b = base[s], ws = wstar[s];
  int inc = 0;
  if (Ws > 0) inc = (2 * (b + ws) - Ws) < (Ws - 2 * b) ? 1 : 0;
  long long lo = b + (inc ? ws : 0);
  if (Ws == 0) lo = 0;
  incl[s] = inc;
  Wnext[2 * s] = lo;
  Wnext[2 * s + 1] = Ws - lo;
}

template <typename K>
__global__ void k_assign(int64_t n, const K *keys, int32_t *part, const K *pord,
                         const uint32_t *pid, const int *incl, const long long *W) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int s = part[i];
    K o = keys[i];
    uint32_t id = (uint32_t)i;
    K po = pord[s];
    uint32_t pi = pid[s];
    bool low;
    if (W[s] == 0) low = false;
    else if (o != po) low = o < po;
    else if (id != pi) low = id < pi;
    else low = incl[s] != 0;
    part[i] = 2 * s + (low ? 0 : 1);
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
  int64_t ns = K < 1 ? 1 : K;
  size_t b = 0;
  b += align_up(sizeof(uint64_t) * n, 256);                 // keys
  b += align_up(sizeof(unsigned long long) * ns * 256, 256); // hist (K/2 sections max)
  b += align_up(sizeof(uint64_t) * ns, 256);                // pord
  b += align_up(sizeof(uint32_t) * ns, 256);                // pid
  b += align_up(sizeof(long long) * ns, 256) * 3;           // base, wstar, W
  b += align_up(sizeof(long long) * 2 * ns, 256);           // Wnext
  b += align_up(sizeof(int) * ns, 256);                     // incl
  b += 1024;
  return b;
}

template <typename T>
int split_pow2(sphx_graph *g, const T *coords, int ld, int ncoord, int K, int32_t *part,
               void *scratch, void *pinned, hipStream_t s, std::string *err) {
  using KT = typename Ord<T>::K;
  const int64_t n = g->n;
  int levels = 0;
  while ((1 << levels) < K) ++levels;
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
  long long *Wnext = a.take<long long>(2 * (size_t)K);
  int *incl = a.take<int>(K);
  int *flag = a.take<int>(4);
  hipMemsetAsync(part, 0, sizeof(int32_t) * n, s);
  hipMemsetAsync(hist, 0, sizeof(unsigned long long) * (size_t)K * 256, s);
  hipMemsetAsync(W, 0, sizeof(long long) * K, s);
  hipMemsetAsync(flag, 0, sizeof(int) * 4, s);
  hipLaunchKernelGGL(k_wsum, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, n, g->vwgt, W);
  const int nd = (int)sizeof(KT) + 4;
  const unsigned gn = grid_for(n, 256, 4096);
  for (int l = 0; l < levels; ++l) {
    const int nsec = 1 << l;
    const int c = l % ncoord;
    hipLaunchKernelGGL((k_keys<T>), dim3(gn), dim3(256), 0, s, coords, ld, c, n, keys, flag);
    hipLaunchKernelGGL((k_reset<KT>), dim3(grid_for(nsec, 256, 1 << 16)), dim3(256), 0, s,
                       nsec, pord, pid, base);
    for (int d = 0; d < nd; ++d) {
      if (nsec <= kLdsSections)
        hipLaunchKernelGGL((k_hist<KT, true>), dim3(gn), dim3(256), 0, s, n, keys, part,
                           g->vwgt, d, nsec, pord, pid, hist);
      else
        hipLaunchKernelGGL((k_hist<KT, false>), dim3(gn), dim3(256), 0, s, n, keys, part,
                           g->vwgt, d, nsec, pord, pid, hist);
      hipLaunchKernelGGL((k_select<KT>), dim3(grid_for(nsec, 256, 1 << 16)), dim3(256), 0, s,
                         nsec, d, nd, hist, pord, pid, base, W, wstar);
    }
    hipLaunchKernelGGL(k_finish_level, dim3(grid_for(nsec, 256, 1 << 16)), dim3(256), 0, s,
                       nsec, base, W, wstar, incl, Wnext);
    hipLaunchKernelGGL((k_assign<KT>), dim3(gn), dim3(256), 0, s, n, keys, part, pord, pid,
                       incl, W);
    hipMemcpyAsync(W, Wnext, sizeof(long long) * 2 * nsec, hipMemcpyDeviceToDevice, s);
  }
  if (hipGetLastError() != hipSuccess) {
    *err = "split kernel launch failed";
    return SPHX_E_HIP;
  }
  int *fh = static_cast<int *>(pinned);
  hipMemcpyAsync(fh, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) {
    *err = "split: stream error";
    return SPHX_E_HIP;
  }
  if (*fh) {
    *err = "NaN coordinate";
    return SPHX_E_INVALID_ARG;
  }
  return SPHX_OK;
}

template int split_pow2<float>(sphx_graph *, const float *, int, int, int, int32_t *, void *,
                               void *, hipStream_t, std::string *);
template int split_pow2<double>(sphx_graph *, const double *, int, int, int, int32_t *, void *,
                                void *, hipStream_t, std::string *);

}  // namespace sphx
