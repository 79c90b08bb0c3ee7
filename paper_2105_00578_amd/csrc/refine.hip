// Greedy refinement of a K-way partition: Sec. 7 proposes a greedy
// improvement step after the spectral split (moves of single vertices, which
// parallelise where KL/FM does not); balance as defined in Sec. 3.1, every
// part weight below W_avg (1 + eps).
//
// One pass over the current partition pi (c_v vertex weights, w edge weights,
// conn(v, p) the weight of v's edges into part p, C the capacity):
//  1. gains: t(v) = the neighbour part p != pi(v) of largest conn(v, p), the
//     smallest p on ties; g(v) = conn(v, t) - conn(v, pi(v)).  Candidates
//     have g > 0 and 1 <= deg(v) <= kRefineMaxDeg.
//  2. conflicts: candidates are ranked by (g descending, id ascending); v
//     stays a mover when its gain, recomputed with every higher-ranked
//     candidate at its target, is still positive.
//  3. balance: the movers into part p, in increasing id, are accepted while
//     W_p plus their cumulative weight stays <= C (departures not credited).
//  4. accepted movers take their targets.  The pass is kept only when the
//     exact cut drops, and passes repeat while it does.
//
// Every sum is exact (edge counts for unit weights; for float weights the
// 128-bit fixed point of the quality kernel, in units of 2^e0), so every
// comparison is exact and independent of the order of the additions.
#include <cmath>
#include <vector>

#include "fixed.h"
#include "kernels.h"

namespace sphx {
namespace {

using S = __int128;

constexpr int kThreadDeg = 32;        // rows up to this degree: one thread each
constexpr int kRefineMaxDeg = 2048;   // rows above this degree never move
constexpr int kScanBlocks = 1024;

template <typename WT>
__device__ __forceinline__ S wfix(const WT *w, int64_t k, int e0) {
  if constexpr (std::is_same_v<WT, Unit>) {
    return 1;
  } else {
    unsigned long long lo, hi;
    fixed_of(w[k], e0, lo, hi);
    return (S)(((unsigned __int128)hi << 64) | lo);
  }
}

// (c, p) beats (best, t): a larger connection, the smaller part on ties
__device__ __forceinline__ bool better(S c, int p, S best, int t) {
  return p >= 0 && (t < 0 || c > best || (c == best && p < t));
}

// Step 1 for rows of degree <= kThreadDeg (one thread per row, the row's
// neighbour parts in this thread's LDS column).  Rows of larger degree are
// flagged for k_gain_block; empty rows are no candidates.
template <typename IdxT, typename WT>
__global__ __launch_bounds__(256) void k_gain_thread(int64_t n, const IdxT *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     const WT *__restrict__ w, int e0,
                                                     const int32_t *__restrict__ part,
                                                     int32_t *tgt, S *gain, uint8_t *big) {
  __shared__ int32_t sp[kThreadDeg * 256];
  const int tid = threadIdx.x;
  for (int64_t v = (int64_t)blockIdx.x * 256 + tid; v < n; v += (int64_t)gridDim.x * 256) {
    const int64_t lo = rp[v];
    const int64_t d = (int64_t)rp[v + 1] - lo;
    int t = -1;
    S g = 0;
    if (d >= 1 && d <= kThreadDeg) {
      const int a = part[v];
      const int dd = (int)d;
      for (int j = 0; j < dd; ++j) sp[j * 256 + tid] = part[col[lo + j]];
      S ca = 0, best = 0;
      for (int j = 0; j < dd; ++j) {
        const int p = sp[j * 256 + tid];
        if (p == a) {
          ca += wfix(w, lo + j, e0);
          continue;
        }
        bool first = true;
        for (int q = 0; q < j; ++q)
          if (sp[q * 256 + tid] == p) {
            first = false;
            break;
          }
        if (!first) continue;
        S c = 0;
        for (int q = j; q < dd; ++q)
          if (sp[q * 256 + tid] == p) c += wfix(w, lo + q, e0);
        if (better(c, p, best, t)) {
          best = c;
          t = p;
        }
      }
      if (t >= 0 && best - ca > 0) g = best - ca;
      else t = -1;
    }
    tgt[v] = t;
    gain[v] = g;
    big[v] = (d > kThreadDeg && d <= kRefineMaxDeg) ? 1 : 0;
  }
}

// Step 1 for the listed rows (kThreadDeg < degree <= kRefineMaxDeg): one
// block per row, the row's neighbour parts in LDS.  With unit weights and at
// most kLdsParts parts, conn(v, p) is counted in an LDS table indexed by part
// (integer counts: the order of the increments does not matter); otherwise
// each distinct part's connection is summed over the row (first occurrence
// of the part owns the sum).
constexpr int kLdsParts = 8192;

template <typename IdxT, typename WT>
__global__ __launch_bounds__(256) void k_gain_block(const int32_t *__restrict__ rows,
                                                    const int32_t *__restrict__ nrows,
                                                    const IdxT *__restrict__ rp,
                                                    const int32_t *__restrict__ col,
                                                    const WT *__restrict__ w, int e0,
                                                    const int32_t *__restrict__ part, int K,
                                                    int32_t *tgt, S *gain) {
  __shared__ int32_t sp[kRefineMaxDeg];
  __shared__ int32_t cnt[kLdsParts];
  // per-thread candidates and own-part sums, combined by a tree in LDS (the
  // combination is exact and order-free: a maximum under a total order and
  // an integer sum)
  __shared__ S rc[256], ra[256];
  __shared__ int rt[256];
  constexpr bool kUnit = std::is_same_v<WT, Unit>;
  const bool table = kUnit && K <= kLdsParts;
  const int tid = threadIdx.x;
  if (table) {
    for (int k = tid; k < K; k += 256) cnt[k] = 0;
    __syncthreads();
  }
  const int nr = *nrows;
  for (int r = blockIdx.x; r < nr; r += gridDim.x) {
    const int64_t v = rows[r];
    const int64_t lo = rp[v];
    const int d = (int)((int64_t)rp[v + 1] - lo);   // kThreadDeg < d <= kRefineMaxDeg
    const int a = part[v];
    for (int j = tid; j < d; j += 256) {
      const int p = part[col[lo + j]];
      sp[j] = p;
      if (table) atomicAdd(&cnt[p], 1);
    }
    __syncthreads();
    S ca = 0, best = 0;
    int t = -1;
    if (table) {
      if (tid == 0) ca = cnt[a];
      for (int j = tid; j < d; j += 256) {
        const int p = sp[j];
        if (p != a && better((S)cnt[p], p, best, t)) {
          best = cnt[p];
          t = p;
        }
      }
    } else {
      for (int j = tid; j < d; j += 256) {
        const int p = sp[j];
        if (p == a) {
          ca += wfix(w, lo + j, e0);
          continue;
        }
        bool first = true;
        for (int q = 0; q < j; ++q)
          if (sp[q] == p) {
            first = false;
            break;
          }
        if (!first) continue;
        S c = 0;
        for (int q = j; q < d; ++q)
          if (sp[q] == p) c += wfix(w, lo + q, e0);
        if (better(c, p, best, t)) {
          best = c;
          t = p;
        }
      }
    }
    rc[tid] = best;
    rt[tid] = t;
    ra[tid] = ca;
    __syncthreads();
    if (table)   // clear the counts of this row (every read above is done)
      for (int j = tid; j < d; j += 256) cnt[sp[j]] = 0;
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) {
        S B = rc[tid];
        int T = rt[tid];
        if (better(rc[tid + h], rt[tid + h], B, T)) {
          B = rc[tid + h];
          T = rt[tid + h];
        }
        rc[tid] = B;
        rt[tid] = T;
        ra[tid] += ra[tid + h];
      }
      __syncthreads();
    }
    if (tid == 0) {
      const S B = rc[0], A = ra[0];
      const int T = rt[0];
      const bool cand = T >= 0 && B - A > 0;
      tgt[v] = cand ? T : -1;
      gain[v] = cand ? B - A : (S)0;
    }
    __syncthreads();
  }
}

// Step 2: a candidate stays a mover when its gain, with every higher-ranked
// candidate neighbour at its target, is positive.
template <typename IdxT, typename WT>
__device__ __forceinline__ S moved_gain(int64_t v, int64_t k0, int64_t k1, int64_t step,
                                        const int32_t *__restrict__ col,
                                        const WT *__restrict__ w, int e0,
                                        const int32_t *__restrict__ part,
                                        const int32_t *__restrict__ tgt,
                                        const S *__restrict__ gain, int a, int t, S gv) {
  S g2 = 0;
  for (int64_t k = k0; k < k1; k += step) {
    const int64_t u = col[k];
    int pu = part[u];
    const int tu = tgt[u];
    if (tu >= 0) {
      const S gu = gain[u];
      if (gu > gv || (gu == gv && u < v)) pu = tu;
    }
    if (pu == t) g2 += wfix(w, k, e0);
    else if (pu == a) g2 -= wfix(w, k, e0);
  }
  return g2;
}

// rows of degree <= kThreadDeg (and the rows that never move): one thread each
template <typename IdxT, typename WT>
__global__ __launch_bounds__(256) void k_movers(int64_t n, const IdxT *__restrict__ rp,
                                                const int32_t *__restrict__ col,
                                                const WT *__restrict__ w, int e0,
                                                const int32_t *__restrict__ part,
                                                const int32_t *__restrict__ tgt,
                                                const S *__restrict__ gain, uint8_t *mv) {
  for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * 256) {
    const int64_t k0 = rp[v], k1 = rp[v + 1];
    const int64_t d = k1 - k0;
    if (d > kThreadDeg && d <= kRefineMaxDeg) continue;   // k_movers_wave
    const int t = tgt[v];
    uint8_t f = 0;
    if (t >= 0)
      f = moved_gain<IdxT, WT>(v, k0, k1, 1, col, w, e0, part, tgt, gain, part[v], t,
                               gain[v]) > 0
              ? 1
              : 0;
    mv[v] = f;
  }
}

// the listed rows (kThreadDeg < degree <= kRefineMaxDeg): one wave each
template <typename IdxT, typename WT>
__global__ __launch_bounds__(256) void k_movers_wave(const int32_t *__restrict__ rows,
                                                     const int32_t *__restrict__ nrows,
                                                     const IdxT *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     const WT *__restrict__ w, int e0,
                                                     const int32_t *__restrict__ part,
                                                     const int32_t *__restrict__ tgt,
                                                     const S *__restrict__ gain, uint8_t *mv) {
  // lane sums through LDS, added by a tree per wave (exact integer sums: the
  // order does not matter); the row loop is uniform over the block (rows
  // r0 + wave) so every wave reaches the barriers
  __shared__ S lanes[256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nr = *nrows;
  for (int64_t r0 = (int64_t)blockIdx.x * 4; r0 < nr; r0 += (int64_t)gridDim.x * 4) {
    const int64_t r = r0 + wave;
    int64_t v = -1;
    int t = -1;
    S g2 = 0;
    if (r < nr) {
      v = rows[r];
      t = tgt[v];
      if (t >= 0) {
        const int64_t k0 = rp[v], k1 = rp[v + 1];
        g2 = moved_gain<IdxT, WT>(v, k0 + lane, k1, 64, col, w, e0, part, tgt, gain, part[v],
                                  t, gain[v]);
      }
    }
    lanes[threadIdx.x] = g2;
    __syncthreads();
    for (int h = 32; h > 0; h >>= 1) {
      if (lane < h) lanes[threadIdx.x] += lanes[threadIdx.x + h];
      __syncthreads();
    }
    if (lane == 0 && v >= 0) mv[v] = (t >= 0 && lanes[threadIdx.x] > 0) ? 1 : 0;
    __syncthreads();
  }
}

// ---- stable compaction of flagged vertices (increasing id)

__global__ __launch_bounds__(256) void k_flag_count(int64_t n, const uint8_t *__restrict__ f,
                                                    int32_t *cnt) {
  const int64_t per = (n + kScanBlocks - 1) / kScanBlocks;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(n, r0 + per);
  int c = 0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) c += f[i];
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
  __shared__ int sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) cnt[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// exclusive scan of the kScanBlocks counts (one block); total at cnt[kScanBlocks]
__global__ __launch_bounds__(1024) void k_flag_scan(int32_t *cnt) {
  __shared__ int sh[kScanBlocks];
  const int t = threadIdx.x;
  sh[t] = cnt[t];
  __syncthreads();
  for (int off = 1; off < kScanBlocks; off <<= 1) {
    const int x = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  cnt[t] = t ? sh[t - 1] : 0;
  if (t == kScanBlocks - 1) cnt[kScanBlocks] = sh[t];
}

__global__ __launch_bounds__(256) void k_flag_scatter(int64_t n, const uint8_t *__restrict__ f,
                                                      const int32_t *__restrict__ cnt,
                                                      int32_t *list) {
  const int64_t per = (n + kScanBlocks - 1) / kScanBlocks;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(n, r0 + per);
  __shared__ int wc[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int base = cnt[blockIdx.x];
  for (int64_t c0 = r0; c0 < r1; c0 += 256) {
    const int64_t i = c0 + threadIdx.x;
    const bool on = i < r1 && f[i];
    const unsigned long long m = __ballot(on);
    const int below = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wc[wv] = __popcll(m);
    __syncthreads();
    int off = base + below;
    for (int q = 0; q < wv; ++q) off += wc[q];
    if (on) list[off] = (int32_t)i;
    base += wc[0] + wc[1] + wc[2] + wc[3];
    __syncthreads();
  }
}

// ---- step 3: balance

__global__ void k_zero_u64(unsigned long long *x, int64_t cnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0;
}

// total weight of the movers into each part; up to kLdsParts parts are
// summed in LDS first (integer sums: the order does not matter)
__global__ __launch_bounds__(256) void k_arrivals(const int32_t *__restrict__ list,
                                                  const int32_t *__restrict__ count,
                                                  const int32_t *__restrict__ tgt,
                                                  const int32_t *__restrict__ vwgt, int K,
                                                  unsigned long long *arr) {
  __shared__ unsigned long long hst[kLdsParts];
  const bool lds = K <= kLdsParts;
  if (lds) {
    for (int k = threadIdx.x; k < K; k += 256) hst[k] = 0;
    __syncthreads();
  }
  const int M = *count;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < M; i += gridDim.x * 256) {
    const int v = list[i];
    const unsigned long long c = (unsigned long long)(vwgt ? vwgt[v] : 1);
    if (lds) atomicAdd(&hst[tgt[v]], c);
    else atomicAdd(&arr[tgt[v]], c);
  }
  if (lds) {
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += 256)
      if (hst[k]) atomicAdd(&arr[k], hst[k]);
  }
}

// movers into parts that take all their arrivals
__global__ __launch_bounds__(256) void k_accept_all(const int32_t *__restrict__ list,
                                                    const int32_t *__restrict__ count,
                                                    const int32_t *__restrict__ tgt,
                                                    const unsigned long long *__restrict__ W,
                                                    const unsigned long long *__restrict__ arr,
                                                    unsigned long long cap, int32_t *nxt,
                                                    unsigned long long *moved) {
  const int M = *count;
  unsigned long long c = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < M; i += gridDim.x * 256) {
    const int v = list[i];
    const int t = tgt[v];
    if (W[t] + arr[t] <= cap) {
      nxt[v] = t;
      ++c;
    }
  }
  if (c) atomicAdd(moved, c);
}

// Parts whose arrivals exceed the capacity ("overflowing": some but not all
// of their movers fit) accept the prefix of their movers, in list (= vertex)
// order, that fits.  The list is cut into kPrefChunks chunks: per
// (overflowing part, chunk) the movers' weight is summed, scanned over the
// chunks, and each chunk then accepts its movers with a block scan from that
// offset.
constexpr int kPrefChunks = 256;
constexpr int kMaxOver = 16384;   // overflowing parts handled per launch batch

__global__ void k_over_flags(int K, const unsigned long long *__restrict__ W,
                             const unsigned long long *__restrict__ arr, unsigned long long cap,
                             uint8_t *of) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < K; p += gridDim.x * blockDim.x)
    of[p] = (W[p] + arr[p] > cap && W[p] < cap) ? 1 : 0;
}

__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long x,
                                                            unsigned long long *ws) {
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = x;
  __syncthreads();
  return ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ __launch_bounds__(256) void k_over_sums(const int32_t *__restrict__ list,
                                                   const int32_t *__restrict__ count,
                                                   const int32_t *__restrict__ tgt,
                                                   const int32_t *__restrict__ vwgt,
                                                   const int32_t *__restrict__ olist,
                                                   const int32_t *__restrict__ ocount, int o0,
                                                   unsigned long long *sums) {
  __shared__ unsigned long long ws[4];
  const int M = *count, O = min(*ocount, o0 + kMaxOver);
  const int per = (M + kPrefChunks - 1) / kPrefChunks;
  const int i0 = blockIdx.x * per, i1 = min(M, i0 + per);
  for (int o = o0 + blockIdx.y; o < O; o += gridDim.y) {
    const int p = olist[o];
    unsigned long long acc = 0;
    for (int i = i0 + threadIdx.x; i < i1; i += 256) {
      const int v = list[i];
      if (tgt[v] == p) acc += (unsigned long long)(vwgt ? vwgt[v] : 1);
    }
    acc = block_sum_u64(acc, ws);
    if (threadIdx.x == 0) sums[(int64_t)(o - o0) * kPrefChunks + blockIdx.x] = acc;
  }
}

// exclusive scan of each overflowing part's chunk sums
__global__ __launch_bounds__(kPrefChunks) void k_over_scan(const int32_t *__restrict__ ocount,
                                                           int o0, unsigned long long *sums) {
  __shared__ unsigned long long sh[kPrefChunks];
  const int O = min(*ocount, o0 + kMaxOver);
  const int t = threadIdx.x;
  for (int o = o0 + blockIdx.x; o < O; o += gridDim.x) {
    unsigned long long *row = sums + (int64_t)(o - o0) * kPrefChunks;
    sh[t] = row[t];
    __syncthreads();
    for (int off = 1; off < kPrefChunks; off <<= 1) {
      const unsigned long long x = t >= off ? sh[t - off] : 0ull;
      __syncthreads();
      sh[t] += x;
      __syncthreads();
    }
    row[t] = t ? sh[t - 1] : 0ull;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_over_accept(const int32_t *__restrict__ list,
                                                     const int32_t *__restrict__ count,
                                                     const int32_t *__restrict__ tgt,
                                                     const int32_t *__restrict__ vwgt,
                                                     const int32_t *__restrict__ olist,
                                                     const int32_t *__restrict__ ocount, int o0,
                                                     const unsigned long long *__restrict__ W,
                                                     const unsigned long long *__restrict__ sums,
                                                     unsigned long long cap, int32_t *nxt,
                                                     unsigned long long *moved) {
  __shared__ unsigned long long ws[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int M = *count, O = min(*ocount, o0 + kMaxOver);
  const int per = (M + kPrefChunks - 1) / kPrefChunks;
  const int i0 = blockIdx.x * per, i1 = min(M, i0 + per);
  unsigned long long acc = 0;
  for (int o = o0 + blockIdx.y; o < O; o += gridDim.y) {
    const int p = olist[o];
    const unsigned long long base = W[p] + sums[(int64_t)(o - o0) * kPrefChunks + blockIdx.x];
    if (base >= cap) continue;   // block-uniform: no mover of this chunk fits
    unsigned long long run = 0;
    for (int b = i0; b < i1; b += 256) {
      const int i = b + tid;
      int v = -1;
      unsigned long long x = 0;
      if (i < i1) {
        v = list[i];
        if (tgt[v] == p) x = (unsigned long long)(vwgt ? vwgt[v] : 1);
      }
      unsigned long long sc = x;   // inclusive scan over the block
      for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long y = __shfl_up(sc, off);
        if (lane >= off) sc += y;
      }
      if (lane == 63) ws[wv] = sc;
      __syncthreads();
      unsigned long long pre = 0;
      for (int q = 0; q < wv; ++q) pre += ws[q];
      const unsigned long long tot = ws[0] + ws[1] + ws[2] + ws[3];
      if (x && base + run + pre + sc <= cap) {
        nxt[v] = p;
        ++acc;
      }
      run += tot;
      __syncthreads();
      if (base + run > cap) break;   // block-uniform: every later mover is rejected
    }
  }
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0 && acc) atomicAdd(moved, acc);
}

__global__ void k_copy_i32(const int32_t *__restrict__ a, int32_t *b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

}  // namespace

size_t refine_scratch_bytes(int64_t n, int K) {
  size_t b = 0;
  b += align_up(sizeof(int32_t) * n, 256) * 4;                       // nxt, tgt, list, rows
  b += align_up(sizeof(S) * n, 256);                                 // gain
  b += align_up(n, 256) * 2;                                         // flags (big, mover)
  b += align_up(sizeof(int32_t) * (kScanBlocks + 1), 256) * 2;       // block counts
  b += align_up(sizeof(unsigned long long) * (size_t)K, 256) * 2;    // W, arrivals
  b += align_up(sizeof(unsigned long long) * 4, 256);                // counters
  b += align_up((size_t)K, 256) + align_up(sizeof(int32_t) * (size_t)K, 256);   // overflow
  b += align_up(sizeof(int32_t) * (kScanBlocks + 1), 256);
  b += align_up(sizeof(unsigned long long) * (size_t)std::min(K, kMaxOver) * kPrefChunks, 256);
  b += quality_scratch_bytes(K) + 256;
  return b;
}

int refine(sphx_graph *g, int32_t *part, int K, double eps, int max_passes, double *cut,
           double *imbalance, int *passes, int64_t *moves, void *scratch, void *pinned,
           hipStream_t s, std::string *err) {
  const int64_t n = g->n;
  Arena a;
  a.base = static_cast<char *>(scratch);
  int32_t *nxt = a.take<int32_t>(n);
  int32_t *tgt = a.take<int32_t>(n);
  int32_t *list = a.take<int32_t>(n);
  int32_t *rows = a.take<int32_t>(n);
  S *gain = a.take<S>(n);
  uint8_t *big = a.take<uint8_t>(n);
  uint8_t *mv = a.take<uint8_t>(n);
  int32_t *cnt_rows = a.take<int32_t>(kScanBlocks + 1);
  int32_t *cnt_mv = a.take<int32_t>(kScanBlocks + 1);
  unsigned long long *W = a.take<unsigned long long>(K);
  unsigned long long *arr = a.take<unsigned long long>(K);
  unsigned long long *ctr = a.take<unsigned long long>(4);
  uint8_t *oflag = a.take<uint8_t>(K);
  int32_t *olist = a.take<int32_t>(K);
  int32_t *cnt_of = a.take<int32_t>(kScanBlocks + 1);
  unsigned long long *osums =
      a.take<unsigned long long>((size_t)std::min(K, kMaxOver) * kPrefChunks);
  char *qscratch = a.take<char>(quality_scratch_bytes(K));
  int e0 = 0;
  if (g->wdt == SPHX_F32) e0 = fixed_exponent<float>(g->wmin);
  if (g->wdt == SPHX_F64) e0 = fixed_exponent<double>(g->wmin);

  // current partition: its exact cut, part weights (and the range check)
  std::vector<int64_t> pw(K);
  std::vector<unsigned long long> hW(K);
  unsigned __int128 cut_cur = 0;
  double c_d = 0.0, imb = 1.0;
  SPHX_TRY(quality(g, part, K, &c_d, &imb, pw.data(), qscratch, pinned, s, err, &cut_cur));
  unsigned long long Wtot = 0;
  for (int k = 0; k < K; ++k) Wtot += (unsigned long long)pw[k];
  // largest integer part weight strictly below (W / K)(1 + eps)
  const double x = ((double)Wtot / (double)K) * (1.0 + eps);
  const double cap_d = std::ceil(x) - 1.0;
  const unsigned long long cap =
      cap_d < 0.0 ? 0ull : (cap_d >= 1.8e19 ? ~0ull : (unsigned long long)cap_d);

  int32_t *cur = part, *alt = nxt;
  int kept = 0;
  int64_t nmoves = 0;
  const unsigned gv = grid_for(n, 256, 8192);
  auto go = [&](auto idx_tag, auto w_tag) -> int {
    using IdxT = decltype(idx_tag);
    using WT = decltype(w_tag);
    const IdxT *rp = static_cast<const IdxT *>(g->rowptr);
    const WT *w = static_cast<const WT *>(g->w);
    for (int pass = 0; pass < max_passes; ++pass) {
      // 1. gains
      hipLaunchKernelGGL((k_gain_thread<IdxT, WT>), dim3(gv), dim3(256), 0, s, n, rp, g->col, w,
                         e0, (const int32_t *)cur, tgt, gain, big);
      hipLaunchKernelGGL(k_flag_count, dim3(kScanBlocks), dim3(256), 0, s, n,
                         (const uint8_t *)big, cnt_rows);
      hipLaunchKernelGGL(k_flag_scan, dim3(1), dim3(kScanBlocks), 0, s, cnt_rows);
      hipLaunchKernelGGL(k_flag_scatter, dim3(kScanBlocks), dim3(256), 0, s, n,
                         (const uint8_t *)big, (const int32_t *)cnt_rows, rows);
      const int32_t *nbig = cnt_rows + kScanBlocks;
      hipLaunchKernelGGL((k_gain_block<IdxT, WT>), dim3(2048), dim3(256), 0, s,
                         (const int32_t *)rows, nbig, rp, g->col, w, e0, (const int32_t *)cur, K,
                         tgt, gain);
      // 2. conflicts
      hipLaunchKernelGGL((k_movers<IdxT, WT>), dim3(gv), dim3(256), 0, s, n, rp, g->col, w, e0,
                         (const int32_t *)cur, (const int32_t *)tgt, (const S *)gain, mv);
      hipLaunchKernelGGL((k_movers_wave<IdxT, WT>), dim3(2048), dim3(256), 0, s,
                         (const int32_t *)rows, nbig, rp, g->col, w, e0, (const int32_t *)cur,
                         (const int32_t *)tgt, (const S *)gain, mv);
      hipLaunchKernelGGL(k_flag_count, dim3(kScanBlocks), dim3(256), 0, s, n,
                         (const uint8_t *)mv, cnt_mv);
      hipLaunchKernelGGL(k_flag_scan, dim3(1), dim3(kScanBlocks), 0, s, cnt_mv);
      hipLaunchKernelGGL(k_flag_scatter, dim3(kScanBlocks), dim3(256), 0, s, n,
                         (const uint8_t *)mv, (const int32_t *)cnt_mv, list);
      // 3. balance, 4. moves (into a copy of the current partition)
      const int32_t *M = cnt_mv + kScanBlocks;
      // part weights of the current partition (from its quality pass)
      for (int k = 0; k < K; ++k) hW[k] = (unsigned long long)pw[k];
      SPHX_HIP(g->h, hipMemcpyAsync(W, hW.data(), sizeof(unsigned long long) * K,
                                    hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(K, 256, 1024)), dim3(256), 0, s, arr,
                         (int64_t)K);
      hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, ctr, (int64_t)4);
      hipLaunchKernelGGL(k_arrivals, dim3(grid_for(n, 256 * 16, 1024)), dim3(256), 0, s,
                         (const int32_t *)list, M, (const int32_t *)tgt, g->vwgt, K, arr);
      hipLaunchKernelGGL(k_copy_i32, dim3(gv), dim3(256), 0, s, (const int32_t *)cur, alt, n);
      hipLaunchKernelGGL(k_accept_all, dim3(gv), dim3(256), 0, s, (const int32_t *)list, M,
                         (const int32_t *)tgt, (const unsigned long long *)W,
                         (const unsigned long long *)arr, cap, alt, ctr);
      // overflowing parts: prefix acceptance in vertex order
      hipLaunchKernelGGL(k_over_flags, dim3(grid_for(K, 256, 1024)), dim3(256), 0, s, K,
                         (const unsigned long long *)W, (const unsigned long long *)arr, cap,
                         oflag);
      hipLaunchKernelGGL(k_flag_count, dim3(kScanBlocks), dim3(256), 0, s, (int64_t)K,
                         (const uint8_t *)oflag, cnt_of);
      hipLaunchKernelGGL(k_flag_scan, dim3(1), dim3(kScanBlocks), 0, s, cnt_of);
      hipLaunchKernelGGL(k_flag_scatter, dim3(kScanBlocks), dim3(256), 0, s, (int64_t)K,
                         (const uint8_t *)oflag, (const int32_t *)cnt_of, olist);
      const int32_t *O = cnt_of + kScanBlocks;
      for (int o0 = 0; o0 < K; o0 += kMaxOver) {
        const unsigned gy = (unsigned)std::min(std::min(K - o0, kMaxOver), 64);
        hipLaunchKernelGGL(k_over_sums, dim3(kPrefChunks, gy), dim3(256), 0, s,
                           (const int32_t *)list, M, (const int32_t *)tgt, g->vwgt,
                           (const int32_t *)olist, O, o0, osums);
        hipLaunchKernelGGL(k_over_scan, dim3(std::min(std::min(K - o0, kMaxOver), 1024)),
                           dim3(kPrefChunks), 0, s, O, o0, osums);
        hipLaunchKernelGGL(k_over_accept, dim3(kPrefChunks, gy), dim3(256), 0, s,
                           (const int32_t *)list, M, (const int32_t *)tgt, g->vwgt,
                           (const int32_t *)olist, O, o0, (const unsigned long long *)W,
                           (const unsigned long long *)osums, cap, alt, ctr);
      }
      if (hipGetLastError() != hipSuccess) {
        *err = "refinement kernel launch failed";
        return SPHX_E_HIP;
      }
      unsigned long long moved = 0;
      if (hipMemcpyAsync(&moved, ctr, sizeof(moved), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        *err = "refinement: copy failed";
        return SPHX_E_HIP;
      }
      if (moved == 0) break;
      unsigned __int128 cut_new = 0;
      double cn = 0.0, in = 1.0;
      SPHX_TRY(quality(g, alt, K, &cn, &in, pw.data(), qscratch, pinned, s, err, &cut_new));
      if (!(cut_new < cut_cur)) break;
      std::swap(cur, alt);
      cut_cur = cut_new;
      c_d = cn;
      imb = in;
      ++kept;
      nmoves += (int64_t)moved;
    }
    return SPHX_OK;
  };
  int r;
  if (g->rp64) {
    if (g->wdt == SPHX_UNIT) r = go(int64_t{}, Unit{});
    else if (g->wdt == SPHX_F32) r = go(int64_t{}, float{});
    else r = go(int64_t{}, double{});
  } else {
    if (g->wdt == SPHX_UNIT) r = go(int32_t{}, Unit{});
    else if (g->wdt == SPHX_F32) r = go(int32_t{}, float{});
    else r = go(int32_t{}, double{});
  }
  if (r != SPHX_OK) return r;
  if (cur != part) {
    hipLaunchKernelGGL(k_copy_i32, dim3(gv), dim3(256), 0, s, (const int32_t *)cur, part, n);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
      *err = "refinement: copy failed";
      return SPHX_E_HIP;
    }
  }
  if (cut) *cut = c_d;
  if (imbalance) *imbalance = imb;
  if (passes) *passes = kept;
  if (moves) *moves = nmoves;
  return SPHX_OK;
}

}  // namespace sphx
