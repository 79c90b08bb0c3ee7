// Laplacian block product Y = L_C X over padded row-major blocks (Eq. 2 with
// weights, difference form y_i = sum_j w_ij (x_i - x_j)).
//
// The LOBPCG blocks are n x ld with ld * sizeof(T) a multiple of 16 bytes,
// so a row is NV = ld * sizeof(T) / 16 aligned 16-byte vectors.  Short rows
// are handled one thread per row: the thread keeps x_i and the NV-vector
// accumulator in registers and gathers each neighbour row with NV vector
// loads (adjacent threads take adjacent rows, so on mesh-like graphs the
// gathers of a wavefront are contiguous).  Blocks of rows are mapped so that
// each of the 8 XCDs (hardware places consecutive workgroups round robin on
// them) works on one contiguous eighth of the rows, which keeps the gathered
// neighbours of a mesh in that XCD's L2.  Mid-degree rows use a wavefront
// per row (lanes over the neighbours, butterfly reduction in a fixed order),
// hub rows fixed-size chunks combined in a second pass.  All sums are in a
// fixed order, so results are bitwise reproducible.
//
// Epilogues (whole rows): Store, Residual (r = acc - b_i theta_c x_i, output r
// or the Jacobi step r / d_i, FP64 norm partials of ||r||^2_{B^-1} and
// ||x||^2_B per column c < m), and one Chebyshev step of the iteration for
// L h = r (Sec. 5.2).
#include <hip/hip_ext.h>

#include <algorithm>

#include "kernels.h"

namespace sphx {
namespace {

// Row vectors of VB bytes: 16 (float4 / double2), or 8 (float2) for FP32
// rows of an even, non-multiple-of-4 width.
template <typename T, int VB> struct Vec;
template <> struct Vec<float, 16> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int E = 4;
};
template <> struct Vec<float, 8> {
  typedef float type __attribute__((ext_vector_type(2)));
  static constexpr int E = 2;
};
template <> struct Vec<double, 16> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int E = 2;
};

// Unit weights with the column indices stored as int16 offsets from the row
// (graphs whose every neighbour lies within 32767 rows: two bytes per entry
// instead of four in the index stream).
struct UnitD16 {};
template <typename WT>
constexpr bool kUnitW = std::is_same_v<WT, Unit> || std::is_same_v<WT, UnitD16>;
template <typename WT> struct ColOf { using type = int32_t; };
template <> struct ColOf<UnitD16> { using type = int16_t; };

template <typename IdxT, typename WT>
struct Csr {
  const IdxT *rp;
  const typename ColOf<WT>::type *col;
  const WT *w;
  // neighbour of row i stored at entry k, and the entry's weight
  __device__ __forceinline__ int64_t nbr(int64_t i, int64_t k) const {
    if constexpr (std::is_same_v<WT, UnitD16>) return i + (int64_t)col[k];
    else return (int64_t)col[k];
  }
  __device__ __forceinline__ WT wk(int64_t k) const { return w[k]; }
};

// The same entries read from an LDS copy of a contiguous run of them
// (entries k0 ..; staged by the row-chunk kernel below).
template <typename WT>
struct LdsCsr {
  using CT = typename ColOf<WT>::type;
  using WS = std::conditional_t<kUnitW<WT>, float, WT>;
  const CT *col;
  const WS *w;
  int64_t k0;
  __device__ __forceinline__ int64_t nbr(int64_t i, int64_t k) const {
    if constexpr (std::is_same_v<WT, UnitD16>) return i + (int64_t)col[k - k0];
    else return (int64_t)col[k - k0];
  }
  __device__ __forceinline__ WS wk(int64_t k) const { return w[k - k0]; }
};

// Block id remap: XCD x = b % 8 receives a contiguous range of block ids.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
  const int64_t q = nb / 8, r = nb % 8;
  const int64_t x = b % 8, pos = b / 8;
  return x * q + (x < r ? x : r) + pos;
}

// acc = sum over entries k0, k0 + step, ... < k1 of w_k (x_i - x_col[k]).
// U independent partial sums (U gathers in flight per lane), combined in a
// fixed order.
template <typename T, int VB, int NV, typename WT, typename Src>
__device__ __forceinline__ void vrow_acc(const Src &A, int64_t i, int64_t k0, int64_t k1,
                                         int step, const typename Vec<T, VB>::type *__restrict__ X,
                                         int ldv, const typename Vec<T, VB>::type (&xi)[NV],
                                         typename Vec<T, VB>::type (&acc)[NV]) {
  using V = typename Vec<T, VB>::type;
  constexpr int U = NV <= 2 ? 4 : 2;
  V a[U][NV];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int v = 0; v < NV; ++v) a[u][v] = V(0);
  int64_t k = k0;
  for (; k + (U - 1) * step < k1; k += U * step) {
    int64_t j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) j[u] = A.nbr(i, k + u * step);
    V x[U][NV];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int v = 0; v < NV; ++v) x[u][v] = X[j[u] * ldv + v];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (kUnitW<WT>) {
#pragma unroll
        for (int v = 0; v < NV; ++v) a[u][v] += xi[v] - x[u][v];
      } else {
        const T wk = T(A.wk(k + u * step));
#pragma unroll
        for (int v = 0; v < NV; ++v) a[u][v] += wk * (xi[v] - x[u][v]);
      }
    }
  }
  // tail: fewer than U entries left, into the partial sums in order
#pragma unroll
  for (int u = 0; u < U - 1; ++u) {
    if (k < k1) {
      const int64_t j0 = A.nbr(i, k);
      if constexpr (kUnitW<WT>) {
#pragma unroll
        for (int v = 0; v < NV; ++v) a[u][v] += xi[v] - X[j0 * ldv + v];
      } else {
        const T w0 = T(A.wk(k));
#pragma unroll
        for (int v = 0; v < NV; ++v) a[u][v] += w0 * (xi[v] - X[j0 * ldv + v]);
      }
      k += step;
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if constexpr (U == 4) acc[v] = (a[0][v] + a[1][v]) + (a[2][v] + a[3][v]);
    else acc[v] = a[0][v] + a[1][v];
  }
}

// ------------------------------------------------------------- epilogues
template <typename T, int VB, int NV>
struct VStore {
  EpiStoreP<T> p;
  static constexpr bool kNorms = false;
  using V = typename Vec<T, VB>::type;
  __device__ void row(int64_t i, const V (&xi)[NV], const V (&acc)[NV], double *, double *) const {
    V *y = reinterpret_cast<V *>(p.Y + i * p.ldy);
#pragma unroll
    for (int v = 0; v < NV; ++v) y[v] = acc[v];
  }
};

template <typename T, int VB, int NV>
struct VResidual {
  EpiResidualP<T> p;
  int m;
  bool store_lx = true;   // false: L X is already in p.LX (streaming pass)
  static constexpr bool kNorms = true;
  using V = typename Vec<T, VB>::type;
  static constexpr int E = Vec<T, VB>::E;
  __device__ void row(int64_t i, const V (&xi)[NV], const V (&acc)[NV], double *n1,
                      double *n2) const {
    const double di = p.d64 ? p.d64[i] : 1.0;
    const double b = p.generalized ? di : 1.0;
    // one division per row for the B^-1-norm terms (exactly 1 when B = I)
    const double ib = p.generalized ? 1.0 / di : 1.0;
    V *lx = reinterpret_cast<V *>(p.LX + i * p.ld);
    V *out = reinterpret_cast<V *>(p.OUT + i * p.ld);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      V o;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int c = v * E + e;
        const double x = double(xi[v][e]);
        const double th = c < m ? p.theta[c] : 0.0;
        const double r = double(acc[v][e]) - b * th * x;
        o[e] = T(p.jacobi ? r / di : r);
        if (c < m) {
          n1[c] += r * r * ib;
          n2[c] += b * x * x;
        }
      }
      if (store_lx) lx[v] = acc[v];
      out[v] = o;
    }
  }
};

template <typename T, int VB, int NV>
struct VShiftDot {
  EpiShiftDotP<T> p;
  int m;
  static constexpr bool kNorms = true;
  using V = typename Vec<T, VB>::type;
  static constexpr int E = Vec<T, VB>::E;
  __device__ void row(int64_t i, const V (&xi)[NV], const V (&acc)[NV], double *n1,
                      double *) const {
    const double b = p.bd ? p.bd[i] : 1.0;
    V *out = reinterpret_cast<V *>(p.OUT + i * p.ld);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      V o;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int c = v * E + e;
        const double x = double(xi[v][e]);
        const double lc = c < m ? p.lam[c] : 0.0;
        const double y = double(acc[v][e]) - b * lc * x;
        o[e] = T(y);
        if (c < m) n1[c] += x * y;
      }
      out[v] = o;
    }
  }
};

template <typename T, int VB, int NV>
struct VCheb {
  EpiChebP<T> p;
  static constexpr bool kNorms = false;
  using V = typename Vec<T, VB>::type;
  static constexpr int E = Vec<T, VB>::E;
  __device__ void row(int64_t i, const V (&xi)[NV], const V (&acc)[NV], double *, double *) const {
    const double si = p.dinv ? p.dinv[i] : 1.0;
    const V *rr = reinterpret_cast<const V *>(p.R + i * p.ld);
    const V *pp = p.prev ? reinterpret_cast<const V *>(p.prev + i * p.ld) : nullptr;
    V *out = reinterpret_cast<V *>(p.OUT + i * p.ld);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const V r = rr[v];
      const V pv = pp ? pp[v] : V(0);
      V o;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const double xs = p.src_scale * double(xi[v][e]);
        const double pr = p.prev_scale * double(pv[e]);
        const double res = double(r[e]) - p.src_scale * double(acc[v][e]);
        o[e] = T(xs + p.alpha * (xs - pr) + p.beta * si * res);
      }
      out[v] = o;
    }
  }
};

template <typename T, int VB, int NV>
struct VPoly {
  EpiPolyP<T> p;
  static constexpr bool kNorms = false;
  using V = typename Vec<T, VB>::type;
  static constexpr int E = Vec<T, VB>::E;
  __device__ void row(int64_t i, const V (&xi)[NV], const V (&acc)[NV], double *, double *) const {
    const double si = p.dinv ? p.dinv[i] : 1.0;
    const V *yi = p.Yin ? reinterpret_cast<const V *>(p.Yin + i * p.ld) : nullptr;
    V *yo = reinterpret_cast<V *>(p.Yout + i * p.ld);
    V *po = p.last ? nullptr : reinterpret_cast<V *>(p.Pout + i * p.ld);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const V y0 = yi ? yi[v] : V(0);
      V y, pn;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const double pv = double(xi[v][e]);
        const double pnew = pv - si * double(acc[v][e]) * p.inv_t;
        double yv = double(y0[e]) + pv * p.inv_t;
        if (p.last) yv += pnew * p.inv_t_next;
        y[e] = T(yv);
        pn[e] = T(pnew);
      }
      yo[v] = y;
      if (po) po[v] = pn;
    }
  }
};

// Per-column block sums of the thread norms (columns < m), fixed order:
// butterfly within each wavefront, then the 4 wavefronts in order.
template <int LD>
__device__ void block_norms(const double (&n1)[LD], const double (&n2)[LD], int m,
                            double *partials, int slot) {
  __shared__ double sh[4][2 * kMaxNev];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < LD; ++c) {
    if (c >= m) break;
    double a = n1[c], b = n2[c];
    for (int off = 32; off >= 1; off >>= 1) {
      a += __shfl_xor(a, off);
      b += __shfl_xor(b, off);
    }
    if (lane == 0) {
      sh[wave][c] = a;
      sh[wave][kMaxNev + c] = b;
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < m) {
    double a = sh[0][t] + sh[1][t] + sh[2][t] + sh[3][t];
    double b = sh[0][kMaxNev + t] + sh[1][kMaxNev + t] + sh[2][kMaxNev + t] +
               sh[3][kMaxNev + t];
    partials[(int64_t)t * kMaxNormBlocks + slot] = a;
    partials[(int64_t)(kMaxNev + t) * kMaxNormBlocks + slot] = b;
  }
}

// ----------------------------------------------------------------- kernels
// Short rows, one thread per row; `rpt` rows per thread, 256-row strides.
template <typename T, int VB, int NV, typename IdxT, typename WT, typename Epi>
__global__ __launch_bounds__(256) void k_vrow(Csr<IdxT, WT> A, const int32_t *__restrict__ rows,
                                              int64_t nrows, const T *__restrict__ Xs, int ld,
                                              int rpt, Epi epi, double *partials, int slot0,
                                              int m) {
  using V = typename Vec<T, VB>::type;
  constexpr int LD = NV * Vec<T, VB>::E;
  const V *X = reinterpret_cast<const V *>(Xs);
  const int ldv = ld / Vec<T, VB>::E;
  const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
  double n1[LD], n2[LD];
#pragma unroll
  for (int c = 0; c < LD; ++c) { n1[c] = 0.0; n2[c] = 0.0; }
  for (int q = 0; q < rpt; ++q) {
    const int64_t r = (b * rpt + q) * 256 + threadIdx.x;
    if (r >= nrows) break;
    const int64_t i = rows ? rows[r] : r;
    V xi[NV], acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) xi[v] = X[i * ldv + v];
    vrow_acc<T, VB, NV, WT>(A, i, (int64_t)A.rp[i], (int64_t)A.rp[i + 1], 1, X, ldv, xi, acc);
    epi.row(i, xi, acc, n1, n2);
  }
  if constexpr (Epi::kNorms) block_norms<LD>(n1, n2, m, partials, slot0 + (int)blockIdx.x);
}

template <typename T, int VB, int NV>
__device__ __forceinline__ void wave_sum(typename Vec<T, VB>::type (&acc)[NV]) {
  constexpr int E = Vec<T, VB>::E;
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      T a = acc[v][e];
      for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off);
      acc[v][e] = a;
    }
}

template <typename T, int VB, int NV, int G>
__device__ __forceinline__ void group_sum(typename Vec<T, VB>::type (&acc)[NV]) {
  constexpr int E = Vec<T, VB>::E;
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      T a = acc[v][e];
#pragma unroll
      for (int off = G / 2; off >= 1; off >>= 1) a += __shfl_xor(a, off);
      acc[v][e] = a;
    }
}

// G lanes per row (G = 2, 4, 16 or 64): the lanes of a group take every G-th
// neighbour of the row, so a group reads a contiguous run of the column
// indices; the group's partial sums are combined by a butterfly in a fixed
// order and the group's first lane runs the epilogue.  rows = null: natural
// order over all n rows.
// rpb > 0: each block takes a contiguous range of rpb rows (a multiple of the
// groups per block), and block ids are remapped so that each XCD works on one
// contiguous stretch of ranges (as the one-lane kernel does): the gathered
// neighbour rows of a mesh then stay in that XCD's L2.  rpb == 0: blocks
// stride over the rows (the degree-binned lists of power-law graphs, whose
// neighbours are random anyway and whose row costs vary within a bin).
template <typename T, int VB, int NV, int G, typename IdxT, typename WT, typename Epi>
__global__ __launch_bounds__(256) void k_vgroup(Csr<IdxT, WT> A,
                                                const int32_t *__restrict__ rows,
                                                int64_t nrows, const T *__restrict__ Xs,
                                                int ld, int64_t rpb, Epi epi, double *partials,
                                                int slot0, int m) {
  using V = typename Vec<T, VB>::type;
  constexpr int LD = NV * Vec<T, VB>::E;
  constexpr int GPB = 256 / G;   // groups per block
  const V *X = reinterpret_cast<const V *>(Xs);
  const int ldv = ld / Vec<T, VB>::E;
  const int gl = threadIdx.x & (G - 1);
  const bool strided = rpb == 0;
  const int64_t b = strided ? (int64_t)blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
  const int64_t rend = strided ? nrows : min(nrows, (b + 1) * rpb);
  const int64_t step = strided ? (int64_t)gridDim.x * GPB : GPB;
  double n1[LD], n2[LD];
#pragma unroll
  for (int c = 0; c < LD; ++c) { n1[c] = 0.0; n2[c] = 0.0; }
  for (int64_t r = (strided ? b * GPB : b * rpb) + threadIdx.x / G; r < rend; r += step) {
    const int64_t i = rows ? rows[r] : r;
    V xi[NV], acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) xi[v] = X[i * ldv + v];
    vrow_acc<T, VB, NV, WT>(A, i, (int64_t)A.rp[i] + gl, (int64_t)A.rp[i + 1], G, X, ldv, xi, acc);
    group_sum<T, VB, NV, G>(acc);
    if (gl == 0) epi.row(i, xi, acc, n1, n2);
  }
  if constexpr (Epi::kNorms) block_norms<LD>(n1, n2, m, partials, slot0 + (int)blockIdx.x);
}

// Rows of 13..48 neighbours in natural order (mesh-like graphs), G lanes per
// row, with the column indices (and weights) staged in LDS: the block takes
// its rows in chunks of 256 / G consecutive rows, whose CSR entries form one
// contiguous run; the block loads that run with coalesced loads (adjacent
// threads, adjacent entries) into LDS, and the groups then walk their rows
// from LDS.  Read per lane from global memory instead, the index and weight
// lines of all resident waves exceed the L2 and are fetched again (measured:
// about twice the algorithmic bytes on the weighted 27-point mesh).  A chunk
// with more than kLdsEntries entries is read from global memory.  Blocks take
// contiguous chunk ranges, remapped per XCD as above.  The summation order is
// the same as k_vgroup's.
constexpr int kLdsEntries = 4096;

template <typename T, int VB, int NV, int G, typename IdxT, typename WT, typename Epi>
__global__ __launch_bounds__(256) void k_vlds(Csr<IdxT, WT> A, int64_t nrows,
                                              const T *__restrict__ Xs, int ld, int64_t rpb,
                                              Epi epi, double *partials, int slot0, int m) {
  using V = typename Vec<T, VB>::type;
  using L = LdsCsr<WT>;
  constexpr int LD = NV * Vec<T, VB>::E;
  constexpr int R = 256 / G;   // rows per chunk
  __shared__ typename L::CT scol[kLdsEntries];
  __shared__ typename L::WS sw[kUnitW<WT> ? 1 : kLdsEntries];
  const V *X = reinterpret_cast<const V *>(Xs);
  const int ldv = ld / Vec<T, VB>::E;
  const int gl = threadIdx.x & (G - 1);
  const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t rend = min(nrows, (b + 1) * rpb);
  double n1[LD], n2[LD];
#pragma unroll
  for (int c = 0; c < LD; ++c) { n1[c] = 0.0; n2[c] = 0.0; }
  for (int64_t r0 = b * rpb; r0 < rend; r0 += R) {
    const int64_t r1 = min(rend, r0 + (int64_t)R);
    const int64_t k0 = A.rp[r0], k1 = A.rp[r1];
    const bool staged = k1 - k0 <= kLdsEntries;
    if (staged) {
      for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) {
        scol[k - k0] = A.col[k];
        if constexpr (!kUnitW<WT>) sw[k - k0] = A.w[k];
      }
    }
    __syncthreads();
    const int64_t i = r0 + threadIdx.x / G;
    if (i < r1) {                       // uniform over each group of G lanes
      V xi[NV], acc[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) xi[v] = X[i * ldv + v];
      const int64_t ka = (int64_t)A.rp[i] + gl, kb = (int64_t)A.rp[i + 1];
      if (staged) {
        const L S{scol, sw, k0};
        vrow_acc<T, VB, NV, WT>(S, i, ka, kb, G, X, ldv, xi, acc);
      } else {
        vrow_acc<T, VB, NV, WT>(A, i, ka, kb, G, X, ldv, xi, acc);
      }
      group_sum<T, VB, NV, G>(acc);
      if (gl == 0) epi.row(i, xi, acc, n1, n2);
    }
    __syncthreads();
  }
  if constexpr (Epi::kNorms) block_norms<LD>(n1, n2, m, partials, slot0 + (int)blockIdx.x);
}

// Hub rows, pass 1: one wavefront per chunk -> partial row sums (as double).
template <typename T, int VB, int NV, typename IdxT, typename WT>
__global__ __launch_bounds__(256) void k_vhub_partial(
    Csr<IdxT, WT> A, const int32_t *__restrict__ hub_rows,
    const int32_t *__restrict__ hub_chunk_begin, int64_t n_hub,
    const int64_t *__restrict__ k0s, const int64_t *__restrict__ k1s, int64_t n_chunks,
    const T *__restrict__ Xs, int ld, double *out) {
  using V = typename Vec<T, VB>::type;
  constexpr int E = Vec<T, VB>::E;
  const V *X = reinterpret_cast<const V *>(Xs);
  const int ldv = ld / E;
  const int lane = threadIdx.x & 63;
  for (int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); q < n_chunks;
       q += (int64_t)gridDim.x * 4) {
    int64_t lo = 0, hi = n_hub - 1;
    while (lo < hi) {
      int64_t mid = (lo + hi + 1) / 2;
      if (hub_chunk_begin[mid] <= q) lo = mid; else hi = mid - 1;
    }
    const int64_t i = hub_rows[lo];
    V xi[NV], acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) xi[v] = X[i * ldv + v];
    vrow_acc<T, VB, NV, WT>(A, i, k0s[q] + lane, k1s[q], 64, X, ldv, xi, acc);
    wave_sum<T, VB, NV>(acc);
    if (lane == 0)
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < E; ++e) out[q * kMaxNev + v * E + e] = double(acc[v][e]);
  }
}

// Hub rows, pass 2: one thread per hub row sums its chunks in order.
template <typename T, int VB, int NV, typename Epi>
__global__ __launch_bounds__(256) void k_vhub_combine(const int32_t *__restrict__ hub_rows,
                                                      const int32_t *__restrict__ hub_chunk_begin,
                                                      int64_t n_hub, const double *part,
                                                      const T *__restrict__ Xs, int ld, Epi epi,
                                                      double *partials, int slot0, int m) {
  using V = typename Vec<T, VB>::type;
  constexpr int E = Vec<T, VB>::E;
  constexpr int LD = NV * E;
  const V *X = reinterpret_cast<const V *>(Xs);
  const int ldv = ld / E;
  double n1[LD], n2[LD];
#pragma unroll
  for (int c = 0; c < LD; ++c) { n1[c] = 0.0; n2[c] = 0.0; }
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < n_hub;
       h += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = hub_rows[h];
    V xi[NV], acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      xi[v] = X[i * ldv + v];
      acc[v] = V(0);
    }
    for (int64_t q = hub_chunk_begin[h]; q < hub_chunk_begin[h + 1]; ++q)
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < E; ++e) acc[v][e] += T(part[q * kMaxNev + v * E + e]);
    epi.row(i, xi, acc, n1, n2);
  }
  if constexpr (Epi::kNorms) block_norms<LD>(n1, n2, m, partials, slot0 + (int)blockIdx.x);
}

// The residual epilogue as a streaming pass over an L X that a store product
// has already written: one thread per row, `rpt` rows per thread in 256-row
// strides, the same arithmetic and norm partials as the fused epilogue.
template <typename T, int VB, int NV>
__global__ __launch_bounds__(256) void k_resid_rows(int64_t n, const T *__restrict__ Xs,
                                                    VResidual<T, VB, NV> epi, int rpt,
                                                    double *partials, int m) {
  using V = typename Vec<T, VB>::type;
  constexpr int LD = NV * Vec<T, VB>::E;
  const V *X = reinterpret_cast<const V *>(Xs);
  const V *LXv = reinterpret_cast<const V *>(epi.p.LX);
  const int ldv = epi.p.ld / Vec<T, VB>::E;
  double n1[LD], n2[LD];
#pragma unroll
  for (int c = 0; c < LD; ++c) { n1[c] = 0.0; n2[c] = 0.0; }
  for (int q = 0; q < rpt; ++q) {
    const int64_t i = ((int64_t)blockIdx.x * rpt + q) * 256 + threadIdx.x;
    if (i >= n) break;
    V xi[NV], acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      xi[v] = X[i * ldv + v];
      acc[v] = LXv[i * ldv + v];
    }
    epi.row(i, xi, acc, n1, n2);
  }
  block_norms<LD>(n1, n2, m, partials, (int)blockIdx.x);
}

template <typename T>
int resid_stream(int64_t n, const T *X, int ld, int m, const EpiResidualP<T> &p,
                 double *partials, int *nparts, hipStream_t s) {
  const int64_t nb0 = ceil_div(n, 256);
  const int rpt = (int)ceil_div(nb0, kMaxNormBlocks);
  const unsigned nb = (unsigned)ceil_div(n, 256 * (int64_t)rpt);
  const int row_bytes = ld * (int)sizeof(T);
  if (row_bytes % 16) return SPHX_E_INVALID_ARG;
#define SPHX_RS(NV_)                                                                        \
  case NV_: {                                                                               \
    VResidual<T, 16, NV_> e{p};                                                             \
    e.m = m;                                                                                \
    e.store_lx = false;                                                                     \
    hipLaunchKernelGGL((k_resid_rows<T, 16, NV_>), dim3(nb), dim3(256), 0, s, n, X, e, rpt, \
                       partials, m);                                                        \
    break;                                                                                  \
  }
  switch (row_bytes / 16) {
    SPHX_RS(1) SPHX_RS(2) SPHX_RS(3) SPHX_RS(4)
    default:
      if constexpr (std::is_same_v<T, double>) {
        switch (row_bytes / 16) {
          SPHX_RS(5) SPHX_RS(6) SPHX_RS(7) SPHX_RS(8)
          default: return SPHX_E_INVALID_ARG;
        }
      } else {
        return SPHX_E_INVALID_ARG;
      }
  }
#undef SPHX_RS
  if (nparts) *nparts = (int)nb;
  return hipGetLastError() == hipSuccess ? SPHX_OK : SPHX_E_HIP;
}

// ----------------------------------------------------------------- dispatch
constexpr int kMaxShortBlocks = 8192;
constexpr int kGroupBlocks = 8192;
constexpr int kBinnedShortBlocks = 4096;
constexpr int kBinnedGroupBlocks = 1536;
constexpr int kWaveBlocks = 1024;
constexpr int kHubBlocks = 16;
static_assert(kMaxShortBlocks <= kMaxNormBlocks && kGroupBlocks <= kMaxNormBlocks &&
                  kBinnedShortBlocks + (kNumBins - 1) * kBinnedGroupBlocks + kHubBlocks <=
                      kMaxNormBlocks,
              "norm partial slots");

template <typename T, int VB, int NV, typename IdxT, typename WT, typename Epi>
void run_vec(const Csr<IdxT, WT> &A, int64_t n, const SpmmPlan &plan, const T *X, int ld,
             const Epi &epi, double *partials, int *nparts, int m, hipStream_t s,
             const LaunchEvents *ev) {
  // Every launch writes one norm-partial slot per block: the grids below
  // stay within kMaxNormBlocks in total (grid-stride loops cover the rest).
  int used = 0;
  // an unbinned plan is one launch, which ev (if given) times exactly
  const bool stamp = ev && !plan.binned;
  hipEvent_t e0 = stamp ? ev->start : nullptr, e1 = stamp ? ev->stop : nullptr;
  if (ev && !stamp) (void)hipEventRecord(ev->start, s);
  auto short_rows = [&](const int32_t *rows, int64_t nr, int64_t maxb) {
    int64_t nb = ceil_div(nr, 256);
    int rpt = (int)ceil_div(nb, maxb);
    nb = ceil_div(nr, 256 * (int64_t)rpt);
    hipExtLaunchKernelGGL((k_vrow<T, VB, NV, IdxT, WT, Epi>), dim3((unsigned)nb), dim3(256), 0,
                          s, e0, e1, 0, A, rows, nr, X, ld, rpt, epi, partials, used, m);
    used += (int)nb;
  };
  auto grouped = [&](int G, const int32_t *rows, int64_t nr, int64_t maxb) {
    // natural order: contiguous ranges of whole group-steps per block;
    // row lists (binned): blocks stride over the list.  At most maxb blocks.
    const int64_t gpb = 256 / G;
    int64_t rpb = 0;
    unsigned gb = grid_for(nr, gpb, maxb);
    if (!rows) {
      const int64_t steps = ceil_div(nr, gpb);
      rpb = ceil_div(steps, maxb) * gpb;
      gb = (unsigned)std::max<int64_t>(1, ceil_div(nr, rpb));
    }
    if (G == 2)
      hipExtLaunchKernelGGL((k_vgroup<T, VB, NV, 2, IdxT, WT, Epi>), dim3(gb), dim3(256), 0, s,
                            e0, e1, 0, A, rows, nr, X, ld, rpb, epi, partials, used, m);
    else if (G == 4)
      hipExtLaunchKernelGGL((k_vgroup<T, VB, NV, 4, IdxT, WT, Epi>), dim3(gb), dim3(256), 0, s,
                            e0, e1, 0, A, rows, nr, X, ld, rpb, epi, partials, used, m);
    else if (G == 16)
      hipExtLaunchKernelGGL((k_vgroup<T, VB, NV, 16, IdxT, WT, Epi>), dim3(gb), dim3(256), 0,
                            s, e0, e1, 0, A, rows, nr, X, ld, rpb, epi, partials, used, m);
    else
      hipExtLaunchKernelGGL((k_vgroup<T, VB, NV, 64, IdxT, WT, Epi>), dim3(gb), dim3(256), 0,
                            s, e0, e1, 0, A, rows, nr, X, ld, rpb, epi, partials, used, m);
    used += (int)gb;
  };
  auto staged = [&](int G, int64_t nr, int64_t maxb) {
    const int64_t R = 256 / G;
    const int64_t chunks = ceil_div(nr, R);
    const int64_t cpb = ceil_div(chunks, maxb);
    const int64_t rpb = cpb * R;
    const unsigned gb = (unsigned)std::max<int64_t>(1, ceil_div(nr, rpb));
    if (G == 2)
      hipExtLaunchKernelGGL((k_vlds<T, VB, NV, 2, IdxT, WT, Epi>), dim3(gb), dim3(256), 0, s,
                            e0, e1, 0, A, nr, X, ld, rpb, epi, partials, used, m);
    else
      hipExtLaunchKernelGGL((k_vlds<T, VB, NV, 4, IdxT, WT, Epi>), dim3(gb), dim3(256), 0, s,
                            e0, e1, 0, A, nr, X, ld, rpb, epi, partials, used, m);
    used += (int)gb;
  };
  if (!plan.binned) {
    // rows of 13..48 neighbours: wide gathered rows (>= 32 bytes) take two
    // lanes per row (measured on the 27-point meshes against one and four
    // lanes, FP32 and FP64), narrow rows four
    int G = plan.group;
    if (G > 1 && VB * NV >= 32) G = 2;
    // the LDS-staged index stream pays off for the light epilogues (store,
    // polynomial steps: 8..20 % faster on the weighted 27-point mesh); with
    // the residual epilogue's per-thread norm sums the extra LDS costs more
    // occupancy than it saves (measured 11..30 % slower), so that one reads
    // its indices per lane
    if (G == 1) short_rows(nullptr, n, kMaxShortBlocks);
    else if (Epi::kNorms) grouped(G, nullptr, n, kGroupBlocks);
    else staged(G, n, kGroupBlocks);
  } else {
    for (int c = 0; c < kNumBins; ++c) {
      if (plan.nrows[c] == 0) continue;
      if (bin_group(c) == 1) short_rows(plan.rows[c], plan.nrows[c], kBinnedShortBlocks);
      else grouped(bin_group(c), plan.rows[c], plan.nrows[c], kBinnedGroupBlocks);
    }
    if (plan.n_hub > 0) {
      unsigned gb = grid_for(plan.n_chunks, 4, kWaveBlocks);
      hipLaunchKernelGGL((k_vhub_partial<T, VB, NV, IdxT, WT>), dim3(gb), dim3(256), 0, s, A,
                         plan.hub_rows, plan.hub_chunk_begin, plan.n_hub, plan.chunk_k0,
                         plan.chunk_k1, plan.n_chunks, X, ld, plan.hub_partial);
      unsigned gc = grid_for(plan.n_hub, 256, kHubBlocks);
      hipLaunchKernelGGL((k_vhub_combine<T, VB, NV, Epi>), dim3(gc), dim3(256), 0, s,
                         plan.hub_rows, plan.hub_chunk_begin, plan.n_hub,
                         (const double *)plan.hub_partial, X, ld, epi, partials, used, m);
      used += (int)gc;
    }
  }
  if (ev && !stamp) (void)hipEventRecord(ev->stop, s);
  if (nparts) *nparts = used;
}

template <typename T, int VB, int NV, template <typename, int, int> class EpiT, typename P>
int dispatch_types(sphx_graph *g, const SpmmPlan &plan, const T *X, int ld, const P &p,
                   int m, double *partials, int *nparts, hipStream_t s,
                   const LaunchEvents *ev) {
  auto go = [&](auto idx_tag, auto w_tag) {
    using IdxT = decltype(idx_tag);
    using WT = decltype(w_tag);
    const typename ColOf<WT>::type *col;
    if constexpr (std::is_same_v<WT, UnitD16>) col = plan.dcol;
    else col = g->col;
    Csr<IdxT, WT> A{static_cast<const IdxT *>(g->rowptr), col, static_cast<const WT *>(g->w)};
    EpiT<T, VB, NV> epi{p};
    if constexpr (std::is_same_v<EpiT<T, VB, NV>, VResidual<T, VB, NV>> ||
                  std::is_same_v<EpiT<T, VB, NV>, VShiftDot<T, VB, NV>>)
      epi.m = m;
    run_vec<T, VB, NV>(A, g->n, plan, X, ld, epi, partials, nparts, m, s, ev);
  };
  if (g->rp64) {
    if (g->wdt == SPHX_UNIT) go(int64_t{}, Unit{});
    else if (g->wdt == SPHX_F32) go(int64_t{}, float{});
    else go(int64_t{}, double{});
  } else {
    if (g->wdt == SPHX_UNIT && plan.dcol) go(int32_t{}, UnitD16{});
    else if (g->wdt == SPHX_UNIT) go(int32_t{}, Unit{});
    else if (g->wdt == SPHX_F32) go(int32_t{}, float{});
    else go(int32_t{}, double{});
  }
  return hipGetLastError() == hipSuccess ? SPHX_OK : SPHX_E_HIP;
}

template <typename T, template <typename, int, int> class EpiT, typename P>
int dispatch_nv(sphx_graph *g, const SpmmPlan &plan, const T *X, int ld, const P &p, int m,
                double *partials, int *nparts, hipStream_t s,
                const LaunchEvents *ev = nullptr) {
  if (ld < m || ld > kMaxNev || m < 1) return SPHX_E_INVALID_ARG;
  const int row_bytes = ld * (int)sizeof(T);
#define SPHX_NV(VB_, NV_)                                                                 \
  case NV_:                                                                               \
    return dispatch_types<T, VB_, NV_, EpiT>(g, plan, X, ld, p, m, partials, nparts, s, ev);
  if (row_bytes % 16 == 0) {
    switch (row_bytes / 16) {
      SPHX_NV(16, 1) SPHX_NV(16, 2) SPHX_NV(16, 3) SPHX_NV(16, 4)
      default: break;
    }
    if constexpr (std::is_same_v<T, double>) {
      switch (row_bytes / 16) {
        SPHX_NV(16, 5) SPHX_NV(16, 6) SPHX_NV(16, 7) SPHX_NV(16, 8)
        default: break;
      }
    }
  } else if constexpr (std::is_same_v<T, float>) {
    // FP32 rows of 2, 6, 10 or 14 values: 8-byte vectors
    if (row_bytes % 8 == 0) {
      switch (row_bytes / 8) {
        SPHX_NV(8, 1) SPHX_NV(8, 3) SPHX_NV(8, 5) SPHX_NV(8, 7)
        default: break;
      }
    }
  }
#undef SPHX_NV
  return SPHX_E_INVALID_ARG;
}

}  // namespace

int padded_ld(int m, int elem_bytes) {
  const int e = 16 / elem_bytes;
  return (m + e - 1) / e * e;
}

template <typename T>
int vspmm_store(sphx_graph *g, const SpmmPlan &plan, const T *X, int ld, int m,
                EpiStoreP<T> epi, hipStream_t s) {
  return dispatch_nv<T, VStore>(g, plan, X, ld, epi, m, nullptr, nullptr, s);
}
template <typename T>
int vspmm_residual(sphx_graph *g, const SpmmPlan &plan, const T *X, int ld, int m,
                   EpiResidualP<T> epi, double *norm_partials, int *n_norm_blocks,
                   hipStream_t s) {
  if (!plan.binned && plan.group > 1 && (ld * (int)sizeof(T)) % 16 == 0) {
    // 13..48-neighbour meshes: the LDS-staged store product writes L X, then
    // a streaming pass forms the residual, the Jacobi step and the norms
    // (the fused residual epilogue keeps per-lane index reads and ran at
    // about two thirds of the store product's rate there)
    int r = dispatch_nv<T, VStore>(g, plan, X, ld, EpiStoreP<T>{epi.LX, ld}, m, nullptr,
                                   nullptr, s);
    if (r != SPHX_OK) return r;
    return resid_stream<T>(g->n, X, ld, m, epi, norm_partials, n_norm_blocks, s);
  }
  return dispatch_nv<T, VResidual>(g, plan, X, ld, epi, m, norm_partials, n_norm_blocks, s);
}
template <typename T>
int vspmm_shiftdot(sphx_graph *g, const SpmmPlan &plan, const T *X, int ld, int m,
                   EpiShiftDotP<T> epi, double *partials, int *n_blocks, hipStream_t s) {
  return dispatch_nv<T, VShiftDot>(g, plan, X, ld, epi, m, partials, n_blocks, s);
}
template <typename T>
int vspmm_cheb(sphx_graph *g, const SpmmPlan &plan, const T *X, int ld, int m,
               EpiChebP<T> epi, hipStream_t s, const LaunchEvents *ev) {
  return dispatch_nv<T, VCheb>(g, plan, X, ld, epi, m, nullptr, nullptr, s, ev);
}

template <typename T>
int vspmm_poly(sphx_graph *g, const SpmmPlan &plan, const T *X, int ld, int m,
               EpiPolyP<T> epi, hipStream_t s, const LaunchEvents *ev) {
  return dispatch_nv<T, VPoly>(g, plan, X, ld, epi, m, nullptr, nullptr, s, ev);
}

#define SPHX_VINST(T)                                                                       \
  template int vspmm_store<T>(sphx_graph *, const SpmmPlan &, const T *, int, int,         \
                              EpiStoreP<T>, hipStream_t);                                  \
  template int vspmm_residual<T>(sphx_graph *, const SpmmPlan &, const T *, int, int,      \
                                 EpiResidualP<T>, double *, int *, hipStream_t);           \
  template int vspmm_shiftdot<T>(sphx_graph *, const SpmmPlan &, const T *, int, int,      \
                                 EpiShiftDotP<T>, double *, int *, hipStream_t);           \
  template int vspmm_cheb<T>(sphx_graph *, const SpmmPlan &, const T *, int, int,          \
                             EpiChebP<T>, hipStream_t, const LaunchEvents *);              \
  template int vspmm_poly<T>(sphx_graph *, const SpmmPlan &, const T *, int, int,          \
                             EpiPolyP<T>, hipStream_t, const LaunchEvents *);
SPHX_VINST(float)
SPHX_VINST(double)
#undef SPHX_VINST

}  // namespace sphx
