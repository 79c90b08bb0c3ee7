// Dense block kernels of LOBPCG (Algorithm 1): initial blocks, Gram matrices
// on FP64 matrix cores, Rayleigh-Ritz in one workgroup, the fused block
// update, the convergence check, and final normalisation.
//
// Blocks are row-major n x ld (ld >= m; columns m..ld-1 are padding).  The
// Rayleigh-Ritz basis is
// S = [X, H_a, P_a] where a lists the active (unconverged) columns.
#include <cmath>

#include "kernels.h"

namespace sphx {
namespace {

// ------------------------------------------------------------ random init
// Counter-based normal draws: splitmix64 (Steele, Lea, Flood 2014) of the
// element counter gives two uniforms, Box-Muller turns them into N(0, 1).
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Element (i, c) draws from the counter i * m + c, independent of the padding.
template <typename T>
__global__ void k_init_random(T *X, int64_t n, int m, int ld, uint64_t seed) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * ld;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / ld;
    const int c = (int)(e - i * ld);
    if (c >= m) {
      X[e] = T(0);
      continue;
    }
    const uint64_t ctr = (uint64_t)(i * m + c);
    uint64_t a = splitmix64(seed ^ splitmix64(2 * ctr));
    uint64_t b = splitmix64(seed ^ splitmix64(2 * ctr + 1));
    double u1 = (double)((a >> 11) + 1) * 0x1.0p-53;   // (0, 1]
    double u2 = (double)(b >> 11) * 0x1.0p-53;         // [0, 1)
    X[e] = T(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
  }
}

// Sec. 6.2.1: column 0 is the constant vector; column j >= 1 is the indicator
// of index block j-1 of d blocks [floor(b n / d), floor((b+1) n / d)).
template <typename T>
__global__ void k_init_piecewise(T *X, int64_t n, int m, int ld) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * ld;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e / ld;
    int c = (int)(e - i * ld);
    T v = T(0);
    if (c == 0) v = T(1);
    else if (c < m) {
      int64_t b = c - 1;
      int64_t lo = b * n / m, hi = (b + 1) * n / m;
      v = (i >= lo && i < hi) ? T(1) : T(0);
    }
    X[e] = v;
  }
}

// ------------------------------------------------------------------ Gram
typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kCh = 64;   // rows per LDS chunk

struct GramDev {
  int64_t n;
  int m, ld, w;
  int offH, offP;           // column offsets of the H and P parts in S
  int use_h, use_p;
  int inv[kMaxNev];         // inverse active map: column -> position or -1
  const double *bdiag;
};

// Source s of the basis: 0 X, 1 LX, 2 H, 3 LH, 4 P, 5 LP.  Even sources
// feed S, odd ones L S.  Column c of source s lands at S column
// off[s/2] + pos, pos = c (X) or the active position of c (H, P).
template <typename T>
struct GramSrc {
  const T *p[6];
};

constexpr int kPre = (kCh * kMaxNev + 255) / 256;   // staged values per thread and source

// Tiles: NT x NT tiles of 16 columns cover the padded width W = 16 NT; the
// upper ones (NT (NT + 1) / 2 per matrix) are formed.  kCompact (NT = 2,
// w <= 24): two tiles per matrix instead -- T1 = columns 0..15 against
// 0..15, and T2 = columns w-16..w-1 (rows) against 16..w-1 followed by
// 0..w-17 (columns), whose entries give the pairs with a column >= 16 (the
// ones against 0..w-17 by symmetry, stored transposed); one tile per wave.
template <typename T, int NT, bool kCompact = false>
__global__ __launch_bounds__(256) void k_gram(GramDev a, GramSrc<T> src,
                                              int64_t rows_per_block, double *partials) {
  static_assert(!kCompact || NT == 2, "compact tiles are for two-tile widths");
  constexpr int W = 16 * NT;
  constexpr int WP = W + 1;
  constexpr int NTILES = kCompact ? 4 : NT * (NT + 1);   // tiles of both matrices
  constexpr int TPW = (NTILES + 3) / 4;
  __shared__ double sS[kCh * WP];
  __shared__ double sL[kCh * WP];
  __shared__ double sb[kCh];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int m = a.m;
  const int ld = a.ld;
  for (int e = t; e < kCh * WP; e += blockDim.x) {
    sS[e] = 0.0;
    sL[e] = 0.0;
  }
  // tile ownership, and the S columns of this lane's tile row / column
  const int i16 = lane & 15;
  const int k4 = lane >> 4;
  const int wc = a.w - 16;      // compact: T2 row offset, and the width of its two column runs
  int tmat[TPW], tti[TPW], ttj[TPW], tci[TPW], tcj[TPW];
  d4 acc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    int tt = wave + 4 * q;
    tmat[q] = -1;
    tti[q] = ttj[q] = 0;
    if (tt < NTILES) {
      if (kCompact) {
        tmat[q] = tt >> 1;
        tti[q] = tt & 1;          // 0: T1, 1: T2
      } else {
        int mat = tt / (NT * (NT + 1) / 2);
        int r = tt % (NT * (NT + 1) / 2);
        int ti = 0;
        while (r >= NT - ti) { r -= NT - ti; ++ti; }
        tmat[q] = mat;
        tti[q] = ti;
        ttj[q] = ti + r;
      }
    }
    if (kCompact) {
      const bool t2 = tti[q] == 1;
      tci[q] = t2 ? wc + i16 : i16;
      // T2 columns: 16..w-1, then 0..w-17, then a zero padding column
      tcj[q] = !t2 ? i16 : (i16 < wc ? 16 + i16 : (i16 < 2 * wc ? i16 - wc : W - 1));
    } else {
      tci[q] = tti[q] * 16 + i16;
      tcj[q] = ttj[q] * 16 + i16;
    }
    acc[q] = d4{0.0, 0.0, 0.0, 0.0};
  }
  // per staged slot: destination (row, S column) or -1
  const bool use[6] = {true, true, a.use_h != 0, a.use_h != 0, a.use_p != 0, a.use_p != 0};
  const int offs[3] = {0, a.offH, a.offP};
  int dst[3][kPre];
#pragma unroll
  for (int r = 0; r < kPre; ++r) {
    int e = t + 256 * r;
    int row = e / ld, c = e - row * ld;
    bool in = e < kCh * ld && c < m;
    dst[0][r] = in ? row * WP + c : -1;
    int pos = (in && a.inv[c] >= 0) ? a.inv[c] : -1;
    dst[1][r] = pos >= 0 ? row * WP + offs[1] + pos : -1;
    dst[2][r] = pos >= 0 ? row * WP + offs[2] + pos : -1;
  }
  const int64_t rb = (int64_t)blockIdx.x * rows_per_block;
  const int64_t re = min(a.n, rb + rows_per_block);
  T st[6][kPre];
  auto fetch = [&](int64_t r0) {
    const int64_t base = r0 * ld;
    const int64_t lim = (re - r0) * ld;   // valid elements of this chunk
#pragma unroll
    for (int s = 0; s < 6; ++s) {
#pragma unroll
      for (int r = 0; r < kPre; ++r) {
        int e = t + 256 * r;
        st[s][r] = (use[s] && dst[s >> 1][r] >= 0 && e < lim) ? src.p[s][base + e] : T(0);
      }
    }
  };
  __syncthreads();
  if (rb < re) fetch(rb);
  for (int64_t r0 = rb; r0 < re; r0 += kCh) {
    // stage the fetched chunk into LDS
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      if (!use[s]) continue;
      double *dstm = (s & 1) ? sL : sS;
#pragma unroll
      for (int r = 0; r < kPre; ++r) {
        int d = dst[s >> 1][r];
        if (d >= 0) dstm[d] = double(st[s][r]);
      }
    }
    if (t < kCh) {
      int64_t gr = r0 + t;
      sb[t] = gr < re ? (a.bdiag ? a.bdiag[gr] : 1.0) : 0.0;
    }
    __syncthreads();
    // the next chunk's loads overlap the products below
    if (r0 + kCh < re) fetch(r0 + kCh);
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      if (tmat[q] < 0) continue;
      const int ci = tci[q];
      const int cj = tcj[q];
      if (tmat[q] == 0) {
#pragma unroll 4
        for (int kk = 0; kk < kCh; kk += 4) {
          int k = kk + k4;
          double av = sS[k * WP + ci];
          double bv = sL[k * WP + cj];
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
        }
      } else {
#pragma unroll 4
        for (int kk = 0; kk < kCh; kk += 4) {
          int k = kk + k4;
          double av = sS[k * WP + ci];
          double bv = sS[k * WP + cj] * sb[k];
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // D layout of the 16x16x4 FP64 product: accumulator register r of a lane
  // holds row 4*r + lane/16, column lane%16.
  double *out = partials + (int64_t)blockIdx.x * 2 * W * W;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    if (tmat[q] < 0) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (kCompact && tti[q] == 1) {
        // T2 entry (row R, column C): the upper entry (R, C) for C >= 16,
        // R <= C; the upper entry (C, R) for C < w-16, R >= 16 (pairs with
        // both below 16 come from T1); nothing for the padding column
        const int R = wc + 4 * r + k4, C = tcj[q];
        int gi = -1, gj = -1;
        if (C >= 16 && C < a.w && R <= C) { gi = R; gj = C; }
        if (C < wc && R >= 16) { gi = C; gj = R; }
        if (gi >= 0) out[(int64_t)tmat[q] * W * W + gi * W + gj] = acc[q][r];
      } else {
        int gi = (kCompact ? 0 : tti[q] * 16) + 4 * r + k4;
        int gj = (kCompact ? 0 : ttj[q] * 16) + i16;
        out[(int64_t)tmat[q] * W * W + gi * W + gj] = acc[q][r];
      }
    }
  }
}

// Sum the block partials of upper tiles in block order: each block takes 16
// entries, 16 thread groups sum interleaved subsets of the partial blocks,
// and the 16 subset sums are added in a fixed order.
__global__ __launch_bounds__(256) void k_gram_reduce(const double *partials, int nblocks,
                                                     int NT, int w, double *out) {
  const int W = 16 * NT;
  const int E = 2 * W * W;
  const int t = threadIdx.x;
  const int e = blockIdx.x * 16 + (t & 15);
  const int sub = t >> 4;
  __shared__ double sh[256];
  double s0 = 0.0, s1 = 0.0;
  if (e < E) {
    int ij = e % (W * W);
    int i = ij / W, j = ij - i * W;
    if (i <= j && j < w) {
      int b = sub;
      for (; b + 16 < nblocks; b += 32) {
        s0 += partials[(int64_t)b * E + e];
        s1 += partials[(int64_t)(b + 16) * E + e];
      }
      if (b < nblocks) s0 += partials[(int64_t)b * E + e];
    }
  }
  sh[t] = s0 + s1;
  __syncthreads();
  if (t < 16 && e < E) {
    double tot = 0.0;
    for (int u = 0; u < 16; ++u) tot += sh[u * 16 + t];
    int mat = e / (W * W);
    int ij = e - mat * W * W;
    int i = ij / W, j = ij - i * W;
    out[mat * kMaxW * kMaxW + i * kMaxW + j] = tot;
  }
}

// --------------------------------------------------------- Rayleigh-Ritz
constexpr int LDA = kMaxW + 1;
static_assert(kMaxW < 64, "Rayleigh-Ritz pivot search: one candidate per lane of a wave");

// Cyclic Jacobi eigensolver (round-robin parallel ordering) on the k x k
// symmetric matrix in A (LDS, stride LDA); V receives the eigenvectors, and
// the returned pointer (A or B) the rotated matrix.  For odd k the matrices
// carry one zero row and column k (its pairs never rotate), so that every
// pair of a round has two rows.  The pairs of one round are disjoint, so
// A <- R^T A R splits into independent 2 x 2 blocks (pair I's rows, pair J's
// columns).  In every wave, lane I computes the angle of pair I from the
// matrix of the previous round; each thread then takes one block, fetches
// the angles of I and J from those lanes, rotates its rows with I's angle,
// then its columns with J's (a row pass followed by a column pass; a pair
// that does not rotate has c = 1, s = 0, which leaves its entries exactly as
// they are), and writes the block into the other buffer; V <- V R likewise
// by blocks, in place.  One barrier per round.  Before each sweep every pair
// is tested once: the sweeps stop when no pair would rotate.
__device__ __forceinline__ void jacobi_pair(int r, int t, int kk, int &p, int &q) {
  // written with selects (t varies across lanes)
  int a = r + t, b = r - t;
  a = a >= kk - 1 ? a - (kk - 1) : a;
  b = b < 0 ? b + (kk - 1) : b;
  a = t == 0 ? kk - 1 : a;
  b = t == 0 ? r : b;
  p = min(a, b);
  q = max(a, b);
}

// rotations stop once an off-diagonal entry is at rounding level (a few ulps
// of ||A||), or negligible next to both diagonal entries:
// |a_pq| > 2e-16 sqrt(|a_pp a_qq|), compared in squares
__device__ __forceinline__ bool jacobi_rotates(double apq, double app, double aqq,
                                               double abs_floor) {
  return (fabs(apq) > abs_floor) & (apq * apq > 4e-32 * fabs(app * aqq));
}

// 1/x and 1/sqrt(x) from the hardware estimates and two Newton steps each
// (quadratic convergence from the estimate's error to a few ulps)
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  for (int i = 0; i < 2; ++i) {
    const double h = fma(-0.5 * x * y, y, 0.5);   // (1 - x y^2) / 2
    y = fma(y, h, y);
  }
  return y;
}

// Rotation (c, s) that annihilates a_pq (Rutishauser's form: the tangent
// t = sgn(th) / (|th| + sqrt(th^2 + 1)), th = (a_qq - a_pp) / (2 a_pq), the
// smaller root; c = 1 / sqrt(1 + t^2), s = t c); (1, 0) if the pair does not
// rotate.  th is clamped at 1e150 (then t ~ 1 / (2 th) underflows to a
// negligible rotation either way).
__device__ __forceinline__ void jacobi_rotation(double app, double aqq, double apq, bool rot,
                                                double &c, double &s) {
  const double h = rot ? 2.0 * apq : 1.0;
  double th = (aqq - app) * recip(h);
  th = fmin(fmax(th, -1e150), 1e150);
  const double q = fma(th, th, 1.0);
  const double sq = q * rsqrt_nr(q);
  const double tt = (th >= 0 ? 1.0 : -1.0) * recip(fabs(th) + sq);
  const double cc = rsqrt_nr(fma(tt, tt, 1.0));
  c = rot ? cc : 1.0;
  s = rot ? tt * cc : 0.0;
}

constexpr int kJacobiThreads = 256;
// blocks per thread and round: 2 (kMaxW / 2)^2 over kJacobiThreads threads
constexpr int kJacobiItems = (2 * (kMaxW / 2) * (kMaxW / 2) + kJacobiThreads - 1) / kJacobiThreads;

// The matrices are at offsets ao (A), bo (B) and vo (V) of the LDS array S;
// returns the offset of the rotated matrix.
__device__ __forceinline__ int jacobi_eig(double *S, int ao, int bo, int vo, int k, int *flags) {
  double *A = S + ao;
  double *V = S + vo;
  __shared__ double anorm;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int kk = k + (k & 1);
  for (int e = t; e < kk * kk; e += blockDim.x) {
    const int i = e / kk, j = e - i * kk;
    V[i * LDA + j] = (i == j) ? 1.0 : 0.0;
    if (i == k || j == k) A[i * LDA + j] = 0.0;   // odd k: the zero row and column
  }
  if (t < 64) {
    double s = 0.0;
    for (int e = t; e < k * k; e += 64) {
      int i = e / k, j = e - i * k;
      s += A[i * LDA + j] * A[i * LDA + j];
    }
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (t == 0) anorm = sqrt(s);
  }
  if (t < 3) flags[t] = 0;
  __syncthreads();
  if (k < 2) return ao;
  const double abs_floor = 4e-16 * anorm + 1e-300;
  const int npair = kk / 2;              // <= kMaxW / 2 < 64: one pair per lane
  const int nblk = npair * npair;
  const int nwork = 2 * nblk;
  const int npq = k * (k - 1) / 2;
  // this thread's blocks (fixed over the rounds): pair indices and kind
  int bI[kJacobiItems], bJ[kJacobiItems];
  bool bV[kJacobiItems], bOk[kJacobiItems];
#pragma unroll
  for (int u = 0; u < kJacobiItems; ++u) {
    const int e = t + u * kJacobiThreads;
    bOk[u] = e < nwork;
    bV[u] = e >= nblk;
    const int b = e < nblk ? e : (e < nwork ? e - nblk : 0);
    bI[u] = b / npair;
    bJ[u] = b - bI[u] * npair;
  }
  int cur = ao, nxt = bo;
  for (int sweep = 0; sweep < 40; ++sweep) {
    // flags cycle through three words: the one tested now was cleared two
    // sweeps ago, and read by every thread before the barriers of the last
    // sweep, when it is cleared again
    int *rot = flags + sweep % 3;
    if (t == 0) flags[(sweep + 1) % 3] = 0;
    for (int e = t; e < npq; e += blockDim.x) {
      // pair (p, q), p < q: e = q (q - 1) / 2 + p
      int q = (int)((1.0 + sqrt(1.0 + 8.0 * e)) * 0.5);
      while (q * (q - 1) / 2 > e) --q;
      while ((q + 1) * q / 2 <= e) ++q;
      const int p = e - q * (q - 1) / 2;
      if (jacobi_rotates(S[cur + p * LDA + q], S[cur + p * LDA + p], S[cur + q * LDA + q],
                         abs_floor))
        *rot = 1;
    }
    __syncthreads();
    if (*rot == 0) break;
    for (int r = 0; r < kk - 1; ++r) {
      double c, s;
      {
        int p, q;
        jacobi_pair(r, lane < npair ? lane : 0, kk, p, q);
        const double apq = S[cur + p * LDA + q];
        const double app = S[cur + p * LDA + p], aqq = S[cur + q * LDA + q];
        const bool rr = (lane < npair) & (q < k) & jacobi_rotates(apq, app, aqq, abs_floor);
        jacobi_rotation(app, aqq, apq, rr, c, s);
      }
#pragma unroll
      for (int u = 0; u < kJacobiItems; ++u) {
        if (u * kJacobiThreads >= nwork) break;     // uniform
        const int I = bI[u], J = bJ[u];
        const double cI0 = __shfl(c, I), sI0 = __shfl(s, I);
        const double cJ = __shfl(c, J), sJ = __shfl(s, J);
        if (!bOk[u]) continue;
        const bool isv = bV[u];
        const double cI = isv ? 1.0 : cI0, sI = isv ? 0.0 : sI0;
        int p0, q0, p1, q1;
        jacobi_pair(r, I, kk, p0, q0);
        jacobi_pair(r, J, kk, p1, q1);
        const int mi = isv ? vo : cur, oi = isv ? vo : nxt;
        double a00 = S[mi + p0 * LDA + p1], a01 = S[mi + p0 * LDA + q1];
        double a10 = S[mi + q0 * LDA + p1], a11 = S[mi + q0 * LDA + q1];
        {
          const double b00 = cI * a00 - sI * a10, b10 = sI * a00 + cI * a10;
          const double b01 = cI * a01 - sI * a11, b11 = sI * a01 + cI * a11;
          a00 = b00; a10 = b10; a01 = b01; a11 = b11;
        }
        {
          const double b00 = cJ * a00 - sJ * a01, b01 = sJ * a00 + cJ * a01;
          const double b10 = cJ * a10 - sJ * a11, b11 = sJ * a10 + cJ * a11;
          a00 = b00; a01 = b01; a10 = b10; a11 = b11;
        }
        S[oi + p0 * LDA + p1] = a00;
        S[oi + p0 * LDA + q1] = a01;
        S[oi + q0 * LDA + p1] = a10;
        S[oi + q0 * LDA + q1] = a11;
      }
      __syncthreads();
      const int tmp = cur;
      cur = nxt;
      nxt = tmp;
    }
  }
  return cur;
}

// Rayleigh-Ritz (Algorithm 1, RR(S, nev)) on the reduced Gram matrices.
//
// The columns of S are scaled to unit B-norm (Gs = D G_B D, As = D G_A D with
// D = diag(G_B)^-1/2).  A pivoted Cholesky factorisation of Gs picks, at each
// step, the column with the largest remaining Schur-complement diagonal and
// stops when that is at most drop_tol: the k chosen columns span the others
// up to the tolerance (those are dropped as linearly dependent), and
// Gs(piv, piv) = L L^T.  The rows of W = L^-1 are formed along with the
// columns of L: row k is W[k][c] = -(1 / l_kk) sum_j L[k][j] W[j][c] for
// c < k and 1 / l_kk for c = k, where the sums are accumulated step by step
// for every row not chosen yet (acc[i][c] += l_ik W[k][c], right-looking),
// so L itself is never stored.  With C = W^T, S(:, piv) C is B-orthonormal
// and the projected matrix A' = W As(piv, piv) W^T is diagonalised by cyclic
// Jacobi; the m smallest Ritz pairs give Y = D P W^T Z.  If fewer than m
// columns survive, the P block is dropped and the step retried once.
constexpr int kRRThreads = kJacobiThreads;

// (v, i) or (ov, oi), whichever comes first in the order: larger value,
// then lower index; an index < 0 marks no candidate
__device__ __forceinline__ void take_better(double &v, int &i, double ov, int oi) {
  // non-short-circuit operators: selects, no branches
  const bool b = (oi >= 0) & ((i < 0) | (ov > v) | ((ov == v) & (oi < i)));
  v = b ? ov : v;
  i = b ? oi : i;
}

// Value and index of lane (lane ^ pattern) within rows of 16 lanes (DPP).
template <int kCtrl>
__device__ __forceinline__ void dpp_take(double &v, int &i) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), kCtrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), kCtrl, 0xF, 0xF, false);
  const int oi = __builtin_amdgcn_update_dpp(-1, i, kCtrl, 0xF, 0xF, false);
  take_better(v, i, __hiloint2double(hi, lo), oi);
}

// The first (value, index) of the wave in the order above, in every lane
// (all 64 lanes active): within each row of 16 lanes by DPP moves (swap of
// neighbours, of pairs, then the half-row and row mirrors, each pairing
// every lane with one holding the other half's best so far), then across the
// four rows by lane reads.
__device__ __forceinline__ void wave_argmax(double &v, int &i) {
  dpp_take<0xB1>(v, i);    // quad_perm(1, 0, 3, 2)
  dpp_take<0x4E>(v, i);    // quad_perm(2, 3, 0, 1)
  dpp_take<0x141>(v, i);   // row_half_mirror
  dpp_take<0x140>(v, i);   // row_mirror
  const int lo = __double2loint(v), hi = __double2hiint(v);
  double bv = __hiloint2double(__builtin_amdgcn_readlane(hi, 0), __builtin_amdgcn_readlane(lo, 0));
  int bi = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
  for (int r = 1; r < 4; ++r)
    take_better(bv, bi,
                __hiloint2double(__builtin_amdgcn_readlane(hi, 16 * r),
                                 __builtin_amdgcn_readlane(lo, 16 * r)),
                __builtin_amdgcn_readlane(i, 16 * r));
  v = bv;
  i = bi;
}
constexpr int kRRItems = (kMaxW * kMaxW + kRRThreads - 1) / kRRThreads;

__global__ __launch_bounds__(kRRThreads) void k_rr(const double *__restrict__ gram, RRArgs a,
                                                   double *Y, double *theta, DevStatus *st) {
  constexpr int MS = kMaxW * LDA;
  __shared__ double Msh[4 * MS];
  double *M1 = Msh, *M2 = Msh + MS, *M3 = Msh + 2 * MS, *Wi = Msh + 3 * MS;
  __shared__ double sc[kMaxW], lam[kMaxW], dg[2][kMaxW];
  __shared__ int piv[kMaxW], ipiv[kMaxW], perm[kMaxW];
  __shared__ int flags[3];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = a.w, m = a.m;
  const double *GA = gram;
  const double *GB = gram + kMaxW * kMaxW;
  int restarted = 0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    const int wl = attempt == 0 ? w : a.p_begin;   // drop P on retry
    if (t < kMaxW) {
      double g = (t < wl) ? GB[t * kMaxW + t] : 0.0;
      sc[t] = (t < wl && g > 0.0) ? 1.0 / sqrt(g) : 0.0;
      ipiv[t] = -1;
    }
    __syncthreads();
    // M1 = Gs (then its Schur complements, diagonal also in dg), M3 = As,
    // M2 = the accumulated sums acc[i][c] of the rows of W; after the
    // factorisation M1, M2 and M3 take As(piv, piv), As(piv, piv) W^T and A'
    // in turn
    for (int e = t; e < wl * wl; e += blockDim.x) {
      int i = e / wl, j = e - i * wl;
      int lo = i < j ? i : j, hi = i < j ? j : i;
      double sij = sc[i] * sc[j];
      const double gs = GB[lo * kMaxW + hi] * sij;
      M1[i * LDA + j] = gs;
      if (i == j) dg[0][i] = gs;
      M3[i * LDA + j] = GA[lo * kMaxW + hi] * sij;
      M2[i * LDA + j] = 0.0;
    }
    // this thread's entries (i, j) of the wl x wl matrices, fixed over the
    // steps, and whether row i / column j has been chosen (the same for every
    // thread: the pivots are)
    int ei[kRRItems], ej[kRRItems];
    bool ci[kRRItems], cj[kRRItems];
#pragma unroll
    for (int u = 0; u < kRRItems; ++u) {
      const int e = t + u * kRRThreads;
      const bool ok = e < wl * wl;
      ei[u] = ok ? e / wl : 0;
      ej[u] = ok ? e - ei[u] * wl : 0;
      ci[u] = !ok;                 // nothing to do for entries past the matrix
      cj[u] = false;
    }
    bool ct = t >= wl;             // column t chosen (or past the matrix)
    __syncthreads();
    // ---- pivoted Cholesky of Gs, one barrier per step: every wave finds
    // the pivot itself from the diagonal of the previous step (dg[k & 1],
    // which this step does not write; chosen columns hold 0 there)
    int k = 0;
    for (; k < wl; ++k) {
      // the largest positive remaining diagonal entry, the lowest index on
      // ties (one candidate per lane: wl <= kMaxW < 64)
      double bv = lane < wl ? dg[k & 1][lane] : 0.0;
      int best = bv > 0.0 ? lane : -1;
      wave_argmax(bv, best);
      const int p = (best >= 0 && bv > a.drop_tol) ? best : -1;
      if (p < 0) break;
      const double pval = bv;
      const double rd = 1.0 / sqrt(pval);
      if (t == 0) {
        piv[k] = p;
        ipiv[p] = k;
      }
      // row k of W
      if (t <= k) Wi[k * LDA + t] = t == k ? rd : -rd * M2[p * LDA + t];
      // chosen columns leave the diagonal search
      if (t == p) ct = true;
      if (t < wl && ct) dg[(k + 1) & 1][t] = 0.0;
      // Schur complement on the columns not chosen yet, and the sums of the
      // rows of W not formed yet (column p of M1 and row p of M2 are not
      // written in this step); all loads of an entry are issued first
#pragma unroll
      for (int u = 0; u < kRRItems; ++u) {
        const int i = ei[u], j = ej[u];
        if (i == p) ci[u] = true;
        if (j == p) cj[u] = true;
        if (ci[u]) continue;
        const double mip = M1[i * LDA + p], mjp = M1[j * LDA + p], mij = M1[i * LDA + j];
        const double apj = M2[p * LDA + j], aij = M2[i * LDA + j];
        const double li = mip * rd;
        if (!cj[u]) {
          const double v = mij - li * (mjp * rd);
          M1[i * LDA + j] = v;
          if (i == j) dg[(k + 1) & 1][i] = v;
        }
        if (j <= k) M2[i * LDA + j] = aij + li * (j == k ? rd : -rd * apj);
      }
      __syncthreads();
    }
    if (k >= m || attempt == 1 || a.p_begin >= w) {
      if (k < m) {
        // breakdown: keep X as it is
        for (int e = t; e < kMaxW * kMaxNev; e += blockDim.x) {
          int i = e / kMaxNev, c = e - i * kMaxNev;
          Y[e] = (i == c && c < m) ? 1.0 : 0.0;
        }
        if (t == 0) {
          st->kept = k;
          st->restarted = restarted;
          st->breakdown = 1;
        }
        return;
      }
      // Ap = As(piv, piv) -> M1
      for (int e = t; e < k * k; e += blockDim.x) {
        const int i = e / k, j = e - i * k;
        M1[i * LDA + j] = M3[piv[i] * LDA + piv[j]];
      }
      __syncthreads();
      // T = Ap W^T -> M2 (W lower triangular: j <= c)
      for (int e = t; e < k * k; e += blockDim.x) {
        const int i = e / k, c = e - i * k;
        double s0 = 0.0, s1 = 0.0;
        int j = 0;
        for (; j + 1 <= c; j += 2) {
          s0 += M1[i * LDA + j] * Wi[c * LDA + j];
          s1 += M1[i * LDA + j + 1] * Wi[c * LDA + j + 1];
        }
        if (j <= c) s0 += M1[i * LDA + j] * Wi[c * LDA + j];
        M2[i * LDA + c] = s0 + s1;
      }
      __syncthreads();
      // A' = W T -> M3 (j <= i), upper triangle computed and mirrored
      for (int e = t; e < k * k; e += blockDim.x) {
        const int i = e / k, c = e - i * k;
        if (i > c) continue;
        double s0 = 0.0, s1 = 0.0;
        int j = 0;
        for (; j + 1 <= i; j += 2) {
          s0 += Wi[i * LDA + j] * M2[j * LDA + c];
          s1 += Wi[i * LDA + j + 1] * M2[(j + 1) * LDA + c];
        }
        if (j <= i) s0 += Wi[i * LDA + j] * M2[j * LDA + c];
        M3[i * LDA + c] = s0 + s1;
        M3[c * LDA + i] = s0 + s1;
      }
      __syncthreads();
      // eigenpairs of A': values on the diagonal, vectors in M2
      const int af = jacobi_eig(Msh, 2 * MS, 0, MS, k, flags);
      if (t < k) lam[t] = Msh[af + t * LDA + t];
      __syncthreads();
      if (t < k) {
        int rank = 0;
        double v = lam[t];
        for (int j = 0; j < k; ++j)
          if (lam[j] < v || (lam[j] == v && j < t)) ++rank;
        perm[rank] = t;
      }
      __syncthreads();
      // Y (basis row i, Ritz vector c) = sc_i (W^T z_perm[c])[position of
      // i], 0 if dropped
      for (int e = t; e < kMaxW * kMaxNev; e += blockDim.x) {
        int i = e / kMaxNev, c = e - i * kMaxNev;
        double v = 0.0;
        if (i < wl && c < m && ipiv[i] >= 0) {
          const int r = ipiv[i], zc = perm[c];
          double s0 = 0.0, s1 = 0.0;
          int j = r;
          for (; j + 1 < k; j += 2) {
            s0 += Wi[j * LDA + r] * M2[j * LDA + zc];
            s1 += Wi[(j + 1) * LDA + r] * M2[(j + 1) * LDA + zc];
          }
          if (j < k) s0 += Wi[j * LDA + r] * M2[j * LDA + zc];
          v = sc[i] * (s0 + s1);
        }
        Y[e] = v;
      }
      if (t < m) theta[t] = lam[perm[t]];
      if (t == 0) {
        st->kept = k;
        st->restarted = restarted;
        st->breakdown = 0;
      }
      return;
    }
    restarted = 1;
    __syncthreads();
  }
}

// --------------------------------------------------- polynomial roots
// Harmonic Ritz values of a Lanczos projection (the roots of the GMRES
// residual polynomial): H is (k1 + 1) x k1 row-major (stride k1).  They are
// the eigenvalues of the pencil (H^T H, H_k) with H_k the leading k1 x k1
// block (symmetrised): H_k = L L^T (Cholesky), C = L^-1 H^T H L^-T, cyclic
// Jacobi.  The roots are written in modified Leja order: the largest first,
// then each maximising the sum of log distances to those already chosen
// (lowest index on ties).  status: 0, or 1 if H_k is not positive definite.
__global__ __launch_bounds__(kJacobiThreads) void k_harmonic_ritz(const double *__restrict__ Hg, int k1,
                                                       double *theta, int *status) {
  constexpr int MS = kMaxW * LDA;
  __shared__ double Msh[3 * MS];
  double *Mk = Msh, *Mc = Msh + MS, *Mv = Msh + 2 * MS;
  __shared__ double lam[kMaxW];
  __shared__ int flags[3], bad;
  const int t = threadIdx.x;
  // Mk = sym(H_k), Mc = H^T H
  for (int e = t; e < k1 * k1; e += blockDim.x) {
    const int i = e / k1, j = e - i * k1;
    Mk[i * LDA + j] = 0.5 * (Hg[i * k1 + j] + Hg[j * k1 + i]);
    double sum = 0.0;
    for (int r = 0; r <= k1; ++r) sum += Hg[r * k1 + i] * Hg[r * k1 + j];
    Mc[i * LDA + j] = sum;
  }
  if (t == 0) bad = 0;
  __syncthreads();
  // Cholesky of Mk in place (lower), one thread
  if (t == 0) {
    for (int j = 0; j < k1 && !bad; ++j) {
      double d = Mk[j * LDA + j];
      for (int q = 0; q < j; ++q) d -= Mk[j * LDA + q] * Mk[j * LDA + q];
      if (!(d > 0.0)) { bad = 1; break; }
      d = sqrt(d);
      Mk[j * LDA + j] = d;
      for (int i = j + 1; i < k1; ++i) {
        double v = Mk[i * LDA + j];
        for (int q = 0; q < j; ++q) v -= Mk[i * LDA + q] * Mk[j * LDA + q];
        Mk[i * LDA + j] = v / d;
      }
    }
  }
  __syncthreads();
  if (bad) {
    if (t == 0) *status = 1;
    return;
  }
  // T = L^-1 Mc (column per thread) -> Mv
  if (t < k1) {
    for (int i = 0; i < k1; ++i) {
      double v = Mc[i * LDA + t];
      for (int q = 0; q < i; ++q) v -= Mk[i * LDA + q] * Mv[q * LDA + t];
      Mv[i * LDA + t] = v / Mk[i * LDA + i];
    }
  }
  __syncthreads();
  // C = L^-1 T^T (column c has right-hand side row c of T) -> Mc
  if (t < k1) {
    for (int i = 0; i < k1; ++i) {
      double v = Mv[t * LDA + i];
      for (int q = 0; q < i; ++q) v -= Mk[i * LDA + q] * Mc[q * LDA + t];
      Mc[i * LDA + t] = v / Mk[i * LDA + i];
    }
  }
  __syncthreads();
  for (int e = t; e < k1 * k1; e += blockDim.x) {
    const int i = e / k1, j = e - i * k1;
    if (i < j) {
      const double v = 0.5 * (Mc[i * LDA + j] + Mc[j * LDA + i]);
      Mc[i * LDA + j] = v;
      Mc[j * LDA + i] = v;
    }
  }
  __syncthreads();
  // Mk (the factor) is free now: the second buffer of the rotations
  const int af = jacobi_eig(Msh, MS, 0, 2 * MS, k1, flags);
  if (t < k1) lam[t] = Msh[af + t * LDA + t];
  __syncthreads();
  if (t == 0) {
    bool used[kMaxW];
    for (int i = 0; i < k1; ++i) used[i] = false;
    int first = 0;
    for (int i = 1; i < k1; ++i)
      if (fabs(lam[i]) > fabs(lam[first])) first = i;
    theta[0] = lam[first];
    used[first] = true;
    double score[kMaxW];
    for (int i = 0; i < k1; ++i) score[i] = 0.0;
    int last = first;
    for (int q = 1; q < k1; ++q) {
      int best = -1;
      for (int i = 0; i < k1; ++i) {
        if (used[i]) continue;
        score[i] += log(fabs(lam[i] - lam[last]));
        if (best < 0 || score[i] > score[best]) best = i;
      }
      theta[q] = lam[best];
      used[best] = true;
      last = best;
    }
    *status = 0;
  }
}

// --------------------------------------------------------------- update
struct UpdDev {
  int64_t n;
  int m, ld;
  int na;
  int act[kMaxNev];
  int use_h, use_p;
  int offH, offP;     // rows of Y for the H and P parts
  int update_lp;      // also LP <- LH y_H + LP y_P
};

// Rows of all blocks have stride ld, a multiple of E (4 floats: 16-byte
// loads; FP64 elements are loaded one by one, which measured faster than
// pairs).  A chunk of 256 E elements (256 E / ld rows) of each block is read
// with one load per thread and block into LDS (kept in T; widened to double
// where used); thread t then computes the elements t + 256 j of the chunk
// (column c = e % ld < m; padding columns untouched), each as a sum in a
// fixed order: the X part over k, plus the H and P parts over the active
// columns.
template <typename T> struct UpdVec;
template <> struct UpdVec<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int E = 4;
};
template <> struct UpdVec<double> {
  typedef double type;
  static constexpr int E = 1;
};

template <typename T>
__global__ __launch_bounds__(256) void k_update(T *X, const T *__restrict__ H, T *P,
                                                const T *__restrict__ LH, T *LP,
                                                const double *__restrict__ Yg, UpdDev a) {
  using V = typename UpdVec<T>::type;
  constexpr int E = UpdVec<T>::E;
  constexpr int CH = 256 * E;
  __shared__ double sY[kMaxW * kMaxNev];
  __shared__ V sX[256], sH[256], sP[256], sLH[256], sLP[256];
  const T *lX = reinterpret_cast<const T *>(sX);
  const T *lH = reinterpret_cast<const T *>(sH);
  const T *lP = reinterpret_cast<const T *>(sP);
  const T *lLH = reinterpret_cast<const T *>(sLH);
  const T *lLP = reinterpret_cast<const T *>(sLP);
  const bool upd_lp = a.update_lp;
  const int m = a.m, ld = a.ld;
  const int rc = CH / ld;       // rows per chunk
  const int t = threadIdx.x;
  for (int e = t; e < kMaxW * kMaxNev; e += blockDim.x) sY[e] = Yg[e];
  const bool write_p = a.use_h || a.use_p;
  for (int64_t r0 = (int64_t)blockIdx.x * rc; r0 < a.n; r0 += (int64_t)gridDim.x * rc) {
    const int64_t base = r0 * ld;
    const int lim = (int)min((int64_t)rc, a.n - r0) * ld;
    __syncthreads();
    if (t * E < lim) {
      const int64_t vb = base / E + t;
      sX[t] = reinterpret_cast<const V *>(X)[vb];
      if (a.use_h) {
        sH[t] = reinterpret_cast<const V *>(H)[vb];
        if (upd_lp) sLH[t] = reinterpret_cast<const V *>(LH)[vb];
      }
      if (a.use_p) {
        sP[t] = reinterpret_cast<const V *>(P)[vb];
        if (upd_lp) sLP[t] = reinterpret_cast<const V *>(LP)[vb];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int e = t + 256 * j;
      if (e >= lim) break;
      const int row = e / ld;
      const int c = e - row * ld;
      if (c >= m) continue;
      double p = 0.0, lp = 0.0, x = 0.0;
      const int o = row * ld;
      if (a.use_h)
        for (int q = 0; q < a.na; ++q) {
          const double y = sY[(a.offH + q) * kMaxNev + c];
          p += double(lH[o + a.act[q]]) * y;
          if (upd_lp) lp += double(lLH[o + a.act[q]]) * y;
        }
      if (a.use_p)
        for (int q = 0; q < a.na; ++q) {
          const double y = sY[(a.offP + q) * kMaxNev + c];
          p += double(lP[o + a.act[q]]) * y;
          if (upd_lp) lp += double(lLP[o + a.act[q]]) * y;
        }
      for (int k = 0; k < m; ++k) x += double(lX[o + k]) * sY[k * kMaxNev + c];
      x += p;
      X[base + e] = T(x);
      if (write_p) {
        P[base + e] = T(p);
        if (upd_lp) LP[base + e] = T(lp);
      }
    }
  }
}

// ------------------------------------------------------------- finalize
// Sum the sum-major partials (sum q of block b at partials[q * stride + b])
// over b in a fixed order -> out[q] for the 2m sums q < m and
// kMaxNev <= q < kMaxNev + m.  One wavefront per sum: lanes stride over the
// blocks into eight accumulators (independent loads in flight), which are
// combined in a fixed tree, then a butterfly across lanes.
constexpr int kSumThreads = 1024;
__device__ void sum_partials_block(const double *partials, int nblocks, int stride, int m,
                                   double *out) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  for (int j = wave; j < 2 * m; j += nw) {
    const int q = j < m ? j : kMaxNev + (j - m);
    const double *p = partials + (int64_t)q * stride;
    double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int b = lane;
    for (; b + 7 * 64 < nblocks; b += 8 * 64) {
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] += p[b + u * 64];
    }
#pragma unroll
    for (int u = 0; u < 7; ++u)
      if (b + u * 64 < nblocks) v[u] += p[b + u * 64];
    double r = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    for (int off = 32; off >= 1; off >>= 1) r += __shfl_xor(r, off);
    if (lane == 0) out[q] = r;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kSumThreads) void k_finalize(const double *partials, int nblocks,
                                                          int m, const double *theta,
                                                          double tol, int locking,
                                                          DevStatus *st) {
  __shared__ double sums[2 * kMaxNev];
  sum_partials_block(partials, nblocks, kMaxNormBlocks, m, sums);
  if (threadIdx.x == 0) {
    double floor_th = m > 1 ? theta[1] : theta[0];
    int nconv = 0, na = 0;
    bool conv[kMaxNev];
    for (int c = 0; c < m; ++c) {
      double scale = fmax(theta[c], floor_th);
      if (!(scale > 0.0)) scale = 1.0;
      double rn = sqrt(sums[c]), xn = sqrt(sums[kMaxNev + c]);
      double rho = xn > 0.0 ? rn / (scale * xn) : INFINITY;
      st->rho[c] = rho;
      st->theta[c] = theta[c];
      conv[c] = rho <= tol;
      nconv += conv[c] ? 1 : 0;
    }
    for (int c = 0; c < m; ++c)
      if (!conv[c] || (!locking && nconv < m)) st->act[na++] = c;
    st->nact = na;
    st->nconv = nconv;
  }
}

__global__ __launch_bounds__(kSumThreads) void k_sum_partials(const double *partials,
                                                              int nblocks, int stride, int m,
                                                              double *out) {
  __shared__ double sums[2 * kMaxNev];
  if (threadIdx.x < 2 * kMaxNev) sums[threadIdx.x] = 0.0;
  __syncthreads();
  sum_partials_block(partials, nblocks, stride, m, sums);
  if (threadIdx.x < 2 * kMaxNev) out[threadIdx.x] = sums[threadIdx.x];
}

// Per-column block sums with a fixed lane -> column assignment, stored
// sum-major with stride kRqStride.
__device__ void colsum2(int c, double v1, double v2, int m, double *partials) {
  __shared__ double s1[256], s2[256];
  __shared__ int sc[256];
  int t = threadIdx.x;
  s1[t] = v1;
  s2[t] = v2;
  sc[t] = c;
  __syncthreads();
  if (t < m) {
    double a = 0.0, b = 0.0;
    for (int u = 0; u < (int)blockDim.x; ++u)
      if (sc[u] == t) { a += s1[u]; b += s2[u]; }
    partials[(int64_t)t * kRqStride + blockIdx.x] = a;
    partials[(int64_t)(kMaxNev + t) * kRqStride + blockIdx.x] = b;
  }
}

// Rayleigh quotient partials: sum x.lx and sum b x^2 per column (blocks of
// row stride ld; thread t takes column t % ld of rows t / ld).
template <typename T>
__global__ __launch_bounds__(256) void k_rq(const T *X, const double *LX, int64_t n, int m,
                                            int ld, const double *bdiag, double *partials) {
  const int rc = 256 / ld;
  const int row = threadIdx.x / ld;
  const int c = threadIdx.x % ld;
  const bool live = threadIdx.x < rc * ld && c < m;
  double a = 0.0, b = 0.0;
  if (live)
    for (int64_t r = (int64_t)blockIdx.x * rc + row; r < n; r += (int64_t)gridDim.x * rc) {
      double x = double(X[r * ld + c]);
      double bd = bdiag ? bdiag[r] : 1.0;
      a += x * LX[r * ld + c];
      b += bd * x * x;
    }
  colsum2(live ? c : -1, a, b, m, partials);
}

// Residual partials: sum (lx - theta b x)^2 / b and sum b x^2 per column.
template <typename T>
__global__ __launch_bounds__(256) void k_res(const T *X, const double *LX, int64_t n, int m,
                                             int ld, const double *bdiag, const double *theta,
                                             double *partials) {
  const int rc = 256 / ld;
  const int row = threadIdx.x / ld;
  const int c = threadIdx.x % ld;
  const bool live = threadIdx.x < rc * ld && c < m;
  double a = 0.0, b = 0.0;
  if (live) {
    double th = theta[c];
    for (int64_t r = (int64_t)blockIdx.x * rc + row; r < n; r += (int64_t)gridDim.x * rc) {
      double x = double(X[r * ld + c]);
      double bd = bdiag ? bdiag[r] : 1.0;
      double res = LX[r * ld + c] - th * bd * x;
      a += res * res / bd;
      b += bd * x * x;
    }
  }
  colsum2(live ? c : -1, a, b, m, partials);
}

// Column argmax |x| (lowest index on ties): block partials (value, index).
template <typename T>
__global__ __launch_bounds__(256) void k_colmax(const T *X, int64_t n, int m, double *pv,
                                                int64_t *pi) {
  const int rc = 256 / m;
  const int row = threadIdx.x / m;
  const int c = threadIdx.x % m;
  const bool live = threadIdx.x < rc * m;
  double bv = -1.0;
  int64_t bi = INT64_MAX;
  if (live)
    for (int64_t r = (int64_t)blockIdx.x * rc + row; r < n; r += (int64_t)gridDim.x * rc) {
      double v = fabs(double(X[r * m + c]));
      if (v > bv || (v == bv && r < bi)) { bv = v; bi = r; }
    }
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  __shared__ int scol[256];
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  scol[threadIdx.x] = live ? c : -1;
  __syncthreads();
  if (threadIdx.x < m) {
    double v = -1.0;
    int64_t ix = INT64_MAX;
    for (int u = 0; u < (int)blockDim.x; ++u)
      if (scol[u] == (int)threadIdx.x)
        if (sv[u] > v || (sv[u] == v && si[u] < ix)) { v = sv[u]; ix = si[u]; }
    pv[blockIdx.x * kMaxNev + threadIdx.x] = v;
    pi[blockIdx.x * kMaxNev + threadIdx.x] = ix;
  }
}

template <typename T>
__global__ void k_colsign(const T *X, int m, int nblocks, const double *pv,
                          const int64_t *pi, double *sign) {
  int c = threadIdx.x;
  if (c >= m) return;
  double v = -1.0;
  int64_t ix = INT64_MAX;
  for (int b = 0; b < nblocks; ++b) {
    double bv = pv[b * kMaxNev + c];
    int64_t bi = pi[b * kMaxNev + c];
    if (bv > v || (bv == v && bi < ix)) { v = bv; ix = bi; }
  }
  double x = (ix == INT64_MAX) ? 1.0 : double(X[ix * m + c]);
  sign[c] = x < 0 ? -1.0 : 1.0;
}

struct Scales { double s[kMaxNev]; };

template <typename T>
__global__ void k_colscale(T *X, int64_t n, int m, const double *sign, Scales sc) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * m;
       e += (int64_t)gridDim.x * blockDim.x) {
    int c = (int)(e % m);
    X[e] = T(double(X[e]) * sign[c] * sc.s[c]);
  }
}

template <typename Tin, typename Tout>
__global__ void k_convert(const Tin *in, Tout *out, int64_t count) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = Tout(in[e]);
}

template <typename T>
__global__ void k_copy_cols(const T *in, int ldin, T *out, int ldout, int64_t n, int m) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * m;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e / m;
    int c = (int)(e - i * m);
    out[i * ldout + c] = in[i * ldin + c];
  }
}

}  // namespace

// ------------------------------------------------------------ launchers
template <typename T>
void launch_init_random(T *X, int64_t n, int m, int ld, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL((k_init_random<T>), dim3(grid_for(n * ld, 256, 4096)), dim3(256), 0, s,
                     X, n, m, ld, seed);
}
template <typename T>
void launch_init_piecewise(T *X, int64_t n, int m, int ld, hipStream_t s) {
  hipLaunchKernelGGL((k_init_piecewise<T>), dim3(grid_for(n * ld, 256, 4096)), dim3(256), 0,
                     s, X, n, m, ld);
}

size_t gram_partial_doubles(int max_blocks) {
  return (size_t)max_blocks * 2 * kMaxW * kMaxW;
}

template <typename T>
int gram(const T *X, const T *LX, const T *H, const T *LH, const T *P, const T *LP,
         const GramArgs &a, double *partials, int max_blocks, double *gram_out,
         hipStream_t s) {
  GramDev d;
  d.n = a.n;
  d.m = a.m;
  d.ld = a.ld;
  int na = a.act.count;
  d.use_h = a.use_h && na > 0;
  d.use_p = a.use_p && na > 0;
  d.offH = a.m;
  d.offP = a.m + (d.use_h ? na : 0);
  d.w = a.m + (d.use_h ? na : 0) + (d.use_p ? na : 0);
  for (int c = 0; c < kMaxNev; ++c) d.inv[c] = -1;
  for (int q = 0; q < na; ++q) d.inv[a.act.col[q]] = q;
  d.bdiag = a.bdiag;
  int NT = (d.w + 15) / 16;
  int64_t rows_per_block = ceil_div(a.n, max_blocks);
  rows_per_block = ceil_div(rows_per_block, kCh) * kCh;
  int nb = (int)ceil_div(a.n, rows_per_block);
  if (nb < 1) nb = 1;
  GramSrc<T> sp{{X, LX, H, LH, P, LP}};
  switch (NT) {
    case 1:
      hipLaunchKernelGGL((k_gram<T, 1>), dim3(nb), dim3(256), 0, s, d, sp, rows_per_block,
                         partials);
      break;
    case 2:
      if (d.w <= 24)
        hipLaunchKernelGGL((k_gram<T, 2, true>), dim3(nb), dim3(256), 0, s, d, sp,
                           rows_per_block, partials);
      else
        hipLaunchKernelGGL((k_gram<T, 2>), dim3(nb), dim3(256), 0, s, d, sp, rows_per_block,
                           partials);
      break;
    case 3:
      hipLaunchKernelGGL((k_gram<T, 3>), dim3(nb), dim3(256), 0, s, d, sp, rows_per_block,
                         partials);
      break;
    default:
      return SPHX_E_INVALID_ARG;
  }
  int W = 16 * NT;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)ceil_div(2 * W * W, 16)), dim3(256), 0, s,
                     (const double *)partials, nb, NT, d.w, gram_out);
  return hipGetLastError() == hipSuccess ? SPHX_OK : SPHX_E_HIP;
}

void launch_harmonic_ritz(const double *H, int k1, double *theta, int *status,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_harmonic_ritz, dim3(1), dim3(kJacobiThreads), 0, s, H, k1, theta, status);
}

void launch_rr(const double *gram_out, const RRArgs &a, double *Y, double *theta,
               DevStatus *st, hipStream_t s) {
  hipLaunchKernelGGL(k_rr, dim3(1), dim3(kRRThreads), 0, s, gram_out, a, Y, theta, st);
}

template <typename T>
int launch_update(T *X, const T *H, T *P, const T *LH, T *LP, const double *Y,
                  const UpdateArgs &a, hipStream_t s) {
  UpdDev d;
  d.n = a.n;
  d.m = a.m;
  d.ld = a.ld;
  d.na = a.act.count;
  for (int q = 0; q < kMaxNev; ++q) d.act[q] = q < d.na ? a.act.col[q] : 0;
  d.use_h = a.use_h && d.na > 0;
  d.use_p = a.use_p && d.na > 0;
  d.offH = a.m;
  d.offP = a.m + (d.use_h ? d.na : 0);
  d.update_lp = LP != nullptr && (d.use_h || d.use_p);
  // rows of whole load vectors (the solver pads every block to 16 bytes)
  constexpr int E = UpdVec<T>::E;
  if (a.ld % E != 0 || a.ld > 256 || a.m > a.ld) return SPHX_E_INVALID_ARG;
  int rc = 256 * E / a.ld;
  hipLaunchKernelGGL((k_update<T>), dim3(grid_for(a.n, rc, 8192)), dim3(256), 0, s, X, H, P,
                     LH, LP, Y, d);
  return hipGetLastError() == hipSuccess ? SPHX_OK : SPHX_E_HIP;
}

void launch_finalize(const double *norm_partials, int n_blocks, int m, const double *theta,
                     double tol, int locking, DevStatus *st, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kSumThreads), 0, s, norm_partials, n_blocks, m,
                     theta, tol, locking, st);
}

template <typename T>
void launch_rq_partials(const T *X, const double *LX, int64_t n, int m, int ld,
                        const double *bdiag, double *partials, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL((k_rq<T>), dim3(nblocks), dim3(256), 0, s, X, LX, n, m, ld, bdiag,
                     partials);
}
template <typename T>
void launch_res_partials(const T *X, const double *LX, int64_t n, int m, int ld,
                         const double *bdiag, const double *theta, double *partials,
                         int nblocks, hipStream_t s) {
  hipLaunchKernelGGL((k_res<T>), dim3(nblocks), dim3(256), 0, s, X, LX, n, m, ld, bdiag, theta,
                     partials);
}
void launch_sum_partials(const double *partials, int nblocks, int cols, double *out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kSumThreads), 0, s, partials, nblocks,
                     kRqStride, cols, out);
}

constexpr int kColBlocks = 256;
size_t normalize_scratch_bytes() {
  return (size_t)kColBlocks * kMaxNev * (sizeof(double) + sizeof(int64_t)) + 256 * 8;
}

template <typename T>
int normalize_columns(T *X, int64_t n, int m, const double *scale_host, void *scratch,
                      hipStream_t s) {
  double *pv = static_cast<double *>(scratch);
  int64_t *pi = reinterpret_cast<int64_t *>(pv + kColBlocks * kMaxNev);
  double *sign = reinterpret_cast<double *>(pi + kColBlocks * kMaxNev);
  int nb = (int)grid_for(n, 256 / m, kColBlocks);
  hipLaunchKernelGGL((k_colmax<T>), dim3(nb), dim3(256), 0, s, X, n, m, pv, pi);
  hipLaunchKernelGGL((k_colsign<T>), dim3(1), dim3(64), 0, s, X, m, nb, pv, pi, sign);
  Scales sc;
  for (int c = 0; c < kMaxNev; ++c) sc.s[c] = c < m ? scale_host[c] : 1.0;
  hipLaunchKernelGGL((k_colscale<T>), dim3(grid_for(n * m, 256, 4096)), dim3(256), 0, s, X, n,
                     m, (const double *)sign, sc);
  return hipGetLastError() == hipSuccess ? SPHX_OK : SPHX_E_HIP;
}

template <typename Tin, typename Tout>
void launch_convert(const Tin *in, Tout *out, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<Tin, Tout>), dim3(grid_for(count, 256, 4096)), dim3(256), 0, s,
                     in, out, count);
}
template <typename T>
void launch_copy_cols(const T *in, int ldin, T *out, int ldout, int64_t n, int m,
                      hipStream_t s) {
  hipLaunchKernelGGL((k_copy_cols<T>), dim3(grid_for(n * m, 256, 4096)), dim3(256), 0, s, in,
                     ldin, out, ldout, n, m);
}

#define SPHX_INST(T)                                                                        \
  template void launch_init_random<T>(T *, int64_t, int, int, uint64_t, hipStream_t);      \
  template void launch_init_piecewise<T>(T *, int64_t, int, int, hipStream_t);             \
  template int gram<T>(const T *, const T *, const T *, const T *, const T *, const T *,   \
                       const GramArgs &, double *, int, double *, hipStream_t);            \
  template int launch_update<T>(T *, const T *, T *, const T *, T *, const double *,      \
                                 const UpdateArgs &, hipStream_t);                         \
  template void launch_rq_partials<T>(const T *, const double *, int64_t, int, int,        \
                                      const double *, double *, int, hipStream_t);         \
  template void launch_res_partials<T>(const T *, const double *, int64_t, int, int,       \
                                       const double *, const double *, double *, int,      \
                                       hipStream_t);                                       \
  template int normalize_columns<T>(T *, int64_t, int, const double *, void *, hipStream_t); \
  template void launch_copy_cols<T>(const T *, int, T *, int, int64_t, int, hipStream_t);
SPHX_INST(float)
SPHX_INST(double)
#undef SPHX_INST
template void launch_convert<float, double>(const float *, double *, int64_t, hipStream_t);
template void launch_convert<double, float>(const double *, float *, int64_t, hipStream_t);
template void launch_convert<double, double>(const double *, double *, int64_t, hipStream_t);
template void launch_convert<float, float>(const float *, float *, int64_t, hipStream_t);

}  // namespace sphx
