// Gradient of a loss l(lambda, V) with respect to the edge weights, through
// the eigenpairs of L_C v = lambda B v (weighted Laplacian of Sec. 3.2).
//
// Raising w_e of edge e = {i, j} changes L_C by (e_i - e_j)(e_i - e_j)^T and,
// for the generalized problem, B = D by e_i e_i^T + e_j e_j^T.  First-order
// perturbation of B-orthonormal eigenpairs (simple eigenvalues) gives, with
// a = V[i,:], b = V[j,:]:
//   eigenvalue terms   g_lam_k [(a_k-b_k)^2 - gen lam_k (a_k^2+b_k^2)]
//   in-block terms     c_kl [(a_k-b_k)(a_l-b_l) - gen lam_k (a_k a_l + b_k b_l)],
//                      c_kl = (g_k . v_l) / (lam_k - lam_l), l != k
//   normalisation      -gen/2 (g_k . v_k)(a_k^2 + b_k^2)
//   out-of-block terms -(mu_ki-mu_kj)(a_k-b_k) + gen lam_k (mu_ki a_k + mu_kj b_k)
// where mu_k solves (L - lam_k B) mu_k = g_k - B V V^T g_k with V^T B mu_k = 0.
// The first three groups are the bilinear forms (a-b)^T M1 (a-b) and
// a^T M2 a + b^T M2 b with small nev x nev matrices built on the host.
//
// The normalized problem L_N y = lambda y has the eigenpairs (lambda, D^1/2 x)
// of the generalized one.  With x = D^-1/2 y, the loss sees y through x and
// through D^1/2, whose entries i and j move by 1/(2 sqrt(d)) when w_e does:
//   dl/dw_e = [generalized gradient with dl/dx = D^1/2 dl/dy]
//             + t_i + t_j,   t_i = sum_k (dl/dy_ik) y_ik / (2 d_i).
//
// mu_k comes from a projected preconditioned conjugate gradient run on all
// columns at once (one Laplacian product per step): iterates stay in the
// B-orthogonal complement of V through z = (I - V V^T B) J r, J the diagonal
// of L - lam_k B inverted; residuals stay orthogonal to V.  The CG blocks are
// n x ld row-major (ld even: 16-byte rows), so the product is the vector-row
// Laplacian kernel with the shift lam_k B and the dots p^T A p fused into its
// epilogue.  The CG scalars (r^T z, alpha, beta, convergence flags) live on
// the device and are computed by one-block reductions in a fixed order; the
// host reads the flags every kCgCheck steps only.  Convergence: the relative
// residual in the preconditioner's norm, sqrt(r^T z / f^T J f) <= cg_tol.
#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace sphx {
namespace {

struct Small {
  double a[kMaxNev * kMaxNev];
};

struct AdjParams {
  int nev;
  int gen;
  double lam[kMaxNev];
};

// Gram partials: out[block][j * nev + k] = sum_i A[i,j] * wgt_i * B[i,k] over
// the block's rows (A, B row-major with row strides lda, ldb).  The 256
// threads form 256 / nev^2 groups, each covering every group-th row of the
// block for all nev^2 pairs (four independent sums per thread keep loads in
// flight); the groups are added in LDS in group order.
__global__ __launch_bounds__(256) void k_small_gram(const double *A, int lda, const double *Bm,
                                                    int ldb, const double *wgt, int64_t n,
                                                    int nev, double *partials,
                                                    int64_t rows_per_block) {
  __shared__ double sh[256];
  const int np = nev * nev;
  const int ng = 256 / np;
  const int t = threadIdx.x;
  const int grp = t / np, pr = t - grp * np;
  const int j = pr / nev, k = pr - j * nev;
  const bool live = grp < ng;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(n, r0 + rows_per_block);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (live) {
    int64_t i = r0 + grp;
    const int64_t st = ng;
    for (; i + 3 * st < r1; i += 4 * st) {
      const double a0 = A[i * lda + j], b0 = Bm[i * ldb + k];
      const double a1 = A[(i + st) * lda + j], b1 = Bm[(i + st) * ldb + k];
      const double a2 = A[(i + 2 * st) * lda + j], b2 = Bm[(i + 2 * st) * ldb + k];
      const double a3 = A[(i + 3 * st) * lda + j], b3 = Bm[(i + 3 * st) * ldb + k];
      if (wgt) {
        s0 += a0 * wgt[i] * b0;
        s1 += a1 * wgt[i + st] * b1;
        s2 += a2 * wgt[i + 2 * st] * b2;
        s3 += a3 * wgt[i + 3 * st] * b3;
      } else {
        s0 += a0 * b0;
        s1 += a1 * b1;
        s2 += a2 * b2;
        s3 += a3 * b3;
      }
    }
    for (; i < r1; i += st) s0 += A[i * lda + j] * (wgt ? wgt[i] : 1.0) * Bm[i * ldb + k];
  }
  sh[t] = live ? (s0 + s1) + (s2 + s3) : 0.0;
  __syncthreads();
  if (t < np) {
    double a = 0.0;
    for (int g = 0; g < ng; ++g) a += sh[g * np + t];
    partials[(int64_t)blockIdx.x * kMaxNev * kMaxNev + t] = a;
  }
}

// out[p] = sum over blocks of partials[block][p], p < cnt: one wavefront per
// output, lanes strided over the blocks, then a butterfly (fixed order).
__global__ __launch_bounds__(1024) void k_small_sum(const double *partials, int nblocks,
                                                    int cnt, double *out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int p = wave; p < cnt; p += 16) {
    double a = 0.0;
    for (int b = lane; b < nblocks; b += 64) a += partials[(int64_t)b * kMaxNev * kMaxNev + p];
    for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off);
    if (lane == 0) out[p] = a;
  }
}

// Vp (n x ld) = V (n x nev) with zero padding columns
__global__ void k_pad_cols(const double *V, int nev, double *Vp, int ld, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * ld;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / ld;
    const int c = (int)(e - i * ld);
    Vp[e] = (V && c < nev) ? V[i * nev + c] : 0.0;
  }
}

// r = g - B V (V^T g)  (M = V^T g, nev x nev, device; g stride nev, V and r
// stride ld, padding columns of r zero)
__global__ void k_project_rhs(const double *G, const double *Vp, const double *bd,
                              const double *M, int64_t n, int nev, int ld, double *R) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * ld;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / ld;
    const int k = (int)(e - i * ld);
    if (k >= nev) { R[e] = 0.0; continue; }
    double s = 0.0;
    for (int j = 0; j < nev; ++j) s += Vp[i * ld + j] * M[j * nev + k];
    R[e] = G[i * nev + k] - (bd ? bd[i] : 1.0) * s;
  }
}

// Device state of the projected CG (one entry per column).
struct CgState {
  double rz[kMaxNev], rz0[kMaxNev], alpha[kMaxNev], beta[kMaxNev];
  int done[kMaxNev];
  int iters;       // steps with at least one active column
  int breakdown;   // a column met p^T A p <= 0 before converging
};

// Optional step x += alpha p, r -= alpha Ap (state given), then z = J r with
// J_ik = 1 / (d_i - lam_k b_i) (1 / d_i where that is not positive).
__global__ void k_cg_step_jac(double *MU, double *R, const double *P, const double *AP,
                              const CgState *st, const double *d, const double *bd,
                              AdjParams p, int64_t n, int ld, double *Z) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * ld;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / ld;
    const int k = (int)(e - i * ld);
    if (k >= p.nev) { Z[e] = 0.0; continue; }
    double r = R[e];
    if (st) {
      const double al = st->alpha[k];
      MU[e] += al * P[e];
      r -= al * AP[e];
      R[e] = r;
    }
    double diag = d[i] - p.lam[k] * (bd ? bd[i] : 1.0);
    if (!(diag > 0.0)) diag = d[i];
    Z[e] = r / diag;
  }
}

// z <- z - V M (M = V^T B z, device) and per-block partial sums of r^T z per
// column (fixed order: rows within a thread, then threads in LDS order).
__global__ __launch_bounds__(256) void k_cg_project(double *Z, const double *Vp,
                                                    const double *M, const double *R,
                                                    int64_t n, int nev, int ld,
                                                    double *rz_partials) {
  __shared__ double sh[256];
  const int rc = 256 / ld;                 // rows per block step (ld <= 16)
  const int row = threadIdx.x / ld, c = threadIdx.x % ld;
  const bool live = threadIdx.x < rc * ld && c < nev;
  double acc = 0.0;
  if (live)
    for (int64_t i = (int64_t)blockIdx.x * rc + row; i < n; i += (int64_t)gridDim.x * rc) {
      double s = 0.0;
      for (int j = 0; j < nev; ++j) s += Vp[i * ld + j] * M[j * nev + c];
      const double z = Z[i * ld + c] - s;
      Z[i * ld + c] = z;
      acc += R[i * ld + c] * z;
    }
  sh[threadIdx.x] = live ? acc : 0.0;
  __syncthreads();
  if (threadIdx.x < nev) {
    double a = 0.0;
    for (int r = 0; r < rc; ++r) a += sh[r * ld + threadIdx.x];
    rz_partials[(int64_t)blockIdx.x * kMaxNev + threadIdx.x] = a;
  }
}

// Fixed-order block sum of column c's partials (stride between blocks given).
__device__ double block_reduce_col(const double *parts, int64_t stride, int nparts) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) a += parts[(int64_t)b * stride];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int off = blockDim.x / 2; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// r^T z of the step: init (first preconditioned residual) or update with beta
// and the convergence test r^T z <= tol^2 f^T J f.
__global__ __launch_bounds__(256) void k_cg_rz(const double *rz_partials, int nparts, int nev,
                                               double tol2, int init, CgState *st) {
  for (int c = 0; c < nev; ++c) {
    const double rz = block_reduce_col(rz_partials + c, kMaxNev, nparts);
    if (threadIdx.x == 0) {
      if (init) {
        st->rz0[c] = rz;
        st->rz[c] = rz;
        st->done[c] = !(rz > 0.0);
        st->alpha[c] = 0.0;
        st->beta[c] = 0.0;
      } else {
        const bool was = st->done[c] != 0;
        const bool conv = was || rz <= tol2 * st->rz0[c];
        st->beta[c] = conv ? 0.0 : rz / st->rz[c];
        st->rz[c] = rz;
        st->done[c] = conv ? 1 : 0;
      }
    }
  }
  if (threadIdx.x == 0 && init) {
    st->iters = 0;
    st->breakdown = 0;
  }
}

// alpha = r^T z / p^T A p from the product's per-block p^T A p partials
// (sum-major, kMaxNormBlocks apart); a column whose p^T A p is not positive
// stops (breakdown flag).
__global__ __launch_bounds__(256) void k_cg_alpha(const double *pap_partials, int nparts,
                                                  int nev, CgState *st) {
  bool any = false;
  for (int c = 0; c < nev; ++c) {
    const double pap = block_reduce_col(pap_partials + (int64_t)c * kMaxNormBlocks, 1, nparts);
    if (threadIdx.x == 0) {
      double al = 0.0;
      if (!st->done[c]) {
        if (pap > 0.0) {
          al = st->rz[c] / pap;
          any = true;
        } else {
          st->done[c] = 1;
          st->breakdown = 1;
        }
      }
      st->alpha[c] = al;
    }
  }
  if (threadIdx.x == 0 && any) st->iters += 1;
}

// p = z + beta p (first step: p = z)
__global__ void k_cg_xpby(double *P, const double *Z, const CgState *st, int first,
                          int64_t n, int ld, int nev) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * ld;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e % ld);
    if (k >= nev) { P[e] = 0.0; continue; }
    P[e] = first ? Z[e] : Z[e] + st->beta[k] * P[e];
  }
}

// Edge gradient: one wavefront per row, lanes over its entries.
template <typename IdxT>
__global__ __launch_bounds__(256) void k_edge_grad(int64_t n, const IdxT *rp,
                                                   const int32_t *col, const double *V,
                                                   const double *MU, int ldmu, Small M1,
                                                   Small M2, AdjParams p, int use_mu,
                                                   double *grad) {
  __shared__ double s1[kMaxNev * kMaxNev], s2[kMaxNev * kMaxNev];
  const int nev = p.nev;
  for (int e = threadIdx.x; e < nev * nev; e += blockDim.x) {
    s1[e] = M1.a[e];
    s2[e] = M2.a[e];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x / 64;
  for (int64_t i = (int64_t)blockIdx.x * wpb + threadIdx.x / 64; i < n;
       i += (int64_t)gridDim.x * wpb) {
    double a[kMaxNev], ci[kMaxNev];
    for (int k = 0; k < nev; ++k) {
      a[k] = V[i * nev + k];
      ci[k] = use_mu ? MU[i * ldmu + k] : 0.0;
    }
    for (int64_t q = (int64_t)rp[i] + lane; q < (int64_t)rp[i + 1]; q += 64) {
      int64_t j = col[q];
      double b[kMaxNev], df[kMaxNev];
      for (int k = 0; k < nev; ++k) {
        b[k] = V[j * nev + k];
        df[k] = a[k] - b[k];
      }
      double g1 = 0.0, g2 = 0.0;
      for (int k = 0; k < nev; ++k) {
        double t1 = 0.0, ta = 0.0, tb = 0.0;
        for (int l = 0; l < nev; ++l) {
          t1 += s1[k * nev + l] * df[l];
          ta += s2[k * nev + l] * a[l];
          tb += s2[k * nev + l] * b[l];
        }
        g1 += df[k] * t1;
        g2 += a[k] * ta + b[k] * tb;
      }
      double g3 = 0.0;
      if (use_mu)
        for (int k = 0; k < nev; ++k) {
          double cj = MU[j * ldmu + k];
          g3 -= (ci[k] - cj) * df[k];
          if (p.gen) g3 += p.lam[k] * (ci[k] * a[k] + cj * b[k]);
        }
      grad[q] = g1 - g2 + g3;
    }
  }
}

// normalized problem: X = D^-1/2 Y, GX = D^1/2 GY, t_i = sum_k GY_ik Y_ik / (2 d_i)
__global__ void k_norm_prep(const double *Y, const double *GY, const double *d, int64_t n,
                            int nev, double *X, double *GX, double *t) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double di = d[i];
    const double r = sqrt(di);
    double acc = 0.0;
    for (int k = 0; k < nev; ++k) {
      const double y = Y[i * nev + k];
      X[i * nev + k] = y / r;
      if (GY) {
        const double gy = GY[i * nev + k];
        GX[i * nev + k] = gy * r;
        acc += gy * y;
      }
    }
    t[i] = acc / (2.0 * di);
  }
}

// grad[q] += t_i + t_j for every CSR entry q = (i, j); one wave per row
template <typename IdxT>
__global__ __launch_bounds__(256) void k_add_vertex_terms(int64_t n, const IdxT *rp,
                                                          const int32_t *col, const double *t,
                                                          double *grad) {
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x / 64;
  for (int64_t i = (int64_t)blockIdx.x * wpb + threadIdx.x / 64; i < n;
       i += (int64_t)gridDim.x * wpb) {
    const double ti = t[i];
    for (int64_t q = (int64_t)rp[i] + lane; q < (int64_t)rp[i + 1]; q += 64)
      grad[q] += ti + t[col[q]];
  }
}

constexpr int kSmallBlocks = 1024;
constexpr int kDotBlocks = 1024;
constexpr int kCgCheck = 8;   // CG steps between host reads of the flags

}  // namespace

size_t adjoint_scratch_bytes(int64_t n, int nev) {
  const int ld = padded_ld(nev, 8);
  size_t blk = align_up(sizeof(double) * n * nev, 256);
  size_t blkp = align_up(sizeof(double) * n * ld, 256);
  // 2 blocks of the normalized transform and t, 6 padded CG blocks (V, mu,
  // r, z, p, Ap), the product's dot partials, Gram and r^T z partials
  return 2 * blk + align_up(sizeof(double) * n, 256) + 6 * blkp +
         align_up(sizeof(double) * 2 * kMaxNev * kMaxNormBlocks, 256) +
         align_up(sizeof(double) * kSmallBlocks * kMaxNev * kMaxNev, 256) +
         align_up(sizeof(double) * kDotBlocks * kMaxNev, 256) +
         align_up(sizeof(double) * kMaxNev * kMaxNev, 256) * 2 +
         align_up(sizeof(CgState), 256) + 4096;
}

int eig_backward(sphx_graph *g, const SpmmPlan &plan, int problem, int nev,
                 const double *lam, const double *V, const double *g_vals, const double *gV,
                 double cg_tol, int cg_max_iter, const double *d64, double *grad,
                 void *scratch, void *pinned, hipStream_t s, std::string *err,
                 int *cg_iters, double *cg_relres) {
  const int64_t n = g->n;
  Arena a;
  a.base = static_cast<char *>(scratch);
  size_t blk = (size_t)n * nev;
  if (cg_iters) *cg_iters = 0;
  if (cg_relres) *cg_relres = 0.0;
  if (problem == SPHX_NORMALIZED) {
    double *Xn = a.take<double>(blk);
    double *GXn = a.take<double>(blk);
    double *t = a.take<double>(n);
    hipLaunchKernelGGL(k_norm_prep, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, V, gV, d64,
                       n, nev, Xn, GXn, t);
    int r = eig_backward(g, plan, SPHX_GENERALIZED, nev, lam, Xn, g_vals, gV ? GXn : nullptr,
                         cg_tol, cg_max_iter, d64, grad, a.base + align_up(a.off, 256), pinned, s,
                         err, cg_iters, cg_relres);
    if (r < 0 || !gV) return r;
    unsigned gb = grid_for(n, 4, 1 << 16);
    if (g->rp64)
      hipLaunchKernelGGL((k_add_vertex_terms<int64_t>), dim3(gb), dim3(256), 0, s, n,
                         (const int64_t *)g->rowptr, g->col, (const double *)t, grad);
    else
      hipLaunchKernelGGL((k_add_vertex_terms<int32_t>), dim3(gb), dim3(256), 0, s, n,
                         (const int32_t *)g->rowptr, g->col, (const double *)t, grad);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
      *err = "adjoint kernel failed";
      return SPHX_E_HIP;
    }
    return r;
  }
  const bool gen = problem == SPHX_GENERALIZED;
  const double *bd = gen ? d64 : nullptr;
  const int ld = padded_ld(nev, 8);
  const size_t blkp = (size_t)n * ld;
  double *Vp = a.take<double>(blkp);
  double *MU = a.take<double>(blkp);
  double *Rr = a.take<double>(blkp);
  double *Z = a.take<double>(blkp);
  double *Pp = a.take<double>(blkp);
  double *AP = a.take<double>(blkp);
  double *pap_parts = a.take<double>((size_t)2 * kMaxNev * kMaxNormBlocks);
  double *parts = a.take<double>((size_t)kSmallBlocks * kMaxNev * kMaxNev);
  double *rz_parts = a.take<double>((size_t)kDotBlocks * kMaxNev);
  double *Mdev = a.take<double>(kMaxNev * kMaxNev);
  double *Mdev2 = a.take<double>(kMaxNev * kMaxNev);
  CgState *st = a.take<CgState>(1);
  (void)Mdev2;
  double *host = static_cast<double *>(pinned);
  const int64_t rpb = ceil_div(n, kSmallBlocks);
  const int nsb = (int)ceil_div(n, rpb);
  const unsigned gew = grid_for((int64_t)blkp, 256, 4096);
  auto gram_small = [&](const double *A, int lda, const double *B, int ldb, const double *w,
                        double *out) {
    hipLaunchKernelGGL(k_small_gram, dim3(nsb), dim3(256), 0, s, A, lda, B, ldb, w, n, nev,
                       parts, rpb);
    hipLaunchKernelGGL(k_small_sum, dim3(1), dim3(1024), 0, s, (const double *)parts, nsb,
                       nev * nev, out);
  };
  AdjParams prm;
  prm.nev = nev;
  prm.gen = gen ? 1 : 0;
  for (int k = 0; k < kMaxNev; ++k) prm.lam[k] = k < nev ? lam[k] : 0.0;
  Small M1{}, M2{};
  for (int k = 0; k < nev; ++k) {
    double gl = g_vals ? g_vals[k] : 0.0;
    M1.a[k * nev + k] += gl;
    if (gen) M2.a[k * nev + k] += lam[k] * gl;
  }
  int status = SPHX_OK;
  bool use_mu = false;
  if (gV) {
    // G^T V: GtV[j * nev + k] = sum_i g_ij v_ik  -> c_kl = GtV[k][l] / (lam_k - lam_l)
    gram_small(gV, nev, V, nev, nullptr, Mdev);
    double gtv[kMaxNev * kMaxNev];
    if (hipMemcpyAsync(gtv, Mdev, sizeof(double) * nev * nev, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return SPHX_E_HIP;
    for (int k = 0; k < nev; ++k)
      for (int l = 0; l < nev; ++l) {
        if (l == k) {
          if (gen) M2.a[k * nev + k] += 0.5 * gtv[k * nev + k];
          continue;
        }
        double c = gtv[k * nev + l] / (lam[k] - lam[l]);
        M1.a[k * nev + l] += c;
        if (gen) M2.a[k * nev + l] += lam[k] * c;
      }
    // ---- mu: projected PCG on all columns, scalars on the device
    use_mu = true;
    hipLaunchKernelGGL(k_pad_cols, dim3(gew), dim3(256), 0, s, V, nev, Vp, ld, n);
    // r0 = g - B V (V^T g); mu0 = 0
    gram_small(V, nev, gV, nev, nullptr, Mdev);
    hipLaunchKernelGGL(k_project_rhs, dim3(gew), dim3(256), 0, s, gV, (const double *)Vp, bd,
                       (const double *)Mdev, n, nev, ld, Rr);
    hipLaunchKernelGGL(k_pad_cols, dim3(gew), dim3(256), 0, s, (const double *)nullptr, 0, MU,
                       ld, n);
    const unsigned gproj = grid_for(n, 256 / ld, kDotBlocks);
    // z = (I - V V^T B) J r and r^T z; first == the step that has no update
    auto precond = [&](bool update) {
      hipLaunchKernelGGL(k_cg_step_jac, dim3(gew), dim3(256), 0, s, MU, Rr,
                         (const double *)Pp, (const double *)AP,
                         update ? (const CgState *)st : nullptr, d64, bd, prm, n, ld, Z);
      gram_small(Vp, ld, Z, ld, bd, Mdev);   // V^T B Z
      hipLaunchKernelGGL(k_cg_project, dim3(gproj), dim3(256), 0, s, Z, (const double *)Vp,
                         (const double *)Mdev, (const double *)Rr, n, nev, ld, rz_parts);
      hipLaunchKernelGGL(k_cg_rz, dim3(1), dim3(256), 0, s, (const double *)rz_parts,
                         (int)gproj, nev, cg_tol * cg_tol, update ? 0 : 1, st);
    };
    precond(false);
    hipLaunchKernelGGL(k_cg_xpby, dim3(gew), dim3(256), 0, s, Pp, (const double *)Z,
                       (const CgState *)st, 1, n, ld, nev);
    if (hipGetLastError() != hipSuccess) {
      *err = "adjoint CG launch failed";
      return SPHX_E_HIP;
    }
    EpiShiftDotP<double> ep{AP, ld, nullptr, bd};
    double *lam_dev = Mdev2;   // lam_k on the device for the product's epilogue
    if (hipMemcpyAsync(lam_dev, prm.lam, sizeof(double) * kMaxNev, hipMemcpyHostToDevice, s) !=
        hipSuccess) {
      *err = "adjoint: copy failed";
      return SPHX_E_HIP;
    }
    ep.lam = lam_dev;
    CgState hs{};
    int it = 0;
    bool all = false;
    while (it < cg_max_iter) {
      const int steps = std::min(kCgCheck, cg_max_iter - it);
      for (int q = 0; q < steps; ++q) {
        int np = 0;
        int r = vspmm_shiftdot<double>(g, plan, Pp, ld, nev, ep, pap_parts, &np, s);
        if (r != SPHX_OK) {
          *err = "adjoint CG product failed";
          return r;
        }
        hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(256), 0, s, (const double *)pap_parts, np,
                           nev, st);
        precond(true);
        hipLaunchKernelGGL(k_cg_xpby, dim3(gew), dim3(256), 0, s, Pp, (const double *)Z,
                           (const CgState *)st, 0, n, ld, nev);
      }
      it += steps;
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(&hs, st, sizeof(CgState), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        *err = "adjoint CG failed";
        return SPHX_E_HIP;
      }
      all = true;
      for (int k = 0; k < nev; ++k) all = all && hs.done[k];
      if (all) break;
    }
    (void)host;
    double worst = 0.0;
    for (int k = 0; k < nev; ++k)
      if (hs.rz0[k] > 0.0) worst = std::max(worst, std::sqrt(std::max(0.0, hs.rz[k] / hs.rz0[k])));
    if (cg_iters) *cg_iters = hs.iters;
    if (cg_relres) *cg_relres = worst;
    if (!all) status = SPHX_NOT_CONVERGED;
    if (hs.breakdown) {
      *err = "adjoint CG: p^T A p not positive (eigenvalues not separated from the rest)";
      status = SPHX_NOT_CONVERGED;
    }
  }
  unsigned gb = grid_for(n, 4, 1 << 16);
  if (g->rp64)
    hipLaunchKernelGGL((k_edge_grad<int64_t>), dim3(gb), dim3(256), 0, s, n,
                       (const int64_t *)g->rowptr, g->col, V, (const double *)MU, ld, M1, M2,
                       prm, use_mu ? 1 : 0, grad);
  else
    hipLaunchKernelGGL((k_edge_grad<int32_t>), dim3(gb), dim3(256), 0, s, n,
                       (const int32_t *)g->rowptr, g->col, V, (const double *)MU, ld, M1, M2,
                       prm, use_mu ? 1 : 0, grad);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    *err = "adjoint kernel failed";
    return SPHX_E_HIP;
  }
  return status;
}

}  // namespace sphx
