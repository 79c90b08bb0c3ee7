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
// of L - lam_k B inverted; residuals stay orthogonal to V.
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

// Gram partials: out[block][j * nev + k] = sum_i A[i,j] * wgt_i * B[i,k]
__global__ __launch_bounds__(256) void k_small_gram(const double *A, const double *Bm,
                                                    const double *wgt, int64_t n, int nev,
                                                    double *partials, int64_t rows_per_block) {
  int t = threadIdx.x;
  int j = t / nev, k = t % nev;
  bool live = t < nev * nev;
  int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  int64_t r1 = min(n, r0 + rows_per_block);
  double s = 0.0;
  if (live)
    for (int64_t i = r0; i < r1; ++i)
      s += A[i * nev + j] * (wgt ? wgt[i] : 1.0) * Bm[i * nev + k];
  if (live) partials[(int64_t)blockIdx.x * kMaxNev * kMaxNev + t] = s;
}

__global__ void k_small_sum(const double *partials, int nblocks, int cnt, double *out) {
  int t = threadIdx.x;
  if (t >= cnt) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partials[(int64_t)b * kMaxNev * kMaxNev + t];
  out[t] = s;
}

// per-column partial dots: out[block][c] = sum_i X[i,c] Y[i,c] (cols < nev)
__global__ __launch_bounds__(256) void k_coldot(const double *X, const double *Y,
                                                int64_t n, int nev, double *partials) {
  const int rc = 256 / nev;
  const int row = threadIdx.x / nev, c = threadIdx.x % nev;
  const bool live = threadIdx.x < rc * nev;
  double s = 0.0;
  if (live)
    for (int64_t r = (int64_t)blockIdx.x * rc + row; r < n; r += (int64_t)gridDim.x * rc)
      s += X[r * nev + c] * Y[r * nev + c];
  __shared__ double sh[256];
  __shared__ int sc[256];
  sh[threadIdx.x] = s;
  sc[threadIdx.x] = live ? c : -1;
  __syncthreads();
  if (threadIdx.x < nev) {
    double a = 0.0;
    for (int u = 0; u < 256; ++u)
      if (sc[u] == (int)threadIdx.x) a += sh[u];
    partials[(int64_t)blockIdx.x * kMaxNev * kMaxNev + threadIdx.x] = a;
  }
}

// f = g - B V (V^T g)  (M = V^T g, nev x nev, device)
__global__ void k_project_rhs(const double *G, const double *V, const double *bd,
                              const double *M, int64_t n, int nev, double *F) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * nev;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e / nev;
    int k = (int)(e - i * nev);
    double s = 0.0;
    for (int j = 0; j < nev; ++j) s += V[i * nev + j] * M[j * nev + k];
    F[e] = G[e] - (bd ? bd[i] : 1.0) * s;
  }
}

// zt = J r, J_i,k = 1 / (d_i - lam_k b_i) (1/d_i if not positive)
__global__ void k_jac(const double *R, const double *d, const double *bd, AdjParams p,
                      int64_t n, double *Z) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * p.nev;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e / p.nev;
    int k = (int)(e - i * p.nev);
    double diag = d[i] - p.lam[k] * (bd ? bd[i] : 1.0);
    if (!(diag > 0.0)) diag = d[i];
    Z[e] = R[e] / diag;
  }
}

// Z <- Z - V M   (M = V^T B Z, device)
__global__ void k_sub_vm(double *Z, const double *V, const double *M, int64_t n, int nev) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * nev;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e / nev;
    int k = (int)(e - i * nev);
    double s = 0.0;
    for (int j = 0; j < nev; ++j) s += V[i * nev + j] * M[j * nev + k];
    Z[e] -= s;
  }
}

// AP = LP - lam_k B P (in place in LP)
__global__ void k_shift(double *LP, const double *P, const double *bd, AdjParams p, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * p.nev;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = e / p.nev;
    int k = (int)(e - i * p.nev);
    LP[e] -= p.lam[k] * (bd ? bd[i] : 1.0) * P[e];
  }
}

struct Coef {
  double c[kMaxNev];
};

// x += alpha p ; r -= alpha Ap
__global__ void k_axpy2(double *X, double *R, const double *P, const double *AP, Coef al,
                        int64_t n, int nev) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * nev;
       e += (int64_t)gridDim.x * blockDim.x) {
    int k = (int)(e % nev);
    X[e] += al.c[k] * P[e];
    R[e] -= al.c[k] * AP[e];
  }
}

// p = z + beta p
__global__ void k_xpby(double *P, const double *Z, Coef be, int64_t n, int nev) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * nev;
       e += (int64_t)gridDim.x * blockDim.x) {
    int k = (int)(e % nev);
    P[e] = Z[e] + be.c[k] * P[e];
  }
}

// Edge gradient: one wavefront per row, lanes over its entries.
template <typename IdxT>
__global__ __launch_bounds__(256) void k_edge_grad(int64_t n, const IdxT *rp,
                                                   const int32_t *col, const double *V,
                                                   const double *MU, Small M1, Small M2,
                                                   AdjParams p, int use_mu, double *grad) {
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
      ci[k] = use_mu ? MU[i * nev + k] : 0.0;
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
          double cj = MU[j * nev + k];
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

constexpr int kSmallBlocks = 256;
constexpr int kDotBlocks = 256;

}  // namespace

size_t adjoint_scratch_bytes(int64_t n, int nev) {
  size_t blk = align_up(sizeof(double) * n * nev, 256);
  // 7 blocks of the solve, 2 of the normalized transform, t
  return 9 * blk + align_up(sizeof(double) * n, 256) +
         align_up(sizeof(double) * kSmallBlocks * kMaxNev * kMaxNev, 256) +
         align_up(sizeof(double) * kMaxNev * kMaxNev, 256) * 2 + 4096;
}

int eig_backward(sphx_graph *g, const SpmmPlan &plan, int problem, int nev,
                 const double *lam, const double *V, const double *g_vals, const double *gV,
                 double cg_tol, int cg_max_iter, const double *d64, double *grad,
                 void *scratch, void *pinned, hipStream_t s, std::string *err) {
  const int64_t n = g->n;
  Arena a;
  a.base = static_cast<char *>(scratch);
  size_t blk = (size_t)n * nev;
  if (problem == SPHX_NORMALIZED) {
    double *Xn = a.take<double>(blk);
    double *GXn = a.take<double>(blk);
    double *t = a.take<double>(n);
    hipLaunchKernelGGL(k_norm_prep, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, V, gV, d64,
                       n, nev, Xn, GXn, t);
    int r = eig_backward(g, plan, SPHX_GENERALIZED, nev, lam, Xn, g_vals, gV ? GXn : nullptr,
                         cg_tol, cg_max_iter, d64, grad, a.base + align_up(a.off, 256), pinned, s,
                         err);
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
  double *MU = a.take<double>(blk);
  double *Rr = a.take<double>(blk);
  double *Z = a.take<double>(blk);
  double *Pp = a.take<double>(blk);
  double *AP = a.take<double>(blk);
  double *F = a.take<double>(blk);
  double *Gz = a.take<double>(blk);
  double *parts = a.take<double>((size_t)kSmallBlocks * kMaxNev * kMaxNev);
  double *Mdev = a.take<double>(kMaxNev * kMaxNev);
  double *Mdev2 = a.take<double>(kMaxNev * kMaxNev);
  double *host = static_cast<double *>(pinned);
  const int64_t rpb = ceil_div(n, kSmallBlocks);
  const int nsb = (int)ceil_div(n, rpb);
  auto gram_small = [&](const double *A, const double *B, const double *w, double *out) {
    hipLaunchKernelGGL(k_small_gram, dim3(nsb), dim3(256), 0, s, A, B, w, n, nev, parts, rpb);
    hipLaunchKernelGGL(k_small_sum, dim3(1), dim3(256), 0, s, (const double *)parts, nsb,
                       nev * nev, out);
  };
  auto coldot = [&](const double *X, const double *Y, double *out_host) -> int {
    int nb = (int)grid_for(n, 256 / nev, kDotBlocks);
    hipLaunchKernelGGL(k_coldot, dim3(nb), dim3(256), 0, s, X, Y, n, nev, parts);
    hipLaunchKernelGGL(k_small_sum, dim3(1), dim3(256), 0, s, (const double *)parts, nb, nev,
                       Mdev2);
    if (hipMemcpyAsync(out_host, Mdev2, sizeof(double) * nev, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return SPHX_E_HIP;
    return SPHX_OK;
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
    gram_small(gV, V, nullptr, Mdev);
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
    // ---- mu: projected PCG on all columns
    use_mu = true;
    // M = V^T g (nev x nev) ; F = g - B V M
    gram_small(V, gV, nullptr, Mdev);
    hipLaunchKernelGGL(k_project_rhs, dim3(grid_for(blk, 256, 4096)), dim3(256), 0, s, gV, V,
                       bd, (const double *)Mdev, n, nev, F);
    if (hipMemsetAsync(MU, 0, sizeof(double) * blk, s) != hipSuccess ||
        hipMemcpyAsync(Rr, F, sizeof(double) * blk, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return SPHX_E_HIP;
    auto precond = [&]() {
      hipLaunchKernelGGL(k_jac, dim3(grid_for(blk, 256, 4096)), dim3(256), 0, s,
                         (const double *)Rr, d64, bd, prm, n, Z);
      gram_small(V, Z, bd, Mdev);   // V^T B Z
      hipLaunchKernelGGL(k_sub_vm, dim3(grid_for(blk, 256, 4096)), dim3(256), 0, s, Z, V,
                         (const double *)Mdev, n, nev);
    };
    precond();
    if (hipMemcpyAsync(Pp, Z, sizeof(double) * blk, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return SPHX_E_HIP;
    double rz[kMaxNev], f2[kMaxNev], r2[kMaxNev], pap[kMaxNev];
    SPHX_TRY(coldot(Rr, Z, host));
    for (int k = 0; k < nev; ++k) rz[k] = host[k];
    SPHX_TRY(coldot(F, F, host));
    for (int k = 0; k < nev; ++k) f2[k] = host[k];
    bool done[kMaxNev];
    for (int k = 0; k < nev; ++k) done[k] = !(f2[k] > 0.0);
    ColMap idm;
    idm.count = nev;
    for (int q = 0; q < kMaxNev; ++q) idm.col[q] = q < nev ? q : 0;
    int it = 0;
    for (; it < cg_max_iter; ++it) {
      bool all = true;
      for (int k = 0; k < nev; ++k) all = all && done[k];
      if (all) break;
      SPHX_TRY(spmm_store<double>(g, plan, Pp, nev, idm, EpiStoreP<double>{AP, nev}, s));
      hipLaunchKernelGGL(k_shift, dim3(grid_for(blk, 256, 4096)), dim3(256), 0, s, AP,
                         (const double *)Pp, bd, prm, n);
      SPHX_TRY(coldot(Pp, AP, host));
      Coef al{};
      for (int k = 0; k < nev; ++k) {
        pap[k] = host[k];
        al.c[k] = (done[k] || !(pap[k] > 0.0)) ? 0.0 : rz[k] / pap[k];
      }
      hipLaunchKernelGGL(k_axpy2, dim3(grid_for(blk, 256, 4096)), dim3(256), 0, s, MU, Rr,
                         (const double *)Pp, (const double *)AP, al, n, nev);
      SPHX_TRY(coldot(Rr, Rr, host));
      for (int k = 0; k < nev; ++k) {
        r2[k] = host[k];
        if (!done[k] && r2[k] <= cg_tol * cg_tol * f2[k]) done[k] = true;
      }
      precond();
      SPHX_TRY(coldot(Rr, Z, host));
      Coef be{};
      for (int k = 0; k < nev; ++k) {
        double nz = host[k];
        be.c[k] = (done[k] || !(rz[k] != 0.0)) ? 0.0 : nz / rz[k];
        rz[k] = nz;
      }
      hipLaunchKernelGGL(k_xpby, dim3(grid_for(blk, 256, 4096)), dim3(256), 0, s, Pp,
                         (const double *)Z, be, n, nev);
    }
    bool all = true;
    for (int k = 0; k < nev; ++k) all = all && done[k];
    if (!all) status = SPHX_NOT_CONVERGED;
  }
  unsigned gb = grid_for(n, 4, 1 << 16);
  if (g->rp64)
    hipLaunchKernelGGL((k_edge_grad<int64_t>), dim3(gb), dim3(256), 0, s, n,
                       (const int64_t *)g->rowptr, g->col, V, (const double *)MU, M1, M2, prm,
                       use_mu ? 1 : 0, grad);
  else
    hipLaunchKernelGGL((k_edge_grad<int32_t>), dim3(gb), dim3(256), 0, s, n,
                       (const int32_t *)g->rowptr, g->col, V, (const double *)MU, M1, M2, prm,
                       use_mu ? 1 : 0, grad);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    *err = "adjoint kernel failed";
    return SPHX_E_HIP;
  }
  (void)Gz;
  return status;
}

}  // namespace sphx
