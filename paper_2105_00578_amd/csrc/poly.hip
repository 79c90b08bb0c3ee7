// GMRES polynomial preconditioner (Sec. 5.2): setup and apply.
//
// The polynomial p of degree k is the one of the GMRES residual polynomial
// pi(x) = prod_{i=1}^{k+1} (1 - x / theta_i) = 1 - x p(x) of a (k+1)-step
// Krylov process from a start vector b.  The operators are self-adjoint in
// the B-inner product (L_C with B = I; D^-1 L_C with B = D), so the process
// is Lanczos with full reorthogonalisation (classical Gram-Schmidt, twice) in
// FP64, and the roots theta_i are the harmonic Ritz values: eigenvalues of the
// pencil (H^T H, H_k) of the (k+2) x (k+1) projection H (dense.hip).  The
// start vector is first made B-orthogonal to the trivial eigenvector (the
// constant), so the polynomial addresses the non-trivial spectrum.
//
// Apply (product form, roots in modified Leja order):
//   P_1 = s r (s = D^-1 for the generalized problem), Y = 0,
//   step i = 1..k:  Y += P_i / theta_i,  P_{i+1} = P_i - s L P_i / theta_i,
//   and finally Y += P_{k+1} / theta_{k+1}, fused into step k.
// Every step is one Laplacian product with the update in its epilogue.
#include <cmath>
#include <vector>

#include "kernels.h"

namespace sphx {
namespace {

constexpr int kDotBlocks = 512;

// partials[q * kDotBlocks + b] = sum over the block's rows of V_q(i) bd(i) w(i)
// (V column-major, column q at V + q * n), fixed order within a block.
__global__ __launch_bounds__(256) void k_bdots(const double *__restrict__ V, int64_t n, int nq,
                                               const double *__restrict__ w,
                                               const double *__restrict__ bd,
                                               double *partials) {
  __shared__ double sh[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = min(n, r0 + per);
  for (int q = 0; q < nq; ++q) {
    double acc = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x)
      acc += V[(int64_t)q * n + i] * (bd ? bd[i] : 1.0) * w[i];
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) sh[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
      partials[(int64_t)q * gridDim.x + blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
  }
}

__global__ void k_sum_parts(const double *partials, int nb, int nq, double *out) {
  const int q = threadIdx.x;
  if (q >= nq) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partials[(int64_t)q * nb + b];
  out[q] = s;
}

// w -= sum_q h_q V_q
__global__ void k_basis_axpy(const double *__restrict__ V, int64_t n, int nq,
                             const double *__restrict__ h, double *w) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = w[i];
    for (int q = 0; q < nq; ++q) v -= h[q] * V[(int64_t)q * n + i];
    w[i] = v;
  }
}

// y = a * x (optionally times dinv_i)
__global__ void k_scale_vec(const double *x, int64_t n, double a, const double *dinv,
                            double *y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] * (dinv ? dinv[i] : 1.0);
}

// x -= c * 1
__global__ void k_shift_vec(double *x, int64_t n, const double *c) {
  const double cc = *c;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] -= cc;
}

__global__ void k_fill(double *x, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

// c = (1^T B x) / (1^T B 1) from the two reduced sums
__global__ void k_ratio(const double *sums, double *c) {
  if (threadIdx.x == 0) *c = sums[0] / sums[1];
}

}  // namespace

size_t poly_scratch_bytes(int64_t n, int degree) {
  const int k1 = degree + 1;
  size_t b = 0;
  b += align_up(sizeof(double) * n * (k1 + 1), 256);              // basis
  b += align_up(sizeof(double) * n, 256) * 2;                     // w, ones
  b += align_up(sizeof(double) * kDotBlocks * (kMaxW + 2), 256);  // partials
  b += align_up(sizeof(double) * (kMaxW + 2) * 2, 256);           // sums
  b += align_up(sizeof(double) * (kMaxW + 1) * kMaxW, 256);       // H
  b += align_up(sizeof(double) * kMaxW, 256) + 1024;              // roots, status
  return b;
}

int poly_roots(sphx_graph *g, const SpmmPlan &plan, bool gen, const double *d64,
               const double *dinv, const double *b, int degree, double *roots, int *nroots,
               void *scratch, void *pinned, hipStream_t s, std::string *err) {
  const int64_t n = g->n;
  int k1 = degree + 1;
  if (degree < 1 || k1 > kMaxW) {
    *err = "polynomial degree must be in [1, 47]";
    return SPHX_E_INVALID_ARG;
  }
  Arena a;
  a.base = static_cast<char *>(scratch);
  double *V = a.take<double>((size_t)n * (k1 + 1));
  double *w = a.take<double>(n);
  double *ones = a.take<double>(n);
  double *parts = a.take<double>((size_t)kDotBlocks * (kMaxW + 2));
  double *sums = a.take<double>((kMaxW + 2) * 2);
  double *Hd = a.take<double>((size_t)(kMaxW + 1) * kMaxW);
  double *th = a.take<double>(kMaxW);
  int *status = a.take<int>(4);
  double *host = static_cast<double *>(pinned);
  const double *bd = gen ? d64 : nullptr;
  const unsigned ge = grid_for(n, 256, 4096);
  auto dots = [&](const double *Vq, int nq, const double *x, double *out_dev) {
    hipLaunchKernelGGL(k_bdots, dim3(kDotBlocks), dim3(256), 0, s, Vq, n, nq, x, bd, parts);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, (const double *)parts, kDotBlocks,
                       nq, out_dev);
  };
  auto fetch = [&](const double *dev, int cnt) -> int {
    if (hipMemcpyAsync(host, dev, sizeof(double) * cnt, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return SPHX_E_HIP;
    return SPHX_OK;
  };
  // v0 = b - c 1 with 1^T B v0 = 0, then B-normalised
  hipLaunchKernelGGL(k_scale_vec, dim3(ge), dim3(256), 0, s, b, n, 1.0, (const double *)nullptr,
                     V);
  hipLaunchKernelGGL(k_fill, dim3(ge), dim3(256), 0, s, ones, n, 1.0);
  dots(V, 1, ones, sums);              // 1^T B b
  dots(ones, 1, ones, sums + 1);       // 1^T B 1
  hipLaunchKernelGGL(k_ratio, dim3(1), dim3(64), 0, s, (const double *)sums, sums + 2);
  hipLaunchKernelGGL(k_shift_vec, dim3(ge), dim3(256), 0, s, V, n, (const double *)(sums + 2));
  dots(V, 1, V, sums);
  SPHX_TRY(fetch(sums, 1));
  if (!(host[0] > 0.0)) {
    *err = "polynomial start vector is zero after removing the trivial component";
    return SPHX_E_INVALID_ARG;
  }
  hipLaunchKernelGGL(k_scale_vec, dim3(ge), dim3(256), 0, s, (const double *)V, n,
                     1.0 / std::sqrt(host[0]), (const double *)nullptr, V);
  std::vector<double> H((size_t)(k1 + 1) * k1, 0.0);
  ColMap one;
  one.count = 1;
  for (int q = 0; q < kMaxNev; ++q) one.col[q] = 0;
  int kk = k1;
  for (int j = 0; j < k1; ++j) {
    const double *vj = V + (size_t)j * n;
    // w = A v_j (A = L, or D^-1 L)
    SPHX_TRY(spmm_store<double>(g, plan, vj, 1, one, EpiStoreP<double>{w, 1}, s));
    if (gen)
      hipLaunchKernelGGL(k_scale_vec, dim3(ge), dim3(256), 0, s, (const double *)w, n, 1.0,
                         dinv, w);
    for (int pass = 0; pass < 2; ++pass) {
      dots(V, j + 1, w, sums);
      hipLaunchKernelGGL(k_basis_axpy, dim3(ge), dim3(256), 0, s, (const double *)V, n, j + 1,
                         (const double *)sums, w);
      SPHX_TRY(fetch(sums, j + 1));
      for (int q = 0; q <= j; ++q) H[(size_t)q * k1 + j] += host[q];
    }
    dots(w, 1, w, sums);
    SPHX_TRY(fetch(sums, 1));
    const double beta = std::sqrt(std::max(host[0], 0.0));
    double hmax = 0.0;
    for (int q = 0; q <= j; ++q) hmax = std::max(hmax, std::fabs(H[(size_t)q * k1 + j]));
    if (!(beta > 1e-12 * hmax)) {
      // invariant Krylov space: its j + 1 Ritz values are exact roots
      kk = j + 1;
      break;
    }
    H[(size_t)(j + 1) * k1 + j] = beta;
    hipLaunchKernelGGL(k_scale_vec, dim3(ge), dim3(256), 0, s, (const double *)w, n, 1.0 / beta,
                       (const double *)nullptr, V + (size_t)(j + 1) * n);
  }
  // (kk + 1) x kk projection, row-major with stride kk
  std::vector<double> Hc((size_t)(kk + 1) * kk, 0.0);
  for (int i = 0; i <= kk; ++i)
    for (int j = 0; j < kk; ++j)
      Hc[(size_t)i * kk + j] = (i < kk || kk == k1) ? H[(size_t)i * k1 + j] : 0.0;
  SPHX_HIP(g->h, hipMemcpyAsync(Hd, Hc.data(), sizeof(double) * Hc.size(),
                                hipMemcpyHostToDevice, s));
  launch_harmonic_ritz(Hd, kk, th, status, s);
  int st = 0;
  SPHX_HIP(g->h, hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, s));
  SPHX_HIP(g->h, hipMemcpyAsync(roots, th, sizeof(double) * kk, hipMemcpyDeviceToHost, s));
  SPHX_HIP(g->h, hipStreamSynchronize(s));
  if (st != 0) {
    *err = "Lanczos projection not positive definite";
    return SPHX_E_BREAKDOWN;
  }
  *nroots = kk;
  return SPHX_OK;
}

}  // namespace sphx
