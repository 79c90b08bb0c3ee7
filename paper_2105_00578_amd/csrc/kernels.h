// Host-side launch interfaces of the HIP kernels.
#pragma once

#include "common.h"

namespace sphx {

// ------------------------------------------------------------------ setup
// Row classes of the Laplacian product by neighbour count.  Class c < kNumBins
// holds rows with at most bin_max_deg(c) neighbours (and more than the class
// below), served by bin_group(c) lanes per row; rows beyond kHubDeg are hubs,
// split into kHubChunk-entry chunks of one wavefront each.
constexpr int kHubDeg = 16384;
constexpr int kHubChunk = 4096;
constexpr int kNumBins = 4;
__host__ __device__ constexpr int bin_max_deg(int c) {
  return c == 0 ? 12 : (c == 1 ? 48 : (c == 2 ? 192 : kHubDeg));
}
__host__ __device__ constexpr int bin_group(int c) {
  return c == 0 ? 1 : (c == 1 ? 4 : (c == 2 ? 16 : 64));
}
// Graphs whose rows all have at most this many neighbours are not binned:
// every row in natural order, `group` lanes per row (for rows of more than 12
// neighbours the product picks 1, 2 or 4 lanes from the gathered row width
// and the weight stream).
constexpr int kUnbinnedMaxDeg = 48;

struct SpmmPlan {
  bool binned = false;          // false: natural row order, `group` lanes per row
  int group = 1;
  // unbinned unit-weight graphs with 32-bit row pointers whose neighbours all
  // lie within 32767 rows: column offsets from the row, 2 bytes per entry
  const int16_t *dcol = nullptr;
  const int32_t *rows[kNumBins] = {};    // row lists of the classes (binned)
  int64_t nrows[kNumBins] = {};
  const int32_t *hub_rows = nullptr;     // hub rows
  int64_t n_hub = 0;
  const int64_t *chunk_k0 = nullptr;     // per chunk: first entry
  const int64_t *chunk_k1 = nullptr;     // per chunk: one past last entry
  const int32_t *hub_chunk_begin = nullptr;  // per hub: first chunk (n_hub+1)
  int64_t n_chunks = 0;
  double *hub_partial = nullptr;         // n_chunks * kMaxNev scratch (T-sized)
};

// Degree statistics of a graph (pattern and weighted).
struct DegreeStats {
  int64_t max_deg, sum_deg, min_deg;
  double max_wdeg, min_wdeg;
};

int validate_graph(sphx_graph *g, hipStream_t s, int32_t *flags_dev, int *flags_host);
// d64[i] = weighted degree; dT (float or double copy, may be null);
// returns statistics through a device buffer then host.
// Edge-weight range of a weighted graph (g->wmin, g->wmax; unit graphs: no
// work), cached in the graph.  scratch: device, 2 doubles per block of at most
// kWrangeBlocks blocks; pinned: host, as many.  Weights spanning more than
// 2^40 give SPHX_E_BAD_WEIGHT (the exact fixed-point sums need less).
constexpr int kWrangeBlocks = 1024;
int weight_range(sphx_graph *g, void *scratch, void *pinned, hipStream_t s);
int compute_degrees(sphx_graph *g, double *d64, float *d32, void *scratch,
                    DegreeStats *out, void *pinned, hipStream_t s);
int build_plan(sphx_graph *g, Arena &ws, SpmmPlan *plan, const DegreeStats &st,
               void *pinned, hipStream_t s);
size_t plan_bytes(sphx_graph *g);
// Degree order of a graph: rows sorted by floor(log2 degree), descending,
// ties in increasing id.  *out is a copy of g over permuted arrays in
// scratch (degree_order_bytes(g)); perm[new] = old, inv[old] = new.
size_t degree_order_bytes(const sphx_graph *g);
int build_degree_order(sphx_graph *g, void *scratch, sphx_graph *out, int32_t **perm,
                       int32_t **inv, hipStream_t s);

// ------------------------------------------------------------------ spmm
// Epilogue parameters.
template <typename T>
struct EpiStoreP { T *Y; int ldy; };
template <typename T>
struct EpiResidualP {
  T *LX;             // L x output (ld)
  T *OUT;            // residual (or Jacobi-preconditioned residual) output
  int ld;
  const double *theta;   // device, per column
  const double *d64;     // weighted degrees
  int generalized;
  int jacobi;
};
// One step of the GMRES-polynomial apply (product form over the roots):
//   Y <- Y + P / theta_i  (Y = 0 on the first step),
//   P' = P - s (L P) / theta_i  (s = 1 / d_i for the generalized problem),
// and on the last step Y <- Y + P' / theta_{k+1} instead of storing P'.
template <typename T>
struct EpiPolyP {
  const T *Yin;        // nullable on the first step
  T *Yout;
  T *Pout;             // unused on the last step
  int ld;
  double inv_t, inv_t_next;
  const double *dinv;  // nullable: 1
  int last;
};

// Shifted product with dots: out = L p - lam_c b_i p (b = bd or 1), and
// per-block partials of p^T out per column (the norm-partial layout).
template <typename T>
struct EpiShiftDotP {
  T *OUT;
  int ld;
  const double *lam;   // device, per column
  const double *bd;    // nullable: B = I
};

template <typename T>
struct EpiChebP {
  const T *prev;       // previous iterate is prev_scale * prev (nullable = 0)
  const T *R;          // right-hand side
  T *OUT;
  int ld;
  double src_scale;    // the gathered source is src_scale * X
  double prev_scale;
  double alpha, beta;
  const double *dinv;  // nullable: 1
};

// Norm partials: 2*kMaxNev sums, each over up to kMaxNormBlocks blocks,
// stored sum-major (sum q of block b at q * kMaxNormBlocks + b).
constexpr int kMaxNormBlocks = 10240;
// Rayleigh-quotient partials: up to kRqStride blocks, sum-major.
constexpr int kRqStride = 256;

template <typename T>
int spmm_store(sphx_graph *g, const SpmmPlan &plan, const T *X, int ldx,
               const ColMap &cm, EpiStoreP<T> epi, hipStream_t s);
template <typename T>
int spmm_residual(sphx_graph *g, const SpmmPlan &plan, const T *X, int ldx,
                  const ColMap &cm, EpiResidualP<T> epi, double *norm_partials,
                  int *n_norm_blocks, hipStream_t s);
template <typename T>
int spmm_cheb(sphx_graph *g, const SpmmPlan &plan, const T *X, int ldx,
              const ColMap &cm, EpiChebP<T> epi, hipStream_t s);

// Padded blocks: n x ld with ld * sizeof(T) a multiple of 16 bytes (columns
// m..ld-1 are padding).  Thread-per-row products with 16-byte vector loads.
int padded_ld(int m, int elem_bytes);

// Events that bracket the kernels of one product: a single launch is stamped
// by its own dispatch (start and end of execution); several launches are
// bracketed by stream records.
struct LaunchEvents {
  hipEvent_t start, stop;
};

template <typename T>
int vspmm_store(sphx_graph *g, const SpmmPlan &plan, const T *X, int ld, int m,
                EpiStoreP<T> epi, hipStream_t s);
template <typename T>
int vspmm_residual(sphx_graph *g, const SpmmPlan &plan, const T *X, int ld, int m,
                   EpiResidualP<T> epi, double *norm_partials, int *n_norm_blocks,
                   hipStream_t s);
template <typename T>
int vspmm_shiftdot(sphx_graph *g, const SpmmPlan &plan, const T *X, int ld, int m,
                   EpiShiftDotP<T> epi, double *partials, int *n_blocks, hipStream_t s);
template <typename T>
int vspmm_cheb(sphx_graph *g, const SpmmPlan &plan, const T *X, int ld, int m,
               EpiChebP<T> epi, hipStream_t s, const LaunchEvents *ev = nullptr);
template <typename T>
int vspmm_poly(sphx_graph *g, const SpmmPlan &plan, const T *X, int ld, int m,
               EpiPolyP<T> epi, hipStream_t s, const LaunchEvents *ev = nullptr);

// ------------------------------------------------------------------ dense
// Initial blocks (n x ld, columns >= m zero).
template <typename T>
void launch_init_random(T *X, int64_t n, int m, int ld, uint64_t seed, hipStream_t s);
template <typename T>
void launch_init_piecewise(T *X, int64_t n, int m, int ld, hipStream_t s);

// Gram matrices of S = [X(all m), H(act), P(act, if have_p)] against
// LS = [LX, LH, LP] and B S.  Output: reduced upper-tile entries in
// gram_out[2][kMaxW][kMaxW] (A then B), row-major, only i <= j meaningful.
struct GramArgs {
  int64_t n;
  int m;               // X width
  int ld;              // row stride of every block (>= m)
  ColMap act;          // active columns for H and P
  int use_h, use_p;
  const double *bdiag; // nullable: B = I
};
template <typename T>
int gram(const T *X, const T *LX, const T *H, const T *LH, const T *P,
         const T *LP, const GramArgs &a, double *partials, int max_blocks,
         double *gram_out, hipStream_t s);
size_t gram_partial_doubles(int max_blocks);
constexpr int kGramBlocks = 1024;

// Rayleigh-Ritz on the reduced Gram matrices (one workgroup, FP64).
// Writes Y (kMaxW x kMaxNev, row-major: Y[k * kMaxNev + c]) and theta
// into `rr_out`, and kept / restarted / breakdown into the status.
struct RRArgs {
  int m;            // nev
  int w;            // total basis width
  int p_begin;      // first P column in the basis (== w if no P)
  double drop_tol;
};
void launch_rr(const double *gram_out, const RRArgs &a, double *Y, double *theta,
               DevStatus *st, hipStream_t s);
// GMRES polynomial (poly.hip): scratch bytes, and the roots (Leja order)
// from start vector b (x variables; B-inner product D if gen).
size_t poly_scratch_bytes(int64_t n, int degree);
int poly_roots(sphx_graph *g, const SpmmPlan &plan, bool gen, const double *d64,
               const double *dinv, const double *b, int degree, double *roots, int *nroots,
               void *scratch, void *pinned, hipStream_t s, std::string *err);
// Roots of the GMRES residual polynomial from a (k1 + 1) x k1 Lanczos
// projection (k1 <= kMaxW), modified Leja order; status 1 if H_k is not SPD.
void launch_harmonic_ritz(const double *H, int k1, double *theta, int *status,
                          hipStream_t s);

// X <- [X, H_a, P_a] Y ; P <- [0, H_a, P_a] Y ; LP <- [0, LH_a, LP_a] Y
struct UpdateArgs {
  int64_t n;
  int m;
  int ld;              // row stride of every block (>= m)
  ColMap act;
  int use_h, use_p;
};
// SPHX_E_INVALID_ARG unless ld is at most 256, at least m and, for FP32, a
// multiple of 4.  With LP non-null, LP is updated along with P from LH and
// LP (otherwise the caller forms L P by a product).
template <typename T>
int launch_update(T *X, const T *H, T *P, const T *LH, T *LP, const double *Y,
                  const UpdateArgs &a, hipStream_t s);

// Reduce norm partials -> rho, convergence, active list (one workgroup).
void launch_finalize(const double *norm_partials, int n_blocks, int m,
                     const double *theta, double tol, int locking,
                     DevStatus *st, hipStream_t s);

// Rayleigh quotients / residual norms in FP64 of a final block.
template <typename T>
void launch_rq_partials(const T *X, const double *LX, int64_t n, int m, int ld,
                        const double *bdiag, double *partials, int nblocks,
                        hipStream_t s);
template <typename T>
void launch_res_partials(const T *X, const double *LX, int64_t n, int m, int ld,
                         const double *bdiag, const double *theta,
                         double *partials, int nblocks, hipStream_t s);
// Sum partials[nblocks][2*kMaxNev] into out[2*kMaxNev] (fixed order).
void launch_sum_partials(const double *partials, int nblocks, int cols,
                         double *out, hipStream_t s);
// Per-column argmax |x| (lowest index on ties) -> sign; scale columns.
template <typename T>
int normalize_columns(T *X, int64_t n, int m, const double *scale_dev,
                      void *scratch, hipStream_t s);
size_t normalize_scratch_bytes();

template <typename Tin, typename Tout>
void launch_convert(const Tin *in, Tout *out, int64_t count, hipStream_t s);
template <typename T>
void launch_copy_cols(const T *in, int ldin, T *out, int ldout, int64_t n,
                      int m, hipStream_t s);

// ------------------------------------------------------------------ split
size_t split_scratch_bytes(int64_t n, int K);
template <typename T>
int split_mj(sphx_graph *g, const T *coords, int ld, int ncoord, int K,
             int32_t *part, void *scratch, void *pinned, hipStream_t s,
             std::string *err);

// ---------------------------------------------------------------- quality
size_t quality_scratch_bytes(int K);
// 64-bit words of the pinned host buffer `quality` reads its results through
// (the handle's kPinnedSmallBytes): the 2 x 1024 cut partials and a flag fit,
// part weights come back in chunks of this many
constexpr int kQualityPinnedWords = (int)(kPinnedSmallBytes / 8);
// cut_fixed (optional): the exact cut as an integer multiple of 2^e0 (unit
// weights: the number of cut edges), for exact comparisons
int quality(sphx_graph *g, const int32_t *part, int K, double *cut,
            double *imbalance, int64_t *part_weights, void *scratch,
            void *pinned, hipStream_t s, std::string *err,
            unsigned __int128 *cut_fixed = nullptr);

// ----------------------------------------------------------------- refine
size_t refine_scratch_bytes(int64_t n, int K);
int refine(sphx_graph *g, int32_t *part, int K, double eps, int max_passes, double *cut,
           double *imbalance, int *passes, int64_t *moves, void *scratch, void *pinned,
           hipStream_t s, std::string *err);

// ---------------------------------------------------------------- adjoint
size_t adjoint_scratch_bytes(int64_t n, int nev);
// cg_iters, cg_relres (nullable): CG steps taken and the largest final
// relative residual (preconditioner norm) over the columns
int eig_backward(sphx_graph *g, const SpmmPlan &plan, int problem, int nev,
                 const double *eigvals, const double *V, const double *g_vals,
                 const double *gV, double cg_tol, int cg_max_iter,
                 const double *d64, double *grad, void *scratch, void *pinned,
                 hipStream_t s, std::string *err, int *cg_iters = nullptr,
                 double *cg_relres = nullptr);

}  // namespace sphx
