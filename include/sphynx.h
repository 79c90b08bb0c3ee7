/*
 * sphynx.h -- C ABI of an MI355X (gfx950) spectral graph partitioner.
 *
 * Method: Sphynx (Acer, Boman, Glusa, Rajamanickam, arXiv 2105.00578).  Given
 * a symmetric graph G = (V, E) with edge weights and a part count K, compute
 * the d = floor(log2 K) + 1 smallest eigenpairs of the graph Laplacian by
 * preconditioned LOBPCG, embed each vertex at its entries of eigenvectors
 * 2..d, and split the embedding into K parts (Algorithm 2).
 *
 * Conventions shared by every entry point
 *   - Graphs are CSR: row_ptr[n+1] (int32 or int64), col[nnz] (int32),
 *     optional edge weights w[nnz] (float32 or float64; NULL = unit), optional
 *     vertex weights vwgt[n] (positive int32; NULL = unit).  The pattern and
 *     the weights must be symmetric, with no self-loops and no duplicate
 *     entries, and the column indices of each row strictly increasing.
 *   - Dense blocks of vectors are row-major (vertex-major): entry (i, c) of an
 *     n x m block lives at X[i * m + c].
 *   - "device" pointers are HIP device memory on the handle's device; "host"
 *     pointers are ordinary host memory.  All device pointers are borrowed:
 *     the caller keeps them alive (and unmodified, for graph arrays) for as
 *     long as the object that uses them.
 *   - Every call is ordered on the handle's HIP stream.  Calls that return
 *     host results synchronise that stream before returning.
 *   - Return value: SPHX_OK (0), SPHX_NOT_CONVERGED (+1, a warning: outputs
 *     hold the best iterate), or a negative error code.  No C++ exception
 *     crosses this interface.  sphx_last_error() gives a message.
 *   - A handle must not be used by two host threads at once.
 */
#ifndef SPHYNX_H
#define SPHYNX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
enum {
    SPHX_OK = 0,
    SPHX_NOT_CONVERGED = 1,     /* warning: max_iter reached               */
    SPHX_E_INVALID_ARG = -1,    /* bad size, pointer, option or K          */
    SPHX_E_BAD_GRAPH = -2,      /* row_ptr not monotone, col out of range,
                                   duplicate entries                       */
    SPHX_E_NOT_SYMMETRIC = -3,  /* pattern or weights not symmetric        */
    SPHX_E_BAD_WEIGHT = -4,     /* edge weight not finite and > 0, or
                                   vertex weight < 1                       */
    SPHX_E_SELF_LOOP = -5,      /* an entry (i, i)                          */
    SPHX_E_BREAKDOWN = -6,      /* Rayleigh-Ritz basis lost rank even after
                                   restarting without the P block          */
    SPHX_E_HIP = -7,            /* a HIP runtime call failed               */
    SPHX_E_WORKSPACE = -8       /* workspace too small / allocation failed */
};

/* dtype tags for untyped pointers */
enum { SPHX_UNIT = 0, SPHX_F32 = 1, SPHX_F64 = 2 };

/* eigenvalue problem (Sec. 3.2): L_C x = lambda x, L_C x = lambda D x, or
 * L_N y = lambda y with L_N = I - D^-1/2 A D^-1/2 (the normalized Laplacian).
 * The normalized problem is solved as the generalized one in the variables
 * x = D^-1/2 y (the same pencil up to the congruence D^1/2, so the same
 * eigenvalues, LOBPCG iterates and relative residuals in exact arithmetic);
 * its initial block is given in y and its eigenvectors are returned as
 * y = D^1/2 x with unit 2-norm.  It needs every weighted degree > 0. */
enum { SPHX_COMBINATORIAL = 0, SPHX_GENERALIZED = 1, SPHX_NORMALIZED = 2 };

/* preconditioner (Sec. 5): none, Jacobi (Sec. 5.1), Chebyshev polynomial,
 * or the GMRES polynomial the paper uses (Sec. 5.2; degree 25 by default) */
enum { SPHX_PRECOND_NONE = 0, SPHX_PRECOND_JACOBI = 1, SPHX_PRECOND_CHEBYSHEV = 2,
       SPHX_PRECOND_GMRES = 3 };

/* arithmetic: all FP64, or FP32 sparse products / preconditioner / vector
 * updates with FP64 Gram matrices, Rayleigh-Ritz and norms */
enum { SPHX_FP64 = 0, SPHX_MIXED = 1 };

/* initial block (Sec. 6.2.1): random (default on regular graphs),
 * piecewise constant (default on irregular graphs), or caller supplied */
enum { SPHX_INIT_RANDOM = 0, SPHX_INIT_PIECEWISE = 1, SPHX_INIT_USER = 2 };

/* graph flags */
enum { SPHX_SKIP_VALIDATE = 1u };

typedef struct sphx_handle sphx_handle;
typedef struct sphx_graph sphx_graph;

typedef struct sphx_options {
    int problem;          /* SPHX_COMBINATORIAL / _GENERALIZED / _NORMALIZED */
    int precond;          /* SPHX_PRECOND_*                                  */
    int cheb_degree;      /* degree of the polynomial preconditioner: SpMMs
                             per apply (default 25; GMRES: 1..47)             */
    double cheb_ratio;    /* Chebyshev interval [hi/ratio, hi]; hi bounds the
                             spectrum: 2 max_i d_i (Gershgorin) for L_C, 2 for
                             D^-1 L_C and L_N                                */
    int precision;        /* SPHX_FP64 / SPHX_MIXED                          */
    double tol;           /* bound on every relative residual rho_i:
                             ||L x_i - theta_i B x_i||_{B^-1}
                               / (max(theta_i, theta_1) ||x_i||_B)
                             (B = I for L_N)                                  */
    int max_iter;         /* LOBPCG iterations (default 10000)               */
    int init;             /* SPHX_INIT_*                                      */
    uint64_t seed;        /* for SPHX_INIT_RANDOM                             */
    int locking;          /* soft locking (Algorithm 1 "I" subsets), 1/0     */
    double drop_tol;      /* Rayleigh-Ritz basis directions with relative
                             Gram eigenvalue below this are dropped; 0 picks
                             1e-10 (MIXED) or 1e-14 (FP64)                   */
    int promote_window;   /* MIXED only.  FP32 vectors cannot get closer to
                             an eigenvector than their rounding, so a
                             tolerance near that floor can stall: when, over
                             this many iterations, neither an eigenpair
                             converged nor the largest unconverged rho_i fell
                             below 0.7 of its value at the last such
                             progress, the iteration continues in FP64 from
                             the current vectors (stats.promoted = 1; the
                             returned vectors stay FP32; max_iter bounds
                             both parts together).  0 = 100, < 0 = never.    */
    int reorder;          /* 1 (default): graphs with rows of more than 48
                             neighbours are solved on a copy whose rows are
                             ordered by floor(log2 degree), descending (ties
                             by id), so that the frequently gathered rows of
                             high degree share cache lines; initial blocks and
                             results stay in the caller's order.  0: the
                             caller's order.                                  */
} sphx_options;

typedef struct sphx_stats {
    int iterations;       /* LOBPCG iterations done                           */
    int converged;        /* number of eigenpairs with rho_i <= tol           */
    int restarts;         /* Rayleigh-Ritz restarts without the P block       */
    int graph_regular;    /* 1 iff max degree / average degree <= 10          */
    int64_t max_degree;
    double avg_degree;
    double rho[32];       /* final rho_i from one FP64 product L X (first 32) */
    double ms_total;      /* device time of the call (HIP events)             */
    double ms_setup, ms_spmm, ms_precond, ms_gram, ms_rr, ms_update,
           ms_split, ms_quality;   /* per-phase device time from HIP events
                                      around the launches, only when the
                                      handle's timing flag is on; ms_spmm
                                      covers the plain and residual Laplacian
                                      products, ms_precond the Chebyshev
                                      steps (each a fused Laplacian product)  */
    int64_t spmm_calls;   /* Laplacian products launched (all kinds)         */
    int64_t precond_calls;     /* Chebyshev steps launched                   */
    double gb_spmm, gb_precond;  /* algorithmic GB moved by the launches timed
                                    in ms_spmm / ms_precond: index arrays
                                    once, each block entry read or written
                                    once (gathered rows counted once)         */
    int64_t precond_cols; /* sum over preconditioner applies of the number of
                             active (unconverged) columns they served         */
    int32_t promoted;     /* 1 if a MIXED solve continued in FP64 (see
                             sphx_options.promote_window); iterations count
                             both parts                                       */
    int32_t col_index_bytes; /* bytes per column index the vector products
                                read: 2 when the graph (unit weights, 32-bit
                                row pointers, at most 48 neighbours per row,
                                every neighbour within 32767 rows) is stored
                                as int16 offsets from the row, else 4.  The
                                algorithmic GB above count 4 (the int32 CSR
                                the caller passed).                           */
} sphx_stats;

/* ---------------------------------------------------------------- basics */

/* Message for a status code (static string). */
const char *sphx_status_string(int status);

/* Create a handle on HIP device `device`, ordering work on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  *h receives the handle. */
int sphx_create(sphx_handle **h, int device, void *hip_stream);
int sphx_destroy(sphx_handle *h);
int sphx_set_stream(sphx_handle *h, void *hip_stream);
/* Last error message of this handle ("" if none). */
const char *sphx_last_error(const sphx_handle *h);
/* Per-phase timing with HIP events (adds synchronisation; off by default). */
int sphx_set_timing(sphx_handle *h, int on);

/* Eq. 4: number of eigenvectors d = floor(log2 K) + 1 (K >= 1), else -1. */
int sphx_num_eigenvectors(int K);

/* Defaults of Sec. 6.3.1 for a preconditioner: regular graphs use the
 * combinatorial problem; irregular graphs the normalized one with a
 * polynomial (Chebyshev or GMRES) preconditioner and the generalized one
 * otherwise; the tolerance is 1e-3 on regular graphs and 1e-2 on irregular
 * ones; initial vectors are random on regular graphs and piecewise constant
 * on irregular ones (Sec. 6.2.1).  The other fields: degree 25, ratio 1000,
 * FP64, max_iter 10000, locking on, drop_tol 0 (automatic),
 * promote_window 0 (100 iterations), reorder 1. */
void sphx_options_default(sphx_options *opt, int graph_is_regular, int precond);

/* ---------------------------------------------------------------- graphs */

/* Wrap a device CSR graph (Sec. 3.1).  row_ptr: device int32[n+1]
 * (row_ptr_is_64 = 0) or int64[n+1] (= 1).  col: device int32[nnz].
 * w: device edge weights of type w_dtype (SPHX_F32/SPHX_F64) or NULL with
 * SPHX_UNIT.  vwgt: device int32[n] vertex weights (>= 1) or NULL (unit).
 * Unless flags has SPHX_SKIP_VALIDATE, the arrays are checked on the device
 * (row_ptr monotone from 0 to nnz, 0 <= col < n, columns strictly increasing
 * within each row -- hence no duplicates --, no self-loops, symmetric pattern
 * and weights, weights finite and > 0): errors SPHX_E_BAD_GRAPH,
 * SPHX_E_SELF_LOOP, SPHX_E_NOT_SYMMETRIC, SPHX_E_BAD_WEIGHT.  Connectivity is
 * not checked: with c components, eigenvalue 0 has multiplicity c.
 * Requires 1 <= n < 2^31 and nnz < 2^31 (int32 row_ptr) or < 2^62. */
int sphx_graph_create(sphx_handle *h, int64_t n, int64_t nnz,
                      const void *row_ptr, int row_ptr_is_64,
                      const int32_t *col, const void *w, int w_dtype,
                      const int32_t *vwgt, uint32_t flags, sphx_graph **g);
int sphx_graph_destroy(sphx_graph *g);

/* Degree statistics of Sec. 6.1: regular iff max/avg degree <= 10.
 * Pattern degrees (neighbour counts). Synchronises. */
int sphx_graph_info(sphx_handle *h, sphx_graph *g, int *is_regular,
                    int64_t *max_degree, double *avg_degree);

/* --------------------------------------------------------------- workspace */

/* Device bytes needed by sphx_eigensolve (nev), sphx_partition (any K with
 * floor(log2 K) + 1 = nev), sphx_eig_backward (nev) and the operator calls
 * (m <= nev) for this graph and options: an upper bound for all of them. */
int sphx_workspace_size(sphx_handle *h, sphx_graph *g, int nev,
                        const sphx_options *opt, size_t *bytes);
/* Hand the library a device workspace (borrowed, at least 256-byte aligned).
 * A call that needs more than `bytes` allocates (and caches in the handle)
 * its own instead; with a workspace of sphx_workspace_size bytes the calls
 * above allocate no device memory.  NULL detaches it. */
int sphx_set_workspace(sphx_handle *h, void *dev_ptr, size_t bytes);
/* Device bytes the handle currently owns as its own cached workspace (0 when
 * every call so far fit the caller's workspace). */
int sphx_workspace_owned(const sphx_handle *h, size_t *bytes);
/* Free the handle's own cached workspace (synchronises the stream). */
int sphx_workspace_release(sphx_handle *h);

/* -------------------------------------------------------------- operators */

/* Y = L X for the matrix of `problem`: L_C (Eq. 2 with weights) for the
 * combinatorial and generalized problems, L_N = D^-1/2 L_C D^-1/2 (the
 * normalized Laplacian, Sec. 3.2) for SPHX_NORMALIZED.  X and Y are device
 * n x m row-major blocks of dtype SPHX_F32 or SPHX_F64 (1 <= m <= 16), not
 * overlapping.  L_C is summed per row as sum_j w_ij (x_i - x_j), so constant
 * vectors map to exact zeros; L_N scales the rows of X by D^-1/2 (rounded to
 * dtype), applies L_C and scales the result by D^-1/2, and needs every
 * weighted degree > 0 (else SPHX_E_INVALID_ARG). */
int sphx_laplacian_apply(sphx_handle *h, sphx_graph *g, int problem, int m, int dtype,
                         const void *X, void *Y);

/* H = T R for the LOBPCG preconditioner T of `opt` (Sec. 5; Algorithm 1
 * "solve M H = R"): Jacobi h_ic = r_ic / diag(L)_i (d_i; 1 for L_N, a copy);
 * Chebyshev: cheb_degree steps of the Chebyshev iteration for L h = r
 * (generalized: D^-1 L_C h = D^-1 r; normalized: L_N h = r, computed as
 * D^1/2 p(D^-1 L_C) D^-1 (D^1/2 r)) from h = 0 on [hi/cheb_ratio, hi];
 * NONE copies.  R, H: device n x m, dtype. */
int sphx_precond_apply(sphx_handle *h, sphx_graph *g, const sphx_options *opt,
                       int m, int dtype, const void *R, void *H);

/* -------------------------------------------------------------- eigensolve */

/* The nev smallest eigenpairs of L_C x = lambda B x (B = I or D), by LOBPCG
 * (Algorithm 1) with block size nev (Sec. 4).
 * X0: device n x nev initial block (dtype of the precision: F32 for MIXED,
 *     F64 for FP64), read only when opt->init == SPHX_INIT_USER, else NULL.
 * eigvals: host double[nev], ascending.
 * eigvecs: device n x nev (F32 for MIXED, F64 for FP64), B-orthonormal, each
 *     column's largest-magnitude entry (lowest index on ties) positive.
 * stats: host, may be NULL.  1 <= nev <= 32, nev < n.
 * Returns SPHX_NOT_CONVERGED if max_iter was reached first. */
int sphx_eigensolve(sphx_handle *h, sphx_graph *g, int nev,
                    const sphx_options *opt, const void *X0,
                    double *eigvals, void *eigvecs, sphx_stats *stats);

/* ------------------------------------------------------------ split, cut */

/* Part vector from coordinates (Algorithm 2; the multi-jagged split of
 * Sec. 4): one level per prime factor p of K, largest first, level l
 * splitting every section into p children along coordinate l mod ncoord.
 * Members are ordered by (value, vertex id) with -0 == +0; cut j (1 <= j < p)
 * of a section of weight W follows the prefix whose weight C minimises
 * |p C - j W|, the shorter prefix on ties (p = 2: |2 W_lo - W|); part ids are
 * the mixed-radix digits, most significant first (for K = 2^m, branch bits).
 * coords: device, entry (i, c) at coords[i * ld + c], dtype F32 or F64,
 * 1 <= ncoord <= ld.  part: device int32[n].  1 <= K <= min(n, 2^30); the
 * total vertex weight times the largest prime factor of K must stay below
 * 2^62.  NaN coordinates give SPHX_E_INVALID_ARG. */
int sphx_split(sphx_handle *h, sphx_graph *g, const void *coords, int ld,
               int ncoord, int dtype, int K, int32_t *part);

/* Partition quality (Sec. 3.1): cut = Eq. 1 (each undirected edge once),
 * cut2x = 2 cut (the paper's table convention), part weights W_k and
 * imbalance = max_k W_k * K / sum_k W_k.  Sums are exact before a single
 * final rounding (weights must span at most 2^40 in ratio).
 * part: device int32[n] with values in [0, K).  cut, cut2x, imbalance: host
 * (each may be NULL).  part_weights: host int64[K] or NULL. */
int sphx_quality(sphx_handle *h, sphx_graph *g, const int32_t *part, int K,
                 double *cut, double *cut2x, double *imbalance,
                 int64_t *part_weights);

/* sphx_quality with no allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as sphx_quality.
 * Its scratch (cut partials, part-weight counters, flag) is a fixed 1 MiB
 * array in the library's code object, one copy per GPU, resolved when the
 * first handle on that GPU is created; results come back through the
 * handle's pinned host buffer.  No device or host memory is allocated.
 * K above 65536 gives SPHX_E_WORKSPACE.  Every call on one GPU shares that
 * GPU's array and leaves its contents behind (each call clears what it
 * needs): calls that overlap on one GPU (other threads, other streams)
 * race and must not be issued. */
int sphx_quality_noalloc(sphx_handle *h, sphx_graph *g, const int32_t *part, int K,
                         double *cut, double *cut2x, double *imbalance,
                         int64_t *part_weights);

/* Greedy refinement of a K-way partition (Sec. 7 proposes a greedy
 * improvement step for the cut of the spectral partition; balance as in
 * Sec. 3.1: every part weight W_k below W_avg (1 + eps), eps = 0.01 in the
 * experiments of Sec. 6).  One pass:
 *  1. each vertex v of degree 1..2048 in part a targets the neighbour part
 *     t != a with the largest edge weight conn(v, t) from v (smallest t on
 *     ties); gain g = conn(v, t) - conn(v, a); candidates have g > 0;
 *  2. candidates are ranked by (g descending, id ascending); v remains a
 *     mover when its gain, with every higher-ranked candidate at its target,
 *     stays positive;
 *  3. the movers into part p, in increasing id, are accepted while W_p plus
 *     their cumulative weight stays <= C, C the largest integer below
 *     (W / K)(1 + eps) (departures are not credited);
 *  4. accepted movers take their targets.
 * A pass is kept only when the exact cut drops; passes repeat while it does,
 * at most max_passes.  All sums are exact (float weights in 128-bit fixed
 * point, ratio of weights at most 2^40), so the result does not depend on
 * the order of the additions.
 * part: device int32[n] with values in [0, K), refined in place.
 * eps >= 0.  cut, imbalance (host, may be NULL): of the returned partition,
 * as in sphx_quality.  passes (host, may be NULL): passes kept.  moves
 * (host, may be NULL): accepted moves over the kept passes.
 * Warm-start repartitioning (Sec. 1: partitions recomputed as the data
 * changes, on the accelerator) passes the previous eigenvectors as X0 with
 * SPHX_INIT_USER to sphx_partition and may refine its part vector here. */
int sphx_refine(sphx_handle *h, sphx_graph *g, int K, int32_t *part,
                double eps, int max_passes, double *cut, double *imbalance,
                int *passes, int64_t *moves);

/* Algorithm 2 end to end: nev = d = floor(log2 K) + 1 eigenpairs, the
 * embedding = eigenvector columns 1..d-1 (the trivial one dropped), the
 * split into any 2 <= K <= n parts and its quality.  eigvals host double[d]; eigvecs device n x d (as
 * in sphx_eigensolve; may be NULL to use workspace); part device int32[n];
 * cut, imbalance host (may be NULL). */
int sphx_partition(sphx_handle *h, sphx_graph *g, int K, const sphx_options *opt,
                   const void *X0, double *eigvals, void *eigvecs,
                   int32_t *part, double *cut, double *imbalance,
                   sphx_stats *stats);

/* GMRES polynomial (Sec. 5.2).  The preconditioner is p(A) with p of degree
 * k the polynomial of the GMRES residual polynomial
 * pi(x) = prod_{i=1}^{k+1} (1 - x / theta_i) = 1 - x p(x) of a (k+1)-step
 * Krylov process from a start vector b; A = L_C (combinatorial), D^-1 L_C
 * applied to D^-1 r (generalized), L_N (normalized).  b is made orthogonal
 * (in the problem's B-inner product) to the trivial eigenvector first.
 *
 * sphx_poly_roots: the roots theta_i (harmonic Ritz values of a Lanczos
 * process with full reorthogonalisation in FP64), modified Leja order (the
 * largest first, then each maximising the product of distances to those
 * before).  b: device FP64[n] in the problem's variables (y for L_N).
 * roots: host double[degree + 1]; *nroots = degree + 1, or fewer when the
 * Krylov space becomes invariant.  1 <= degree <= 47.
 * The solver (SPHX_PRECOND_GMRES) draws b from its seed. */
int sphx_poly_roots(sphx_handle *h, sphx_graph *g, int problem, int degree,
                    const double *b, double *roots, int *nroots);
/* H = p(A) R (generalized: p(D^-1 L_C) D^-1 R) for the polynomial with the
 * given nonzero roots (host, applied in the given order): nroots - 1
 * Laplacian products, p(A) v = sum_i pi_{i-1}(A) v / theta_i.  R, H: device
 * n x m row-major of dtype F32/F64, 1 <= m <= 16, not overlapping. */
int sphx_poly_apply(sphx_handle *h, sphx_graph *g, int problem, int nroots,
                    const double *roots, int m, int dtype, const void *R, void *H);

/* ---------------------------------------------------------------- adjoint */

/* Gradient of a loss l(lambda, V) with respect to the edge weights, through
 * the eigenpairs of L_C x = lambda B x (weighted Laplacian, Sec. 3.2).
 * Inputs: eigvals host double[nev] (simple eigenvalues), eigvecs device F64
 * n x nev (B-orthonormal eigenvectors, e.g. from sphx_eigensolve in FP64),
 * g_vals host double[nev] (dl/dlambda, NULL = 0), g_vecs device F64 n x nev
 * (dl/dV, NULL = 0).  Output grad_w: device F64[nnz]; both stored directions
 * of an undirected edge receive dl/dw_e for that edge.
 * Eigenvector terms inside the block use the computed pairs; the rest of the
 * spectrum enters through mu_k solving (L - lambda_k B) mu_k =
 * g_k - B V V^T g_k with V^T B mu_k = 0 (projected, Jacobi-preconditioned
 * conjugate gradients, all columns at once, at most cg_max_iter steps, until
 * every column's residual r satisfies sqrt(r^T J r) <= cg_tol sqrt(f^T J f),
 * f the right-hand side and J the inverted diagonal of L - lambda_k B).  The
 * solve needs lambda_k separated from the eigenvalues outside the block.
 * For SPHX_NORMALIZED (eigvecs y = D^1/2 x of unit 2-norm) the gradient is
 * the generalized one for x with dl/dx = D^1/2 dl/dy, plus, on each edge
 * {i, j}, t_i + t_j with t_i = sum_k (dl/dy_ik) y_ik / (2 d_i) from the
 * dependence of D^1/2 on w.
 * The graph must carry F64 weights or unit weights.
 * Returns SPHX_NOT_CONVERGED if a CG solve stopped at cg_max_iter (or lost
 * positive curvature); grad_w then holds the gradient of the last iterate. */
int sphx_eig_backward(sphx_handle *h, sphx_graph *g, int problem, int nev,
                      const double *eigvals, const void *eigvecs,
                      const double *g_vals, const void *g_vecs,
                      double cg_tol, int cg_max_iter, void *grad_w);
/* CG steps of the handle's last sphx_eig_backward and the largest final
 * relative residual over its columns (0 when no eigenvector term). */
int sphx_backward_info(const sphx_handle *h, int *cg_iterations,
                       double *cg_rel_residual);

/* ------------------------------------------------------- kernel test hooks */
/* The dense kernels of one LOBPCG iteration (Algorithm 1: the block Gram
 * products and RR(S, nev)), exposed so that tests can check them alone.
 *
 * sphx_block_gram: Gram matrices of the basis S = [X, H_a, P_a] (a = the nact
 * columns listed in act, host int32; H_a only if use_h, P_a only if use_p):
 * GA = S^T [LX, LH_a, LP_a] and GB = S^T B S with B = diag(bdiag) (device
 * double[n]) or I (NULL).  X, LX, H, LH, P, LP: device n x m blocks of dtype
 * (unused ones may be NULL).  GA, GB: host double[w*w], w = m + nact*(use_h +
 * use_p), row-major; accumulated in FP64 on the matrix cores.
 *
 * sphx_rayleigh_ritz: Ritz pairs of the w x w pencil (GA, GB) (host, only the
 * upper triangle i <= j is read), the m smallest: Y host double[w*m]
 * (row-major, columns GB-orthonormal), theta host double[m] ascending.
 * Basis columns from p_begin on are dropped if the pencil is numerically
 * rank deficient (kept < m); kept and breakdown (host int) report the rank
 * used and whether fewer than m directions remained. */
int sphx_block_gram(sphx_handle *h, int64_t n, int m, int dtype, const void *X,
                    const void *LX, const void *H, const void *LH, const void *P,
                    const void *LP, int nact, const int32_t *act, int use_h,
                    int use_p, const double *bdiag, double *GA, double *GB);
int sphx_rayleigh_ritz(sphx_handle *h, int m, int w, int p_begin,
                       double drop_tol, const double *GA, const double *GB,
                       double *Y, double *theta, int *kept, int *breakdown);

#ifdef __cplusplus
}
#endif
#endif /* SPHYNX_H */
