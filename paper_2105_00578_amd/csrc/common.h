// Internal definitions shared by the host driver and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <type_traits>
#include <vector>

#include "sphynx.h"

namespace sphx {

constexpr int kMaxNev = 16;              // block size limit (Rayleigh-Ritz <= 48)
constexpr int kMaxW = 3 * kMaxNev;       // [X, H, P] width
constexpr int kWave = 64;

struct Unit {};                          // marker type: unit edge weights

// Column map: lane c of a row group works on column col[c] of an ld-wide row.
struct ColMap {
  int count;
  int col[kMaxNev];
};

// Device-side LOBPCG status, mirrored to pinned host memory every iteration.
struct DevStatus {
  int nact;              // unconverged columns
  int act[kMaxNev];      // their indices, ascending
  int nconv;             // converged columns
  int kept;              // Rayleigh-Ritz basis rank
  int restarted;         // Rayleigh-Ritz dropped the P block this iteration
  int breakdown;         // rank < nev even without P
  int pad[2];
  double rho[kMaxNev];
  double theta[kMaxNev];
};

}  // namespace sphx

namespace sphx {
// Phase timing with HIP events (recorded around launches, read at the end).
enum Phase { PH_SETUP, PH_SPMM, PH_PRECOND, PH_GRAM, PH_RR, PH_UPDATE, PH_SPLIT,
             PH_QUALITY, PH_OTHER, PH_COUNT };
struct PhaseLog {
  struct Rec {
    int phase;
    double bytes;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t next = 0;
  bool on = false;
  hipEvent_t take() {
    if (next == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[next++];
  }
  void reset() {
    recs.clear();
    next = 0;
  }
  // begin/end a timed launch group on stream s
  int begin(int phase, double bytes, hipStream_t s) {
    if (!on) return -1;
    Rec r{phase, bytes, take(), take()};
    if (!r.a || !r.b) return -1;
    (void)hipEventRecord(r.a, s);
    recs.push_back(r);
    return (int)recs.size() - 1;
  }
  void end(int id, hipStream_t s) {
    if (id >= 0) (void)hipEventRecord(recs[id].b, s);
  }
  // a launch group whose kernels record the two events themselves; false
  // when timing is off
  bool begin_stamped(int phase, double bytes, hipEvent_t *a, hipEvent_t *b) {
    if (!on) return false;
    Rec r{phase, bytes, take(), take()};
    if (!r.a || !r.b) return false;
    recs.push_back(r);
    *a = r.a;
    *b = r.b;
    return true;
  }
  ~PhaseLog() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};
}  // namespace sphx

namespace sphx {
constexpr size_t kPinnedSmallBytes = 65536;
}  // namespace sphx

struct sphx_handle {
  sphx::PhaseLog plog;
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  void *ws_user = nullptr;
  size_t ws_user_bytes = 0;
  void *ws_own = nullptr;
  size_t ws_own_bytes = 0;
  int timing = 0;
  sphx::DevStatus *pinned_status = nullptr;   // hipHostMalloc'ed
  void *pinned_small = nullptr;               // kPinnedSmallBytes of pinned host
                                              // memory for small D2H reads
  int32_t *flags_dev = nullptr;               // 256 device bytes: validation flags
  int last_cg_iters = 0;                      // of the last sphx_eig_backward
  double last_cg_relres = 0.0;
};

struct sphx_graph {
  sphx_handle *h = nullptr;
  int64_t n = 0, nnz = 0;
  const void *rowptr = nullptr;
  int rp64 = 0;
  const int32_t *col = nullptr;
  const void *w = nullptr;
  int wdt = SPHX_UNIT;
  const int32_t *vwgt = nullptr;
  // cached statistics (computed on first use)
  int stats_valid = 0;
  int64_t max_deg = 0;
  int64_t sum_deg = 0;
  double max_wdeg = 0.0;
  double wmin = 0.0, wmax = 0.0;   // edge weight range (weighted graphs)
  int wrange_valid = 0;            // wmin / wmax computed
};

// ----------------------------------------------------------------- helpers
namespace sphx {

inline int set_err(sphx_handle *h, int code, const std::string &msg) {
  if (h) h->err = msg;
  return code;
}

#define SPHX_HIP(h, call)                                                    \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      return ::sphx::set_err((h), SPHX_E_HIP,                                \
                             std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define SPHX_TRY(expr)              \
  do {                              \
    int s_ = (expr);                \
    if (s_ < 0) return s_;          \
  } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over a workspace region.
struct Arena {
  char *base = nullptr;
  size_t cap = 0, off = 0;
  bool count_only = false;
  template <class T>
  T *take(size_t count) {
    off = align_up(off, 256);
    T *p = count_only ? nullptr : reinterpret_cast<T *>(base + off);
    off += count * sizeof(T);
    return p;
  }
};

// Launch helper: grid size for n items with `per_block` items per block,
// capped so that grid-stride loops cover the rest.
inline unsigned grid_for(int64_t n, int64_t per_block, int64_t cap = 1 << 20) {
  int64_t g = ceil_div(n, per_block);
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<unsigned>(g);
}

}  // namespace sphx
