// Exact summation of positive floating-point weights in 128-bit fixed point.
//
// With e0 the exponent of the last mantissa bit of the smallest weight, every
// weight is an integer multiple of 2^e0.  Sums of such integers are exact in
// 128 bits (for weight ratios up to 2^40 and up to 2^31 terms), and a single
// correctly rounded conversion (to nearest, ties to even) gives the double
// nearest to the exact sum, independent of the order of the additions.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

namespace sphx {

struct U128 {
  unsigned long long lo, hi;
};

__host__ __device__ __forceinline__ void add128(U128 &a, unsigned long long lo,
                                                unsigned long long hi) {
  unsigned long long l = a.lo + lo;
  a.hi += hi + (l < a.lo ? 1ull : 0ull);
  a.lo = l;
}

// e0 for weights of type WT whose minimum is wmin (> 0)
template <typename WT>
inline int fixed_exponent(double wmin) {
  int ex;
  std::frexp(wmin, &ex);
  return ex - (std::is_same_v<WT, float> ? 24 : 53);
}

// w / 2^e0 as a 128-bit integer (w > 0 finite, 2^e0 divides w)
template <typename WT>
__device__ __forceinline__ void fixed_of(WT w, int e0, unsigned long long &lo,
                                         unsigned long long &hi) {
  int ex;
  double f = frexp(double(w), &ex);   // w = f 2^ex, f in [0.5, 1)
  constexpr int MB = std::is_same_v<WT, float> ? 24 : 53;
  unsigned long long M = (unsigned long long)ldexp(f, MB);   // exact
  int sh = ex - MB - e0;                                      // >= 0
  if (sh <= 0) { lo = M >> (-sh); hi = 0; }                   // sh < 0 only if misuse
  else if (sh < 64) { lo = M << sh; hi = M >> (64 - sh); }
  else { lo = 0; hi = M << (sh - 64); }
}

// (hi, lo) * 2^e0 rounded to the nearest double, ties to even
__host__ __device__ inline double fixed_to_double(U128 v, int e0) {
  if (v.hi == 0 && v.lo < (1ull << 53)) return ldexp((double)v.lo, e0);
  int nb;
  if (v.hi) {
    int lz = 0;
    for (unsigned long long t = v.hi; !(t & 0x8000000000000000ull); t <<= 1) ++lz;
    nb = 128 - lz;
  } else {
    int lz = 0;
    for (unsigned long long t = v.lo; !(t & 0x8000000000000000ull); t <<= 1) ++lz;
    nb = 64 - lz;
  }
  int sh = nb - 53;   // > 0
  // top = v >> sh (53 bits), rem = v mod 2^sh
  unsigned long long top, rem_hi, rem_lo;
  if (sh < 64) {
    top = (v.lo >> sh) | (sh ? (v.hi << (64 - sh)) : 0ull);
    rem_hi = 0;
    rem_lo = v.lo & ((1ull << sh) - 1);
  } else {
    top = v.hi >> (sh - 64);
    rem_hi = (sh == 64) ? 0ull : (v.hi & ((1ull << (sh - 64)) - 1));
    rem_lo = v.lo;
  }
  // half = 2^(sh-1)
  unsigned long long half_hi = 0, half_lo = 0;
  if (sh - 1 < 64) half_lo = 1ull << (sh - 1);
  else half_hi = 1ull << (sh - 1 - 64);
  bool gt = rem_hi > half_hi || (rem_hi == half_hi && rem_lo > half_lo);
  bool eq = rem_hi == half_hi && rem_lo == half_lo;
  if (gt || (eq && (top & 1ull))) top += 1;
  return ldexp((double)top, sh + e0);
}

}  // namespace sphx
