// Shared definitions of the HIP implementation (product path).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/nep.h"

namespace nep {

// ---------------------------------------------------------------------------
// Complex scalar of precision P (interleaved re, im), usable on host/device.
// ---------------------------------------------------------------------------
template <typename P>
struct cx {
  P re, im;
};
using c64 = cx<float>;
using c128 = cx<double>;

template <typename P>
__host__ __device__ __forceinline__ cx<P> mk(P r, P i) { return cx<P>{r, i}; }
template <typename P>
__host__ __device__ __forceinline__ cx<P> operator+(cx<P> a, cx<P> b) { return {a.re + b.re, a.im + b.im}; }
template <typename P>
__host__ __device__ __forceinline__ cx<P> operator-(cx<P> a, cx<P> b) { return {a.re - b.re, a.im - b.im}; }
template <typename P>
__host__ __device__ __forceinline__ cx<P> operator*(cx<P> a, cx<P> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename P>
__host__ __device__ __forceinline__ cx<P> operator*(P s, cx<P> b) { return {s * b.re, s * b.im}; }
template <typename P>
__host__ __device__ __forceinline__ cx<P> operator-(cx<P> a) { return {-a.re, -a.im}; }
template <typename P>
__host__ __device__ __forceinline__ cx<P> conj(cx<P> a) { return {a.re, -a.im}; }
__host__ __device__ __forceinline__ float pfma(float a, float b, float c) { return fmaf(a, b, c); }
__host__ __device__ __forceinline__ double pfma(double a, double b, double c) { return fma(a, b, c); }
// a - b*c  (the update step of every elimination / substitution)
template <typename P>
__host__ __device__ __forceinline__ cx<P> fms(cx<P> a, cx<P> b, cx<P> c) {
  return {pfma(-b.re, c.re, pfma(b.im, c.im, a.re)), pfma(-b.re, c.im, pfma(-b.im, c.re, a.im))};
}
// acc + a*b as four fused multiply-adds
template <typename P>
__host__ __device__ __forceinline__ cx<P> cmac(cx<P> acc, cx<P> a, cx<P> b) {
  return {pfma(a.re, b.re, pfma(-a.im, b.im, acc.re)), pfma(a.re, b.im, pfma(a.im, b.re, acc.im))};
}
// c ? a : b on values, component by component.  (A conditional between two
// complex lvalues would select their addresses, which keeps register arrays
// from being promoted to registers.)
template <typename P>
__host__ __device__ __forceinline__ cx<P> csel(bool c, cx<P> a, cx<P> b) {
  return {c ? a.re : b.re, c ? a.im : b.im};
}
template <typename P>
__host__ __device__ __forceinline__ P abs1(cx<P> a) {  // |Re| + |Im|, +0 for signed zeros
  return std::fabs(a.re) + std::fabs(a.im);
}
template <typename P>
__host__ __device__ __forceinline__ P norm2(cx<P> a) { return a.re * a.re + a.im * a.im; }
// Maximum that keeps NaN (fmax drops it): a norm taken over values that hold a
// NaN must come out NaN, so that tests on it can see the failure.
__host__ __device__ __forceinline__ double nanmax(double a, double b) { return (a > b || a != a) ? a : b; }

// Reciprocal 1/a computed in double and rounded once to P.
template <typename P>
__host__ __device__ __forceinline__ cx<P> recip(cx<P> a) {
  double ar = a.re, ai = a.im;
  double d = ar * ar + ai * ai;
  if (d == 0.0) return {P(0), P(0)};
  return {P(ar / d), P(-ai / d)};
}
// 1/a in FP32: a is scaled by a power of two to |a| ~ 1 (exact), the
// hardware reciprocal of |a|^2 is refined by one Newton step (about one
// ulp), and 1/a = conj(a)/|a|^2 is scaled back.  Zero maps to zero.
__device__ __forceinline__ c64 recip_f32(c64 a) {
  const float m = fmaxf(fabsf(a.re), fabsf(a.im));
  if (m == 0.f) return {0.f, 0.f};
  const int e = __builtin_amdgcn_frexp_expf(m);
  const float xr = ldexpf(a.re, -e), xi = ldexpf(a.im, -e);
  const float d = xr * xr + xi * xi;
  float r = __builtin_amdgcn_rcpf(d);
  r = r * (2.f - d * r);
  return {ldexpf(xr * r, -e), ldexpf(-xi * r, -e)};
}
// a / b in double precision.
__host__ __device__ __forceinline__ c128 cdiv(c128 a, c128 b) {
  // Smith's scaling to avoid overflow
  double br = b.re, bi = b.im;
  if ((br < 0 ? -br : br) >= (bi < 0 ? -bi : bi)) {
    double r = bi / br, den = br + bi * r;
    return {(a.re + a.im * r) / den, (a.im - a.re * r) / den};
  } else {
    double r = br / bi, den = bi + br * r;
    return {(a.re * r + a.im) / den, (a.im * r - a.re) / den};
  }
}

template <typename P>
struct Prec;
template <>
struct Prec<float> {
  static constexpr int id = NEP_PREC_C32_IR64;
};
template <>
struct Prec<double> {
  static constexpr int id = NEP_PREC_FP64;
};

__host__ __device__ __forceinline__ c64 to64(c128 a) { return {float(a.re), float(a.im)}; }
__host__ __device__ __forceinline__ c128 to128(c64 a) { return {double(a.re), double(a.im)}; }
template <typename P>
__host__ __device__ __forceinline__ cx<P> cvt(c128 a);
template <>
__host__ __device__ __forceinline__ c64 cvt<float>(c128 a) { return to64(a); }
template <>
__host__ __device__ __forceinline__ c128 cvt<double>(c128 a) { return a; }

// ---------------------------------------------------------------------------
// Per-matrix descriptor of a (possibly ragged) batch of n x n factor blocks.
// Factor blocks are stored row-major with leading dimension ld; row_at maps a
// logical (pivoted) row to its physical row, so pivoting never moves data.
// ---------------------------------------------------------------------------
struct MatDesc {
  int n;          // size
  int ld;         // row stride (elements)
  long long offT; // element offset of the block in the factor buffer
  int offRow;     // offset of row_at (n ints) in the row buffer
  int node;       // global node index (problem-major) for Y/R addressing
};

// Work-table entry: prefix sums of tiles over the active matrices of a step.
struct StepTable {
  int nact;       // active matrices (prefix of the size-sorted list)
  int offPrefix;  // offset into the prefix buffer (nact+1 ints)
  int total;      // total tiles of the step
};

// Error reporting -----------------------------------------------------------
void set_error(const char* fmt, ...);
const char* last_error();

#define NEP_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) {                                                  \
      ::nep::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                       __FILE__, __LINE__);                                  \
      return NEP_ERR_DEVICE;                                                 \
    }                                                                        \
  } while (0)

#define NEP_CHECK(cond, code, ...) \
  do {                             \
    if (!(cond)) {                 \
      ::nep::set_error(__VA_ARGS__); \
      return (code);               \
    }                              \
  } while (0)

#define NEP_TRY(expr)            \
  do {                           \
    nep_status s_ = (expr);      \
    if (s_ != NEP_OK) return s_; \
  } while (0)

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
inline long long ceil_div_ll(long long a, long long b) { return (a + b - 1) / b; }

// Device binary search: largest k with prefix[k] <= x (prefix[0] = 0).
__device__ __forceinline__ int find_slot(const int* prefix, int cnt, int x) {
  int lo = 0, hi = cnt;  // prefix[lo] <= x < prefix[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (prefix[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// XCD-aware work-group order: consecutive virtual ids run on the same XCD
// (hardware dispatches work-group i to XCD i % 8), so tiles of one matrix
// share an L2.  Returns -1 for the padding groups of the last round.
__device__ __forceinline__ int xcd_remap(int bid, int grid, int total) {
  const int per = grid >> 3;  // grid is a multiple of 8
  int v = (bid & 7) * per + (bid >> 3);
  return v < total ? v : -1;
}
inline int xcd_grid(int total) { return ((total + 7) / 8) * 8; }

}  // namespace nep
