// Scalar functions with the FN semantics of Section 3.2.2, evaluated in
// complex FP64 on the device: beta * g(alpha * z) with g rational (Horner,
// coefficients highest degree first), exp, log, principal sqrt, inverse sqrt,
// phi_k, or a combination (add, mul, div, compose) of two functions.
#pragma once

#include "common.hpp"

namespace nep {

constexpr int kMaxFnNodes = 64;
constexpr int kMaxFnDepth = 4;
constexpr int kMaxCoeffs = 33;

// Flattened FN tree node (device-resident, built at handle creation).
struct FnNode {
  int type;        // nep_fn_type
  c128 alpha, beta;
  int num_off, nnum, den_off, nden;  // into the coefficient array
  int phi_k;
  int op;          // combine op
  int a, b;        // child node indices (combine)
};

// Bits reported by the evaluators.
enum : int { kFnBadCut = 1, kFnBadPole = 2 };

__device__ __forceinline__ c128 zexp(c128 x) {
  double s, c;
  sincos(x.im, &s, &c);
  double e = exp(x.re);
  return {e * c, e * s};
}

// Principal square root; its cut is the non-positive real axis.
__device__ __forceinline__ c128 zsqrt(c128 x) {
  double r = hypot(x.re, x.im);
  if (r == 0.0) return {0.0, 0.0};
  if (x.re >= 0.0) {
    double t = sqrt(0.5 * (r + x.re));
    return {t, x.im / (2.0 * t)};
  }
  double t = sqrt(0.5 * (r - x.re));
  return {fabs(x.im) / (2.0 * t), copysign(t, x.im)};
}

__device__ __forceinline__ c128 zlog(c128 x) { return {log(hypot(x.re, x.im)), atan2(x.im, x.re)}; }

__device__ __forceinline__ bool on_cut(c128 x) { return x.im == 0.0 && x.re <= 0.0; }

// phi_k(x) = sum_m x^m/(m+k)!  (summed directly for |x| < 1/2), otherwise the
// recurrence phi_k = (phi_{k-1} - 1/(k-1)!)/x started from e^x.
__device__ inline c128 zphi(int k, c128 x) {
  double ax = hypot(x.re, x.im);
  if (ax < 0.5) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    c128 term = {1.0 / f, 0.0}, s = {0.0, 0.0};
    for (int m = 0; m < 40; ++m) {
      s = s + term;
      term = (1.0 / double(m + k + 1)) * (term * x);
    }
    return s;
  }
  c128 v = zexp(x);
  double fact = 1.0;  // (j-1)!
  for (int j = 1; j <= k; ++j) {
    if (j > 1) fact *= (j - 1);
    v = cdiv(v - c128{1.0 / fact, 0.0}, x);
  }
  return v;
}

__device__ inline c128 horner(const c128* c, int cnt, c128 x) {
  c128 acc = {0.0, 0.0};
  for (int i = 0; i < cnt; ++i) acc = acc * x + c[i];
  return acc;
}

// Depth-bounded evaluation (compile-time recursion, no device call stack).
template <int D>
struct FnEval {
  __device__ static c128 run(const FnNode* nd, const c128* cf, int k, c128 z, int& bad) {
    const FnNode f = nd[k];
    c128 x = f.alpha * z;
    c128 g;
    switch (f.type) {
      case NEP_FN_RATIONAL: {
        g = horner(cf + f.num_off, f.nnum, x);
        if (f.nden > 0) {
          c128 q = horner(cf + f.den_off, f.nden, x);
          if (q.re == 0.0 && q.im == 0.0) { bad |= kFnBadPole; return {0.0, 0.0}; }
          g = cdiv(g, q);
        }
        break;
      }
      case NEP_FN_EXP: g = zexp(x); break;
      case NEP_FN_LOG:
        if (on_cut(x)) { bad |= kFnBadCut; return {0.0, 0.0}; }
        g = zlog(x);
        break;
      case NEP_FN_SQRT:
        if (on_cut(x)) { bad |= kFnBadCut; return {0.0, 0.0}; }
        g = zsqrt(x);
        break;
      case NEP_FN_INVSQRT:
        if (on_cut(x)) { bad |= kFnBadCut; return {0.0, 0.0}; }
        g = cdiv(c128{1.0, 0.0}, zsqrt(x));
        break;
      case NEP_FN_PHI: g = zphi(f.phi_k, x); break;
      case NEP_FN_COMBINE: {
        c128 a = FnEval<D - 1>::run(nd, cf, f.a, x, bad);
        if (f.op == NEP_COMB_COMPOSE) {
          g = FnEval<D - 1>::run(nd, cf, f.b, a, bad);
        } else {
          c128 b = FnEval<D - 1>::run(nd, cf, f.b, x, bad);
          if (f.op == NEP_COMB_ADD) g = a + b;
          else if (f.op == NEP_COMB_MUL) g = a * b;
          else {
            if (b.re == 0.0 && b.im == 0.0) { bad |= kFnBadPole; return {0.0, 0.0}; }
            g = cdiv(a, b);
          }
        }
        break;
      }
      default: g = {0.0, 0.0}; bad |= kFnBadPole;
    }
    return f.beta * g;
  }
};
template <>
struct FnEval<0> {
  __device__ static c128 run(const FnNode*, const c128*, int, c128, int& bad) {
    bad |= kFnBadPole;
    return {0.0, 0.0};
  }
};

__device__ __forceinline__ c128 fn_eval(const FnNode* nd, const c128* cf, int root, c128 z, int& bad) {
  return FnEval<kMaxFnDepth>::run(nd, cf, root, z, bad);
}

// Value and derivative (the derivative of FNEvaluateDerivative, Section 3.2.2):
// f(z) = beta g(alpha z) has f'(z) = alpha beta g'(alpha z); the rational
// part carries p and p' through one Horner pass (p' by synthetic division),
// g' = (p' q - p q')/q^2; exp' = exp, log' = 1/x, sqrt' = 1/(2 sqrt x),
// (x^{-1/2})' = -x^{-1/2}/(2x); phi_k' = phi_k - k phi_{k+1} (termwise from the
// series sum_m x^m/(m+k)!); sum, product, quotient and chain rules for the
// combinations.
__device__ inline void horner_d(const c128* c, int cnt, c128 x, c128& p, c128& dp) {
  p = {0.0, 0.0};
  dp = {0.0, 0.0};
  for (int i = 0; i < cnt; ++i) {
    dp = dp * x + p;
    p = p * x + c[i];
  }
}

template <int D>
struct FnEvalD {
  __device__ static c128 run(const FnNode* nd, const c128* cf, int k, c128 z, int& bad, c128& dz) {
    const FnNode f = nd[k];
    c128 x = f.alpha * z;
    c128 g, dg;  // g(x) and g'(x)
    switch (f.type) {
      case NEP_FN_RATIONAL: {
        c128 p, dp;
        horner_d(cf + f.num_off, f.nnum, x, p, dp);
        if (f.nden > 0) {
          c128 q, dq;
          horner_d(cf + f.den_off, f.nden, x, q, dq);
          if (q.re == 0.0 && q.im == 0.0) { bad |= kFnBadPole; dz = {0.0, 0.0}; return {0.0, 0.0}; }
          g = cdiv(p, q);
          dg = cdiv(dp - g * dq, q);
        } else {
          g = p;
          dg = dp;
        }
        break;
      }
      case NEP_FN_EXP: g = zexp(x); dg = g; break;
      case NEP_FN_LOG:
        if (on_cut(x)) { bad |= kFnBadCut; dz = {0.0, 0.0}; return {0.0, 0.0}; }
        g = zlog(x);
        dg = cdiv(c128{1.0, 0.0}, x);
        break;
      case NEP_FN_SQRT:
        if (on_cut(x)) { bad |= kFnBadCut; dz = {0.0, 0.0}; return {0.0, 0.0}; }
        g = zsqrt(x);
        dg = cdiv(c128{0.5, 0.0}, g);
        break;
      case NEP_FN_INVSQRT:
        if (on_cut(x)) { bad |= kFnBadCut; dz = {0.0, 0.0}; return {0.0, 0.0}; }
        g = cdiv(c128{1.0, 0.0}, zsqrt(x));
        dg = cdiv(-0.5 * g, x);
        break;
      case NEP_FN_PHI:
        g = zphi(f.phi_k, x);
        dg = g - double(f.phi_k) * zphi(f.phi_k + 1, x);
        break;
      case NEP_FN_COMBINE: {
        c128 da, db;
        c128 a = FnEvalD<D - 1>::run(nd, cf, f.a, x, bad, da);
        if (f.op == NEP_COMB_COMPOSE) {
          g = FnEvalD<D - 1>::run(nd, cf, f.b, a, bad, db);
          dg = db * da;
        } else {
          c128 b = FnEvalD<D - 1>::run(nd, cf, f.b, x, bad, db);
          if (f.op == NEP_COMB_ADD) {
            g = a + b;
            dg = da + db;
          } else if (f.op == NEP_COMB_MUL) {
            g = a * b;
            dg = da * b + a * db;
          } else {
            if (b.re == 0.0 && b.im == 0.0) { bad |= kFnBadPole; dz = {0.0, 0.0}; return {0.0, 0.0}; }
            g = cdiv(a, b);
            dg = cdiv(da - g * db, b);
          }
        }
        break;
      }
      default: g = {0.0, 0.0}; dg = {0.0, 0.0}; bad |= kFnBadPole;
    }
    dz = f.alpha * (f.beta * dg);
    return f.beta * g;
  }
};
template <>
struct FnEvalD<0> {
  __device__ static c128 run(const FnNode*, const c128*, int, c128, int& bad, c128& dz) {
    bad |= kFnBadPole;
    dz = {0.0, 0.0};
    return {0.0, 0.0};
  }
};

__device__ __forceinline__ c128 fn_eval_d(const FnNode* nd, const c128* cf, int root, c128 z, int& bad, c128& dz) {
  return FnEvalD<kMaxFnDepth>::run(nd, cf, root, z, bad, dz);
}

}  // namespace nep
