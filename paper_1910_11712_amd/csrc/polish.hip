// Eigenpair polish by residual inverse iteration (Section 4.1, Algorithm
// "RII", eqs. (rii) and (rii-scalar)), in FP64 on the device, for many pairs
// at once.
//
// For a pair (lambda, x) the target is sigma = lambda (the paper's option of
// updating sigma, taken once), T(sigma) is assembled and factored in complex
// FP64 on the matrix cores (one plan over every pair's shift), and each outer
// step is:
//   scalar equation  x^* T(sigma)^{-1} T(z) x = sum_i f_i(z) (x^* s_i) = 0 with
//                    s_i = T(sigma)^{-1} A_i x (the split form turns the
//                    equation into l scalars; one solve launch with l
//                    right-hand sides per pair), solved by Newton's method
//                    with the derivatives f_i' (mu = g/g', stop when
//                    |mu| < sqrt(eps) |z|);
//   residual         r = T(lambda) x = sum_i f_i(lambda) A_i x and eta(x, lambda);
//   correction       v = T(sigma)^{-1} r by a second solve, x <- (x - v)/||x - v||.
// The correction is solved from r itself: sigma lies near the eigenvalue, so
// the s_i are large (~ 1/|sigma - lambda|) while v is small, and forming v as
// sum_i f_i(lambda) s_i would cancel away its digits.  The scalar equation
// does not suffer from this: g and g' carry the same large factor.  The loop
// stops for a pair when eta < tol.
#include <algorithm>
#include <cmath>
#include <vector>

#include "dense.hpp"
#include "handle.hpp"

namespace nep {

constexpr int kPolishNewton = 50;  // scalar Newton steps per outer step, at most

// R[(row*P + q)*ell + i] = (A_i x_q)[row]: one group per (64 rows, 16 pairs,
// term), A tile staged through LDS.
__global__ __launch_bounds__(256) void k_term_apply(int n, int ell, int P, const double* const* __restrict__ A,
                                                    const int* __restrict__ cplx, const c128* __restrict__ X,
                                                    c128* __restrict__ R) {
  __shared__ c128 As[64][33];
  __shared__ c128 Xs[32][17];
  const int row0 = blockIdx.x * 64, q0 = blockIdx.y * 16, i = blockIdx.z;
  const int tr = threadIdx.x >> 2, tq = (threadIdx.x & 3) * 4;
  c128 acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  for (int s0 = 0; s0 < n; s0 += 32) {
    for (int e = threadIdx.x; e < 64 * 32; e += 256) {
      const int r = e >> 5, s = e & 31;
      const int gr = row0 + r, gs = s0 + s;
      c128 a = {0.0, 0.0};
      if (gr < n && gs < n) {
        if (cplx[i]) a = reinterpret_cast<const c128*>(A[i])[(long long)gr * n + gs];
        else a.re = A[i][(long long)gr * n + gs];
      }
      As[r][s] = a;
    }
    for (int e = threadIdx.x; e < 32 * 16; e += 256) {
      const int s = e >> 4, q = e & 15;
      const int gs = s0 + s, gq = q0 + q;
      Xs[s][q] = (gs < n && gq < P) ? X[(long long)gq * n + gs] : c128{0.0, 0.0};
    }
    __syncthreads();
    for (int s = 0; s < 32; ++s) {
      const c128 a = As[tr][s];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = acc[u] + a * Xs[s][tq + u];
    }
    __syncthreads();
  }
  const int gr = row0 + tr;
  if (gr < n)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int gq = q0 + tq + u;
      if (gq < P) R[((long long)gr * P + gq) * ell + i] = acc[u];
    }
}

hipError_t term_apply(int n, int ell, int P, const double* const* A, const int* cplx, const c128* X, c128* R,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_term_apply, dim3(ceil_div(n, 64), ceil_div(P, 16), ell), dim3(256), 0, st, n, ell, P, A, cplx,
                     X, R);
  return hipGetLastError();
}

__device__ __forceinline__ c128 block_sum256(c128 v, c128* red) {
  for (int o = 32; o >= 1; o >>= 1) {
    v.re += __shfl_xor(v.re, o, 64);
    v.im += __shfl_xor(v.im, o, 64);
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// d[q*ell + i] = x_q^* s_{q,i} with s = Y (layout of R); one group per pair.
__global__ __launch_bounds__(256) void k_polish_dots(int n, int ell, int P, const c128* __restrict__ X,
                                                     const c128* __restrict__ Y, c128* __restrict__ d) {
  __shared__ c128 red[4];
  const int q = blockIdx.x;
  for (int i = 0; i < ell; ++i) {
    c128 acc = {0.0, 0.0};
    for (int r = threadIdx.x; r < n; r += 256) acc = acc + conj(X[(long long)q * n + r]) * Y[((long long)r * P + q) * ell + i];
    const c128 s = block_sum256(acc, red);
    if (threadIdx.x == 0) d[q * ell + i] = s;
  }
}

// Newton's method on g(z) = sum_i f_i(z) d_i (eq. (rii-scalar) in split form),
// one thread per pair, from lam[q]; writes the root, f_i there and a flag
// (1: a pole or cut was met, or the iteration left the finite numbers).
__global__ void k_polish_newton(int ell, int P, const FnNode* __restrict__ nodes, const c128* __restrict__ coef,
                                const int* __restrict__ roots, const c128* __restrict__ d, c128* __restrict__ lam,
                                c128* __restrict__ fz, int* __restrict__ bad, int* __restrict__ steps) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P) return;
  const double rtol = sqrt(2.220446049250313e-16);
  c128 z = lam[q];
  int b = 0, it = 0;
  for (; it < kPolishNewton; ++it) {
    c128 g = {0.0, 0.0}, dg = {0.0, 0.0};
    for (int i = 0; i < ell; ++i) {
      c128 df;
      const c128 f = fn_eval_d(nodes, coef, roots[i], z, b, df);
      g = g + f * d[q * ell + i];
      dg = dg + df * d[q * ell + i];
    }
    if (b || (dg.re == 0.0 && dg.im == 0.0)) {
      b |= 1;
      break;
    }
    const c128 mu = cdiv(g, dg);
    z = z - mu;
    if (!isfinite(z.re) || !isfinite(z.im)) {
      b |= 1;
      break;
    }
    if (sqrt(norm2(mu)) < rtol * sqrt(norm2(z))) {
      ++it;
      break;
    }
  }
  for (int i = 0; i < ell; ++i) fz[q * ell + i] = fn_eval(nodes, coef, roots[i], z, b);
  lam[q] = z;
  bad[q] = b ? 1 : 0;
  steps[q] = it;
}

// Residual r = sum_i f_i(lambda) y_i (y_i = A_i x in R), written over R's
// first column as the right-hand side of the correction solve, and
// eta = max|r| / (sum_i |f_i| ||A_i||_inf max|x|) (eq. (sressplit), infinity
// norms).  One group per pair.
__global__ __launch_bounds__(256) void k_polish_residual(int n, int ell, int P, c128* __restrict__ R,
                                                         const c128* __restrict__ fz, const double* __restrict__ normA,
                                                         const c128* __restrict__ X, double* __restrict__ eta) {
  __shared__ double rmax[256], xmax[256];
  const int q = blockIdx.x;
  double rm = 0.0, xm = 0.0;
  for (int r = threadIdx.x; r < n; r += 256) {
    c128 rv = {0.0, 0.0};
    const long long k0 = ((long long)r * P + q) * ell;
    for (int i = 0; i < ell; ++i) rv = rv + fz[q * ell + i] * R[k0 + i];
    R[k0] = rv;  // this thread alone reads and writes row r of pair q
    rm = nanmax(rm, sqrt(norm2(rv)));
    xm = nanmax(xm, sqrt(norm2(X[(long long)q * n + r])));
  }
  rmax[threadIdx.x] = rm;
  xmax[threadIdx.x] = xm;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      rmax[threadIdx.x] = nanmax(rmax[threadIdx.x], rmax[threadIdx.x + s]);
      xmax[threadIdx.x] = nanmax(xmax[threadIdx.x], xmax[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double den = 0.0;
    for (int i = 0; i < ell; ++i) den += sqrt(norm2(fz[q * ell + i])) * normA[i];
    den *= xmax[0];
    eta[q] = den > 0.0 ? rmax[0] / den : NAN;
  }
}

// x_new = x - v with v = T(sigma)^{-1} r in Y's first column, and ||x_new||_2.
__global__ __launch_bounds__(256) void k_polish_correct(int n, int ell, int P, const c128* __restrict__ Y,
                                                        const c128* __restrict__ X, c128* __restrict__ Xn,
                                                        double* __restrict__ nrm) {
  __shared__ double ss[256];
  const int q = blockIdx.x;
  double s2 = 0.0;
  for (int r = threadIdx.x; r < n; r += 256) {
    const c128 xn = X[(long long)q * n + r] - Y[((long long)r * P + q) * ell];
    Xn[(long long)q * n + r] = xn;
    s2 += norm2(xn);
  }
  ss[threadIdx.x] = s2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) ss[threadIdx.x] += ss[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) nrm[q] = sqrt(ss[0]);
}

// x_q <- Xn_q / nrm_q for the pairs flagged in upd.
__global__ void k_polish_update(int n, int P, const c128* __restrict__ Xn, const double* __restrict__ nrm,
                                const int* __restrict__ upd, c128* __restrict__ X) {
  const int q = blockIdx.y;
  if (!upd[q]) return;
  const double s = 1.0 / nrm[q];
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
    X[(long long)q * n + r] = s * Xn[(long long)q * n + r];
}

// ||x||_2 = 1 and the largest-modulus entry (lowest index on ties) real and
// positive: the normalization of the extracted eigenvectors.
__global__ __launch_bounds__(256) void k_polish_normalize(int n, c128* __restrict__ X) {
  __shared__ double am[256], s2[256];
  __shared__ int ai[256];
  const int q = blockIdx.x;
  c128* x = X + (long long)q * n;
  double best = -1.0, ss = 0.0;
  int bi = 0;
  for (int r = threadIdx.x; r < n; r += 256) {
    const double a = norm2(x[r]);
    ss += a;
    if (a > best) {
      best = a;
      bi = r;
    }
  }
  am[threadIdx.x] = best;
  ai[threadIdx.x] = bi;
  s2[threadIdx.x] = ss;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double o = am[threadIdx.x + s];
      const int oi = ai[threadIdx.x + s];
      if (o > am[threadIdx.x] || (o == am[threadIdx.x] && oi < ai[threadIdx.x])) {
        am[threadIdx.x] = o;
        ai[threadIdx.x] = oi;
      }
      s2[threadIdx.x] += s2[threadIdx.x + s];
    }
    __syncthreads();
  }
  const c128 p = x[ai[0]];
  const double ap = sqrt(norm2(p)), nr = sqrt(s2[0]);
  const c128 ph = ap > 0.0 ? c128{p.re / ap, -p.im / ap} : c128{1.0, 0.0};
  const c128 sc = (1.0 / nr) * ph;
  __syncthreads();
  for (int r = threadIdx.x; r < n; r += 256) x[r] = sc * x[r];
}

nep_status backward_errors_dev(Split& h, int m, const c128* lam, const c128* X, double* eta, ExtractWork* w,
                               hipStream_t st);

nep_status rii_polish(Split& h, int m, zc* lam, c128* X, double* eta, const char* sel, double tol, int max_it,
                      int* iters, ExtractWork* w, hipStream_t st) {
  const int n = h.op.n, ell = h.op.ell;
  std::vector<int> idx;
  for (int q = 0; q < m; ++q)
    if (sel == nullptr || sel[q]) idx.push_back(q);
  if (iters)
    for (int q = 0; q < m; ++q) iters[q] = 0;
  const int P = (int)idx.size();
  if (P == 0) return NEP_OK;
  // shifts sigma_q = lambda_q and the plan that factors T(sigma_q) in FP64
  DevMem dz, dXw, dXn, dd, dfz, dlam, dsmall, dA;
  NEP_TRY(dz.alloc(sizeof(c128) * P));
  NEP_TRY(dXw.alloc(sizeof(c128) * (size_t)n * P));
  NEP_TRY(dXn.alloc(sizeof(c128) * (size_t)n * P));
  NEP_TRY(dd.alloc(sizeof(c128) * (size_t)P * ell));
  NEP_TRY(dfz.alloc(sizeof(c128) * (size_t)P * ell));
  NEP_TRY(dlam.alloc(sizeof(c128) * P));
  NEP_TRY(dsmall.alloc((sizeof(double) * 2 + sizeof(int) * 3) * (size_t)P));
  NEP_TRY(dA.alloc(sizeof(void*) * kMaxTerms + sizeof(int) * kMaxTerms));
  std::vector<c128> sig(P);
  for (int k = 0; k < P; ++k) sig[k] = c128{lam[idx[k]].real(), lam[idx[k]].imag()};
  NEP_HIP(hipMemcpyAsync(dz.p, sig.data(), sizeof(c128) * P, hipMemcpyHostToDevice, st));
  for (int k = 0; k < P; ++k)
    NEP_HIP(hipMemcpyAsync(dXw.as<c128>() + (size_t)k * n, X + (size_t)idx[k] * n, sizeof(c128) * n,
                           hipMemcpyDeviceToDevice, st));
  const double* hA[kMaxTerms];
  for (int i = 0; i < ell; ++i) hA[i] = reinterpret_cast<const double*>(h.op.dA[i]);
  const double** dAp = dA.as<const double*>();
  int* dcp = reinterpret_cast<int*>(dA.as<char>() + sizeof(void*) * kMaxTerms);
  NEP_HIP(hipMemcpyAsync(dAp, hA, sizeof(void*) * ell, hipMemcpyHostToDevice, st));
  NEP_HIP(hipMemcpyAsync(dcp, h.op.is_cplx, sizeof(int) * ell, hipMemcpyHostToDevice, st));
  double* deta = dsmall.as<double>();
  double* dnrm = deta + P;
  int* dbad = reinterpret_cast<int*>(dnrm + P);
  int* dupd = dbad + P;
  int* dsteps = dupd + P;

  MomentsPlan plan;
  nep_contour g0{};
  g0.kind = 0;
  g0.rho = 1.0;
  g0.v = 1.0;
  PlanOptions po;
  po.N = P;
  po.L = ell;
  po.K = 1;
  po.prec = NEP_PREC_FP64;
  po.max_refine = 0;
  po.fallback = 0;
  std::vector<PlanProblem> probs{PlanProblem{&h.op, g0, nullptr, nullptr, dz.as<c128>()}};
  NEP_TRY(plan.build(probs, po, st));
  NEP_TRY(plan.factor(st));
  std::vector<int> info(P), active(P, 1), upd(P, 0), bad(P), steps(P);
  NEP_HIP(hipMemcpyAsync(info.data(), plan.info(), sizeof(int) * P, hipMemcpyDeviceToHost, st));
  NEP_HIP(hipStreamSynchronize(st));
  for (int k = 0; k < P; ++k)
    if (info[k] < n) active[k] = 0;  // T(sigma) exactly singular: sigma is an eigenvalue to working precision
  std::vector<c128> lcur(sig), lnew(P);
  std::vector<double> et(P);
  NEP_HIP(hipMemcpyAsync(dlam.p, lcur.data(), sizeof(c128) * P, hipMemcpyHostToDevice, st));
  int it = 0;
  for (; it < max_it; ++it) {
    bool any = false;
    for (int k = 0; k < P; ++k) any |= active[k] != 0;
    if (!any) break;
    hipLaunchKernelGGL(k_term_apply, dim3(ceil_div(n, 64), ceil_div(P, 16), ell), dim3(256), 0, st, n, ell, P, dAp,
                       dcp, dXw.as<c128>(), plan.R_mut());
    NEP_HIP(hipGetLastError());
    NEP_TRY(plan.solve_rhs(st));
    hipLaunchKernelGGL(k_polish_dots, dim3(P), dim3(256), 0, st, n, ell, P, dXw.as<c128>(), plan.Y_mut(),
                       dd.as<c128>());
    NEP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_polish_newton, dim3(ceil_div(P, 64)), dim3(64), 0, st, ell, P, h.op.dfn_nodes,
                       h.op.dfn_coef, h.fn_roots.as<int>(), dd.as<c128>(), dlam.as<c128>(), dfz.as<c128>(), dbad,
                       dsteps);
    NEP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_polish_residual, dim3(P), dim3(256), 0, st, n, ell, P, plan.R_mut(), dfz.as<c128>(),
                       h.op.dnormA, dXw.as<c128>(), deta);
    NEP_HIP(hipGetLastError());
    NEP_TRY(plan.solve_rhs(st));  // v = T(sigma)^{-1} r (first column)
    hipLaunchKernelGGL(k_polish_correct, dim3(P), dim3(256), 0, st, n, ell, P, plan.Y_mut(), dXw.as<c128>(),
                       dXn.as<c128>(), dnrm);
    NEP_HIP(hipGetLastError());
    NEP_HIP(hipMemcpyAsync(lnew.data(), dlam.p, sizeof(c128) * P, hipMemcpyDeviceToHost, st));
    NEP_HIP(hipMemcpyAsync(et.data(), deta, sizeof(double) * P, hipMemcpyDeviceToHost, st));
    NEP_HIP(hipMemcpyAsync(bad.data(), dbad, sizeof(int) * P, hipMemcpyDeviceToHost, st));
    NEP_HIP(hipStreamSynchronize(st));
    bool more = false;
    for (int k = 0; k < P; ++k) {
      upd[k] = 0;
      if (!active[k]) continue;
      if (bad[k] || !std::isfinite(et[k])) {
        active[k] = 0;  // left as it was
        lnew[k] = lcur[k];
        continue;
      }
      lcur[k] = lnew[k];
      if (iters) iters[idx[k]] = it + 1;
      if (et[k] < tol) {
        active[k] = 0;  // (x^{(k)}, lambda^{(k+1)}) is the result
      } else {
        upd[k] = 1;
        more = true;
      }
    }
    // inactive pairs restart the scalar Newton from their kept value
    NEP_HIP(hipMemcpyAsync(dlam.p, lcur.data(), sizeof(c128) * P, hipMemcpyHostToDevice, st));
    if (!more) break;
    NEP_HIP(hipMemcpyAsync(dupd, upd.data(), sizeof(int) * P, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_polish_update, dim3(ceil_div(n, 256), P), dim3(256), 0, st, n, P, dXn.as<c128>(), dnrm,
                       dupd, dXw.as<c128>());
    NEP_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_polish_normalize, dim3(P), dim3(256), 0, st, n, dXw.as<c128>());
  NEP_HIP(hipGetLastError());
  // the polished pairs' backward errors as the extraction reports them; a
  // pair is replaced only where that improves on what it had
  std::vector<double> eta_new(P);
  NEP_TRY(backward_errors_dev(h, P, lcur.data(), dXw.as<c128>(), eta_new.data(), w, st));
  for (int k = 0; k < P; ++k) {
    const int q = idx[k];
    if (!(eta_new[k] < eta[q])) continue;  // not better (or not comparable): the pair stays as it was
    lam[q] = zc(lcur[k].re, lcur[k].im);
    eta[q] = eta_new[k];
    NEP_HIP(hipMemcpyAsync(X + (size_t)q * n, dXw.as<c128>() + (size_t)k * n, sizeof(c128) * n,
                           hipMemcpyDeviceToDevice, st));
  }
  NEP_HIP(hipStreamSynchronize(st));
  return NEP_OK;
}

}  // namespace nep

using namespace nep;

extern "C" {

nep_status nep_rii_polish(nep_split h, int m, double* lambda, void* X, double* eta, double tol, int max_it,
                          int* iters) {
  NEP_CHECK(h != nullptr, NEP_ERR_ARG, "null handle");
  NEP_CHECK(m >= 1 && lambda && X && eta, NEP_ERR_ARG, "bad arguments");
  NEP_CHECK(tol >= 0.0 && max_it >= 1 && max_it <= 100, NEP_ERR_ARG, "need tol >= 0 and 1 <= max_it <= 100");
  Split& s = h->impl;
  std::vector<zc> lam(m);
  for (int q = 0; q < m; ++q) lam[q] = zc(lambda[2 * q], lambda[2 * q + 1]);
  std::vector<c128> lc(m);
  for (int q = 0; q < m; ++q) lc[q] = c128{lam[q].real(), lam[q].imag()};
  NEP_TRY(backward_errors_dev(s, m, lc.data(), (const c128*)X, eta, nullptr, s.stream));
  NEP_TRY(rii_polish(s, m, lam.data(), (c128*)X, eta, nullptr, tol > 0.0 ? tol : 1e-14, max_it, iters, nullptr,
                     s.stream));
  for (int q = 0; q < m; ++q) {
    lambda[2 * q] = lam[q].real();
    lambda[2 * q + 1] = lam[q].imag();
  }
  return NEP_OK;
}

}  // extern "C"
