// Left eigenvectors and the resolvent (Section 2, eqs. (nep-left) and
// (resolvent); Section 3.2.5, NEPGetLeftEigenvector / NEPApplyResolvent).
//
// Left eigenvectors y^* T(lambda) = 0 are right eigenvectors of the adjoint
// operator T^*(z) = T(conj z)^* = sum_i conj(f_i(conj z)) A_i^*, at the
// eigenvalue conj(lambda).  nep_split_adjoint builds that operator as a
// handle of its own (so the whole moment path and the extraction run on it);
// nep_left_eigenvectors computes y for given eigenvalues by residual inverse
// iteration on T^* with the target sigma = conj(lambda).
//
// Keldysh's expansion gives, for semisimple eigenvalues inside the region,
// T^{-1}(z) = sum_i (z - lambda_i)^{-1} x_i y_i^* + R(z) with
// y_i^* T'(lambda_i) x_i = 1.  nep_apply_resolvent applies the sum to a block
// of vectors (the normalization is applied explicitly: c_i = y_i^* T'(lambda_i)
// x_i divides each term), and nep_solve_at applies the full T(z)^{-1} at given
// points by factorization and solves.
#include <cmath>
#include <vector>

#include "dense.hpp"
#include "handle.hpp"

namespace nep {

hipError_t fn_points_d(const FnNode* nodes, const c128* coef, const int* roots, int ell, const c128* z, int m,
                       c128* out, int* bad, hipStream_t st);
nep_status backward_errors_dev(Split& h, int m, const c128* lam, const c128* X, double* eta, ExtractWork* w,
                               hipStream_t st);
nep_status rii_polish(Split& h, int m, zc* lam, c128* X, double* eta, const char* sel, double tol, int max_it,
                      int* iters, ExtractWork* w, hipStream_t st);

hipError_t term_apply(int n, int ell, int P, const double* const* A, const int* cplx, const c128* X, c128* R,
                      hipStream_t st);

// c_q = y_q^* T'(lambda_q) x_q = sum_r conj(y_q[r]) sum_i f_i'(lambda_q) (A_i x_q)[r],
// with R[(r*m + q)*ell + i] = (A_i x_q)[r] from term_apply.  One group per pair.
__global__ __launch_bounds__(256) void k_keldysh_scale(int n, int ell, int m, const c128* __restrict__ R,
                                                       const c128* __restrict__ fd, const c128* __restrict__ Y,
                                                       c128* __restrict__ c) {
  __shared__ c128 red[4];
  const int q = blockIdx.x;
  c128 acc = {0.0, 0.0};
  for (int r = threadIdx.x; r < n; r += 256) {
    c128 tr = {0.0, 0.0};
    for (int i = 0; i < ell; ++i) tr = tr + fd[(long long)i * m + q] * R[((long long)r * m + q) * ell + i];
    acc = acc + conj(Y[(long long)q * n + r]) * tr;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    acc.re += __shfl_xor(acc.re, o, 64);
    acc.im += __shfl_xor(acc.im, o, 64);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) c[q] = red[0] + red[1] + red[2] + red[3];
}

// G[q + c*m] = coef_q * y_q^* v_c  (coef_q = 1/((z - lambda_q) c_q)).
__global__ __launch_bounds__(256) void k_resolvent_g(int n, int m, const c128* __restrict__ Y,
                                                     const c128* __restrict__ V, const c128* __restrict__ coef,
                                                     c128* __restrict__ G) {
  __shared__ c128 red[4];
  const int q = blockIdx.x, col = blockIdx.y;
  c128 acc = {0.0, 0.0};
  for (int r = threadIdx.x; r < n; r += 256) acc = acc + conj(Y[(long long)q * n + r]) * V[(long long)col * n + r];
  for (int o = 32; o >= 1; o >>= 1) {
    acc.re += __shfl_xor(acc.re, o, 64);
    acc.im += __shfl_xor(acc.im, o, 64);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) G[q + (long long)col * m] = coef[q] * (red[0] + red[1] + red[2] + red[3]);
}

// W[:, c] = sum_q x_q G[q, c]
__global__ void k_resolvent_w(int n, int m, int L, const c128* __restrict__ X, const c128* __restrict__ G,
                              c128* __restrict__ W) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * L) return;
  const int col = (int)(e / n), r = (int)(e - (long long)col * n);
  c128 s = {0.0, 0.0};
  for (int q = 0; q < m; ++q) s = s + X[(long long)q * n + r] * G[q + (long long)col * m];
  W[e] = s;
}

// Y_out[k][c][r] (column-major n x L per point) from the plan layout
// [row][point][column].
__global__ void k_points_out(int n, int P, int L, const c128* __restrict__ Yp, c128* __restrict__ out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * P * L) return;
  const int k = (int)(e / ((long long)n * L));
  const long long rem = e - (long long)k * n * L;
  const int c = (int)(rem / n), r = (int)(rem - (long long)c * n);
  out[e] = Yp[((long long)r * P + k) * L + c];
}

static nep_status ensure_adjoint(Split& s) {
  if (s.adj) return NEP_OK;
  auto a = std::make_unique<nep_split_s>();
  NEP_TRY(a->impl.init_adjoint(s));
  s.adj = a.release();
  return NEP_OK;
}

}  // namespace nep

using namespace nep;

extern "C" {

nep_status nep_split_adjoint(nep_split h, nep_split* out) {
  NEP_CHECK(h != nullptr && out != nullptr, NEP_ERR_ARG, "null handle or output");
  *out = nullptr;
  auto a = std::make_unique<nep_split_s>();
  NEP_TRY(a->impl.init_adjoint(h->impl));
  *out = a.release();
  return NEP_OK;
}

nep_status nep_left_eigenvectors(nep_split h, int m, double* lambda, void* Y, double* eta, int max_it) {
  NEP_CHECK(h != nullptr, NEP_ERR_ARG, "null handle");
  NEP_CHECK(m >= 1 && lambda && Y && eta, NEP_ERR_ARG, "bad arguments");
  NEP_CHECK(max_it >= 1 && max_it <= 100, NEP_ERR_ARG, "max_it must be in 1..100");
  Split& s = h->impl;
  NEP_TRY(ensure_adjoint(s));
  Split& a = s.adj->impl;
  std::vector<zc> mu(m);
  std::vector<c128> muc(m);
  for (int q = 0; q < m; ++q) {
    mu[q] = zc(lambda[2 * q], -lambda[2 * q + 1]);  // eigenvalues of T^* are conj(lambda)
    muc[q] = c128{mu[q].real(), mu[q].imag()};
  }
  NEP_TRY(backward_errors_dev(a, m, muc.data(), (const c128*)Y, eta, nullptr, s.stream));
  NEP_TRY(rii_polish(a, m, mu.data(), (c128*)Y, eta, nullptr, 1e-14, max_it, nullptr, nullptr, s.stream));
  for (int q = 0; q < m; ++q) {
    lambda[2 * q] = mu[q].real();
    lambda[2 * q + 1] = -mu[q].imag();
  }
  return NEP_OK;
}

nep_status nep_apply_resolvent(nep_split h, int m, const double* lambda, const void* X, const void* Y,
                               const double* z, int L, const void* V, void* W) {
  NEP_CHECK(h != nullptr, NEP_ERR_ARG, "null handle");
  NEP_CHECK(m >= 1 && m <= 4096 && L >= 1 && lambda && X && Y && z && V && W, NEP_ERR_ARG, "bad arguments");
  Split& s = h->impl;
  const int n = s.op.n, ell = s.op.ell;
  const hipStream_t st = s.stream;
  DevMem dlam, dfd, dbad, dc, dcoef, dG, dA, dR;
  NEP_TRY(dlam.alloc(sizeof(c128) * m));
  NEP_TRY(dfd.alloc(sizeof(c128) * (size_t)m * ell));
  NEP_TRY(dbad.alloc(sizeof(int) * m));
  NEP_TRY(dc.alloc(sizeof(c128) * m));
  NEP_TRY(dcoef.alloc(sizeof(c128) * m));
  NEP_TRY(dG.alloc(sizeof(c128) * (size_t)m * L));
  NEP_TRY(dA.alloc(sizeof(void*) * kMaxTerms + sizeof(int) * kMaxTerms));
  NEP_TRY(dR.alloc(sizeof(c128) * (size_t)n * m * ell));
  NEP_HIP(hipMemcpyAsync(dlam.p, lambda, sizeof(c128) * m, hipMemcpyHostToDevice, st));
  NEP_HIP(fn_points_d(s.op.dfn_nodes, s.op.dfn_coef, s.fn_roots.as<int>(), ell, dlam.as<c128>(), m, dfd.as<c128>(),
                      dbad.as<int>(), st));
  const double* hA[kMaxTerms];
  for (int i = 0; i < ell; ++i) hA[i] = reinterpret_cast<const double*>(s.op.dA[i]);
  const double** dAp = dA.as<const double*>();
  int* dcp = reinterpret_cast<int*>(dA.as<char>() + sizeof(void*) * kMaxTerms);
  NEP_HIP(hipMemcpyAsync(dAp, hA, sizeof(void*) * ell, hipMemcpyHostToDevice, st));
  NEP_HIP(hipMemcpyAsync(dcp, s.op.is_cplx, sizeof(int) * ell, hipMemcpyHostToDevice, st));
  NEP_HIP(term_apply(n, ell, m, dAp, dcp, (const c128*)X, dR.as<c128>(), st));
  hipLaunchKernelGGL(k_keldysh_scale, dim3(m), dim3(256), 0, st, n, ell, m, dR.as<c128>(), dfd.as<c128>(),
                     (const c128*)Y, dc.as<c128>());
  NEP_HIP(hipGetLastError());
  std::vector<c128> c(m), coef(m);
  std::vector<int> bad(m);
  NEP_HIP(hipMemcpyAsync(c.data(), dc.p, sizeof(c128) * m, hipMemcpyDeviceToHost, st));
  NEP_HIP(hipMemcpyAsync(bad.data(), dbad.p, sizeof(int) * m, hipMemcpyDeviceToHost, st));
  NEP_HIP(hipStreamSynchronize(st));
  const zc zz(z[0], z[1]);
  for (int q = 0; q < m; ++q) {
    NEP_CHECK(!bad[q], NEP_ERR_NOT_HOLOMORPHIC, "eigenvalue %d lies on a pole or branch cut of some f_i", q);
    const zc lq(lambda[2 * q], lambda[2 * q + 1]);
    const zc cq(c[q].re, c[q].im);
    NEP_CHECK(std::abs(cq) > 0.0 && zz != lq, NEP_ERR_ARG,
              "pair %d: y^* T'(lambda) x = 0 (not a simple eigenvalue) or z equals lambda", q);
    const zc k = 1.0 / ((zz - lq) * cq);
    coef[q] = c128{k.real(), k.imag()};
  }
  NEP_HIP(hipMemcpyAsync(dcoef.p, coef.data(), sizeof(c128) * m, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_resolvent_g, dim3(m, L), dim3(256), 0, st, n, m, (const c128*)Y, (const c128*)V,
                     dcoef.as<c128>(), dG.as<c128>());
  NEP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_resolvent_w, dim3((unsigned)ceil_div_ll((long long)n * L, 256)), dim3(256), 0, st, n, m, L,
                     (const c128*)X, dG.as<c128>(), (c128*)W);
  NEP_HIP(hipGetLastError());
  NEP_HIP(hipStreamSynchronize(st));
  return NEP_OK;
}

nep_status nep_solve_at(nep_split h, int m, const double* z, int L, const void* V, int prec, void* Y,
                        nep_ciss_stats* st_out) {
  NEP_CHECK(h != nullptr, NEP_ERR_ARG, "null handle");
  NEP_CHECK(m >= 1 && m <= 4096 && L >= 1 && L <= 64 && z && V && Y, NEP_ERR_ARG, "bad arguments");
  NEP_CHECK(prec == NEP_PREC_FP64 || prec == NEP_PREC_C32_IR64, NEP_ERR_ARG, "unknown precision %d", prec);
  Split& s = h->impl;
  const int n = s.op.n;
  const hipStream_t st = s.stream;
  DevMem dz, dS;
  NEP_TRY(dz.alloc(sizeof(c128) * m));
  NEP_TRY(dS.alloc(sizeof(c128) * (size_t)n * L * 2));  // the (zero-weight) moments the plan writes
  NEP_HIP(hipMemcpyAsync(dz.p, z, sizeof(c128) * m, hipMemcpyHostToDevice, st));
  MomentsPlan plan;
  nep_contour g0{};
  g0.kind = 0;
  g0.rho = 1.0;
  g0.v = 1.0;
  PlanOptions po;
  po.N = m;
  po.L = L;
  po.K = 1;
  po.prec = prec;
  po.max_refine = prec == NEP_PREC_FP64 ? 0 : 5;
  po.fallback = 1;
  std::vector<PlanProblem> probs{PlanProblem{&s.op, g0, (const c128*)V, dS.as<c128>(), dz.as<c128>()}};
  NEP_TRY(plan.build(probs, po, st));
  NEP_TRY(plan.enqueue(st, true));
  RunResult rr;
  const nep_status rs = plan.finish(st, rr, true);
  if (st_out && !rr.stats.empty()) *st_out = rr.stats[0];
  NEP_TRY(rs);
  hipLaunchKernelGGL(k_points_out, dim3((unsigned)ceil_div_ll((long long)n * m * L, 256)), dim3(256), 0, st, n, m, L,
                     plan.Y(), (c128*)Y);
  NEP_HIP(hipGetLastError());
  NEP_HIP(hipStreamSynchronize(st));
  return NEP_OK;
}

}  // extern "C"
