// Quadrature coefficients, split-form assembly and moment accumulation.
//
//   coefficients: nodes z_j = c + rho zeta_j with zeta_j = cos t_j + i v sin t_j,
//                 t_j = 2 pi (j + 1/2)/N, weights w_j = rho (v cos t_j + i sin t_j)/N
//                 (trapezoid rule for the contour integral of eq. (invpair) over
//                 the RG circle/ellipse), f_i(z_j) under FN semantics, and the
//                 moment weights w_j zeta_j^p.
//   assembly:     T(z_j) = sum_i f_i(z_j) A_i (eq. (split)), FP64 multiply-adds in
//                 the order i = 1..ell, rounded once to the factor precision.
//                 Each A_i element is read once and reused for every node.
//   moments:      S_p = sum_j w_j zeta_j^p Y_j, j ascending, FP64 (the
//                 quadrature of the Keldysh-expanded resolvent, eq. (resolvent)).
#include "engine.hpp"

namespace nep {

// ---------------------------------------------------------------------------
__global__ void k_coef(const ProbDesc* __restrict__ pd, NodeArrays na, int nnodes, IrState ir) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nnodes) return;
  const int p = na.prob[g], j = na.jnode[g];
  const ProbDesc& P = pd[p];
  if (!P.active) {  // sits out this pass: nothing of its operator is read
    na.bad[g] = 0;
    ir.conv[g] = 1;
    return;
  }
  const double th = 2.0 * M_PI * (j + 0.5) / P.N;
  double s, c;
  sincos(th, &s, &c);
  const double v = P.kind == 1 ? P.v : 1.0;
  c128 zeta = {c, v * s};
  c128 z = {P.c.re + P.rho * zeta.re, P.c.im + P.rho * zeta.im};
  c128 w = {P.rho * v * c / P.N, P.rho * s / P.N};
  if (P.zpts != nullptr) {  // explicit points (shifted solves): no quadrature weights
    z = P.zpts[j];
    zeta = z;
    w = {0.0, 0.0};
  }
  na.z[g] = z;
  na.zeta[g] = zeta;
  na.w[g] = w;
  int bad = 0;
  double fn = 0.0;
  for (int i = 0; i < P.ell; ++i) {
    const c128 f = P.fpts != nullptr ? P.fpts[j * P.ell + i] : fn_eval(P.fn_nodes, P.fn_coef, P.fn_root[i], z, bad);
    na.fz[g * kMaxTerms + i] = f;
    fn += sqrt(norm2(f)) * P.normA[i];
  }
  na.fnorm[g] = fn;
  c128 zp = {1.0, 0.0};
  for (int q = 0; q < P.KK; ++q) {
    na.mcoef[g * kMaxMoments + q] = w * zp;
    zp = zp * zeta;
  }
  na.bad[g] = bad ? 1 : 0;
  if (bad) {
    atomicAdd(&ir.counters[1], 1);
    atomicMin(&ir.counters[3], g);
  }
}

hipError_t launch_coef(const ProbDesc* pd, const NodeArrays& na, int nnodes, IrState ir, hipStream_t st) {
  hipLaunchKernelGGL(k_coef, dim3(ceil_div(nnodes, 64)), dim3(64), 0, st, pd, na, nnodes, ir);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Assembly.  One thread per element (r, c) of one problem; loops over nodes.
// ---------------------------------------------------------------------------
constexpr int kAsmThreads = 256;

template <typename P, bool CPLX>
__device__ __forceinline__ void assemble_elem(const ProbDesc& D, const NodeArrays& na, long long e, cx<P>* T,
                                              const int* skip) {
  const int n = D.n;
  const int r = (int)(e / n), col = (int)(e - (long long)r * n);
  double ar[kMaxTerms], ai[kMaxTerms];
#pragma unroll
  for (int i = 0; i < kMaxTerms; ++i) {
    if (i < D.ell) {
      if (CPLX && D.a_is_cplx[i]) {
        const c128 a = reinterpret_cast<const c128*>(D.A[i])[e];
        ar[i] = a.re;
        ai[i] = a.im;
      } else {
        ar[i] = reinterpret_cast<const double*>(D.A[i])[e];
        ai[i] = 0.0;
      }
    }
  }
  const long long off = (long long)r * D.ld + col;
  for (int j = 0; j < D.N; ++j) {
    const int g = D.node0 + j;
    if (skip != nullptr && skip[g]) continue;
    const c128* f = na.fz + (long long)g * kMaxTerms;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxTerms; ++i) {
      if (i < D.ell) {
        const c128 fi = f[i];
        if (CPLX) {
          sr += fi.re * ar[i] - fi.im * ai[i];
          si += fi.re * ai[i] + fi.im * ar[i];
        } else {
          sr += fi.re * ar[i];
          si += fi.im * ar[i];
        }
      }
    }
    T[D.offT0 + (long long)j * D.strideT + off] = cx<P>{P(sr), P(si)};
  }
}

template <typename P>
__global__ __launch_bounds__(kAsmThreads) void k_assemble(const ProbDesc* __restrict__ pd,
                                                          const int* __restrict__ prefix, int cnt, int total,
                                                          NodeArrays na, cx<P>* __restrict__ T,
                                                          const int* __restrict__ skip) {
  const int v = xcd_remap(blockIdx.x, gridDim.x, total);
  if (v < 0) return;
  const int p = find_slot(prefix, cnt, v);
  const ProbDesc& D = pd[p];
  const long long e = (long long)(v - prefix[p]) * kAsmThreads + threadIdx.x;
  if (e >= (long long)D.n * D.n) return;
  if (D.a_cplx) assemble_elem<P, true>(D, na, e, T, skip);
  else assemble_elem<P, false>(D, na, e, T, skip);
}

template <typename P>
hipError_t launch_assemble(const ProbDesc* pd, const int* prefix, const Table& t, const NodeArrays& na, cx<P>* T,
                           const int* skip, hipStream_t st) {
  if (t.total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_assemble<P>, dim3(xcd_grid(t.total)), dim3(kAsmThreads), 0, st, pd, prefix + t.off, t.cnt,
                     t.total, na, T, skip);
  return hipGetLastError();
}
template hipError_t launch_assemble<float>(const ProbDesc*, const int*, const Table&, const NodeArrays&, c64*,
                                           const int*, hipStream_t);
template hipError_t launch_assemble<double>(const ProbDesc*, const int*, const Table&, const NodeArrays&, c128*,
                                            const int*, hipStream_t);

// ---------------------------------------------------------------------------
// Moments.  One thread per (row r, probe c) of one problem.
// Y: row-major n x (N*L) per problem; S: column-major n x L per moment p.
// ---------------------------------------------------------------------------
constexpr int kMomThreads = 256;
constexpr int kMomQ = 8;  // moments per thread

// One thread per (row r, probe column c, group of kMomQ moments); the sum
// over nodes runs in ascending j for every moment.  Lanes of a wave cover
// consecutive (c, r) pairs of one moment group, so Y loads are contiguous
// per row and the coefficients w_j zeta_j^p are wave-uniform.
__global__ __launch_bounds__(kMomThreads) void k_moments(const ProbDesc* __restrict__ pd,
                                                         const int* __restrict__ prefix, int cnt, int total,
                                                         NodeArrays na, const c128* __restrict__ Y) {
  const int v = xcd_remap(blockIdx.x, gridDim.x, total);
  if (v < 0) return;
  const int p = find_slot(prefix, cnt, v);
  const ProbDesc& D = pd[p];
  if (!D.active) return;
  const int n = D.n, L = D.L, NL = D.N * D.L, KK = D.KK, N = D.N, node0 = D.node0;
  const int ngrp = (KK + kMomQ - 1) / kMomQ;
  const int nl = n * L;
  const int blocks_per_grp = (nl + kMomThreads - 1) / kMomThreads;
  const int local = v - prefix[p];
  const int qg = local / blocks_per_grp;
  const int e = (local - qg * blocks_per_grp) * kMomThreads + threadIdx.x;
  if (qg >= ngrp || e >= nl) return;
  const int r = e / L, c = e - r * L;
  const int q0 = qg * kMomQ;
  c128 acc[kMomQ];
#pragma unroll
  for (int q = 0; q < kMomQ; ++q) acc[q] = {0.0, 0.0};
  const c128* y = Y + D.offY + (long long)r * NL + c;
  const c128* mc0 = na.mcoef + (long long)node0 * kMaxMoments + q0;
  for (int j = 0; j < N; ++j) {
    const c128 yv = y[j * L];
    const c128* mc = mc0 + (long long)j * kMaxMoments;
#pragma unroll
    for (int q = 0; q < kMomQ; ++q) acc[q] = cmac(acc[q], mc[q], yv);
  }
#pragma unroll
  for (int q = 0; q < kMomQ; ++q)
    if (q0 + q < KK) D.S[(long long)(q0 + q) * D.s_stride + (long long)c * n + r] = acc[q];
}

hipError_t launch_moments(const ProbDesc* pd, const int* prefix, const Table& t, const NodeArrays& na,
                          const c128* Y, hipStream_t st) {
  if (t.total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_moments, dim3(xcd_grid(t.total)), dim3(kMomThreads), 0, st, pd, prefix + t.off, t.cnt,
                     t.total, na, Y);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// max |V| per probe column: one block per (problem, column), a wave max by
// shuffles, then the four waves through LDS
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_vnorm(const ProbDesc* __restrict__ pd, IrState ir) {
  const ProbDesc& D = pd[blockIdx.x];
  const int c = blockIdx.y;
  if (c >= D.L || !D.active) return;  // uniform
  const c128* __restrict__ v = D.V + (long long)c * D.n;
  double m = 0.0;
  for (int r = threadIdx.x; r < D.n; r += blockDim.x) m = nanmax(m, sqrt(norm2(v[r])));
  for (int o = 32; o >= 1; o >>= 1) m = nanmax(m, __shfl_xor(m, o, 64));
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) ir.vnorm[blockIdx.x * 64 + c] = nanmax(nanmax(red[0], red[1]), nanmax(red[2], red[3]));
}

hipError_t launch_vnorm(const ProbDesc* pd, int nprob, int L, IrState ir, hipStream_t st) {
  hipLaunchKernelGGL(k_vnorm, dim3(nprob, L), dim3(256), 0, st, pd, ir);
  return hipGetLastError();
}

void build_prefix(std::vector<int>& buf, Table& t, const std::vector<int>& counts) {
  t.off = (int)buf.size();
  t.cnt = (int)counts.size();
  int acc = 0;
  buf.push_back(0);
  for (int c : counts) {
    acc += c;
    buf.push_back(acc);
  }
  t.total = acc;
}

}  // namespace nep
