// Batched triangular solves with the factors of k_lu_*: Y_j = T(z_j)^{-1} B.
//
//   gather : W = P B  (row r of W is row row_at[r] of B; B is the probe block V
//            or a refinement residual R), rounded to the factor precision.
//   steps  : blocked substitution, 64-row blocks, one launch per block step.
//            In step s every remaining block receives the update from the
//            block solved in step s-1 (W_r -= L_rq W_q, one work-group per
//            (matrix, block)); the group that owns the next diagonal block then
//            solves it in registers, one wave per right-hand column with the
//            64 rows spread over the lanes (no block barrier in the sweep).
//            Forward: unit lower L.  Backward: U, dividing by its diagonal.
//   scatter: Y = W (initial solve) or Y += W (refinement correction), in FP64,
//            and the column maxima of |Y| used by the refinement test.
#include "engine.hpp"

namespace nep {

constexpr int kSolveThreads = 256;

template <typename P>
__device__ __forceinline__ cx<P> cdivp(cx<P> a, cx<P> b) {
  const c128 q = cdiv(c128{double(a.re), double(a.im)}, c128{double(b.re), double(b.im)});
  return cx<P>{P(q.re), P(q.im)};
}

// ---------------------------------------------------------------------------
template <typename P>
__global__ __launch_bounds__(kSolveThreads) void k_solve_gather(const MatDesc* __restrict__ md,
                                                               const int* __restrict__ prefix, int cnt, int total,
                                                               const ProbDesc* __restrict__ pd, NodeArrays na,
                                                               const int* __restrict__ rows, cx<P>* __restrict__ Wk,
                                                               const c128* __restrict__ R, int refine,
                                                               const int* __restrict__ conv) {
  const int v = xcd_remap(blockIdx.x, gridDim.x, total);
  if (v < 0) return;
  const int b = find_slot(prefix, cnt, v);
  const MatDesc d = md[b];
  const int g = d.node;
  if (conv != nullptr && conv[g]) return;
  const int p = na.prob[g], j = na.jnode[g];
  const ProbDesc& D = pd[p];
  const int L = D.L, n = d.n;
  const int e = (v - prefix[b]) * kSolveThreads + threadIdx.x;
  if (e >= n * L) return;
  const int r = e / L, c = e - r * L;
  const int pr = rows[d.offRow + r];
  c128 val;
  if (refine) val = R[D.offY + (long long)pr * D.N * L + (long long)j * L + c];
  else val = D.V[(long long)c * n + pr];
  Wk[D.offW0 + (long long)j * n * L + e] = cvt<P>(val);
}

template <typename P>
__global__ __launch_bounds__(kSolveThreads) void k_solve_scatter(const MatDesc* __restrict__ md,
                                                                const int* __restrict__ prefix, int cnt, int total,
                                                                const ProbDesc* __restrict__ pd, NodeArrays na,
                                                                const cx<P>* __restrict__ Wk, c128* __restrict__ Y,
                                                                int refine, const int* __restrict__ conv,
                                                                IrState ir) {
  const int v = xcd_remap(blockIdx.x, gridDim.x, total);
  if (v < 0) return;
  const int b = find_slot(prefix, cnt, v);
  const MatDesc d = md[b];
  const int g = d.node;
  if (conv != nullptr && conv[g]) return;
  const int p = na.prob[g], j = na.jnode[g];
  const ProbDesc& D = pd[p];
  const int L = D.L, n = d.n;
  const int e = (v - prefix[b]) * kSolveThreads + threadIdx.x;
  double m = 0.0;
  int c = 0;
  if (e < n * L) {
    const int r = e / L;
    c = e - r * L;
    const cx<P> w = Wk[D.offW0 + (long long)j * n * L + e];
    c128* y = Y + D.offY + (long long)r * D.N * L + (long long)j * L + c;
    c128 nv = {double(w.re), double(w.im)};
    if (refine) nv = *y + nv;
    *y = nv;
    m = sqrt(norm2(nv));
  }
  // column maxima: for L a power of two <= 64 the lanes of one wave that hold
  // the same column c sit L apart, so they reduce before the atomic.
  const int lane = threadIdx.x & 63;
  if ((L & (L - 1)) == 0 && L <= 64) {
    for (int off = L; off < 64; off <<= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if (e < n * L && lane < L)
      atomicMax(&ir.ynorm[(long long)g * kNormStride + c], (unsigned long long)__double_as_longlong(m));
  } else if (e < n * L) {
    atomicMax(&ir.ynorm[(long long)g * kNormStride + c], (unsigned long long)__double_as_longlong(m));
  }
}

// ---------------------------------------------------------------------------
template <typename P, bool LOWER>
__global__ __launch_bounds__(kSolveThreads) void k_solve_step(const MatDesc* __restrict__ md,
                                                             const int* __restrict__ prefix, int cnt, int total,
                                                             int s, const ProbDesc* __restrict__ pd, NodeArrays na,
                                                             const cx<P>* __restrict__ Tb,
                                                             const int* __restrict__ rows, cx<P>* __restrict__ Wk,
                                                             const int* __restrict__ conv) {
  const int v = xcd_remap(blockIdx.x, gridDim.x, total);
  if (v < 0) return;
  const int b = find_slot(prefix, cnt, v);
  const int t = v - prefix[b];
  const MatDesc d = md[b];
  const int g = d.node;
  if (conv != nullptr && conv[g]) return;
  const int p = na.prob[g], j = na.jnode[g];
  const ProbDesc& D = pd[p];
  const int n = d.n, L = D.L, ld = d.ld;
  const int nblk = (n + kSolveBlk - 1) / kSolveBlk;
  const cx<P>* __restrict__ T = Tb + d.offT;
  const int* __restrict__ rat = rows + d.offRow;
  cx<P>* __restrict__ W = Wk + D.offW0 + (long long)j * n * L;

  int rblk, qblk, dblk;
  if (LOWER) {
    rblk = s + t;
    qblk = s - 1;
    dblk = s;
  } else {
    const int cb = nblk - 1 - s;
    rblk = t;
    qblk = cb + 1;
    dblk = cb;
  }
  const int R0 = rblk * kSolveBlk, nr = min(kSolveBlk, n - R0);

  extern __shared__ unsigned char smem_raw[];
  cx<P>* Ls = reinterpret_cast<cx<P>*>(smem_raw);            // 64 x 65
  cx<P>* Xs = Ls + kSolveBlk * (kSolveBlk + 1);               // 64 x L
  constexpr int LDL = kSolveBlk + 1;

  if (s > 0) {
    const int Q0 = qblk * kSolveBlk, nq = min(kSolveBlk, n - Q0);
    for (int e = threadIdx.x; e < kSolveBlk * kSolveBlk; e += kSolveThreads) {
      const int i = e / kSolveBlk, k = e - i * kSolveBlk;
      Ls[i * LDL + k] = (i < nr && k < nq) ? T[(long long)rat[R0 + i] * ld + Q0 + k] : cx<P>{P(0), P(0)};
    }
    for (int e = threadIdx.x; e < kSolveBlk * L; e += kSolveThreads) {
      const int k = e / L;
      Xs[e] = (k < nq) ? W[(long long)Q0 * L + e] : cx<P>{P(0), P(0)};
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nr * L; e += kSolveThreads) {
      const int i = e / L, c = e - i * L;
      cx<P> acc = W[(long long)R0 * L + e];
#pragma unroll 8
      for (int k = 0; k < kSolveBlk; ++k) acc = fms(acc, Ls[i * LDL + k], Xs[k * L + c]);
      W[(long long)R0 * L + e] = acc;
    }
  }
  if (rblk != dblk) return;
  __syncthreads();
  // diagonal block solve
  for (int e = threadIdx.x; e < kSolveBlk * kSolveBlk; e += kSolveThreads) {
    const int i = e / kSolveBlk, k = e - i * kSolveBlk;
    cx<P> val = {P(0), P(0)};
    if (i < nr && k < nr && (LOWER ? (k < i) : (k >= i))) val = T[(long long)rat[R0 + i] * ld + R0 + k];
    Ls[i * LDL + k] = val;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = wave; c < L; c += kSolveThreads / 64) {
    cx<P> x = (lane < nr) ? W[(long long)(R0 + lane) * L + c] : cx<P>{P(0), P(0)};
    if (LOWER) {
      for (int q = 0; q < nr; ++q) {
        cx<P> xs;
        xs.re = __shfl(x.re, q, 64);
        xs.im = __shfl(x.im, q, 64);
        if (lane > q) x = fms(x, Ls[lane * LDL + q], xs);
      }
    } else {
      for (int q = nr - 1; q >= 0; --q) {
        if (lane == q) x = cdivp(x, Ls[q * LDL + q]);
        cx<P> xs;
        xs.re = __shfl(x.re, q, 64);
        xs.im = __shfl(x.im, q, 64);
        if (lane < q) x = fms(x, Ls[lane * LDL + q], xs);
      }
    }
    if (lane < nr) W[(long long)(R0 + lane) * L + c] = x;
  }
}

// ---------------------------------------------------------------------------
template <typename P>
static size_t step_lds(int Lmax) {
  return (size_t)(kSolveBlk * (kSolveBlk + 1) + kSolveBlk * Lmax) * sizeof(cx<P>);
}

template <typename P>
hipError_t solve_run(const SolvePlan& sp, const int* d_prefix, const ProbDesc* pd, const MatDesc* md,
                     const NodeArrays& na, const cx<P>* T, const int* rows, cx<P>* Wk, const c128* R, c128* Y,
                     bool refine, const int* conv, IrState ir, int Lmax, hipStream_t st) {
  const Table& tg = sp.gather;
  if (tg.total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_solve_gather<P>, dim3(xcd_grid(tg.total)), dim3(kSolveThreads), 0, st, md,
                     d_prefix + tg.off, tg.cnt, tg.total, pd, na, rows, Wk, R, refine ? 1 : 0, conv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = step_lds<P>(Lmax);
  for (int s = 0; s < sp.nblk_max; ++s) {
    const Table& t = sp.fwd[s];
    hipLaunchKernelGGL((k_solve_step<P, true>), dim3(xcd_grid(t.total)), dim3(kSolveThreads), lds, st, md,
                       d_prefix + t.off, t.cnt, t.total, s, pd, na, T, rows, Wk, conv);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  for (int s = 0; s < sp.nblk_max; ++s) {
    const Table& t = sp.bwd[s];
    hipLaunchKernelGGL((k_solve_step<P, false>), dim3(xcd_grid(t.total)), dim3(kSolveThreads), lds, st, md,
                       d_prefix + t.off, t.cnt, t.total, s, pd, na, T, rows, Wk, conv);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_solve_scatter<P>, dim3(xcd_grid(tg.total)), dim3(kSolveThreads), 0, st, md,
                     d_prefix + tg.off, tg.cnt, tg.total, pd, na, Wk, Y, refine ? 1 : 0, conv, ir);
  return hipGetLastError();
}

template hipError_t solve_run<float>(const SolvePlan&, const int*, const ProbDesc*, const MatDesc*,
                                     const NodeArrays&, const c64*, const int*, c64*, const c128*, c128*, bool,
                                     const int*, IrState, int, hipStream_t);
template hipError_t solve_run<double>(const SolvePlan&, const int*, const ProbDesc*, const MatDesc*,
                                      const NodeArrays&, const c128*, const int*, c128*, const c128*, c128*, bool,
                                      const int*, IrState, int, hipStream_t);

void SolvePlan_build(SolvePlan& sp, std::vector<int>& buf, const std::vector<MatDesc>& sorted,
                     const std::vector<int>& Lof) {
  // Lof[b]: probe count of sorted matrix b
  std::vector<int> cnt;
  for (size_t b = 0; b < sorted.size(); ++b) cnt.push_back(ceil_div(sorted[b].n * Lof[b], kSolveThreads));
  build_prefix(buf, sp.gather, cnt);
  sp.nblk_max = sorted.empty() ? 0 : ceil_div(sorted[0].n, kSolveBlk);
  sp.fwd.assign(sp.nblk_max, Table());
  sp.bwd.assign(sp.nblk_max, Table());
  for (int s = 0; s < sp.nblk_max; ++s) {
    std::vector<int> c2;
    for (size_t b = 0; b < sorted.size(); ++b) {
      const int nb = ceil_div(sorted[b].n, kSolveBlk);
      if (nb <= s) break;
      c2.push_back(nb - s);
    }
    build_prefix(buf, sp.fwd[s], c2);
    sp.bwd[s] = sp.fwd[s];
  }
}

hipError_t solve_configure() {
  hipError_t e = hipFuncSetAttribute((const void*)k_solve_step<float, true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, step_lds<float>(64));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_solve_step<float, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          step_lds<float>(64));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_solve_step<double, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          step_lds<double>(64));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_solve_step<double, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             step_lds<double>(64));
}

}  // namespace nep
