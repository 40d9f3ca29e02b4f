// Batched triangular solves with the factors of k_lu_*: Y_j = T(z_j)^{-1} B,
// with P T = L U (P through the row map), B the probe block V or a
// refinement residual R.
//
//   k_diag_inv : after each factorization, the 64 x 64 diagonal blocks of L
//                (unit lower) and U are inverted once, in FP64, and stored in
//                the factor precision.  One group per block; one wave per
//                column of the inverse with the rows spread over the lanes.
//   k_trsv     : one launch per solve.  A group owns one node and a group of
//                Lg right-hand columns and runs forward then backward
//                substitution over 64-row blocks: each block first gathers the
//                products of the finished part (the four waves split the
//                inner dimension, then reduce through LDS), then multiplies by
//                the stored inverse of its diagonal block.  The right-hand
//                side is gathered through the row map on the fly; the result
//                is stored to (or, for a correction, added to) Y in FP64,
//                together with the column maxima of |Y| for the refinement test.
#include "engine.hpp"

namespace nep {

constexpr int kTrsvThreads = 256;
constexpr int kInvBlk = kSolveBlk;  // 64

// ---------------------------------------------------------------------------
// Diagonal-block inverses.  Dinv layout per matrix: [blk][which][64][64]
// (which 0: L^{-1}, 1: U^{-1}), row-major, padded with the identity.
// ---------------------------------------------------------------------------
template <typename P>
__global__ __launch_bounds__(256) void k_diag_inv(const MatDesc* __restrict__ md, const int* __restrict__ prefix,
                                                  int cnt, int total, const cx<P>* __restrict__ Tb,
                                                  const int* __restrict__ rows, cx<P>* __restrict__ Dinv,
                                                  const long long* __restrict__ dinv_off,
                                                  const int* __restrict__ skip) {
  const int v = xcd_remap(blockIdx.x, gridDim.x, total);
  if (v < 0) return;
  const int b = find_slot(prefix, cnt, v);
  const int t = v - prefix[b];
  const MatDesc d = md[b];
  if (skip != nullptr && skip[d.node]) return;
  const int blk = t >> 1, which = t & 1;
  const int n = d.n, ld = d.ld;
  const int R0 = blk * kInvBlk, nr = min(kInvBlk, n - R0);
  const cx<P>* __restrict__ T = Tb + d.offT;
  const int* __restrict__ rat = rows + d.offRow;
  __shared__ c128 A[kInvBlk][kInvBlk + 1];
  for (int e = threadIdx.x; e < kInvBlk * kInvBlk; e += 256) {
    const int i = e / kInvBlk, k = e - i * kInvBlk;
    c128 val = {0.0, 0.0};
    if (i < nr && k < nr) {
      const bool keep = which == 0 ? (k < i) : (k >= i);
      if (keep) {
        const cx<P> x = T[(long long)rat[R0 + i] * ld + R0 + k];
        val = c128{double(x.re), double(x.im)};
      }
    } else if (which == 1 && i == k) {
      val = c128{1.0, 0.0};  // identity padding of U
    }
    A[i][k] = val;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  cx<P>* __restrict__ out = Dinv + dinv_off[b] + ((long long)blk * 2 + which) * kInvBlk * kInvBlk;
  for (int c = wave; c < kInvBlk; c += 4) {
    c128 x = {lane == c ? 1.0 : 0.0, 0.0};
    if (which == 0) {
      for (int s = c; s < kInvBlk; ++s) {
        c128 xs;
        xs.re = __shfl(x.re, s, 64);
        xs.im = __shfl(x.im, s, 64);
        if (lane > s) x = fms(x, A[lane][s], xs);
      }
    } else {
      for (int s = c; s >= 0; --s) {
        if (lane == s) x = cdiv(x, A[s][s]);
        c128 xs;
        xs.re = __shfl(x.re, s, 64);
        xs.im = __shfl(x.im, s, 64);
        if (lane < s) x = fms(x, A[lane][s], xs);
      }
    }
    out[lane * kInvBlk + c] = cx<P>{P(x.re), P(x.im)};
  }
}

// ---------------------------------------------------------------------------
// Fused forward + backward substitution.
// ---------------------------------------------------------------------------
template <typename P, int LG>
__global__ __launch_bounds__(kTrsvThreads) void k_trsv(const MatDesc* __restrict__ md, int nmat, int groups,
                                                      const ProbDesc* __restrict__ pd, NodeArrays na,
                                                      const cx<P>* __restrict__ Tb, const int* __restrict__ rows,
                                                      const cx<P>* __restrict__ Dinv,
                                                      const long long* __restrict__ dinv_off, cx<P>* __restrict__ Wk,
                                                      const c128* __restrict__ R, c128* __restrict__ Y, int refine,
                                                      const int* __restrict__ conv, IrState ir) {
  const int b = blockIdx.x / groups, grp = blockIdx.x - b * groups;
  if (b >= nmat) return;
  const MatDesc d = md[b];
  const int g = d.node;
  if (conv != nullptr && conv[g]) return;
  const int p = na.prob[g], j = na.jnode[g];
  const ProbDesc& D = pd[p];
  const int n = d.n, ld = d.ld, L = D.L;
  const int c0 = grp * LG;
  const int nc = min(LG, L - c0);
  if (nc <= 0) return;
  const cx<P>* __restrict__ T = Tb + d.offT;
  const int* __restrict__ rat = rows + d.offRow;
  const cx<P>* __restrict__ Di = Dinv + dinv_off[b];
  cx<P>* __restrict__ W = Wk + D.offW0 + (long long)j * n * L;  // n x L, row-major
  const int nblk = (n + kSolveBlk - 1) / kSolveBlk;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  __shared__ cx<P> red[3][kSolveBlk][LG];
  __shared__ double cmax[4][LG];

  double ymax[LG];
#pragma unroll
  for (int c = 0; c < LG; ++c) ymax[c] = 0.0;

  for (int pass = 0; pass < 2; ++pass) {  // 0: L y = P b, 1: U x = y
    for (int qq = 0; qq < nblk; ++qq) {
      const int q = pass == 0 ? qq : nblk - 1 - qq;
      const int R0 = q * kSolveBlk, nr = min(kSolveBlk, n - R0);
      const int row = R0 + lane;
      // inner dimension of the finished part, split over the four waves
      const int s_lo = pass == 0 ? 0 : R0 + nr;
      const int s_hi = pass == 0 ? R0 : n;
      cx<P> acc[LG];
#pragma unroll
      for (int c = 0; c < LG; ++c) acc[c] = cx<P>{P(0), P(0)};
      if (lane < nr && s_hi > s_lo) {
        const cx<P>* __restrict__ trow = T + (long long)rat[row] * ld;
        for (int s = s_lo + wave; s < s_hi; s += 4) {
          const cx<P> a = trow[s];
          const cx<P>* __restrict__ ys = W + (long long)s * L + c0;
#pragma unroll
          for (int c = 0; c < LG; ++c)
            if (c < nc) acc[c] = acc[c] + a * ys[c];
        }
      }
      if (wave > 0) {
#pragma unroll
        for (int c = 0; c < LG; ++c) red[wave - 1][lane][c] = acc[c];
      }
      __syncthreads();
      // right-hand side of the block: t = rhs - sum
      if (wave == 0) {
#pragma unroll
        for (int c = 0; c < LG; ++c) {
          cx<P> tv = {P(0), P(0)};
          if (lane < nr && c < nc) {
            cx<P> rhs;
            if (pass == 0) {
              const int pr = rat[row];
              const c128 bv = refine ? R[D.offY + (long long)pr * D.N * L + (long long)j * L + c0 + c]
                                     : D.V[(long long)(c0 + c) * n + pr];
              rhs = cvt<P>(bv);
            } else {
              rhs = W[(long long)row * L + c0 + c];
            }
            tv = rhs - (acc[c] + red[0][lane][c] + red[1][lane][c] + red[2][lane][c]);
          }
          red[0][lane][c] = tv;
        }
      }
      __syncthreads();
      // x_q = Dinv_q t, rows over lanes, columns over waves
      const cx<P>* __restrict__ inv = Di + ((long long)q * 2 + pass) * kSolveBlk * kSolveBlk + lane * kSolveBlk;
#pragma unroll
      for (int c = 0; c < LG; ++c) {
        if ((c & 3) == wave && c < nc && lane < nr) {
          cx<P> x = {P(0), P(0)};
          for (int k = 0; k < nr; ++k) x = x + inv[k] * red[0][k][c];
          W[(long long)row * L + c0 + c] = x;
          if (pass == 1) {
            c128* y = Y + D.offY + (long long)row * D.N * L + (long long)j * L + c0 + c;
            c128 nv = {double(x.re), double(x.im)};
            if (refine) nv = *y + nv;
            *y = nv;
            ymax[c] = fmax(ymax[c], sqrt(norm2(nv)));
          }
        }
      }
      __syncthreads();
    }
  }
  // column maxima of the new Y
#pragma unroll
  for (int c = 0; c < LG; ++c) {
    double m = ymax[c];
    for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0) cmax[wave][c] = m;
  }
  __syncthreads();
  if (threadIdx.x < nc) {
    const int c = threadIdx.x;
    const double m = fmax(fmax(cmax[0][c], cmax[1][c]), fmax(cmax[2][c], cmax[3][c]));
    atomicMax(&ir.ynorm[(long long)g * kNormStride + c0 + c], (unsigned long long)__double_as_longlong(m));
  }
}

// ---------------------------------------------------------------------------
template <typename P>
hipError_t diag_inv_run(const SolvePlan& sp, const int* d_prefix, const MatDesc* md, const cx<P>* T,
                        const int* rows, cx<P>* Dinv, const long long* dinv_off, const int* skip, hipStream_t st) {
  const Table& t = sp.diag;
  if (t.total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_inv<P>, dim3(xcd_grid(t.total)), dim3(256), 0, st, md, d_prefix + t.off, t.cnt, t.total,
                     T, rows, Dinv, dinv_off, skip);
  return hipGetLastError();
}

template <typename P>
hipError_t solve_run(const SolvePlan& sp, const ProbDesc* pd, const MatDesc* md, const NodeArrays& na,
                     const cx<P>* T, const int* rows, const cx<P>* Dinv, const long long* dinv_off, cx<P>* Wk,
                     const c128* R, c128* Y, bool refine, const int* conv, IrState ir, hipStream_t st) {
  if (sp.nmat == 0) return hipSuccess;
  const dim3 grid(sp.nmat * sp.groups), blk(kTrsvThreads);
  const int rf = refine ? 1 : 0;
  switch (sp.lg) {
    case 2: hipLaunchKernelGGL((k_trsv<P, 2>), grid, blk, 0, st, md, sp.nmat, sp.groups, pd, na, T, rows, Dinv,
                               dinv_off, Wk, R, Y, rf, conv, ir); break;
    case 4: hipLaunchKernelGGL((k_trsv<P, 4>), grid, blk, 0, st, md, sp.nmat, sp.groups, pd, na, T, rows, Dinv,
                               dinv_off, Wk, R, Y, rf, conv, ir); break;
    case 8: hipLaunchKernelGGL((k_trsv<P, 8>), grid, blk, 0, st, md, sp.nmat, sp.groups, pd, na, T, rows, Dinv,
                               dinv_off, Wk, R, Y, rf, conv, ir); break;
    default: hipLaunchKernelGGL((k_trsv<P, 16>), grid, blk, 0, st, md, sp.nmat, sp.groups, pd, na, T, rows, Dinv,
                                dinv_off, Wk, R, Y, rf, conv, ir); break;
  }
  return hipGetLastError();
}

template hipError_t diag_inv_run<float>(const SolvePlan&, const int*, const MatDesc*, const c64*, const int*, c64*,
                                        const long long*, const int*, hipStream_t);
template hipError_t diag_inv_run<double>(const SolvePlan&, const int*, const MatDesc*, const c128*, const int*,
                                         c128*, const long long*, const int*, hipStream_t);
template hipError_t solve_run<float>(const SolvePlan&, const ProbDesc*, const MatDesc*, const NodeArrays&, const c64*,
                                     const int*, const c64*, const long long*, c64*, const c128*, c128*, bool,
                                     const int*, IrState, hipStream_t);
template hipError_t solve_run<double>(const SolvePlan&, const ProbDesc*, const MatDesc*, const NodeArrays&,
                                      const c128*, const int*, const c128*, const long long*, c128*, const c128*,
                                      c128*, bool, const int*, IrState, hipStream_t);

// Column-group size: enough groups to occupy the device when there are few
// matrices, bounded by L (the group is an unrolled register tile).
static int pick_lg(int nmat, int L) {
  int lg = 16;
  while (lg > 2 && (lg >= 2 * L || (long long)nmat * ceil_div(L, lg) < 512)) lg >>= 1;
  return lg;
}

void SolvePlan_build(SolvePlan& sp, std::vector<int>& buf, const std::vector<MatDesc>& sorted, int L,
                     std::vector<long long>& dinv_off, long long& dinv_elems) {
  sp.nmat = (int)sorted.size();
  sp.lg = pick_lg(sp.nmat, L);
  sp.groups = ceil_div(L, sp.lg);
  std::vector<int> cnt;
  dinv_off.clear();
  long long off = 0;
  for (const auto& m : sorted) {
    const int nb = ceil_div(m.n, kSolveBlk);
    cnt.push_back(2 * nb);
    dinv_off.push_back(off);
    off += (long long)nb * 2 * kSolveBlk * kSolveBlk;
  }
  dinv_elems = off;
  build_prefix(buf, sp.diag, cnt);
}

hipError_t solve_configure() { return hipSuccess; }

}  // namespace nep
