// Batched triangular solves with the factors of k_lu_*: Y_j = T(z_j)^{-1} B,
// with P T = L U (P through the row map), B the probe block V or a
// refinement residual R.
//
// The LU writes, as its panels complete, the inverses of the 64 x 64 diagonal
// blocks of L (unit lower) and U.  k_trsv runs one launch per solve: a group
// owns one node and a group of Lg right-hand columns and runs forward then
// backward substitution over 64-row blocks (right-looking, accumulators in
// registers; see the kernel).  The right-hand side is gathered through the
// row map; the result is stored to (or, for a correction, added to) Y in
// FP64, with the column maxima of |Y| for the refinement test.
#include "engine.hpp"

namespace nep {

// Threads per group: 512 for matrices of more than 512 rows, 256 below
// (two rows per thread up to 512 rows, one up to 256), so that small matrices
// of a ragged batch do not leave most of a large group idle.
constexpr int kTrsvThreads = 512, kTrsvThreadsSmall = 256;

// ---------------------------------------------------------------------------
// Right-looking substitution with the accumulators in registers: thread t
// owns the logical rows t, t+512, ...  For each 64-row block (in order for
// L, reversed for U):
//   1. the owners of the block's rows publish t = acc (their pending sums)
//      and the group stages the stored inverse of the diagonal block;
//   2. x_q = Dinv_q t (all threads, 64 rows x LG columns);
//   3. every row not yet solved pulls its 64-wide segment of the factor and
//      subtracts segment * x_q from its accumulators.
// Step 3 issues many independent row loads, so the solve streams the factor
// instead of waiting on one dependent chain.
// 16 consecutive elements of a factor row; the segment starts at a multiple
// of 64 elements of a row whose stride is a multiple of 16, so it is 16-byte
// aligned.
__device__ __forceinline__ void load_seg16(const c64* __restrict__ s, c64 (&v)[16]) {
  const float4* q = reinterpret_cast<const float4*>(s);
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const float4 t = q[u];
    v[2 * u] = {t.x, t.y};
    v[2 * u + 1] = {t.z, t.w};
  }
}
__device__ __forceinline__ void load_seg16(const c128* __restrict__ s, c128 (&v)[16]) {
  const double2* q = reinterpret_cast<const double2*>(s);
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const double2 t = q[u];
    v[u] = {t.x, t.y};
  }
}

template <int Q, typename P>
__device__ __forceinline__ void load_seg(const cx<P>* __restrict__ s, cx<P> (&v)[Q]) {
  static_assert(Q % 16 == 0, "segments of 16 elements");
#pragma unroll
  for (int k = 0; k < Q; k += 16) {
    cx<P> t[16];
    load_seg16(s + k, t);
#pragma unroll
    for (int u = 0; u < 16; ++u) v[k + u] = t[u];
  }
}

// 256-thread groups with four rows per thread (the large class of big
// batches, two or more groups per CU) are held to three waves per SIMD: 168
// registers with a small spill, three groups per CU instead of two (the
// 256-problem batch 204.4 -> 203.1 ms)
template <typename P, int LG, int RPT, int NT>
__global__ __launch_bounds__(NT, (NT == 256 && RPT == 4) ? 3 : 1) void k_trsv(const MatDesc* __restrict__ md, int nmat, int groups,
                                                      const ProbDesc* __restrict__ pd, NodeArrays na,
                                                      const cx<P>* __restrict__ Tb, const int* __restrict__ rows,
                                                      const cx<P>* __restrict__ Dinv,
                                                      const long long* __restrict__ dinv_off,
                                                      const c128* __restrict__ R, c128* __restrict__ Y, int refine,
                                                      const int* __restrict__ conv, IrState ir) {
  constexpr int B = kSolveBlk;  // 64
  // register budget (32-bit words per thread) of the prefetched segment
  // columns (PF per row) and of the rows whose 16-column chunks load together
  // (GR): accumulators + prefetch + one chunk per grouped row stay within it
  constexpr int FW = 2 * (int)(sizeof(P) / 4);  // words per complex
  constexpr int kBudget = sizeof(P) == 8 ? 112 : 176;
  constexpr int PF = RPT * FW * (32 + 16 + LG) <= kBudget   ? 32
                     : RPT * FW * (16 + 16 + LG) <= kBudget ? 16
                                                            : 0;
  constexpr int GR = RPT * FW * (PF + 16 + LG) <= kBudget ? RPT : 1;
  // full blocks as a pipeline of 16-column chunks in two register buffers
  // (the prefetched first chunk is one of them): each chunk's loads are in
  // flight while the previous chunk is applied
  constexpr bool PIPE = PF == 16 && RPT * FW * (2 * 16 + LG) <= 160;
  // the column groups of one matrix run on one XCD and share its L2
  const int v = xcd_remap(blockIdx.x, gridDim.x, nmat * groups);
  if (v < 0) return;
  const int b = v / groups, grp = v - b * groups;
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
  const int nblk = (n + B - 1) / B;
  const int tid = threadIdx.x;

  __shared__ cx<P> Ds[B][B + 1];   // diagonal-block inverse
  __shared__ cx<P> Ts[B][LG];      // block right-hand side
  __shared__ cx<P> Xs[B][LG];      // block solution
  __shared__ double cmax[NT / 64][LG];

  // rows of this thread: slot i holds row i*T + tid (i even) or
  // (i+1)*T - 1 - tid (i odd), so every thread has rows from both ends and
  // the pending rows of a block are spread evenly over the waves
  auto row_of = [&](int i) { return (i & 1) ? (i + 1) * NT - 1 - tid : i * NT + tid; };
  // right-hand side P b gathered into the owners' accumulators
  cx<P> acc[RPT][LG];
  long long rowoff[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = row_of(i);
    const int pr = r < n ? rat[r] : 0;
    rowoff[i] = (long long)pr * ld;
#pragma unroll
    for (int c = 0; c < LG; ++c) {
      c128 bv = {0.0, 0.0};
      if (r < n && c < nc)
        bv = refine ? R[D.offY + (long long)pr * D.N * L + (long long)j * L + c0 + c] : D.V[(long long)(c0 + c) * n + pr];
      acc[i][c] = cvt<P>(bv);
    }
  }
  double ymax[LG];
#pragma unroll
  for (int c = 0; c < LG; ++c) ymax[c] = 0.0;

  constexpr int DPT = B * B / NT;  // inverse elements per thread
  static_assert(DPT * NT == B * B, "inverse staging");
  cx<P> dreg[DPT];
#pragma unroll
  for (int u = 0; u < DPT; ++u) {  // block 0 of L
    const cx<P>* src = Di + tid + u * NT;
    dreg[u] = cx<P>{src->re, src->im};
  }
  for (int pass = 0; pass < 2; ++pass) {  // 0: L y = P b, 1: U x = y
    for (int qq = 0; qq < nblk; ++qq) {
      const int q = pass == 0 ? qq : nblk - 1 - qq;
      const int R0 = q * B, nr = min(B, n - R0);
      // 0. the factor segments of the pending rows do not depend on this
      // block's solution: the first PF columns are loaded now and arrive
      // while the block is solved
      cx<P> pre[RPT][PF > 0 ? PF : 1];
      if constexpr (PF > 0) {
        if (nr == B) {
#pragma unroll
          for (int i = 0; i < RPT; ++i) {
            const int r = row_of(i);
            if (r < n && (pass == 0 ? r >= R0 + B : r < R0)) load_seg<PF>(T + rowoff[i] + R0, pre[i]);
          }
        }
      }
      // 1. publish the block's pending sums; stage the inverse
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = row_of(i);
        if (r >= R0 && r < R0 + B) {
#pragma unroll
          for (int c = 0; c < LG; ++c) Ts[r - R0][c] = r < n ? acc[i][c] : cx<P>{P(0), P(0)};
        }
      }
      // the block's inverse arrived in registers during the previous block
      // (identity-padded past nr, so no masking is needed)
#pragma unroll
      for (int u = 0; u < DPT; ++u) {
        const int e = tid + u * NT;
        Ds[e / B][e % B] = cx<P>{dreg[u].re, dreg[u].im};
      }
      __syncthreads();
      // 2. x_q = Dinv_q t
      for (int e = tid; e < B * LG; e += NT) {
        const int i = e / LG, c = e - i * LG;
        cx<P> x = {P(0), P(0)};
#pragma unroll 16
        for (int k = 0; k < B; ++k) x = cmac(x, Ds[i][k], Ts[k][c]);
        Xs[i][c] = x;
      }
      __syncthreads();
      // prefetch the next block's inverse (forward order in pass 0, then
      // backward in pass 1)
      {
        const bool last = pass == 1 && qq + 1 == nblk;
        const int nq = pass == 0 ? (qq + 1 < nblk ? q + 1 : nblk - 1) : q - 1;
        const int npass = (pass == 0 && qq + 1 == nblk) ? 1 : pass;
        if (!last) {
          const cx<P>* __restrict__ nx = Di + ((long long)nq * 2 + npass) * B * B;
#pragma unroll
          for (int u = 0; u < DPT; ++u) {
            const cx<P>* src = nx + tid + u * NT;
            dreg[u] = cx<P>{src->re, src->im};
          }
        }
      }
      // 3. rows still pending subtract (factor segment) * x_q; the block's own
      // rows take their solution
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = row_of(i);
        if (r >= n) continue;
        if (r >= R0 && r < R0 + nr) {
#pragma unroll
          for (int c = 0; c < LG; ++c) acc[i][c] = Xs[r - R0][c];
          continue;
        }
        const bool pending = pass == 0 ? r >= R0 + nr : r < R0;
        if (!pending) continue;
        const cx<P>* __restrict__ seg = T + rowoff[i] + R0;
        if (nr == B && PIPE) continue;  // applied by the pipeline below
        if (nr == B) {  // full block: prefetched part first
#pragma unroll
          for (int u = 0; u < PF; ++u)
#pragma unroll
            for (int c = 0; c < LG; ++c) acc[i][c] = fms(acc[i][c], pre[i][u], Xs[u][c]);
        } else {  // ragged last block
          for (int k = 0; k < nr; ++k) {
            const cx<P> lv = seg[k];
#pragma unroll
            for (int c = 0; c < LG; ++c) acc[i][c] = fms(acc[i][c], lv, Xs[k][c]);
          }
        }
      }
      if constexpr (PIPE) {
        if (nr == B) {
          bool pend[RPT];
#pragma unroll
          for (int i = 0; i < RPT; ++i) {
            const int r = row_of(i);
            pend[i] = r < n && (pass == 0 ? r >= R0 + B : r < R0);
          }
          cx<P> nb[RPT][16];
          auto issue = [&](cx<P> (&buf)[RPT][PF > 0 ? PF : 1], int k0) {
#pragma unroll
            for (int i = 0; i < RPT; ++i)
              if (pend[i]) load_seg16(T + rowoff[i] + R0 + k0, reinterpret_cast<cx<P>(&)[16]>(buf[i]));
          };
          auto issue_nb = [&](int k0) {
#pragma unroll
            for (int i = 0; i < RPT; ++i)
              if (pend[i]) load_seg16(T + rowoff[i] + R0 + k0, nb[i]);
          };
          auto apply_pre = [&](int k0) {
#pragma unroll
            for (int i = 0; i < RPT; ++i)
              if (pend[i]) {
#pragma unroll
                for (int u = 0; u < 16; ++u)
#pragma unroll
                  for (int c = 0; c < LG; ++c) acc[i][c] = fms(acc[i][c], pre[i][u], Xs[k0 + u][c]);
              }
          };
          auto apply_nb = [&](int k0) {
#pragma unroll
            for (int i = 0; i < RPT; ++i)
              if (pend[i]) {
#pragma unroll
                for (int u = 0; u < 16; ++u)
#pragma unroll
                  for (int c = 0; c < LG; ++c) acc[i][c] = fms(acc[i][c], nb[i][u], Xs[k0 + u][c]);
              }
          };
          issue_nb(16);
          apply_pre(0);
          issue(pre, 32);
          apply_nb(16);
          issue_nb(48);
          apply_pre(32);
          apply_nb(48);
        }
      }
      // rest of the full-block segments, 16 columns at a time, every row's
      // loads issued together
      if (!PIPE && nr == B) {
#pragma unroll
        for (int i0 = 0; i0 < RPT; i0 += GR) {
          for (int k0 = PF; k0 < B; k0 += 16) {
            cx<P> lv[GR][16];
#pragma unroll
            for (int g = 0; g < GR; ++g) {
              const int r = row_of(i0 + g);
              if (r < n && (pass == 0 ? r >= R0 + B : r < R0)) load_seg16(T + rowoff[i0 + g] + R0 + k0, lv[g]);
            }
#pragma unroll
            for (int g = 0; g < GR; ++g) {
              const int r = row_of(i0 + g);
              const bool pending = r < n && (pass == 0 ? r >= R0 + B : r < R0);
              if (pending) {
#pragma unroll
                for (int u = 0; u < 16; ++u)
#pragma unroll
                  for (int c = 0; c < LG; ++c) acc[i0 + g][c] = fms(acc[i0 + g][c], lv[g][u], Xs[k0 + u][c]);
              }
            }
          }
        }
      }
      // (the next block's barrier after step 1 orders Xs reuse)
    }
    __syncthreads();
  }
  // acc now holds x for the owned rows: store to Y (FP64) and take maxima
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = row_of(i);
    if (r < n) {
      c128* y = Y + D.offY + (long long)r * D.N * L + (long long)j * L + c0;
#pragma unroll
      for (int c = 0; c < LG; ++c) {
        if (c < nc) {
          c128 nv = {double(acc[i][c].re), double(acc[i][c].im)};
          if (refine) nv = y[c] + nv;
          y[c] = nv;
          ymax[c] = nanmax(ymax[c], sqrt(norm2(nv)));
        }
      }
    }
  }
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int c = 0; c < LG; ++c) {
    double m = ymax[c];
    for (int o = 32; o >= 1; o >>= 1) m = nanmax(m, __shfl_xor(m, o, 64));
    if (lane == 0) cmax[wave][c] = m;
  }
  __syncthreads();
  if (tid < nc) {
    double m = 0.0;
    for (int w = 0; w < NT / 64; ++w) m = nanmax(m, cmax[w][tid]);
    atomicMax(&ir.ynorm[(long long)g * kNormStride + c0 + tid], (unsigned long long)__double_as_longlong(m));
  }
}

// ---------------------------------------------------------------------------

template <typename P, int LG, int RPT, int NT>
static void launch_trsv_class(const SolvePlan& sp, int b0, int cnt, const ProbDesc* pd, const MatDesc* md,
                              const NodeArrays& na, const cx<P>* T, const int* rows, const cx<P>* Dinv,
                              const long long* dinv_off, const c128* R, c128* Y, int rf, const int* conv, IrState ir,
                              hipStream_t st) {
  if (cnt <= 0) return;
  hipLaunchKernelGGL((k_trsv<P, LG, RPT, NT>), dim3(xcd_grid(cnt * sp.groups)), dim3(NT), 0, st, md + b0, cnt,
                     sp.groups, pd, na, T, rows, Dinv, dinv_off + b0, R, Y, rf, conv, ir);
}

// One launch per size class of the (size-sorted) matrices: more than 512
// rows (512 threads, sp.rpt rows each), 257..512 rows and up to 256 rows
// (256 threads, two and one rows each).
template <typename P, int LG>
static void launch_trsv(const SolvePlan& sp, const ProbDesc* pd, const MatDesc* md, const NodeArrays& na,
                        const cx<P>* T, const int* rows, const cx<P>* Dinv, const long long* dinv_off, const c128* R,
                        c128* Y, int rf, const int* conv, IrState ir, hipStream_t st) {
  // the first nblk matrices took the blocked solve (complex FP32 only)
  const int b0 = sizeof(P) == 4 ? sp.nblk : 0;
  const int nb = sp.nbig - b0, nm = sp.nmid, ns = sp.nmat - sp.nbig - sp.nmid;
  // many large matrices (several rounds of groups): 256-thread groups with
  // twice the rows each, two per CU, so one group's barrier waits are
  // covered by the other's work
  // (complex FP32 with at most 8 columns per group: two such groups fit a CU's registers)
  constexpr bool kPaired = sizeof(P) == 4 && LG <= 8;
  if (kPaired && sp.rpt <= 2 && nb > 0 && (sp.paired == 1 || (sp.paired < 0 && (long long)nb * sp.groups >= 2048))) {
    if constexpr (kPaired)
      launch_trsv_class<P, LG, 4, kTrsvThreadsSmall>(sp, b0, nb, pd, md, na, T, rows, Dinv, dinv_off, R, Y, rf, conv,
                                                     ir, st);
  } else switch (sp.rpt) {
    case 1:
    case 2: launch_trsv_class<P, LG, 2, kTrsvThreads>(sp, b0, nb, pd, md, na, T, rows, Dinv, dinv_off, R, Y, rf, conv, ir, st); break;
    case 4: launch_trsv_class<P, LG, 4, kTrsvThreads>(sp, b0, nb, pd, md, na, T, rows, Dinv, dinv_off, R, Y, rf, conv, ir, st); break;
    default: launch_trsv_class<P, LG, 8, kTrsvThreads>(sp, b0, nb, pd, md, na, T, rows, Dinv, dinv_off, R, Y, rf, conv, ir, st); break;
  }
  launch_trsv_class<P, LG, 2, kTrsvThreadsSmall>(sp, sp.nbig, nm, pd, md, na, T, rows, Dinv, dinv_off, R, Y, rf, conv, ir,
                                                 st);
  launch_trsv_class<P, LG, 1, kTrsvThreadsSmall>(sp, sp.nbig + nm, ns, pd, md, na, T, rows, Dinv, dinv_off, R, Y, rf,
                                                 conv, ir, st);
}

template <typename P>
hipError_t solve_run(const SolvePlan& sp, const ProbDesc* pd, const MatDesc* md, const NodeArrays& na,
                     const cx<P>* T, const int* rows, const cx<P>* Dinv, const long long* dinv_off,
                     const c128* R, c128* Y, bool refine, const int* conv, IrState ir, hipStream_t st) {
  if (sp.nmat == 0) return hipSuccess;
  const int rf = refine ? 1 : 0;
  if constexpr (sizeof(P) == 4) {
    if (sp.nblk > 0) {
      const hipError_t e = solve_blocked(sp, pd, md, na, T, rows, Dinv, dinv_off, R, Y, refine, conv, ir, st);
      if (e != hipSuccess) return e;
      if (sp.nblk == sp.nmat) return hipSuccess;
    }
  }
  switch (sp.lg) {
    case 4: launch_trsv<P, 4>(sp, pd, md, na, T, rows, Dinv, dinv_off, R, Y, rf, conv, ir, st); break;
    case 8: launch_trsv<P, 8>(sp, pd, md, na, T, rows, Dinv, dinv_off, R, Y, rf, conv, ir, st); break;
    default: launch_trsv<P, 16>(sp, pd, md, na, T, rows, Dinv, dinv_off, R, Y, rf, conv, ir, st); break;
  }
  return hipGetLastError();
}

template hipError_t solve_run<float>(const SolvePlan&, const ProbDesc*, const MatDesc*, const NodeArrays&, const c64*,
                                     const int*, const c64*, const long long*, const c128*, c128*, bool,
                                     const int*, IrState, hipStream_t);
template hipError_t solve_run<double>(const SolvePlan&, const ProbDesc*, const MatDesc*, const NodeArrays&,
                                      const c128*, const int*, const c128*, const long long*, const c128*,
                                      c128*, bool, const int*, IrState, hipStream_t);

// Column-group size: enough groups to occupy the device when there are few
// matrices, bounded by L (the group is an unrolled register tile).
static int pick_lg(int nmat, int L) {
  // Each column group re-reads the node's factor (from the XCD's L2), so
  // prefer few groups per node; split only when there are too few nodes to
  // occupy the device.
  int lg = 16;
  while (lg > 4 && lg >= 2 * L) lg >>= 1;
  while (lg > 4 && (long long)nmat * ceil_div(L, lg) < 256) lg >>= 1;
  return lg;
}

void SolvePlan_build(SolvePlan& sp, std::vector<int>& /*buf*/, const std::vector<MatDesc>& sorted, int L, int prec,
                     std::vector<long long>& dinv_off, long long& dinv_elems) {
  sp.nmat = (int)sorted.size();
  const int nmax = sorted.empty() ? 0 : sorted[0].n;
  sp.rpt = nmax <= 512 ? 1 : nmax <= 1024 ? 2 : nmax <= 2048 ? 4 : 8;  // rows per thread of the 512-thread class
  sp.nbig = sp.nmid = 0;
  for (const auto& m : sorted) {
    if (m.n > 2 * kTrsvThreadsSmall) ++sp.nbig;
    else if (m.n > kTrsvThreadsSmall) ++sp.nmid;
  }
  // complex FP32 with an even number (at most 64) of right-hand sides: the
  // matrices of at least kSolveBlockedMinN rows take the blocked solve
  sp.nblk = 0;
  sp.L = L;
  if (prec != NEP_PREC_FP64 && L % 2 == 0 && L <= 64)
    while (sp.nblk < sp.nmat && sorted[sp.nblk].n >= kSolveBlockedMinN) ++sp.nblk;
  sp.npad = sp.nblk > 0 ? ceil_div(sorted[0].n, kSolveBlk) * kSolveBlk : 0;
  sp.nbk = 256;
  sp.W = nullptr;
  sp.lg = pick_lg(sp.nmat - sp.nblk, L);
  while (sp.lg > 4 && !solve_lg_fits(sp, sp.lg, L, prec)) sp.lg >>= 1;
  sp.groups = ceil_div(L, sp.lg);
  sp.paired = -1;
  dinv_off.clear();
  long long off = 0;
  for (const auto& m : sorted) {
    const int nb = ceil_div(m.n, kSolveBlk);
    dinv_off.push_back(off);
    off += (long long)nb * 2 * kSolveBlk * kSolveBlk;
  }
  dinv_elems = off;
}

bool solve_lg_fits(const SolvePlan& sp, int lg, int L, int prec) {
  if (lg != 4 && lg != 8 && lg != 16) return false;
  if (lg == 4) return true;  // the narrowest group always fits
  // accumulators live in registers: at most 32 complex FP32 (8 complex FP64)
  // values per thread
  const int cap = prec == NEP_PREC_FP64 ? 8 : 32;
  return lg < 2 * L && sp.rpt * lg <= cap;
}

void solve_set_lg(SolvePlan& sp, int lg, int L) {
  sp.lg = lg;
  sp.groups = ceil_div(L, lg);
}

hipError_t solve_configure() { return hipSuccess; }

}  // namespace nep
