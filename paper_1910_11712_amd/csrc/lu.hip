// Batched complex LU with partial pivoting (P T = L U) for gfx950.
//
// The factorizations of T(z_j) at every quadrature node (and, for batches, of
// every problem) are the dominant cost of the contour-integral path; the
// paper likewise reports factorizations as the dominant cost of its solvers
// (Sections 4 and 5, and the "PC build" column of its accuracy table).
//
// Storage: every matrix is row-major with leading dimension ld.  Pivoting is
// done through a logical-to-physical row map (row_at); no row is ever moved,
// so every kernel reads logical row r from physical row row_at[r].  Rows are
// contiguous, so gathered row segments stay coalesced.
//
// Right-looking blocked algorithm, one step per panel of jb columns:
//   k_lu_panel : one work-group per matrix factors the n-k0 by jb panel; leaves
//                of W columns live in registers (one logical row per thread and
//                slot), loaded and stored through LDS in whole-row pieces;
//                pivots are found by DPP wave reductions and one LDS atomic
//                max, modulus |Re|+|Im|, ties to the lowest row.  At its end
//                the group inverts the unit lower block L11 (recursive
//                doubling in LDS), used for U12 and, block by block, by the
//                solves.
//   k_lu_inv_u : inverses of the 64 x 64 diagonal blocks of U11 (FP64).
//   k_lu_part0_c64: U12 and the update of the first 64 trailing columns (the
//                next panel's) in one launch, complex FP32.
//   k_lu_gemm<1>: U12 = L11^{-1} A12 on the matrix cores (block-row solve).
//   k_lu_gemm<0>: A22 -= L21 U12 on the matrix cores.  Complex products use the
//                real 2x2 embedding [ar -ai; ai ar] built in the operand
//                registers, so one real MFMA k-pair is one complex k.
//                c64: v_mfma_f32_32x32x2f32, 128x128 complex tile per group.
//                c128: v_mfma_f64_16x16x4f64, 128x64 complex tile per group.
#include "lu.hpp"

#include <algorithm>
#include <climits>
#include <vector>

namespace nep {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kPanelThreads = 512;
constexpr int kPanelSmall = 256;  // threads of the panel groups of at most 256 rows
constexpr int kMaxPanelRows = 4096;  // n - k0 held by one panel group

// ---------------------------------------------------------------------------
// init: row_at = identity, info = n (no zero pivot)
// ---------------------------------------------------------------------------
__global__ void k_lu_init(const MatDesc* __restrict__ md, int nmat, int* __restrict__ rowb,
                          int* __restrict__ info) {
  const int b = blockIdx.x;
  if (b >= nmat) return;
  const MatDesc d = md[b];
  for (int r = threadIdx.x; r < d.n; r += blockDim.x) rowb[d.offRow + r] = r;
  if (threadIdx.x == 0) info[d.node] = d.n;
}

// ---------------------------------------------------------------------------
// Inverses of the panel's diagonal blocks.
//
// tri_inv_lds inverts, in place, an m x m triangular block held in LDS (row
// stride lx, m = 64 or 128) with NT threads: the 8 x 8 diagonal blocks by
// substitution (one thread per column), then neighbouring blocks are merged
// with sizes 8 -> 16 -> ... -> m.  For lower [A 0; B C] the inverse's
// off-diagonal block is -C^{-1} B A^{-1}; for upper [A B; 0 C] it is
// -A^{-1} B C^{-1}; both are formed as two products against the already
// inverted diagonal blocks.  The opposite triangle holds zeros; the diagonal
// holds 1 (unit lower) or u_ii (upper).
// ---------------------------------------------------------------------------
template <typename S>
__device__ __forceinline__ cx<S> cdiv_s(cx<S> a, cx<S> b) {
  const c128 q = cdiv(c128{double(a.re), double(a.im)}, c128{double(b.re), double(b.im)});
  return cx<S>{S(q.re), S(q.im)};
}

template <typename S, bool UPPER, int NT = 256>
__device__ void tri_inv_lds(cx<S>* X, int lx, int m) {
  constexpr int NQ = 1024 / NT;  // groups per thread
  const int tid = threadIdx.x;
  const cx<S> zero = {S(0), S(0)};
  {  // 8 x 8 diagonal blocks: thread (block, column c)
    cx<S> col[8];
    const int o = (tid >> 3) * 8, c = tid & 7;
    const bool act = tid < m;
    if (act) {
      if (!UPPER) {
#pragma unroll
        for (int i = 0; i < 8; ++i) col[i] = i == c ? cx<S>{S(1), S(0)} : zero;
#pragma unroll
        for (int i = 1; i < 8; ++i) {
          cx<S> sum = zero;
#pragma unroll
          for (int k = 0; k < i; ++k) sum = cmac(sum, X[(o + i) * lx + o + k], col[k]);
          if (i > c) col[i] = -sum;
        }
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) col[i] = zero;
#pragma unroll
        for (int i = 7; i >= 0; --i) {
          cx<S> sum = zero;
#pragma unroll
          for (int k = i + 1; k < 8; ++k) sum = cmac(sum, X[(o + i) * lx + o + k], col[k]);
          const cx<S> rhs = i == c ? cx<S>{S(1) - sum.re, -sum.im} : -sum;
          const cx<S> x = cdiv_s(rhs, X[(o + i) * lx + o + i]);
          if (i <= c) col[i] = x;
        }
      }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (UPPER ? i <= c : i >= c) X[(o + i) * lx + o + c] = col[i];
    }
    __syncthreads();
  }
  // merges: thread groups of 4 consecutive columns of one row of the
  // off-diagonal block; at most m*s/8 / NT groups per thread
  for (int s = 8; s < m; s <<= 1) {
    const int gpb = s * (s >> 2);            // groups per block pair
    const int ng = (m / (2 * s)) * gpb;
    cx<S> acc[NQ][4];
    // step 1: T = B A^{-1} (lower) or T = B C^{-1} (upper)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int g = tid + NT * q;
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[q][j] = zero;
      if (g < ng) {
        const int pr = g / gpb, rem = g - pr * gpb;
        const int r = rem / (s >> 2), c0 = (rem - r * (s >> 2)) * 4;
        const int a0 = pr * 2 * s, a1 = a0 + s;
        if (!UPPER) {
          for (int k = c0; k < s; ++k) {
            const cx<S> bv = X[(a1 + r) * lx + a0 + k];
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[q][j] = cmac(acc[q][j], bv, X[(a0 + k) * lx + a0 + c0 + j]);
          }
        } else {
          for (int k = 0; k < c0 + 4; ++k) {
            const cx<S> bv = X[(a0 + r) * lx + a1 + k];
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[q][j] = cmac(acc[q][j], bv, X[(a1 + k) * lx + a1 + c0 + j]);
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int g = tid + NT * q;
      if (g < ng) {
        const int pr = g / gpb, rem = g - pr * gpb;
        const int r = rem / (s >> 2), c0 = (rem - r * (s >> 2)) * 4;
        const int a0 = pr * 2 * s, a1 = a0 + s;
        cx<S>* dst = UPPER ? X + (a0 + r) * lx + a1 + c0 : X + (a1 + r) * lx + a0 + c0;
#pragma unroll
        for (int j = 0; j < 4; ++j) dst[j] = acc[q][j];
      }
    }
    __syncthreads();
    // step 2: -C^{-1} T (lower) or -A^{-1} T (upper)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int g = tid + NT * q;
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[q][j] = zero;
      if (g < ng) {
        const int pr = g / gpb, rem = g - pr * gpb;
        const int r = rem / (s >> 2), c0 = (rem - r * (s >> 2)) * 4;
        const int a0 = pr * 2 * s, a1 = a0 + s;
        if (!UPPER) {
          for (int k = 0; k <= r; ++k) {
            const cx<S> cv = X[(a1 + r) * lx + a1 + k];
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[q][j] = cmac(acc[q][j], cv, X[(a1 + k) * lx + a0 + c0 + j]);
          }
        } else {
          for (int k = r; k < s; ++k) {
            const cx<S> av = X[(a0 + r) * lx + a0 + k];
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[q][j] = cmac(acc[q][j], av, X[(a0 + k) * lx + a1 + c0 + j]);
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int g = tid + NT * q;
      if (g < ng) {
        const int pr = g / gpb, rem = g - pr * gpb;
        const int r = rem / (s >> 2), c0 = (rem - r * (s >> 2)) * 4;
        const int a0 = pr * 2 * s, a1 = a0 + s;
        cx<S>* dst = UPPER ? X + (a0 + r) * lx + a1 + c0 : X + (a1 + r) * lx + a0 + c0;
#pragma unroll
        for (int j = 0; j < 4; ++j) dst[j] = -acc[q][j];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Panel
// ---------------------------------------------------------------------------
template <typename P>
__device__ __forceinline__ P shfl_xor_p(P v, int m) { return __shfl_xor(v, m, 64); }

// Component-wise read / write of a complex element: whole-struct copies of
// the register-resident leaf are lowered as 64-bit moves, which keeps the
// leaf array out of registers.
template <typename P>
__device__ __forceinline__ cx<P> cget(const cx<P>& x) { return cx<P>{x.re, x.im}; }
template <typename P>
__device__ __forceinline__ void cput(cx<P>& d, const cx<P> v) { d.re = v.re; d.im = v.im; }

// Pivot key of a candidate: the bits of its modulus |Re|+|Im| (non-negative,
// so the bits order like the values) plus one, 0 for "no candidate".  FP32
// keys are exact; FP64 keys keep the high word of the double (sign, exponent
// and 20 mantissa bits), so moduli within 2^-20 of each other tie.  Ties go to
// the lowest row, which keeps the choice deterministic.
__device__ __forceinline__ unsigned pivot_key(float v) { return __float_as_uint(v) + 1u; }
__device__ __forceinline__ unsigned pivot_key(double v) {
  return (unsigned)((unsigned long long)__double_as_longlong(v) >> 32) + 1u;
}

// Maximum / minimum of a 32-bit value over the wave with DPP row operations
// (quad swaps, half-row and row mirrors, then the row broadcasts that carry
// rows 0-2 into row 3); lane 63 holds the result, returned uniform.  Lanes a
// broadcast does not reach keep their value (the "old" operand is the
// operation's identity).
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  int x = (int)v;
  auto mx = [](int a, int b) { return (int)max((unsigned)a, (unsigned)b); };
  x = mx(x, __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
  x = mx(x, __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
  x = mx(x, __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false));  // row_half_mirror
  x = mx(x, __builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false));  // row_mirror
  x = mx(x, __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false));  // row_bcast15 -> rows 1, 3
  x = mx(x, __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false));  // row_bcast31 -> rows 2, 3
  return (unsigned)__builtin_amdgcn_readlane(x, 63);
}
__device__ __forceinline__ unsigned wave_min_u32(unsigned v) {
  int x = (int)v;
  auto mn = [](int a, int b) { return (int)min((unsigned)a, (unsigned)b); };
  x = mn(x, __builtin_amdgcn_update_dpp(-1, x, 0xB1, 0xF, 0xF, false));
  x = mn(x, __builtin_amdgcn_update_dpp(-1, x, 0x4E, 0xF, 0xF, false));
  x = mn(x, __builtin_amdgcn_update_dpp(-1, x, 0x141, 0xF, 0xF, false));
  x = mn(x, __builtin_amdgcn_update_dpp(-1, x, 0x140, 0xF, 0xF, false));
  x = mn(x, __builtin_amdgcn_update_dpp(-1, x, 0x142, 0xA, 0xF, false));
  x = mn(x, __builtin_amdgcn_update_dpp(-1, x, 0x143, 0xC, 0xF, false));
  return (unsigned)__builtin_amdgcn_readlane(x, 63);
}

// Leaf rows between the row-major factor and the LDS block S (one chunk of
// NT logical rows from rbase, NT the panel group's threads).  A row's W-column segment is 128
// bytes (64 for the 8-rows-per-thread leaves) split into 16-byte pieces, one
// per lane, so every load or store instruction of a wave covers whole rows
// instead of one row per lane.  The segment start is 16-byte aligned (the
// leading dimension is a multiple of 16 elements and c0 a multiple of W), and
// a whole segment lies inside the padded row, so loads need no column bound;
// stores stop at column c0 + wc.
template <typename P, int W, int NT = kPanelThreads>
__device__ __forceinline__ void leaf_to_lds(const cx<P>* __restrict__ T, const int* rat, int ld, int k0, int c0,
                                            int rbase, int nrow, cx<P> (&S)[NT][W + 1]) {
  constexpr int CP = 16 / (int)sizeof(cx<P>);  // elements per piece
  constexpr int LPR = W / CP;                   // pieces per row
  constexpr int RPP = NT / LPR;      // rows per pass
  static_assert(W % CP == 0 && NT % LPR == 0, "whole pieces per row");
  const int q = threadIdx.x % LPR, rr = threadIdx.x / LPR;
#pragma unroll
  for (int p = 0; p < LPR; ++p) {
    const int lr = p * RPP + rr;
    if (lr < nrow) {
      const cx<P>* src = T + (long long)rat[rbase + lr - k0] * ld + c0 + q * CP;
      if constexpr (CP == 2) {
        const float4 t = *reinterpret_cast<const float4*>(src);
        cput(S[lr][2 * q], cx<P>{t.x, t.y});
        cput(S[lr][2 * q + 1], cx<P>{t.z, t.w});
      } else {
        const double2 t = *reinterpret_cast<const double2*>(src);
        cput(S[lr][q], cx<P>{t.x, t.y});
      }
    }
  }
}

template <typename P, int W, int NT = kPanelThreads>
__device__ __forceinline__ void lds_to_leaf(cx<P>* __restrict__ T, const int* rat, int ld, int k0, int c0, int rbase,
                                            int nrow, int wc, const cx<P> (&S)[NT][W + 1]) {
  constexpr int CP = 16 / (int)sizeof(cx<P>);
  constexpr int LPR = W / CP;
  constexpr int RPP = NT / LPR;
  const int q = threadIdx.x % LPR, rr = threadIdx.x / LPR;
#pragma unroll
  for (int p = 0; p < LPR; ++p) {
    const int lr = p * RPP + rr;
    if (lr < nrow && q * CP < wc) {
      cx<P>* dst = T + (long long)rat[rbase + lr - k0] * ld + c0 + q * CP;
      if constexpr (CP == 2) {
        const cx<P> x0 = cget(S[lr][2 * q]), x1 = cget(S[lr][2 * q + 1]);
        if (2 * q + 1 < wc)
          *reinterpret_cast<float4*>(dst) = make_float4(x0.re, x0.im, x1.re, x1.im);
        else
          *reinterpret_cast<float2*>(dst) = make_float2(x0.re, x0.im);  // odd last column
      } else {
        const cx<P> x0 = cget(S[lr][q]);
        *reinterpret_cast<double2*>(dst) = make_double2(x0.re, x0.im);
      }
    }
  }
}

// The end of a leaf (columns c0 .. c0+wc-1, held in registers as a[i][w] for
// logical rows c0 + tid + i*NT): the leaf's top rows make the
// panel columns right of it (c0+wc .. k0+jb-1) rows of U by a unit lower
// solve with the leaf's top block; then, one chunk of NT rows at a
// time, the chunk's leaf rows go to LDS, from there to the factor (coalesced),
// and, as the L operand, into the rank-wc update of the right columns.  The
// row map must hold the leaf's physical rows before the call.
template <typename P, int W, int RPT, int NT = kPanelThreads>
__device__ __forceinline__ void panel_right_update(cx<P>* __restrict__ T, const int* rat, int ld, int n, int k0,
                                                   int jb, int c0, int wc, const cx<P> (&a)[RPT][W],
                                                   cx<P> (&Ltop)[W][W], cx<P> (&Utop)[W][kLuMaxJB],
                                                   cx<P> (&Lc)[NT][W + 1]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // ---- update the panel columns right of the leaf
  const int rc0 = c0 + wc;
  const int nr = k0 + jb - rc0;
  if (nr > 0) {
    if (tid < wc) {
#pragma unroll
      for (int w = 0; w < W; ++w) cput(Ltop[tid][w], cget(a[0][w]));
    }
    __syncthreads();
    static_assert(kLuMaxJB <= NT, "one thread per right-hand column of the panel");
    if (tid < nr) {  // nr < jb <= kLuMaxJB: one column per thread
      const int j = tid;
      cx<P> x[W];
#pragma unroll
      for (int w = 0; w < W; ++w)
        if (w < wc) x[w] = T[(long long)rat[c0 + w - k0] * ld + rc0 + j];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        if (w < wc) {
#pragma unroll
          for (int v = 0; v < W; ++v)
            if (v < w) x[w] = fms(x[w], Ltop[w][v], x[v]);
          T[(long long)rat[c0 + w - k0] * ld + rc0 + j] = x[w];
          Utop[w][j] = x[w];
        }
      }
    }
    // (the chunk loop's first barrier orders Utop before its readers)
  }
  // rows >= rc0: A[r][right] -= L[r][leaf] U[leaf][right], one chunk of
  // NT rows at a time, the chunk's L rows in LDS
  for (int i = 0; i < RPT; ++i) {
    const int rbase = c0 + i * NT;
    if (rbase >= n) break;  // uniform
    const int nrow = min(NT, n - rbase);
    // this thread's row of chunk i (selects: a[][] stays in registers)
#pragma unroll
    for (int w = 0; w < W; ++w) {
      cx<P> v = cget(a[0][w]);
#pragma unroll
      for (int u = 1; u < RPT; ++u) v = csel(i == u, cget(a[u][w]), v);
      cput(Lc[tid][w], w < wc ? v : cx<P>{P(0), P(0)});
    }
    __syncthreads();
    lds_to_leaf<P, W, NT>(T, rat, ld, k0, c0, rbase, nrow, wc, Lc);
    if (nr > 0) {
      if constexpr (sizeof(P) == 4) {
        // Complex FP32: on the matrix cores.  A wave takes four 16-row blocks
        // of one 32-column block of the right part; C is loaded into the
        // accumulators, the leaf's W complex k run as W v_mfma_f32_32x32x2f32
        // on the real 2x2 embedding (A operand negated, so the sum is C - L U),
        // and the blocks are stored back.  Rows of a block below rc0 or past n
        // compute discarded values.
        // four row blocks per unit; two where the leaf rows held in registers
        // (RPT * W complex) leave too few for four blocks' accumulators.
        // A last column block of at most 16 columns (the right part is 48 or
        // 16 columns wide after the first and third 16-column leaves) runs as
        // 16-column units on v_mfma_f32_16x16x4f32 instead of half-empty
        // 32-column ones, where the leaf registers leave room (panels of at
        // most 2 * NT rows).
        constexpr int RB = 16, CB = 32, NRB = RPT * W > 32 ? 2 : 4;
        constexpr bool k16 = RPT * W <= 32;
        static_assert(W % 2 == 0, "16-column units take the leaf's k in pairs");
        const bool has16 = k16 && (nr & (CB - 1)) != 0 && (nr & (CB - 1)) <= 16;
        const int ncb = has16 ? nr / CB : (nr + CB - 1) / CB;  // 32-column blocks
        const int at = lane & 1, au = lane >> 5, arow = (lane & 31) >> 1;
        const int acomp = at ^ au;
        const float asign = (at == 0 && au == 1) ? 1.f : -1.f;
        const int rb_lo = max(0, rc0 - rbase) / RB;
        const int rb_hi = (nrow + RB - 1) / RB;
        const int nquad = (rb_hi - rb_lo + NRB - 1) / NRB;
        if (k16 && has16) {
          // 16-column units: a 16-row block is two 8-complex-row MFMA blocks;
          // lane l holds column l%16 of complex rows 2(l/16) and 2(l/16)+1 of
          // a block (re, im, re, im), and feeds A row (l%16)/2, component
          // l%2, and B/A k-slot l/16 = (complex k of the pair, component)
          const int h0 = CB * ncb;  // first column of the block, relative to rc0
          const int t16 = lane & 1, kq = lane >> 4, ka = kq >> 1, ku = kq & 1;
          const int acomp16 = t16 ^ ku, arow16 = (lane & 15) >> 1;
          const float asign16 = (t16 == 0 && ku == 1) ? 1.f : -1.f;
          const int col = rc0 + h0 + (lane & 15);
          const bool cok = col < k0 + jb;
          const int cc = cok ? col : rc0;
          const int ucol = min(h0, kLuMaxJB - 16) + (lane & 15);
          // numbered after the 32-column units, dealt to the waves in turn
          int u0 = (wave - nquad * ncb) % (NT / 64);
          if (u0 < 0) u0 += NT / 64;
          for (int unit = u0; unit < nquad; unit += NT / 64) {
            const int rb0 = rb_lo + NRB * unit;
            floatx4 acc[2 * NRB];
            int roff[2 * NRB][2];
            bool rok[2 * NRB][2];
            int rbq[NRB];
#pragma unroll
            for (int q = 0; q < NRB; ++q) {
              const bool vq = rb0 + q < rb_hi;  // uniform
              rbq[q] = vq ? rb0 + q : rb0;
#pragma unroll
              for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                  const int r = rbase + RB * (rb0 + q) + 8 * h + 2 * kq + e;
                  rok[2 * q + h][e] = vq && r >= rc0 && r < n;
                  roff[2 * q + h][e] = rat[(rok[2 * q + h][e] ? r : rc0) - k0] * ld;
                }
            }
#pragma unroll
            for (int g = 0; g < 2 * NRB; ++g)
#pragma unroll
              for (int e = 0; e < 2; ++e) {
                const cx<P> cv = T[roff[g][e] + cc];
                const bool ok = cok && rok[g][e];
                acc[g][2 * e] = ok ? cv.re : 0.f;
                acc[g][2 * e + 1] = ok ? cv.im : 0.f;
              }
#pragma unroll 2
            for (int k = 0; k < W; k += 2) {
              const cx<P> uv = Utop[k + ka][ucol];
              const float bv = ku ? uv.im : uv.re;
#pragma unroll
              for (int g = 0; g < 2 * NRB; ++g) {
                const cx<P> lv = Lc[RB * rbq[g >> 1] + 8 * (g & 1) + arow16][k + ka];
                const float av = asign16 * (acomp16 ? lv.im : lv.re);
                acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[g], 0, 0, 0);
              }
            }
            if (cok) {
#pragma unroll
              for (int g = 0; g < 2 * NRB; ++g)
#pragma unroll
                for (int e = 0; e < 2; ++e)
                  if (rok[g][e]) T[roff[g][e] + col] = cx<P>{acc[g][2 * e], acc[g][2 * e + 1]};
            }
          }
        }
        for (int unit = wave; unit < nquad * ncb; unit += NT / 64) {
          const int cb = unit / nquad, rb0 = rb_lo + NRB * (unit - cb * nquad);
          const int col = rc0 + CB * cb + (lane & 31);
          const bool cok = col < k0 + jb;
          floatx16 acc[NRB];
          int roff[NRB][8];
          bool rok[NRB][8];
          int rbq[NRB];
#pragma unroll
          for (int q = 0; q < NRB; ++q) {
            const bool vq = rb0 + q < rb_hi;  // uniform
            rbq[q] = vq ? rb0 + q : rb0;
#pragma unroll
            for (int e = 0; e < 16; e += 2) {
              const int r = rbase + RB * (rb0 + q) + 4 * (e >> 2) + 2 * (lane >> 5) + ((e & 3) >> 1);
              rok[q][e >> 1] = vq && r >= rc0 && r < n;
              roff[q][e >> 1] = rat[(rok[q][e >> 1] ? r : rc0) - k0] * ld;
            }
          }
          const int cc = cok ? col : rc0;
#pragma unroll
          for (int q = 0; q < NRB; ++q)
#pragma unroll
            for (int e = 0; e < 16; e += 2) {
              const cx<P> cv = T[roff[q][e >> 1] + cc];
              const bool ok = cok && rok[q][e >> 1];
              acc[q][e] = ok ? cv.re : 0.f;
              acc[q][e + 1] = ok ? cv.im : 0.f;
            }
#pragma unroll
          for (int k = 0; k < W; ++k) {
            const cx<P> uv = Utop[k][min(CB * cb, kLuMaxJB - CB) + (lane & 31)];
            const float bv = au ? uv.im : uv.re;
#pragma unroll
            for (int q = 0; q < NRB; ++q) {
              const cx<P> lv = Lc[RB * rbq[q] + arow][k];
              const float av = asign * (acomp ? lv.im : lv.re);
              acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc[q], 0, 0, 0);
            }
          }
          if (cok) {
#pragma unroll
            for (int q = 0; q < NRB; ++q)
#pragma unroll
              for (int e = 0; e < 16; e += 2)
                if (rok[q][e >> 1]) T[roff[q][e >> 1] + col] = cx<P>{acc[q][e], acc[q][e + 1]};
          }
        }
      } else {
        const int rlo = max(rbase, rc0), rhi = rbase + nrow;
        // each wave takes kRows rows at a time so that their loads are in
        // flight together (fewer where the leaf rows held in registers are
        // many); full leaves and full row batches run branch-free
        constexpr int kLeafWords = RPT * W * (int)sizeof(cx<P>) / 4;
        constexpr int kRows = kLeafWords >= 128 ? 2 : kLeafWords > 64 ? 4 : 8;
        for (int r0 = rlo + wave * kRows; r0 < rhi; r0 += (NT / 64) * kRows) {
          const int nrw = min(kRows, rhi - r0);
          for (int j = lane; j < nr; j += 64) {
            long long off[kRows];
            cx<P> acc[kRows];
#pragma unroll
            for (int u = 0; u < kRows; ++u) {
              const int r = r0 + min(u, nrw - 1);
              off[u] = (long long)rat[r - k0] * ld + rc0 + j;
            }
#pragma unroll
            for (int u = 0; u < kRows; ++u) acc[u] = T[off[u]];
            if (wc == W) {
#pragma unroll
              for (int u = 0; u < kRows; ++u) {
                const int lr = r0 + min(u, nrw - 1) - rbase;
#pragma unroll
                for (int w = 0; w < W; ++w) acc[u] = fms(acc[u], Lc[lr][w], Utop[w][j]);
              }
            } else {
#pragma unroll
              for (int u = 0; u < kRows; ++u) {
                const int lr = r0 + min(u, nrw - 1) - rbase;
                for (int w = 0; w < wc; ++w) acc[u] = fms(acc[u], Lc[lr][w], Utop[w][j]);
              }
            }
            // duplicated tail rows compute identical values, so storing them
            // twice is harmless
#pragma unroll
            for (int u = kRows - 1; u >= 0; --u) T[off[u]] = acc[u];
          }
        }
      }
    }
    __syncthreads();
  }
}

template <typename P, int W, int RPT, int NT = kPanelThreads>
__global__ __launch_bounds__(NT) void k_lu_panel(const MatDesc* __restrict__ md, int k0, int jbmax,
                                                           cx<P>* __restrict__ Tb, const int* __restrict__ rsrc,
                                                           int* __restrict__ rdst, int* __restrict__ info,
                                                           const int* __restrict__ skip, cx<P>* __restrict__ Linv,
                                                           cx<P>* __restrict__ Dinv,
                                                           const long long* __restrict__ dinv_off) {
  const int b = blockIdx.x;
  const MatDesc d = md[b];
  const int n = d.n;
  if (k0 >= n) return;
  if (skip != nullptr && skip[d.node]) return;
  const int jb = min(jbmax, n - k0);  // jbmax <= kLuMaxJB, a multiple of kSolveBlkLu
  cx<P>* __restrict__ T = Tb + d.offT;
  const int ld = d.ld;
  const int* __restrict__ rowg = rsrc + d.offRow;
  int* __restrict__ rowo = rdst + d.offRow;

  // the row map of the panel's rows (at most NT * RPT below 512 threads)
  __shared__ int rat[NT < kPanelThreads ? NT * RPT : kMaxPanelRows];
  // the column's best candidate, (key << 32) | ~row, by an LDS atomic max of
  // every wave's candidate; three slots in rotation, so that a slot is
  // cleared a column after its last read and a column before its next use
  __shared__ unsigned long long redm[3];
  __shared__ cx<P> xbuf[2][W];                    // row c, for the pivot row's owner
  __shared__ int xph[2];
  __shared__ cx<P> wrow[2][NT / 64][W];  // per wave: its candidate row
  __shared__ int wph[2][NT / 64];
  __shared__ cx<P> Ltop[W][W];
  __shared__ cx<P> Utop[W][kLuMaxJB];
  // the right update's L rows (+1: rows in distinct banks), and afterwards
  // the panel's diagonal block for its inverse
  constexpr int kLcBytes = NT * (W + 1) * (int)sizeof(cx<P>);
  constexpr int kXBytes = kSolveBlkLu * (kSolveBlkLu + 1) * (int)sizeof(cx<P>);
  __shared__ __align__(16) unsigned char pool[kLcBytes > kXBytes ? kLcBytes : kXBytes];
  auto& Lc = *reinterpret_cast<cx<P>(*)[NT][W + 1]>(pool);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int m = n - k0;
  for (int r = tid; r < m; r += NT) rat[r] = rowg[k0 + r];
  for (int r = tid; r < k0; r += NT) rowo[r] = rowg[r];  // rows above the panel: unchanged
  if (tid < 3) redm[tid] = 0ull;
  __syncthreads();

  int zp = n;  // first zero pivot (uniform)
  int par = 0, slot = 0;
  for (int c0 = k0; c0 < k0 + jb; c0 += W) {
    const int wc = min(W, k0 + jb - c0);
    // the leaf: logical rows c0 + tid + i*512 with their physical rows ph;
    // row exchanges move data and physical row together, and the row map is
    // written once at the end of the leaf
    // (staged through LDS one chunk of NT rows at a time so that
    // the loads are coalesced; columns from wc on are zero)
    cx<P> a[RPT][W];
    int ph[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int rbase = c0 + i * NT, r = rbase + tid;
#pragma unroll
      for (int w = 0; w < W; ++w) a[i][w] = cx<P>{P(0), P(0)};
      ph[i] = 0;
      if (rbase < n) {  // uniform
        if (i > 0) __syncthreads();  // the previous chunk has been read
        leaf_to_lds<P, W, NT>(T, rat, ld, k0, c0, rbase, min(NT, n - rbase), Lc);
        __syncthreads();
        if (r < n) {
          ph[i] = rat[r - k0];
#pragma unroll
          for (int w = 0; w < W; ++w)
            if (w < wc) cput(a[i][w], cget(Lc[tid][w]));
        }
      }
    }

#pragma unroll
    for (int w = 0; w < W; ++w) {
      if (w < wc) {
        const int c = c0 + w;
        // ---- pivot search: largest key over logical rows >= c, lowest row on ties
        unsigned key = 0u;
        int row = INT_MAX;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const int r = c0 + tid + i * NT;
          const unsigned ki = (r >= c && r < n) ? pivot_key(abs1(cget(a[i][w]))) : 0u;
          const bool take = ki > key;  // rows ascend with i: ties keep the lower
          key = take ? ki : key;
          row = take ? r : row;
        }
        // wave: the largest key, then the lowest row holding it; the lane that
        // holds it publishes the row (a branch taken by that lane alone)
        const unsigned wkey = wave_max_u32(key);
        const unsigned wr = wave_min_u32(key == wkey ? (unsigned)row : 0xffffffffu);
        if (lane == 0) atomicMax(&redm[slot], ((unsigned long long)wkey << 32) | (0xffffffffu - wr));
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          if (wkey != 0u && c0 + tid + i * NT == (int)wr) {
#pragma unroll
            for (int v = 0; v < W; ++v) {  // component copies keep a[][] in registers
              wrow[par][wave][v].re = a[i][v].re;
              wrow[par][wave][v].im = a[i][v].im;
            }
            wph[par][wave] = ph[i];
          }
        }
        if (tid == w) {  // the owner of row c (slot 0) publishes it
#pragma unroll
          for (int v = 0; v < W; ++v) {
            xbuf[par][v].re = a[0][v].re;
            xbuf[par][v].im = a[0][v].im;
          }
          xph[par] = ph[0];
        }
        __syncthreads();
        // the previous column's slot has been read by every thread
        if (tid == 0) redm[slot == 0 ? 2 : slot - 1] = 0ull;
        const int p = (int)(0xffffffffu - (unsigned)redm[slot]);
        slot = slot == 2 ? 0 : slot + 1;
        const int wq = ((p - c0) & (NT - 1)) >> 6;  // the wave that owns logical row p
        const cx<P>* prow = wrow[par][wq];  // pivot row (LDS, read where used)
        // ---- exchange logical rows c and p (registers only)
        if (p != c) {  // uniform
          if (tid == w) {
#pragma unroll
            for (int v = 0; v < W; ++v) {
              a[0][v].re = prow[v].re;
              a[0][v].im = prow[v].im;
            }
            ph[0] = wph[par][wq];
          }
#pragma unroll
          for (int i = 0; i < RPT; ++i) {
            if (c0 + tid + i * NT == p) {  // the pivot row's owner takes row c
#pragma unroll
              for (int v = 0; v < W; ++v) {
                a[i][v].re = xbuf[par][v].re;
                a[i][v].im = xbuf[par][v].im;
              }
              ph[i] = xph[par];
            }
          }
        }
        // ---- scale the column and update the rest of the leaf (selects, no branches)
        const cx<P> pv = prow[w];
        if (pv.re == P(0) && pv.im == P(0) && zp == n) zp = c;
        cx<P> inv;
        if constexpr (sizeof(P) == 4) inv = recip_f32(pv);
        else inv = recip(pv);
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const int r = c0 + tid + i * NT;
          const bool below = r > c && r < n;
          const cx<P> l = cget(a[i][w]) * inv;
          const cx<P> lm = csel(below, l, cx<P>{P(0), P(0)});
          cput(a[i][w], csel(below, l, cget(a[i][w])));
#pragma unroll
          for (int v = 0; v < W; ++v)  // constant trip count: unrolled before w is
            if (v > w) cput(a[i][v], fms(cget(a[i][v]), lm, cget(prow[v])));
        }
        par ^= 1;
      }
    }

    // ---- record the leaf's row exchanges in the row map (visible after the
    // next barrier), then store the leaf and update the columns right of it
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = c0 + tid + i * NT;
      if (r < n) rat[r - k0] = ph[i];
    }

    panel_right_update<P, W, RPT, NT>(T, rat, ld, n, k0, jb, c0, wc, a, Ltop, Utop, Lc);
  }
  __syncthreads();
  for (int r = tid; r < m; r += NT) rowo[k0 + r] = rat[r];
  if (tid == 0 && zp < n) atomicMin(&info[d.node], zp);

  // ---- inverses of the unit lower 64 x 64 diagonal blocks of L11
  // (recursive doubling in LDS): the 64 x 64 diagonal-block inverses of L
  // that the triangular solves use (Dinv layout per matrix: [blk][0: L, 1:
  // U][64][64], row-major, identity-padded) and, when trailing columns
  // follow, inv(L11) for the U12 product.  A 128-wide panel's L11 = [A 0; C B]
  // has the inverse [inv(A) 0; -inv(B) C inv(A)  inv(B)]: with inv(A) still
  // in LDS, Y = C inv(A) goes (FP64 sums, rounded once) to the block of Linv
  // that -inv(B) Y later replaces.
  {
    constexpr int B = kSolveBlkLu, lx = B + 1;
    constexpr int YPT = B * B / NT;  // off-diagonal entries per thread
    cx<P>* X = reinterpret_cast<cx<P>*>(pool);
    const bool trailing = n - k0 - jb > 0;
    cx<P>* __restrict__ Li0 = Linv + (long long)b * kLuMaxJB * kLuMaxJB;
    for (int q0 = 0; q0 < jb; q0 += B) {
      const int nb = min(B, jb - q0);
      __syncthreads();  // the pool is free
      for (int e = tid; e < B * B; e += NT) {
        const int i = e / B, k = e - i * B;
        cx<P> v = {P(i == k ? 1 : 0), P(0)};
        if (i < nb && k < i) v = cget(T[(long long)rat[q0 + i] * ld + k0 + q0 + k]);
        cput(X[i * lx + k], v);
      }
      __syncthreads();
      tri_inv_lds<P, false, NT>(X, lx, B);
      if (trailing) {
        cx<P>* __restrict__ Li = Li0 + (long long)q0 * kLuMaxJB + q0;
        for (int e = tid; e < nb * nb; e += NT) {
          const int i = e / nb, k = e - i * nb;
          cput(Li[(long long)i * kLuMaxJB + k], cget(X[i * lx + k]));
        }
      }
      cx<P>* __restrict__ out = Dinv + dinv_off[b] + ((long long)((k0 + q0) / B) * 2 + 0) * B * B;
      for (int e = tid; e < B * B; e += NT) cput(out[e], cget(X[(e / B) * lx + (e % B)]));
      if (trailing && q0 == 0 && jb > B) {  // Y = C inv(A) into Linv[B.., 0..B)
        __syncthreads();  // inv(A) in X is complete
        for (int u = 0; u < YPT; ++u) {
          const int e = tid + NT * u, i = e / B, j = e - i * B;
          const cx<P>* __restrict__ crow = T + (long long)rat[B + i] * ld + k0;
          c128 acc = {0.0, 0.0};
          for (int k = j; k < B; ++k) {  // inv(A) is lower triangular
            const cx<P> c = crow[k], m = cget(X[k * lx + j]);
            acc = acc + c128{double(c.re), double(c.im)} * c128{double(m.re), double(m.im)};
          }
          Li0[(long long)(B + i) * kLuMaxJB + j] = cx<P>{P(acc.re), P(acc.im)};
        }
      }
    }
    if (trailing && jb > B) {  // X = -inv(B) Y (inv(B) in LDS), the upper block zero
      __syncthreads();  // Y is in Linv for every thread
      cx<P> xo[YPT];
      for (int u = 0; u < YPT; ++u) {
        const int e = tid + NT * u, i = e / B, j = e - i * B;
        c128 acc = {0.0, 0.0};
        for (int k = 0; k <= i; ++k) {  // inv(B) is lower triangular
          const cx<P> m = cget(X[i * lx + k]), y = Li0[(long long)(B + k) * kLuMaxJB + j];
          acc = acc + c128{double(m.re), double(m.im)} * c128{double(y.re), double(y.im)};
        }
        xo[u] = cx<P>{P(-acc.re), P(-acc.im)};
      }
      __syncthreads();  // every thread has read Y
      for (int u = 0; u < YPT; ++u) {
        const int e = tid + NT * u, i = e / B, j = e - i * B;
        Li0[(long long)(B + i) * kLuMaxJB + j] = xo[u];
        Li0[(long long)i * kLuMaxJB + B + j] = cx<P>{P(0), P(0)};
      }
    }
  }
}

// U part: inverses of the 64 x 64 diagonal blocks of U11, in FP64, stored in
// the factor precision.  One group per (matrix, 64-row block of the panel).
template <typename P>
__global__ __launch_bounds__(256) void k_lu_inv_u(const MatDesc* __restrict__ md, int k0, int jbmax,
                                                  const cx<P>* __restrict__ Tb, const int* __restrict__ rowb,
                                                  cx<P>* __restrict__ Dinv, const long long* __restrict__ dinv_off,
                                                  const int* __restrict__ skip) {
  constexpr int B = kSolveBlkLu;
  const int nbp = jbmax / B;
  const int b = blockIdx.x / nbp, q = blockIdx.x - b * nbp;
  const MatDesc d = md[b];
  const int n = d.n;
  if (k0 >= n) return;
  if (skip != nullptr && skip[d.node]) return;
  const int R0 = k0 + q * B;
  const int jb = min(jbmax, n - k0);
  if (q * B >= jb) return;
  const int nr = min(B, n - R0);
  const cx<P>* __restrict__ T = Tb + d.offT;
  const int ld = d.ld;
  const int* __restrict__ rat = rowb + d.offRow + R0;
  __shared__ c128 X[B * (B + 1)];
  for (int e = threadIdx.x; e < B * B; e += 256) {
    const int i = e / B, k = e - i * B;
    c128 v = {i == k ? 1.0 : 0.0, 0.0};
    if (i < nr && k < nr && k >= i) {
      const cx<P> t = T[(long long)rat[i] * ld + R0 + k];
      v = c128{double(t.re), double(t.im)};
    }
    X[i * (B + 1) + k] = v;
  }
  __syncthreads();
  tri_inv_lds<double, true>(X, B + 1, B);
  cx<P>* __restrict__ out = Dinv + dinv_off[b] + ((long long)(R0 / B) * 2 + 1) * B * B;
  for (int e = threadIdx.x; e < B * B; e += 256) {
    const int i = e / B, k = e - i * B;
    const c128 v = X[i * (B + 1) + k];
    out[e] = cx<P>{P(v.re), P(v.im)};
  }
}

// ---------------------------------------------------------------------------
// GEMM: A22 -= L21 * U12  (complex, on the matrix cores)
// ---------------------------------------------------------------------------
// c64 variant: 256 threads = 4 waves (2 x 2), each wave 64 x 64 complex.
constexpr int kG32TM = 128, kG32TN = 128, kG32KC = 16;
constexpr int kG32Waves = 8;  // waves per group of the complex-FP32 GEMM

// MODE 0: trailing update A22 -= L21 U12 (rows/cols >= k0+jb).
// MODE 1: block-row solve U12 = L11^{-1} A12 with the stored inverse (rows
//         k0..k0+jb-1, cols >= k0+jb), result stored in place.
template <int MODE, int NW>
__global__ __launch_bounds__(64 * NW) void k_lu_gemm_c64(const MatDesc* __restrict__ md, const int* __restrict__ prefix,
                                                     int nact, int total, int k0, int jbmax, c64* __restrict__ Tb,
                                                     const int* __restrict__ rowb, const int* __restrict__ skip,
                                                     const c64* __restrict__ Linv, const int* __restrict__ rowa,
                                                     int coff, int ntn) {
  const int v = xcd_remap(blockIdx.x, gridDim.x, total);
  if (v < 0) return;
  const int b = find_slot(prefix, nact, v);
  const int t = v - prefix[b];
  const MatDesc d = md[b];
  if (skip != nullptr && skip[d.node]) return;
  const int n = d.n;
  const int jb = min(jbmax, n - k0);  // == jbmax whenever a trailing block exists (a multiple of kG32KC)
  const int s0 = k0 + jb;             // first trailing row/col
  const int mt = n - s0;              // trailing size
  // tile columns 0 .. ntn - 1 of the trailing columns from coff on (clipped)
  const int tiles_n = min(ntn, (mt - coff + kG32TN - 1) / kG32TN);
  const int tm = t / tiles_n, tn = t - tm * tiles_n;
  const int row0 = (MODE == 0 ? s0 : k0) + tm * kG32TM, col0 = s0 + coff + tn * kG32TN;
  const int row_end = MODE == 0 ? n : k0 + jb;
  c64* __restrict__ T = Tb + d.offT;
  const int ld = d.ld;
  const int* __restrict__ rat = rowb + d.offRow;    // B rows (and U12 rows in MODE 1)
  const int* __restrict__ rata = rowa + d.offRow;   // A and C rows of the trailing update
  const c64* __restrict__ Asrc = MODE == 1 ? Linv + (long long)b * kLuMaxJB * kLuMaxJB : T;
  // NW waves as WR x 2, each (kG32TM / WR) complex rows x 64 complex columns
  constexpr int NT = 64 * NW, WR = NW / 2, MI = kG32TM / WR / 16;
  constexpr int AQ = kG32TM * kG32KC / 2 / NT, BQ = kG32KC * kG32TN / 2 / NT;  // staged pairs per thread
  static_assert(AQ >= 1 && BQ >= 1 && MI >= 1, "tile shape");

  // LDS: A as [k][row] complex (stride kG32TM+2), B as re/im planes [k][col].
  __shared__ float As[2][kG32KC][2 * kG32TM + 4];
  __shared__ float Bs[2][kG32KC][2][kG32TN + 4];
  // element offsets of the tile's A rows (-1: outside) and of the jb B rows
  __shared__ int aoff_s[kG32TM];
  __shared__ int boff_s[kLuMaxJB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * (kG32TM / WR), wcn = (wave & 1) * 64;
  // a wave whose rows or columns lie wholly outside the matrix (edge tiles of
  // the shrinking trailing block, the lower half of the U12 tiles) stages its
  // share of the operands but issues no products (uniform per wave)
  const bool wlive = row0 + wr < row_end && col0 + wcn < n;
  if (tid < kG32TM) {
    const int gr = row0 + tid;
    aoff_s[tid] = gr < row_end ? (MODE == 0 ? rata[gr] * ld : (gr - k0) * kLuMaxJB) : -1;
  }
  for (int i = tid; i < jb; i += NT) boff_s[i] = rat[k0 + i] * ld;
  __syncthreads();

  // per-thread staging roles: A (row r = tid/8 + (NT/8) q, k-pair kp = tid%8),
  // B (k row kr = tid/64 + NW q, column pair cp = tid%64)
  const int kp = tid & 7, cp = tid & 63;
  int aoff[AQ];
  bool aval[AQ];
#pragma unroll
  for (int q = 0; q < AQ; ++q) {
    const int o = aoff_s[(tid >> 3) + (NT / 8) * q];
    aval[q] = o >= 0;
    aoff[q] = o >= 0 ? o : 0;
  }
  const int gc = col0 + 2 * cp;
  const int gcl = min(gc, ld - 2);  // clamped: the load stays inside the row
  const bool bval0 = gc < n, bval1 = gc + 1 < n;

  // Loads go to clamped, always-valid addresses; the zero masks are applied
  // when the staged values are written to LDS, so the loads stay in flight
  // across the products of the current chunk.
  float4 ra[AQ], rb[BQ];
  auto load_tile = [&](int kk) {  // kk: chunk offset relative to k0
#pragma unroll
    for (int q = 0; q < AQ; ++q)
      ra[q] = *reinterpret_cast<const float4*>(Asrc + aoff[q] + (MODE == 0 ? k0 : 0) + kk + 2 * kp);
#pragma unroll
    for (int q = 0; q < BQ; ++q)
      rb[q] = *reinterpret_cast<const float4*>(T + boff_s[kk + (tid >> 6) + NW * q] + gcl);
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int q = 0; q < AQ; ++q) {
      const int r = (tid >> 3) + (NT / 8) * q;
      const bool va = aval[q];
      As[buf][2 * kp][2 * r] = va ? ra[q].x : 0.f;
      As[buf][2 * kp][2 * r + 1] = va ? ra[q].y : 0.f;
      As[buf][2 * kp + 1][2 * r] = va ? ra[q].z : 0.f;
      As[buf][2 * kp + 1][2 * r + 1] = va ? ra[q].w : 0.f;
    }
#pragma unroll
    for (int q = 0; q < BQ; ++q) {
      const int kr = (tid >> 6) + NW * q;
      Bs[buf][kr][0][2 * cp] = bval0 ? rb[q].x : 0.f;
      Bs[buf][kr][1][2 * cp] = bval0 ? rb[q].y : 0.f;
      Bs[buf][kr][0][2 * cp + 1] = bval1 ? rb[q].z : 0.f;
      Bs[buf][kr][1][2 * cp + 1] = bval1 ? rb[q].w : 0.f;
    }
  };

  // Accumulators.  acc reg r of block (i, j) holds real row 8(r/4) + 4(l/32)
  // + r%4 of the 32-row block, i.e. complex row 4(r/4) + 2(l/32) + (r%4)/2
  // (component r%2), and complex column l%32.  MODE 0 starts from C and
  // accumulates -L21 U12, so the epilogue only stores; MODE 1 starts from 0.
  floatx16 acc[MI][2];
  if (MODE == 0 && wlive) {
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int gcol = col0 + wcn + j * 32 + (lane & 31);
        const int gcl2 = min(gcol, ld - 1);
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
          const int lr = wr + i * 16 + 4 * (r >> 2) + 2 * (lane >> 5) + ((r & 3) >> 1);
          const int o = aoff_s[lr];
          const c64 cv = T[(o >= 0 ? o : 0) + gcl2];
          const bool ok = o >= 0 && gcol < n;
          acc[i][j][r] = ok ? cv.re : 0.f;
          acc[i][j][r + 1] = ok ? cv.im : 0.f;
        }
      }
  } else {
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  }

  // operand lane roles: A row (l%32)/2 with component t=l%2; k-half u=l/32
  const int at = lane & 1, au = lane >> 5, arow = (lane & 31) >> 1;
  const int acomp = at ^ au;                      // 0: re, 1: im
  const float asign = ((at == 0 && au == 1) ? -1.f : 1.f) * (MODE == 0 ? -1.f : 1.f);
  const int bcol = lane & 31, bu = lane >> 5;

  const int nk = jb / kG32KC;
  load_tile(0);
  store_tile(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) load_tile((kc + 1) * kG32KC);
    if (wlive) {
    // operands of step k+1 are read while the products of step k issue
    float af[2][MI], bf[2][2];
    auto frag = [&](int k, float (&a)[MI], float (&bb)[2]) {
#pragma unroll
      for (int i = 0; i < MI; ++i) a[i] = asign * As[buf][k][2 * (wr + i * 16 + arow) + acomp];
#pragma unroll
      for (int j = 0; j < 2; ++j) bb[j] = Bs[buf][k][bu][wcn + j * 32 + bcol];
    };
    frag(0, af[0], bf[0]);
    __builtin_amdgcn_sched_group_barrier(0x100, (MI + 2) / 2, 0);
    __builtin_amdgcn_sched_group_barrier(0x002, MI, 0);
#pragma unroll
    for (int k = 0; k < kG32KC; ++k) {
      if (k + 1 < kG32KC) frag(k + 1, af[(k + 1) & 1], bf[(k + 1) & 1]);
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[k & 1][i], bf[k & 1][j], acc[i][j], 0, 0, 0);
      // issue order: the next step's LDS reads, then this step's products
      if (k + 1 < kG32KC) {
        __builtin_amdgcn_sched_group_barrier(0x100, (MI + 2) / 2, 0);  // DS reads
        __builtin_amdgcn_sched_group_barrier(0x002, MI, 0);  // sign multiplies
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 2 * MI, 0);    // MFMA
    }
    }
    if (kc + 1 < nk) {
      store_tile(buf ^ 1);
      __syncthreads();
    }
  }
  if (!wlive) return;

  // epilogue: store the block (C - L21 U12 in MODE 0, U12 in MODE 1)
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int gcol = col0 + wcn + j * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        const int lr = wr + i * 16 + 4 * (r >> 2) + 2 * (lane >> 5) + ((r & 3) >> 1);
        const int gr = row0 + lr;
        if (gr < row_end && gcol < n)
          T[(MODE == 0 ? aoff_s[lr] : rat[gr] * ld) + gcol] = c64{acc[i][j][r], acc[i][j][r + 1]};
      }
    }
}

// Part 0 of a step, complex FP32: the first kP0TN trailing columns, which
// hold the next panel.  Every group first forms U12 = inv(L11) A12 for those
// columns on the matrix cores (inv(L11) and A12 staged in LDS; the group of
// the first row tile also stores U12), then applies C -= L21 U12 to its
// 128 x 64 block with U12 kept in LDS.  One launch instead of a block-row
// product followed by an update, on the factorization's critical path.
// U12 replaces A12 in place, so it is stored by the last group of the matrix
// to have staged A12 (a per-matrix arrival count, reset by that group): every
// other group has read A12 by then.
// Grid: the row tiles of all active matrices (prefix table).  Operand lane
// roles and the accumulator layout are those of k_lu_gemm_c64.
constexpr int kP0TM = 128, kP0TN = kPart0Cols, kP0KC = 16;  // (64-wide panels only)
constexpr int kP0Waves = 8;  // waves per group

template <int NW>
__global__ __launch_bounds__(64 * NW) void k_lu_part0_c64(const MatDesc* __restrict__ md,
                                                      const int* __restrict__ prefix, int nact, int total, int k0,
                                                      int jbmax, c64* __restrict__ Tb, const int* __restrict__ rowb,
                                                      const int* __restrict__ skip, const c64* __restrict__ Linv,
                                                      int* __restrict__ arrivals) {
  const int v = xcd_remap(blockIdx.x, gridDim.x, total);
  if (v < 0) return;
  const int b = find_slot(prefix, nact, v);
  const int tm = v - prefix[b];
  const MatDesc d = md[b];
  if (skip != nullptr && skip[d.node]) return;
  const int n = d.n;
  const int s0 = k0 + jbmax;   // a trailing block exists, so the panel was jbmax (= 64) wide
  const int mt = n - s0;
  const int ncol = min(kP0TN, mt);
  c64* __restrict__ T = Tb + d.offT;
  const int ld = d.ld;
  const int* __restrict__ rat = rowb + d.offRow;
  const c64* __restrict__ Li = Linv + (long long)b * kLuMaxJB * kLuMaxJB;

  constexpr int K = kSolveBlkLu;          // 64 = jbmax
  constexpr int NT = 64 * NW;
  // U12 (64 x 64): 4 row blocks x 2 column blocks of 16 x 32, CB1 per wave;
  // update (128 x 64): each wave 128/NW rows (MI3 blocks of 16) x 64 columns
  constexpr int CB1 = 8 / NW, MI3 = kP0TM / NW / 16, AQ3 = kP0TM * kP0KC / 2 / NT;
  static_assert(CB1 >= 1 && MI3 >= 1 && AQ3 >= 1, "wave layout");
  constexpr int SA = 2 * K + 4;           // phase 1: inv(L11) as [k][2 row + comp]
  constexpr int SC = 2 * kP0TM + 4;       // phase 2: L21 chunks as [buf][k][2 row + comp]
  constexpr int kSa = K * SA > 2 * kP0KC * SC ? K * SA : 2 * kP0KC * SC;
  __shared__ float Sa[kSa];
  __shared__ float Sb[K][2][kP0TN + 4];   // A12, then U12: re/im planes [k][col]
  __shared__ int aoff_s[kP0TM];
  __shared__ int store_u12;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int at = lane & 1, au = lane >> 5, arow = (lane & 31) >> 1;
  const int acomp = at ^ au;
  const float asign = (at == 0 && au == 1) ? -1.f : 1.f;
  const int bcol = lane & 31, bu = lane >> 5;

  // ---- stage inv(L11) (64 x 64, row-major, stride kLuMaxJB) and A12 (the
  // panel's rows, columns s0 .. s0+63; zero beyond the matrix)
  for (int e = tid; e < K * K / 2; e += NT) {
    const int r = e / (K / 2), kp = e - r * (K / 2);
    const float4 x = *reinterpret_cast<const float4*>(Li + (long long)r * kLuMaxJB + 2 * kp);
    Sa[(2 * kp) * SA + 2 * r] = x.x;
    Sa[(2 * kp) * SA + 2 * r + 1] = x.y;
    Sa[(2 * kp + 1) * SA + 2 * r] = x.z;
    Sa[(2 * kp + 1) * SA + 2 * r + 1] = x.w;
  }
  for (int e = tid; e < K * kP0TN / 2; e += NT) {
    const int k = e / (kP0TN / 2), cp = e - k * (kP0TN / 2);
    const int gc = s0 + 2 * cp;
    const float4 x = *reinterpret_cast<const float4*>(T + (long long)rat[k0 + k] * ld + min(gc, ld - 2));
    const bool v0 = 2 * cp < ncol, v1 = 2 * cp + 1 < ncol;
    Sb[k][0][2 * cp] = v0 ? x.x : 0.f;
    Sb[k][1][2 * cp] = v0 ? x.y : 0.f;
    Sb[k][0][2 * cp + 1] = v1 ? x.z : 0.f;
    Sb[k][1][2 * cp + 1] = v1 ? x.w : 0.f;
  }
  if (tid < kP0TM) {
    const int gr = s0 + tm * kP0TM + tid;
    aoff_s[tid] = gr < n ? rat[gr] * ld : -1;
  }
  __syncthreads();  // A12 is in LDS
  if (tid == 0) {
    const int ntiles = (mt + kP0TM - 1) / kP0TM;
    __threadfence();
    const int before = atomicAdd(&arrivals[b], 1);
    store_u12 = before == ntiles - 1;
    if (store_u12) arrivals[b] = 0;  // every group of this matrix has arrived
  }

  // ---- U12: wave w takes row block rb1 (rows 16 rb1 .. 16 rb1 + 15) and
  // CB1 column blocks from cb1 on (inv(L11) is lower triangular: k runs to
  // the block's last row)
  const int rb1 = wave * CB1 / 2, cb1 = (wave * CB1) % 2;
  floatx16 u[CB1];
#pragma unroll
  for (int j = 0; j < CB1; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) u[j][r] = 0.f;
  const int kend = 16 * rb1 + 16;
  for (int k = 0; k < kend; ++k) {
    const float a = asign * Sa[k * SA + 2 * (16 * rb1 + arow) + acomp];
#pragma unroll
    for (int j = 0; j < CB1; ++j)
      u[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, Sb[k][bu][(cb1 + j) * 32 + bcol], u[j], 0, 0, 0);
  }
  __syncthreads();  // every wave is done with A12 and inv(L11)
#pragma unroll
  for (int j = 0; j < CB1; ++j) {
    const int col = (cb1 + j) * 32 + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; r += 2) {
      const int k = 16 * rb1 + 4 * (r >> 2) + 2 * (lane >> 5) + ((r & 3) >> 1);
      Sb[k][0][col] = u[j][r];
      Sb[k][1][col] = u[j][r + 1];
      if (store_u12 && col < ncol) T[(long long)rat[k0 + k] * ld + s0 + col] = c64{u[j][r], u[j][r + 1]};
    }
  }

  // ---- C -= L21 U12: wave w takes rows (128/NW) w .. (MI3 16-row blocks)
  // and both 32-column blocks; C is loaded into the accumulators
  const int kp = tid & 7;
  const int wr3 = wave * MI3 * 16;
  int aoff[AQ3];
  bool aval[AQ3];
#pragma unroll
  for (int q = 0; q < AQ3; ++q) {
    const int o = aoff_s[(tid >> 3) + (NT / 8) * q];
    aval[q] = o >= 0;
    aoff[q] = o >= 0 ? o : 0;
  }
  float4 ra[AQ3];
  auto load_chunk = [&](int kk) {
#pragma unroll
    for (int q = 0; q < AQ3; ++q) ra[q] = *reinterpret_cast<const float4*>(T + aoff[q] + k0 + kk + 2 * kp);
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int q = 0; q < AQ3; ++q) {
      const int r = (tid >> 3) + (NT / 8) * q;
      float* base = Sa + (buf * kP0KC) * SC;
      base[(2 * kp) * SC + 2 * r] = aval[q] ? ra[q].x : 0.f;
      base[(2 * kp) * SC + 2 * r + 1] = aval[q] ? ra[q].y : 0.f;
      base[(2 * kp + 1) * SC + 2 * r] = aval[q] ? ra[q].z : 0.f;
      base[(2 * kp + 1) * SC + 2 * r + 1] = aval[q] ? ra[q].w : 0.f;
    }
  };
  // a wave whose rows all lie past the matrix stages its share of L21 but
  // issues no products (uniform per wave; the tile's rows are consecutive)
  const bool wlive = aoff_s[wr3] >= 0;
  floatx16 acc[MI3][2];
#pragma unroll
  for (int i = 0; i < MI3; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (!wlive) continue;
      const int gcol = s0 + j * 32 + (lane & 31);
      const int gcl = min(gcol, ld - 1);
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        const int lr = wr3 + 16 * i + 4 * (r >> 2) + 2 * (lane >> 5) + ((r & 3) >> 1);
        const int o = aoff_s[lr];
        const c64 cv = T[(o >= 0 ? o : 0) + gcl];
        const bool ok = o >= 0 && j * 32 + (lane & 31) < ncol;
        acc[i][j][r] = ok ? cv.re : 0.f;
        acc[i][j][r + 1] = ok ? cv.im : 0.f;
      }
    }
  load_chunk(0);
  __syncthreads();  // U12 in Sb; Sa free for the L21 chunks
  store_chunk(0);
  __syncthreads();
  constexpr int nk = K / kP0KC;
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) load_chunk((kc + 1) * kP0KC);
    const float* base = Sa + (buf * kP0KC) * SC;
    if (wlive) {
#pragma unroll
      for (int k = 0; k < kP0KC; ++k) {
        float a[MI3];
#pragma unroll
        for (int i = 0; i < MI3; ++i) a[i] = -asign * base[k * SC + 2 * (wr3 + 16 * i + arow) + acomp];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const float bb = Sb[kc * kP0KC + k][bu][j * 32 + bcol];
#pragma unroll
          for (int i = 0; i < MI3; ++i)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], bb, acc[i][j], 0, 0, 0);
        }
      }
    }
    if (kc + 1 < nk) {
      store_chunk(buf ^ 1);
      __syncthreads();
    }
  }
  if (!wlive) return;
#pragma unroll
  for (int i = 0; i < MI3; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = j * 32 + (lane & 31);
      if (col >= ncol) continue;
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        const int lr = wr3 + 16 * i + 4 * (r >> 2) + 2 * (lane >> 5) + ((r & 3) >> 1);
        const int o = aoff_s[lr];
        if (o >= 0) T[o + s0 + col] = c64{acc[i][j][r], acc[i][j][r + 1]};
      }
    }
}

// c128 variant: 256 threads = 4 waves (2 x 2), each wave 64 x 32 complex.
constexpr int kG64TM = 128, kG64TN = 64, kG64KC = 8;
constexpr int kG64Waves = 8;  // waves per group of the complex-FP64 GEMM

template <int MODE, int NW>
__global__ __launch_bounds__(64 * NW) void k_lu_gemm_c128(const MatDesc* __restrict__ md, const int* __restrict__ prefix,
                                                      int nact, int total, int k0, int jbmax, c128* __restrict__ Tb,
                                                      const int* __restrict__ rowb, const int* __restrict__ skip,
                                                      const c128* __restrict__ Linv, const int* __restrict__ rowa,
                                                      int coff, int ntn) {
  const int v = xcd_remap(blockIdx.x, gridDim.x, total);
  if (v < 0) return;
  const int b = find_slot(prefix, nact, v);
  const int t = v - prefix[b];
  const MatDesc d = md[b];
  if (skip != nullptr && skip[d.node]) return;
  const int n = d.n;
  const int jb = min(jbmax, n - k0);  // == jbmax whenever a trailing block exists (a multiple of kG64KC)
  const int s0 = k0 + jb;
  const int mt = n - s0;
  const int tiles_n = min(ntn, (mt - coff + kG64TN - 1) / kG64TN);
  const int tm = t / tiles_n, tn = t - tm * tiles_n;
  const int row0 = (MODE == 0 ? s0 : k0) + tm * kG64TM, col0 = s0 + coff + tn * kG64TN;
  const int row_end = MODE == 0 ? n : k0 + jb;
  c128* __restrict__ T = Tb + d.offT;
  const int ld = d.ld;
  const int* __restrict__ rat = rowb + d.offRow;    // B rows (and U12 rows in MODE 1)
  const int* __restrict__ rata = rowa + d.offRow;   // A and C rows of the trailing update
  const c128* __restrict__ Asrc = MODE == 1 ? Linv + (long long)b * kLuMaxJB * kLuMaxJB : T;
  // NW waves as WR x 2, each (kG64TM / WR) complex rows x 32 complex columns
  constexpr int NT = 64 * NW, WR = NW / 2, MI = kG64TM / WR / 8;
  constexpr int AQ = kG64TM * kG64KC / NT, BQ = kG64KC * kG64TN / NT;  // staged complex per thread
  static_assert(AQ >= 1 && BQ >= 1 && MI >= 1, "tile shape");

  __shared__ double As[2][kG64KC][2 * kG64TM + 2];
  __shared__ double Bs[2][kG64KC][2][kG64TN + 2];
  __shared__ int aoff_s[kG64TM];
  __shared__ int boff_s[kLuMaxJB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * (kG64TM / WR), wcn = (wave & 1) * 32;
  // waves wholly outside the matrix stage operands but issue no products
  const bool wlive = row0 + wr < row_end && col0 + wcn < n;
  if (tid < kG64TM) {
    const int gr = row0 + tid;
    aoff_s[tid] = gr < row_end ? (MODE == 0 ? rata[gr] * ld : (gr - k0) * kLuMaxJB) : -1;
  }
  for (int i = tid; i < jb; i += NT) boff_s[i] = rat[k0 + i] * ld;
  __syncthreads();

  // staging roles: A (row tid/8 + (NT/8) q, k tid%8), B (k row tid/64 + NW q, column tid%64)
  const int kq8 = tid & 7, cb = tid & 63;
  int aoff[AQ];
  bool aval[AQ];
#pragma unroll
  for (int q = 0; q < AQ; ++q) {
    const int o = aoff_s[(tid >> 3) + (NT / 8) * q];
    aval[q] = o >= 0;
    aoff[q] = o >= 0 ? o : 0;
  }
  const int gcb = col0 + cb;
  const bool bval = gcb < n;
  const int gcbl = min(gcb, ld - 1);

  double2 ra[AQ], rb[BQ];
  auto load_tile = [&](int kk) {  // kk: chunk offset relative to k0
#pragma unroll
    for (int q = 0; q < AQ; ++q)
      ra[q] = *reinterpret_cast<const double2*>(Asrc + aoff[q] + (MODE == 0 ? k0 : 0) + kk + kq8);
#pragma unroll
    for (int q = 0; q < BQ; ++q)
      rb[q] = *reinterpret_cast<const double2*>(T + boff_s[kk + (tid >> 6) + NW * q] + gcbl);
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int q = 0; q < AQ; ++q) {
      const int r = (tid >> 3) + (NT / 8) * q;
      As[buf][kq8][2 * r] = aval[q] ? ra[q].x : 0.0;
      As[buf][kq8][2 * r + 1] = aval[q] ? ra[q].y : 0.0;
    }
#pragma unroll
    for (int q = 0; q < BQ; ++q) {
      const int kr = (tid >> 6) + NW * q;
      Bs[buf][kr][0][cb] = bval ? rb[q].x : 0.0;
      Bs[buf][kr][1][cb] = bval ? rb[q].y : 0.0;
    }
  };

  // acc reg r of lane l: real row l/16 + 4r -> complex row (l/16)/2 + 2r,
  // component (l/16)%2; col l%16.  MODE 0 starts from C and accumulates
  // -L21 U12; MODE 1 starts from 0.
  const int tcomp = (lane >> 4) & 1, rbase = (lane >> 4) >> 1;
  doublex4 acc[MI][2];
  if (MODE == 0 && wlive) {
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int gc = col0 + wcn + j * 16 + (lane & 15);
        const int gcl = min(gc, ld - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int o = aoff_s[wr + i * 8 + rbase + 2 * r];
          const double cv = reinterpret_cast<const double*>(T + (o >= 0 ? o : 0) + gcl)[tcomp];
          acc[i][j][r] = (o >= 0 && gc < n) ? cv : 0.0;
        }
      }
  } else {
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;
  }

  // f64 16x16x4 operand roles: A real row l%16 -> complex row (l%16)/2, t=l%2;
  // real k l/16 -> complex k (l/16)/2 within the pair, u=(l/16)%2.
  const int at = lane & 1, arow = (lane & 15) >> 1;
  const int kq = lane >> 4, ak = kq >> 1, au = kq & 1;
  const int acomp = at ^ au;
  const double asign = ((at == 0 && au == 1) ? -1.0 : 1.0) * (MODE == 0 ? -1.0 : 1.0);
  const int bcol = lane & 15;

  const int nk = jb / kG64KC;
  load_tile(0);
  store_tile(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) load_tile((kc + 1) * kG64KC);
    if (wlive) {
#pragma unroll
    for (int k2 = 0; k2 < kG64KC; k2 += 2) {
      double af[MI], bf[2];
#pragma unroll
      for (int i = 0; i < MI; ++i) af[i] = asign * As[buf][k2 + ak][2 * (wr + i * 8 + arow) + acomp];
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = Bs[buf][k2 + ak][au][wcn + j * 16 + bcol];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    }
    if (kc + 1 < nk) {
      store_tile(buf ^ 1);
      __syncthreads();
    }
  }
  if (!wlive) return;
  // epilogue: store-only
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int gc = col0 + wcn + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int lr = wr + i * 8 + rbase + 2 * r;
        const int gr = row0 + lr;
        if (gr < row_end && gc < n)
          reinterpret_cast<double*>(T + (MODE == 0 ? aoff_s[lr] : rat[gr] * ld) + gc)[tcomp] = acc[i][j][r];
      }
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
// Leaf width: complex FP32 panels of one row per thread take 16-column
// leaves (half the passes over the panel's right part); otherwise 8 (c64) or
// 4 (c128), which keeps the unrolled leaf in registers.
// rpt 0: panels of at most kPanelSmall rows, one row per thread of a
// kPanelSmall-thread group (several groups share a CU).
template <typename P>
static hipError_t launch_panel(int rpt, int nact, const MatDesc* md, int k0, int jb, cx<P>* T, const int* rsrc,
                               int* rdst, int* info, const int* skip, cx<P>* Linv, cx<P>* Dinv,
                               const long long* dinv_off, hipStream_t st) {
  dim3 g(nact), blk(rpt == 0 ? kPanelSmall : kPanelThreads);
  // leaf width: as wide as the registers allow (RPT rows x W complex per thread)
  constexpr bool f32 = sizeof(P) == 4;
  constexpr int W1 = f32 ? 16 : 8, W8 = f32 ? 8 : 4;
#define NEP_PANEL(W, R, NT)                                                                                    \
  hipLaunchKernelGGL((k_lu_panel<P, W, R, NT>), g, blk, 0, st, md, k0, jb, T, rsrc, rdst, info, skip, Linv, Dinv, \
                     dinv_off)
  switch (rpt) {
    case 0: NEP_PANEL(W1, 1, kPanelSmall); break;
    case 1: NEP_PANEL(W1, 1, kPanelThreads); break;
    case 2: NEP_PANEL(W1, 2, kPanelThreads); break;
    case 4: NEP_PANEL(W1, 4, kPanelThreads); break;
    default: NEP_PANEL(W8, 8, kPanelThreads); break;
  }
#undef NEP_PANEL
  return hipGetLastError();
}

// Panel width: 128 when every matrix has at least kLuWideMinN rows (the
// trailing update then runs with k = 128, half the C traffic per product),
// else 64.  A matrix's factors depend on the width, so a matrix factors
// identically in every plan of the same width.
int lu_jb(int /*prec*/, int nmin) { return nmin >= kLuWideMinN ? 128 : 64; }

void LuPlan::build(const std::vector<MatDesc>& sorted, int prec_, int jb_force) {
  prec = prec_;
  jb = jb_force > 0 ? jb_force : lu_jb(prec, sorted.empty() ? 0 : sorted.back().n);
  const int p0cols = jb;  // part 0: the columns of the next panel
  nmat = (int)sorted.size();
  nvec.clear();
  for (const auto& m : sorted) nvec.push_back(m.n);
  nmax = nmat ? sorted[0].n : 0;
  steps.clear();
  prefix.clear();
  for (int k0 = 0; k0 < nmax; k0 += jb) {
    Step s;
    s.k0 = k0;
    int nact = 0;
    while (nact < nmat && sorted[nact].n > k0) ++nact;
    s.nact = nact;
    s.n8 = 0;
    while (s.n8 < nact && sorted[s.n8].n - k0 > 4 * kPanelThreads) ++s.n8;
    s.n4 = s.n8;
    while (s.n4 < nact && sorted[s.n4].n - k0 > 2 * kPanelThreads) ++s.n4;
    s.nwide = s.n4;
    while (s.nwide < nact && sorted[s.nwide].n - k0 > kPanelThreads) ++s.nwide;
    s.nsmall = s.nwide;
    while (s.nsmall < nact && sorted[s.nsmall].n - k0 > kPanelSmall) ++s.nsmall;
    // tile prefixes of the block-row product (U12) and of the trailing
    // update, each in two parts: part 0 = the first jb trailing columns
    // (they hold the next panel), part 1 = the rest.  Complex FP32 with
    // 64-wide panels runs part 0 as one fused kernel (128-row tiles, U12
    // formed in each); 128-wide panels take the two products.
    const bool f32 = prec != NEP_PREC_FP64;
    const bool fused0 = f32 && jb == kPart0Cols;
    const int TM = f32 ? kG32TM : kG64TM;
    for (int part = 0; part < 2; ++part) {
      // part 0 covers the next panel's columns: one 128-column tile column
      // (complex FP32), or p0cols / 64 of the complex-FP64 update's tiles
      const int TN = part == 0 ? (f32 ? p0cols : kG64TN) : (f32 ? kG32TN : kG64TN);
      for (int kind = 0; kind < 2; ++kind) {  // 0: U12 product, 1: trailing update
        int& off = kind == 0 ? s.off_trsm[part] : s.off_gemm[part];
        int& tot = kind == 0 ? s.tot_trsm[part] : s.tot_gemm[part];
        off = (int)prefix.size();
        int acc = 0;
        prefix.push_back(0);
        for (int b = 0; b < nact; ++b) {
          const int n = sorted[b].n, jbb = std::min(jb, n - k0), mt = n - k0 - jbb;
          const int ncols = part == 0 ? std::min(mt, p0cols) : std::max(0, mt - p0cols);
          const int ntn = ncols > 0 ? ceil_div(ncols, TN) : 0;
          if (kind == 0) acc += (fused0 && part == 0) ? 0 : ntn;
          else acc += (mt > 0 ? ceil_div(mt, TM) : 0) * ntn;
          prefix.push_back(acc);
        }
        tot = acc;
      }
    }
    steps.push_back(s);
  }
}

// ---------------------------------------------------------------------------
// Optional kernel timing (events around each trailing-update GEMM launch).
// ---------------------------------------------------------------------------
static KernelProf g_prof;
KernelProf& kernel_prof() { return g_prof; }

// Final row maps: a matrix's map is in the buffer its own last panel wrote
// (matrices leave the schedule when their panels end); copy it to rows
// where that is the second buffer.
__global__ void k_lu_map_final(const MatDesc* __restrict__ md, int jb, const int* __restrict__ alt,
                               int* __restrict__ rows, const int* __restrict__ skip) {
  const MatDesc d = md[blockIdx.x];
  if (skip != nullptr && skip[d.node]) return;
  if ((((d.n + jb - 1) / jb) & 1) == 0) return;  // an even number of panels ends in rows
  for (int r = threadIdx.x; r < d.n; r += blockDim.x) rows[d.offRow + r] = alt[d.offRow + r];
}

// Panel of a step (which also inverts its L11 block) and the inverses of its
// U diagonal blocks.  The U inverses are needed only by the solves: with a
// side stream they run there, off the factorization's critical path (the
// side stream is joined at the end).  The panel reads the row map from rsrc
// and writes the updated map to rdst.
template <typename P>
static hipError_t lu_panel_step(const LuPlan& plan, const LuPlan::Step& s, const MatDesc* d_md, cx<P>* T,
                                const int* rsrc, int* rdst, int* info, const int* skip, cx<P>* Linv, cx<P>* Dinv,
                                const long long* dinv_off, hipStream_t st, hipStream_t side, hipEvent_t ev_side) {
  hipError_t e;
  // the multi-row classes: 8, 4 and 2 rows per thread
  const int wb[4] = {0, s.n8, s.n4, s.nwide}, wr[3] = {8, 4, 2};
  for (int c = 0; c < 3; ++c)
    if (wb[c + 1] > wb[c] &&
        (e = launch_panel<P>(wr[c], wb[c + 1] - wb[c], d_md + wb[c], s.k0, plan.jb, T, rsrc, rdst, info, skip,
                             Linv + (long long)wb[c] * kLuMaxJB * kLuMaxJB, Dinv, dinv_off + wb[c], st)) != hipSuccess)
      return e;
  // panels of at most kPanelSmall rows take the kPanelSmall-thread groups
  // when they are many (two groups share a CU; complex FP32 only, where two
  // fit); the two variants give the same bits (per-row arithmetic and the
  // inverse's per-element sums do not depend on the group size), so the
  // choice by batch size does not change any matrix's factors
  const bool small = sizeof(P) == 4 && s.nact > s.nsmall && s.nact - s.nsmall >= plan.small_min;
  const int mid_end = small ? s.nsmall : s.nact;
  if (s.nwide < mid_end &&
      (e = launch_panel<P>(1, mid_end - s.nwide, d_md + s.nwide, s.k0, plan.jb, T, rsrc, rdst, info, skip,
                           Linv + (long long)s.nwide * kLuMaxJB * kLuMaxJB, Dinv, dinv_off + s.nwide, st)) !=
          hipSuccess)
    return e;
  if (small &&
      (e = launch_panel<P>(0, s.nact - s.nsmall, d_md + s.nsmall, s.k0, plan.jb, T, rsrc, rdst, info, skip,
                           Linv + (long long)s.nsmall * kLuMaxJB * kLuMaxJB, Dinv, dinv_off + s.nsmall, st)) !=
          hipSuccess)
    return e;
  hipStream_t su = st;
  if (side != nullptr) {
    if ((e = hipEventRecord(ev_side, st)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(side, ev_side, 0)) != hipSuccess) return e;
    su = side;
  }
  hipLaunchKernelGGL(k_lu_inv_u<P>, dim3(s.nact * (plan.jb / kSolveBlkLu)), dim3(256), 0, su, d_md, s.k0, plan.jb, T,
                     rdst, Dinv, dinv_off, skip);
  return hipGetLastError();
}

// U12 product and trailing update of one part of a step's tile columns.
template <typename P>
static hipError_t lu_update_part(const LuPlan& plan, const LuPlan::Step& s, int part, const MatDesc* d_md,
                                 const int* d_prefix, cx<P>* T, const int* rows, const int* rows_ac, const int* skip,
                                 const cx<P>* Linv, int* arrivals, hipStream_t st) {
  const int coff = part == 0 ? 0 : plan.jb;
  const int ntn = part == 0 ? (sizeof(P) == 4 ? 1 : plan.jb / kG64TN) : INT_MAX;  // part 0: the next panel's columns
  if constexpr (sizeof(P) == 4) {
    if (part == 0 && plan.jb == kPart0Cols) {  // fused U12 product and update of the first columns
      if (s.tot_gemm[0] > 0) {
        hipLaunchKernelGGL((k_lu_part0_c64<kP0Waves>), dim3(xcd_grid(s.tot_gemm[0])), dim3(64 * kP0Waves), 0, st, d_md,
                           d_prefix + s.off_gemm[0], s.nact, s.tot_gemm[0], s.k0, plan.jb, T, rows, skip, Linv,
                           arrivals);
        return hipGetLastError();
      }
      return hipSuccess;
    }
  }
  if (s.tot_trsm[part] > 0) {
    if constexpr (sizeof(P) == 4)
      hipLaunchKernelGGL((k_lu_gemm_c64<1, kG32Waves>), dim3(xcd_grid(s.tot_trsm[part])), dim3(64 * kG32Waves), 0, st, d_md,
                         d_prefix + s.off_trsm[part], s.nact, s.tot_trsm[part], s.k0, plan.jb, T, rows, skip, Linv,
                         rows, coff, ntn);
    else
      hipLaunchKernelGGL((k_lu_gemm_c128<1, kG64Waves>), dim3(xcd_grid(s.tot_trsm[part])), dim3(64 * kG64Waves), 0, st, d_md,
                         d_prefix + s.off_trsm[part], s.nact, s.tot_trsm[part], s.k0, plan.jb, T, rows, skip, Linv,
                         rows, coff, ntn);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (s.tot_gemm[part] > 0) {
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (g_prof.on) {
      (void)hipEventCreate(&ev0);
      (void)hipEventCreate(&ev1);
      (void)hipEventRecord(ev0, st);
    }
    if constexpr (sizeof(P) == 4)
      hipLaunchKernelGGL((k_lu_gemm_c64<0, kG32Waves>), dim3(xcd_grid(s.tot_gemm[part])), dim3(64 * kG32Waves), 0, st, d_md,
                         d_prefix + s.off_gemm[part], s.nact, s.tot_gemm[part], s.k0, plan.jb, T, rows, skip, Linv,
                         rows_ac, coff, ntn);
    else
      hipLaunchKernelGGL((k_lu_gemm_c128<0, kG64Waves>), dim3(xcd_grid(s.tot_gemm[part])), dim3(64 * kG64Waves), 0, st, d_md,
                         d_prefix + s.off_gemm[part], s.nact, s.tot_gemm[part], s.k0, plan.jb, T, rows, skip, Linv,
                         rows_ac, coff, ntn);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (g_prof.on) {
      (void)hipEventRecord(ev1, st);
      double flops = 0.0;  // 8 real flops per complex multiply-add of the update
      for (int b = 0; b < s.nact; ++b) {
        const int n = plan.nvec[b], jbb = std::min(plan.jb, n - s.k0), mt = n - s.k0 - jbb;
        if (mt <= 0) continue;
        const int c_lo = part == 0 ? 0 : std::min(mt, plan.jb), c_hi = part == 0 ? std::min(mt, plan.jb) : mt;
        flops += 8.0 * mt * (double)(c_hi - c_lo) * jbb;
      }
      g_prof.add(sizeof(P) == 4 ? 0 : 1, ev0, ev1, flops);
    }
  }
  return hipSuccess;
}

// Look-ahead schedule.  The rest of step k's update (the tile columns after
// the first, which hold the next panel) forks to the auxiliary stream while
// st updates the first tile columns and runs the next panel (the panels and
// the first tile columns form the factorization's critical path, so they stay
// on one stream); st joins the auxiliary stream before step k+1's update.
// The two parts touch disjoint columns and only read panel k's factors.  In
// complex FP32 the fork comes as soon as panel k is done, so the auxiliary
// stream's updates of consecutive steps follow each other without waiting for
// st; in complex FP64 it comes after the first columns' update, whose two
// kernels were slowed more by the overlap than the auxiliary stream gained.
// Row maps alternate between two buffers: step k's kernels use map k, and
// panel k+1 reads map k and writes map k+1 into the other buffer, so the rest
// of step k's update keeps addressing its rows through map k while the next
// panel permutes rows (the rows that update touches form the same set under
// either map, and the panel writes only its own columns).  The L11 inverses
// are kept in two halves of Linv by step parity for the same reason: the next
// panel's inverse is written while the rest of step k's U12 product still
// reads step k's.  Without a second buffer (rows_alt null) or an auxiliary
// stream the steps run in order on st with one map.
template <typename P>
hipError_t lu_run(const LuPlan& plan, const MatDesc* d_md, const int* d_prefix, cx<P>* T, int* rows, int* rows_alt,
                  int rows_total, int* info, const int* skip, cx<P>* Linv, cx<P>* Dinv, const long long* dinv_off,
                  int* arrivals, hipStream_t st, const LuStreams& ls) {
  (void)rows_total;
  hipStream_t aux = ls.aux, side = ls.side;
  hipEvent_t ev_fork = ls.ev_fork, ev_join = ls.ev_join;
  hipError_t e;
  hipLaunchKernelGGL(k_lu_init, dim3(plan.nmat), dim3(256), 0, st, d_md, plan.nmat, rows, info);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int nsteps = (int)plan.steps.size();
  if (nsteps == 0) return hipSuccess;
  // panels of 64 or 128 columns (64-column diagonal blocks)
  if (plan.jb % kSolveBlkLu != 0 || plan.jb > kLuMaxJB) return hipErrorInvalidValue;
  const bool lookahead = aux != nullptr && rows_alt != nullptr;
  int* const R[2] = {rows, lookahead ? rows_alt : rows};
  auto map = [&](int k) { return R[(k + 1) & 1]; };  // map of step k (map -1: the initial one)
  const long long half = (long long)plan.nmat * kLuMaxJB * kLuMaxJB;
  auto linv = [&](int k) { return Linv + (k & 1) * half; };
  if ((e = lu_panel_step<P>(plan, plan.steps[0], d_md, T, map(-1), map(0), info, skip, linv(0), Dinv, dinv_off, st,
                            side, ls.ev_side[0])) != hipSuccess)
    return e;
  bool joined = true;  // st has waited for the last work forked to aux
  for (int k = 0; k < nsteps; ++k) {
    const auto& s = plan.steps[k];
    const bool has_next = k + 1 < nsteps;
    const bool overlap = lookahead && has_next && (s.tot_gemm[1] > 0 || s.tot_trsm[1] > 0);
    // fork before the first columns' update: built in for 64-wide complex
    // FP32 panels; with 128-wide panels the late fork lets the next panel
    // start before the update takes the CUs (n = 4096: 172.8 against 206.1 ms
    // per moment pass)
    const bool early = plan.early_fork >= 0 ? plan.early_fork != 0 : (sizeof(P) == 4 && plan.jb == kSolveBlkLu);
    auto fork = [&]() -> hipError_t {
      hipError_t r;
      if ((r = hipEventRecord(ev_fork, st)) != hipSuccess) return r;
      if ((r = hipStreamWaitEvent(aux, ev_fork, 0)) != hipSuccess) return r;
      if ((r = lu_update_part<P>(plan, s, 1, d_md, d_prefix, T, map(k), map(k), skip, linv(k), arrivals, aux)) !=
          hipSuccess)
        return r;
      joined = false;
      return hipEventRecord(ev_join, aux);
    };
    if (overlap && early && (e = fork()) != hipSuccess) return e;
    if ((e = lu_update_part<P>(plan, s, 0, d_md, d_prefix, T, map(k), map(k), skip, linv(k), arrivals, st)) != hipSuccess)
      return e;
    if (overlap && !early && (e = fork()) != hipSuccess) return e;
    if (!overlap &&
        (e = lu_update_part<P>(plan, s, 1, d_md, d_prefix, T, map(k), map(k), skip, linv(k), arrivals, st)) != hipSuccess)
      return e;
    if (has_next && (e = lu_panel_step<P>(plan, plan.steps[k + 1], d_md, T, map(k), map(k + 1), info, skip,
                                          linv(k + 1), Dinv, dinv_off, st, side, ls.ev_side[(k + 1) & 1])) !=
                        hipSuccess)
      return e;
    if (!joined) {
      if ((e = hipStreamWaitEvent(st, ev_join, 0)) != hipSuccess) return e;
      joined = true;
    }
  }
  if (side != nullptr) {  // join the U inverses
    if ((e = hipEventRecord(ls.ev_side_done, side)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(st, ls.ev_side_done, 0)) != hipSuccess) return e;
  }
  if (lookahead) {  // the final maps go to rows
    hipLaunchKernelGGL(k_lu_map_final, dim3(plan.nmat), dim3(256), 0, st, d_md, plan.jb, rows_alt, rows, skip);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t lu_configure() { return hipSuccess; }

template hipError_t lu_run<float>(const LuPlan&, const MatDesc*, const int*, c64*, int*, int*, int, int*, const int*,
                                  c64*, c64*, const long long*, int*, hipStream_t, const LuStreams&);
template hipError_t lu_run<double>(const LuPlan&, const MatDesc*, const int*, c128*, int*, int*, int, int*, const int*,
                                   c128*, c128*, const long long*, int*, hipStream_t, const LuStreams&);

}  // namespace nep
