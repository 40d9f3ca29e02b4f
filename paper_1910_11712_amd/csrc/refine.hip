// FP64 iterative refinement of the node solves.
//
// Residual in split form (the way the paper evaluates T(lambda) x for a split
// operator, Section 5): R_j = V - sum_i A_i (f_i(z_j) Y_j), computed for every
// node at once as one FP64 GEMM per term over all N*L columns [Y_1 .. Y_N], on
// the FP64 matrix cores (v_mfma_f64_16x16x4f64).  The complex columns are
// viewed as pairs of real columns (re, im); for a real A_i this is a plain
// real GEMM, for a complex A_i the 2x2 real embedding is built in the B tile.
// The scalar f_i(z_j) of each column block is applied while staging Y.
//
// Control: a node is converged when, for every probe column c,
//   ||r_c||_inf <= tol (sum_i |f_i(z_j)| ||A_i||_inf ||y_c||_inf + ||v_c||_inf),
// a normwise backward-error test (moduli of complex entries), or when its
// scaled residual stops halving within 10 tol.  A node whose scaled residual
// does not at least halve in a sweep above that is marked stalled.
#include <algorithm>
#include <climits>

#include "engine.hpp"

namespace nep {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kRTM = 64;   // rows per tile
constexpr int kRTQ = 64;   // real columns per tile (32 complex)
constexpr int kRKC = 16;   // real k per stage

template <bool ACPLX>
__global__ __launch_bounds__(256) void k_resid(const ProbDesc* __restrict__ pd, const int* __restrict__ prefix,
                                               int cnt, int total, NodeArrays na, const c128* __restrict__ Y,
                                               c128* __restrict__ R, IrState ir) {
  const int v = xcd_remap(blockIdx.x, gridDim.x, total);
  if (v < 0) return;
  const int p = find_slot(prefix, cnt, v);
  const ProbDesc& D = pd[p];
  if (ACPLX != (D.a_cplx != 0)) return;
  const int t = v - prefix[p];
  const int n = D.n, L = D.L, NL = D.N * D.L, Q = 2 * NL;
  const int tiles_q = (Q + kRTQ - 1) / kRTQ;
  const int tm = t / tiles_q, tq = t - tm * tiles_q;
  const int row0 = tm * kRTM, q0 = tq * kRTQ;
  // skip when every node covered by this column tile has converged
  {
    const int cc0 = q0 / 2, cc1 = min(NL, cc0 + kRTQ / 2) - 1;
    bool any = false;
    for (int j = cc0 / L; j <= cc1 / L; ++j) any |= (ir.conv[D.node0 + j] == 0);
    if (!any) return;
  }
  __shared__ double As[kRKC][kRTM + 1];
  __shared__ double Bs[kRKC][kRTQ + 2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wq = (wave & 1) * 32;
  const double* __restrict__ Yd = reinterpret_cast<const double*>(Y + D.offY);

  doublex4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;

  for (int term = 0; term < D.ell; ++term) {
    if (D.a_is_diag[term]) continue;  // applied in the epilogue
    const double* __restrict__ A = reinterpret_cast<const double*>(D.A[term]);
    const int acplx = ACPLX ? D.a_is_cplx[term] : 0;
    const int Kd = acplx ? 2 * n : n;            // real k extent of this term
    const int lda = acplx ? 2 * n : n;
    for (int k0 = 0; k0 < Kd; k0 += kRKC) {
      // A tile: 64 rows x 16 k
      for (int e = tid; e < kRTM * kRKC; e += 256) {
        const int r = e >> 4, k = e & 15;
        const int gr = row0 + r, gk = k0 + k;
        As[k][r] = (gr < n && gk < Kd) ? A[(long long)gr * lda + gk] : 0.0;
      }
      if (!acplx) {
        // B tile: 16 rows s of Y x 32 complex columns -> re/im real columns
        for (int e = tid; e < kRKC * (kRTQ / 2); e += 256) {
          const int k = e >> 5, cl = e & 31;
          const int s = k0 + k, cc = q0 / 2 + cl;
          double br = 0.0, bi = 0.0;
          if (s < n && cc < NL) {
            const c128 y = {Yd[2 * ((long long)s * NL + cc)], Yd[2 * ((long long)s * NL + cc) + 1]};
            const c128 f = na.fz[(long long)(D.node0 + cc / L) * kMaxTerms + term];
            const c128 fy = f * y;
            br = fy.re;
            bi = fy.im;
          }
          Bs[k][2 * cl] = br;
          Bs[k][2 * cl + 1] = bi;
        }
      } else {
        // complex A: real k = (s, u); B[(s,u)][(cc,t)] = [[re, im], [-im, re]]
        for (int e = tid; e < (kRKC / 2) * (kRTQ / 2); e += 256) {
          const int ks = e >> 5, cl = e & 31;
          const int s = k0 / 2 + ks, cc = q0 / 2 + cl;
          double br = 0.0, bi = 0.0;
          if (s < n && cc < NL) {
            const c128 y = {Yd[2 * ((long long)s * NL + cc)], Yd[2 * ((long long)s * NL + cc) + 1]};
            const c128 f = na.fz[(long long)(D.node0 + cc / L) * kMaxTerms + term];
            const c128 fy = f * y;
            br = fy.re;
            bi = fy.im;
          }
          Bs[2 * ks][2 * cl] = br;
          Bs[2 * ks][2 * cl + 1] = bi;
          Bs[2 * ks + 1][2 * cl] = -bi;
          Bs[2 * ks + 1][2 * cl + 1] = br;
        }
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < kRKC; kk += 4) {
        double af[2], bf[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) af[i] = As[kk + (lane >> 4)][wr + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < 2; ++j) bf[j] = Bs[kk + (lane >> 4)][wq + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
      __syncthreads();
    }
  }
  // epilogue: lane l, reg r -> row (l/16) + 4r, real column l%16 of the block
  double* __restrict__ Rd = reinterpret_cast<double*>(R + D.offY);
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int q = q0 + wq + j * 16 + (lane & 15);
    const int cc = q >> 1, tcomp = q & 1;
    const int node = cc / L, c = cc - node * L;
    double cm = 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wr + i * 16 + (lane >> 4) + 4 * r;
        double val = 0.0;
        if (gr < n && q < Q) {
          const c128 vv = D.V[(long long)c * n + gr];
          double s = acc[i][j][r];
          for (int term = 0; term < D.ell; ++term) {
            if (!D.a_is_diag[term]) continue;
            const c128 y = {Yd[2 * ((long long)gr * NL + cc)], Yd[2 * ((long long)gr * NL + cc) + 1]};
            const c128 f = na.fz[(long long)(D.node0 + node) * kMaxTerms + term];
            const c128 dy = (f * D.Adiag[term][gr]) * y;
            s += tcomp ? dy.im : dy.re;
          }
          val = (tcomp ? vv.im : vv.re) - s;
          Rd[(long long)gr * Q + q] = val;
        }
        const double other = __shfl_xor(val, 1, 64);
        cm = nanmax(cm, sqrt(val * val + other * other));
      }
    cm = nanmax(cm, __shfl_xor(cm, 16, 64));
    cm = nanmax(cm, __shfl_xor(cm, 32, 64));
    if (lane < 16 && tcomp == 0 && q < Q)
      atomicMax(&ir.rnorm[(long long)(D.node0 + node) * kNormStride + c], (unsigned long long)__double_as_longlong(cm));
  }
}

// ---------------------------------------------------------------------------
// Real A_i (every term real): tiles of TM rows x TQ real columns per group of
// WR x WQ waves, each wave (TM/WR) x (TQ/WQ) as blocks of
// v_mfma_f64_16x16x4f64.  The next stage's A and f_i(z_j) Y tiles are loaded
// into registers while the current stage runs from LDS (double-buffered).
// ---------------------------------------------------------------------------
template <int TM, int TQ, int WR, int WQ, int kR2KC>
__global__ __launch_bounds__(64 * WR * WQ, 4) void k_resid_real(const ProbDesc* __restrict__ pd,
                                                              const int* __restrict__ prefix, int cnt, int total,
                                                              NodeArrays na, const c128* __restrict__ Y,
                                                              c128* __restrict__ R, IrState ir) {
  constexpr int NT = 64 * WR * WQ;
  constexpr int MI = TM / WR / 16, MJ = TQ / WQ / 16;  // 16 x 16 blocks per wave
  constexpr int AU = TM * kR2KC / 2 / NT;              // A k-pairs staged per thread
  constexpr int BU = kR2KC * (TQ / 2) / NT;            // B complex entries staged per thread
  static_assert(MI >= 1 && MJ >= 1 && AU >= 1 && BU >= 1, "tile shape");
  static_assert(AU * 2 * NT == TM * kR2KC && BU * NT == kR2KC * (TQ / 2), "staging");
  const int v = xcd_remap(blockIdx.x, gridDim.x, total);
  if (v < 0) return;
  const int p = find_slot(prefix, cnt, v);
  const ProbDesc& D = pd[p];
  const int t = v - prefix[p];
  const int n = D.n, L = D.L, NL = D.N * D.L, Q = 2 * NL;
  const int tiles_q = (Q + TQ - 1) / TQ;
  const int tm = t / tiles_q, tq = t - tm * tiles_q;
  const int row0 = tm * TM, q0 = tq * TQ;
  {
    const int cc0 = q0 / 2, cc1 = min(NL, cc0 + TQ / 2) - 1;
    bool any = false;
    for (int j = cc0 / L; j <= cc1 / L; ++j) any |= (ir.conv[D.node0 + j] == 0);
    if (!any) return;
  }
  __shared__ double As[2][kR2KC][TM + 1];
  __shared__ double Bs[2][kR2KC][TQ + 2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave / WQ) * (TM / WR), wq = (wave % WQ) * (TQ / WQ);
  const c128* __restrict__ Yp = Y + D.offY;

  // staging roles: A element e = tid + NT u is (row e / KP, k pair e % KP);
  // B element e is (k row e / (TQ/2), complex column e % (TQ/2))
  constexpr int KP = kR2KC / 2;
  static_assert(NT % KP == 0 && NT % (TQ / 2) == 0, "staging roles");
  const int akp = tid % KP, bcl = tid % (TQ / 2);
  const int bcc = q0 / 2 + bcl;
  const bool bcol_ok = bcc < NL;
  const int bnode = bcol_ok ? bcc / L : 0;

  doublex4 acc[MI][MJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < MJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;

  for (int term = 0; term < D.ell; ++term) {
    if (D.a_is_diag[term]) continue;  // applied in the epilogue
    // a low-rank term G H^T runs as the product of G (n x r) with Z = H^T Y
    // (r x N*L, formed before this kernel): the same loop over k < r; a
    // banded term of half-width w runs over the k of the tile rows' band
    // only, [row0 - w, row0 + TM + w) (the other products are by zeros)
    const int lr = D.a_lr[term], bw = D.a_bw[term];
    const double* __restrict__ A = lr > 0 ? D.LrG[term] : reinterpret_cast<const double*>(D.A[term]);
    const int lda = lr > 0 ? lr : n;
    const int kend = lr > 0 ? lr : (bw > 0 ? min(n, row0 + TM + bw) : n);
    const int kbeg = (lr == 0 && bw > 0) ? (max(0, row0 - bw) / kR2KC) * kR2KC : 0;
    const c128* __restrict__ Bsrc = lr > 0 ? D.LrZ[term] : Yp;
    const c128 f = bcol_ok ? na.fz[(long long)(D.node0 + bnode) * kMaxTerms + term] : c128{0.0, 0.0};
    double ra[AU][2];
    c128 rb[BU];
    auto load = [&](int k0) {
#pragma unroll
      for (int u = 0; u < AU; ++u) {
        const int gr = row0 + tid / KP + (NT / KP) * u, gk = k0 + 2 * akp;
        const double* src = A + (long long)min(gr, n - 1) * lda;
        const double a0 = src[min(gk, kend - 1)], a1 = src[min(gk + 1, kend - 1)];
        ra[u][0] = (gr < n && gk < kend) ? a0 : 0.0;
        ra[u][1] = (gr < n && gk + 1 < kend) ? a1 : 0.0;
      }
#pragma unroll
      for (int u = 0; u < BU; ++u) {
        const int s = k0 + tid / (TQ / 2) + (2 * NT / TQ) * u;
        const c128 y = Bsrc[(long long)min(s, kend - 1) * NL + (bcol_ok ? bcc : 0)];
        rb[u] = (s < kend && bcol_ok) ? f * y : c128{0.0, 0.0};
      }
    };
    auto store = [&](int buf) {
#pragma unroll
      for (int u = 0; u < AU; ++u) {
        const int r = tid / KP + (NT / KP) * u;
        As[buf][2 * akp][r] = ra[u][0];
        As[buf][2 * akp + 1][r] = ra[u][1];
      }
#pragma unroll
      for (int u = 0; u < BU; ++u) {
        const int k = tid / (TQ / 2) + (2 * NT / TQ) * u;
        Bs[buf][k][2 * bcl] = rb[u].re;
        Bs[buf][k][2 * bcl + 1] = rb[u].im;
      }
    };
    const int nk = (kend - kbeg + kR2KC - 1) / kR2KC;
    load(kbeg);
    store(0);
    __syncthreads();
    for (int ks = 0; ks < nk; ++ks) {
      const int buf = ks & 1;
      if (ks + 1 < nk) load(kbeg + (ks + 1) * kR2KC);
#pragma unroll
      for (int kk = 0; kk < kR2KC; kk += 4) {
        double af[MI], bf[MJ];
#pragma unroll
        for (int i = 0; i < MI; ++i) af[i] = As[buf][kk + (lane >> 4)][wr + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < MJ; ++j) bf[j] = Bs[buf][kk + (lane >> 4)][wq + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < MJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
      if (ks + 1 < nk) {
        store(buf ^ 1);
        __syncthreads();
      }
    }
    __syncthreads();  // the next term restages buffer 0
  }
  // epilogue: lane l, reg r -> row (l/16) + 4r, real column l%16 of the block
  const double* __restrict__ Yd = reinterpret_cast<const double*>(Yp);
  double* __restrict__ Rd = reinterpret_cast<double*>(R + D.offY);
#pragma unroll
  for (int j = 0; j < MJ; ++j) {
    const int q = q0 + wq + j * 16 + (lane & 15);
    const int cc = q >> 1, tcomp = q & 1;
    const int node = cc / L, c = cc - node * L;
    double cm = 0.0;
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = row0 + wr + i * 16 + (lane >> 4) + 4 * r;
        double val = 0.0;
        if (gr < n && q < Q) {
          const c128 vv = D.V[(long long)c * n + gr];
          double s = acc[i][j][r];
          for (int term = 0; term < D.ell; ++term) {
            if (!D.a_is_diag[term]) continue;
            const c128 y = {Yd[2 * ((long long)gr * NL + cc)], Yd[2 * ((long long)gr * NL + cc) + 1]};
            const c128 fz = na.fz[(long long)(D.node0 + node) * kMaxTerms + term];
            const c128 dy = (fz * D.Adiag[term][gr]) * y;
            s += tcomp ? dy.im : dy.re;
          }
          val = (tcomp ? vv.im : vv.re) - s;
          Rd[(long long)gr * Q + q] = val;
        }
        const double other = __shfl_xor(val, 1, 64);
        cm = nanmax(cm, sqrt(val * val + other * other));
      }
    cm = nanmax(cm, __shfl_xor(cm, 16, 64));
    cm = nanmax(cm, __shfl_xor(cm, 32, 64));
    if (lane < 16 && tcomp == 0 && q < Q)
      atomicMax(&ir.rnorm[(long long)(D.node0 + node) * kNormStride + c], (unsigned long long)__double_as_longlong(cm));
  }
}

// Z = H^T Y for one low-rank term of one problem: H n x r (row-major, real),
// Y n x NL (row-major, complex), Z r x NL.  Tiles of 64 rows of Z by 32
// columns, 4 x 2 outputs per thread (rows 4 tk .. 4 tk + 3, columns tc and
// tc + 16), so that each value read from LDS feeds several products; the sum
// over s is cut into S ranges of srows rows (a multiple of 32, s ascending
// in chunks of 32 inside each), one group per tile and range, writing its
// partial sum to slice sp of Zp (Z itself when S == 1); k_lr_zsum then adds
// the S slices in order, so the result does not depend on scheduling.  The
// row tiles of one column tile and range read the same Y rows and are
// consecutive virtual ids: they run on one XCD and share its L2.
__global__ __launch_bounds__(256) void k_lr_z(const double* __restrict__ H, const c128* __restrict__ Y,
                                              c128* __restrict__ Zp, int n, int r, int NL, int S, int srows,
                                              int total) {
  constexpr int KC = 32;
  __shared__ __align__(16) double Hs[KC][66];
  __shared__ c128 Ys[KC][33];
  const int v = xcd_remap(blockIdx.x, gridDim.x, total);
  if (v < 0) return;
  const int rb = (r + 63) / 64;
  const int pair = v / rb, sp = pair % S;
  const int k0 = (v % rb) * 64, c0 = (pair / S) * 32;
  const int sbeg = sp * srows, send = min(n, sbeg + srows);
  const int tk = threadIdx.x >> 4, tc = threadIdx.x & 15;
  c128 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i][0] = acc[i][1] = c128{0.0, 0.0};
  for (int s0 = sbeg; s0 < send; s0 += KC) {
    for (int e = threadIdx.x; e < KC * 64; e += 256) {
      const int s = e >> 6, j = e & 63;
      const int gs = s0 + s;
      Hs[s][j] = (gs < send && k0 + j < r) ? H[(long long)gs * r + k0 + j] : 0.0;
    }
    for (int e = threadIdx.x; e < KC * 32; e += 256) {
      const int s = e >> 5, j = e & 31;
      const int gs = s0 + s;
      Ys[s][j] = (gs < send && c0 + j < NL) ? Y[(long long)gs * NL + c0 + j] : c128{0.0, 0.0};
    }
    __syncthreads();
#pragma unroll 4
    for (int s = 0; s < KC; ++s) {
      const double2 ha = *reinterpret_cast<const double2*>(&Hs[s][4 * tk]);
      const double2 hb = *reinterpret_cast<const double2*>(&Hs[s][4 * tk + 2]);
      const c128 y0 = Ys[s][tc], y1 = Ys[s][tc + 16];
      const double h[4] = {ha.x, ha.y, hb.x, hb.y};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        acc[i][0].re += h[i] * y0.re;
        acc[i][0].im += h[i] * y0.im;
        acc[i][1].re += h[i] * y1.re;
        acc[i][1].im += h[i] * y1.im;
      }
    }
    __syncthreads();
  }
  c128* out = Zp + (long long)sp * r * NL;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = k0 + 4 * tk + i;
    if (k >= r) break;
    if (c0 + tc < NL) out[(long long)k * NL + c0 + tc] = acc[i][0];
    if (c0 + tc + 16 < NL) out[(long long)k * NL + c0 + tc + 16] = acc[i][1];
  }
}

// Z[i] = sum over sp = 0..S-1 of Zp[sp m + i], in that order.
__global__ __launch_bounds__(256) void k_lr_zsum(const c128* __restrict__ Zp, c128* __restrict__ Z, int S,
                                                 long long m) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  c128 a = Zp[i];
  for (int sp = 1; sp < S; ++sp) {
    const c128 b = Zp[(long long)sp * m + i];
    a.re += b.re;
    a.im += b.im;
  }
  Z[i] = a;
}

// t: tiles of the complex-term kernel (64 x 64); tr: tiles of the real-term
// kernel (resid_big: kResidBigTM x kResidBigTQ, else kResidRealTM x
// kResidRealTQ).  A problem counts in exactly one of them.  Every tile shape
// issues the same products in the same order for each element (terms in
// order, k ascending in steps of 4), so the choice does not change results.
hipError_t resid_run(const ProbDesc* pd, const int* prefix, const Table& t, const Table& tr, int resid_big,
                     const NodeArrays& na, const c128* Y, c128* R, IrState ir, int /*nnodes*/, hipStream_t st,
                     const LrJob* lr, int nlr) {
  for (int j = 0; j < nlr; ++j) {  // Z = H^T Y of every low-rank term, before the products that use it
    const LrJob& J = lr[j];
    const int total = ((J.r + 63) / 64) * ((J.NL + 31) / 32) * J.S;
    hipLaunchKernelGGL(k_lr_z, dim3(xcd_grid(total)), dim3(256), 0, st, J.H, Y + J.offY, J.S > 1 ? J.Zp : J.Z, J.n,
                       J.r, J.NL, J.S, J.srows, total);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (J.S > 1) {
      const long long m = (long long)J.r * J.NL;
      hipLaunchKernelGGL(k_lr_zsum, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, J.Zp, J.Z, J.S, m);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  if (tr.total > 0) {
    constexpr int WR = 4, WQ = 2;  // 8 waves
    if (resid_big)  // waves of 32 x 64: twice the reuse of each staged element
      hipLaunchKernelGGL((k_resid_real<kResidBigTM, kResidBigTQ, WR, WQ, 8>), dim3(xcd_grid(tr.total)),
                         dim3(64 * WR * WQ), 0, st, pd, prefix + tr.off, tr.cnt, tr.total, na, Y, R, ir);
    else  // waves of 16 x 32
      hipLaunchKernelGGL((k_resid_real<kResidRealTM, kResidRealTQ, WR, WQ, 32>), dim3(xcd_grid(tr.total)),
                         dim3(64 * WR * WQ), 0, st, pd, prefix + tr.off, tr.cnt, tr.total, na, Y, R, ir);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (t.total > 0) {
    hipLaunchKernelGGL(k_resid<true>, dim3(xcd_grid(t.total)), dim3(256), 0, st, pd, prefix + t.off, t.cnt, t.total,
                       na, Y, R, ir);
    return hipGetLastError();
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// One group over every node: the unconverged count is reduced in LDS and
// stored once, so the counter needs no clearing launch before the sweep.
constexpr int kIrControlThreads = 1024;

__device__ __forceinline__ bool ir_control_node(const ProbDesc* __restrict__ pd, const NodeArrays& na,
                                                const IrState& ir, int g, int sweep, double tol) {
  const int p = na.prob[g];
  const ProbDesc& D = pd[p];
  const double fn = na.fnorm[g];
  double rho = 0.0;
  for (int c = 0; c < D.L; ++c) {
    const double rn = __longlong_as_double((long long)ir.rnorm[(long long)g * kNormStride + c]);
    const double yn = __longlong_as_double((long long)ir.ynorm[(long long)g * kNormStride + c]);
    const double den = fn * yn + ir.vnorm[p * 64 + c];
    // a non-finite residual, solution or scale (an overflow in the factor
    // precision, a NaN anywhere) never counts as converged
    const bool finite = isfinite(rn) && isfinite(yn) && isfinite(den);
    const double q = !finite ? 1e300 : den > 0.0 ? rn / den : (rn > 0.0 ? 1e300 : 0.0);
    rho = fmax(rho, q);
    ir.rnorm[(long long)g * kNormStride + c] = 0ull;
    ir.ynorm[(long long)g * kNormStride + c] = 0ull;
  }
  const double prev = ir.rho[g];
  ir.rho[g] = rho;
  ir.sweeps[g] = sweep + 1;
  const bool stalls = sweep > 0 && !(rho <= 0.5 * prev);
  // converged: below the tolerance, or stalled within 10x of it (the level
  // the factor's contraction reaches at this node; further sweeps or an FP64
  // re-solve would not change the moments beyond that)
  if (rho <= tol || (stalls && rho <= 10.0 * tol)) {
    ir.conv[g] = 1;
    return false;
  }
  if (stalls) ir.stalled[g] = 1;
  return true;
}

__global__ __launch_bounds__(kIrControlThreads) void k_ir_control(const ProbDesc* __restrict__ pd, NodeArrays na,
                                                                   IrState ir, int nnodes, int sweep, double tol) {
  __shared__ int unconv;
  if (threadIdx.x == 0) unconv = 0;
  __syncthreads();
  int mine = 0;
  for (int g = threadIdx.x; g < nnodes; g += blockDim.x)
    if (!ir.conv[g] && ir_control_node(pd, na, ir, g, sweep, tol)) ++mine;
  if (mine > 0) atomicAdd(&unconv, mine);
  __syncthreads();
  if (threadIdx.x == 0) ir.counters[0] = unconv;
}

__global__ void k_ir_reset(IrState ir, int nnodes) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nnodes * kNormStride) {
    ir.rnorm[i] = 0ull;
    ir.ynorm[i] = 0ull;
  }
  if (i < nnodes) {
    ir.conv[i] = 0;
    ir.stalled[i] = 0;
    ir.sweeps[i] = 0;
    ir.rho[i] = 1e300;
  }
  if (i == 0) {
    ir.counters[0] = 0;
    ir.counters[1] = 0;
    ir.counters[2] = 0;
    ir.counters[3] = INT_MAX;
  }
}

hipError_t ir_control(const ProbDesc* pd, const NodeArrays& na, IrState ir, int nnodes, int sweep, double tol,
                      hipStream_t st) {
  const int nt = std::min(kIrControlThreads, std::max(64, ceil_div(nnodes, 64) * 64));
  hipLaunchKernelGGL(k_ir_control, dim3(1), dim3(nt), 0, st, pd, na, ir, nnodes, sweep, tol);
  return hipGetLastError();
}

// Per-node status for the host in one block (one copy instead of one per
// array): rho[G] and the smallest pivot modulus pmin[G] (double), then info,
// conv, sweeps, bad (int each), then the four counters.
__global__ void k_gather_status(IrState ir, const int* __restrict__ info, const int* __restrict__ bad, int G,
                                char* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  double* rho = reinterpret_cast<double*>(out);
  int* iv = reinterpret_cast<int*>(out + 2 * (size_t)G * sizeof(double));
  if (g < G) {
    rho[g] = ir.rho[g];
    iv[g] = info[g];
    iv[G + g] = ir.conv[g];
    iv[2 * G + g] = ir.sweeps[g];
    iv[3 * G + g] = bad[g];
  }
  if (g < 4) iv[4 * G + g] = ir.counters[g];
}

size_t status_bytes(int G) { return (size_t)G * (2 * sizeof(double) + 4 * sizeof(int)) + 4 * sizeof(int); }

// Smallest pivot modulus |u_kk| of each node's factorization: logical row k
// of a factor sits at the physical row rows[k], so u_kk is T[rows[k], k].
// One group per matrix; a NaN pivot makes the minimum NaN.
template <typename P>
__global__ __launch_bounds__(256) void k_min_pivot(const MatDesc* __restrict__ md, const cx<P>* __restrict__ T,
                                                   const int* __restrict__ rows, double* __restrict__ out) {
  const MatDesc d = md[blockIdx.x];
  double m = INFINITY;
  for (int k = threadIdx.x; k < d.n; k += blockDim.x) {
    const cx<P> u = T[d.offT + (long long)rows[d.offRow + k] * d.ld + k];
    const double a = sqrt(double(u.re) * double(u.re) + double(u.im) * double(u.im));
    m = (a < m || a != a) ? a : m;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    const double x = __shfl_xor(m, o, 64);
    m = (x < m || x != x) ? x : m;
  }
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) m = (red[w] < m || red[w] != red[w]) ? red[w] : m;
    out[d.node] = (red[0] < m || red[0] != red[0]) ? red[0] : m;
  }
}

template <typename P>
hipError_t min_pivot(const MatDesc* md, int nmat, const cx<P>* T, const int* rows, int G, void* status,
                     hipStream_t st) {
  double* out = reinterpret_cast<double*>(static_cast<char*>(status) + (size_t)G * sizeof(double));
  hipLaunchKernelGGL(k_min_pivot<P>, dim3(nmat), dim3(256), 0, st, md, T, rows, out);
  return hipGetLastError();
}
template hipError_t min_pivot<float>(const MatDesc*, int, const c64*, const int*, int, void*, hipStream_t);

// log|det T| and arg det T of each node's factorization P T = L U (unit L):
// det T = sign(P) prod_k u_kk, with u_kk = T[rows[k], k] and sign(P) the
// parity of the row map k -> rows[k], counted by walking its cycles (one
// thread, an LDS bitmap of visited rows; n <= 4096).  out[node] = log|det|,
// out[nnodes + node] = arg det in (-pi, pi].
constexpr int kLogdetMaxN = 4096;

template <typename P>
__global__ __launch_bounds__(256) void k_logdet(const MatDesc* __restrict__ md, const cx<P>* __restrict__ T,
                                                const int* __restrict__ rows, int nnodes, double* __restrict__ out) {
  __shared__ unsigned seen[kLogdetMaxN / 32];
  __shared__ double rla[256], rar[256];
  __shared__ int parity;
  const MatDesc d = md[blockIdx.x];
  double la = 0.0, ar = 0.0;
  for (int k = threadIdx.x; k < d.n; k += blockDim.x) {
    const cx<P> u = T[d.offT + (long long)rows[d.offRow + k] * d.ld + k];
    const double re = double(u.re), im = double(u.im);
    la += log(hypot(re, im));
    ar += atan2(im, re);
  }
  for (int w = threadIdx.x; w < kLogdetMaxN / 32; w += blockDim.x) seen[w] = 0u;
  rla[threadIdx.x] = la;
  rar[threadIdx.x] = ar;
  __syncthreads();
  if (threadIdx.x == 0) {
    int cycles = 0;
    for (int s = 0; s < d.n; ++s) {
      if (seen[s >> 5] & (1u << (s & 31))) continue;
      ++cycles;
      int k = s;
      for (int step = 0; step < d.n && k >= 0 && k < d.n && !(seen[k >> 5] & (1u << (k & 31))); ++step) {
        seen[k >> 5] |= 1u << (k & 31);
        k = rows[d.offRow + k];
      }
    }
    parity = (d.n - cycles) & 1;
  }
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      rla[threadIdx.x] += rla[threadIdx.x + s];
      rar[threadIdx.x] += rar[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double a = rar[0] + (parity ? M_PI : 0.0);
    a = remainder(a, 2.0 * M_PI);  // into [-pi, pi]
    out[d.node] = rla[0];
    out[nnodes + d.node] = a;
  }
}

template <typename P>
hipError_t logdet_run(const MatDesc* md, int nmat, const cx<P>* T, const int* rows, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_logdet<P>, dim3(nmat), dim3(256), 0, st, md, T, rows, nmat, out);
  return hipGetLastError();
}
template hipError_t logdet_run<float>(const MatDesc*, int, const c64*, const int*, double*, hipStream_t);
template hipError_t logdet_run<double>(const MatDesc*, int, const c128*, const int*, double*, hipStream_t);
template hipError_t min_pivot<double>(const MatDesc*, int, const c128*, const int*, int, void*, hipStream_t);

hipError_t gather_status(IrState ir, const int* info, const int* bad, int G, void* out, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_status, dim3(ceil_div(std::max(G, 4), 256)), dim3(256), 0, st, ir, info, bad, G,
                     static_cast<char*>(out));
  return hipGetLastError();
}

hipError_t ir_reset(IrState ir, int nnodes, hipStream_t st) {
  hipLaunchKernelGGL(k_ir_reset, dim3(ceil_div(std::max(nnodes * kNormStride, 1), 256)), dim3(256), 0, st, ir, nnodes);
  return hipGetLastError();
}

}  // namespace nep
