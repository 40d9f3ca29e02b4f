// Blocked triangular solves for large matrices with many right-hand sides
// (complex FP32 factors): Y_j = T(z_j)^{-1} B with P T = L U.
//
// The per-node solve (k_trsv) streams a node's factor once per group of a
// few right-hand columns, and its update work runs on VALU.  For matrices of
// thousands of rows with tens of right-hand sides, the update work dominates
// and belongs on the matrix cores.  Here the right-hand sides of a node sit
// in a complex FP32 work buffer W (padded rows are zero), and each
// substitution runs over big blocks of nbk rows (a multiple of 64):
//   k_bs_diag : one group per (node, 4 right-hand columns) solves the big
//               block's diagonal part in LDS: for each 64-row sub-block,
//               x = Dinv t with the stored inverse of the LU, then the later
//               sub-blocks of the big block subtract (factor block) x;
//   k_bs_gemm : every row outside the big block (below it for L, above for
//               U) subtracts (factor rows) x_big on v_mfma_f32_32x32x2f32,
//               128 rows x 32 right-hand columns per group, the factor read
//               once per step;
//   k_bs_gather / k_bs_store: P b into W (through the row map), and the
//               result back to Y in FP64 (or added to it for a correction)
//               with the column maxima of |Y| for the refinement test.
// The arithmetic of a node depends on its own size only (the big-block
// partition starts at row 0 for every node), so a node solves identically
// alone and in a ragged batch.
#include "engine.hpp"

namespace nep {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kBsSub = 64;       // stored diagonal-block inverses: 64 x 64
constexpr int kBsBigMax = 256;   // largest big block
constexpr int kBsDiagCols = 4;   // right-hand columns per diagonal-solve group (256 threads: 64 rows x 4)
constexpr int kBsTM = 128, kBsTN = 32, kBsKC = 16;  // update tile (complex) and k chunk

__device__ __forceinline__ int bs_pad(int n) { return (n + kBsSub - 1) / kBsSub * kBsSub; }

// W = P b, complex FP32, rows past n zero.  Grid (chunks of npad*L, matrices).
__global__ __launch_bounds__(256) void k_bs_gather(const MatDesc* __restrict__ md, const ProbDesc* __restrict__ pd,
                                                   NodeArrays na, const int* __restrict__ rows,
                                                   const c128* __restrict__ R, int refine,
                                                   const int* __restrict__ conv, c64* __restrict__ W,
                                                   long long wstride, int npad) {
  const int b = blockIdx.y;
  const MatDesc d = md[b];
  const int g = d.node;
  if (conv != nullptr && conv[g]) return;
  const int p = na.prob[g], j = na.jnode[g];
  const ProbDesc& D = pd[p];
  const int L = D.L, n = d.n;
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long long)bs_pad(n) * L || e >= (long long)npad * L) return;
  const int r = (int)(e / L), c = (int)(e - (long long)r * L);
  c64 v = {0.f, 0.f};
  if (r < n) {
    const int pr = rows[d.offRow + r];
    const c128 bv =
        refine ? R[D.offY + (long long)pr * D.N * L + (long long)j * L + c] : D.V[(long long)c * n + pr];
    v = c64{float(bv.re), float(bv.im)};
  }
  W[(long long)b * wstride + e] = v;
}

// Diagonal part of big block kb.  Grid: matrices x column groups.  The
// blocks it needs form one list, in order: for each 64-row sub-block s (in
// solve order) the stored inverse of its diagonal block, then the factor
// blocks that carry x_s into the big block's later sub-blocks.  Each block
// is loaded into registers while the previous one is applied, and staged in
// one of two LDS buffers.
template <bool UPPER>
__global__ __launch_bounds__(256) void k_bs_diag(const MatDesc* __restrict__ md, const ProbDesc* __restrict__ pd,
                                                 NodeArrays na, const c64* __restrict__ Tb,
                                                 const int* __restrict__ rows, const c64* __restrict__ Dinv,
                                                 const long long* __restrict__ dinv_off,
                                                 const int* __restrict__ conv, c64* __restrict__ W,
                                                 long long wstride, int kb, int nbk, int cgroups) {
  constexpr int B = kBsSub, C = kBsDiagCols, PER = B * B / 256;
  const int b = blockIdx.x / cgroups, cg = blockIdx.x - b * cgroups;
  const MatDesc d = md[b];
  const int g = d.node;
  if (conv != nullptr && conv[g]) return;
  const int n = d.n, ld = d.ld;
  const int R0 = kb * nbk;
  if (R0 >= n) return;
  const int L = pd[na.prob[g]].L;
  const int c0 = cg * C;
  const int nsub = min(nbk, bs_pad(n) - R0) / B;
  const c64* __restrict__ T = Tb + d.offT;
  const int* __restrict__ rat = rows + d.offRow;
  const c64* __restrict__ Di0 = Dinv + dinv_off[b];
  c64* __restrict__ Wb = W + (long long)b * wstride;

  __shared__ c64 Ts[kBsBigMax][C];   // the big block's right-hand sides, then solutions
  __shared__ c64 Fs[2][B][B + 1];    // stored inverses and factor blocks, double-buffered
  __shared__ c64 Xs[B][C];           // the current sub-block's solution
  const int tid = threadIdx.x;
  const int ti = tid / C, tc = tid % C;  // this thread's row and column

  // list entry e -> (s, s2): s2 == s is the inverse of sub-block s, otherwise
  // the factor block (s2, s); the list has nsub (nsub + 1) / 2 entries
  auto entry = [&](int e, int& s, int& s2) {
    for (int ss = 0; ss < nsub; ++ss) {
      const int sv = UPPER ? nsub - 1 - ss : ss;
      const int cnt = UPPER ? sv + 1 : nsub - sv;  // the inverse and the blocks after it
      if (e < cnt) {
        s = sv;
        s2 = UPPER ? sv - e : sv + e;
        return;
      }
      e -= cnt;
    }
    s = s2 = 0;
  };
  c64 pf[PER];
  auto load = [&](int e) {
    int s, s2;
    entry(e, s, s2);
    const int blk = R0 / B + s;
    if (s2 == s) {
      const c64* __restrict__ Di = Di0 + ((long long)blk * 2 + (UPPER ? 1 : 0)) * B * B;
#pragma unroll
      for (int u = 0; u < PER; ++u) pf[u] = Di[tid + 256 * u];
    } else {
      const int rb = (R0 / B + s2) * B;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int ee = tid + 256 * u, i = ee / B, k = ee % B;
        const int r = rb + i, col = blk * B + k;
        pf[u] = (r < n && col < n) ? T[(long long)rat[r] * ld + col] : c64{0.f, 0.f};
      }
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int ee = tid + 256 * u;
      Fs[buf][ee / B][ee % B] = pf[u];
    }
  };

  for (int e = tid; e < nsub * B * C; e += 256) {
    const int r = e / C, c = e - r * C;
    Ts[r][c] = c0 + c < L ? Wb[(long long)(R0 + r) * L + c0 + c] : c64{0.f, 0.f};
  }
  const int ne = nsub * (nsub + 1) / 2;
  load(0);
  stage(0);
  __syncthreads();
  int xs_of = -1;  // sub-block whose solution is in Xs, not yet copied to Ts
  for (int e = 0; e < ne; ++e) {
    if (e + 1 < ne) load(e + 1);  // in flight while this block is applied
    int s, s2;
    entry(e, s, s2);
    const int buf = e & 1;
    if (s2 == s) {  // x_s = Dinv t_s (the inverse is identity-padded past n)
      if (xs_of >= 0) Ts[xs_of * B + ti][tc] = Xs[ti][tc];  // the previous solution, own element
      c64 a = {0.f, 0.f};
#pragma unroll 16
      for (int k = 0; k < B; ++k) a = cmac(a, Fs[buf][ti][k], Ts[s * B + k][tc]);
      __syncthreads();  // every thread has read Xs and Ts[s]
      Xs[ti][tc] = a;
      xs_of = s;
    } else {  // t_s2 -= F(s2, s) x_s
      c64 a = Ts[s2 * B + ti][tc];
#pragma unroll 16
      for (int k = 0; k < B; ++k) a = fms(a, Fs[buf][ti][k], Xs[k][tc]);
      Ts[s2 * B + ti][tc] = a;
    }
    if (e + 1 < ne) stage(buf ^ 1);
    __syncthreads();
  }
  if (xs_of >= 0) Ts[xs_of * B + ti][tc] = Xs[ti][tc];
  __syncthreads();
  for (int e = tid; e < nsub * B * C; e += 256) {
    const int r = e / C, c = e - r * C;
    if (c0 + c < L) Wb[(long long)(R0 + r) * L + c0 + c] = Ts[r][c];
  }
}

// Rows [rlo, min(rhi, n)) outside big block kb subtract (factor rows over the
// block's columns) times the block's solution.  Grid: matrices x row tiles x
// column tiles.
// Operand lane roles and the accumulator layout follow the LU's trailing
// update: the A operand carries the real 2 x 2 embedding of the complex
// factor entries (with the sign of the subtraction), B the real and
// imaginary planes of x, and C is loaded into the accumulators.
template <bool UPPER>
__global__ __launch_bounds__(256) void k_bs_gemm(const MatDesc* __restrict__ md, const ProbDesc* __restrict__ pd,
                                                 NodeArrays na, const c64* __restrict__ Tb,
                                                 const int* __restrict__ rows, const int* __restrict__ conv,
                                                 c64* __restrict__ W, long long wstride, int kb, int nbk,
                                                 int rlo, int rhi, int tiles_m, int tiles_n) {
  const int per = tiles_m * tiles_n;
  const int v = blockIdx.x;
  const int b = v / per, t = v - b * per;
  const int tm = t / tiles_n, tn = t - tm * tiles_n;
  const MatDesc d = md[b];
  const int g = d.node;
  if (conv != nullptr && conv[g]) return;
  const int n = d.n, ld = d.ld;
  const int K0 = kb * nbk;
  if (K0 >= n) return;
  const int KB = min(nbk, bs_pad(n) - K0);
  const int rbeg = rlo, rend = min(rhi, n);
  const int row0 = rbeg + tm * kBsTM;
  if (row0 >= rend) return;
  const int L = pd[na.prob[g]].L;
  const int col0 = tn * kBsTN;
  if (col0 >= L) return;
  const c64* __restrict__ T = Tb + d.offT;
  const int* __restrict__ rat = rows + d.offRow;
  c64* __restrict__ Wb = W + (long long)b * wstride;

  __shared__ float As[2][kBsKC][2 * kBsTM + 4];
  __shared__ float Bs[2][kBsKC][2][kBsTN + 4];
  __shared__ long long aoff_s[kBsTM];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < kBsTM) {
    const int r = row0 + tid;
    aoff_s[tid] = r < rend ? (long long)rat[r] * ld : -1;
  }
  __syncthreads();

  constexpr int AQ = kBsTM * kBsKC / 2 / 256;  // 4 k-pairs per thread
  const int kp = tid & 7;
  long long aoff[AQ];
  bool aval[AQ];
#pragma unroll
  for (int q = 0; q < AQ; ++q) {
    const long long o = aoff_s[(tid >> 3) + 32 * q];
    aval[q] = o >= 0;
    aoff[q] = o >= 0 ? o : 0;
  }
  const int bk = tid >> 4, bcp = tid & 15;  // B: k row, column pair
  const int gc = col0 + 2 * bcp;
  const bool bv0 = gc < L, bv1 = gc + 1 < L;
  const int gcl = min(gc, L - 2);  // clamped inside the row (L is even)

  float4 ra[AQ], rb;
  auto load_chunk = [&](int kk) {
    // columns past n (up to the 64-row padding) are masked when staged; the
    // address is clamped inside the row (ld is even and at least n)
    const int kc2 = min(K0 + kk + 2 * kp, ld - 2);
#pragma unroll
    for (int q = 0; q < AQ; ++q) ra[q] = *reinterpret_cast<const float4*>(T + aoff[q] + kc2);
    rb = *reinterpret_cast<const float4*>(Wb + (long long)(K0 + kk + bk) * L + gcl);
  };
  auto store_chunk = [&](int buf, int kk) {
    const int kg = K0 + kk + 2 * kp;  // factor columns kg, kg + 1
    const bool k0ok = kg < n, k1ok = kg + 1 < n;
#pragma unroll
    for (int q = 0; q < AQ; ++q) {
      const int r = (tid >> 3) + 32 * q;
      const bool va = aval[q];
      As[buf][2 * kp][2 * r] = va && k0ok ? ra[q].x : 0.f;
      As[buf][2 * kp][2 * r + 1] = va && k0ok ? ra[q].y : 0.f;
      As[buf][2 * kp + 1][2 * r] = va && k1ok ? ra[q].z : 0.f;
      As[buf][2 * kp + 1][2 * r + 1] = va && k1ok ? ra[q].w : 0.f;
    }
    Bs[buf][bk][0][2 * bcp] = bv0 ? rb.x : 0.f;
    Bs[buf][bk][1][2 * bcp] = bv0 ? rb.y : 0.f;
    Bs[buf][bk][0][2 * bcp + 1] = bv1 ? rb.z : 0.f;
    Bs[buf][bk][1][2 * bcp + 1] = bv1 ? rb.w : 0.f;
  };

  // each wave: 32 complex rows (two 16-row blocks) x 32 columns
  const int wr = wave * 32;
  const bool wlive = row0 + wr < rend;
  floatx16 acc[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int gcol = col0 + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; r += 2) {
      const int lr = wr + i * 16 + 4 * (r >> 2) + 2 * (lane >> 5) + ((r & 3) >> 1);
      const bool ok = wlive && row0 + lr < rend && gcol < L;
      c64 cv = {0.f, 0.f};
      if (ok) cv = Wb[(long long)(row0 + lr) * L + gcol];
      acc[i][r] = cv.re;
      acc[i][r + 1] = cv.im;
    }
  }
  const int at = lane & 1, au = lane >> 5, arow = (lane & 31) >> 1;
  const int acomp = at ^ au;
  const float asign = ((at == 0 && au == 1) ? -1.f : 1.f) * -1.f;  // C -= A B
  const int bcol = lane & 31, bu = lane >> 5;

  const int nk = KB / kBsKC;
  load_chunk(0);
  store_chunk(0, 0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) load_chunk((kc + 1) * kBsKC);
    if (wlive) {
#pragma unroll
      for (int k = 0; k < kBsKC; ++k) {
        const float a0 = asign * As[buf][k][2 * (wr + arow) + acomp];
        const float a1 = asign * As[buf][k][2 * (wr + 16 + arow) + acomp];
        const float bb = Bs[buf][k][bu][bcol];
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, bb, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, bb, acc[1], 0, 0, 0);
      }
    }
    if (kc + 1 < nk) {
      store_chunk(buf ^ 1, (kc + 1) * kBsKC);
      __syncthreads();
    }
  }
  if (!wlive) return;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int gcol = col0 + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; r += 2) {
      const int lr = wr + i * 16 + 4 * (r >> 2) + 2 * (lane >> 5) + ((r & 3) >> 1);
      if (row0 + lr < rend && gcol < L) Wb[(long long)(row0 + lr) * L + gcol] = c64{acc[i][r], acc[i][r + 1]};
    }
  }
}

// Y = x (or Y += x), FP64, with the column maxima of |Y|.  Grid (row chunks,
// matrices); each group takes kBsStoreRows rows.
constexpr int kBsStoreRows = 64;
__global__ __launch_bounds__(256) void k_bs_store(const MatDesc* __restrict__ md, const ProbDesc* __restrict__ pd,
                                                  NodeArrays na, const int* __restrict__ conv,
                                                  const c64* __restrict__ W, long long wstride,
                                                  c128* __restrict__ Y, int refine, IrState ir) {
  const int b = blockIdx.y;
  const MatDesc d = md[b];
  const int g = d.node;
  if (conv != nullptr && conv[g]) return;
  const int p = na.prob[g], j = na.jnode[g];
  const ProbDesc& D = pd[p];
  const int n = d.n, L = D.L;
  const int r0 = blockIdx.x * kBsStoreRows;
  if (r0 >= n) return;
  __shared__ unsigned long long cm[64];
  if (threadIdx.x < 64) cm[threadIdx.x] = 0ull;
  __syncthreads();
  const int nr = min(kBsStoreRows, n - r0);
  const c64* __restrict__ Wb = W + (long long)b * wstride;
  for (int e = threadIdx.x; e < nr * L; e += 256) {
    const int r = r0 + e / L, c = e % L;
    const c64 x = Wb[(long long)r * L + c];
    c128* y = Y + D.offY + (long long)r * D.N * L + (long long)j * L + c;
    c128 nv = {double(x.re), double(x.im)};
    if (refine) nv = *y + nv;
    *y = nv;
    // non-negative doubles order as their bits; a NaN's bits order above
    // every finite value, so the maximum stays NaN
    atomicMax(&cm[c], (unsigned long long)__double_as_longlong(sqrt(norm2(nv))));
  }
  __syncthreads();
  if ((int)threadIdx.x < L)
    atomicMax(&ir.ynorm[(long long)g * kNormStride + threadIdx.x], cm[threadIdx.x]);
}

// Substitution order: per big block, the diagonal part, then every row
// beyond it in solve order.  (Splitting that update into the next big
// block's rows and the rest, the rest on a second stream beside the next
// diagonal part, measured slower at n = 4096: the concurrent update took the
// CUs the diagonal part needed, 5.95 ms per solve against 4.3.)
hipError_t solve_blocked(const SolvePlan& sp, const ProbDesc* pd, const MatDesc* md, const NodeArrays& na,
                         const c64* T, const int* rows, const c64* Dinv, const long long* dinv_off,
                         const c128* R, c128* Y, bool refine, const int* conv, IrState ir, hipStream_t st) {
  const int nm = sp.nblk, L = sp.L, npad = sp.npad, nbk = sp.nbk;
  if (nm <= 0) return hipSuccess;
  if (sp.W == nullptr || nbk % kBsSub != 0 || nbk > kBsBigMax || L % 2 != 0 || L > 64) return hipErrorInvalidValue;
  const long long wstride = (long long)npad * L;
  const int rf = refine ? 1 : 0;
  hipLaunchKernelGGL(k_bs_gather, dim3(ceil_div(npad * L, 256), nm), dim3(256), 0, st, md, pd, na, rows, R, rf, conv,
                     sp.W, wstride, npad);
  const int nkb = ceil_div(npad, nbk);
  const int cgroups = ceil_div(L, kBsDiagCols), tiles_n = ceil_div(L, kBsTN);
  for (int kb = 0; kb < nkb; ++kb) {  // L y = P b
    hipLaunchKernelGGL(k_bs_diag<false>, dim3(nm * cgroups), dim3(256), 0, st, md, pd, na, T, rows, Dinv, dinv_off,
                       conv, sp.W, wstride, kb, nbk, cgroups);
    const int r0 = (kb + 1) * nbk;
    if (r0 < npad) {
      const int tiles_m = ceil_div(npad - r0, kBsTM);
      hipLaunchKernelGGL(k_bs_gemm<false>, dim3(nm * tiles_m * tiles_n), dim3(256), 0, st, md, pd, na, T, rows, conv,
                         sp.W, wstride, kb, nbk, r0, npad, tiles_m, tiles_n);
    }
  }
  for (int kb = nkb - 1; kb >= 0; --kb) {  // U x = y
    hipLaunchKernelGGL(k_bs_diag<true>, dim3(nm * cgroups), dim3(256), 0, st, md, pd, na, T, rows, Dinv, dinv_off,
                       conv, sp.W, wstride, kb, nbk, cgroups);
    if (kb > 0) {
      const int tiles_m = ceil_div(kb * nbk, kBsTM);
      hipLaunchKernelGGL(k_bs_gemm<true>, dim3(nm * tiles_m * tiles_n), dim3(256), 0, st, md, pd, na, T, rows, conv,
                         sp.W, wstride, kb, nbk, 0, kb * nbk, tiles_m, tiles_n);
    }
  }
  hipLaunchKernelGGL(k_bs_store, dim3(ceil_div(npad, kBsStoreRows), nm), dim3(256), 0, st, md, pd, na, conv, sp.W,
                     wstride, Y, rf, ir);
  return hipGetLastError();
}

}  // namespace nep
