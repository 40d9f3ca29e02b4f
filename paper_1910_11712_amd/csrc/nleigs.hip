// NLEIGS (Section 4.5).  The split operator is replaced by a rational
// interpolant R_d in the rational Newton basis (eqs. (nleigsbj), (nleigsq))
// whose nodes and poles are Leja--Bagby points (eq. (nleigsleja)); the
// eigenvalues near a shift sigma are those of the linearization pencil of
// eq. (nleigsmatlin), found by Arnoldi on its shift-and-invert operator
// (eq. (nleigssinvert)) with the Krylov basis in the TOAR representation
// (Algorithm "Arnoldi for NLEIGS with TOAR representation").
//
// Work split.  The host takes the scalar set-up (boundary discretization,
// greedy Leja--Bagby selection, basis scaling, divided differences, degree)
// and the coefficient recurrences of the TOAR representation, which act on
// vectors of length k + d.  The device takes everything of size n: the
// function values at the nodes, the assembly and LU of
// R_d(sigma) = sum_i rho_i A_i with the moment plan's kernels (explicit
// coefficients rho_i in place of f_i(z)), and per Arnoldi step the
// reconstruction U q_i of the vector that multiplies each A_i, the split-form
// product -sum_i A_i (U q_i), the solve with the resident factors of
// R_d(sigma), and classical Gram--Schmidt with one reorthogonalization of the
// new vector against U.  A step reads every A_i once and the factors once, so
// it is bound by HBM bandwidth (for one large matrix, by the latency of the
// solve's chain of 64-row blocks).  nep_nleigs_batch runs many problems at
// once: one batched LU of every R_d(sigma_p), and each step's products,
// solves (the moment plan's batched solve) and Gram--Schmidt as single launches
// over all problems, with the per-problem host work on a thread pool.
//
// The divided-difference matrices D_j are never formed (Section 4.5): with
// q_i = sum_{j<d-1} d_i^j g~^{j+1} + (d_i^d / beta_d) g^{d-1}, the right-hand
// side -sum_j D_j y^{j+1} - D_d v^{d-1} / beta_d of eq. (nleigs-toar2) is
// -sum_i A_i U q_i.
//
// Readings where the text leaves a choice: b_0 = 1 (so beta_0 = 1); sigma_0
// is the boundary point at angle 0; ties of the greedy selections go to the
// lowest index among candidates within a relative 1e-10 of the extreme;
// |s_j| is infinite at a point already taken as a pole, so each point of the
// singularity set serves at most once and the remaining poles are infinite;
// the degree is the first j >= 2 with max_i |d_i^j| / max_i |d_i^0| < tol; the
// last pole is then set to infinity and beta_d, d_i^d recomputed.  The scalar
// divided differences follow the interpolation recurrence of eq. (nleigsdd)
// applied to each f_i (the quantity eq. (nleigsfdd) evaluates through a
// matrix function).  No Krylov--Schur restart: one Arnoldi run of k steps.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "dense.hpp"
#include "fn_device.hpp"
#include "handle.hpp"
#include "lu.hpp"

namespace nep {

namespace {

constexpr int kNlMaxK = 256;       // Arnoldi steps
constexpr int kNlMaxDeg = 100;     // interpolation degree
constexpr int kNlMaxPts = 16384;   // boundary discretization
constexpr double kNlTie = 1e-10;   // relative tie window of the greedy selections
constexpr double kNlDep = 1e-12;   // a new vector this small after Gram--Schmidt
                                   // (relative) does not extend U

// ---------------------------------------------------------------------------
// Device kernels
// ---------------------------------------------------------------------------

__device__ __forceinline__ c128 wave_sum(c128 v) {
  for (int o = 32; o >= 1; o >>= 1) {
    v.re += __shfl_xor(v.re, o, 64);
    v.im += __shfl_xor(v.im, o, 64);
  }
  return v;
}

// Sum over a 256-thread group; every thread gets the total.
__device__ __forceinline__ c128 group_sum(c128 v, c128* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  c128 s = red[0];
  for (int i = 1; i < 4; ++i) s = s + red[i];
  __syncthreads();
  return s;
}

// Z[:, c] = U[:, 0:m] Q[:, c] (sub = 0) or Z[:, c] -= U[:, 0:m] Q[:, c]
// (sub = 1).  U column-major with leading dimension n, Q column-major with
// leading dimension m.  One thread per row, one grid row per column c.
__global__ __launch_bounds__(64) void k_nl_comb(int n, int m, const c128* __restrict__ U,
                                                const c128* __restrict__ Q, c128* __restrict__ Z, int sub) {
  const int r = blockIdx.x * 64 + threadIdx.x, c = blockIdx.y;
  if (r >= n) return;
  const c128* q = Q + (long long)c * m;
  c128 a0 = {0.0, 0.0}, a1 = {0.0, 0.0};
  int t = 0;
  for (; t + 1 < m; t += 2) {  // two independent chains keep two loads in flight
    a0 = a0 + U[(long long)t * n + r] * q[t];
    a1 = a1 + U[(long long)(t + 1) * n + r] * q[t + 1];
  }
  if (t < m) a0 = a0 + U[(long long)t * n + r] * q[t];
  const c128 acc = a0 + a1;
  c128* z = Z + (long long)c * n + r;
  *z = sub ? *z - acc : acc;
}

// ---------------------------------------------------------------------------
// Triangular solves with the factors of one matrix, one right-hand side.
//
// The batched solve kernels give a whole matrix to one group, which suits
// many matrices and probe columns; a Krylov step solves with one matrix and
// one vector, so here the 64-row blocks of the triangle go to separate
// groups (n/64 of them) and each group streams its own block row of the
// factor while the solutions of the blocks before it appear:
//   y_q = Dinv_q (b_q - sum_{c<q} L_qc y_c)   (forward; U backwards)
// with the stored inverses of the 64 x 64 diagonal blocks.  Thread (wave w,
// lane l) owns rows 16w..16w+15 of the block and column l of every column
// block (coalesced row segments); its 16 partial sums are reduced over the
// wave once, at the end.  A group takes its block from a ticket counter, so
// blocks are taken in launch order and a group only waits for blocks already
// held by running groups; the waits are bounded (a wait that runs out sets
// *err and the group finishes with wrong values instead of hanging).  Block
// solutions are published by a release store of the solve's epoch into the
// block's flag; readers acquire it at agent scope before loading the block.
// ---------------------------------------------------------------------------
constexpr int kNlBlk = 64;
constexpr int kNlSpinMax = 1 << 22;  // polls of one wait (about 0.3 s)

// Waits until *flag == epoch (relaxed polls; the caller's acquire fence
// follows the wait once).  Once any wait has run out (*err set), no group
// waits any more, so a failed solve costs one bound, not one per block.
__device__ __forceinline__ void wait_flag(const int* flag, int epoch, int* err) {
  int it = 0;
  while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
    if (++it > kNlSpinMax || ((it & 1023) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
      atomicExch(err, 1);
      break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// UPPER = 0: out = L^{-1} P b with b gathered through the row map (b in
// physical row order); UPPER = 1: out = U^{-1} b.  T: row-major factor with
// leading dimension ld, rat: the row map, Di: the diagonal-block inverses.
// A group of 512 threads owns two consecutive 64-row blocks: waves 0-3 the
// one solved first (the lower-indexed for L, the higher for U), waves 4-7 the
// other, whose coupling to the first is applied inside the group (LDS and a
// barrier instead of a flag round trip through memory), so the chain of
// cross-group waits is n/128 long.
template <bool UPPER>
__global__ __launch_bounds__(512) void k_nl_tri(int n, int ld, const c128* __restrict__ T,
                                                const int* __restrict__ rat, const c128* __restrict__ Di,
                                                const c128* __restrict__ b, c128* out, int* flags, int* ticket,
                                                int epoch, int* err) {
  constexpr int B = kNlBlk;
  __shared__ c128 Dsh[2][B][B + 1];
  __shared__ c128 tq[2][B];
  __shared__ c128 ysh[2][B];
  __shared__ int s_t;
  const int nblk = (n + B - 1) / B, npair = (nblk + 1) / 2;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int half = w >> 2;            // 0: the block solved first, 1: the other
  const int hw = w & 3, htid = tid & 255;
  if (tid == 0) s_t = atomicAdd(ticket, 1) - (epoch - 1) * npair;
  __syncthreads();
  const int tk = s_t;
  if (tk < 0 || tk >= npair) return;  // not reached with npair groups per epoch
  const int pr = UPPER ? npair - 1 - tk : tk;
  // the group's blocks in solve order; the higher one may lie past n (odd nblk)
  const int qf = UPPER ? min(2 * pr + 1, nblk - 1) : 2 * pr;
  const int qs = UPPER ? (2 * pr + 1 < nblk ? 2 * pr : -1) : (2 * pr + 1 < nblk ? 2 * pr + 1 : -1);
  const int qmine = half == 0 ? qf : qs;  // this wave's block (-1: none)
  // the diagonal-block inverses (identity past n)
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int qq = h == 0 ? qf : qs;
    if (qq < 0) continue;
    const c128* D = Di + ((long long)qq * 2 + (UPPER ? 1 : 0)) * B * B;
    for (int e = tid; e < B * B; e += 512) Dsh[h][e / B][e % B] = D[e];
  }
  // physical rows of this thread's 16 logical rows
  long long roff[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int r = qmine < 0 ? n : qmine * B + 16 * hw + i;
    roff[i] = r < n ? (long long)rat[r] * ld : -1;
  }
  c128 acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = c128{0.0, 0.0};
  // this wave's 16 right-hand-side entries, loaded now (they do not depend on
  // the chain): lane i < 16 holds row 16 hw + i
  c128 rhs_mine = {0.0, 0.0};
  if (lane < 16 && qmine >= 0) {
    const int r = qmine * B + 16 * hw + lane;
    if (r < n) rhs_mine = UPPER ? b[r] : b[rat[r]];
  }
  // column blocks solved by other groups, in the order they appear
  const int c_first = UPPER ? nblk - 1 : 0;
  const int ncb = UPPER ? max(0, nblk - 1 - max(qf, qs)) : 2 * pr;
  auto cb = [&](int s) { return UPPER ? c_first - s : c_first + s; };
  c128 seg[16];
  auto load_seg = [&](int c) {
    const int col = c * B + lane;
#pragma unroll
    for (int i = 0; i < 16; ++i) seg[i] = (roff[i] >= 0 && col < n) ? T[roff[i] + col] : c128{0.0, 0.0};
  };
  // waves 4-7 also need the segment of the first block (their coupling)
  const int nseg = ncb + (half == 1 ? 1 : 0);
  auto seg_col = [&](int s) { return s < ncb ? cb(s) : qf; };
  if (nseg > 0) load_seg(seg_col(0));
  // Blocks are published in the order cb(0), cb(1), ... (a group publishes
  // only after consuming every block before its own), so once the flag of
  // cb(ncb - 1) is seen, every block this group needs is there: one wait and
  // one acquire cover them all, and each block's solution can be loaded one
  // block ahead like the factor segments.
  int known = 0;  // blocks cb(0..known-1) are acquired
  c128 ynext = {0.0, 0.0};
  for (int s = 0; s < ncb; ++s) {
    const int c = cb(s);
    const int col = c * B + lane;
    c128 yc;
    if (s >= known) {
      int kn = s + 1;
      if (lane == 0) {
        wait_flag(flags + c, epoch, err);
        if (s + 1 < ncb &&
            __hip_atomic_load(flags + cb(ncb - 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch)
          kn = ncb;
      }
      known = __shfl(kn, 0, 64);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      yc = col < n ? out[col] : c128{0.0, 0.0};
    } else {
      yc = ynext;
    }
    if (s + 1 < known) {
      const int ncol = cb(s + 1) * B + lane;
      ynext = ncol < n ? out[ncol] : c128{0.0, 0.0};
    }
    c128 cur[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) cur[i] = seg[i];
    if (s + 1 < nseg) load_seg(seg_col(s + 1));  // the next segment loads during this one's use
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = acc[i] + cur[i] * yc;
  }
  // solve the group's blocks in order: t_q = b_q - row sums, y_q = Dinv_q t_q
  auto publish_sums = [&](int h) {  // waves of half h
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = wave_sum(acc[i]);
    if (lane < 16) {
      c128 v = {0.0, 0.0};
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (i == lane) v = acc[i];
      tq[h][16 * hw + lane] = rhs_mine - v;
    }
  };
  auto apply_inverse = [&](int h) {  // the 256 threads of half h: four per row
    const int i = htid >> 2, k0 = (htid & 3) * 16;
    c128 y = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 16; ++k) y = y + Dsh[h][i][k0 + k] * tq[h][k0 + k];
    y.re += __shfl_xor(y.re, 1, 64);
    y.im += __shfl_xor(y.im, 1, 64);
    y.re += __shfl_xor(y.re, 2, 64);
    y.im += __shfl_xor(y.im, 2, 64);
    if ((htid & 3) == 0) ysh[h][i] = y;
  };
  auto store_publish = [&](int h, int q) {  // one wave: its release orders its own stores before the flag
    if (q * B + lane < n) out[q * B + lane] = ysh[h][lane];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0) __hip_atomic_store(flags + q, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  if (half == 0) publish_sums(0);
  __syncthreads();
  if (half == 0) apply_inverse(0);
  __syncthreads();
  if (w == 0) store_publish(0, qf);
  if (qs < 0) return;  // wave-uniform: no second block
  if (half == 1) {
    // coupling to the first block: seg holds its segment
    const c128 yc = ysh[0][lane];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = acc[i] + seg[i] * yc;
    publish_sums(1);
  }
  __syncthreads();
  if (half == 1) apply_inverse(1);
  __syncthreads();
  if (w == 4) store_publish(1, qs);
}

struct NlTerms {
  const void* A[kMaxTerms];     // row-major n x n, double or complex
  const c128* diag[kMaxTerms];  // diagonal of a diagonal A_i
  int cplx[kMaxTerms];
  int isdiag[kMaxTerms];
};

// out[r] = -sum_i (A_i Z[:, i])[r].  One wavefront per row (lanes stride the
// row, so each load of a wavefront is 64 consecutive entries), four rows per
// group; a diagonal A_i contributes d_r z_r.
__global__ __launch_bounds__(256) void k_nl_splitmv(int n, int ell, NlTerms T, const c128* __restrict__ Z,
                                                    c128* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  c128 acc = {0.0, 0.0};
  for (int i = 0; i < ell; ++i) {
    const c128* z = Z + (long long)i * n;
    if (T.isdiag[i]) {
      if (lane == 0) acc = acc + T.diag[i][r] * z[r];
    } else if (T.cplx[i]) {
      const c128* a = reinterpret_cast<const c128*>(T.A[i]) + (long long)r * n;
#pragma unroll 4
      for (int c = lane; c < n; c += 64) acc = acc + a[c] * z[c];
    } else {
      const double* a = reinterpret_cast<const double*>(T.A[i]) + (long long)r * n;
#pragma unroll 4
      for (int c = lane; c < n; c += 64) {
        const double v = a[c];
        const c128 zc = z[c];
        acc.re += v * zc.re;
        acc.im += v * zc.im;
      }
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) out[r] = -acc;
}

// h[t] = U[:, t]^H y, t < m: one group per column.
__global__ __launch_bounds__(256) void k_nl_dots(int n, const c128* __restrict__ U, const c128* __restrict__ y,
                                                 c128* __restrict__ h) {
  __shared__ c128 red[4];
  const c128* u = U + (long long)blockIdx.x * n;
  c128 acc = {0.0, 0.0};
  for (int r = threadIdx.x; r < n; r += 256) acc = acc + conj(u[r]) * y[r];
  const c128 s = group_sum(acc, red);
  if (threadIdx.x == 0) h[blockIdx.x] = s;
}

// out = ||y||_2 (one group).
__global__ __launch_bounds__(256) void k_nl_norm(int n, const c128* __restrict__ y, double* __restrict__ out) {
  __shared__ c128 red[4];
  double acc = 0.0;
  for (int r = threadIdx.x; r < n; r += 256) acc += norm2(y[r]);
  const c128 s = group_sum(c128{acc, 0.0}, red);
  if (threadIdx.x == 0) *out = sqrt(s.re);
}

// u = y / nrm (nrm read on the device; 0 leaves u = 0).
// (y and u may be the same vector.)
__global__ __launch_bounds__(256) void k_nl_store(int n, const c128* y, const double* nrm, c128* u) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double s = *nrm > 0.0 ? 1.0 / *nrm : 0.0;
  u[r] = s * y[r];
}

// x = U[:, 0:m] s, scaled to 2-norm 1 with its largest-modulus entry (lowest
// index among equals) real and positive: the body of one 256-thread group.
__device__ void nl_vector(int n, int m, const c128* __restrict__ U, const c128* __restrict__ s,
                          c128* __restrict__ x) {
  __shared__ c128 red[4];
  __shared__ double wmax[4];
  __shared__ int widx[4];
  double ss = 0.0, bm = -1.0;
  int bi = 0x7fffffff;
  for (int r = threadIdx.x; r < n; r += 256) {
    c128 acc = {0.0, 0.0};
    for (int t = 0; t < m; ++t) acc = acc + U[(long long)t * n + r] * s[t];
    x[r] = acc;
    const double a2 = norm2(acc);
    ss += a2;
    if (a2 > bm) {
      bm = a2;
      bi = r;
    }
  }
  const c128 tot = group_sum(c128{ss, 0.0}, red);
  for (int o = 32; o >= 1; o >>= 1) {
    const double ov = __shfl_xor(bm, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (ov > bm || (ov == bm && oi < bi)) {
      bm = ov;
      bi = oi;
    }
  }
  if ((threadIdx.x & 63) == 0) {
    wmax[threadIdx.x >> 6] = bm;
    widx[threadIdx.x >> 6] = bi;
  }
  __syncthreads();
  bm = wmax[0];
  bi = widx[0];
  for (int w = 1; w < 4; ++w)
    if (wmax[w] > bm || (wmax[w] == bm && widx[w] < bi)) {
      bm = wmax[w];
      bi = widx[w];
    }
  const c128 piv = x[bi];
  const double ap = sqrt(norm2(piv)), nrm = sqrt(tot.re);
  const c128 sc = (ap > 0.0 && nrm > 0.0) ? c128{piv.re / (ap * nrm), -piv.im / (ap * nrm)} : c128{0.0, 0.0};
  __syncthreads();
  for (int r = threadIdx.x; r < n; r += 256) x[r] = sc * x[r];
}

// X[:, q] = U[:, 0:m] S[:, q] (normalized as above): one group per column
__global__ __launch_bounds__(256) void k_nl_vectors(int n, int m, const c128* __restrict__ U,
                                                    const c128* __restrict__ S, c128* __restrict__ X) {
  nl_vector(n, m, U, S + (long long)blockIdx.x * m, X + (long long)blockIdx.x * n);
}

// ---------------------------------------------------------------------------
// Batched NLEIGS: one run over many problems at once.  Every problem has its
// own basis U_p, terms and sizes (descriptor below); the per-step basis size
// m_p comes from a device array (negative: the problem takes no part).  The
// factorizations and solves are the moment plan's batched LU and solve
// kernels over one node per problem.
// ---------------------------------------------------------------------------
struct NlbProb {
  int n, ell;
  long long offU;  // U_p: column-major n x (mmax+1) at U + offU
  long long offZ;  // U_p q_i: n x ell at Z + offZ
  long long offY;  // right-hand side (R) and solution (Y) in the plan's buffers
  NlTerms t;
  const double* normA;  // ell infinity norms
  const FnNode* fn_nodes;
  const c128* fn_coef;
  int fn_root[kMaxTerms];
};

// Z_p[:, c] = U_p[:, 0:m_p] Q_p[:, c], c < ell_p; Q_p at Q + p * qstride
__global__ __launch_bounds__(64) void k_nlb_rhs(const NlbProb* __restrict__ pb, const int* __restrict__ dm,
                                                const c128* __restrict__ U, const c128* __restrict__ Q,
                                                long long qstride, c128* __restrict__ Z) {
  const int p = blockIdx.z, c = blockIdx.y, r = blockIdx.x * 64 + threadIdx.x;
  const NlbProb& P = pb[p];
  const int m = dm[p];
  if (m < 0 || c >= P.ell || r >= P.n) return;
  const c128* u = U + P.offU + r;
  const c128* q = Q + p * qstride + (long long)c * m;
  c128 a0 = {0.0, 0.0}, a1 = {0.0, 0.0};
  int t = 0;
  for (; t + 1 < m; t += 2) {
    a0 = a0 + u[(long long)t * P.n] * q[t];
    a1 = a1 + u[(long long)(t + 1) * P.n] * q[t + 1];
  }
  if (t < m) a0 = a0 + u[(long long)t * P.n] * q[t];
  Z[P.offZ + (long long)c * P.n + r] = a0 + a1;
}

// R_p = -sum_i A_i Z_p[:, i]: one wavefront per row, four rows per group
__global__ __launch_bounds__(256) void k_nlb_splitmv(const NlbProb* __restrict__ pb, const int* __restrict__ dm,
                                                     const c128* __restrict__ Z, c128* __restrict__ R) {
  const int p = blockIdx.y;
  const NlbProb& P = pb[p];
  const int lane = threadIdx.x & 63, r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (dm[p] < 0 || r >= P.n) return;
  const int n = P.n;
  c128 acc = {0.0, 0.0};
  for (int i = 0; i < P.ell; ++i) {
    const c128* z = Z + P.offZ + (long long)i * n;
    if (P.t.isdiag[i]) {
      if (lane == 0) acc = acc + P.t.diag[i][r] * z[r];
    } else if (P.t.cplx[i]) {
      const c128* a = reinterpret_cast<const c128*>(P.t.A[i]) + (long long)r * n;
      for (int c = lane; c < n; c += 64) acc = acc + a[c] * z[c];
    } else {
      const double* a = reinterpret_cast<const double*>(P.t.A[i]) + (long long)r * n;
      for (int c = lane; c < n; c += 64) {
        const double v = a[c];
        const c128 zc = z[c];
        acc.re += v * zc.re;
        acc.im += v * zc.im;
      }
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) R[P.offY + r] = -acc;
}

// h_p[t] = U_p[:, t]^H y_p, t < m_p: one group per (column, problem)
__global__ __launch_bounds__(256) void k_nlb_dots(const NlbProb* __restrict__ pb, const int* __restrict__ dm,
                                                  const c128* __restrict__ U, c128* const* __restrict__ yp,
                                                  c128* __restrict__ h, long long hstride) {
  __shared__ c128 red[4];
  const int p = blockIdx.y, t = blockIdx.x;
  const NlbProb& P = pb[p];
  if (t >= dm[p]) return;  // group-uniform (dm < 0: done)
  const c128* u = U + P.offU + (long long)t * P.n;
  const c128* y = yp[p];
  c128 acc = {0.0, 0.0};
  for (int r = threadIdx.x; r < P.n; r += 256) acc = acc + conj(u[r]) * y[r];
  const c128 sum = group_sum(acc, red);
  if (threadIdx.x == 0) h[p * hstride + t] = sum;
}

// y_p -= U_p[:, 0:m_p] h_p
__global__ __launch_bounds__(64) void k_nlb_sub(const NlbProb* __restrict__ pb, const int* __restrict__ dm,
                                                const c128* __restrict__ U, const c128* __restrict__ h,
                                                long long hstride, c128* const* __restrict__ yp) {
  const int p = blockIdx.y, r = blockIdx.x * 64 + threadIdx.x;
  const NlbProb& P = pb[p];
  const int m = dm[p];
  if (m <= 0 || r >= P.n) return;
  const c128* u = U + P.offU + r;
  const c128* q = h + p * hstride;
  c128 a0 = {0.0, 0.0}, a1 = {0.0, 0.0};
  int t = 0;
  for (; t + 1 < m; t += 2) {
    a0 = a0 + u[(long long)t * P.n] * q[t];
    a1 = a1 + u[(long long)(t + 1) * P.n] * q[t + 1];
  }
  if (t < m) a0 = a0 + u[(long long)t * P.n] * q[t];
  c128* y = yp[p] + r;
  *y = *y - (a0 + a1);
}

// nrm[p * nstride + slot] = ||y_p||_2: one group per problem
__global__ __launch_bounds__(256) void k_nlb_norm(const NlbProb* __restrict__ pb, const int* __restrict__ dm,
                                                  c128* const* __restrict__ yp, double* __restrict__ nrm,
                                                  long long nstride, int slot) {
  __shared__ c128 red[4];
  const int p = blockIdx.x;
  const NlbProb& P = pb[p];
  if (dm[p] < 0) return;
  const c128* y = yp[p];
  double acc = 0.0;
  for (int r = threadIdx.x; r < P.n; r += 256) acc += norm2(y[r]);
  const c128 sum = group_sum(c128{acc, 0.0}, red);
  if (threadIdx.x == 0) nrm[p * nstride + slot] = sqrt(sum.re);
}

// U_p[:, m_p] = y_p / nrm (y_p may be that column)
__global__ __launch_bounds__(256) void k_nlb_store(const NlbProb* __restrict__ pb, const int* __restrict__ dm,
                                                   c128* U, c128* const* __restrict__ yp, const double* __restrict__ nrm,
                                                   long long nstride) {
  const int p = blockIdx.y, r = blockIdx.x * 256 + threadIdx.x;
  const NlbProb& P = pb[p];
  const int m = dm[p];
  if (m < 0 || r >= P.n) return;
  const double v = nrm[p * nstride + 1];
  const double sc = v > 0.0 ? 1.0 / v : 0.0;
  U[P.offU + (long long)m * P.n + r] = sc * yp[p][r];
}

// One Ritz pair of a batched run: its problem, eigenvalue, the offset of its
// coefficients on U_p and of its vector in the work buffer.
struct NlbPair {
  int p, m;
  c128 lam;
  long long soff, xoff;
};

// X[:, a] = U_p S_a, scaled to 2-norm 1 with its largest-modulus entry (lowest
// index among equals) real and positive; one group per pair
__global__ __launch_bounds__(256) void k_nlb_vectors(const NlbProb* __restrict__ pb, const NlbPair* __restrict__ pr,
                                                     const c128* __restrict__ U, const c128* __restrict__ S,
                                                     c128* __restrict__ X) {
  const NlbPair a = pr[blockIdx.x];
  nl_vector(pb[a.p].n, a.m, U + pb[a.p].offU, S + a.soff, X + a.xoff);
}

// Backward error of eq. (sressplit) for one pair per group: the row maxima of
// |T(lambda) x| and |x| and sum_i |f_i(lambda)| ||A_i||_inf (f_i on the
// device, NaN if lambda lies on a pole or cut)
__global__ __launch_bounds__(256) void k_nlb_eta(const NlbProb* __restrict__ pb, const NlbPair* __restrict__ pr,
                                                 const c128* __restrict__ X, double* __restrict__ eta) {
  __shared__ double red[4];
  __shared__ double xr_[4];
  const NlbPair a = pr[blockIdx.x];
  const NlbProb& P = pb[a.p];
  const int n = P.n, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  c128 f[kMaxTerms];
  int bad = 0;
  double den = 0.0;
  for (int i = 0; i < P.ell; ++i) {
    f[i] = fn_eval(P.fn_nodes, P.fn_coef, P.fn_root[i], a.lam, bad);
    den += sqrt(norm2(f[i])) * P.normA[i];
  }
  const c128* x = X + a.xoff;
  double rmax = 0.0, xmax = 0.0;
  for (int r = w; r < n; r += 4) {
    c128 acc = {0.0, 0.0};
    for (int i = 0; i < P.ell; ++i) {
      c128 ai = {0.0, 0.0};
      if (P.t.isdiag[i]) {
        if (lane == 0) ai = P.t.diag[i][r] * x[r];
      } else if (P.t.cplx[i]) {
        const c128* A = reinterpret_cast<const c128*>(P.t.A[i]) + (long long)r * n;
        for (int c = lane; c < n; c += 64) ai = ai + A[c] * x[c];
      } else {
        const double* A = reinterpret_cast<const double*>(P.t.A[i]) + (long long)r * n;
        for (int c = lane; c < n; c += 64) {
          const double v = A[c];
          ai.re += v * x[c].re;
          ai.im += v * x[c].im;
        }
      }
      acc = acc + f[i] * ai;
    }
    acc = wave_sum(acc);
    rmax = nanmax(rmax, sqrt(norm2(acc)));
    if (lane == 0) xmax = nanmax(xmax, sqrt(norm2(x[r])));
  }
  if (lane == 0) {
    red[w] = rmax;
    xr_[w] = xmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double rm = 0.0, xm = 0.0;
    for (int i = 0; i < 4; ++i) {
      rm = nanmax(rm, red[i]);
      xm = nanmax(xm, xr_[i]);
    }
    const double dd = den * xm;
    eta[blockIdx.x] = (bad || !(dd > 0.0)) ? NAN : rm / dd;
  }
}

// f_i(z_pj) for every problem p and node j < stride, one thread each:
// out[(p * kMaxTerms + i) * stride + j], bad[p * stride + j]
__global__ __launch_bounds__(64) void k_nlb_fn(const NlbProb* __restrict__ pb, int nprob, int stride,
                                               const c128* __restrict__ z, c128* __restrict__ out,
                                               int* __restrict__ bad) {
  const int e = blockIdx.x * 64 + threadIdx.x;
  const int p = e / stride, j = e - p * stride;
  if (p >= nprob) return;
  const NlbProb& P = pb[p];
  int b = 0;
  for (int i = 0; i < P.ell; ++i)
    out[((long long)p * kMaxTerms + i) * stride + j] = fn_eval(P.fn_nodes, P.fn_coef, P.fn_root[i], z[e], b);
  bad[e] = b;
}

// Y_dst[a] = X[:, a] for the kept pairs: one group per pair
__global__ __launch_bounds__(256) void k_nlb_gather(const NlbPair* __restrict__ pr, const int* __restrict__ keep,
                                                    c128* const* __restrict__ dst, const c128* __restrict__ X,
                                                    const NlbProb* __restrict__ pb) {
  const NlbPair a = pr[keep[blockIdx.x]];
  const int n = pb[a.p].n;
  c128* out = dst[blockIdx.x];
  for (int r = threadIdx.x; r < n; r += 256) out[r] = X[a.xoff + r];
}

// ---------------------------------------------------------------------------
// Host set-up: Leja--Bagby points, basis scaling, divided differences
// ---------------------------------------------------------------------------

using zc = std::complex<double>;

struct Interp {
  int d = 0, met = 0;
  std::vector<zc> sigma, xi;   // d + 1 each (xi[0] unused, infinite)
  std::vector<double> beta;    // d + 1
  std::vector<zc> dd;          // ell x (d + 1): dd[i * (d + 1) + j] = d_i^j
};

bool inf_pole(zc x) { return std::isinf(x.real()) || std::isinf(x.imag()); }
zc pole_factor(zc z, zc xi) { return inf_pole(xi) ? zc(1.0, 0.0) : zc(1.0, 0.0) - z / xi; }

int argmax_tie(const std::vector<double>& a) {
  const double m = *std::max_element(a.begin(), a.end());
  for (size_t k = 0; k < a.size(); ++k)
    if (a[k] >= m * (1.0 - kNlTie)) return (int)k;
  return 0;
}

// -1 when every value is infinite
int argmin_tie(const std::vector<double>& a) {
  double m = INFINITY;
  for (double v : a) m = std::min(m, v);
  if (!std::isfinite(m)) return -1;
  for (size_t k = 0; k < a.size(); ++k)
    if (a[k] <= m * (1.0 + kNlTie)) return (int)k;
  return -1;
}

double mag(zc x) {
  const double a = std::abs(x);
  return std::isnan(a) ? INFINITY : a;
}

// The interpolant in two phases around the evaluation of the f_i at the
// nodes (done on the device, for one problem or for a batch at once).
struct InterpWork {
  int npts = 0, dmax = 0;
  double tol = 0.0;
  std::vector<zc> zb, sig, xi;
  std::vector<int> idx;
};

// Leja--Bagby nodes and poles (host)
void interp_nodes(const nep_contour& g, const nep_nleigs_opts& o, InterpWork& w) {
  const int npts = o.npts > 0 ? o.npts : 1024;
  const int dmax = o.dmax > 0 ? o.dmax : 50;
  w.npts = npts;
  w.dmax = dmax;
  w.tol = o.tol > 0.0 ? o.tol : 1e-12;
  // boundary of the region
  const double v = g.kind == 1 ? g.v : 1.0;
  std::vector<zc> zb(npts);
  for (int k = 0; k < npts; ++k) {
    const double t = 2.0 * M_PI * k / npts;
    zb[k] = zc(g.c[0] + g.rho * std::cos(t), g.c[1] + g.rho * v * std::sin(t));
  }
  std::vector<zc> xs(o.nxi);
  for (int k = 0; k < o.nxi; ++k) xs[k] = zc(o.xi[2 * k], o.xi[2 * k + 1]);
  // Leja--Bagby: s_j kept on the candidates, rescaled every step (the
  // selections only compare values)
  std::vector<int> idx{0};
  std::vector<zc> sig{zb[0]}, xi{zc(INFINITY, 0.0)};
  std::vector<zc> sb(npts), sx(xs.size());
  for (int k = 0; k < npts; ++k) sb[k] = zb[k] - sig[0];
  for (size_t k = 0; k < xs.size(); ++k) sx[k] = xs[k] - sig[0];
  std::vector<double> a(npts), ax(xs.size());
  std::vector<char> used(xs.size(), 0);  // |s_j| is infinite at a pole
  for (int j = 0; j < dmax; ++j) {
    double sc = 0.0;
    for (int k = 0; k < npts; ++k) sc = std::max(sc, std::abs(sb[k]));
    for (int k = 0; k < npts; ++k) {
      sb[k] /= sc;
      a[k] = std::abs(sb[k]);
    }
    for (size_t k = 0; k < xs.size(); ++k) {
      sx[k] /= sc;
      ax[k] = used[k] ? INFINITY : mag(sx[k]);
    }
    const int kb = argmax_tie(a);
    idx.push_back(kb);
    sig.push_back(zb[kb]);
    const int kx = xs.empty() ? -1 : argmin_tie(ax);
    const zc xn = kx >= 0 ? xs[kx] : zc(INFINITY, 0.0);
    if (kx >= 0)
      for (size_t k = 0; k < xs.size(); ++k) used[k] |= xs[k] == xn;
    xi.push_back(xn);
    for (int k = 0; k < npts; ++k) sb[k] = sb[k] * (zb[k] - sig.back()) / pole_factor(zb[k], xn);
    for (size_t k = 0; k < xs.size(); ++k)
      if (!used[k]) sx[k] = sx[k] * (xs[k] - sig.back()) / pole_factor(xs[k], xn);
  }
  w.zb = std::move(zb);
  w.sig = std::move(sig);
  w.xi = std::move(xi);
  w.idx = std::move(idx);
}

// basis scaling, divided differences from f_i at the nodes (fv: ell x
// (dmax+1), fv[i * (dmax+1) + j] = f_i(sigma_j)), degree, last pole at infinity
nep_status interp_finish(const InterpWork& w, int ell, const c128* fv, const int* bad, Interp& it) {
  const int npts = w.npts, dmax = w.dmax;
  const double tol = w.tol;
  const std::vector<zc>& zb = w.zb;
  const std::vector<zc>& sig = w.sig;
  const std::vector<zc>& xi = w.xi;
  const std::vector<int>& idx = w.idx;
  for (int j = 0; j <= dmax; ++j)
    NEP_CHECK(!bad[j], NEP_ERR_NOT_HOLOMORPHIC, "interpolation node %d lies on a pole or branch cut", j);
  auto f = [&](int i, int j) { return zc(fv[(size_t)i * (dmax + 1) + j].re, fv[(size_t)i * (dmax + 1) + j].im); };
  // b_j on the boundary points, beta_j scaling max |b_j| to 1
  std::vector<zc> bb((size_t)(dmax + 1) * npts);
  std::vector<double> beta(dmax + 1, 1.0);
  for (int k = 0; k < npts; ++k) bb[k] = zc(1.0, 0.0);
  std::vector<zc> t(npts);
  for (int j = 1; j <= dmax; ++j) {
    double mx = 0.0;
    for (int k = 0; k < npts; ++k) {
      t[k] = bb[(size_t)(j - 1) * npts + k] * (zb[k] - sig[j - 1]) / pole_factor(zb[k], xi[j]);
      mx = std::max(mx, std::abs(t[k]));
    }
    beta[j] = mx;
    for (int k = 0; k < npts; ++k) bb[(size_t)j * npts + k] = t[k] / mx;
  }
  auto B = [&](int j, int k) { return bb[(size_t)j * npts + k]; };
  // divided differences by the interpolation conditions
  std::vector<zc> dd((size_t)ell * (dmax + 1));
  for (int i = 0; i < ell; ++i)
    for (int j = 0; j <= dmax; ++j) {
      zc acc = f(i, j);
      for (int q = 0; q < j; ++q) acc -= B(q, idx[j]) * dd[(size_t)i * (dmax + 1) + q];
      dd[(size_t)i * (dmax + 1) + j] = acc / B(j, idx[j]);
    }
  std::vector<double> delta(dmax + 1, 0.0);
  for (int j = 0; j <= dmax; ++j)
    for (int i = 0; i < ell; ++i) delta[j] = std::max(delta[j], std::abs(dd[(size_t)i * (dmax + 1) + j]));
  int d = dmax, met = 0;
  for (int j = 2; j <= dmax; ++j)
    if (delta[j] / delta[0] < tol) {
      d = j;
      met = 1;
      break;
    }
  // last pole at infinity
  double mx = 0.0;
  for (int k = 0; k < npts; ++k) {
    t[k] = B(d - 1, k) * (zb[k] - sig[d - 1]);
    mx = std::max(mx, std::abs(t[k]));
  }
  beta[d] = mx;
  const zc bd = t[idx[d]] / mx;
  it.d = d;
  it.met = met;
  it.sigma.assign(sig.begin(), sig.begin() + d + 1);
  it.xi.assign(xi.begin(), xi.begin() + d + 1);
  it.xi[d] = zc(INFINITY, 0.0);
  it.beta.assign(beta.begin(), beta.begin() + d + 1);
  it.dd.assign((size_t)ell * (d + 1), zc());
  for (int i = 0; i < ell; ++i) {
    for (int j = 0; j < d; ++j) it.dd[(size_t)i * (d + 1) + j] = dd[(size_t)i * (dmax + 1) + j];
    zc acc = f(i, d);
    for (int q = 0; q < d; ++q) acc -= B(q, idx[d]) * dd[(size_t)i * (dmax + 1) + q];
    it.dd[(size_t)i * (d + 1) + d] = acc / bd;
  }
  return NEP_OK;
}

nep_status interp_build(Split& s, const nep_contour& g, const nep_nleigs_opts& o, Interp& it) {
  InterpWork w;
  interp_nodes(g, o, w);
  std::vector<c128> zn(w.dmax + 1), fv;
  std::vector<int> bad;
  for (int j = 0; j <= w.dmax; ++j) zn[j] = c128{w.sig[j].real(), w.sig[j].imag()};
  NEP_TRY(s.eval_fns(w.dmax + 1, zn.data(), fv, bad, false));
  return interp_finish(w, s.op.ell, fv.data(), bad.data(), it);
}

// b_0(z)..b_d(z) of the interpolant
std::vector<zc> basis_at(const Interp& it, zc z) {
  std::vector<zc> b(it.d + 1);
  b[0] = zc(1.0, 0.0);
  for (int j = 1; j <= it.d; ++j) b[j] = b[j - 1] * (z - it.sigma[j - 1]) / (it.beta[j] * pole_factor(z, it.xi[j]));
  return b;
}

// complex product without the library's inf/nan recovery (the operands
// here are finite)
inline zc cmul(zc a, zc b) {
  return zc(a.real() * b.real() - a.imag() * b.imag(), a.real() * b.imag() + a.imag() * b.real());
}

// sum over d blocks (stride ld, first len entries) of conj(a) b, and
// v -= h g over the same entries: plain real arithmetic (these loops run
// on the host once per Arnoldi step over (k + d) d entries per vector)
zc dot_blocks(const zc* a, const zc* b, int d, int ld, int len) {
  double sr = 0.0, si = 0.0;
  for (int i = 0; i < d; ++i) {
    const double* x = reinterpret_cast<const double*>(a + (size_t)i * ld);
    const double* y = reinterpret_cast<const double*>(b + (size_t)i * ld);
    for (int t = 0; t < 2 * len; t += 2) {
      sr += x[t] * y[t] + x[t + 1] * y[t + 1];
      si += x[t] * y[t + 1] - x[t + 1] * y[t];
    }
  }
  return zc(sr, si);
}

void axpy_blocks(zc* v, const zc* g, zc h, int d, int ld, int len) {
  const double hr = h.real(), hi = h.imag();
  for (int i = 0; i < d; ++i) {
    double* x = reinterpret_cast<double*>(v + (size_t)i * ld);
    const double* y = reinterpret_cast<const double*>(g + (size_t)i * ld);
    for (int t = 0; t < 2 * len; t += 2) {
      x[t] -= y[t] * hr - y[t + 1] * hi;
      x[t + 1] -= y[t] * hi + y[t + 1] * hr;
    }
  }
}

// fn(p) for p < count on a few host threads (the per-problem coefficient work
// of a batched run)
template <typename F>
void parallel_for(int count, F&& fn) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int nt = std::min<int>({16, (int)hw, (count + 7) / 8});
  if (nt <= 1) {
    for (int p = 0; p < count; ++p) fn(p);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(nt);
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      for (int p = t; p < count; p += nt) fn(p);
    });
  for (auto& x : th) x.join();
}

// A few host threads kept for the length of a batched run: run(count, fn)
// calls fn(p) for every p < count across them and the calling thread (the
// per-problem coefficient work of each Arnoldi step, without starting threads
// every step).
class HostPool {
 public:
  explicit HostPool(int nworkers) {
    for (int t = 0; t < nworkers; ++t)
      th_.emplace_back([this] {
        unsigned seen = 0;
        for (;;) {
          {
            std::unique_lock<std::mutex> lk(mu_);
            cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
            if (stop_) return;
            seen = gen_;
          }
          drain();
          std::lock_guard<std::mutex> lk(mu_);
          if (--busy_ == 0) done_.notify_all();
        }
      });
  }
  HostPool(const HostPool&) = delete;
  HostPool& operator=(const HostPool&) = delete;
  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  void run(int count, std::function<void(int)> fn) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = std::move(fn);
      count_ = count;
      next_ = 0;
      busy_ = (int)th_.size();
      ++gen_;
    }
    cv_.notify_all();
    drain();
    std::unique_lock<std::mutex> lk(mu_);
    done_.wait(lk, [&] { return busy_ == 0; });
  }

 private:
  void drain() {
    for (int p; (p = next_.fetch_add(1)) < count_;) job_(p);
  }
  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable cv_, done_;
  std::function<void(int)> job_;
  int count_ = 0, busy_ = 0;
  std::atomic<int> next_{0};
  unsigned gen_ = 0;
  bool stop_ = false;
};

// Host side of Arnoldi in the TOAR representation for one problem: the
// coefficient recurrences of eqs. (nleigs-toar1), (nleigs-toar4), the
// coefficients of the right-hand side of eq. (nleigs-toar2) per term, and the
// Gram--Schmidt of the coefficient vectors (Algorithm "Arnoldi for NLEIGS with
// TOAR representation").  G holds g_1, g_2, ...: d blocks of mmax entries
// (the first m meaningful), H the (k+1) x k Hessenberg matrix.
struct ToarHost {
  int d = 0, k = 0, ell = 0, mmax = 0, m = 0, kd = 0;
  double hlast = 0.0;
  bool done = false;  // breakdown (invariant subspace) or k steps
  zc sg;
  std::vector<zc> bs, xr, rds, bom, ddl, dd;
  std::vector<std::vector<zc>> G, gt;
  std::vector<zc> H;

  void init(const Interp& it, zc sigma, int nterms, int ksteps) {
    d = it.d;
    k = ksteps;
    ell = nterms;
    mmax = d + k;
    sg = sigma;
    bs = basis_at(it, sg);
    dd = it.dd;
    xr.assign(d + 1, zc());
    rds.assign(d, zc());
    bom.assign(d, zc());
    ddl.assign(ell, zc());
    for (int j = 1; j <= d; ++j) {
      const zc om = inf_pole(it.xi[j]) ? zc(1.0, 0.0) : zc(1.0, 0.0) - sg / it.xi[j];
      xr[j] = inf_pole(it.xi[j]) ? zc() : it.beta[j] / it.xi[j];
      if (j < d) {
        rds[j] = 1.0 / (it.sigma[j - 1] - sg);
        bom[j] = it.beta[j] * om;
      }
    }
    for (int i = 0; i < ell; ++i) ddl[i] = dd[(size_t)i * (d + 1) + d] / it.beta[d];
    gt.assign(d, std::vector<zc>(mmax));
    H.assign((size_t)(k + 1) * k, zc());
    G.clear();
  }
  // coefficients rho_i of R_d(sigma) = sum_i rho_i A_i
  void rho(c128* out) const {
    for (int i = 0; i < ell; ++i) {
      zc acc;
      for (int j = 0; j <= d; ++j) acc += bs[j] * dd[(size_t)i * (d + 1) + j];
      out[i] = c128{acc.real(), acc.imag()};
    }
  }
  // g_1 = vec(R) / ||vec(R)|| from the Gram--Schmidt QR of the starting
  // block: R[q * d + t] = coefficient of w^q on basis vector t
  void start(const std::vector<zc>& R) {
    G.assign(1, std::vector<zc>((size_t)d * mmax, zc()));
    double fro = 0.0;
    for (const zc& v : R) fro += std::norm(v);
    fro = std::sqrt(fro);
    for (int q = 0; q < d; ++q)
      for (int t = 0; t < d; ++t) G[0][(size_t)q * mmax + t] = R[(size_t)q * d + t] / fro;
    m = d;
  }
  // step j: Q (m x ell, column-major) such that the right-hand side of eq.
  // (nleigs-toar2) is -sum_i A_i U q_i
  void rhs(int j, c128* Q) {
    const std::vector<zc>& gj = G[j];
    auto gb = [&](int i, int t) { return gj[(size_t)i * mmax + t]; };
    for (int t = 0; t < m; ++t)
      gt[d - 1][t] = cmul(gb(d - 2, t) + cmul(xr[d - 1], gb(d - 1, t)), rds[d - 1]);
    for (int i = d - 2; i >= 1; --i)
      for (int t = 0; t < m; ++t)
        gt[i][t] = cmul(gb(i - 1, t) + cmul(xr[i], gb(i, t)) - cmul(bom[i], gt[i + 1][t]), rds[i]);
    for (int i = 0; i < ell; ++i)
      for (int t = 0; t < m; ++t) {
        zc acc = cmul(ddl[i], gb(d - 1, t));
        for (int q = 0; q + 1 < d; ++q) acc += cmul(dd[(size_t)i * (d + 1) + q], gt[q + 1][t]);
        Q[(size_t)i * m + t] = c128{acc.real(), acc.imag()};
      }
  }
  // step j: y^0 = U c + n1 u (u the new basis vector unless y^0 was
  // dependent); forms g (eq. (nleigs-toar4)), orthogonalizes it against
  // g_1..g_{j+1} and appends g_{j+2} and column j of H
  void absorb(int j, const std::vector<zc>& c, double n0, double n1) {
    const bool grow_u = n1 > kNlDep * n0;
    const int mn = m + (grow_u ? 1 : 0);
    std::vector<zc> g0v(mn, zc());
    for (int t = 0; t < m; ++t) g0v[t] = c[t];
    if (grow_u) g0v[m] = n1;
    std::vector<zc> v((size_t)d * mmax, zc());
    for (int i = 0; i + 1 < d; ++i)
      for (int t = 0; t < mn; ++t) v[(size_t)i * mmax + t] = (t < m ? gt[i + 1][t] : zc()) + cmul(bs[i], g0v[t]);
    for (int t = 0; t < mn; ++t) v[(size_t)(d - 1) * mmax + t] = cmul(bs[d - 1], g0v[t]);
    std::vector<zc> hh(j + 1, zc());
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<zc> hp(j + 1, zc());
      for (int q = 0; q <= j; ++q) hp[q] = dot_blocks(G[q].data(), v.data(), d, mmax, mn);
      for (int q = 0; q <= j; ++q) {
        axpy_blocks(v.data(), G[q].data(), hp[q], d, mmax, mn);
        hh[q] += hp[q];
      }
    }
    const double nv = std::sqrt(dot_blocks(v.data(), v.data(), d, mmax, mn).real());
    for (int q = 0; q <= j; ++q) H[(size_t)j * (k + 1) + q] = hh[q];
    H[(size_t)j * (k + 1) + j + 1] = nv;
    m = mn;
    kd = j + 1;
    hlast = nv;
    if (!(nv > 0.0) || kd == k) {  // invariant subspace, or the last step
      done = true;
      if (!(nv > 0.0)) return;
    }
    for (zc& e : v) e /= nv;
    G.push_back(std::move(v));
  }
  // Ritz values lambda = sigma + 1/theta of H_kd; S: the eigenvectors
  // (kd x kd, column-major)
  bool ritz(std::vector<zc>& lam, std::vector<zc>& S) const {
    std::vector<zc> Hk((size_t)kd * kd), th;
    for (int q = 0; q < kd; ++q)
      for (int r = 0; r < kd; ++r) Hk[(size_t)q * kd + r] = H[(size_t)q * (k + 1) + r];
    if (!eig_general(kd, Hk, th, S)) return false;
    lam.assign(kd, zc(INFINITY, 0.0));
    for (int q = 0; q < kd; ++q)
      if (th[q] != zc(0.0, 0.0)) lam[q] = sg + 1.0 / th[q];
    return true;
  }
  // coefficients of the first block of Ritz vector q on U: G^0 s / ||s||
  void ritz_coeffs(const std::vector<zc>& S, int q, c128* out) const {
    double sn = 0.0;
    for (int r = 0; r < kd; ++r) sn += std::norm(S[(size_t)q * kd + r]);
    sn = std::sqrt(sn);
    for (int t = 0; t < m; ++t) {
      zc acc;
      for (int r = 0; r < kd; ++r) acc += cmul(G[r][t], S[(size_t)q * kd + r]);
      acc /= sn;
      out[t] = c128{acc.real(), acc.imag()};
    }
  }
};

// inside the region g (circle or ellipse)
bool inside_region(const nep_contour& g, zc z) {
  const double v = g.kind == 1 ? g.v : 1.0;
  const zc mu = (z - zc(g.c[0], g.c[1])) / g.rho;
  const double r2 = mu.real() * mu.real() + (mu.imag() / v) * (mu.imag() / v);
  return std::isfinite(r2) && r2 < 1.0;
}

nep_status check_nleigs_opts(const nep_nleigs_opts* o) {
  NEP_CHECK(o != nullptr, NEP_ERR_ARG, "null options");
  NEP_CHECK(o->dmax == 0 || (o->dmax >= 2 && o->dmax <= kNlMaxDeg), NEP_ERR_ARG, "need 2 <= dmax <= %d", kNlMaxDeg);
  NEP_CHECK(o->npts == 0 || (o->npts >= 8 && o->npts <= kNlMaxPts), NEP_ERR_ARG, "need 8 <= npts <= %d", kNlMaxPts);
  NEP_CHECK(o->tol >= 0.0 && o->tol < 1.0, NEP_ERR_ARG, "need 0 <= tol < 1");
  NEP_CHECK(o->nxi >= 0 && o->nxi <= 65536 && (o->nxi == 0 || o->xi != nullptr), NEP_ERR_ARG,
            "bad singularity set");
  return NEP_OK;
}

}  // namespace

}  // namespace nep

using namespace nep;

extern "C" {

nep_status nep_nleigs_interp(nep_split h, const nep_contour* g, const nep_nleigs_opts* o, int* d, int* met,
                             double* sigma, double* xi, double* beta, double* dd) {
  NEP_CHECK(h != nullptr, NEP_ERR_ARG, "null handle");
  NEP_TRY(check_contour(g));
  NEP_TRY(check_nleigs_opts(o));
  NEP_CHECK(d && met && sigma && xi && beta && dd, NEP_ERR_ARG, "null output");
  Split& s = h->impl;
  Interp it;
  NEP_TRY(interp_build(s, *g, *o, it));
  const int dmax = o->dmax > 0 ? o->dmax : 50;
  *d = it.d;
  *met = it.met;
  for (int j = 0; j <= dmax; ++j) {
    const bool in = j <= it.d;
    sigma[2 * j] = in ? it.sigma[j].real() : 0.0;
    sigma[2 * j + 1] = in ? it.sigma[j].imag() : 0.0;
    xi[2 * j] = in ? it.xi[j].real() : 0.0;
    xi[2 * j + 1] = in ? it.xi[j].imag() : 0.0;
    beta[j] = in ? it.beta[j] : 0.0;
    for (int i = 0; i < s.op.ell; ++i) {
      const zc v = in ? it.dd[(size_t)i * (it.d + 1) + j] : zc();
      dd[2 * ((size_t)i * (dmax + 1) + j)] = v.real();
      dd[2 * ((size_t)i * (dmax + 1) + j) + 1] = v.imag();
    }
  }
  return NEP_OK;
}

nep_status nep_nleigs(nep_split h, const nep_contour* g, const nep_nleigs_opts* o, const void* W0, int* m_out,
                      double* lambda, void* X, double* eta, double* Hout, nep_nleigs_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  NEP_CHECK(h != nullptr, NEP_ERR_ARG, "null handle");
  NEP_TRY(check_contour(g));
  NEP_TRY(check_nleigs_opts(o));
  NEP_CHECK(o->k >= 1 && o->k <= kNlMaxK, NEP_ERR_ARG, "need 1 <= k <= %d", kNlMaxK);
  NEP_CHECK(o->max_eigs >= 1, NEP_ERR_ARG, "need max_eigs >= 1");
  NEP_CHECK(o->eta_tol >= 0.0, NEP_ERR_ARG, "need eta_tol >= 0");
  NEP_CHECK(W0 && m_out && lambda && X && eta, NEP_ERR_ARG, "null argument");
  Split& s = h->impl;
  const int n = s.op.n, ell = s.op.ell, k = o->k;
  const hipStream_t st = s.stream;
  const zc sg(o->sigma[0], o->sigma[1]);
  const double eta_tol = o->eta_tol > 0.0 ? o->eta_tol : 1e-10;

  Interp it;
  NEP_TRY(interp_build(s, *g, *o, it));
  const int d = it.d;
  for (int j = 0; j < d; ++j)
    NEP_CHECK(it.sigma[j] != sg, NEP_ERR_ARG, "the shift equals interpolation node %d", j);
  for (int j = 1; j <= d; ++j)
    NEP_CHECK(inf_pole(it.xi[j]) || it.xi[j] != sg, NEP_ERR_ARG, "the shift equals pole %d", j);
  ToarHost tz;
  tz.init(it, sg, ell, k);
  std::vector<c128> rho(ell);
  tz.rho(rho.data());

  // device buffers
  const int mmax = d + k;  // basis columns at most
  DevMem dU, dZ, dQ, dsc, dsig, drho;
  NEP_TRY(dU.alloc(sizeof(c128) * (size_t)n * (mmax + 1)));
  NEP_TRY(dZ.alloc(sizeof(c128) * (size_t)n * std::max(ell, 1)));
  NEP_TRY(dQ.alloc(sizeof(c128) * (size_t)(mmax + 1) * std::max(ell, k)));
  NEP_TRY(dsc.alloc(sizeof(c128) * (size_t)(2 * (mmax + 1) + 2)));
  NEP_HIP(hipMemsetAsync(dsc.p, 0, dsc.bytes, st));
  NEP_TRY(dsig.alloc(sizeof(c128)));
  NEP_TRY(drho.alloc(sizeof(c128) * ell));
  c128* U = dU.as<c128>();
  c128* h1 = dsc.as<c128>();
  c128* h2 = h1 + (mmax + 1);
  double* nrm = reinterpret_cast<double*>(h2 + (mmax + 1));  // [0]: before, [1]: after Gram--Schmidt
  const c128 csg{sg.real(), sg.imag()};
  NEP_HIP(hipMemcpyAsync(dsig.p, &csg, sizeof(c128), hipMemcpyHostToDevice, st));
  NEP_HIP(hipMemcpyAsync(drho.p, rho.data(), sizeof(c128) * ell, hipMemcpyHostToDevice, st));

  NlTerms terms{};
  for (int i = 0; i < ell; ++i) {
    terms.A[i] = s.op.dA[i];
    terms.diag[i] = s.op.dDiag[i];
    terms.cplx[i] = s.op.is_cplx[i];
    terms.isdiag[i] = s.op.is_diag[i];
  }

  // R_d(sigma) = sum_i rho_i A_i: assembly and LU in complex FP64
  MomentsPlan plan;
  nep_contour g0{};
  g0.kind = 0;
  g0.rho = 1.0;
  g0.v = 1.0;
  PlanOptions po;
  po.N = 1;
  po.L = 1;
  po.K = 1;
  po.prec = NEP_PREC_FP64;
  po.max_refine = 0;
  po.fallback = 0;
  PlanProblem pp{&s.op, g0, nullptr, nullptr, dsig.as<c128>()};
  pp.fpts = drho.as<c128>();
  std::vector<PlanProblem> probs{pp};
  NEP_TRY(plan.build(probs, po, st));
  {
    // one matrix: its panels run alone, with nothing to overlap them, and a
    // 64-wide panel does half the serial work of a 128-wide one (n = 4096:
    // 80 ms against 112 ms for the factorization)
    MomentsPlan::Knobs kn = plan.knobs();
    if (kn.jb != 64) {
      kn.jb = 64;
      NEP_TRY(plan.apply(kn, st));
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  NEP_HIP(hipEventCreate(&e0));
  NEP_HIP(hipEventCreate(&e1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } evg{e0, e1};
  NEP_HIP(hipEventRecord(e0, st));
  NEP_TRY(plan.factor(st));
  NEP_HIP(hipEventRecord(e1, st));
  int pinfo = 0;
  NEP_HIP(hipMemcpyAsync(&pinfo, plan.info(), sizeof(int), hipMemcpyDeviceToHost, st));
  NEP_HIP(hipStreamSynchronize(st));
  NEP_CHECK(pinfo >= n, NEP_ERR_SINGULAR, "R_d(sigma) is exactly singular (zero pivot at step %d)", pinfo);
  float ms_lu = 0.0f;
  NEP_HIP(hipEventElapsedTime(&ms_lu, e0, e1));
  const auto t1 = std::chrono::steady_clock::now();
  c128* Rv = plan.R_mut();
  c128* Yv = plan.Y_mut();
  const dim3 grow(ceil_div(n, 256)), g256(256);
  // y = R_d(sigma)^{-1} rhs with the resident factors: forward then backward,
  // n/64 groups each (flags and tickets zeroed once; each solve has its epoch)
  const MatDesc md0 = plan.mat0();
  NEP_CHECK(md0.n == n, NEP_ERR_DEVICE, "factor plan holds a matrix of size %d, expected %d", md0.n, n);
  const int nblk = ceil_div(n, kNlBlk);
  DevMem dflag;
  NEP_TRY(dflag.alloc(sizeof(int) * (2 * (size_t)nblk + 4)));
  NEP_HIP(hipMemsetAsync(dflag.p, 0, dflag.bytes, st));
  int* fl_l = dflag.as<int>();
  int* fl_u = fl_l + nblk;
  int* tick = fl_u + nblk;  // [0]: forward, [1]: backward
  // set when a solve's wait ran out; read back with every step's coefficients
  int* overrun_flag = reinterpret_cast<int*>(h1 + 2 * (mmax + 1) + 1);
  const c128* Tf = reinterpret_cast<const c128*>(plan.factor_base()) + md0.offT;
  const int* rat = plan.row_map() + md0.offRow;
  const c128* Dv = reinterpret_cast<const c128*>(plan.dinv0());
  DevMem dyf;
  NEP_TRY(dyf.alloc(sizeof(c128) * (size_t)n));
  int epoch = 0;
  // algorithmic HBM bytes of one triangle: the factor outside the diagonal
  // blocks, the diagonal-block inverses, and the right-hand side, solution
  // and row map (for event profiling)
  double tri_bytes = 0.0;
  {
    double diag = 0.0;
    for (int q = 0; q < nblk; ++q) {
      const double nr = std::min(kNlBlk, n - q * kNlBlk);
      diag += nr * nr;
    }
    tri_bytes = 16.0 * (((double)n * n - diag) / 2.0 + (double)nblk * kNlBlk * kNlBlk + 2.0 * n) + 4.0 * n;
  }
  KernelProf& prof = kernel_prof();
  auto timed = [&](int kind, double bytes, auto&& launch) {
    hipEvent_t a = nullptr, z = nullptr;
    if (prof.on) {
      (void)hipEventCreate(&a);
      (void)hipEventCreate(&z);
      (void)hipEventRecord(a, st);
    }
    launch();
    if (prof.on) {
      (void)hipEventRecord(z, st);
      prof.add(kind, a, z, bytes);
    }
  };
  auto solve = [&](const c128* rhs, c128* x) -> nep_status {
    ++epoch;
    const dim3 gp((nblk + 1) / 2), g512(512);
    timed(2, tri_bytes, [&] {
      hipLaunchKernelGGL(k_nl_tri<false>, gp, g512, 0, st, n, md0.ld, Tf, rat, Dv, rhs, dyf.as<c128>(), fl_l, tick,
                         epoch, overrun_flag);
    });
    timed(2, tri_bytes, [&] {
      hipLaunchKernelGGL(k_nl_tri<true>, gp, g512, 0, st, n, md0.ld, Tf, rat, Dv, dyf.as<c128>(), x, fl_u,
                         tick + 1, epoch, overrun_flag);
    });
    NEP_HIP(hipGetLastError());
    return NEP_OK;
  };
  // algorithmic HBM bytes of the split-form product: every A_i once (its
  // diagonal if diagonal), the ell vectors and the result
  double smv_bytes = 16.0 * n * (ell + 1);
  for (int i = 0; i < ell; ++i)
    smv_bytes += s.op.is_diag[i] ? 16.0 * n : (s.op.is_cplx[i] ? 16.0 : 8.0) * (double)n * n;

  // Gram--Schmidt of y against U[:, 0:m] with one reorthogonalization; the
  // normalized remainder goes to U[:, m].  Returns the coefficients and the
  // norms before and after.
  std::vector<c128> hb(2 * (mmax + 1) + 2);
  auto orth = [&](c128* y, int m, std::vector<zc>& coef, double& n0, double& n1) -> nep_status {
    hipLaunchKernelGGL(k_nl_norm, dim3(1), g256, 0, st, n, y, nrm);
    if (m > 0) {
      hipLaunchKernelGGL(k_nl_dots, dim3(m), g256, 0, st, n, U, y, h1);
      hipLaunchKernelGGL(k_nl_comb, dim3(ceil_div(n, 64), 1), dim3(64), 0, st, n, m, U, h1, y, 1);
      hipLaunchKernelGGL(k_nl_dots, dim3(m), g256, 0, st, n, U, y, h2);
      hipLaunchKernelGGL(k_nl_comb, dim3(ceil_div(n, 64), 1), dim3(64), 0, st, n, m, U, h2, y, 1);
    }
    hipLaunchKernelGGL(k_nl_norm, dim3(1), g256, 0, st, n, y, nrm + 1);
    hipLaunchKernelGGL(k_nl_store, grow, g256, 0, st, n, y, nrm + 1, U + (long long)m * n);
    NEP_HIP(hipGetLastError());
    NEP_HIP(hipMemcpyAsync(hb.data(), dsc.p, sizeof(c128) * hb.size(), hipMemcpyDeviceToHost, st));
    NEP_HIP(hipStreamSynchronize(st));
    coef.assign(m, zc());
    for (int t = 0; t < m; ++t)
      coef[t] = zc(hb[t].re + hb[(mmax + 1) + t].re, hb[t].im + hb[(mmax + 1) + t].im);
    const double* hn = reinterpret_cast<const double*>(hb.data() + 2 * (mmax + 1));
    n0 = hn[0];
    n1 = hn[1];
    NEP_CHECK(*reinterpret_cast<const int*>(hb.data() + 2 * (mmax + 1) + 1) == 0, NEP_ERR_DEVICE,
              "a triangular-solve group ran out of its wait bound");
    return NEP_OK;
  };

  // starting block: QR of [w^0 .. w^{d-1}] by Gram--Schmidt, g_1 = vec(R)/||vec(R)||
  NEP_HIP(hipMemcpyAsync(U, W0, sizeof(c128) * (size_t)n * d, hipMemcpyDeviceToDevice, st));
  {
    std::vector<zc> c, R((size_t)d * d, zc());
    double n0 = 0.0, n1 = 0.0;
    for (int q = 0; q < d; ++q) {
      NEP_TRY(orth(U + (long long)q * n, q, c, n0, n1));
      NEP_CHECK(n1 > kNlDep * n0 && n0 > 0.0, NEP_ERR_ARG, "starting block column %d is linearly dependent", q);
      for (int t = 0; t < q; ++t) R[(size_t)q * d + t] = c[t];
      R[(size_t)q * d + q] = n1;
    }
    tz.start(R);
  }
  std::vector<c128> Qh((size_t)(mmax + 1) * std::max(ell, 1));
  std::vector<zc> c;
  for (int j = 0; j < k && !tz.done; ++j) {
    const int m = tz.m;
    tz.rhs(j, Qh.data());
    NEP_HIP(hipMemcpyAsync(dQ.p, Qh.data(), sizeof(c128) * (size_t)m * ell, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_nl_comb, dim3(ceil_div(n, 64), ell), dim3(64), 0, st, n, m, U, dQ.as<c128>(),
                       dZ.as<c128>(), 0);
    timed(3, smv_bytes, [&] {
      hipLaunchKernelGGL(k_nl_splitmv, dim3(ceil_div(n, 4)), g256, 0, st, n, ell, terms, dZ.as<c128>(), Rv);
    });
    NEP_HIP(hipGetLastError());
    NEP_TRY(solve(Rv, Yv));  // y^0 = R_d(sigma)^{-1} rhs
    double n0 = 0.0, n1 = 0.0;
    NEP_TRY(orth(Yv, m, c, n0, n1));
    tz.absorb(j, c, n0, n1);
  }
  const float ms_krylov = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t1).count();

  // Ritz pairs: theta of H_k, lambda = sigma + 1/theta, x = U G^0 s
  std::vector<zc> lam, S;
  NEP_CHECK(tz.ritz(lam, S), NEP_ERR_DEVICE, "eigenvalues of the Hessenberg matrix did not converge");
  const int kd = tz.kd, m = tz.m;
  std::vector<int> cand;
  for (int q = 0; q < kd; ++q)
    if (inside_region(*g, lam[q])) cand.push_back(q);
  int mret = 0;
  std::vector<double> et;
  if (!cand.empty()) {
    const int nc = (int)cand.size();
    std::vector<c128> Sx((size_t)m * nc);
    for (int a = 0; a < nc; ++a) tz.ritz_coeffs(S, cand[a], Sx.data() + (size_t)a * m);
    DevMem dS, dX;
    NEP_TRY(dS.alloc(sizeof(c128) * Sx.size()));
    NEP_TRY(dX.alloc(sizeof(c128) * (size_t)n * nc));
    NEP_HIP(hipMemcpyAsync(dS.p, Sx.data(), sizeof(c128) * Sx.size(), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_nl_vectors, dim3(nc), g256, 0, st, n, m, U, dS.as<c128>(), dX.as<c128>());
    NEP_HIP(hipGetLastError());
    std::vector<double> lh(2 * nc), eh(nc);
    for (int a = 0; a < nc; ++a) {
      lh[2 * a] = lam[cand[a]].real();
      lh[2 * a + 1] = lam[cand[a]].imag();
    }
    NEP_TRY(nep_backward_error(h, nc, lh.data(), dX.p, eh.data()));
    std::vector<int> keep;
    for (int a = 0; a < nc; ++a)
      if (eh[a] <= eta_tol) keep.push_back(a);
    std::sort(keep.begin(), keep.end(), [&](int x, int y) {
      const zc lx = lam[cand[x]], ly = lam[cand[y]];
      return lx.real() != ly.real() ? lx.real() < ly.real() : lx.imag() < ly.imag();
    });
    mret = std::min((int)keep.size(), o->max_eigs);
    for (int a = 0; a < mret; ++a) {
      const int b = keep[a];
      lambda[2 * a] = lh[2 * b];
      lambda[2 * a + 1] = lh[2 * b + 1];
      eta[a] = eh[b];
      NEP_HIP(hipMemcpyAsync(reinterpret_cast<c128*>(X) + (size_t)a * n, dX.as<c128>() + (size_t)b * n,
                             sizeof(c128) * n, hipMemcpyDeviceToDevice, st));
    }
    NEP_HIP(hipStreamSynchronize(st));
  }
  *m_out = mret;
  if (Hout)
    for (size_t e = 0; e < tz.H.size(); ++e) {
      Hout[2 * e] = tz.H[e].real();
      Hout[2 * e + 1] = tz.H[e].imag();
    }
  if (info) {
    info->d = d;
    info->met = it.met;
    info->k_done = kd;
    info->basis = m;
    info->h_last = tz.hlast;
    info->ms_lu = ms_lu;
    info->ms_krylov = ms_krylov;
    info->ms_total = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return NEP_OK;
}


nep_status nep_nleigs_batch(int nprob, const nep_split* h, const nep_contour* g, const nep_nleigs_opts* o,
                            const void* const* W0, int* m_out, double* lambda, void* const* X, double* eta,
                            nep_nleigs_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  NEP_CHECK(nprob >= 1 && nprob <= 4096, NEP_ERR_ARG, "need 1 <= nprob <= 4096");
  NEP_CHECK(h && g && o && W0 && m_out && lambda && X && eta, NEP_ERR_ARG, "null argument");
  const int P = nprob, k = o[0].k, maxe = o[0].max_eigs;
  NEP_CHECK(k >= 1 && k <= kNlMaxK, NEP_ERR_ARG, "need 1 <= k <= %d", kNlMaxK);
  NEP_CHECK(maxe >= 1, NEP_ERR_ARG, "need max_eigs >= 1");
  for (int p = 0; p < P; ++p) {
    NEP_CHECK(h[p] != nullptr && W0[p] && X[p], NEP_ERR_ARG, "problem %d: null handle or buffer", p);
    NEP_TRY(check_contour(&g[p]));
    NEP_TRY(check_nleigs_opts(&o[p]));
    NEP_CHECK(o[p].k == k && o[p].max_eigs == maxe, NEP_ERR_ARG, "problem %d: k and max_eigs must match problem 0's",
              p);
    NEP_CHECK(o[p].eta_tol >= 0.0, NEP_ERR_ARG, "need eta_tol >= 0");
  }
  const hipStream_t st = h[0]->impl.stream;
  // per-problem descriptors (offsets filled in below)
  std::vector<NlbProb> hpb(P);
  for (int p = 0; p < P; ++p) {
    const SplitOperator& op = h[p]->impl.op;
    NlbProb& B = hpb[p];
    B = NlbProb{};
    B.n = op.n;
    B.ell = op.ell;
    for (int i = 0; i < op.ell; ++i) {
      B.t.A[i] = op.dA[i];
      B.t.diag[i] = op.dDiag[i];
      B.t.cplx[i] = op.is_cplx[i];
      B.t.isdiag[i] = op.is_diag[i];
      B.fn_root[i] = op.fn_root[i];
    }
    B.normA = op.dnormA;
    B.fn_nodes = op.dfn_nodes;
    B.fn_coef = op.dfn_coef;
  }
  DevMem dpb;
  NEP_TRY(dpb.alloc(sizeof(NlbProb) * P));
  NEP_HIP(hipMemcpyAsync(dpb.p, hpb.data(), sizeof(NlbProb) * P, hipMemcpyHostToDevice, st));
  const NlbProb* pb = dpb.as<NlbProb>();
  // interpolants: nodes on the host, every problem's f_i at its nodes in one
  // launch, divided differences on the host
  std::vector<InterpWork> iw(P);
  parallel_for(P, [&](int p) { interp_nodes(g[p], o[p], iw[p]); });
  int fstride = 1;
  for (int p = 0; p < P; ++p) fstride = std::max(fstride, iw[p].dmax + 1);
  std::vector<Interp> its(P);
  {
    std::vector<c128> zh((size_t)P * fstride, c128{0.0, 0.0});
    for (int p = 0; p < P; ++p)
      for (int j = 0; j <= iw[p].dmax; ++j) zh[(size_t)p * fstride + j] = c128{iw[p].sig[j].real(), iw[p].sig[j].imag()};
    DevMem dz, dfv, dbad;
    NEP_TRY(dz.alloc(sizeof(c128) * zh.size()));
    NEP_TRY(dfv.alloc(sizeof(c128) * zh.size() * kMaxTerms));
    NEP_TRY(dbad.alloc(sizeof(int) * zh.size()));
    NEP_HIP(hipMemcpyAsync(dz.p, zh.data(), sizeof(c128) * zh.size(), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_nlb_fn, dim3(ceil_div(P * fstride, 64)), dim3(64), 0, st, pb, P, fstride, dz.as<c128>(),
                       dfv.as<c128>(), dbad.as<int>());
    NEP_HIP(hipGetLastError());
    std::vector<c128> fv(zh.size() * kMaxTerms);
    std::vector<int> bad(zh.size());
    NEP_HIP(hipMemcpyAsync(fv.data(), dfv.p, sizeof(c128) * fv.size(), hipMemcpyDeviceToHost, st));
    NEP_HIP(hipMemcpyAsync(bad.data(), dbad.p, sizeof(int) * bad.size(), hipMemcpyDeviceToHost, st));
    NEP_HIP(hipStreamSynchronize(st));
    std::vector<nep_status> rs(P, NEP_OK);
    parallel_for(P, [&](int p) {
      const int ell = hpb[p].ell, dm1 = iw[p].dmax + 1;
      std::vector<c128> f((size_t)ell * dm1);
      for (int i = 0; i < ell; ++i)
        for (int j = 0; j < dm1; ++j) f[(size_t)i * dm1 + j] = fv[((size_t)p * kMaxTerms + i) * fstride + j];
      rs[p] = interp_finish(iw[p], ell, f.data(), bad.data() + (size_t)p * fstride, its[p]);
    });
    for (int p = 0; p < P; ++p)
      NEP_CHECK(rs[p] == NEP_OK, rs[p], "problem %d: an interpolation node lies on a pole or branch cut", p);
  }
  std::vector<ToarHost> tz(P);
  int mmax = 0, ellmax = 1, nmax = 1, dmaxd = 0;
  for (int p = 0; p < P; ++p) {
    Split& s = h[p]->impl;
    const zc sg(o[p].sigma[0], o[p].sigma[1]);
    for (int j = 0; j < its[p].d; ++j)
      NEP_CHECK(its[p].sigma[j] != sg, NEP_ERR_ARG, "problem %d: the shift equals interpolation node %d", p, j);
    for (int j = 1; j <= its[p].d; ++j)
      NEP_CHECK(inf_pole(its[p].xi[j]) || its[p].xi[j] != sg, NEP_ERR_ARG, "problem %d: the shift equals pole %d",
                p, j);
    tz[p].init(its[p], sg, s.op.ell, k);
    mmax = std::max(mmax, its[p].d + k);
    ellmax = std::max(ellmax, s.op.ell);
    nmax = std::max(nmax, s.op.n);
    dmaxd = std::max(dmaxd, its[p].d);
  }
  // device buffers: bases, products, coefficients, Gram--Schmidt results
  std::vector<long long> offU(P), offZ(P);
  long long totU = 0, totZ = 0;
  for (int p = 0; p < P; ++p) {
    const int n = h[p]->impl.op.n;
    offU[p] = totU;
    offZ[p] = totZ;
    totU += (long long)n * (mmax + 1);
    totZ += (long long)n * ellmax;
  }
  const long long qstride = (long long)(mmax + 1) * ellmax;
  const long long hs = 2LL * (mmax + 1) + 1;  // per problem: h1, h2, two norms
  DevMem dU, dZ, dQ, dsc, dm, dyp, dsig, drho;
  NEP_TRY(dU.alloc(sizeof(c128) * (size_t)totU));
  NEP_TRY(dZ.alloc(sizeof(c128) * (size_t)totZ));
  NEP_TRY(dQ.alloc(sizeof(c128) * (size_t)(qstride * P)));
  NEP_TRY(dsc.alloc(sizeof(c128) * (size_t)(hs * P)));
  NEP_TRY(dm.alloc(sizeof(int) * P));
  NEP_TRY(dyp.alloc(sizeof(c128*) * P));
  NEP_TRY(dsig.alloc(sizeof(c128) * P));
  NEP_TRY(drho.alloc(sizeof(c128) * (size_t)P * kMaxTerms));
  c128* U = dU.as<c128>();
  std::vector<c128> hsig(P), hrho((size_t)P * kMaxTerms);
  for (int p = 0; p < P; ++p) {
    hsig[p] = c128{o[p].sigma[0], o[p].sigma[1]};
    tz[p].rho(hrho.data() + (size_t)p * kMaxTerms);
  }
  NEP_HIP(hipMemcpyAsync(dsig.p, hsig.data(), sizeof(c128) * P, hipMemcpyHostToDevice, st));
  NEP_HIP(hipMemcpyAsync(drho.p, hrho.data(), sizeof(c128) * hrho.size(), hipMemcpyHostToDevice, st));

  // R_d(sigma_p) for every problem: one batched assembly and LU in complex FP64
  MomentsPlan plan;
  nep_contour g0{};
  g0.kind = 0;
  g0.rho = 1.0;
  g0.v = 1.0;
  PlanOptions po;
  po.N = 1;
  po.L = 1;
  po.K = 1;
  po.prec = NEP_PREC_FP64;
  po.max_refine = 0;
  po.fallback = 0;
  std::vector<PlanProblem> probs;
  probs.reserve(P);
  for (int p = 0; p < P; ++p) {
    PlanProblem pp{&h[p]->impl.op, g0, nullptr, nullptr, dsig.as<c128>() + p};
    pp.fpts = drho.as<c128>() + (size_t)p * kMaxTerms;
    probs.push_back(pp);
  }
  NEP_TRY(plan.build(probs, po, st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  NEP_HIP(hipEventCreate(&e0));
  NEP_HIP(hipEventCreate(&e1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } evg{e0, e1};
  NEP_HIP(hipEventRecord(e0, st));
  NEP_TRY(plan.factor(st));
  NEP_HIP(hipEventRecord(e1, st));
  {
    std::vector<int> pinfo(P);
    NEP_HIP(hipMemcpyAsync(pinfo.data(), plan.info(), sizeof(int) * P, hipMemcpyDeviceToHost, st));
    NEP_HIP(hipStreamSynchronize(st));
    for (int p = 0; p < P; ++p)
      NEP_CHECK(pinfo[p] >= h[p]->impl.op.n, NEP_ERR_SINGULAR, "problem %d: R_d(sigma) is exactly singular", p);
  }
  float ms_lu = 0.0f;
  NEP_HIP(hipEventElapsedTime(&ms_lu, e0, e1));
  const auto t1 = std::chrono::steady_clock::now();
  c128* Rb = plan.R_mut();
  c128* Yb = plan.Y_mut();
  for (int p = 0; p < P; ++p) {
    hpb[p].offU = offU[p];
    hpb[p].offZ = offZ[p];
    hpb[p].offY = plan.y_offset(p);
  }
  NEP_HIP(hipMemcpyAsync(dpb.p, hpb.data(), sizeof(NlbProb) * P, hipMemcpyHostToDevice, st));
  int* dms = dm.as<int>();
  c128** yp = dyp.as<c128*>();
  c128* hbase = dsc.as<c128>();
  double* nbase = reinterpret_cast<double*>(hbase + 2 * (mmax + 1));
  const long long nstride = 2 * hs;  // doubles
  const dim3 g256(256), g64(64);
  std::vector<int> hm(P);
  std::vector<c128*> hy(P);
  std::vector<c128> hb((size_t)(hs * P));
  // Gram--Schmidt of every y_p against U_p[:, 0:m_p] (m_p < 0: skipped), as
  // in the single-problem run; results read back in one copy
  auto orth = [&]() -> nep_status {
    NEP_HIP(hipMemcpyAsync(dms, hm.data(), sizeof(int) * P, hipMemcpyHostToDevice, st));
    NEP_HIP(hipMemcpyAsync(yp, hy.data(), sizeof(c128*) * P, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_nlb_norm, dim3(P), g256, 0, st, pb, dms, yp, nbase, nstride, 0);
    hipLaunchKernelGGL(k_nlb_dots, dim3(mmax, P), g256, 0, st, pb, dms, U, yp, hbase, hs);
    hipLaunchKernelGGL(k_nlb_sub, dim3(ceil_div(nmax, 64), P), g64, 0, st, pb, dms, U, hbase, hs, yp);
    hipLaunchKernelGGL(k_nlb_dots, dim3(mmax, P), g256, 0, st, pb, dms, U, yp, hbase + (mmax + 1), hs);
    hipLaunchKernelGGL(k_nlb_sub, dim3(ceil_div(nmax, 64), P), g64, 0, st, pb, dms, U, hbase + (mmax + 1), hs, yp);
    hipLaunchKernelGGL(k_nlb_norm, dim3(P), g256, 0, st, pb, dms, yp, nbase, nstride, 1);
    hipLaunchKernelGGL(k_nlb_store, dim3(ceil_div(nmax, 256), P), g256, 0, st, pb, dms, U, yp, nbase, nstride);
    NEP_HIP(hipGetLastError());
    NEP_HIP(hipMemcpyAsync(hb.data(), dsc.p, sizeof(c128) * hb.size(), hipMemcpyDeviceToHost, st));
    NEP_HIP(hipStreamSynchronize(st));
    return NEP_OK;
  };
  auto coef = [&](int p, int m, std::vector<zc>& c, double& n0, double& n1) {
    const c128* b = hb.data() + (size_t)p * hs;
    c.assign(m, zc());
    for (int t = 0; t < m; ++t) c[t] = zc(b[t].re + b[(mmax + 1) + t].re, b[t].im + b[(mmax + 1) + t].im);
    const double* nn = reinterpret_cast<const double*>(b + 2 * (mmax + 1));
    n0 = nn[0];
    n1 = nn[1];
  };

  // starting blocks: QR of [w^0 .. w^{d-1}] per problem by Gram--Schmidt
  for (int p = 0; p < P; ++p)
    NEP_HIP(hipMemcpyAsync(U + offU[p], W0[p], sizeof(c128) * (size_t)h[p]->impl.op.n * its[p].d,
                           hipMemcpyDeviceToDevice, st));
  {
    std::vector<std::vector<zc>> R(P);
    for (int p = 0; p < P; ++p) R[p].assign((size_t)its[p].d * its[p].d, zc());
    std::vector<zc> c;
    for (int q = 0; q < dmaxd; ++q) {
      for (int p = 0; p < P; ++p) {
        hm[p] = q < its[p].d ? q : -1;
        hy[p] = U + offU[p] + (long long)q * h[p]->impl.op.n;
      }
      NEP_TRY(orth());
      for (int p = 0; p < P; ++p) {
        if (q >= its[p].d) continue;
        double n0 = 0.0, n1 = 0.0;
        coef(p, q, c, n0, n1);
        NEP_CHECK(n1 > kNlDep * n0 && n0 > 0.0, NEP_ERR_ARG, "problem %d: starting block column %d is linearly "
                  "dependent", p, q);
        const int d = its[p].d;
        for (int t = 0; t < q; ++t) R[p][(size_t)q * d + t] = c[t];
        R[p][(size_t)q * d + q] = n1;
      }
    }
    for (int p = 0; p < P; ++p) tz[p].start(R[p]);
  }
  // Arnoldi steps, all problems together
  std::vector<c128> Qh((size_t)(qstride * P));
  for (int p = 0; p < P; ++p) hy[p] = Yb + hpb[p].offY;
  const unsigned hwc = std::max(1u, std::thread::hardware_concurrency());
  HostPool pool(std::max(0, std::min<int>({15, (int)hwc - 1, P / 8})));
  for (int j = 0; j < k; ++j) {
    bool any = false;
    for (int p = 0; p < P; ++p) any |= !tz[p].done;
    if (!any) break;
    pool.run(P, [&](int p) {
      hm[p] = tz[p].done ? -1 : tz[p].m;
      if (!tz[p].done) tz[p].rhs(j, Qh.data() + p * qstride);
    });
    NEP_HIP(hipMemcpyAsync(dms, hm.data(), sizeof(int) * P, hipMemcpyHostToDevice, st));
    NEP_HIP(hipMemcpyAsync(dQ.p, Qh.data(), sizeof(c128) * Qh.size(), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_nlb_rhs, dim3(ceil_div(nmax, 64), ellmax, P), g64, 0, st, pb, dms, U, dQ.as<c128>(), qstride,
                       dZ.as<c128>());
    hipLaunchKernelGGL(k_nlb_splitmv, dim3(ceil_div(nmax, 4), P), g256, 0, st, pb, dms, dZ.as<c128>(), Rb);
    NEP_HIP(hipGetLastError());
    NEP_TRY(plan.solve_rhs(st));  // y^0_p = R_d(sigma_p)^{-1} rhs_p, every problem
    NEP_TRY(orth());
    pool.run(P, [&](int p) {
      if (hm[p] < 0) return;
      std::vector<zc> c;
      double n0 = 0.0, n1 = 0.0;
      coef(p, hm[p], c, n0, n1);
      tz[p].absorb(j, c, n0, n1);
    });
  }
  const float ms_krylov = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t1).count();

  // Ritz pairs inside each region, their vectors and backward errors
  std::vector<NlbPair> pairs;
  std::vector<c128> Sx;
  long long xtot = 0;
  std::vector<std::vector<zc>> lams(P), Ss(P);
  std::vector<char> rok(P, 1);
  parallel_for(P, [&](int p) { rok[p] = tz[p].ritz(lams[p], Ss[p]) ? 1 : 0; });
  for (int p = 0; p < P; ++p) {
    NEP_CHECK(rok[p], NEP_ERR_DEVICE, "problem %d: eigenvalues of the Hessenberg matrix did not converge", p);
    const std::vector<zc>& lam = lams[p];
    const std::vector<zc>& S = Ss[p];
    for (int q = 0; q < tz[p].kd; ++q) {
      if (!inside_region(g[p], lam[q])) continue;
      NlbPair a{};
      a.p = p;
      a.m = tz[p].m;
      a.lam = c128{lam[q].real(), lam[q].imag()};
      a.soff = (long long)Sx.size();
      a.xoff = xtot;
      Sx.resize(Sx.size() + tz[p].m);
      tz[p].ritz_coeffs(S, q, Sx.data() + a.soff);
      xtot += h[p]->impl.op.n;
      pairs.push_back(a);
    }
  }
  const int npair = (int)pairs.size();
  std::vector<double> et(npair);
  std::vector<std::vector<int>> keep(P);
  DevMem dpr, dS, dX, deta, dkeep, ddst;
  if (npair > 0) {
    NEP_TRY(dpr.alloc(sizeof(NlbPair) * npair));
    NEP_TRY(dS.alloc(sizeof(c128) * Sx.size()));
    NEP_TRY(dX.alloc(sizeof(c128) * (size_t)xtot));
    NEP_TRY(deta.alloc(sizeof(double) * npair));
    NEP_HIP(hipMemcpyAsync(dpr.p, pairs.data(), sizeof(NlbPair) * npair, hipMemcpyHostToDevice, st));
    NEP_HIP(hipMemcpyAsync(dS.p, Sx.data(), sizeof(c128) * Sx.size(), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_nlb_vectors, dim3(npair), g256, 0, st, pb, dpr.as<NlbPair>(), U, dS.as<c128>(),
                       dX.as<c128>());
    hipLaunchKernelGGL(k_nlb_eta, dim3(npair), g256, 0, st, pb, dpr.as<NlbPair>(), dX.as<c128>(), deta.as<double>());
    NEP_HIP(hipGetLastError());
    NEP_HIP(hipMemcpyAsync(et.data(), deta.p, sizeof(double) * npair, hipMemcpyDeviceToHost, st));
    NEP_HIP(hipStreamSynchronize(st));
    for (int a = 0; a < npair; ++a) {
      const int p = pairs[a].p;
      const double tol = o[p].eta_tol > 0.0 ? o[p].eta_tol : 1e-10;
      if (et[a] <= tol) keep[p].push_back(a);
    }
  }
  std::vector<int> kept;
  std::vector<c128*> dst;
  for (int p = 0; p < P; ++p) {
    auto& kp = keep[p];
    std::sort(kp.begin(), kp.end(), [&](int x, int y) {
      const c128 lx = pairs[x].lam, ly = pairs[y].lam;
      return lx.re != ly.re ? lx.re < ly.re : lx.im < ly.im;
    });
    const int mr = std::min((int)kp.size(), maxe);
    m_out[p] = mr;
    for (int a = 0; a < mr; ++a) {
      const NlbPair& pr = pairs[kp[a]];
      lambda[2 * ((size_t)p * maxe + a)] = pr.lam.re;
      lambda[2 * ((size_t)p * maxe + a) + 1] = pr.lam.im;
      eta[(size_t)p * maxe + a] = et[kp[a]];
      kept.push_back(kp[a]);
      dst.push_back(reinterpret_cast<c128*>(X[p]) + (size_t)a * h[p]->impl.op.n);
    }
  }
  if (!kept.empty()) {
    NEP_TRY(dkeep.alloc(sizeof(int) * kept.size()));
    NEP_TRY(ddst.alloc(sizeof(c128*) * dst.size()));
    NEP_HIP(hipMemcpyAsync(dkeep.p, kept.data(), sizeof(int) * kept.size(), hipMemcpyHostToDevice, st));
    NEP_HIP(hipMemcpyAsync(ddst.p, dst.data(), sizeof(c128*) * dst.size(), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_nlb_gather, dim3((unsigned)kept.size()), g256, 0, st, dpr.as<NlbPair>(), dkeep.as<int>(),
                       ddst.as<c128*>(), dX.as<c128>(), pb);
    NEP_HIP(hipGetLastError());
  }
  NEP_HIP(hipStreamSynchronize(st));
  if (info) {
    const float ms_total = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (int p = 0; p < P; ++p) {
      info[p].d = its[p].d;
      info[p].met = its[p].met;
      info[p].k_done = tz[p].kd;
      info[p].basis = tz[p].m;
      info[p].h_last = tz[p].hlast;
      info[p].ms_lu = ms_lu;
      info[p].ms_krylov = ms_krylov;
      info[p].ms_total = ms_total;
    }
  }
  return NEP_OK;
}

}  // extern "C"
