// Extraction of the eigenpairs inside the contour from the moments.
//
// With B0 = [S_{r+s}] and B1 = [S_{r+s+1}] (r, s = 0..K-1, each Kn x KL), the
// Keldysh expansion (eq. (resolvent)) gives B0 = V_K(X, M) W and
// B1 = V_K(X, M) M W with V_K the block matrix of eq. (invpair-split).  If
// B0 = V0 Sigma0 W0^H is its rank-m truncated SVD, V0^H B1 W0 Sigma0^{-1} is
// similar to M (the eigenvalues mu_i = (lambda_i - c)/rho inside); an
// eigenvector s gives V0 s = [x; mu x; ...], whose first block is x.  The pair
// (X, c + rho M) is a minimal invariant pair (Section 2).
//
// Device: Householder QR of B0 (one reflector at a time), Q applied to the
// small singular vectors, V0^H B1, the eigenvectors, and the split-form
// residual T(lambda) x for the backward error of eq. (sressplit) (inf-norms).
// Host: one-sided Jacobi SVD of the K*L x K*L factor R and the m x m
// eigenproblem (sequential small dense work, as for the projected problems
// of the paper's solvers, Section 5).
#include <algorithm>
#include <cmath>
#include <mutex>
#include <numeric>

#include "dense.hpp"
#include "handle.hpp"

namespace nep {

struct ExtractWork {
  DevMem B0, B1, tau, V0, P, smat, X0, Rt, norms, fz, Rp;
  size_t cap_rows = 0, cap_cols = 0;
};

std::shared_ptr<ExtractWork> make_extract_work() { return std::make_shared<ExtractWork>(); }

// ---------------------------------------------------------------------------
__global__ void k_hankel(const c128* __restrict__ S, int n, int L, int K, long long sstride, c128* __restrict__ B0,
                         c128* __restrict__ B1) {
  const long long M = (long long)K * n, KL = (long long)K * L;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * KL) return;
  const long long col = e / M, row = e - col * M;
  const int r = (int)(row / n), i = (int)(row - (long long)r * n);
  const int s = (int)(col / L), c = (int)(col - (long long)s * L);
  const long long off = (long long)c * n + i;
  B0[e] = S[(long long)(r + s) * sstride + off];
  B1[e] = S[(long long)(r + s + 1) * sstride + off];
}

// R's leading KL x KL block (column-major, leading dimension M) into a
// contiguous KL x KL array, for one plain read-back
__global__ void k_pack_r(const c128* __restrict__ B, long long M, int KL, c128* __restrict__ R) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)KL * KL) return;
  const long long j = e / KL, i = e - j * KL;
  R[e] = B[j * M + i];
}

// block sum over 1024 threads
__device__ __forceinline__ c128 block_sum(c128 v, c128* red) {
  for (int o = 32; o >= 1; o >>= 1) {
    v.re += __shfl_xor(v.re, o, 64);
    v.im += __shfl_xor(v.im, o, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  c128 s = {0.0, 0.0};
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s = s + red[i];
  return s;
}

// Householder vector of column k (zlarfg convention): H^H x = beta e_1 with
// H = I - tau v v^H, v_0 = 1, beta real.  v overwrites x below the diagonal.
// One group of 1024 threads.
__device__ void house_vec(c128* __restrict__ B, long long M, int k, c128* __restrict__ tau, c128* red) {
  c128* x = B + (long long)k * M;
  double ss = 0.0;
  for (long long i = k + 1 + threadIdx.x; i < M; i += blockDim.x) ss += norm2(x[i]);
  const c128 tot = block_sum(c128{ss, 0.0}, red);
  const double sigma2 = tot.re;
  const c128 alpha = x[k];
  __syncthreads();
  if (sigma2 == 0.0 && alpha.im == 0.0) {
    if (threadIdx.x == 0) tau[k] = c128{0.0, 0.0};
    return;
  }
  const double nrm = sqrt(norm2(alpha) + sigma2);
  const double beta = alpha.re >= 0.0 ? -nrm : nrm;
  const c128 t = {(beta - alpha.re) / beta, -alpha.im / beta};
  const c128 scal = cdiv(c128{1.0, 0.0}, c128{alpha.re - beta, alpha.im});
  for (long long i = k + 1 + threadIdx.x; i < M; i += blockDim.x) x[i] = x[i] * scal;
  if (threadIdx.x == 0) {
    tau[k] = t;
    x[k] = c128{beta, 0.0};
  }
}

__global__ __launch_bounds__(1024) void k_house_vec(c128* __restrict__ B, long long M, int k, c128* __restrict__ tau) {
  __shared__ c128 red[16];
  house_vec(B, M, k, tau, red);
}

// b <- H^H b = b - conj(tau) v (v^H b) for columns k+1.. (one group each).
// The group of column k+1 then forms that column's Householder vector (the
// next step's), so a step is one launch: only this group writes column k+1.
__global__ __launch_bounds__(1024) void k_house_apply(c128* __restrict__ B, long long M, int k, int ncol,
                                                      c128* __restrict__ tau) {
  __shared__ c128 red[16];
  const int col = k + 1 + blockIdx.x;
  if (col >= ncol) return;
  const c128* v = B + (long long)k * M;
  c128* b = B + (long long)col * M;
  c128 acc = {0.0, 0.0};
  if (threadIdx.x == 0) acc = b[k];  // v_k = 1
  for (long long i = k + 1 + threadIdx.x; i < M; i += blockDim.x) acc = acc + conj(v[i]) * b[i];
  const c128 w = block_sum(acc, red);
  const c128 f = conj(tau[k]) * w;
  if (threadIdx.x == 0) b[k] = b[k] - f;
  for (long long i = k + 1 + threadIdx.x; i < M; i += blockDim.x) b[i] = b[i] - v[i] * f;
  if (blockIdx.x == 0) {
    __syncthreads();  // the group's updates of column k+1 are visible to all its threads
    house_vec(B, M, col, tau, red);
  }
}

// X <- Q X = H_0 H_1 ... H_{r-1} X, one group per column of X (M x m)
__global__ __launch_bounds__(1024) void k_apply_q(const c128* __restrict__ B, long long M, int r,
                                                  const c128* __restrict__ tau, c128* __restrict__ X) {
  __shared__ c128 red[16];
  c128* x = X + (long long)blockIdx.x * M;
  for (int k = r - 1; k >= 0; --k) {
    const c128* v = B + (long long)k * M;
    c128 acc = {0.0, 0.0};
    if (threadIdx.x == 0) acc = x[k];
    for (long long i = k + 1 + threadIdx.x; i < M; i += blockDim.x) acc = acc + conj(v[i]) * x[i];
    const c128 w = block_sum(acc, red);
    const c128 f = tau[k] * w;
    __syncthreads();
    if (threadIdx.x == 0) x[k] = x[k] - f;
    for (long long i = k + 1 + threadIdx.x; i < M; i += blockDim.x) x[i] = x[i] - v[i] * f;
    __syncthreads();
  }
}

// P[i + j*m] = sum_r conj(V0[r, i]) B1[r, j]; one group per (i, j)
__global__ __launch_bounds__(256) void k_vhb(const c128* __restrict__ V0, const c128* __restrict__ B1, long long M,
                                             int m, c128* __restrict__ P) {
  __shared__ c128 red[16];
  const int i = blockIdx.x % m, j = blockIdx.x / m;
  const c128* a = V0 + (long long)i * M;
  const c128* b = B1 + (long long)j * M;
  c128 acc = {0.0, 0.0};
  for (long long r = threadIdx.x; r < M; r += blockDim.x) acc = acc + conj(a[r]) * b[r];
  const c128 s = block_sum(acc, red);
  if (threadIdx.x == 0) P[(long long)j * m + i] = s;
}

// X[:, q] = V0[0:n, :] s[:, q], normalized (2-norm 1, largest entry real > 0)
__global__ __launch_bounds__(256) void k_eigvec(const c128* __restrict__ V0, long long M, int n, int m,
                                                const c128* __restrict__ smat, c128* __restrict__ X) {
  __shared__ c128 red[16];
  __shared__ double rmax[4];
  __shared__ int ridx[4];
  const int q = blockIdx.x;
  c128* x = X + (long long)q * n;
  double ss = 0.0;
  double bm = -1.0;
  int bi = 0x7fffffff;
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    c128 acc = {0.0, 0.0};
    for (int j = 0; j < m; ++j) acc = acc + V0[(long long)j * M + r] * smat[(long long)q * m + j];
    x[r] = acc;
    const double a2 = norm2(acc);
    ss += a2;
    if (a2 > bm) { bm = a2; bi = r; }
  }
  const c128 tot = block_sum(c128{ss, 0.0}, red);
  for (int o = 32; o >= 1; o >>= 1) {
    const double ov = __shfl_xor(bm, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (ov > bm || (ov == bm && oi < bi)) { bm = ov; bi = oi; }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) { rmax[w] = bm; ridx[w] = bi; }
  __syncthreads();
  bm = rmax[0];
  bi = ridx[0];
  for (int i = 1; i < 4; ++i)
    if (rmax[i] > bm || (rmax[i] == bm && ridx[i] < bi)) { bm = rmax[i]; bi = ridx[i]; }
  const double nrm = sqrt(tot.re);
  const c128 piv = x[bi];
  const double ap = sqrt(norm2(piv));
  // scale = conj(piv)/|piv| / nrm
  const c128 scale = (ap > 0.0 && nrm > 0.0) ? c128{piv.re / (ap * nrm), -piv.im / (ap * nrm)} : c128{0.0, 0.0};
  __syncthreads();
  for (int r = threadIdx.x; r < n; r += blockDim.x) x[r] = x[r] * scale;
}

// Rt[row, q] = sum_i coef[i*m + q] (A_i x_q)[row]  (split-form T(lambda_q) x_q)
// A and x tiles staged through LDS.
__global__ __launch_bounds__(512) void k_split_apply(const ProbDesc* __restrict__ pd_unused, int n, int ell, int m,
                                                     const double* const* __restrict__ A, const int* __restrict__ cplx,
                                                     const c128* __restrict__ coef, const c128* __restrict__ X,
                                                     c128* __restrict__ Rt) {
  // one group per 16 rows x 32 pairs, one output per thread: every A_i row
  // is read by one group only, and n/16 groups keep the CUs busy; each
  // output sums over k in ascending order
  constexpr int RB = 16, QB = 32, KC = 64;
  __shared__ c128 As[RB][KC + 1];
  __shared__ c128 Xs[KC][QB + 1];
  const int row0 = blockIdx.x * RB, q0 = blockIdx.y * QB;
  const int tr = threadIdx.x >> 5, tq = threadIdx.x & 31;
  c128 out = {0.0, 0.0};
  for (int i = 0; i < ell; ++i) {
    c128 acc = {0.0, 0.0};
    for (int s0 = 0; s0 < n; s0 += KC) {
      for (int e = threadIdx.x; e < RB * KC; e += 512) {
        const int r = e / KC, k = e - r * KC;
        const int gr = row0 + r, gs = s0 + k;
        c128 a = {0.0, 0.0};
        if (gr < n && gs < n) {
          if (cplx[i]) a = reinterpret_cast<const c128*>(A[i])[(long long)gr * n + gs];
          else a.re = A[i][(long long)gr * n + gs];
        }
        As[r][k] = a;
      }
      for (int e = threadIdx.x; e < KC * QB; e += 512) {
        const int q = e / KC, k = e - q * KC;
        const int gs = s0 + k, gq = q0 + q;
        Xs[k][q] = (gs < n && gq < m) ? X[(long long)gq * n + gs] : c128{0.0, 0.0};
      }
      __syncthreads();
#pragma unroll 8
      for (int k = 0; k < KC; ++k) acc = acc + As[tr][k] * Xs[k][tq];
      __syncthreads();
    }
    const int gq = q0 + tq;
    if (gq < m) out = out + coef[(long long)i * m + gq] * acc;
  }
  const int gr = row0 + tr, gq = q0 + tq;
  if (gr < n && gq < m) Rt[(long long)gq * n + gr] = out;
}

// per column: max |Rt|, max |X|
__global__ void k_colmax2(const c128* __restrict__ Rt, const c128* __restrict__ X, int n, double* __restrict__ out) {
  __shared__ double r1[256], r2[256];
  const int q = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    a = nanmax(a, sqrt(norm2(Rt[(long long)q * n + r])));
    b = nanmax(b, sqrt(norm2(X[(long long)q * n + r])));
  }
  r1[threadIdx.x] = a;
  r2[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      r1[threadIdx.x] = nanmax(r1[threadIdx.x], r1[threadIdx.x + s]);
      r2[threadIdx.x] = nanmax(r2[threadIdx.x], r2[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * q] = r1[0];
    out[2 * q + 1] = r2[0];
  }
}

// ---------------------------------------------------------------------------
static nep_status grow(DevMem& m, size_t bytes) {
  if (m.bytes >= bytes) return NEP_OK;
  return m.alloc(bytes);
}

// eta for m pairs: X device (n x m column-major), lambda host.
hipError_t fn_points(const FnNode* nodes, const c128* coef, const int* roots, int ell, const c128* z, int m,
                     c128* out, int* bad, hipStream_t st);

// Device buffers of one backward-error evaluation of m pairs.
struct EtaBuffers {
  c128* z;            // m points
  c128* fv;           // f_i(lambda_q) at [i*m + q]
  int* bad;           // m flags: lambda_q on a pole or cut
  c128* Rt;           // n x m residuals T(lambda_q) x_q
  double* norms;      // 2m: max |Rt[:, q]|, max |X[:, q]|
  const double** dA;  // kMaxTerms term pointers
  int* dcp;           // kMaxTerms complex-term flags
};

static size_t eta_small_bytes(int m, int ell) {  // everything but Rt, each part 256-byte aligned
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  return up(sizeof(c128) * m) + up(sizeof(c128) * (size_t)m * ell) + up(sizeof(int) * m) + up(sizeof(double) * 2 * m) +
         up(sizeof(void*) * kMaxTerms) + up(sizeof(int) * kMaxTerms);
}

static EtaBuffers eta_carve(char* small, c128* Rt, int m, int ell) {
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  EtaBuffers b;
  b.z = reinterpret_cast<c128*>(small);
  small += up(sizeof(c128) * m);
  b.fv = reinterpret_cast<c128*>(small);
  small += up(sizeof(c128) * (size_t)m * ell);
  b.bad = reinterpret_cast<int*>(small);
  small += up(sizeof(int) * m);
  b.norms = reinterpret_cast<double*>(small);
  small += up(sizeof(double) * 2 * m);
  b.dA = reinterpret_cast<const double**>(small);
  small += up(sizeof(void*) * kMaxTerms);
  b.dcp = reinterpret_cast<int*>(small);
  b.Rt = Rt;
  return b;
}

// eta of eq. (sressplit) with infinity norms for m pairs: lam host (m
// complex), X device (n x m column-major).  The device computes f_i(lambda_q),
// the split-form residuals T(lambda_q) x_q and the column maxima into b; the
// host reads fv_h (m*ell), bad_h (m), hn_h (2m) back and forms
// eta_q = max|T x| / (sum_i |f_i| ||A_i||_inf max|x|).
static nep_status eta_run(Split& h, int m, const c128* lam, const c128* X, const EtaBuffers& b, c128* fv_h,
                          int* bad_h, double* hn_h, double* eta, hipStream_t st) {
  const int n = h.op.n, ell = h.op.ell;
  const double* hA[kMaxTerms];
  for (int i = 0; i < ell; ++i) hA[i] = reinterpret_cast<const double*>(h.op.dA[i]);
  NEP_HIP(hipMemcpyAsync(b.z, lam, sizeof(c128) * m, hipMemcpyHostToDevice, st));
  NEP_HIP(hipMemcpyAsync(b.dA, hA, sizeof(void*) * ell, hipMemcpyHostToDevice, st));
  NEP_HIP(hipMemcpyAsync(b.dcp, h.op.is_cplx, sizeof(int) * ell, hipMemcpyHostToDevice, st));
  NEP_HIP(fn_points(h.op.dfn_nodes, h.op.dfn_coef, h.fn_roots.as<int>(), ell, b.z, m, b.fv, b.bad, st));
  dim3 grid(ceil_div(n, 16), ceil_div(m, 32));
  hipLaunchKernelGGL(k_split_apply, grid, dim3(512), 0, st, nullptr, n, ell, m, b.dA, b.dcp, b.fv, X, b.Rt);
  NEP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_colmax2, dim3(m), dim3(256), 0, st, b.Rt, X, n, b.norms);
  NEP_HIP(hipGetLastError());
  NEP_HIP(hipMemcpyAsync(fv_h, b.fv, sizeof(c128) * (size_t)m * ell, hipMemcpyDeviceToHost, st));
  NEP_HIP(hipMemcpyAsync(bad_h, b.bad, sizeof(int) * m, hipMemcpyDeviceToHost, st));
  NEP_HIP(hipMemcpyAsync(hn_h, b.norms, sizeof(double) * 2 * m, hipMemcpyDeviceToHost, st));
  NEP_HIP(hipStreamSynchronize(st));
  for (int q = 0; q < m; ++q) {
    if (bad_h[q]) {
      eta[q] = NAN;
      continue;
    }
    double den = 0.0;
    for (int i = 0; i < ell; ++i) {
      const c128 f = fv_h[(size_t)i * m + q];
      den += std::sqrt(f.re * f.re + f.im * f.im) * h.op.normA[i];
    }
    den *= hn_h[2 * q + 1];
    eta[q] = den > 0.0 ? hn_h[2 * q] / den : NAN;
  }
  return NEP_OK;
}

static nep_status backward_errors(Split& h, int m, const std::vector<zc>& lam, const c128* X, std::vector<double>& eta,
                                  ExtractWork& w, hipStream_t st) {
  const int n = h.op.n, ell = h.op.ell;
  // the workspace grows and never shrinks: no device allocation or free once
  // it is large enough
  NEP_TRY(grow(w.fz, eta_small_bytes(m, ell)));
  NEP_TRY(grow(w.Rt, sizeof(c128) * (size_t)n * m));
  const EtaBuffers b = eta_carve(w.fz.as<char>(), w.Rt.as<c128>(), m, ell);
  std::vector<c128> fv((size_t)m * ell);
  std::vector<int> bad(m);
  std::vector<double> hn(2 * m);
  eta.assign(m, 0.0);
  return eta_run(h, m, reinterpret_cast<const c128*>(lam.data()), X, b, fv.data(), bad.data(), hn.data(), eta.data(),
                 st);
}

// eta for m pairs (host points, device vectors) into host eta, with the given
// workspace or the handle's own.
nep_status backward_errors_dev(Split& h, int m, const c128* lam, const c128* X, double* eta, ExtractWork* w,
                               hipStream_t st) {
  if (!w) {
    if (!h.xw) h.xw = std::make_shared<ExtractWork>();
    w = h.xw.get();
  }
  std::vector<zc> lz(m);
  for (int q = 0; q < m; ++q) lz[q] = zc(lam[q].re, lam[q].im);
  std::vector<double> et;
  NEP_TRY(backward_errors(h, m, lz, X, et, *w, st));
  for (int q = 0; q < m; ++q) eta[q] = et[q];
  return NEP_OK;
}

nep_status rii_polish(Split& h, int m, zc* lam, c128* X, double* eta, const char* sel, double tol, int max_it,
                      int* iters, ExtractWork* w, hipStream_t st);

// ---------------------------------------------------------------------------
// Backward errors without allocation.  Callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops) use
// nep_backward_error_noalloc: its scratch is this file-scope device array, one
// copy per GPU, held until the process ends.  Host code must not use the
// array's name as a device address; each device's address comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr int kNoAllocMaxPairs = 256;                       // m
constexpr size_t kNoAllocMaxResid = (size_t)1 << 18;        // n * m complex entries (4 MiB)
constexpr size_t kNoAllocSmall = 128 << 10;                 // points, f values, flags, maxima, term tables
constexpr size_t kNoAllocBytes = kNoAllocMaxResid * sizeof(c128) + kNoAllocSmall;
static __device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {nullptr};

static nep_status scratch_address(void** out) {
  int dev = 0;
  NEP_HIP(hipGetDevice(&dev));
  NEP_CHECK(dev >= 0 && dev < kMaxDevices, NEP_ERR_DEVICE, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      set_error("hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
      return NEP_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return NEP_OK;
}

static nep_status backward_errors_noalloc(Split& h, int m, const double* lambda, const c128* X, double* eta) {
  const int n = h.op.n, ell = h.op.ell;
  NEP_CHECK(m <= kNoAllocMaxPairs, NEP_ERR_ARG, "at most %d pairs per call without allocation (got %d)",
            kNoAllocMaxPairs, m);
  NEP_CHECK((size_t)n * m <= kNoAllocMaxResid, NEP_ERR_ARG,
            "n * m = %lld exceeds the %zu residual entries of the allocation-free scratch", (long long)n * m,
            kNoAllocMaxResid);
  static_assert(sizeof(c128) * kNoAllocMaxPairs + ((sizeof(c128) * kNoAllocMaxPairs * kMaxTerms + 255) / 256 * 256) +
                        sizeof(int) * kNoAllocMaxPairs + sizeof(double) * 2 * kNoAllocMaxPairs + 4 * 256 <=
                    kNoAllocSmall,
                "small scratch region too small");
  void* base = nullptr;
  NEP_TRY(scratch_address(&base));
  char* p = static_cast<char*>(base);
  const EtaBuffers b = eta_carve(p + kNoAllocMaxResid * sizeof(c128), reinterpret_cast<c128*>(p), m, ell);
  // host read-back space on the stack (bounded by the limits above)
  c128 fv[kNoAllocMaxPairs * kMaxTerms];
  int bad[kNoAllocMaxPairs];
  double hn[2 * kNoAllocMaxPairs];
  return eta_run(h, m, reinterpret_cast<const c128*>(lambda), X, b, fv, bad, hn, eta, h.stream);
}

nep_status extract(Split& h, const nep_contour* g, const nep_ciss_opts* o, const void* S,
                   const nep_extract_opts* e, int* m_out, double* lambda, void* X, double* eta, int* inside,
                   double* sigma, ExtractWork* wk) {
  PlanOptions po;
  NEP_TRY(check_opts(o, po));
  return extract_strided(h, g, o, po.L, S, 0, e, m_out, lambda, X, eta, inside, sigma, wk);
}

nep_status extract_strided(Split& h, const nep_contour* g, const nep_ciss_opts* o, int L_eff, const void* S,
                           long long sstride, const nep_extract_opts* e, int* m_out, double* lambda, void* X,
                           double* eta, int* inside, double* sigma, ExtractWork* wk) {
  NEP_TRY(check_contour(g));
  PlanOptions po;
  NEP_TRY(check_opts(o, po));
  NEP_CHECK(e != nullptr && e->max_eigs >= 1, NEP_ERR_ARG, "extract options: max_eigs must be >= 1");
  NEP_CHECK(e->rank_tol >= 0.0 && e->eta_tol >= 0.0, NEP_ERR_ARG, "extract options: tolerances must be >= 0");
  NEP_CHECK(S != nullptr && X != nullptr && m_out && lambda && eta && inside, NEP_ERR_ARG, "null output array");
  const int n = h.op.n, L = L_eff, K = po.K;
  if (sstride <= 0) sstride = (long long)n * L;
  const long long M = (long long)K * n;
  const int KL = K * L;
  NEP_CHECK(KL <= M, NEP_ERR_ARG, "K*L exceeds K*n");
  hipStream_t st = o->stream ? (hipStream_t)o->stream : h.stream;
  if (!wk) {
    if (!h.xw) h.xw = std::make_shared<ExtractWork>();
    wk = h.xw.get();
  }
  ExtractWork& w = *wk;
  NEP_TRY(grow(w.B0, sizeof(c128) * M * KL));
  NEP_TRY(grow(w.B1, sizeof(c128) * M * KL));
  NEP_TRY(grow(w.tau, sizeof(c128) * KL));
  NEP_TRY(grow(w.Rp, sizeof(c128) * (size_t)KL * KL));
  c128* B0 = w.B0.as<c128>();
  c128* B1 = w.B1.as<c128>();
  c128* tau = w.tau.as<c128>();
  const long long tot = M * KL;
  hipLaunchKernelGGL(k_hankel, dim3((unsigned)ceil_div_ll(tot, 256)), dim3(256), 0, st, (const c128*)S, n, L, K,
                     sstride, B0, B1);
  NEP_HIP(hipGetLastError());
  // column 0's vector, then one launch per step: H_k applied to columns
  // k+1.., whose first group then forms column k+1's vector
  hipLaunchKernelGGL(k_house_vec, dim3(1), dim3(1024), 0, st, B0, M, 0, tau);
  NEP_HIP(hipGetLastError());
  for (int k = 0; k + 1 < KL; ++k) {
    hipLaunchKernelGGL(k_house_apply, dim3(KL - k - 1), dim3(1024), 0, st, B0, M, k, KL, tau);
    NEP_HIP(hipGetLastError());
  }
  // R (upper KL x KL) to host
  // (packed on the device and read back in one plain copy: a pitched
  // device-to-host copy read back zeros in a process where a profiler had
  // loaded a second HSA runtime beside the HIP runtime's own)
  std::vector<zc> R((size_t)KL * KL, zc(0.0, 0.0));
  {
    std::vector<zc> tmp((size_t)KL * KL);
    hipLaunchKernelGGL(k_pack_r, dim3((unsigned)ceil_div_ll((long long)KL * KL, 256)), dim3(256), 0, st, B0, M, KL,
                       w.Rp.as<c128>());
    NEP_HIP(hipGetLastError());
    NEP_HIP(hipMemcpyAsync(tmp.data(), w.Rp.p, sizeof(c128) * (size_t)KL * KL, hipMemcpyDeviceToHost, st));
    NEP_HIP(hipStreamSynchronize(st));
    for (int j = 0; j < KL; ++j)
      for (int i = 0; i <= j; ++i) R[(size_t)j * KL + i] = tmp[(size_t)j * KL + i];
  }
  std::vector<double> sv;
  std::vector<zc> Ur, Wr;
  jacobi_svd(KL, R, sv, Ur, Wr);
  if (sigma)
    for (int i = 0; i < KL; ++i) sigma[i] = sv[i];
  const double tol = (e->rank_tol > 0.0 ? e->rank_tol : 1e-12) * sv[0];
  int m = 0;
  while (m < KL && sv[m] > tol) ++m;
  *m_out = m;
  NEP_CHECK(m > 0, NEP_ERR_RANK, "all moments vanish: no eigenvalue inside the contour is visible");
  NEP_CHECK(m < KL, NEP_ERR_RANK, "moment rank %d == K*L: more eigenvalues inside or near the contour pass the "
            "rank threshold than K*L=%d can resolve; increase L or K (or N)", m, KL);
  NEP_CHECK(m <= e->max_eigs, NEP_ERR_ARG, "rank %d exceeds max_eigs %d", m, e->max_eigs);
  // V0 = Q [Ur0; 0]
  NEP_TRY(grow(w.V0, sizeof(c128) * M * m));
  c128* V0 = w.V0.as<c128>();
  {
    std::vector<zc> X0((size_t)M * m, zc(0.0, 0.0));
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < KL; ++i) X0[(size_t)j * M + i] = Ur[(size_t)j * KL + i];
    NEP_HIP(hipMemcpyAsync(V0, X0.data(), sizeof(c128) * M * m, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_apply_q, dim3(m), dim3(1024), 0, st, B0, M, KL, tau, V0);
    NEP_HIP(hipGetLastError());
    NEP_HIP(hipStreamSynchronize(st));  // X0 leaves scope
  }
  // Mt = V0^H B1 W0 Sigma0^{-1}
  NEP_TRY(grow(w.P, sizeof(c128) * (size_t)m * KL));
  hipLaunchKernelGGL(k_vhb, dim3(m * KL), dim3(256), 0, st, V0, B1, M, m, w.P.as<c128>());
  NEP_HIP(hipGetLastError());
  std::vector<zc> P((size_t)m * KL);
  NEP_HIP(hipMemcpyAsync(P.data(), w.P.p, sizeof(c128) * m * KL, hipMemcpyDeviceToHost, st));
  NEP_HIP(hipStreamSynchronize(st));
  std::vector<zc> Mt((size_t)m * m, zc(0.0, 0.0));
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) {
      zc acc = 0.0;
      for (int k = 0; k < KL; ++k) acc += P[(size_t)k * m + i] * Wr[(size_t)j * KL + k];
      Mt[(size_t)j * m + i] = acc / sv[j];
    }
  std::vector<zc> mu, Sv;
  NEP_CHECK(eig_general(m, Mt, mu, Sv), NEP_ERR_RANK, "QR iteration on the projected matrix did not converge");
  // order by (Re lambda, Im lambda)
  const zc c0(g->c[0], g->c[1]);
  std::vector<zc> lam(m);
  for (int i = 0; i < m; ++i) lam[i] = c0 + g->rho * mu[i];
  std::vector<int> ord(m);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    if (lam[a].real() != lam[b].real()) return lam[a].real() < lam[b].real();
    return lam[a].imag() < lam[b].imag();
  });
  std::vector<zc> lam_s(m), Ss((size_t)m * m);
  for (int q = 0; q < m; ++q) {
    lam_s[q] = lam[ord[q]];
    for (int i = 0; i < m; ++i) Ss[(size_t)q * m + i] = Sv[(size_t)ord[q] * m + i];
  }
  NEP_TRY(grow(w.smat, sizeof(c128) * (size_t)m * m));
  NEP_HIP(hipMemcpyAsync(w.smat.p, Ss.data(), sizeof(c128) * m * m, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_eigvec, dim3(m), dim3(256), 0, st, V0, M, n, m, w.smat.as<c128>(), (c128*)X);
  NEP_HIP(hipGetLastError());
  NEP_HIP(hipStreamSynchronize(st));
  std::vector<double> et;
  NEP_TRY(backward_errors(h, m, lam_s, (const c128*)X, et, w, st));
  // The region filter (Section 3.2.4) keeps the eigenvalues inside the
  // contour; of those, a pair counts as converged when its backward error is
  // below the tolerance, the stopping test of the paper's solvers.  A pair
  // inside but above it (typically a spurious one from a numerical rank taken
  // at the moments' noise floor) is flagged apart.
  const double etol = e->eta_tol > 0.0 ? e->eta_tol : 1e-8;
  auto in_region = [&](zc l) {
    const zc mu_q = (l - c0) / g->rho;
    return g->kind == 0 ? (std::abs(mu_q) < 1.0)
                        : (mu_q.real() * mu_q.real() + (mu_q.imag() / g->v) * (mu_q.imag() / g->v) < 1.0);
  };
  if (e->polish_its > 0) {
    // pairs inside but above the tolerance (limited by the quadrature or by
    // the truncation of weakly filtered outside eigenvalues) are polished by
    // residual inverse iteration (Section 4.1) in FP64
    std::vector<char> sel(m, 0);
    int cnt = 0;
    for (int q = 0; q < m; ++q) {
      sel[q] = in_region(lam_s[q]) && !(et[q] <= etol) && std::isfinite(et[q]);
      cnt += sel[q];
    }
    if (cnt > 0) {
      NEP_TRY(rii_polish(h, m, lam_s.data(), (c128*)X, et.data(), sel.data(), 1e-14, e->polish_its, nullptr, &w, st));
      // keep the output sorted by (Re, Im): permute the eigenvectors if
      // polishing changed the order
      std::vector<int> ord2(m);
      std::iota(ord2.begin(), ord2.end(), 0);
      std::stable_sort(ord2.begin(), ord2.end(), [&](int a, int b) {
        if (lam_s[a].real() != lam_s[b].real()) return lam_s[a].real() < lam_s[b].real();
        return lam_s[a].imag() < lam_s[b].imag();
      });
      bool moved = false;
      for (int q = 0; q < m; ++q) moved |= ord2[q] != q;
      if (moved) {
        NEP_TRY(grow(w.X0, sizeof(c128) * (size_t)n * m));
        NEP_HIP(hipMemcpyAsync(w.X0.p, X, sizeof(c128) * (size_t)n * m, hipMemcpyDeviceToDevice, st));
        for (int q = 0; q < m; ++q)
          NEP_HIP(hipMemcpyAsync((c128*)X + (size_t)q * n, w.X0.as<c128>() + (size_t)ord2[q] * n, sizeof(c128) * n,
                                 hipMemcpyDeviceToDevice, st));
        NEP_HIP(hipStreamSynchronize(st));
        std::vector<zc> l2(m);
        std::vector<double> e2(m);
        for (int q = 0; q < m; ++q) {
          l2[q] = lam_s[ord2[q]];
          e2[q] = et[ord2[q]];
        }
        lam_s.swap(l2);
        et.swap(e2);
      }
    }
  }
  for (int q = 0; q < m; ++q) {
    lambda[2 * q] = lam_s[q].real();
    lambda[2 * q + 1] = lam_s[q].imag();
    eta[q] = et[q];
    inside[q] = !in_region(lam_s[q]) ? 0 : (et[q] <= etol ? 1 : 2);
  }
  // two converged pairs with one eigenvalue (a polished spurious pair can
  // land on an eigenvalue another pair already holds): the one with the
  // larger backward error is not counted
  for (int a = 0; a < m; ++a)
    for (int b = a + 1; b < m; ++b)
      if (inside[a] == 1 && inside[b] == 1 && std::abs(lam_s[a] - lam_s[b]) <= 1e-8 * std::abs(lam_s[a]))
        inside[et[a] <= et[b] ? b : a] = 2;
  return NEP_OK;
}

}  // namespace nep

using namespace nep;

extern "C" {

nep_status nep_extract(nep_split h, const nep_contour* g, const nep_ciss_opts* o, const void* S,
                       const nep_extract_opts* e, int* m, double* lambda, void* X, double* eta, int* inside,
                       double* sigma) {
  NEP_CHECK(h != nullptr, NEP_ERR_ARG, "null handle");
  return nep::extract(h->impl, g, o, S, e, m, lambda, X, eta, inside, sigma, nullptr);
}

nep_status nep_backward_error_noalloc(nep_split h, int m, const double* lambda, const void* X, double* eta) {
  NEP_CHECK(h != nullptr, NEP_ERR_ARG, "null handle");
  NEP_CHECK(m >= 1 && lambda && X && eta, NEP_ERR_ARG, "bad arguments");
  return backward_errors_noalloc(h->impl, m, lambda, (const c128*)X, eta);
}

nep_status nep_backward_error(nep_split h, int m, const double* lambda, const void* X, double* eta) {
  NEP_CHECK(h != nullptr, NEP_ERR_ARG, "null handle");
  NEP_CHECK(m >= 1 && lambda && X && eta, NEP_ERR_ARG, "bad arguments");
  if (!h->impl.xw) h->impl.xw = std::make_shared<ExtractWork>();
  std::vector<zc> lam(m);
  for (int q = 0; q < m; ++q) lam[q] = zc(lambda[2 * q], lambda[2 * q + 1]);
  std::vector<double> et;
  NEP_TRY(backward_errors(h->impl, m, lam, (const c128*)X, et, *h->impl.xw, h->impl.stream));
  for (int q = 0; q < m; ++q) eta[q] = et[q];
  return NEP_OK;
}

}  // extern "C"
