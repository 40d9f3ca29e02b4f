// C ABI of libnep: split-operator handles, moments, batches (see nep.h).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <functional>
#include <random>
#include <thread>
#include <memory>
#include <string>
#include <vector>

#include "handle.hpp"

namespace nep {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

const char* last_error() { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// FN trees -> flat node array (children before use; depth-limited)
// ---------------------------------------------------------------------------
static nep_status flatten(const nep_fn* f, int depth, std::vector<FnNode>& nodes, std::vector<c128>& coef,
                          int* out_index) {
  NEP_CHECK(f != nullptr, NEP_ERR_ARG, "null function descriptor");
  NEP_CHECK(depth <= kMaxFnDepth, NEP_ERR_ARG, "function tree deeper than %d", kMaxFnDepth);
  NEP_CHECK((int)nodes.size() < kMaxFnNodes, NEP_ERR_ARG, "function tree larger than %d nodes", kMaxFnNodes);
  FnNode nd{};
  nd.type = f->type;
  nd.alpha = c128{f->alpha[0], f->alpha[1]};
  nd.beta = c128{f->beta[0], f->beta[1]};
  nd.a = nd.b = -1;
  switch (f->type) {
    case NEP_FN_RATIONAL:
      NEP_CHECK(f->nnum >= 1 && f->nnum <= kMaxCoeffs && f->nden >= 0 && f->nden <= kMaxCoeffs, NEP_ERR_ARG,
                "rational function: need 1..%d numerator and 0..%d denominator coefficients", kMaxCoeffs,
                kMaxCoeffs);
      NEP_CHECK(f->num != nullptr && (f->nden == 0 || f->den != nullptr), NEP_ERR_ARG,
                "rational function: null coefficient array");
      nd.num_off = (int)coef.size();
      nd.nnum = f->nnum;
      for (int i = 0; i < f->nnum; ++i) coef.push_back(c128{f->num[2 * i], f->num[2 * i + 1]});
      nd.den_off = (int)coef.size();
      nd.nden = f->nden;
      for (int i = 0; i < f->nden; ++i) coef.push_back(c128{f->den[2 * i], f->den[2 * i + 1]});
      if (f->nden > 0) {
        bool allzero = true;
        for (int i = 0; i < f->nden; ++i) allzero &= (f->den[2 * i] == 0.0 && f->den[2 * i + 1] == 0.0);
        NEP_CHECK(!allzero, NEP_ERR_ARG, "rational function: zero denominator polynomial");
      }
      break;
    case NEP_FN_EXP:
    case NEP_FN_LOG:
    case NEP_FN_SQRT:
    case NEP_FN_INVSQRT:
      break;
    case NEP_FN_PHI:
      NEP_CHECK(f->phi_k >= 0 && f->phi_k <= 20, NEP_ERR_ARG, "phi_k: k must be in 0..20");
      nd.phi_k = f->phi_k;
      break;
    case NEP_FN_COMBINE: {
      NEP_CHECK(f->comb_op >= NEP_COMB_ADD && f->comb_op <= NEP_COMB_COMPOSE, NEP_ERR_ARG, "bad combine op %d",
                f->comb_op);
      nd.op = f->comb_op;
      int ia, ib;
      NEP_TRY(flatten(f->comb_a, depth + 1, nodes, coef, &ia));
      NEP_TRY(flatten(f->comb_b, depth + 1, nodes, coef, &ib));
      nd.a = ia;
      nd.b = ib;
      break;
    }
    default:
      NEP_CHECK(false, NEP_ERR_ARG, "unknown function type %d", f->type);
  }
  *out_index = (int)nodes.size();
  nodes.push_back(nd);
  return NEP_OK;
}

hipError_t to_rowmajor(const void* in, long long ld, int n, int cplx, void* out, hipStream_t st);
hipError_t inf_norm(const void* A, int n, int cplx, unsigned long long* scratch, double* out, hipStream_t st);
hipError_t fn_points(const FnNode* nodes, const c128* coef, const int* roots, int ell, const c128* z, int m,
                     c128* out, int* bad, hipStream_t st);

// Low-rank detection of a real n x n term (column-major h, leading dimension
// ld), by a randomized range finder: Y = A Omega with k = rmax + 8 Gaussian
// columns, Householder QR of Y, numerical rank r from R's diagonal, Q_r, and
// H = A^T Q_r, so that A ~ Q_r H^T.  The factorization is kept only if four
// random probes z give ||A z - Q_r (H^T z)|| <= sqrt(n) u ||A||_F ||z||
// (u = 2^-53): no larger than the typical rounding error of the dense FP64
// product A z itself, which the probe's reference value also carries.
// Returns r (0: not low rank); G = Q_r and H are n x r row-major.
static void par_for(int n, const std::function<void(int, int)>& body) {
  const int nt = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  const int chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int a = t * chunk, b = std::min(n, a + chunk);
    if (a < b) th.emplace_back(body, a, b);
  }
  for (auto& x : th) x.join();
}

static int detect_low_rank(int n, const double* h, long long ld, int rmax, std::vector<double>& G,
                           std::vector<double>& H) {
  const int k = rmax + 8;
  if (n < 4 * k) return 0;
  std::mt19937_64 gen(12345);
  std::normal_distribution<double> nd;
  std::vector<double> Om((size_t)n * k);  // row c: Omega[c][0..k)
  for (auto& x : Om) x = nd(gen);
  std::vector<double> Y((size_t)k * n, 0.0);  // column j of Y at Y[j*n]
  par_for(n, [&](int r0, int r1) {
    for (int c = 0; c < n; ++c) {
      const double* a = h + (long long)c * ld;
      const double* om = &Om[(size_t)c * k];
      for (int j = 0; j < k; ++j) {
        const double w = om[j];
        double* y = &Y[(size_t)j * n];
        for (int r = r0; r < r1; ++r) y[r] += a[r] * w;
      }
    }
  });
  // Householder QR of Y (n x k), reflectors kept in place
  std::vector<double> tau(k, 0.0), diag(k, 0.0);
  for (int j = 0; j < k; ++j) {
    double* x = &Y[(size_t)j * n];
    double s2 = 0.0;
    for (int r = j + 1; r < n; ++r) s2 += x[r] * x[r];
    const double alpha = x[j];
    const double nrm = std::sqrt(alpha * alpha + s2);
    if (nrm == 0.0) { diag[j] = 0.0; continue; }
    const double beta = alpha >= 0.0 ? -nrm : nrm;
    tau[j] = (beta - alpha) / beta;
    const double scal = 1.0 / (alpha - beta);
    for (int r = j + 1; r < n; ++r) x[r] *= scal;
    x[j] = beta;
    diag[j] = std::fabs(beta);
    for (int jj = j + 1; jj < k; ++jj) {
      double* b = &Y[(size_t)jj * n];
      double w = b[j];
      for (int r = j + 1; r < n; ++r) w += x[r] * b[r];
      w *= tau[j];
      b[j] -= w;
      for (int r = j + 1; r < n; ++r) b[r] -= x[r] * w;
    }
  }
  int rk = 0;
  while (rk < k && diag[rk] > 1e-11 * diag[0]) ++rk;
  if (rk == 0 || rk > rmax) return 0;
  // Q_r = H_0 ... H_{k-1} applied to the first rk unit columns
  std::vector<double> Q((size_t)rk * n, 0.0);
  for (int j = 0; j < rk; ++j) {
    double* q = &Q[(size_t)j * n];
    q[j] = 1.0;
    for (int i = k - 1; i >= 0; --i) {
      if (tau[i] == 0.0) continue;
      const double* v = &Y[(size_t)i * n];
      double w = q[i];
      for (int r = i + 1; r < n; ++r) w += v[r] * q[r];
      w *= tau[i];
      q[i] -= w;
      for (int r = i + 1; r < n; ++r) q[r] -= v[r] * w;
    }
  }
  // H = A^T Q_r: H[c][j] = column c of A against q_j
  H.assign((size_t)n * rk, 0.0);
  par_for(n, [&](int c0, int c1) {
    for (int c = c0; c < c1; ++c) {
      const double* a = h + (long long)c * ld;
      for (int j = 0; j < rk; ++j) {
        const double* q = &Q[(size_t)j * n];
        double d = 0.0;
        for (int r = 0; r < n; ++r) d += a[r] * q[r];
        H[(size_t)c * rk + j] = d;
      }
    }
  });
  // a posteriori check with random probes
  double fro2 = 0.0;
  for (int c = 0; c < n; ++c)
    for (int r = 0; r < n; ++r) fro2 += h[(long long)c * ld + r] * h[(long long)c * ld + r];
  const double fro = std::sqrt(fro2);
  std::vector<double> z(n), az(n), hz(rk);
  for (int t = 0; t < 4; ++t) {
    double zn = 0.0;
    for (auto& x : z) { x = nd(gen); zn += x * x; }
    zn = std::sqrt(zn);
    std::fill(az.begin(), az.end(), 0.0);
    for (int c = 0; c < n; ++c) {
      const double* a = h + (long long)c * ld;
      for (int r = 0; r < n; ++r) az[r] += a[r] * z[c];
    }
    for (int j = 0; j < rk; ++j) {
      double d = 0.0;
      for (int c = 0; c < n; ++c) d += H[(size_t)c * rk + j] * z[c];
      hz[j] = d;
    }
    double e2 = 0.0;
    for (int r = 0; r < n; ++r) {
      double g = 0.0;
      for (int j = 0; j < rk; ++j) g += Q[(size_t)j * n + r] * hz[j];
      e2 += (az[r] - g) * (az[r] - g);
    }
    if (!(std::sqrt(e2) <= std::sqrt((double)n) * 0x1p-53 * fro * zn)) return 0;
  }
  G.assign((size_t)n * rk, 0.0);
  for (int j = 0; j < rk; ++j)
    for (int r = 0; r < n; ++r) G[(size_t)r * rk + j] = Q[(size_t)j * n + r];
  return rk;
}

nep_status Split::init(int n_, int ell_, const nep_mat* A, const nep_fn* f, hipStream_t st) {
  stream = st;
  op.n = n_;
  op.ell = ell_;
  NEP_TRY(configure_kernels());
  // functions
  std::vector<FnNode> nodes;
  std::vector<c128> coef;
  for (int i = 0; i < ell_; ++i) NEP_TRY(flatten(&f[i], 1, nodes, coef, &op.fn_root[i]));
  if (coef.empty()) coef.push_back(c128{0.0, 0.0});
  NEP_TRY(fn_nodes.alloc(sizeof(FnNode) * nodes.size()));
  NEP_TRY(fn_coef.alloc(sizeof(c128) * coef.size()));
  NEP_TRY(fn_roots.alloc(sizeof(int) * kMaxTerms));
  // uploads on the handle's stream, which the end of creation waits for: an
  // upload through the null stream is not ordered before work on a
  // non-blocking stream
  NEP_HIP(hipMemcpyAsync(fn_nodes.p, nodes.data(), sizeof(FnNode) * nodes.size(), hipMemcpyHostToDevice, stream));
  NEP_HIP(hipMemcpyAsync(fn_coef.p, coef.data(), sizeof(c128) * coef.size(), hipMemcpyHostToDevice, stream));
  NEP_HIP(hipMemcpyAsync(fn_roots.p, op.fn_root, sizeof(int) * kMaxTerms, hipMemcpyHostToDevice, stream));
  op.dfn_nodes = fn_nodes.as<FnNode>();
  op.dfn_coef = fn_coef.as<c128>();
  h_fn_nodes = nodes;
  h_fn_coef = coef;
  // matrices: upload column-major, convert to row-major on the device
  NEP_TRY(norms.alloc(sizeof(double) * kMaxTerms + sizeof(unsigned long long) * 2));
  op.dnormA = norms.as<double>();
  unsigned long long* scratch = reinterpret_cast<unsigned long long*>(norms.as<char>() + sizeof(double) * kMaxTerms);
  op.a_cplx = 0;
  for (int i = 0; i < ell_; ++i) {
    const int cplx = A[i].type == NEP_MAT_COMPLEX_F64;
    op.is_cplx[i] = cplx;
    op.a_cplx |= cplx;
    const size_t words = cplx ? 2 : 1;
    const size_t bytes = (size_t)n_ * n_ * words * sizeof(double);
    mats[i] = std::make_unique<DevMem>();
    NEP_TRY(mats[i]->alloc(bytes));
    const void* src = A[i].data;
    DevMem staging;
    if (!A[i].on_device) {
      NEP_TRY(staging.alloc((size_t)A[i].ld * n_ * words * sizeof(double)));
      NEP_HIP(hipMemcpyAsync(staging.p, A[i].data, (size_t)A[i].ld * n_ * words * sizeof(double),
                             hipMemcpyHostToDevice, stream));
      src = staging.p;
    }
    NEP_HIP(to_rowmajor(src, A[i].ld, n_, cplx, mats[i]->p, stream));
    if (!A[i].on_device) {  // diagonal terms skip the dense residual product
      const double* h = static_cast<const double*>(A[i].data);
      bool diag = true;
      for (long long c = 0; c < n_ && diag; ++c)
        for (long long r = 0; r < n_; ++r) {
          if (r == c) continue;
          const double* e = h + (r + c * A[i].ld) * words;
          if (e[0] != 0.0 || (cplx && e[1] != 0.0)) {
            diag = false;
            break;
          }
        }
      if (diag) {
        std::vector<c128> dv(n_);
        for (long long r = 0; r < n_; ++r) {
          const double* e = h + (r + r * A[i].ld) * words;
          dv[r] = c128{e[0], cplx ? e[1] : 0.0};
        }
        diags[i] = std::make_unique<DevMem>();
        NEP_TRY(diags[i]->alloc(sizeof(c128) * n_));
        NEP_HIP(hipMemcpyAsync(diags[i]->p, dv.data(), sizeof(c128) * n_, hipMemcpyHostToDevice, stream));
        op.is_diag[i] = 1;
        op.dDiag[i] = diags[i]->as<c128>();
      }
      if (!diag && !cplx) {  // real banded terms: the residual runs over their band only
        long long w = 0;
        for (long long c = 0; c < n_ && w <= kBandMax; ++c)
          for (long long r = 0; r < n_; ++r) {
            const long long d = r > c ? r - c : c - r;
            if (d > w && h[r + c * A[i].ld] != 0.0) w = d;
          }
        if (w >= 1 && w <= kBandMax) {
          op.band_w[i] = (int)w;
        } else if (w > kBandMax) {  // real low-rank terms: the residual applies G (H^T y)
          std::vector<double> hG, hH;
          const int rk = detect_low_rank(n_, h, A[i].ld, std::min(kLowRankMax, n_ / 8), hG, hH);
          if (rk > 0) {
            lrG[i] = std::make_unique<DevMem>();
            lrH[i] = std::make_unique<DevMem>();
            NEP_TRY(lrG[i]->alloc(sizeof(double) * hG.size()));
            NEP_TRY(lrH[i]->alloc(sizeof(double) * hH.size()));
            NEP_HIP(hipMemcpyAsync(lrG[i]->p, hG.data(), sizeof(double) * hG.size(), hipMemcpyHostToDevice, stream));
            NEP_HIP(hipMemcpyAsync(lrH[i]->p, hH.data(), sizeof(double) * hH.size(), hipMemcpyHostToDevice, stream));
            op.lr_rank[i] = rk;
            op.dLrG[i] = lrG[i]->as<double>();
            op.dLrH[i] = lrH[i]->as<double>();
          }
        }
      }
    }
    NEP_HIP(inf_norm(mats[i]->p, n_, cplx, scratch, norms.as<double>() + i, stream));
    NEP_HIP(hipStreamSynchronize(stream));  // staging is released at scope end
    op.dA[i] = mats[i]->p;
  }
  op.normA.assign(ell_, 0.0);
  NEP_HIP(hipMemcpyAsync(op.normA.data(), op.dnormA, sizeof(double) * ell_, hipMemcpyDeviceToHost, stream));
  NEP_HIP(hipStreamSynchronize(stream));
  return NEP_OK;
}

hipError_t fn_points_d(const FnNode* nodes, const c128* coef, const int* roots, int ell, const c128* z, int m,
                       c128* out, int* bad, hipStream_t st);

hipError_t adjoint_copy(const void* src, int n, int cplx, void* dst, hipStream_t st);
hipError_t conj_copy(const c128* src, int n, c128* dst, hipStream_t st);

Split::~Split() {
  if (adj) {
    nep_split a = adj;
    adj = nullptr;
    (void)nep_split_destroy(&a);
  }
}

nep_status Split::init_adjoint(const Split& src) {
  stream = src.stream;
  op.n = src.op.n;
  op.ell = src.op.ell;
  // f^*(z) = conj(f(conj z)) = conj(beta) g^*(conj(alpha) z), g^* the same
  // function with conjugated coefficients (exp, log, sqrt, 1/sqrt and phi_k
  // have real coefficients and cuts symmetric about the real axis)
  h_fn_nodes = src.h_fn_nodes;
  h_fn_coef = src.h_fn_coef;
  for (auto& nd : h_fn_nodes) {
    nd.alpha.im = -nd.alpha.im;
    nd.beta.im = -nd.beta.im;
  }
  for (auto& c : h_fn_coef) c.im = -c.im;
  NEP_TRY(fn_nodes.alloc(sizeof(FnNode) * h_fn_nodes.size()));
  NEP_TRY(fn_coef.alloc(sizeof(c128) * h_fn_coef.size()));
  NEP_TRY(fn_roots.alloc(sizeof(int) * kMaxTerms));
  NEP_HIP(hipMemcpyAsync(fn_nodes.p, h_fn_nodes.data(), sizeof(FnNode) * h_fn_nodes.size(), hipMemcpyHostToDevice,
                         stream));
  NEP_HIP(hipMemcpyAsync(fn_coef.p, h_fn_coef.data(), sizeof(c128) * h_fn_coef.size(), hipMemcpyHostToDevice,
                         stream));
  for (int i = 0; i < kMaxTerms; ++i) op.fn_root[i] = src.op.fn_root[i];
  NEP_HIP(hipMemcpyAsync(fn_roots.p, op.fn_root, sizeof(int) * kMaxTerms, hipMemcpyHostToDevice, stream));
  op.dfn_nodes = fn_nodes.as<FnNode>();
  op.dfn_coef = fn_coef.as<c128>();
  NEP_TRY(norms.alloc(sizeof(double) * kMaxTerms + sizeof(unsigned long long) * 2));
  op.dnormA = norms.as<double>();
  unsigned long long* scratch = reinterpret_cast<unsigned long long*>(norms.as<char>() + sizeof(double) * kMaxTerms);
  op.a_cplx = src.op.a_cplx;
  const int n = op.n;
  for (int i = 0; i < op.ell; ++i) {
    const int cplx = src.op.is_cplx[i];
    op.is_cplx[i] = cplx;
    mats[i] = std::make_unique<DevMem>();
    NEP_TRY(mats[i]->alloc((size_t)n * n * (cplx ? 2 : 1) * sizeof(double)));
    NEP_HIP(adjoint_copy(src.op.dA[i], n, cplx, mats[i]->p, stream));
    if (src.op.is_diag[i]) {
      diags[i] = std::make_unique<DevMem>();
      NEP_TRY(diags[i]->alloc(sizeof(c128) * n));
      NEP_HIP(conj_copy(src.op.dDiag[i], n, diags[i]->as<c128>(), stream));
      op.is_diag[i] = 1;
      op.dDiag[i] = diags[i]->as<c128>();
    }
    NEP_HIP(inf_norm(mats[i]->p, n, cplx, scratch, norms.as<double>() + i, stream));
    NEP_HIP(hipStreamSynchronize(stream));
    op.dA[i] = mats[i]->p;
  }
  op.normA.assign(op.ell, 0.0);
  NEP_HIP(hipMemcpyAsync(op.normA.data(), op.dnormA, sizeof(double) * op.ell, hipMemcpyDeviceToHost, stream));
  NEP_HIP(hipStreamSynchronize(stream));
  return NEP_OK;
}

nep_status Split::eval_fns(int m, const c128* zh, std::vector<c128>& out, std::vector<int>& bad, bool deriv) {
  DevMem dz, dout, dbad;
  NEP_TRY(dz.alloc(sizeof(c128) * m));
  NEP_TRY(dout.alloc(sizeof(c128) * m * op.ell));
  NEP_TRY(dbad.alloc(sizeof(int) * m));
  NEP_HIP(hipMemcpyAsync(dz.p, zh, sizeof(c128) * m, hipMemcpyHostToDevice, stream));
  if (deriv)
    NEP_HIP(fn_points_d(op.dfn_nodes, op.dfn_coef, fn_roots.as<int>(), op.ell, dz.as<c128>(), m, dout.as<c128>(),
                        dbad.as<int>(), stream));
  else
    NEP_HIP(fn_points(op.dfn_nodes, op.dfn_coef, fn_roots.as<int>(), op.ell, dz.as<c128>(), m, dout.as<c128>(),
                      dbad.as<int>(), stream));
  out.resize((size_t)m * op.ell);
  bad.resize(m);
  NEP_HIP(hipMemcpyAsync(out.data(), dout.p, sizeof(c128) * m * op.ell, hipMemcpyDeviceToHost, stream));
  NEP_HIP(hipMemcpyAsync(bad.data(), dbad.p, sizeof(int) * m, hipMemcpyDeviceToHost, stream));
  NEP_HIP(hipStreamSynchronize(stream));
  return NEP_OK;
}

nep_status check_contour(const nep_contour* g) {
  NEP_CHECK(g != nullptr, NEP_ERR_ARG, "null contour");
  NEP_CHECK(g->kind == 0 || g->kind == 1, NEP_ERR_ARG, "contour kind must be 0 (circle) or 1 (ellipse)");
  NEP_CHECK(g->rho > 0.0 && std::isfinite(g->rho), NEP_ERR_ARG, "contour radius must be positive");
  NEP_CHECK(g->kind == 0 || (g->v > 0.0 && std::isfinite(g->v)), NEP_ERR_ARG, "ellipse ratio v must be positive");
  NEP_CHECK(std::isfinite(g->c[0]) && std::isfinite(g->c[1]), NEP_ERR_ARG, "contour centre must be finite");
  return NEP_OK;
}

nep_status check_opts(const nep_ciss_opts* o, PlanOptions& po) {
  NEP_CHECK(o != nullptr, NEP_ERR_ARG, "null options");
  NEP_CHECK(o->N >= 2 && o->N <= 1024, NEP_ERR_ARG, "N must be in 2..1024");
  NEP_CHECK(o->L >= 1 && o->L <= 64, NEP_ERR_ARG, "L must be in 1..64");
  NEP_CHECK(o->K >= 1 && 2 * o->K <= kMaxMoments, NEP_ERR_ARG, "K must be in 1..%d", kMaxMoments / 2);
  NEP_CHECK(2 * o->K - 1 <= o->N - 1, NEP_ERR_ARG, "need 2K-1 <= N-1 (moments beyond the trapezoid's exactness)");
  NEP_CHECK(o->prec == NEP_PREC_FP64 || o->prec == NEP_PREC_C32_IR64, NEP_ERR_ARG, "unknown precision %d", o->prec);
  NEP_CHECK(o->max_refine >= 0 && o->max_refine <= 20, NEP_ERR_ARG, "max_refine must be in 0..20");
  NEP_CHECK(o->refine_tol >= 0.0, NEP_ERR_ARG, "refine_tol must be >= 0");
  po.N = o->N;
  po.L = o->L;
  po.K = o->K;
  po.prec = o->prec;
  po.max_refine = o->max_refine;
  po.fallback = o->fp64_fallback ? 1 : 0;
  po.tol = o->refine_tol > 0.0 ? o->refine_tol : kDefaultRefineTol;
  return NEP_OK;
}

nep_status Split::moments(const nep_contour* g, const nep_ciss_opts* o, const void* V, void* S,
                          nep_ciss_stats* st, long long s_stride) {
  NEP_TRY(check_contour(g));
  PlanOptions po;
  NEP_TRY(check_opts(o, po));
  NEP_CHECK(V != nullptr && S != nullptr, NEP_ERR_ARG, "null V or S");
  NEP_CHECK(s_stride == 0 || s_stride >= (long long)op.n * po.L, NEP_ERR_ARG, "moment stride below n*L");
  hipStream_t s = o->stream ? (hipStream_t)o->stream : stream;
  std::vector<PlanProblem> probs{PlanProblem{&op, *g, (const c128*)V, (c128*)S, nullptr, s_stride}};
  last_g = *g;
  if (!plan || !plan->matches(probs, po) || plan->opt.max_refine != po.max_refine ||
      plan->opt.fallback != po.fallback) {
    plan = std::make_unique<MomentsPlan>();
    nep_status bs = plan->build(probs, po, s);
    if (bs == NEP_OK) bs = tune_plan(*plan, s);
    if (bs != NEP_OK) {
      plan.reset();
      return bs;
    }
  } else {
    plan->opt.tol = po.tol;
    NEP_TRY(plan->rebind(probs, s));
  }
  last_stream = s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (st) {
    NEP_HIP(hipEventCreate(&e0));
    NEP_HIP(hipEventCreate(&e1));
    NEP_HIP(hipEventRecord(e0, s));
  }
  nep_status rs = plan->enqueue(s, true);
  if (rs != NEP_OK) return rs;
  pending = true;
  if (!st) return NEP_OK;
  NEP_HIP(hipEventRecord(e1, s));
  nep_status ws = wait(st);
  float ms = 0.f;
  if (hipEventSynchronize(e1) == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  st->ms_total = ms;
  return ws;
}

nep_status Split::moments_more(const void* V, void* S, long long s_stride, void* strm, nep_ciss_stats* st) {
  NEP_CHECK(plan != nullptr, NEP_ERR_ARG, "no resident factors: call nep_ciss_moments on this handle first");
  NEP_CHECK(!pending, NEP_ERR_ARG, "the last moments call on this handle has not been waited for");
  NEP_CHECK(V != nullptr && S != nullptr, NEP_ERR_ARG, "null V or S");
  NEP_CHECK(s_stride == 0 || s_stride >= (long long)op.n * plan->opt.L, NEP_ERR_ARG, "moment stride below n*L");
  hipStream_t s = strm ? (hipStream_t)strm : (last_stream ? last_stream : stream);
  std::vector<PlanProblem> probs{PlanProblem{&op, last_g, (const c128*)V, (c128*)S, nullptr, s_stride}};
  NEP_TRY(plan->rebind(probs, s));
  last_stream = s;
  NEP_TRY(plan->enqueue(s, true, false));
  pending = true;
  if (!st) return NEP_OK;
  return wait(st);
}

unsigned long long Split::next_uid() {
  static std::atomic<unsigned long long> counter{1};
  return counter.fetch_add(1);
}

void winding_count(const std::vector<double>& arg, int* count, double* max_step, double* winding) {
  const int N = (int)arg.size();
  double tot = 0.0, mx = 0.0;
  for (int j = 0; j < N; ++j) {
    const double d = std::remainder(arg[(j + 1) % N] - arg[j], 2.0 * M_PI);
    tot += d;
    mx = std::max(mx, std::fabs(d));
  }
  const double w = tot / (2.0 * M_PI);
  if (count) *count = (int)std::lround(w);
  if (max_step) *max_step = mx;
  if (winding) *winding = w;
}

nep_status Split::wait(nep_ciss_stats* st) {
  NEP_CHECK(plan != nullptr && pending, NEP_ERR_ARG, "no moments call pending on this handle");
  RunResult rr;
  nep_status s = plan->finish(last_stream, rr, true);
  pending = false;
  if (st && !rr.stats.empty()) *st = rr.stats[0];
  return s;
}

}  // namespace nep

using namespace nep;

extern "C" {

const char* nep_last_error(void) { return nep::last_error(); }
const char* nep_version(void) { return "libnep 0.1 (gfx950)"; }

nep_status nep_split_create(int n, int ell, const nep_mat* A, const nep_fn* f, void* stream, nep_split* out) {
  NEP_CHECK(out != nullptr, NEP_ERR_ARG, "null output handle");
  *out = nullptr;
  NEP_CHECK(n >= 1 && n <= 4096, NEP_ERR_ARG, "n must be in 1..4096");
  NEP_CHECK(ell >= 1 && ell <= kMaxTerms, NEP_ERR_ARG, "ell must be in 1..%d", kMaxTerms);
  NEP_CHECK(A != nullptr && f != nullptr, NEP_ERR_ARG, "null matrix or function array");
  for (int i = 0; i < ell; ++i) {
    NEP_CHECK(A[i].type == NEP_MAT_REAL_F64 || A[i].type == NEP_MAT_COMPLEX_F64, NEP_ERR_ARG,
              "matrix %d: unknown type %d", i, A[i].type);
    NEP_CHECK(A[i].data != nullptr, NEP_ERR_ARG, "matrix %d: null data", i);
    NEP_CHECK(A[i].ld >= n, NEP_ERR_ARG, "matrix %d: ld < n", i);
  }
  auto h = std::make_unique<nep_split_s>();
  nep_status s = h->impl.init(n, ell, A, f, (hipStream_t)stream);
  if (s != NEP_OK) return s;
  *out = h.release();
  return NEP_OK;
}

nep_status nep_split_destroy(nep_split* h) {
  NEP_CHECK(h != nullptr, NEP_ERR_ARG, "null handle pointer");
  if (*h) {
    (void)hipStreamSynchronize((*h)->impl.stream);
    delete *h;
  }
  *h = nullptr;
  return NEP_OK;
}

nep_status nep_split_info(nep_split h, int* n, int* ell) {
  NEP_CHECK(h != nullptr, NEP_ERR_ARG, "null handle");
  if (n) *n = h->impl.op.n;
  if (ell) *ell = h->impl.op.ell;
  return NEP_OK;
}

nep_status nep_ciss_moments(nep_split h, const nep_contour* g, const nep_ciss_opts* o, const void* V, void* S,
                            nep_ciss_stats* st) {
  NEP_CHECK(h != nullptr, NEP_ERR_ARG, "null handle");
  return h->impl.moments(g, o, V, S, st);
}

nep_status nep_ciss_wait(nep_split h, nep_ciss_stats* st) {
  NEP_CHECK(h != nullptr, NEP_ERR_ARG, "null handle");
  return h->impl.wait(st);
}

nep_status nep_fn_eval_derivative(nep_split h, int m, const double* z, double* out) {
  NEP_CHECK(h != nullptr, NEP_ERR_ARG, "null handle");
  NEP_CHECK(m >= 1 && z != nullptr && out != nullptr, NEP_ERR_ARG, "bad point arrays");
  std::vector<c128> vals;
  std::vector<int> bad;
  NEP_TRY(h->impl.eval_fns(m, reinterpret_cast<const c128*>(z), vals, bad, true));
  std::memcpy(out, vals.data(), sizeof(c128) * vals.size());
  for (int k = 0; k < m; ++k)
    NEP_CHECK(bad[k] == 0, NEP_ERR_NOT_HOLOMORPHIC, "point %d lies on a pole or branch cut of some f_i", k);
  return NEP_OK;
}

nep_status nep_fn_eval(nep_split h, int m, const double* z, double* out) {
  NEP_CHECK(h != nullptr, NEP_ERR_ARG, "null handle");
  NEP_CHECK(m >= 1 && z != nullptr && out != nullptr, NEP_ERR_ARG, "bad point arrays");
  std::vector<c128> vals;
  std::vector<int> bad;
  NEP_TRY(h->impl.eval_fns(m, reinterpret_cast<const c128*>(z), vals, bad, false));
  std::memcpy(out, vals.data(), sizeof(c128) * vals.size());
  for (int k = 0; k < m; ++k)
    NEP_CHECK(bad[k] == 0, NEP_ERR_NOT_HOLOMORPHIC, "point %d lies on a pole or branch cut of some f_i", k);
  return NEP_OK;
}

}  // extern "C"

extern "C" {

nep_status nep_prof_enable(int on) {
  KernelProf& p = kernel_prof();
  for (auto& r : p.recs) {
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  p.recs.clear();
  p.on = on != 0;
  return NEP_OK;
}

nep_status nep_prof_read(int kind, int* launches, double* ms, double* flops) {
  NEP_CHECK(launches && ms && flops, NEP_ERR_ARG, "null output");
  KernelProf& p = kernel_prof();
  int cnt = 0;
  double t = 0.0, f = 0.0;
  for (auto& r : p.recs) {
    if (r.kind != kind) continue;
    NEP_HIP(hipEventSynchronize(r.e1));
    float x = 0.f;
    NEP_HIP(hipEventElapsedTime(&x, r.e0, r.e1));
    t += x;
    f += r.flops;
    ++cnt;
  }
  *launches = cnt;
  *ms = t;
  *flops = f;
  return NEP_OK;
}

}  // extern "C"
