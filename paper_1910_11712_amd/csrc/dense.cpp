// Small dense linear algebra of the extraction step (host, double complex).
#include "dense.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace nep {

static inline double abs2(zc a) { return a.real() * a.real() + a.imag() * a.imag(); }

// One-sided (Hestenes) Jacobi: rotate column pairs of A until all pairs are
// orthogonal to working precision; then A = U diag(s) and A_orig W = A.
void jacobi_svd(int k, std::vector<zc>& A, std::vector<double>& s, std::vector<zc>& U, std::vector<zc>& W) {
  W.assign((size_t)k * k, zc(0.0, 0.0));
  for (int i = 0; i < k; ++i) W[(size_t)i * k + i] = 1.0;
  const double eps = 1e-15;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < k - 1; ++p) {
      for (int q = p + 1; q < k; ++q) {
        zc* ap = &A[(size_t)p * k];
        zc* aq = &A[(size_t)q * k];
        double alpha = 0.0, beta = 0.0;
        zc gamma(0.0, 0.0);
        for (int i = 0; i < k; ++i) {
          alpha += abs2(ap[i]);
          beta += abs2(aq[i]);
          gamma += std::conj(ap[i]) * aq[i];
        }
        const double g = std::abs(gamma);
        if (g == 0.0 || g <= eps * std::sqrt(alpha * beta)) continue;
        off = std::max(off, g / std::sqrt(alpha * beta));
        const zc d = gamma / g;  // phase of gamma
        // with b = a_q * conj(d), a_p^H b = g is real: real Jacobi rotation
        const double zeta = (beta - alpha) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        for (int i = 0; i < k; ++i) {
          const zc x = ap[i], y = aq[i] * std::conj(d);
          ap[i] = c * x - sn * y;
          aq[i] = sn * x + c * y;
        }
        zc* wp = &W[(size_t)p * k];
        zc* wq = &W[(size_t)q * k];
        for (int i = 0; i < k; ++i) {
          const zc x = wp[i], y = wq[i] * std::conj(d);
          wp[i] = c * x - sn * y;
          wq[i] = sn * x + c * y;
        }
      }
    }
    if (off <= eps) break;
  }
  std::vector<double> sv(k);
  for (int j = 0; j < k; ++j) {
    double nn = 0.0;
    for (int i = 0; i < k; ++i) nn += abs2(A[(size_t)j * k + i]);
    sv[j] = std::sqrt(nn);
  }
  std::vector<int> ord(k);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return sv[a] > sv[b]; });
  s.assign(k, 0.0);
  U.assign((size_t)k * k, zc(0.0, 0.0));
  std::vector<zc> W2((size_t)k * k);
  for (int jj = 0; jj < k; ++jj) {
    const int j = ord[jj];
    s[jj] = sv[j];
    for (int i = 0; i < k; ++i) {
      U[(size_t)jj * k + i] = sv[j] > 0 ? A[(size_t)j * k + i] / sv[j] : zc(0.0, 0.0);
      W2[(size_t)jj * k + i] = W[(size_t)j * k + i];
    }
  }
  W.swap(W2);
}

// ---------------------------------------------------------------------------
// General complex eigenproblem
// ---------------------------------------------------------------------------
#define H_(i, j) H[(size_t)(j) * m + (i)]
#define Z_(i, j) Z[(size_t)(j) * m + (i)]

// complex Givens: returns (c real, s complex) with [c s; -conj(s) c] [a; b] = [r; 0]
static void givens(zc a, zc b, double& c, zc& s, zc& r) {
  const double ab = std::abs(b);
  if (ab == 0.0) {
    c = 1.0;
    s = 0.0;
    r = a;
    return;
  }
  const double aa = std::abs(a);
  if (aa == 0.0) {
    c = 0.0;
    s = std::conj(b) / ab;
    r = ab;
    return;
  }
  const double nrm = std::hypot(aa, ab);
  c = aa / nrm;
  const zc ph = a / aa;
  s = ph * std::conj(b) / nrm;
  r = ph * nrm;
}

bool eig_general(int m, const std::vector<zc>& M, std::vector<zc>& lam, std::vector<zc>& X) {
  std::vector<zc> H(M), Z((size_t)m * m, zc(0.0, 0.0));
  for (int i = 0; i < m; ++i) Z_(i, i) = 1.0;
  // Householder reduction to upper Hessenberg form: H = Q^H M Q
  std::vector<zc> v(m);
  for (int k = 0; k + 2 < m + 0 && k < m - 2; ++k) {
    double nrm2 = 0.0;
    for (int i = k + 1; i < m; ++i) nrm2 += abs2(H_(i, k));
    const double nrm = std::sqrt(nrm2);
    if (nrm == 0.0) continue;
    const zc a = H_(k + 1, k);
    const double aa = std::abs(a);
    const zc ph = aa > 0 ? a / aa : zc(1.0, 0.0);
    // v = x + ph*||x|| e1 ; H_k = I - 2 v v^H / (v^H v)
    for (int i = 0; i < m; ++i) v[i] = 0.0;
    for (int i = k + 1; i < m; ++i) v[i] = H_(i, k);
    v[k + 1] += ph * nrm;
    double vn = 0.0;
    for (int i = k + 1; i < m; ++i) vn += abs2(v[i]);
    if (vn == 0.0) continue;
    const double tau = 2.0 / vn;
    // H <- P H
    for (int j = 0; j < m; ++j) {
      zc w = 0.0;
      for (int i = k + 1; i < m; ++i) w += std::conj(v[i]) * H_(i, j);
      w *= tau;
      for (int i = k + 1; i < m; ++i) H_(i, j) -= v[i] * w;
    }
    // H <- H P, Z <- Z P
    for (int i = 0; i < m; ++i) {
      zc w = 0.0, wz = 0.0;
      for (int j = k + 1; j < m; ++j) {
        w += H_(i, j) * v[j];
        wz += Z_(i, j) * v[j];
      }
      w *= tau;
      wz *= tau;
      for (int j = k + 1; j < m; ++j) {
        H_(i, j) -= w * std::conj(v[j]);
        Z_(i, j) -= wz * std::conj(v[j]);
      }
    }
    for (int i = k + 2; i < m; ++i) H_(i, k) = 0.0;
  }
  // shifted QR (single complex shift, Wilkinson) with deflation
  const double eps = 2.220446049250313e-16;
  int hi = m - 1, iter = 0, total = 0;
  while (hi > 0) {
    int lo = hi;
    while (lo > 0) {
      const double sc = std::abs(H_(lo, lo)) + std::abs(H_(lo - 1, lo - 1));
      if (std::abs(H_(lo, lo - 1)) <= eps * (sc > 0 ? sc : 1.0)) {
        H_(lo, lo - 1) = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {
      --hi;
      iter = 0;
      continue;
    }
    if (++total > 100 * m) return false;
    ++iter;
    // Wilkinson shift from the trailing 2x2 block
    zc mu;
    {
      const zc a = H_(hi - 1, hi - 1), b = H_(hi - 1, hi), c = H_(hi, hi - 1), d = H_(hi, hi);
      const zc tr = a + d, det = a * d - b * c;
      const zc disc = std::sqrt(tr * tr / 4.0 - det);
      const zc l1 = tr / 2.0 + disc, l2 = tr / 2.0 - disc;
      mu = std::abs(l1 - d) < std::abs(l2 - d) ? l1 : l2;
      if (iter % 11 == 10) mu = d + zc(std::abs(H_(hi, hi - 1)), 0.0);  // exceptional shift
    }
    // QR sweep on rows/cols lo..hi: H - mu I = QR, H <- RQ + mu I
    std::vector<double> cs(hi - lo);
    std::vector<zc> ss(hi - lo);
    for (int k = lo; k <= hi; ++k) H_(k, k) -= mu;
    for (int k = lo; k < hi; ++k) {
      double c;
      zc s, r;
      givens(H_(k, k), H_(k + 1, k), c, s, r);
      cs[k - lo] = c;
      ss[k - lo] = s;
      for (int j = k; j < m; ++j) {
        const zc x = H_(k, j), y = H_(k + 1, j);
        H_(k, j) = c * x + s * y;
        H_(k + 1, j) = -std::conj(s) * x + c * y;
      }
    }
    for (int k = lo; k < hi; ++k) {
      const double c = cs[k - lo];
      const zc s = ss[k - lo];
      const int top = 0;
      for (int i = top; i <= std::min(k + 2, hi); ++i) {
        const zc x = H_(i, k), y = H_(i, k + 1);
        H_(i, k) = c * x + std::conj(s) * y;
        H_(i, k + 1) = -s * x + c * y;
      }
      for (int i = 0; i < m; ++i) {
        const zc x = Z_(i, k), y = Z_(i, k + 1);
        Z_(i, k) = c * x + std::conj(s) * y;
        Z_(i, k + 1) = -s * x + c * y;
      }
    }
    for (int k = lo; k <= hi; ++k) H_(k, k) += mu;
  }
  // eigenvectors of the triangular Schur factor, then back-transform
  lam.assign(m, zc(0.0, 0.0));
  for (int i = 0; i < m; ++i) lam[i] = H_(i, i);
  double hnorm = 0.0;
  for (size_t i = 0; i < H.size(); ++i) hnorm = std::max(hnorm, std::abs(H[i]));
  const double small = eps * std::max(hnorm, 1e-300);
  X.assign((size_t)m * m, zc(0.0, 0.0));
  std::vector<zc> y(m);
  for (int k = 0; k < m; ++k) {
    for (int i = 0; i < m; ++i) y[i] = 0.0;
    y[k] = 1.0;
    for (int i = k - 1; i >= 0; --i) {
      zc acc = 0.0;
      for (int j = i + 1; j <= k; ++j) acc += H_(i, j) * y[j];
      zc den = H_(i, i) - lam[k];
      if (std::abs(den) < small) den = small;
      y[i] = -acc / den;
    }
    for (int i = 0; i < m; ++i) {
      zc acc = 0.0;
      for (int j = 0; j <= k; ++j) acc += Z_(i, j) * y[j];
      X[(size_t)k * m + i] = acc;
    }
  }
  return true;
}

#undef H_
#undef Z_

}  // namespace nep
