// Small dense kernels of the extraction (size <= 256), double complex.
// They act on the K*L x K*L triangular factor of the block-Hankel matrix and
// on the m x m projected matrix; the paper likewise solves its small projected
// problems sequentially (Section 5).
#pragma once

#include <complex>
#include <vector>

namespace nep {

using zc = std::complex<double>;

// One-sided Jacobi SVD of a k x k column-major matrix A (overwritten):
// A = U diag(s) W^H, singular values descending.  U, W column-major k x k.
void jacobi_svd(int k, std::vector<zc>& A, std::vector<double>& s, std::vector<zc>& U, std::vector<zc>& W);

// Eigen-decomposition of a general m x m column-major matrix:
// M X = X diag(lam), via Householder-Hessenberg reduction, shifted complex QR
// to Schur form and back substitution.  Returns false if QR did not converge.
bool eig_general(int m, const std::vector<zc>& M, std::vector<zc>& lam, std::vector<zc>& X);

}  // namespace nep
