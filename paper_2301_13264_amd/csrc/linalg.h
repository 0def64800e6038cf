// Small dense host linear algebra for subspace problems (m <= a few hundred):
// LU solve with partial pivoting and a real non-symmetric eigensolver
// (Householder Hessenberg reduction + complex single-shift QR with Wilkinson
// shifts + back substitution on the Schur form).
#pragma once
#include <complex>
#include <vector>

namespace nm {

// Solves A X = B in place (A n x n row-major, B n x nrhs row-major).
// Returns false when A is numerically singular.
bool lu_solve(std::vector<double> A, std::vector<double>& B, int n, int nrhs);

// Eigen-decomposition of a real m x m row-major matrix G.
// w[k] eigenvalues; V[k*m + i] = component i of the right eigenvector k
// (unit 2-norm).  Returns false if QR did not converge.
bool eig_nonsym(const std::vector<double>& G, int m, std::vector<std::complex<double>>& w,
                std::vector<std::complex<double>>& V);

}  // namespace nm
