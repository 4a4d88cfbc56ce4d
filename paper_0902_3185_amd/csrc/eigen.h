// Host FP64 eigen-solvers (see eigen.cpp).
#pragma once

namespace dmrg {

// Lowest eigenpair of the symmetric tridiagonal matrix with diagonal a[0..n)
// and off-diagonal b[0..n-1).  u (length n) is normalised, first nonzero
// component positive.
void tridiag_lowest(int n, const double* a, const double* b, double* theta, double* u);

// All eigenpairs of the dense symmetric n x n row-major matrix A: on return
// w holds the eigenvalues in ascending order and column c of A the
// eigenvector of w[c].  Returns false if the QR sweeps did not converge.
// nthreads host threads share the eigenvector work (capped at one per 32
// rows); the result is bit-identical for every thread count.
bool sym_eigen(int n, double* A, double* w, int nthreads = 1);

}  // namespace dmrg
