// Host FP64 eigen-solvers (see eigen.cpp).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

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

// The same solve in two phases, for callers that need only some
// eigenvectors.  sym_eigen_reduce: all eigenvalues (w, ascending) and the
// data for the eigenvectors (the Householder reflectors and the
// tridiagonal's eigenvectors); A is not modified.  Returns false if the QR
// sweeps did not converge.
struct SymEig {
  int n = 0, ld = 0;
  std::vector<double> w;          // eigenvalues, ascending
  std::vector<int32_t> row;       // row of Z^T holding the tridiagonal eigenvector of w[c]
  std::vector<double> R, beta;    // reflector k: beta[k], v_k[k+1..n) in R[k * n + ...]
  std::vector<double> zbuf;       // Z^T, n rows of stride ld from zbuf.data() + zoff
  size_t zoff = 0;
  // scratch of sym_eigen_reduce (the working copy of A, the QR rotations);
  // an object reused for later solves keeps its buffers, so the pages are
  // not faulted in again on every call
  std::vector<double> work, rc, rs;
  std::vector<int32_t> rk;
};
bool sym_eigen_reduce(int n, const double* A, SymEig& out, int nthreads = 1);

// Eigenvectors of w[cols[0..k)] into columns 0..k of out (row-major, leading
// dimension ldo >= k): out[r * ldo + q] = component r of the eigenvector of
// w[cols[q]].  Bit-identical for every thread count.
void sym_eigen_vectors(const SymEig& e, int k, const int* cols, double* out, int ldo,
                       int nthreads = 1);

}  // namespace dmrg
