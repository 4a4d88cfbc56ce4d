// Host FP64 eigen-solvers for the two small eigenproblems of the method:
//
// * the Lanczos tridiagonal matrix (Sec. 3.3): its lowest eigenvalue by
//   Sturm-sequence bisection and the matching eigenvector by inverse
//   iteration with a pivoted tridiagonal solve;
// * the per-sector density-matrix blocks (Eqs. (2)-(3)): all eigenpairs by
//   Householder reduction to tridiagonal form followed by implicitly shifted
//   QR sweeps with Wilkinson shifts (Golub & Van Loan, Matrix Computations,
//   Sec. 8.3).  The QR sweeps run on the tridiagonal alone and record their
//   rotations; applying those rotations and the Householder reflectors to
//   the eigenvector matrix, the O(n^3) part, is split over host threads.
#include "eigen.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <numeric>
#include <thread>
#include <vector>

namespace dmrg {

namespace {

// Number of eigenvalues of the tridiagonal (a, b) below x (Sturm count).
int sturm_count(int n, const double* a, const double* b, double x) {
  int cnt = 0;
  double q = 1.0;
  const double tiny = 1e-300;
  for (int i = 0; i < n; ++i) {
    const double off = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
    q = (a[i] - x) - (i > 0 ? off / q : 0.0);
    if (q == 0.0) q = -tiny;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// Solve (T - shift I) x = rhs for tridiagonal T by Gaussian elimination with
// partial pivoting (the fill-in is one extra superdiagonal).  rhs overwritten.
void tridiag_solve(int n, const double* a, const double* b, double shift, double* rhs) {
  // row i: sb[i] at column i-1, dg[i] at i, sp[i] at i+1, sp2[i] at i+2 (fill-in)
  std::vector<double> dg(n), sp(n, 0.0), sp2(n, 0.0), sb(n, 0.0);
  for (int i = 0; i < n; ++i) {
    dg[i] = a[i] - shift;
    if (i + 1 < n) sp[i] = b[i];
    if (i > 0) sb[i] = b[i - 1];
  }
  const double eps = std::numeric_limits<double>::epsilon();
  double scale = 0.0;
  for (int i = 0; i < n; ++i) scale = std::max(scale, std::fabs(dg[i]) + std::fabs(sp[i]) + std::fabs(sb[i]));
  if (scale == 0.0) scale = 1.0;
  for (int i = 0; i + 1 < n; ++i) {
    // rows i and i+1; row i+1 has sb[i+1] at column i
    if (std::fabs(sb[i + 1]) > std::fabs(dg[i])) {
      // swap rows i and i+1 (row i+1: [sb, dg, sp] at columns i, i+1, i+2)
      std::swap(dg[i], sb[i + 1]);
      std::swap(sp[i], dg[i + 1]);
      std::swap(sp2[i], sp[i + 1]);
      std::swap(rhs[i], rhs[i + 1]);
    }
    if (dg[i] == 0.0) dg[i] = eps * scale;
    const double f = sb[i + 1] / dg[i];
    sb[i + 1] = 0.0;
    dg[i + 1] -= f * sp[i];
    sp[i + 1] -= f * sp2[i];
    rhs[i + 1] -= f * rhs[i];
  }
  if (dg[n - 1] == 0.0) dg[n - 1] = eps * scale;
  for (int i = n - 1; i >= 0; --i) {
    double s = rhs[i];
    if (i + 1 < n) s -= sp[i] * rhs[i + 1];
    if (i + 2 < n) s -= sp2[i] * rhs[i + 2];
    rhs[i] = s / dg[i];
  }
}

}  // namespace

void tridiag_lowest(int n, const double* a, const double* b, double* theta, double* u) {
  if (n == 1) {
    *theta = a[0];
    u[0] = 1.0;
    return;
  }
  double lo = a[0], hi = a[0];
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  const double eps = std::numeric_limits<double>::epsilon();
  const double scale = std::max(std::fabs(lo), std::fabs(hi));
  for (int it = 0; it < 200 && hi - lo > 2.0 * eps * std::max(scale, 1e-300); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(n, a, b, mid) >= 1)
      hi = mid;
    else
      lo = mid;
  }
  *theta = 0.5 * (lo + hi);
  // inverse iteration
  std::vector<double> x(n);
  for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.001 * (double)((i * 7919) % 101) / 101.0;
  for (int it = 0; it < 3; ++it) {
    tridiag_solve(n, a, b, *theta, x.data());
    double nn = 0.0;
    for (double v : x) nn += v * v;
    nn = std::sqrt(nn);
    if (!(nn > 0.0) || !std::isfinite(nn)) break;
    for (double& v : x) v /= nn;
  }
  // fixed sign: first nonzero component positive
  double sgn = 1.0;
  for (int i = 0; i < n; ++i)
    if (std::fabs(x[i]) > 1e-300) {
      sgn = x[i] > 0 ? 1.0 : -1.0;
      break;
    }
  for (int i = 0; i < n; ++i) u[i] = sgn * x[i];
}

namespace {

// Run body(t) for t in [0, nthreads) on that many threads (the caller's
// thread takes t = 0).
template <class F>
void parallel(int nthreads, F body) {
  if (nthreads <= 1) {
    body(0);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(nthreads - 1);
  for (int t = 1; t < nthreads; ++t) th.emplace_back(body, t);
  body(0);
  for (auto& x : th) x.join();
}

// sqrt(x^2 + z^2) without the cost of std::hypot where the squares can
// neither overflow nor lose precision to underflow.
inline double safe_hypot(double x, double z) {
  const double m = std::max(std::fabs(x), std::fabs(z));
  if (m > 1e-150 && m < 1e150) return std::sqrt(x * x + z * z);
  return std::hypot(x, z);
}


}  // namespace

bool sym_eigen(int n, double* A, double* w, int nthreads) {
  if (n <= 0) return true;
  nthreads = std::max(1, std::min(nthreads, (n + 31) / 32));
  // 1. Householder reduction to tridiagonal form on the lower triangle.
  //    Reflector k is H_k = I - beta_k v_k v_k^T with v_k[0..k] = 0; its
  //    nonzero part v_k[k+1..n) is kept in R[k][k+1..n).
  std::vector<double> R((size_t)n * n, 0.0), betas(n, 0.0);
  std::vector<double> v(n), p(n);
  for (int k = 0; k + 2 < n; ++k) {
    // The column is scaled by its largest entry first: the reflector does
    // not change, and its norm neither underflows nor overflows (the
    // trailing columns of a low-rank density matrix decay towards the
    // underflow threshold).
    double scale = 0.0;
    for (int i = k + 1; i < n; ++i) scale = std::max(scale, std::fabs(A[(size_t)i * n + k]));
    if (scale == 0.0) continue;
    double sigma = 0.0;
    for (int i = k + 2; i < n; ++i) {
      v[i] = A[(size_t)i * n + k] / scale;
      sigma += v[i] * v[i];
    }
    if (sigma == 0.0) continue;
    const double x0 = A[(size_t)(k + 1) * n + k] / scale;
    const double norm = std::sqrt(x0 * x0 + sigma);
    const double alpha = x0 <= 0.0 ? norm : -norm;
    v[k + 1] = x0 - alpha;
    const double beta = 2.0 / (v[k + 1] * v[k + 1] + sigma);
    // p = beta * A v over the trailing block, reading the lower triangle
    // only: row i contributes A[i][j] v[j] to p[i] and A[i][j] v[i] to p[j]
    // for j < i, both along contiguous memory.
    for (int i = k + 1; i < n; ++i) p[i] = 0.0;
    for (int i = k + 1; i < n; ++i) {
      const double* ai = &A[(size_t)i * n];
      const double vi = v[i];
      double s = 0.0;
      for (int j = k + 1; j < i; ++j) {
        s += ai[j] * v[j];
        p[j] += ai[j] * vi;
      }
      p[i] += s + ai[i] * vi;
    }
    double vtp = 0.0;
    for (int i = k + 1; i < n; ++i) {
      p[i] *= beta;
      vtp += v[i] * p[i];
    }
    const double K = 0.5 * beta * vtp;
    for (int i = k + 1; i < n; ++i) p[i] -= K * v[i];   // p becomes w
    for (int i = k + 1; i < n; ++i) {
      double* ai = &A[(size_t)i * n];
      const double vi = v[i], wi = p[i];
      for (int j = k + 1; j <= i; ++j) ai[j] -= vi * p[j] + wi * v[j];
    }
    A[(size_t)(k + 1) * n + k] = alpha * scale;
    for (int i = k + 2; i < n; ++i) A[(size_t)i * n + k] = 0.0;
    betas[k] = beta;
    std::copy(v.begin() + k + 1, v.end(), R.begin() + (size_t)k * n + k + 1);
  }
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];

  // 2. Implicit symmetric QR with Wilkinson shifts on (d, e).  Each rotation
  //    acts on rows k and k+1 of Z^T (columns of the tridiagonal's
  //    eigenvector matrix Z); it is recorded as (k, c, s) and applied in
  //    step 3.
  std::vector<int32_t> rk;
  std::vector<double> rc, rs;
  rk.reserve((size_t)4 * n * n / 2 + 16);
  rc.reserve(rk.capacity());
  rs.reserve(rk.capacity());
  const double eps = std::numeric_limits<double>::epsilon();
  // An off-diagonal entry is dropped once it is below eps relative to its
  // two diagonal neighbours or below eps * ||T|| (the normwise backward
  // error the Householder reduction already commits); the second test keeps
  // rank-deficient blocks, whose null space is pure rounding noise, from
  // iterating on that noise.
  double anorm = 0.0;
  for (int i = 0; i < n; ++i)
    anorm = std::max(anorm, std::fabs(d[i]) + (i > 0 ? std::fabs(e[i - 1]) : 0.0) +
                                (i + 1 < n ? std::fabs(e[i]) : 0.0));
  const double small = eps * anorm;
  auto negligible = [&](int k) {
    const double a = std::fabs(e[k]);
    return a == 0.0 || a <= small || a <= eps * (std::fabs(d[k]) + std::fabs(d[k + 1]));
  };
  int hi = n - 1;
  long iters = 0;
  const long cap = 60L * n + 100;
  while (hi > 0) {
    if (negligible(hi - 1)) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && !negligible(lo - 1)) --lo;
    if (lo > 0) e[lo - 1] = 0.0;
    if (++iters > cap) return false;
    const double aa = d[hi - 1], bb = e[hi - 1], cc = d[hi];
    const double del = 0.5 * (aa - cc);
    const double den = del + (del >= 0.0 ? 1.0 : -1.0) * std::hypot(del, bb);
    const double mu = den != 0.0 ? cc - bb * bb / den : cc - std::fabs(bb);
    double x = d[lo] - mu, z = e[lo], bulge = 0.0;
    for (int k = lo; k < hi; ++k) {
      if (k > lo) {
        x = e[k - 1];
        z = bulge;
      }
      const double r = safe_hypot(x, z);
      double c = 1.0, s = 0.0;
      if (r != 0.0) {
        const double inv = 1.0 / r;
        c = x * inv;
        s = -z * inv;
      }
      if (k > lo) e[k - 1] = r;
      const double a0 = d[k], b0 = e[k], d1 = d[k + 1];
      // M' = R^T M R with R = [[c, s], [-s, c]]
      const double m00 = a0 * c - b0 * s, m01 = a0 * s + b0 * c;
      const double m10 = b0 * c - d1 * s, m11 = b0 * s + d1 * c;
      d[k] = c * m00 - s * m10;
      e[k] = c * m01 - s * m11;
      d[k + 1] = s * m01 + c * m11;
      if (k + 1 < hi) {
        bulge = -s * e[k + 1];
        e[k + 1] = c * e[k + 1];
      }
      rk.push_back(k);
      rc.push_back(c);
      rs.push_back(s);
    }
  }

  // 3. Z^T = (rotations) applied to the identity; the columns r of Z^T are
  //    independent, so threads take disjoint column ranges and every element
  //    sees the same operations in the same order for any thread count.
  // 4. Eigenvectors V = H_0 H_1 ... H_{n-3} Z: column c of Z (row c of Z^T)
  //    gets the reflectors applied last to first; columns are independent.
  // Rows of Z^T start on 64-byte boundaries with a stride of whole cache
  // lines, so the column ranges of different threads share no line.
  const int ld = (n + 7) / 8 * 8;
  std::vector<double> zbuf((size_t)n * ld + 8, 0.0);
  double* ZT = zbuf.data() + ((8 - (reinterpret_cast<uintptr_t>(zbuf.data()) / 8) % 8) % 8);
  for (int i = 0; i < n; ++i) ZT[(size_t)i * ld + i] = 1.0;
  const size_t nrot = rk.size();
  // One thread sweeps the whole width; several threads take one-line strips
  // round robin (strip i to thread i mod nthreads), which keeps each
  // thread's strip in its first-level cache while the rotation list streams.
  const int width = nthreads == 1 ? ld : 8;
  const int nstrip = ld / width;
  parallel(nthreads, [&](int t) {
    for (int st = t; st < nstrip; st += nthreads) {
      const int c0 = st * width, c1 = std::min(n, c0 + width);
      for (size_t q = 0; q < nrot; ++q) {
        const double c = rc[q], s = rs[q];
        double* zk = &ZT[(size_t)rk[q] * ld];
        double* zk1 = zk + ld;
        for (int r = c0; r < c1; ++r) {
          const double a = zk[r], b = zk1[r];
          zk[r] = c * a - s * b;
          zk1[r] = s * a + c * b;
        }
      }
    }
  });
  parallel(nthreads, [&](int t) {
    const int per = (n + nthreads - 1) / nthreads;
    const int r0 = std::min(n, t * per), r1 = std::min(n, (t + 1) * per);
    for (int row = r0; row < r1; ++row) {
      double* z = &ZT[(size_t)row * ld];
      for (int k = n - 3; k >= 0; --k) {
        if (betas[k] == 0.0) continue;
        const double* vk = &R[(size_t)k * n];
        double s = 0.0;
        for (int i = k + 1; i < n; ++i) s += vk[i] * z[i];
        s *= betas[k];
        for (int i = k + 1; i < n; ++i) z[i] -= s * vk[i];
      }
    }
  });
  // sort ascending; eigenvectors as columns of A
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int c = 0; c < n; ++c) {
    w[c] = d[idx[c]];
    const double* q = &ZT[(size_t)idx[c] * ld];
    for (int r = 0; r < n; ++r) A[(size_t)r * n + c] = q[r];
  }
  return true;
}

}  // namespace dmrg
