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
//   The reflectors are applied per requested eigenvector, so a caller that
//   keeps only some eigenvectors (the density-matrix truncation) pays for
//   those only.
#include "eigen.h"

#include <immintrin.h>

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

namespace {

// sum_{i in [lo, hi)} a[i] * b[i] in four interleaved partial sums (lane u
// takes i = lo + u mod 4), added as (s0 + s1) + (s2 + s3) + tail: a fixed
// order that the compiler keeps in one vector register.
inline double dot4(const double* a, const double* b, int lo, int hi) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = lo;
  for (; i + 4 <= hi; i += 4) {
    s0 += a[i] * b[i];
    s1 += a[i + 1] * b[i + 1];
    s2 += a[i + 2] * b[i + 2];
    s3 += a[i + 3] * b[i + 3];
  }
  double t = 0.0;
  for (; i < hi; ++i) t += a[i] * b[i];
  return ((s0 + s1) + (s2 + s3)) + t;
}

// Row i of the lower triangle (ai = A + i n), columns [lo, i]: with kUpd the
// rank-2 update a_ij -= u_i w_j + w_i u_j first; with kMv its part of A x
// (row i adds a_ij x_j to acc_i and a_ij x_i to acc_j, j < i; the dot in four
// interleaved partial sums so that the loop stays in vector registers).
template <bool kUpd, bool kMv>
inline void row_pass(double* __restrict__ ai, int i, int lo, const double* __restrict__ u,
                     const double* __restrict__ w, const double* __restrict__ x,
                     double* __restrict__ acc) {
  const double ui = kUpd ? u[i] : 0.0, wi = kUpd ? w[i] : 0.0;
  if (!kMv) {
    for (int j = lo; j <= i; ++j) ai[j] -= ui * w[j] + wi * u[j];
    return;
  }
  const double xi = x[i];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int j = lo;
  for (; j + 4 <= i; j += 4) {
    double a0 = ai[j], a1 = ai[j + 1], a2 = ai[j + 2], a3 = ai[j + 3];
    if (kUpd) {
      a0 -= ui * w[j] + wi * u[j];
      a1 -= ui * w[j + 1] + wi * u[j + 1];
      a2 -= ui * w[j + 2] + wi * u[j + 2];
      a3 -= ui * w[j + 3] + wi * u[j + 3];
      ai[j] = a0;
      ai[j + 1] = a1;
      ai[j + 2] = a2;
      ai[j + 3] = a3;
    }
    acc[j] += a0 * xi;
    acc[j + 1] += a1 * xi;
    acc[j + 2] += a2 * xi;
    acc[j + 3] += a3 * xi;
    s0 += a0 * x[j];
    s1 += a1 * x[j + 1];
    s2 += a2 * x[j + 2];
    s3 += a3 * x[j + 3];
  }
  double t = 0.0;
  for (; j < i; ++j) {
    double a = ai[j];
    if (kUpd) {
      a -= ui * w[j] + wi * u[j];
      ai[j] = a;
    }
    acc[j] += a * xi;
    t += a * x[j];
  }
  double a = ai[i];
  if (kUpd) {
    a -= ui * w[i] + wi * u[i];
    ai[i] = a;
  }
  acc[i] += (((s0 + s1) + (s2 + s3)) + t) + a * xi;
}

// Rows i and i + 1 of the lower triangle at once (a0 = A + i n, a1 = A +
// (i + 1) n): with kUpd the rank-2 update of both rows first, then their
// part of A x.  Over the columns [lo, i) the two rows share every load of
// u, w, x and acc (AVX2, four columns per step); column i (row i's
// diagonal, row i + 1's last off-diagonal entry) and row i + 1's diagonal
// follow.  Each row's dot is kept in four lanes added as (l0 + l1) +
// (l2 + l3), then the tail, in a fixed order.
template <bool kUpd>
inline void row_pass2(double* __restrict__ a0, double* __restrict__ a1, int i, int lo,
                      const double* __restrict__ u, const double* __restrict__ w,
                      const double* __restrict__ x, double* __restrict__ acc) {
  const double u0 = kUpd ? u[i] : 0.0, w0 = kUpd ? w[i] : 0.0;
  const double u1 = kUpd ? u[i + 1] : 0.0, w1 = kUpd ? w[i + 1] : 0.0;
  const double x0 = x[i], x1 = x[i + 1];
  const __m256d vu0 = _mm256_set1_pd(u0), vw0 = _mm256_set1_pd(w0);
  const __m256d vu1 = _mm256_set1_pd(u1), vw1 = _mm256_set1_pd(w1);
  const __m256d vx0 = _mm256_set1_pd(x0), vx1 = _mm256_set1_pd(x1);
  __m256d s0 = _mm256_setzero_pd(), s1 = _mm256_setzero_pd();
  int j = lo;
  for (; j + 4 <= i; j += 4) {
    __m256d A0 = _mm256_loadu_pd(a0 + j), A1 = _mm256_loadu_pd(a1 + j);
    if (kUpd) {
      const __m256d W = _mm256_loadu_pd(w + j), U = _mm256_loadu_pd(u + j);
      A0 = _mm256_fnmadd_pd(vw0, U, _mm256_fnmadd_pd(vu0, W, A0));
      A1 = _mm256_fnmadd_pd(vw1, U, _mm256_fnmadd_pd(vu1, W, A1));
      _mm256_storeu_pd(a0 + j, A0);
      _mm256_storeu_pd(a1 + j, A1);
    }
    const __m256d X = _mm256_loadu_pd(x + j);
    __m256d C = _mm256_loadu_pd(acc + j);
    C = _mm256_fmadd_pd(A1, vx1, _mm256_fmadd_pd(A0, vx0, C));
    _mm256_storeu_pd(acc + j, C);
    s0 = _mm256_fmadd_pd(A0, X, s0);
    s1 = _mm256_fmadd_pd(A1, X, s1);
  }
  double t0 = 0.0, t1 = 0.0;
  for (; j < i; ++j) {
    double b0 = a0[j], b1 = a1[j];
    if (kUpd) {
      b0 = std::fma(-w0, u[j], std::fma(-u0, w[j], b0));
      b1 = std::fma(-w1, u[j], std::fma(-u1, w[j], b1));
      a0[j] = b0;
      a1[j] = b1;
    }
    acc[j] = std::fma(b1, x1, std::fma(b0, x0, acc[j]));
    t0 = std::fma(b0, x[j], t0);
    t1 = std::fma(b1, x[j], t1);
  }
  double d0 = a0[i], e1 = a1[i], d1 = a1[i + 1];
  if (kUpd) {
    d0 = std::fma(-w0, u[i], std::fma(-u0, w[i], d0));
    e1 = std::fma(-w1, u[i], std::fma(-u1, w[i], e1));
    d1 = std::fma(-w1, u[i + 1], std::fma(-u1, w[i + 1], d1));
    a0[i] = d0;
    a1[i] = e1;
    a1[i + 1] = d1;
  }
  alignas(32) double l0[4], l1[4];
  _mm256_store_pd(l0, s0);
  _mm256_store_pd(l1, s1);
  acc[i] += ((((l0[0] + l0[1]) + (l0[2] + l0[3])) + t0) + d0 * x0) + e1 * x1;
  acc[i + 1] += ((((l1[0] + l1[1]) + (l1[2] + l1[3])) + t1) + e1 * x0) + d1 * x1;
}

// Rows [r0, n) of the lower triangle, columns [lo, i] of row i, in pairs
// (row_pass2) and a last single row.
template <bool kUpd>
inline void rows_pass(double* A, int n, int r0, int lo, const double* u, const double* w, const double* x,
                      double* acc) {
  int i = r0;
  for (; i + 1 < n; i += 2)
    row_pass2<kUpd>(A + (size_t)i * n, A + (size_t)(i + 1) * n, i, lo, u, w, x, acc);
  if (i < n) row_pass<kUpd, true>(A + (size_t)i * n, i, lo, u, w, x, acc);
}

}  // namespace

bool sym_eigen_reduce(int n, const double* Ain, SymEig& out, int nthreads) {
  out.n = n;
  out.w.assign(n, 0.0);
  out.row.assign(n, 0);
  out.R.assign((size_t)n * n, 0.0);
  out.beta.assign(n, 0.0);
  if (n <= 0) return true;
  nthreads = std::max(1, std::min(nthreads, (n + 31) / 32));
  std::vector<double>& A = out.work;
  A.assign(Ain, Ain + (size_t)n * n);
  std::vector<double>& R = out.R;
  std::vector<double>& betas = out.beta;
  // 1. Householder reduction to tridiagonal form on the lower triangle.
  //    Reflector k is H_k = I - beta_k v_k v_k^T with v_k[0..k] = 0; its
  //    nonzero part v_k[k+1..n) is kept in R[k][k+1..n).  Step k needs
  //    p = beta_k A v_k over the trailing block and then the rank-2 update
  //    A -= v w^T + w v^T.  Column k+1 is updated first, which fixes
  //    reflector k+1; the rest of the update and the next step's p are then
  //    one pass over the trailing rows instead of two.
  std::vector<double> v(n), v2(n), p(n), p2(n);
  // Reflector of column k: v[k+1..n), beta and the new subdiagonal entry.
  // The column is scaled by its largest entry first: the reflector does not
  // change, and its norm neither underflows nor overflows (the trailing
  // columns of a low-rank density matrix decay towards the underflow
  // threshold).  False if the column is zero below the subdiagonal.
  auto reflector = [&](int k, double* vk, double& beta, double& sub) {
    double scale = 0.0;
    for (int i = k + 1; i < n; ++i) scale = std::max(scale, std::fabs(A[(size_t)i * n + k]));
    if (scale == 0.0) return false;
    double sigma = 0.0;
    for (int i = k + 2; i < n; ++i) {
      vk[i] = A[(size_t)i * n + k] / scale;
      sigma += vk[i] * vk[i];
    }
    if (sigma == 0.0) return false;
    const double x0 = A[(size_t)(k + 1) * n + k] / scale;
    const double norm = std::sqrt(x0 * x0 + sigma);
    const double alpha = x0 <= 0.0 ? norm : -norm;
    vk[k + 1] = x0 - alpha;
    beta = 2.0 / (vk[k + 1] * vk[k + 1] + sigma);
    sub = alpha * scale;
    return true;
  };
  double beta = 0.0, sub = 0.0;
  bool have = false;     // reflector k (v, beta, sub) is known and p holds A v_k
  for (int k = 0; k + 2 < n; ++k) {
    if (!have) {
      if (!reflector(k, v.data(), beta, sub)) continue;
      for (int i = k + 1; i < n; ++i) p[i] = 0.0;
      rows_pass<false>(A.data(), n, k + 1, k + 1, nullptr, nullptr, v.data(), p.data());
    }
    double vtp = 0.0;
    for (int i = k + 1; i < n; ++i) {
      p[i] *= beta;
      vtp += v[i] * p[i];
    }
    const double K = 0.5 * beta * vtp;
    for (int i = k + 1; i < n; ++i) p[i] -= K * v[i];   // p becomes w
    // column k+1 of the trailing block, then reflector k+1 from it
    for (int i = k + 1; i < n; ++i) A[(size_t)i * n + k + 1] -= v[i] * p[k + 1] + p[i] * v[k + 1];
    double beta2 = 0.0, sub2 = 0.0;
    const bool next = k + 3 < n && reflector(k + 1, v2.data(), beta2, sub2);
    if (next) {
      for (int i = k + 2; i < n; ++i) p2[i] = 0.0;
      rows_pass<true>(A.data(), n, k + 2, k + 2, v.data(), p.data(), v2.data(), p2.data());
    } else {
      for (int i = k + 2; i < n; ++i) row_pass<true, false>(&A[(size_t)i * n], i, k + 2, v.data(), p.data(), nullptr, nullptr);
    }
    A[(size_t)(k + 1) * n + k] = sub;
    for (int i = k + 2; i < n; ++i) A[(size_t)i * n + k] = 0.0;
    betas[k] = beta;
    std::copy(v.begin() + k + 1, v.end(), R.begin() + (size_t)k * n + k + 1);
    have = next;
    if (next) {
      std::swap(v, v2);
      std::swap(p, p2);
      beta = beta2;
      sub = sub2;
    }
  }
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];

  // 2. Implicit symmetric QR with Wilkinson shifts on (d, e).  Each rotation
  //    acts on rows k and k+1 of Z^T (columns of the tridiagonal's
  //    eigenvector matrix Z); it is recorded as (k, c, s) and applied in
  //    step 3.
  std::vector<int32_t>& rk = out.rk;
  std::vector<double>& rc = out.rc;
  std::vector<double>& rs = out.rs;
  rk.clear();
  rc.clear();
  rs.clear();
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
  // Rows of Z^T start on 64-byte boundaries with a stride of whole cache
  // lines, so the column ranges of different threads share no line.
  const int ld = (n + 7) / 8 * 8;
  out.ld = ld;
  out.zbuf.assign((size_t)n * ld + 8, 0.0);
  out.zoff = (8 - (reinterpret_cast<uintptr_t>(out.zbuf.data()) / 8) % 8) % 8;
  double* ZT = out.zbuf.data() + out.zoff;
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
  // ascending order of the eigenvalues; row[c] is the row of Z^T of w[c]
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int c = 0; c < n; ++c) {
    out.w[c] = d[idx[c]];
    out.row[c] = idx[c];
  }
  return true;
}

void sym_eigen_vectors(const SymEig& E, int k, const int* cols, double* out, int ldo,
                       int nthreads) {
  const int n = E.n;
  if (n <= 0 || k <= 0) return;
  nthreads = std::max(1, std::min(nthreads, (k + 7) / 8));
  const double* ZT = E.zbuf.data() + E.zoff;
  // 4. Eigenvector of w[c] = H_0 H_1 ... H_{n-3} z, z = row row[c] of Z^T:
  //    the reflectors are applied last to first.  Vectors are independent;
  //    four at a time share each reflector's loads, and threads take
  //    disjoint groups of four.
  const int ngroup = (k + 3) / 4;
  parallel(nthreads, [&](int t) {
    const int per = (ngroup + nthreads - 1) / nthreads;
    const int g0 = std::min(ngroup, t * per), g1 = std::min(ngroup, (t + 1) * per);
    std::vector<double> zb((size_t)4 * n);
    for (int g = g0; g < g1; ++g) {
      const int q0 = 4 * g, nq = std::min(4, k - q0);
      double* z[4];
      for (int q = 0; q < 4; ++q) {
        z[q] = zb.data() + (size_t)q * n;
        const double* src = &ZT[(size_t)E.row[cols[q0 + std::min(q, nq - 1)]] * E.ld];
        std::copy(src, src + n, z[q]);
      }
      for (int kk = n - 3; kk >= 0; --kk) {
        const double b = E.beta[kk];
        if (b == 0.0) continue;
        const double* vk = &E.R[(size_t)kk * n];
        double s[4];
        for (int q = 0; q < 4; ++q) s[q] = b * dot4(vk, z[q], kk + 1, n);
        for (int i = kk + 1; i < n; ++i) {
          const double vi = vk[i];
          z[0][i] -= s[0] * vi;
          z[1][i] -= s[1] * vi;
          z[2][i] -= s[2] * vi;
          z[3][i] -= s[3] * vi;
        }
      }
      for (int q = 0; q < nq; ++q)
        for (int r = 0; r < n; ++r) out[(size_t)r * ldo + q0 + q] = z[q][r];
    }
  });
}

bool sym_eigen(int n, double* A, double* w, int nthreads) {
  if (n <= 0) return true;
  SymEig E;
  if (!sym_eigen_reduce(n, A, E, nthreads)) return false;
  std::vector<int> all(n);
  std::iota(all.begin(), all.end(), 0);
  for (int c = 0; c < n; ++c) w[c] = E.w[c];
  sym_eigen_vectors(E, n, all.data(), A, n, nthreads);
  return true;
}

}  // namespace dmrg
