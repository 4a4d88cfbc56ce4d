// FP64 vector kernels for the Lanczos recursion: several dot products against
// the Krylov basis in one pass, the matching update, norms and combinations.
// Reductions go through fixed-shape partial sums, so results are repeatable.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace dmrg {

namespace {
constexpr int kThreads = 256;
constexpr int kPerThread = 4;
constexpr int kSpan = kThreads * kPerThread;   // elements per block
constexpr int kVecsPerBlock = 8;

__device__ inline double block_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}
}  // namespace

int vec_blocks(int64_t n) { return (int)((n + kSpan - 1) / kSpan); }

// partial[j * nblk + blk]
__global__ __launch_bounds__(kThreads) void multi_dot_partial(const double* __restrict__ V,
                                                              int64_t ldv, int nv,
                                                              const double* __restrict__ w,
                                                              int64_t n,
                                                              double* __restrict__ partial) {
  __shared__ double sh[4];
  const int nblk = gridDim.x;
  const int64_t base = (int64_t)blockIdx.x * kSpan + threadIdx.x;
  double wv[kPerThread];
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int64_t i = base + (int64_t)q * kThreads;
    wv[q] = i < n ? w[i] : 0.0;
  }
  const int j0 = blockIdx.y * kVecsPerBlock;
  for (int j = j0; j < j0 + kVecsPerBlock && j < nv; ++j) {
    const double* Vj = V + (int64_t)j * ldv;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
      const int64_t i = base + (int64_t)q * kThreads;
      if (i < n) s += Vj[i] * wv[q];
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) partial[(int64_t)j * nblk + blockIdx.x] = s;
  }
}

// out[j] = sum over blk of partial[j * nblk + blk]  (one block per j)
__global__ __launch_bounds__(kThreads) void sum_partials(const double* __restrict__ partial,
                                                         int nblk, double* __restrict__ out) {
  __shared__ double sh[4];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kThreads) s += partial[(int64_t)j * nblk + b];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[j] = s;
}

__global__ __launch_bounds__(kThreads) void multi_axpy_partial(double* __restrict__ w,
                                                               const double* __restrict__ V,
                                                               int64_t ldv, int nv,
                                                               const double* __restrict__ h,
                                                               int64_t n,
                                                               double* __restrict__ partial) {
  __shared__ double sh[4];
  const int64_t base = (int64_t)blockIdx.x * kSpan + threadIdx.x;
  double acc[kPerThread];
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int64_t i = base + (int64_t)q * kThreads;
    acc[q] = i < n ? w[i] : 0.0;
  }
  for (int j = 0; j < nv; ++j) {
    const double hj = h[j];
    const double* Vj = V + (int64_t)j * ldv;
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
      const int64_t i = base + (int64_t)q * kThreads;
      if (i < n) acc[q] -= hj * Vj[i];
    }
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int64_t i = base + (int64_t)q * kThreads;
    if (i < n) {
      w[i] = acc[q];
      s += acc[q] * acc[q];
    }
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void combine_kernel(double* __restrict__ out,
                                                           const double* __restrict__ V,
                                                           int64_t ldv, int nv,
                                                           const double* __restrict__ u,
                                                           int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < nv; ++j) s += u[j] * V[(int64_t)j * ldv + i];
  out[i] = s;
}

__global__ __launch_bounds__(kThreads) void normalise_kernel(double* __restrict__ dst,
                                                             const double* __restrict__ src,
                                                             const double* __restrict__ nrm2,
                                                             int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const double nn = nrm2[0];
  const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
  if (i < n) dst[i] = src[i] * inv;
}

__global__ void record_kernel(const double* h1, const double* h2, int j, const double* nrm2,
                              double* ab, int it) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ab[2 * it] = h1[j] + (h2 ? h2[j] : 0.0);
    ab[2 * it + 1] = sqrt(nrm2[0] > 0.0 ? nrm2[0] : 0.0);
  }
}

// ---------------------------------------------------------------------------
// One CGS2 step of the Lanczos recursion in bandwidth-shaped launches:
//   dot     partial sums of V^T w   grid (element chunks) x (groups of kDotG vectors)
//   reduce  h1 = sum of the partials, one wave per basis vector
//   axpy    w -= V h1               grid (element chunks), all basis vectors per thread
//   dot, reduce  h2 = V^T w
//   axpy    w -= V h2 and partial sums of ||w||^2
//   finish  (alpha, beta) and v_next = w / beta
// Partial sums are added in a fixed order by the next launch, so results are
// repeatable; the kernel boundary makes them visible across the chip without
// any cache maintenance inside the kernels.
// ---------------------------------------------------------------------------
constexpr int kLzThreads = 256;
constexpr int kDotPer = 4;                       // elements per thread (dot)
constexpr int kDotSpan = kLzThreads * kDotPer;   // elements per block (dot)
constexpr int kDotG = 8;                         // basis vectors per block (dot)
constexpr int kAxPer = 2;                        // elements per thread (axpy)
constexpr int kAxSpan = kLzThreads * kAxPer;     // elements per block (axpy)

int dot_blocks(int64_t n) { return (int)std::max<int64_t>(1, (n + kDotSpan - 1) / kDotSpan); }
int axpy_blocks(int64_t n) { return (int)std::max<int64_t>(1, (n + kAxSpan - 1) / kAxSpan); }

constexpr int kFusedMaxNv = 64;   // basis size up to which axpy and dot share a pass

size_t lz_partial_size(int64_t n, int nv) {
  const size_t fused = (size_t)std::min(nv, kFusedMaxNv) * (size_t)((n + kLzThreads - 1) / kLzThreads);
  return std::max({(size_t)nv * dot_blocks(n), (size_t)axpy_blocks(n), fused});
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of row[0..cnt) by one wave: lane l adds l, l+64, ... in order, then a
// fixed butterfly.  Every lane returns the total.
__device__ inline double wave_row_sum(const double* row, int cnt) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int b = lane; b < cnt; b += 64) s += row[b];
  return wave_sum(s);
}

// partial[(g0 + g) * gridDim.x + blockIdx.x] = block part of <V_{g0+g}, w>,
// g < kDotG; blockIdx.y selects g0.
__global__ __launch_bounds__(kLzThreads) void lz_dot(const double* __restrict__ V, int64_t ldv,
                                                     int nv, const double* __restrict__ w,
                                                     int64_t n, double* __restrict__ partial) {
  __shared__ double sh[kLzThreads / 64][kDotG];
  const int nbx = gridDim.x;
  const int g0 = blockIdx.y * kDotG;
  const int ng = min(kDotG, nv - g0);
  const int64_t start = (int64_t)blockIdx.x * kDotSpan;
  const int64_t base = start + threadIdx.x;
  const bool full = start + kDotSpan <= n;
  double x[kDotPer];
  double s[kDotG];
#pragma unroll
  for (int q = 0; q < kDotPer; ++q) {
    const int64_t i = base + (int64_t)q * kLzThreads;
    x[q] = (full || i < n) ? w[i] : 0.0;
  }
  if (ng == kDotG && full) {
#pragma unroll
    for (int g = 0; g < kDotG; ++g) {
      const double* Vg = V + (int64_t)(g0 + g) * ldv + base;
      double a = 0.0;
#pragma unroll
      for (int q = 0; q < kDotPer; ++q) a += Vg[(int64_t)q * kLzThreads] * x[q];
      s[g] = a;
    }
  } else {
#pragma unroll
    for (int g = 0; g < kDotG; ++g) {
      double a = 0.0;
      if (g < ng) {
        const double* Vg = V + (int64_t)(g0 + g) * ldv;
#pragma unroll
        for (int q = 0; q < kDotPer; ++q) {
          const int64_t i = base + (int64_t)q * kLzThreads;
          if (i < n) a += Vg[i] * x[q];
        }
      }
      s[g] = a;
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int g = 0; g < kDotG; ++g) {
    const double t = wave_sum(s[g]);
    if (lane == 0) sh[wave][g] = t;
  }
  __syncthreads();
  if (threadIdx.x < ng) {
    const int g = threadIdx.x;
    partial[(int64_t)(g0 + g) * nbx + blockIdx.x] = ((sh[0][g] + sh[1][g]) + sh[2][g]) + sh[3][g];
  }
}

// h[i] = sum_b partial[i * nbx + b]: one 64-thread block per basis vector.
__global__ __launch_bounds__(64) void lz_reduce(const double* __restrict__ partial, int nbx,
                                                double* __restrict__ h) {
  const double t = wave_row_sum(partial + (int64_t)blockIdx.x * nbx, nbx);
  if (threadIdx.x == 0) h[blockIdx.x] = t;
}

// w -= sum_{i<nv} h[i] V_i.  With kNorm, also partial[blockIdx.x] = the
// block's part of ||w||^2.
template <bool kNorm>
__global__ __launch_bounds__(kLzThreads) void lz_axpy(double* __restrict__ w,
                                                      const double* __restrict__ V, int64_t ldv,
                                                      int nv, int64_t n,
                                                      const double* __restrict__ h,
                                                      double* __restrict__ partial) {
  const int64_t start = (int64_t)blockIdx.x * kAxSpan;
  const int64_t base = start + threadIdx.x;
  const bool full = start + kAxSpan <= n;
  double x[kAxPer];
#pragma unroll
  for (int q = 0; q < kAxPer; ++q) {
    const int64_t i = base + (int64_t)q * kLzThreads;
    x[q] = (full || i < n) ? w[i] : 0.0;
  }
  if (full) {
    const double* Vb = V + base;
#pragma unroll 8
    for (int i = 0; i < nv; ++i) {
      const double hi = h[i];
      const double* Vi = Vb + (int64_t)i * ldv;
#pragma unroll
      for (int q = 0; q < kAxPer; ++q) x[q] -= hi * Vi[(int64_t)q * kLzThreads];
    }
  } else {
    for (int i = 0; i < nv; ++i) {
      const double hi = h[i];
      const double* Vi = V + (int64_t)i * ldv;
#pragma unroll
      for (int q = 0; q < kAxPer; ++q) {
        const int64_t e = base + (int64_t)q * kLzThreads;
        if (e < n) x[q] -= hi * Vi[e];
      }
    }
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kAxPer; ++q) {
    const int64_t e = base + (int64_t)q * kLzThreads;
    if (full || e < n) {
      w[e] = x[q];
      s += x[q] * x[q];
    }
  }
  if (!kNorm) return;
  __shared__ double sh[kLzThreads / 64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  s = wave_sum(s);
  if (lane == 0) sh[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// beta = sqrt(sum of partial[0..np)) (every block adds the same partials in
// the same order); block 0 writes ab[0] = h1[j] + h2[j] and ab[1] = beta;
// v_next = w / beta where v_next is given.
__global__ __launch_bounds__(kThreads) void lz_finish(double* __restrict__ v,
                                                      const double* __restrict__ w,
                                                      const double* __restrict__ partial, int np,
                                                      const double* __restrict__ h1,
                                                      const double* __restrict__ h2, int j,
                                                      double* __restrict__ ab, int64_t n) {
  __shared__ double beta;
  if (threadIdx.x < 64) {
    const double nrm = wave_row_sum(partial, np);
    if (threadIdx.x == 0) beta = sqrt(nrm > 0.0 ? nrm : 0.0);
  }
  __syncthreads();
  const double b = beta;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ab[0] = h1[j] + h2[j];
    ab[1] = b;
  }
  if (!v) return;
  const double inv = b > 0.0 ? 1.0 / b : 0.0;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) v[i] = w[i] * inv;
}

// w -= sum_{i<nv} h[i] V_i, then partial[i * gridDim.x + blockIdx.x] = the
// block's part of <V_i, w> for the updated w: one pass over the basis for
// both (the first CGS pass's update and the second pass's products).  Each
// thread keeps its element of every basis vector in registers, so kNv (32 or
// 64) bounds nv; one element per thread, 256 per block.  The kNv per-lane
// products are summed over a wave by a reduce-scatter butterfly: at every
// step a lane sends half of its values to its partner and keeps the other
// half, so after the last step lane l holds the wave's sum for vector
// l mod kNv (kNv - 1 exchanges instead of 6 kNv).
template <int kNv>
__global__ __launch_bounds__(kLzThreads) void lz_axpy_dot(double* __restrict__ w,
                                                          const double* __restrict__ V,
                                                          int64_t ldv, int nv, int64_t n,
                                                          const double* __restrict__ h,
                                                          double* __restrict__ partial) {
  static_assert(kNv == 32 || kNv == 64, "the butterfly covers 32 or 64 vectors");
  __shared__ double sh[kLzThreads / 64][kNv];
  const int64_t e = (int64_t)blockIdx.x * kLzThreads + threadIdx.x;
  const bool ok = e < n;
  const int64_t ec = ok ? e : n - 1;   // in-range address for the tail block
  double v[kNv];
#pragma unroll
  for (int i = 0; i < kNv; ++i) v[i] = V[(int64_t)(i < nv ? i : 0) * ldv + ec];
  double x = ok ? w[ec] : 0.0;
#pragma unroll
  for (int i = 0; i < kNv; ++i)
    if (i < nv) x -= h[i] * v[i];
  if (ok) w[e] = x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double p[kNv];
#pragma unroll
  for (int i = 0; i < kNv; ++i) p[i] = (ok && i < nv) ? v[i] * x : 0.0;
  // reduce-scatter over offsets kNv/2, ..., 1: values [0, c) -> [0, c/2)
#pragma unroll
  for (int c = kNv; c > 1; c >>= 1) {
    const int half = c >> 1;
    const bool upper = (lane & half) != 0;
#pragma unroll
    for (int j = 0; j < half; ++j) {
      const double send = upper ? p[j] : p[j + half];
      const double keep = upper ? p[j + half] : p[j];
      p[j] = keep + __shfl_xor(send, half, 64);
    }
  }
  // lane l now holds the sum over its group of kNv lanes for vector l % kNv
  double t = p[0];
  if (kNv == 32) t += __shfl_xor(t, 32, 64);
  if (lane < kNv) sh[wave][lane] = t;
  __syncthreads();
  if (threadIdx.x < nv)
    partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] =
        ((sh[0][threadIdx.x] + sh[1][threadIdx.x]) + sh[2][threadIdx.x]) + sh[3][threadIdx.x];
}

template <int kNv>
void launch_axpy_dot(double* w, const double* V, int64_t ldv, int nv, int64_t n, const double* h,
                     double* partial, int nb, hipStream_t stream) {
  hipLaunchKernelGGL(lz_axpy_dot<kNv>, dim3(nb), dim3(kLzThreads), 0, stream, w, V, ldv, nv, n, h,
                     partial);
}

hipError_t launch_lz_step(double* w, const double* V, int64_t ldv, int nv, int64_t n,
                          double* h1, double* h2, double* partial, double* ab, double* vnext,
                          hipStream_t stream) {
  const dim3 gd(dot_blocks(n), (nv + kDotG - 1) / kDotG);
  const int na = axpy_blocks(n);
  hipLaunchKernelGGL(lz_dot, gd, dim3(kLzThreads), 0, stream, V, ldv, nv, w, n, partial);
  hipLaunchKernelGGL(lz_reduce, dim3(nv), dim3(64), 0, stream, partial, (int)gd.x, h1);
  if (nv <= kFusedMaxNv) {
    // first update and second products in one pass over the basis
    const int nb = (int)((n + kLzThreads - 1) / kLzThreads);
    if (nv <= 32)
      launch_axpy_dot<32>(w, V, ldv, nv, n, h1, partial, nb, stream);
    else
      launch_axpy_dot<64>(w, V, ldv, nv, n, h1, partial, nb, stream);
    hipLaunchKernelGGL(lz_reduce, dim3(nv), dim3(64), 0, stream, partial, nb, h2);
  } else {
    hipLaunchKernelGGL(lz_axpy<false>, dim3(na), dim3(kLzThreads), 0, stream, w, V, ldv, nv, n, h1,
                       partial);
    hipLaunchKernelGGL(lz_dot, gd, dim3(kLzThreads), 0, stream, V, ldv, nv, w, n, partial);
    hipLaunchKernelGGL(lz_reduce, dim3(nv), dim3(64), 0, stream, partial, (int)gd.x, h2);
  }
  hipLaunchKernelGGL(lz_axpy<true>, dim3(na), dim3(kLzThreads), 0, stream, w, V, ldv, nv, n, h2,
                     partial);
  const unsigned nfin = vnext ? (unsigned)((n + kThreads - 1) / kThreads) : 1u;
  hipLaunchKernelGGL(lz_finish, dim3(nfin), dim3(kThreads), 0, stream, vnext, w, partial, na, h1, h2,
                     nv - 1, ab, n);
  return hipGetLastError();
}

hipError_t launch_multi_dot(const double* V, int64_t ldv, int nv, const double* w, int64_t n,
                            double* partial, double* h, hipStream_t stream) {
  if (nv <= 0) return hipSuccess;
  const int nblk = vec_blocks(n);
  dim3 grid(nblk, (nv + kVecsPerBlock - 1) / kVecsPerBlock);
  hipLaunchKernelGGL(multi_dot_partial, grid, dim3(kThreads), 0, stream, V, ldv, nv, w, n, partial);
  hipLaunchKernelGGL(sum_partials, dim3(nv), dim3(kThreads), 0, stream, partial, nblk, h);
  return hipGetLastError();
}

hipError_t launch_multi_axpy_norm(double* w, const double* V, int64_t ldv, int nv,
                                  const double* h, int64_t n, double* partial, double* nrm2,
                                  hipStream_t stream) {
  const int nblk = vec_blocks(n);
  hipLaunchKernelGGL(multi_axpy_partial, dim3(nblk), dim3(kThreads), 0, stream, w, V, ldv, nv, h, n,
                     partial);
  hipLaunchKernelGGL(sum_partials, dim3(1), dim3(kThreads), 0, stream, partial, nblk, nrm2);
  return hipGetLastError();
}

hipError_t launch_combine(double* out, const double* V, int64_t ldv, int nv, const double* u,
                          int64_t n, hipStream_t stream) {
  hipLaunchKernelGGL(combine_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads),
                     0, stream, out, V, ldv, nv, u, n);
  return hipGetLastError();
}

hipError_t launch_normalise(double* dst, const double* src, const double* nrm2, int64_t n,
                            hipStream_t stream) {
  hipLaunchKernelGGL(normalise_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, stream, dst, src, nrm2, n);
  return hipGetLastError();
}

hipError_t launch_record(const double* h1, const double* h2, int j, const double* nrm2,
                         double* ab, int it, hipStream_t stream) {
  hipLaunchKernelGGL(record_kernel, dim3(1), dim3(64), 0, stream, h1, h2, j, nrm2, ab, it);
  return hipGetLastError();
}

}  // namespace dmrg
