// FP64 vector kernels for the Lanczos recursion: several dot products against
// the Krylov basis in one pass, the matching update, norms and combinations.
// Reductions go through fixed-shape partial sums, so results are repeatable.
#include <hip/hip_runtime.h>

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
// Fused CGS2 passes for one Lanczos step.  Each kernel walks the Krylov basis
// once; every block writes its partial sums, and the last block to finish
// (counted with one device-scope atomic) adds them up in a fixed order and
// resets the counter, so results are repeatable and no extra launch is needed.
// ---------------------------------------------------------------------------
constexpr int kLzThreads = 256;
constexpr int kLzPer = 8;                       // elements per thread
constexpr int kLzSpan = kLzThreads * kLzPer;    // elements per block

int lz_blocks(int64_t n) { return (int)((n + kLzSpan - 1) / kLzSpan); }

// Returns true in every thread of the block that finished last.
__device__ inline bool last_block_done(unsigned int* counter) {
  __shared__ bool last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int done = atomicAdd(counter, 1u);
    last = done == gridDim.x - 1;
  }
  __syncthreads();
  if (last) __threadfence();
  return last;
}

// out[j] = sum_b partial[j * nblk + b] (b ascending), by the whole block.
__device__ inline void reduce_partials(const double* partial, int nblk, int nv, double* out,
                                       double* sh) {
  for (int j = 0; j < nv; ++j) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kLzThreads) s += partial[(int64_t)j * nblk + b];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[j] = s;
  }
}

// Mode 0: h1 = V^T w.
// Mode 1: w -= V h1, then h2 = V^T w.
// Mode 2: w -= V h2, then nrm = ||w||^2 and ab[0..1] = (h1[j] + h2[j], sqrt(nrm)).
template <int kMode>
__global__ __launch_bounds__(kLzThreads) void lz_pass(double* __restrict__ w,
                                                      const double* __restrict__ V, int64_t ldv,
                                                      int nv, int64_t n, double* __restrict__ h1,
                                                      double* __restrict__ h2,
                                                      double* __restrict__ partial,
                                                      unsigned int* __restrict__ counter,
                                                      double* __restrict__ ab) {
  __shared__ double sh[4];
  const int nblk = gridDim.x;
  const int64_t base = (int64_t)blockIdx.x * kLzSpan + threadIdx.x;
  double x[kLzPer];
#pragma unroll
  for (int q = 0; q < kLzPer; ++q) {
    const int64_t i = base + (int64_t)q * kLzThreads;
    x[q] = i < n ? w[i] : 0.0;
  }
  if (kMode >= 1) {
    const double* h = kMode == 1 ? h1 : h2;
    for (int j = 0; j < nv; ++j) {
      const double hj = h[j];
      const double* Vj = V + (int64_t)j * ldv;
#pragma unroll
      for (int q = 0; q < kLzPer; ++q) {
        const int64_t i = base + (int64_t)q * kLzThreads;
        if (i < n) x[q] -= hj * Vj[i];
      }
    }
#pragma unroll
    for (int q = 0; q < kLzPer; ++q) {
      const int64_t i = base + (int64_t)q * kLzThreads;
      if (i < n) w[i] = x[q];
    }
  }
  if (kMode <= 1) {
    for (int j = 0; j < nv; ++j) {
      const double* Vj = V + (int64_t)j * ldv;
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < kLzPer; ++q) {
        const int64_t i = base + (int64_t)q * kLzThreads;
        if (i < n) s += Vj[i] * x[q];
      }
      s = block_sum(s, sh);
      if (threadIdx.x == 0) partial[(int64_t)j * nblk + blockIdx.x] = s;
    }
  } else {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kLzPer; ++q) s += x[q] * x[q];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
  if (!last_block_done(counter)) return;
  if (kMode == 2) {
    __shared__ double nrm;
    reduce_partials(partial, nblk, 1, &nrm, sh);
    __syncthreads();
    if (threadIdx.x == 0) {
      ab[0] = h1[nv - 1] + h2[nv - 1];
      ab[1] = sqrt(nrm > 0.0 ? nrm : 0.0);
    }
  } else {
    reduce_partials(partial, nblk, nv, kMode == 0 ? h1 : h2, sh);
  }
  if (threadIdx.x == 0) atomicExch(counter, 0u);
}

// v_next = w / ab[1]
__global__ __launch_bounds__(kThreads) void lz_normalise(double* __restrict__ v,
                                                         const double* __restrict__ w,
                                                         const double* __restrict__ ab,
                                                         int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const double b = ab[1];
  const double inv = b > 0.0 ? 1.0 / b : 0.0;
  if (i < n) v[i] = w[i] * inv;
}

hipError_t launch_lz_step(double* w, const double* V, int64_t ldv, int nv, int64_t n,
                          double* h1, double* h2, double* partial, unsigned int* counter,
                          double* ab, double* vnext, hipStream_t stream) {
  const int nblk = lz_blocks(n);
  hipLaunchKernelGGL(lz_pass<0>, dim3(nblk), dim3(kLzThreads), 0, stream, w, V, ldv, nv, n, h1, h2,
                     partial, counter, ab);
  hipLaunchKernelGGL(lz_pass<1>, dim3(nblk), dim3(kLzThreads), 0, stream, w, V, ldv, nv, n, h1, h2,
                     partial, counter, ab);
  hipLaunchKernelGGL(lz_pass<2>, dim3(nblk), dim3(kLzThreads), 0, stream, w, V, ldv, nv, n, h1, h2,
                     partial, counter, ab);
  if (vnext)
    hipLaunchKernelGGL(lz_normalise, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       stream, vnext, w, ab, n);
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
