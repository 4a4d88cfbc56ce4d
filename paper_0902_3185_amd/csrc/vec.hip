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
// One step of the Lanczos recursion, orthogonalised against the whole basis
// in bandwidth-shaped launches.  Either classical Gram-Schmidt twice:
//   dot     partial sums of V^T w
//   reduce  h1 = sum of the partials, one wave per basis vector
//   axpy+dot  w -= V h1, then partial sums of V^T w for the updated w
//   reduce  h2
//   axpy    w -= V h2 and partial sums of ||w||^2
//   finish  (alpha, beta) and v_next = w / beta
// or the local three-term recurrence followed by one Gram-Schmidt pass,
// w' = w - alpha V_j - beta_{j-1} V_{j-1}, w -= V (V^T w'), in two passes:
//   dotk    partial sums of V^T w and V^T V_j in one sweep (lz_dotk_groups)
//   reduce  the pass's coefficients (lz_reduce_local)
//   axpy    the combined update and partial sums of ||w||^2 (lz_axpy_local)
// or the recurrence alone, w' = w - alpha V_j - beta_{j-1} V_{j-1}, which
// reads three vectors and not the basis:
//   dot     partial sums of <V_j, w> (lz_dot_uw)
//   update  alpha, w' and partial sums of ||w'||^2 (lz_local_update).
// In the last two forms the new vector is left unnormalised: the next
// step sums its norm and scales it on the fly (and writes it back
// normalised), so neither needs a finishing launch.
// One pass over a vector that is already orthogonal to V up to the
// recurrence's small remainder keeps the basis orthogonal to working
// precision; one pass over w itself would not (its error grows by about
// ||H V_j|| / beta_j per step).  The solver alternates the pass and the
// recurrence alone, which keeps the basis semi-orthogonal.
// Every pass gives each thread one element of w (256 per block, a grid of
// ceil(n / 256) blocks) and walks the basis vectors in batches whose loads
// are all issued before the first use, so a wave keeps a batch of basis
// elements in flight instead of one memory latency per vector (the
// single-pass step's sweep instead splits the basis over waves, each with
// four elements per lane: lz_dotk_groups).  Partial sums
// are added in a fixed order by the next launch, so results are repeatable;
// the kernel boundary makes them visible across the chip without any cache
// maintenance inside the kernels.
// ---------------------------------------------------------------------------
constexpr int kLzThreads = 256;
constexpr int kBatch = 32;        // basis vectors per batch of loads
constexpr int kTailBatch = 8;     // batch for the last nv % kBatch vectors
constexpr int kFusedMaxNv = 64;   // basis size up to which axpy and dot share a pass

int lz_blocks(int64_t n) { return (int)std::max<int64_t>(1, (n + kLzThreads - 1) / kLzThreads); }

size_t lz_partial_size(int64_t n, int nv) {
  return (size_t)2 * std::max(nv, 1) * (size_t)lz_blocks(n);
}

size_t lz_norm_partials(int64_t n) { return (size_t)lz_blocks(n); }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of row[0..cnt) by one wave: lane l adds l, l+64, ... in order, then a
// fixed butterfly.  Every lane returns the total.  The loads of a batch of
// kRowBatch values per lane are all issued before the first add, so a row of
// up to 64 * kRowBatch partials costs one memory latency rather than one per
// value (the partials were written by the previous launch and are read from
// another XCD's cache or from memory).
constexpr int kRowBatch = 16;   // the host's wave_order_sum (api.cpp) adds in this order too
__device__ inline double wave_row_sum(const double* __restrict__ row, int cnt) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int b0 = 0; b0 < cnt; b0 += 64 * kRowBatch) {
    double t[kRowBatch];
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      const int b = b0 + lane + 64 * u;
      t[u] = b < cnt ? row[b] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) s += t[u];
  }
  return wave_sum(s);
}

// Reduce-scatter of kB per-lane values over a wave: at the step of width H a
// lane sends half of its values to the lane H away and keeps (and adds) the
// other half, so after log2(kB) steps lane l holds the sum over its group of
// kB lanes of p[l % kB]; the 64 / kB groups are then added by a butterfly.
// kB - 1 + log2(64 / kB) exchanges instead of 6 kB.  Every lane l returns
// the wave's sum for value l % kB.
template <int H, int kB>
__device__ __forceinline__ void rs_step(double (&p)[kB], int lane) {
  const bool upper = (lane & H) != 0;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const double send = upper ? p[j] : p[j + H];
    const double keep = upper ? p[j + H] : p[j];
    p[j] = keep + __shfl_xor(send, H, 64);
  }
}
template <int kB>
__device__ __forceinline__ double wave_reduce_scatter(double (&p)[kB]) {
  static_assert(kB == 8 || kB == 16 || kB == 32 || kB == 64, "batch of 8, 16, 32 or 64 values");
  const int lane = threadIdx.x & 63;
  if constexpr (kB >= 64) rs_step<32>(p, lane);
  if constexpr (kB >= 32) rs_step<16>(p, lane);
  if constexpr (kB >= 16) rs_step<8>(p, lane);
  rs_step<4>(p, lane);
  rs_step<2>(p, lane);
  rs_step<1>(p, lane);
  double t = p[0];
#pragma unroll
  for (int off = kB; off < 64; off <<= 1) t += __shfl_xor(t, off, 64);
  return t;
}

// Block sums of kB per-thread values of one batch of basis vectors [i0,
// i0 + nb) into partial[(i0 + k) * gridDim.x + blockIdx.x].  sh is double
// buffered by batch parity, so one barrier per batch suffices.
template <int kB>
__device__ __forceinline__ void block_batch_partials(double (&p)[kB], double (*sh)[kLzThreads / 64][kBatch],
                                                     int parity, int i0, int nb,
                                                     double* __restrict__ partial) {
  const double t = wave_reduce_scatter<kB>(p);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane < kB) sh[parity][wave][lane] = t;
  __syncthreads();
  if (threadIdx.x < nb) {
    const int k = threadIdx.x;
    partial[(int64_t)(i0 + k) * gridDim.x + blockIdx.x] =
        ((sh[parity][0][k] + sh[parity][1][k]) + sh[parity][2][k]) + sh[parity][3][k];
  }
}

// partial[i * gridDim.x + blockIdx.x] = the block's part of <V_i, w>, i < nv.
__global__ __launch_bounds__(kLzThreads) void lz_dot(const double* __restrict__ V, int64_t ldv,
                                                     int nv, const double* __restrict__ w,
                                                     int64_t n, double* __restrict__ partial) {
  __shared__ double sh[2][kLzThreads / 64][kBatch];
  const int64_t e = (int64_t)blockIdx.x * kLzThreads + threadIdx.x;
  const bool ok = e < n;
  const double* Vb = V + (ok ? e : 0);   // in-range address for the tail block
  const double x = ok ? w[e] : 0.0;
  int i0 = 0, parity = 0;
#pragma unroll 1
  for (; i0 + kBatch <= nv; i0 += kBatch, parity ^= 1) {
    double p[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) p[b] = Vb[(int64_t)(i0 + b) * ldv];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) p[b] = ok ? p[b] * x : 0.0;
    block_batch_partials<kBatch>(p, sh, parity, i0, kBatch, partial);
  }
#pragma unroll 1
  for (; i0 < nv; i0 += kTailBatch, parity ^= 1) {
    const int nb = min(kTailBatch, nv - i0);
    double p[kTailBatch];
#pragma unroll
    for (int b = 0; b < kTailBatch; ++b) p[b] = Vb[(int64_t)(i0 + (b < nb ? b : 0)) * ldv];
#pragma unroll
    for (int b = 0; b < kTailBatch; ++b) p[b] = (ok && b < nb) ? p[b] * x : 0.0;
    block_batch_partials<kTailBatch>(p, sh, parity, i0, nb, partial);
  }
}


// The sweep of a single-pass step: for i < nv and s < 2,
// partial[(s * nv + i) * gridDim.x + blockIdx.x] = the part of <V_i, x_s>
// over elements 256 blockIdx.x .. + 255, with x_0 = w and x_1 = V_{nv-1}
// (nv >= 2).  The basis is split over waves: wave g of block (r, y) takes
// basis vectors kGrpVecs (4 y + g) .. + kGrpVecs - 1 and elements 256 r ..
// 256 r + 255, four per lane (lane, lane + 64, ...), and keeps its
// 2 kGrpVecs sums in registers over them, in element order; one
// reduce-scatter of those sums per wave then gives the wave's parts, so
// there is one cross-lane reduction per 256 elements rather than one per
// 64, and no LDS or barrier.  x_0 and x_1 are read by every wave of a block
// (from the L1 after the first).  OffT: the type of an element offset
// (32 bits below 2^31 elements: fewer registers).  Measured on the
// physical Hubbard headline against one element per thread with a
// reduction per batch of 16 vectors (19.0 us per sweep): groups of 16
// vectors 17.0 us, of 8 vectors (twice the waves, 64 registers) faster
// again by 1-2 % of a solve.
constexpr int kGrpSteps = kLzThreads / 64;   // elements per lane
constexpr int kDotkVecs = 8;                 // basis vectors per wave in the step's sweep

template <int kGrpVecs, class OffT>
__global__ __launch_bounds__(kLzThreads) void lz_dotk_groups(const double* __restrict__ V, int64_t ldv,
                                                             int nv, const double* __restrict__ w,
                                                             int64_t n, double* __restrict__ partial) {
  // the wave index is uniform in a wave: say so, so that the vectors' start
  // addresses stay in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int g0 = (blockIdx.y * (kLzThreads / 64) + wave) * kGrpVecs;
  if (g0 >= nv) return;
  const int nvg = min(kGrpVecs, nv - g0);
  const int64_t eb = (int64_t)blockIdx.x * kLzThreads + lane;
  const double* x1 = V + (int64_t)(nv - 1) * ldv;
  double p[2 * kGrpVecs];
#pragma unroll
  for (int q = 0; q < 2 * kGrpVecs; ++q) p[q] = 0.0;
#pragma unroll 1
  for (int st = 0; st < kGrpSteps; ++st) {
    const int64_t e = eb + 64 * st;
    const bool ok = e < n;
    const OffT ec = ok ? (OffT)e : OffT(0);
    double t[kGrpVecs];
#pragma unroll
    for (int b = 0; b < kGrpVecs; ++b) {
      const double* row = V + (int64_t)(g0 + (b < nvg ? b : 0)) * ldv;   // uniform
      t[b] = row[ec];
    }
    const double x0 = ok ? w[ec] : 0.0, xv = ok ? x1[ec] : 0.0;
#pragma unroll
    for (int b = 0; b < kGrpVecs; ++b) {
      p[b] += t[b] * x0;
      p[kGrpVecs + b] += t[b] * xv;
    }
  }
  const double tot = wave_reduce_scatter<2 * kGrpVecs>(p);   // lane l: value l % (2 kGrpVecs)
  if (lane < 2 * kGrpVecs) {
    const int set = lane / kGrpVecs, b = lane % kGrpVecs;
    if (b < nvg) partial[((int64_t)set * nv + g0 + b) * gridDim.x + blockIdx.x] = tot;
  }
}
// Coefficients of the single Gram-Schmidt pass that follows the local
// three-term recurrence (see launch_lz_step_onepass).  With j = nv - 1, the
// true current vector v_j = s u where u is the stored V_j and s = 1 / ||u||
// when u was left unnormalised (npend: the previous step's partial sums of
// ||u||^2) or s = 1 otherwise; w = H u.  The sweep's two sets of partial
// sums give r_i = <V_i, H v_j> and g_i = <V_i, v_j> (times s, and times s
// again for i = j); alpha = r_j, beta = ||u|| when pending or *beta_prev.
// m_i = <V_i, V_{j-1}> is 1 for i = j - 1, g_{j-1} for i = j and 0 below:
// V_{j-1} left the previous pass orthogonal to V_0..V_{j-2} up to second
// order (the products of the pass's small coefficients and the basis'
// small overlaps), which this pass need not see.  Then
//   h[i] = r_i - alpha g_i - beta m_i + alpha [i == j] + beta [i == j-1],
// so that s w - sum_i h[i] v_i = w' - V (V^T w') for w' = H v_j - alpha v_j
// - beta V_{j-1}.  Block j writes s to *scale, beta to *beta_out (when
// pending) and alpha_j = h[j] to *alpha_out.  One block of five waves per i
// sums its rows in parallel.
__global__ __launch_bounds__(320) void lz_reduce_local(const double* __restrict__ partial, int nbx,
                                                       int nv, const double* __restrict__ beta_prev,
                                                       double* __restrict__ h,
                                                       const double* __restrict__ npend, int nnp,
                                                       double* __restrict__ scale,
                                                       double* __restrict__ beta_out,
                                                       double* __restrict__ alpha_out) {
  __shared__ double sh[5];
  const int i = blockIdx.x, j = nv - 1;
  const int wave = threadIdx.x >> 6;
  // rows: wave 0 R_i, wave 1 G_i, wave 2 G_{j-1} (block j only), wave 3
  // R_j, wave 4 ||u||^2 (pending only)
  const double* row = nullptr;
  int cnt = nbx;
  if (wave < 2) row = partial + (int64_t)(wave * nv + i) * nbx;
  else if (wave == 2) row = i == j ? partial + (int64_t)(nv + j - 1) * nbx : nullptr;
  else if (wave == 3) row = partial + (int64_t)j * nbx;
  else if (npend) {
    row = npend;
    cnt = nnp;
  }
  const double t = row ? wave_row_sum(row, cnt) : 0.0;
  if ((threadIdx.x & 63) == 0) sh[wave] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 1.0, beta = 0.0;
    if (npend) {
      beta = sqrt(sh[4] > 0.0 ? sh[4] : 0.0);
      s = beta > 0.0 ? 1.0 / beta : 0.0;
    } else {
      beta = *beta_prev;
    }
    const double alpha = s * s * sh[3];
    const double r = (i == j ? s * s : s) * sh[0];
    const double g = (i == j ? s * s : s) * sh[1];
    const double m = i == j ? s * sh[2] : (i == j - 1 ? 1.0 : 0.0);
    double c = r - alpha * g - beta * m;
    if (i == j) c += alpha;
    if (i == j - 1) c += beta;
    h[i] = c;
    if (i == j) {
      *scale = s;
      if (npend) *beta_out = beta;
      *alpha_out = c;
    }
  }
}

// h[i] = sum_b partial[i * nbx + b]: one 64-thread block per basis vector.
__global__ __launch_bounds__(64) void lz_reduce(const double* __restrict__ partial, int nbx,
                                                double* __restrict__ h) {
  const double t = wave_row_sum(partial + (int64_t)blockIdx.x * nbx, nbx);
  if (threadIdx.x == 0) h[blockIdx.x] = t;
}

// x -= sum_{i<nv} h[i] V_i[e] for this thread's element (Vb = V + e).
__device__ __forceinline__ double axpy_walk(double x, const double* __restrict__ Vb, int64_t ldv,
                                            int nv, const double* __restrict__ h) {
  int i0 = 0;
#pragma unroll 1
  for (; i0 + kBatch <= nv; i0 += kBatch) {
    double t[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) t[b] = Vb[(int64_t)(i0 + b) * ldv];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) x -= h[i0 + b] * t[b];
  }
#pragma unroll 1
  for (; i0 < nv; i0 += kTailBatch) {
    const int nb = min(kTailBatch, nv - i0);
    double t[kTailBatch];
#pragma unroll
    for (int b = 0; b < kTailBatch; ++b) t[b] = Vb[(int64_t)(i0 + (b < nb ? b : 0)) * ldv];
#pragma unroll
    for (int b = 0; b < kTailBatch; ++b)
      if (b < nb) x -= h[i0 + b] * t[b];
  }
  return x;
}

// w -= sum_{i<nv} h[i] V_i.  With kNorm, also partial[blockIdx.x] = the
// block's part of ||w||^2.
template <bool kNorm>
__global__ __launch_bounds__(kLzThreads) void lz_axpy(double* __restrict__ w,
                                                      const double* __restrict__ V, int64_t ldv,
                                                      int nv, int64_t n,
                                                      const double* __restrict__ h,
                                                      double* __restrict__ partial) {
  const int64_t e = (int64_t)blockIdx.x * kLzThreads + threadIdx.x;
  const bool ok = e < n;
  double x = ok ? w[e] : 0.0;
  x = axpy_walk(x, V + (ok ? e : 0), ldv, nv, h);
  if (ok) w[e] = x;
  if (!kNorm) return;
  __shared__ double sh[kLzThreads / 64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const double s = wave_sum(ok ? x * x : 0.0);
  if (lane == 0) sh[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// The update of a single-pass step: x = s w - sum_{i<j} h[i] V_i - h[j] s u
// (j = nv - 1, u the stored V_j, s = *scale); with pending, V_j is replaced
// by s u in place.  x goes to out (if not null) unnormalised, and
// partial[blockIdx.x] = the block's part of ||x||^2.
__global__ __launch_bounds__(kLzThreads) void lz_axpy_local(const double* __restrict__ w,
                                                            double* __restrict__ V, int64_t ldv,
                                                            int nv, int64_t n,
                                                            const double* __restrict__ h,
                                                            const double* __restrict__ scale,
                                                            bool pending, double* __restrict__ out,
                                                            float* __restrict__ out32,
                                                            double* __restrict__ partial) {
  const int64_t e = (int64_t)blockIdx.x * kLzThreads + threadIdx.x;
  const bool ok = e < n;
  const int64_t ec = ok ? e : 0;
  const int j = nv - 1;
  const double sc = *scale;
  const double u = V[(int64_t)j * ldv + ec];
  double x = ok ? sc * w[ec] : 0.0;
  x = axpy_walk(x, V + ec, ldv, j, h);
  const double vj = pending ? sc * u : u;
  x -= h[j] * vj;
  if (ok) {
    if (pending) V[(int64_t)j * ldv + e] = vj;
    if (out) out[e] = x;
    if (out32) out32[e] = (float)x;
  }
  __shared__ double sh[kLzThreads / 64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const double q = wave_sum(ok ? x * x : 0.0);
  if (lane == 0) sh[wave] = q;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// partial[blockIdx.x] = the block's part of <u, w>.
__global__ __launch_bounds__(kLzThreads) void lz_dot_uw(const double* __restrict__ u,
                                                        const double* __restrict__ w, int64_t n,
                                                        double* __restrict__ partial) {
  const int64_t e = (int64_t)blockIdx.x * kLzThreads + threadIdx.x;
  __shared__ double sh[kLzThreads / 64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const double t = wave_sum(e < n ? u[e] * w[e] : 0.0);
  if (lane == 0) sh[wave] = t;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// The update of a recurrence-only step (j >= 1): V_j is stored unnormalised
// as u, npend holds the partial sums of ||u||^2 and dpart those of <u, w>
// for w = H u (np of each).  With beta_{j-1} = ||u||, s = 1 / ||u|| and
// alpha_j = s^2 <u, w>:  x = s w - alpha_j s u - beta_{j-1} V_{j-1}; V_j is
// replaced by s u in place, x goes to out (if not null) unnormalised and
// nout[blockIdx.x] = the block's part of ||x||^2; block 0 writes ab[-1] =
// beta_{j-1} and ab[0] = alpha_j.  Every block adds the same partials in
// the same order, so all of them use the same s and alpha_j.
__global__ __launch_bounds__(kLzThreads) void lz_local_update(
    const double* __restrict__ w, double* __restrict__ V, int64_t ldv, int j, int64_t n,
    const double* __restrict__ dpart, const double* __restrict__ npend, int np,
    double* __restrict__ out, float* __restrict__ out32, double* __restrict__ nout,
    double* __restrict__ ab) {
  __shared__ double sums[2];
  __shared__ double sh[kLzThreads / 64];
  const int64_t e = (int64_t)blockIdx.x * kLzThreads + threadIdx.x;
  const bool ok = e < n;
  const int64_t ec = ok ? e : 0;
  // the thread's elements are loaded before the sums, so the latencies overlap
  const double wi = w[ec];
  const double ui = V[(int64_t)j * ldv + ec];
  const double pi = V[(int64_t)(j - 1) * ldv + ec];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (wave < 2) {
    const double t = wave_row_sum(wave == 0 ? npend : dpart, np);
    if (lane == 0) sums[wave] = t;
  }
  __syncthreads();
  const double beta = sqrt(sums[0] > 0.0 ? sums[0] : 0.0);
  const double sc = beta > 0.0 ? 1.0 / beta : 0.0;
  const double alpha = sc * sc * sums[1];
  const double vj = sc * ui;
  const double x = ok ? sc * wi - alpha * vj - beta * pi : 0.0;
  if (ok) {
    V[(int64_t)j * ldv + e] = vj;
    if (out) out[e] = x;
    if (out32) out32[e] = (float)x;
  }
  const double q = wave_sum(x * x);
  if (lane == 0) sh[wave] = q;
  __syncthreads();
  if (threadIdx.x == 0) {
    nout[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    if (blockIdx.x == 0) {
      ab[-1] = beta;
      ab[0] = alpha;
    }
  }
}

// beta = sqrt(sum of partial[0..np)) (every block adds the same partials in
// the same order); block 0 writes ab[0] = h1[j] + h2[j] and ab[1] = beta;
// v_next = w / beta where v_next is given.
__global__ __launch_bounds__(kThreads) void lz_finish(double* __restrict__ v,
                                                      const double* __restrict__ w,
                                                      const double* __restrict__ partial, int np,
                                                      const double* __restrict__ h1,
                                                      const double* __restrict__ h2, int j,
                                                      double* __restrict__ ab, int64_t n,
                                                      float* __restrict__ v32) {
  __shared__ double beta;
  // this thread's element of w is loaded before the norm is summed, so the
  // two memory latencies overlap
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const double wi = (v && i < n) ? w[i] : 0.0;
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
  if (i < n) {
    v[i] = wi * inv;
    if (v32) v32[i] = (float)(wi * inv);
  }
}

// w -= sum_{i<nv} h[i] V_i, then partial[i * gridDim.x + blockIdx.x] = the
// block's part of <V_i, w> for the updated w: one pass over the basis for
// both (the first CGS pass's update and the second pass's products).  Each
// thread keeps its element of every basis vector in registers, so kNv (8,
// 16, 32 or 64, the smallest that holds nv) bounds nv.
template <int kNv>
__global__ __launch_bounds__(kLzThreads) void lz_axpy_dot(double* __restrict__ w,
                                                          const double* __restrict__ V,
                                                          int64_t ldv, int nv, int64_t n,
                                                          const double* __restrict__ h,
                                                          double* __restrict__ partial) {
  __shared__ double sh[kLzThreads / 64][kNv];
  const int64_t e = (int64_t)blockIdx.x * kLzThreads + threadIdx.x;
  const bool ok = e < n;
  const int64_t ec = ok ? e : 0;   // in-range address for the tail block
  double v[kNv];
#pragma unroll
  for (int i = 0; i < kNv; ++i) v[i] = V[(int64_t)(i < nv ? i : 0) * ldv + ec];
  double x = ok ? w[ec] : 0.0;
#pragma unroll
  for (int i = 0; i < kNv; ++i)
    if (i < nv) x -= h[i] * v[i];
  if (ok) w[e] = x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < kNv; ++i) v[i] = (ok && i < nv) ? v[i] * x : 0.0;
  const double t = wave_reduce_scatter<kNv>(v);
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
                          hipStream_t stream, float* vnext32) {
  if (nv < 1) return hipErrorInvalidValue;
  const int nb = lz_blocks(n);
  hipLaunchKernelGGL(lz_dot, dim3(nb), dim3(kLzThreads), 0, stream, V, ldv, nv, w, n, partial);
  hipLaunchKernelGGL(lz_reduce, dim3(nv), dim3(64), 0, stream, partial, nb, h1);
  if (nv <= kFusedMaxNv) {
    // first update and second products in one pass over the basis
    if (nv <= 8)
      launch_axpy_dot<8>(w, V, ldv, nv, n, h1, partial, nb, stream);
    else if (nv <= 16)
      launch_axpy_dot<16>(w, V, ldv, nv, n, h1, partial, nb, stream);
    else if (nv <= 32)
      launch_axpy_dot<32>(w, V, ldv, nv, n, h1, partial, nb, stream);
    else
      launch_axpy_dot<64>(w, V, ldv, nv, n, h1, partial, nb, stream);
  } else {
    hipLaunchKernelGGL(lz_axpy<false>, dim3(nb), dim3(kLzThreads), 0, stream, w, V, ldv, nv, n, h1,
                       partial);
    hipLaunchKernelGGL(lz_dot, dim3(nb), dim3(kLzThreads), 0, stream, V, ldv, nv, w, n, partial);
  }
  hipLaunchKernelGGL(lz_reduce, dim3(nv), dim3(64), 0, stream, partial, nb, h2);
  hipLaunchKernelGGL(lz_axpy<true>, dim3(nb), dim3(kLzThreads), 0, stream, w, V, ldv, nv, n, h2,
                     partial);
  const unsigned nfin = vnext ? (unsigned)((n + kThreads - 1) / kThreads) : 1u;
  hipLaunchKernelGGL(lz_finish, dim3(nfin), dim3(kThreads), 0, stream, vnext, w, partial, nb, h1, h2,
                     nv - 1, ab, n, vnext ? vnext32 : nullptr);
  return hipGetLastError();
}

hipError_t launch_lz_step_onepass(double* w, double* V, int64_t ldv, int nv, int64_t n, double* h,
                                  double* partial, const double* npend, const double* beta_prev,
                                  double* nout, double* scale, double* ab, double* out,
                                  hipStream_t stream, float* out32) {
  if (nv < 2 || !nout || !scale || (!npend && !beta_prev)) return hipErrorInvalidValue;
  const int nb = lz_blocks(n);
  const int nbk = nb;   // the sweep's blocks: 256 elements each
  constexpr int kG = kDotkVecs;
  const dim3 grid(nbk, (nv + kG * (kLzThreads / 64) - 1) / (kG * (kLzThreads / 64)));
  if (n < (int64_t(1) << 31))
    hipLaunchKernelGGL((lz_dotk_groups<kG, uint32_t>), grid, dim3(kLzThreads), 0, stream, V, ldv, nv, w, n,
                       partial);
  else
    hipLaunchKernelGGL((lz_dotk_groups<kG, int64_t>), grid, dim3(kLzThreads), 0, stream, V, ldv, nv, w, n,
                       partial);
  // beta_{j-1} into ab[-1] (when pending), alpha_j into ab[0]
  hipLaunchKernelGGL(lz_reduce_local, dim3(nv), dim3(320), 0, stream, partial, nbk, nv, beta_prev, h,
                     npend, nb, scale, ab - 1, ab);
  hipLaunchKernelGGL(lz_axpy_local, dim3(nb), dim3(kLzThreads), 0, stream, w, V, ldv, nv, n, h, scale,
                     npend != nullptr, out, out ? out32 : nullptr, nout);
  return hipGetLastError();
}

hipError_t launch_lz_step_recurrence(const double* w, double* V, int64_t ldv, int nv, int64_t n,
                                     double* partial, const double* npend, double* nout,
                                     double* ab, double* out, hipStream_t stream, float* out32) {
  if (nv < 2 || !npend || !nout) return hipErrorInvalidValue;
  const int nb = lz_blocks(n);
  const int j = nv - 1;
  hipLaunchKernelGGL(lz_dot_uw, dim3(nb), dim3(kLzThreads), 0, stream, V + (int64_t)j * ldv, w, n,
                     partial);
  hipLaunchKernelGGL(lz_local_update, dim3(nb), dim3(kLzThreads), 0, stream, w, V, ldv, j, n,
                     partial, npend, nb, out, out ? out32 : nullptr, nout, ab);
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
