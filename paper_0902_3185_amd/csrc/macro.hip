// The macro-tile FP32 / BF16 product (plan in macro.h).
//
// A workgroup of four waves owns one 64 x 64 output tile at a time; wave w
// computes the 32 x 32 quarter (w / 2, w % 2).  The tile's contraction runs
// in stages of 32 positions of one segment: the workgroup loads the stage's
// two panels -- A (64 output rows x 32) and B (32 x 64 output columns) --
// once, scales them and writes them to LDS ([row][k] and [column][k], rows
// padded to 36 floats so that the matrix-core reads below meet no bank
// conflict), and all four waves read their operands from there, so every
// operand element fetched from memory feeds 64 multiply-adds (a 32 x 32
// tile per workgroup would give each element 32).  Two LDS buffers
// alternate: while the waves work on one stage, the next is being written;
// the loads of the two stages after it are in flight in registers.
//
// Panel loads (256 threads, thread t, wave w, lane l):
//   A rows t/8 and t/8 + 32, positions 4*(t%8) .. +3, one 16-byte load
//     each (SEG_KN: the operator block; SEG_MK: psi row src[m]);
//   B for SEG_KN, psi rows k = 8w .. 8w + 7 at gathered column src[l]: eight
//     4-byte loads, the wave reading 64 (mostly consecutive) columns of a
//     row at once; for SEG_MK, operator rows t/8 and t/8 + 32, four 4-byte
//     loads each.
// The operator blocks are a copy with rows padded by zeros to whole stages.
// Buffer loads carry each buffer's size, so an offset past it reads zero
// with no memory traffic; dead rows or columns start from such an offset.
//
// Matrix-core step (v_mfma_f32_16x16x4f32, per 16 positions): A[i][k] from
// lane i + 16k, B[k][j] from lane j + 16k, D[i][j] in lane j + 16*(i/4),
// register i%4; lane group kk = lane/16 holds positions 4kk .. 4kk + 3 and
// instruction s takes position 4kk + s of each.  The BF16 form writes each
// panel as hi = bf16(x) and lo = bf16(x - hi) and issues
// hi*hi + hi*lo + lo*hi with v_mfma_f32_16x16x16bf16_1k.
//
// A tile shared by several workgroups: each stores its 64 x 64 FP32 partial
// sum (in the lanes' register order) and goes on; a second kernel adds the
// partials of every shared tile in share order in FP64, adds the elementwise
// terms and writes y (the kernel boundary makes all partials visible).
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "kernels.h"
#include "macro.h"

namespace dmrg {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

constexpr int kLd = kMacStage + 4;          // floats per LDS panel row
constexpr int kPanel = kMac * kLd;          // floats per panel
constexpr uint32_t kDead = 0x80000000u;     // past every buffer: reads zero

__device__ inline int rfl(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
// voff: per-lane byte offset; soff: uniform byte offset (the stage's, held
// in a scalar register, so that advancing a stage costs no vector work)
__device__ inline f4 ld16(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}
__device__ inline float ld4(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}

// One stage's loads in registers: A rows (two f4), B (SEG_KN: eight
// gathered values as two f4; SEG_MK: two f4 rows).
struct Raw {
  f4 a[2], b[2];
};
// The fetch side of a segment: its first stage, the first stage past it,
// and per thread the byte offsets of a stage's loads at the segment's first
// stage -- A rows oa[j]; B values j*4 + e at bb[j] + e * step -- and the
// bytes per stage (da, db; uniform).  SEG_KN reads B as psi rows
// 8w + 4j + e at column src[l] (step = one psi row); SEG_MK reads it as
// operator rows t/8 + 32j, positions 4(t%8) + e (step = one float).  Both
// kinds issue the same ten loads, so that the waits for one stage's data
// never cover the next stage's loads.
struct Fetch {
  int seg, kind, st0, next;
  uint32_t oa[2], bb[2];
  uint32_t da, db, step;
};
// The write side of a segment: per-thread scales of the panels and the
// panel elements this thread writes (row * kLd + position).
struct Use {
  int seg, st0, next;
  float sa[2], sb[2];
  int ia[2], ib[2];
};

// sg lives in LDS; `next` is the first stage of the following segment.
__device__ inline void setup_fetch(Fetch& f, int g, const MacSeg& sg, int next, const MacTile& T, int t) {
  f.seg = g;
  f.kind = rfl(sg.kind);
  f.st0 = rfl(sg.st0);
  f.next = next;
  const int w = t >> 6, l = t & 63;
  const int64_t ldp = sg.psi_ld, ldo = sg.op_ld;
  if (f.kind == SEG_KN) {
#pragma unroll
    for (int j = 0; j < 2; ++j)
      f.oa[j] = (uint32_t)(4 * (sg.op_off + (int64_t)(T.m0 + (t >> 3) + 32 * j) * ldo + (t & 7) * 4));
    const int src = sg.src[l];
#pragma unroll
    for (int j = 0; j < 2; ++j)
      f.bb[j] = src >= 0 ? (uint32_t)(4 * (sg.psi_off + (int64_t)(8 * w + 4 * j) * ldp + src)) : kDead;
    f.da = 4 * kMacStage;
    f.db = rfl((int)(4 * kMacStage * ldp));
    f.step = rfl((int)(4 * ldp));
  } else {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int src = sg.src[(t >> 3) + 32 * j];
      f.oa[j] = src >= 0 ? (uint32_t)(4 * (sg.psi_off + (int64_t)src * ldp + (t & 7) * 4)) : kDead;
      f.bb[j] = (uint32_t)(4 * (sg.op_off + (int64_t)(T.n0 + (t >> 3) + 32 * j) * ldo + (t & 7) * 4));
    }
    f.da = 4 * kMacStage;
    f.db = 4 * kMacStage;
    f.step = 4;
  }
}

__device__ inline void setup_use(Use& u, int g, const MacSeg& sg, int next, const MacTile& T, int t) {
  u.seg = g;
  u.st0 = rfl(sg.st0);
  u.next = next;
  const int w = t >> 6, l = t & 63;
  const float c = (float)sg.c;
#pragma unroll
  for (int j = 0; j < 2; ++j) u.ia[j] = ((t >> 3) + 32 * j) * kLd + (t & 7) * 4;
  if (rfl(sg.kind) == SEG_KN) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      u.sa[j] = T.m0 + (t >> 3) + 32 * j < T.a ? c : 0.f;
      u.ib[j] = l * kLd + 8 * w + 4 * j;
    }
    u.sb[0] = sg.src[l] >= 0 ? sg.scl[l] : 0.f;
    u.sb[1] = u.sb[0];
  } else {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int r = (t >> 3) + 32 * j;
      u.sa[j] = sg.src[r] >= 0 ? (float)(sg.c * (double)sg.scl[r]) : 0.f;
      u.sb[j] = T.n0 + r < T.b ? 1.f : 0.f;
      u.ib[j] = u.ia[j];
    }
  }
}

// Loads of stage `st` of the segment: the same ten loads for both kinds,
// the buffers chosen by kind; a dead stage (past the item) reads through
// the empty buffer rz, i.e. zeros with no traffic.
__device__ inline void load(Raw& R, const Fetch& f, int st, bool live, __amdgpu_buffer_rsrc_t rd,
                            __amdgpu_buffer_rsrc_t rp, __amdgpu_buffer_rsrc_t rz) {
  const bool kn = f.kind == SEG_KN;
  const __amdgpu_buffer_rsrc_t ra = live ? (kn ? rd : rp) : rz, rb = live ? (kn ? rp : rd) : rz;
  const uint32_t sa = st * f.da, sb = st * f.db;
#pragma unroll
  for (int j = 0; j < 2; ++j) R.a[j] = ld16(ra, f.oa[j], sa);
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int e = 0; e < 4; ++e) R.b[j][e] = ld4(rb, f.bb[j], sb + e * f.step);
}

template <bool kBF16>
struct Lds;

// FP32 panels: A [64][kLd], B [64][kLd] per buffer.
template <>
struct Lds<false> {
  static constexpr int kFloats = 2 * kPanel;
  __device__ static void put(float* buf, int idx, const f4& v, bool isB) {
    *reinterpret_cast<f4*>(buf + (isB ? kPanel : 0) + idx) = v;
  }
};

__device__ inline void split(const f4& x, s16x4& hi, s16x4& lo) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const __bf16 h = (__bf16)x[j];
    const __bf16 l = (__bf16)(x[j] - (float)h);
    hi[j] = __builtin_bit_cast(short, h);
    lo[j] = __builtin_bit_cast(short, l);
  }
}

// BF16 panels: for A and B, hi and lo halves [64][kLd] each (kLd shorts per
// row; the buffer holds four such panels in the room of two FP32 ones).
template <>
struct Lds<true> {
  static constexpr int kFloats = 2 * kPanel;
  __device__ static void put(float* buf, int idx, const f4& v, bool isB) {
    short* p = reinterpret_cast<short*>(buf) + (isB ? 2 * kPanel : 0);
    s16x4 hi, lo;
    split(v, hi, lo);
    *reinterpret_cast<s16x4*>(p + idx) = hi;
    *reinterpret_cast<s16x4*>(p + kPanel + idx) = lo;
  }
};

// Scaled panels of a stage into buf.  No position past a segment's end needs
// a mask: the operator side reads the zeros that pad its rows to whole
// stages (and finite psi values beyond a block meet those zeros).
template <bool kBF16>
__device__ inline void stage(const Raw& R, const Use& u, float* buf) {
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    Lds<kBF16>::put(buf, u.ia[j], u.sa[j] * R.a[j], false);
    Lds<kBF16>::put(buf, u.ib[j], u.sb[j] * R.b[j], true);
  }
}

struct Acc {
  f32x4 d[4];   // 16 x 16 quarter (qi, qj) of the wave's 32 x 32 at d[2 qi + qj]
};

template <bool kBF16>
__device__ inline void mma(Acc& acc, const float* buf, int w, int lane) {
  const int i = lane & 15, kk = lane >> 4, r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
  if constexpr (!kBF16) {
    const float* As = buf;
    const float* Bs = buf + kPanel;
#pragma unroll
    for (int c = 0; c < kMacStage / 16; ++c) {
      f4 a[2], b[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        a[h] = *reinterpret_cast<const f4*>(As + (r0 + 16 * h + i) * kLd + 16 * c + 4 * kk);
        b[h] = *reinterpret_cast<const f4*>(Bs + (c0 + 16 * h + i) * kLd + 16 * c + 4 * kk);
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int qi = 0; qi < 2; ++qi)
#pragma unroll
          for (int qj = 0; qj < 2; ++qj)
            acc.d[2 * qi + qj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[qi][s], b[qj][s], acc.d[2 * qi + qj], 0, 0, 0);
    }
  } else {
    const short* P = reinterpret_cast<const short*>(buf);
    const short *Ah = P, *Al = P + kPanel, *Bh = P + 2 * kPanel, *Bl = P + 3 * kPanel;
#pragma unroll
    for (int c = 0; c < kMacStage / 16; ++c) {
      s16x4 ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int ra = (r0 + 16 * h + i) * kLd + 16 * c + 4 * kk;
        const int rb = (c0 + 16 * h + i) * kLd + 16 * c + 4 * kk;
        ah[h] = *reinterpret_cast<const s16x4*>(Ah + ra);
        al[h] = *reinterpret_cast<const s16x4*>(Al + ra);
        bh[h] = *reinterpret_cast<const s16x4*>(Bh + rb);
        bl[h] = *reinterpret_cast<const s16x4*>(Bl + rb);
      }
#pragma unroll
      for (int qi = 0; qi < 2; ++qi)
#pragma unroll
        for (int qj = 0; qj < 2; ++qj) {
          f32x4& d = acc.d[2 * qi + qj];
          d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[qi], bh[qj], d, 0, 0, 0);
          d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[qi], bl[qj], d, 0, 0, 0);
          d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[qi], bh[qj], d, 0, 0, 0);
        }
    }
  }
}

// Adds a tile's elementwise terms (FP64) to the lane's sixteen sums and
// writes y.  Register r holds quarter q = r / 4 of the wave's 32 x 32, row
// 16 (q / 2) + 4 (lane / 16) + r % 4, column 16 (q % 2) + lane % 16.
__device__ inline void finish(double (&v)[16], const MacTile& T, const MacGG* __restrict__ mggs,
                              const double* __restrict__ psi64, double* __restrict__ y, double alpha,
                              double beta, int w, int lane) {
  const int ngg = rfl(T.ngg);
  for (int q = 0; q < ngg; ++q) {
    const MacGG& G = mggs[T.gg0 + q];
    const double c = G.c;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int mt = 32 * (w >> 1) + 16 * ((r >> 2) >> 1) + 4 * (lane >> 4) + (r & 3);
      const int nt = 32 * (w & 1) + 16 * ((r >> 2) & 1) + (lane & 15);
      const int64_t row = G.row[mt];
      const int32_t col = G.col[nt];
      const double x = psi64[(row < 0 ? 0 : row) + (col < 0 ? 0 : col)];
      v[r] += c * G.rs[mt] * G.cs[nt] * x;
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int mt = 32 * (w >> 1) + 16 * ((r >> 2) >> 1) + 4 * (lane >> 4) + (r & 3);
    const int nt = 32 * (w & 1) + 16 * ((r >> 2) & 1) + (lane & 15);
    const int m = T.m0 + mt, n = T.n0 + nt;
    if (m < T.a && n < T.b) {
      const int64_t idx = T.y_off + (int64_t)m * T.ldy + n;
      y[idx] = beta == 0.0 ? alpha * v[r] : alpha * v[r] + beta * y[idx];
    }
  }
}

template <bool kBF16>
__global__ __launch_bounds__(kMacThreads, kMacWGsPerCU) void hpsi_macro(
    const MacTile* __restrict__ tiles, const MacSeg* __restrict__ msegs, const MacGG* __restrict__ mggs,
    const MacItem* __restrict__ items, const int32_t* __restrict__ wg_start,
    const float* __restrict__ dense, int64_t ndense, const float* __restrict__ psi32, int64_t npsi,
    const double* __restrict__ psi64, double* __restrict__ y, double alpha, double beta,
    float* __restrict__ part) {
  __shared__ __align__(16) float lds[2 * Lds<kBF16>::kFloats];
  __shared__ __align__(16) MacSeg sl[kMacSegLds];   // the item's segments
  const int t = threadIdx.x, w = rfl(t >> 6), lane = t & 63;
  const __amdgpu_buffer_rsrc_t rd = rsrc(dense, 4 * ndense), rp = rsrc(psi32, 4 * npsi), rz = rsrc(dense, 0);
  float* const buf0 = lds;
  float* const buf1 = lds + Lds<kBF16>::kFloats;
  const int i0 = wg_start[blockIdx.x], i1 = wg_start[blockIdx.x + 1];
  for (int it = i0; it < i1; ++it) {
    const MacItem I = items[it];
    const MacTile T = tiles[I.tile];
    Acc acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc.d[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int s0 = rfl(I.s0), s1 = rfl(I.s1), ng = rfl(I.ng);
    if (s1 > s0) {
      __syncthreads();   // the previous item is done with LDS
      {   // the item's segment records into LDS
        const uint4* src = reinterpret_cast<const uint4*>(msegs + T.seg0 + I.g0);
        uint4* dst = reinterpret_cast<uint4*>(sl);
        const int n16 = ng * (int)(sizeof(MacSeg) / 16);
        for (int x = t; x < n16; x += kMacThreads) dst[x] = src[x];
      }
      __syncthreads();
      auto next_of = [&](int g) { return g + 1 < ng ? rfl(sl[g + 1].st0) : 0x7fffffff; };
      Fetch f;
      Use u;
      setup_fetch(f, 0, sl[0], next_of(0), T, t);
      setup_use(u, 0, sl[0], next_of(0), T, t);
      // loads of tile stage s (dead past the item), fetch segments in order
      // segment bookkeeping (branches) happens before a step's matrix-core
      // work, so that the step's panel writes and loads are straight-line
      // code the scheduler can interleave with it
      auto adv_fetch = [&](int s) {
        while (s < s1 && s >= f.next) setup_fetch(f, f.seg + 1, sl[f.seg + 1], next_of(f.seg + 1), T, t);
      };
      auto adv_use = [&](int s) {
        while (s < s1 && s >= u.next) setup_use(u, u.seg + 1, sl[u.seg + 1], next_of(u.seg + 1), T, t);
      };
      auto fetch = [&](Raw& R, int s) {   // loads of tile stage s (dead past the item)
        const bool live = s < s1;
        load(R, f, (live ? s : f.st0) - f.st0, live, rd, rp, rz);
      };
      auto put = [&](const Raw& R, int s, float* buf) { stage<kBF16>(R, u, buf); };
      // kDepth stages in flight ahead of the one being written: register set
      // R[(r + 1) % kDepth] holds stage s + 1 when stage s = s0 + r is on the
      // matrix cores (the loop is unrolled so that the sets stay registers)
      constexpr int kDepth = 2;
      Raw R0, R1;
      fetch(R0, s0);
      adv_fetch(s0 + 1);
      fetch(R1, s0 + 1);
      __builtin_amdgcn_sched_barrier(0);
      put(R0, s0, buf0);
      adv_fetch(s0 + kDepth);
      fetch(R0, s0 + kDepth);
      __builtin_amdgcn_sched_barrier(0);
      __syncthreads();
      auto step = [&](float* cur, float* nxt, Raw& Rn, int s) {
        adv_use(s + 1);
        adv_fetch(s + 1 + kDepth);
        __builtin_amdgcn_sched_barrier(0);
        mma<kBF16>(acc, cur, w, lane);
        put(Rn, s + 1, nxt);   // past the item: zeros from dead loads, never read
        fetch(Rn, s + 1 + kDepth);
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();
        return s + 1 < s1;
      };
      for (int s = s0;; s += 2) {
        if (!step(buf0, buf1, R1, s)) break;
        if (!step(buf1, buf0, R0, s + 1)) break;
      }
    }
    // epilogue: a shared tile's share stores its partial sum (added up by
    // hpsi_macro_combine after this kernel); an unshared tile is finished here
    const int nsplit = rfl(T.nsplit);
    if (nsplit > 1) {
      float* mine = part + (int64_t)(T.part0 + I.split) * (kMac * kMac);
#pragma unroll
      for (int r = 0; r < 16; ++r) mine[(w * 16 + r) * 64 + lane] = acc.d[r >> 2][r & 3];
      continue;
    }
    double v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = (double)acc.d[r >> 2][r & 3];
    finish(v, T, mggs, psi64, y, alpha, beta, w, lane);
  }
}

// The shared tiles' partial sums in share order (FP64), their elementwise
// terms, and y: four workgroups of 256 threads per shared tile, workgroup q
// the 32 x 32 quarter that wave q of the main kernel stored, thread T of it
// the four stored entries e = 1024 q + 4T .. + 3 (entry e = (w * 16 + r) * 64
// + lane of the storing wave w, register r, lane).  The loads of eight
// shares, and of four elementwise terms, go out together before their sums.
constexpr int kCombineThreads = 256;
constexpr int kCombineBatch = 8;

__global__ __launch_bounds__(kCombineThreads) void hpsi_macro_combine(
    const MacTile* __restrict__ tiles, const int32_t* __restrict__ shared, const MacGG* __restrict__ mggs,
    const float* __restrict__ part, const double* __restrict__ psi64, double* __restrict__ y, double alpha,
    double beta) {
  const MacTile T = tiles[shared[blockIdx.x >> 2]];
  const int nsplit = rfl(T.nsplit), ngg = rfl(T.ngg);
  const int e0 = (blockIdx.x & 3) * (kMac * kMac / 4) + threadIdx.x * 4;
  const float* p0 = part + (int64_t)T.part0 * (kMac * kMac) + e0;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int s = 0; s < nsplit; s += kCombineBatch) {
    f4 x[kCombineBatch];
#pragma unroll
    for (int u = 0; u < kCombineBatch; ++u)
      x[u] = s + u < nsplit ? *reinterpret_cast<const f4*>(p0 + (int64_t)(s + u) * (kMac * kMac))
                            : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < kCombineBatch; ++u)
      if (s + u < nsplit) {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += (double)x[u][k];
      }
  }
  int mt[4], nt[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = e0 + k, w = e >> 10, r = (e >> 6) & 15, lane = e & 63;
    mt[k] = 32 * (w >> 1) + 16 * ((r >> 2) >> 1) + 4 * (lane >> 4) + (r & 3);
    nt[k] = 32 * (w & 1) + 16 * ((r >> 2) & 1) + (lane & 15);
  }
  for (int q = 0; q < ngg; q += 4) {
    double x[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const MacGG& G = mggs[T.gg0 + (q + u < ngg ? q + u : q)];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t row = G.row[mt[k]];
        const int32_t col = G.col[nt[k]];
        x[u][k] = psi64[(row < 0 ? 0 : row) + (col < 0 ? 0 : col)];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (q + u < ngg) {
        const MacGG& G = mggs[T.gg0 + q + u];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += G.c * G.rs[mt[k]] * G.cs[nt[k]] * x[u][k];
      }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int m = T.m0 + mt[k], n = T.n0 + nt[k];
    if (m < T.a && n < T.b) {
      const int64_t idx = T.y_off + (int64_t)m * T.ldy + n;
      y[idx] = beta == 0.0 ? alpha * v[k] : alpha * v[k] + beta * y[idx];
    }
  }
}

}  // namespace

hipError_t launch_hpsi_macro(bool bf16, int nwg, int nshared, const MacTile* tiles, const MacSeg* segs,
                             const MacGG* ggs, const MacItem* items, const int32_t* wg_start,
                             const int32_t* shared, const float* dense, int64_t ndense, const float* psi32,
                             int64_t npsi, const double* psi64, double* y, double alpha, double beta,
                             float* part, hipStream_t stream, hipEvent_t t0, hipEvent_t t1) {
  if (nwg <= 0) return hipSuccess;
  if (4 * ndense >= ((int64_t)1 << 31) || 4 * npsi >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  hipEvent_t end_main = nshared > 0 ? nullptr : t1;
  if (bf16)
    hipExtLaunchKernelGGL(hpsi_macro<true>, dim3(nwg), dim3(kMacThreads), 0, stream, t0, end_main, 0, tiles,
                          segs, ggs, items, wg_start, dense, ndense, psi32, npsi, psi64, y, alpha, beta, part);
  else
    hipExtLaunchKernelGGL(hpsi_macro<false>, dim3(nwg), dim3(kMacThreads), 0, stream, t0, end_main, 0, tiles,
                          segs, ggs, items, wg_start, dense, ndense, psi32, npsi, psi64, y, alpha, beta, part);
  if (nshared > 0)
    hipExtLaunchKernelGGL(hpsi_macro_combine, dim3(4 * nshared), dim3(kCombineThreads), 0, stream, nullptr, t1,
                          0, tiles, shared, ggs, part, psi64, y, alpha, beta);
  return hipGetLastError();
}

}  // namespace dmrg
