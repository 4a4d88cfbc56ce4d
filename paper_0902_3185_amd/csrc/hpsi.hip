// Superblock product kernels for gfx950 (CDNA4).
//
// One workgroup of 4 wave64s owns one 32 x 32 output tile of one target
// block Y_q and reduces every term that writes it (Y_q += c A Psi_q' B^T;
// paper Sec. 3.3, blocking by effective symmetry).  The dense products run on
// the matrix cores; the four waves split the contraction chunks of all of the
// tile's terms and their partial tiles are summed in LDS in a fixed order, so
// the result does not depend on scheduling.  Terms with identity or gather
// operators on both sides are elementwise and are added in FP64 afterwards.
// No atomics are used on y.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace dmrg {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// Per-precision contraction of one segment's chunks into a wave's 32x32 tile.
//
// SEG_KN: Y[m][n] += c * sum_k A[m][k] * B[k][n], A stored k-major
//         (At[k*lda + m]), B[k][n] = sB[n] * Psi'[k][srcB[n]].
//         Lanes of one contraction index read consecutive m / n: coalesced.
// SEG_MK: Y[m][n] += c * sum_k A[m][k] * Bop[n][k], A[m][k] = sA[m] *
//         Psi'[srcA[m]][k], Bop row-major.  Each lane walks a row along k.
// ---------------------------------------------------------------------------

struct GatherLane {
  int32_t src;
  double s;
  bool ok;
};

__device__ inline GatherLane gather_at(const int32_t* gsrc, const double* gscale, int32_t g,
                                       int32_t idx, int32_t limit) {
  GatherLane r;
  r.ok = idx < limit;
  r.src = idx;
  r.s = 1.0;
  if (r.ok && g >= 0) {
    r.src = gsrc[g + idx];
    r.s = gscale[g + idx];
    r.ok = r.src >= 0;
  }
  return r;
}

// FP32 matrix cores: v_mfma_f32_32x32x2f32.  A[i][k] from lane i + 32k,
// B[k][j] from lane j + 32k; D[i][j] in lane j + 32*((i/4)%2), register
// (i%4) + 4*(i/8).
struct CfgF32 {
  using op_t = float;
  struct Acc {
    f32x16 d;
  };
  __device__ static void zero(Acc& a) {
#pragma unroll
    for (int r = 0; r < 16; ++r) a.d[r] = 0.f;
  }
  __device__ static void seg(Acc& acc, const SegDesc& sg, const TileDesc& t, int ch0, int chs,
                             const op_t* dense, const int32_t* gsrc, const double* gscale,
                             const double* psi, int lane) {
    const int i = lane & 31, kh = lane >> 5;
    const double* P = psi + sg.psi_off;
    const int64_t ldp = sg.psi_ld;
    const int nch = (sg.K + kChunk - 1) / kChunk;
    if (sg.kind == SEG_KN) {
      const op_t* At = dense + sg.op_off;
      const int64_t lda = sg.op_ld;
      const int m = t.m0 + i;
      const bool mok = m < t.a;
      GatherLane gb = gather_at(gsrc, gscale, sg.gB, t.n0 + i, t.b);
      const float cs = (float)sg.c, sb = (float)gb.s;
      for (int ch = ch0; ch < nch; ch += chs) {
        const int k0 = ch * kChunk;
        float av[8], bv[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int k = k0 + 2 * s + kh;
          const bool kok = k < sg.K;
          av[s] = (mok && kok) ? cs * At[k * lda + m] : 0.f;
          bv[s] = (gb.ok && kok) ? sb * (float)P[k * ldp + gb.src] : 0.f;
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) acc.d = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s], bv[s], acc.d, 0, 0, 0);
      }
    } else {
      GatherLane ga = gather_at(gsrc, gscale, sg.gA, t.m0 + i, t.a);
      const double* Arow = P + (int64_t)(ga.ok ? ga.src : 0) * ldp;
      const int n = t.n0 + i;
      const bool nok = n < t.b;
      const op_t* Brow = dense + sg.op_off + (int64_t)(nok ? n : 0) * sg.op_ld;
      const float ca = (float)(sg.c * ga.s);
      for (int ch = ch0; ch < nch; ch += chs) {
        const int k0 = ch * kChunk + 8 * kh;
        float av[8], bv[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int k = k0 + s;
          const bool kok = k < sg.K;
          av[s] = (ga.ok && kok) ? ca * (float)Arow[k] : 0.f;
          bv[s] = (nok && kok) ? Brow[k] : 0.f;
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) acc.d = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s], bv[s], acc.d, 0, 0, 0);
      }
    }
  }
  __device__ static double value(const Acc& a, int r) { return (double)a.d[r]; }
  __device__ static void coords(int lane, int r, int& row, int& col) {
    row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    col = lane & 31;
  }
  static constexpr int kRegs = 16;
};

// FP64 matrix cores: v_mfma_f64_16x16x4f64 on a 2 x 2 grid of 16x16 blocks.
// A[i][k] from lane i + 16k, B[k][j] from lane j + 16k; D[i][j] in lane
// j + 16*(i%4), register i/4 (rows interleaved over the four lane groups).
struct CfgF64 {
  using op_t = double;
  struct Acc {
    f64x4 d[4];  // block (bi, bj) at d[2*bi + bj]
  };
  __device__ static void zero(Acc& a) {
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) a.d[b][r] = 0.0;
  }
  __device__ static void seg(Acc& acc, const SegDesc& sg, const TileDesc& t, int ch0, int chs,
                             const op_t* dense, const int32_t* gsrc, const double* gscale,
                             const double* psi, int lane) {
    const int i = lane & 15, kq = lane >> 4;
    const double* P = psi + sg.psi_off;
    const int64_t ldp = sg.psi_ld;
    const int nch = (sg.K + kChunk - 1) / kChunk;
    if (sg.kind == SEG_KN) {
      const op_t* At = dense + sg.op_off;
      const int64_t lda = sg.op_ld;
      const int m0 = t.m0 + i, m1 = t.m0 + 16 + i;
      const bool mok0 = m0 < t.a, mok1 = m1 < t.a;
      GatherLane g0 = gather_at(gsrc, gscale, sg.gB, t.n0 + i, t.b);
      GatherLane g1 = gather_at(gsrc, gscale, sg.gB, t.n0 + 16 + i, t.b);
      const double c = sg.c;
      for (int ch = ch0; ch < nch; ch += chs) {
        const int k0 = ch * kChunk;
        double a0[4], a1[4], b0[4], b1[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = k0 + 4 * s + kq;
          const bool kok = k < sg.K;
          a0[s] = (mok0 && kok) ? c * At[k * lda + m0] : 0.0;
          a1[s] = (mok1 && kok) ? c * At[k * lda + m1] : 0.0;
          b0[s] = (g0.ok && kok) ? g0.s * P[k * ldp + g0.src] : 0.0;
          b1[s] = (g1.ok && kok) ? g1.s * P[k * ldp + g1.src] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          acc.d[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[s], b0[s], acc.d[0], 0, 0, 0);
          acc.d[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[s], b1[s], acc.d[1], 0, 0, 0);
          acc.d[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[s], b0[s], acc.d[2], 0, 0, 0);
          acc.d[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[s], b1[s], acc.d[3], 0, 0, 0);
        }
      }
    } else {
      GatherLane ga0 = gather_at(gsrc, gscale, sg.gA, t.m0 + i, t.a);
      GatherLane ga1 = gather_at(gsrc, gscale, sg.gA, t.m0 + 16 + i, t.a);
      const double* A0 = P + (int64_t)(ga0.ok ? ga0.src : 0) * ldp;
      const double* A1 = P + (int64_t)(ga1.ok ? ga1.src : 0) * ldp;
      const int n0 = t.n0 + i, n1 = t.n0 + 16 + i;
      const bool nok0 = n0 < t.b, nok1 = n1 < t.b;
      const op_t* B0 = dense + sg.op_off + (int64_t)(nok0 ? n0 : 0) * sg.op_ld;
      const op_t* B1 = dense + sg.op_off + (int64_t)(nok1 ? n1 : 0) * sg.op_ld;
      const double c0 = sg.c * ga0.s, c1 = sg.c * ga1.s;
      for (int ch = ch0; ch < nch; ch += chs) {
        const int k0 = ch * kChunk + 4 * kq;
        double a0[4], a1[4], b0[4], b1[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = k0 + s;
          const bool kok = k < sg.K;
          a0[s] = (ga0.ok && kok) ? c0 * A0[k] : 0.0;
          a1[s] = (ga1.ok && kok) ? c1 * A1[k] : 0.0;
          b0[s] = (nok0 && kok) ? B0[k] : 0.0;
          b1[s] = (nok1 && kok) ? B1[k] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          acc.d[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[s], b0[s], acc.d[0], 0, 0, 0);
          acc.d[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[s], b1[s], acc.d[1], 0, 0, 0);
          acc.d[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[s], b0[s], acc.d[2], 0, 0, 0);
          acc.d[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[s], b1[s], acc.d[3], 0, 0, 0);
        }
      }
    }
  }
  __device__ static double value(const Acc& a, int r) { return a.d[r >> 2][r & 3]; }
  __device__ static void coords(int lane, int r, int& row, int& col) {
    const int b = r >> 2, bi = b >> 1, bj = b & 1;
    row = 16 * bi + 4 * (r & 3) + (lane >> 4);
    col = 16 * bj + (lane & 15);
  }
  static constexpr int kRegs = 16;
};

// Elementwise term: c * sA[m] * sB[n] * Psi'[srcA[m]][srcB[n]].
__device__ inline double gg_term(const SegDesc& sg, const TileDesc& t, int m, int n,
                                 const int32_t* gsrc, const double* gscale, const double* psi) {
  GatherLane ga = gather_at(gsrc, gscale, sg.gA, m, t.a);
  GatherLane gb = gather_at(gsrc, gscale, sg.gB, n, t.b);
  if (!ga.ok || !gb.ok) return 0.0;
  return sg.c * ga.s * gb.s * psi[sg.psi_off + (int64_t)ga.src * sg.psi_ld + gb.src];
}

// ---------------------------------------------------------------------------
// y = alpha * H psi + beta * y.  Workgroup slot b takes tile order[b]
// (-1: idle slot), so that the blocks of one target pair share an XCD.
//
// Phase 0  the gather entries of the tile's 32 rows / columns for every
//          matrix-core segment go to LDS; the elementwise (gather-gather)
//          terms of each thread's output elements are loaded.
// Phase 1  the tile's contraction chunks (all matrix-core segments, in
//          order) are dealt round-robin to the waves; each wave loads its
//          next chunk while the current one runs on the matrix cores.
// Phase 2  the waves' 32x32 partial tiles are summed through LDS in wave
//          order, the elementwise terms added in FP64, and y written.
// ---------------------------------------------------------------------------
constexpr int kMaxSeg = 32;   // segments per target block (checked by the host)
constexpr int kMaxGG = 8;     // elementwise segments whose operands are loaded early

struct TileShared {
  int32_t gsrc[kMaxSeg][kTile];
  float gscl[kMaxSeg][kTile];
};

// Gather entry of index idx (row or column of the output block) for segment sg.
__device__ inline void gather_entry(const SegDesc& sg, const TileDesc& t, int i,
                                    const int32_t* gsrc, const double* gscale, int32_t& src,
                                    float& scl) {
  const bool kn = sg.kind == SEG_KN;
  const int idx = (kn ? t.n0 : t.m0) + i;
  const int limit = kn ? t.b : t.a;
  const int32_t g = kn ? sg.gB : sg.gA;
  src = -1;
  scl = 0.f;
  if (idx < limit) {
    if (g < 0) {
      src = idx;
      scl = 1.f;
    } else {
      src = gsrc[g + idx];
      scl = (float)gscale[g + idx];
    }
  }
}

struct F32Tile {
  using op_t = float;
  using red_t = float;
  static constexpr int kWaves = 16;
  struct Acc {
    f32x16 d;
  };
  struct Regs {
    float a[8], b[8];
  };
  __device__ static void zero(Acc& a) {
#pragma unroll
    for (int r = 0; r < 16; ++r) a.d[r] = 0.f;
  }
  __device__ static void load(Regs& R, const SegDesc& sg, const TileDesc& t, int ch, int si,
                              const TileShared& sh, const op_t* dense, const double* psi,
                              int lane) {
    const int i = lane & 31, kh = lane >> 5;
    const double* P = psi + sg.psi_off;
    const int64_t ldp = sg.psi_ld;
    const int32_t src = sh.gsrc[si][i];
    const float scl = sh.gscl[si][i];
    if (sg.kind == SEG_KN) {
      const op_t* At = dense + sg.op_off;
      const int64_t lda = sg.op_ld;
      const int m = t.m0 + i;
      const bool mok = m < t.a;
      const bool nok = src >= 0;
      const float cs = (float)sg.c;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int k = ch * kChunk + 2 * s + kh;
        const bool kok = k < sg.K;
        R.a[s] = (mok && kok) ? cs * At[k * lda + m] : 0.f;
        R.b[s] = (nok && kok) ? scl * (float)P[k * ldp + src] : 0.f;
      }
    } else {
      const bool mok = src >= 0;
      const double* Arow = P + (int64_t)(mok ? src : 0) * ldp;
      const int n = t.n0 + i;
      const bool nok = n < t.b;
      const op_t* Brow = dense + sg.op_off + (int64_t)(nok ? n : 0) * sg.op_ld;
      const float ca = (float)sg.c * scl;
      const int k0 = ch * kChunk + 8 * kh;
      if (k0 + 8 <= sg.K) {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          R.a[s] = mok ? ca * (float)Arow[k0 + s] : 0.f;
          R.b[s] = nok ? Brow[k0 + s] : 0.f;
        }
      } else {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const bool kok = k0 + s < sg.K;
          R.a[s] = (mok && kok) ? ca * (float)Arow[k0 + s] : 0.f;
          R.b[s] = (nok && kok) ? Brow[k0 + s] : 0.f;
        }
      }
    }
  }
  __device__ static void mma(Acc& acc, const Regs& R) {
#pragma unroll
    for (int s = 0; s < 8; ++s) acc.d = __builtin_amdgcn_mfma_f32_32x32x2f32(R.a[s], R.b[s], acc.d, 0, 0, 0);
  }
  static constexpr int kRegs = 16;
  __device__ static float value(const Acc& a, int r) { return a.d[r]; }
  __device__ static void coords(int lane, int r, int& row, int& col) {
    row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    col = lane & 31;
  }
};

struct F64Tile {
  using op_t = double;
  using red_t = double;
  static constexpr int kWaves = 8;
  struct Acc {
    f64x4 d[4];
  };
  struct Regs {
    double a0[4], a1[4], b0[4], b1[4];
  };
  __device__ static void zero(Acc& a) {
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) a.d[b][r] = 0.0;
  }
  __device__ static void load(Regs& R, const SegDesc& sg, const TileDesc& t, int ch, int si,
                              const TileShared& sh, const op_t* dense, const double* psi,
                              int lane) {
    const int i = lane & 15, kq = lane >> 4;
    const double* P = psi + sg.psi_off;
    const int64_t ldp = sg.psi_ld;
    const int32_t src0 = sh.gsrc[si][i], src1 = sh.gsrc[si][16 + i];
    const double scl0 = sh.gscl[si][i], scl1 = sh.gscl[si][16 + i];
    if (sg.kind == SEG_KN) {
      const op_t* At = dense + sg.op_off;
      const int64_t lda = sg.op_ld;
      const int m0 = t.m0 + i, m1 = t.m0 + 16 + i;
      const bool mok0 = m0 < t.a, mok1 = m1 < t.a;
      const double c = sg.c;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = ch * kChunk + 4 * s + kq;
        const bool kok = k < sg.K;
        R.a0[s] = (mok0 && kok) ? c * At[k * lda + m0] : 0.0;
        R.a1[s] = (mok1 && kok) ? c * At[k * lda + m1] : 0.0;
        R.b0[s] = (src0 >= 0 && kok) ? scl0 * P[k * ldp + src0] : 0.0;
        R.b1[s] = (src1 >= 0 && kok) ? scl1 * P[k * ldp + src1] : 0.0;
      }
    } else {
      const double* A0 = P + (int64_t)(src0 >= 0 ? src0 : 0) * ldp;
      const double* A1 = P + (int64_t)(src1 >= 0 ? src1 : 0) * ldp;
      const int n0 = t.n0 + i, n1 = t.n0 + 16 + i;
      const bool nok0 = n0 < t.b, nok1 = n1 < t.b;
      const op_t* B0 = dense + sg.op_off + (int64_t)(nok0 ? n0 : 0) * sg.op_ld;
      const op_t* B1 = dense + sg.op_off + (int64_t)(nok1 ? n1 : 0) * sg.op_ld;
      const double c0 = sg.c * scl0, c1 = sg.c * scl1;
      const int k0 = ch * kChunk + 4 * kq;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const bool kok = k0 + s < sg.K;
        R.a0[s] = (src0 >= 0 && kok) ? c0 * A0[k0 + s] : 0.0;
        R.a1[s] = (src1 >= 0 && kok) ? c1 * A1[k0 + s] : 0.0;
        R.b0[s] = (nok0 && kok) ? B0[k0 + s] : 0.0;
        R.b1[s] = (nok1 && kok) ? B1[k0 + s] : 0.0;
      }
    }
  }
  __device__ static void mma(Acc& acc, const Regs& R) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      acc.d[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(R.a0[s], R.b0[s], acc.d[0], 0, 0, 0);
      acc.d[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(R.a0[s], R.b1[s], acc.d[1], 0, 0, 0);
      acc.d[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(R.a1[s], R.b0[s], acc.d[2], 0, 0, 0);
      acc.d[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(R.a1[s], R.b1[s], acc.d[3], 0, 0, 0);
    }
  }
  static constexpr int kRegs = 16;
  __device__ static double value(const Acc& a, int r) { return a.d[r >> 2][r & 3]; }
  __device__ static void coords(int lane, int r, int& row, int& col) {
    const int b = r >> 2, bi = b >> 1, bj = b & 1;
    row = 16 * bi + 4 * (r & 3) + (lane >> 4);
    col = 16 * bj + (lane & 15);
  }
};

// BF16 hi/lo split on the matrix cores: v_mfma_f32_32x32x16_bf16, A[i][k]
// from lane i + 32*(k/8), element k%8 (B likewise with column j); D as in the
// FP32 32x32 layout.  Every FP32 operand x is split into hi = bf16(x) and
// lo = bf16(x - hi); a product is hi*hi + hi*lo + lo*hi (the lo*lo term and
// the rounding of lo leave a relative error of about 2^-16), accumulated in
// FP32.  The operators are read from the FP32 pool and split on load.
struct BF16Tile {
  using op_t = float;
  using red_t = float;
  static constexpr int kWaves = 16;
  struct Acc {
    f32x16 d;
  };
  struct Regs {
    bf16x8 ah, al, bh, bl;
  };
  __device__ static void zero(Acc& a) {
#pragma unroll
    for (int r = 0; r < 16; ++r) a.d[r] = 0.f;
  }
  __device__ static void split(const float (&x)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const __bf16 h = (__bf16)x[j];
      hi[j] = h;
      lo[j] = (__bf16)(x[j] - (float)h);
    }
  }
  __device__ static void load(Regs& R, const SegDesc& sg, const TileDesc& t, int ch, int si,
                              const TileShared& sh, const op_t* dense, const double* psi,
                              int lane) {
    const int i = lane & 31, kh = lane >> 5;
    const double* P = psi + sg.psi_off;
    const int64_t ldp = sg.psi_ld;
    const int32_t src = sh.gsrc[si][i];
    const float scl = sh.gscl[si][i];
    const int k0 = ch * kChunk + 8 * kh;
    float a[8], b[8];
    if (sg.kind == SEG_KN) {
      const op_t* At = dense + sg.op_off;
      const int64_t lda = sg.op_ld;
      const int m = t.m0 + i;
      const bool mok = m < t.a;
      const bool nok = src >= 0;
      const float cs = (float)sg.c;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = k0 + j;
        const bool kok = k < sg.K;
        a[j] = (mok && kok) ? cs * At[k * lda + m] : 0.f;
        b[j] = (nok && kok) ? scl * (float)P[k * ldp + src] : 0.f;
      }
    } else {
      const bool mok = src >= 0;
      const double* Arow = P + (int64_t)(mok ? src : 0) * ldp;
      const int n = t.n0 + i;
      const bool nok = n < t.b;
      const op_t* Brow = dense + sg.op_off + (int64_t)(nok ? n : 0) * sg.op_ld;
      const float ca = (float)sg.c * scl;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const bool kok = k0 + j < sg.K;
        a[j] = (mok && kok) ? ca * (float)Arow[k0 + j] : 0.f;
        b[j] = (nok && kok) ? Brow[k0 + j] : 0.f;
      }
    }
    split(a, R.ah, R.al);
    split(b, R.bh, R.bl);
  }
  __device__ static void mma(Acc& acc, const Regs& R) {
    acc.d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(R.ah, R.bh, acc.d, 0, 0, 0);
    acc.d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(R.ah, R.bl, acc.d, 0, 0, 0);
    acc.d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(R.al, R.bh, acc.d, 0, 0, 0);
  }
  static constexpr int kRegs = 16;
  __device__ static float value(const Acc& a, int r) { return a.d[r]; }
  __device__ static void coords(int lane, int r, int& row, int& col) {
    row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    col = lane & 31;
  }
};

// Matrix-core segment holding global chunk g of the tile.
__device__ inline int seg_of_chunk(const SegDesc* segs, const TileDesc& t, int g) {
  int found = 0;
  for (int s = 1; s < t.ngemm; ++s)
    if (g >= segs[t.seg0 + s].ch0) found = s;
  return found;
}

template <class Cfg>
__global__ __launch_bounds__(Cfg::kWaves * 64) void hpsi_grouped(
    const int32_t* __restrict__ order, const TileDesc* __restrict__ tiles,
    const SegDesc* __restrict__ segs, const typename Cfg::op_t* __restrict__ dense,
    const int32_t* __restrict__ gsrc, const double* __restrict__ gscale,
    const double* __restrict__ psi, double* __restrict__ y, double alpha, double beta) {
  constexpr int kW = Cfg::kWaves;
  constexpr int kT = kW * 64;
  constexpr int kPer = kTile * kTile / kT;   // output elements per thread
  __shared__ TileShared sh;
  __shared__ typename Cfg::red_t red[kW][kTile * kTile];
  const int ti = order ? order[blockIdx.x] : (int)blockIdx.x;
  if (ti < 0) return;
  const TileDesc t = tiles[ti];
  // the wave index is uniform in a wave: say so, so that chunk and segment
  // bookkeeping stays in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;

  // phase 0: gather entries of the matrix-core segments; elementwise operands
  for (int x = threadIdx.x; x < t.ngemm * kTile; x += kT) {
    const int s = x / kTile, i = x % kTile;
    gather_entry(segs[t.seg0 + s], t, i, gsrc, gscale, sh.gsrc[s][i], sh.gscl[s][i]);
  }
  const int ngg = t.nseg - t.ngemm;
  double gg[kPer];
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int el = threadIdx.x + e * kT;
    const int m = t.m0 + el / kTile, n = t.n0 + el % kTile;
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxGG; ++q)
      if (q < ngg) v += gg_term(segs[t.seg0 + t.ngemm + q], t, m, n, gsrc, gscale, psi);
    gg[e] = v;
  }
  __syncthreads();

  // phase 1: contraction chunks, round-robin over the waves, one chunk ahead
  typename Cfg::Acc acc;
  Cfg::zero(acc);
  const int nw = t.nchunk < kW ? t.nchunk : kW;   // waves that get work
  if (wave < t.nchunk) {
    // two register buffers, used alternately: load chunk g + kW while chunk g
    // is on the matrix cores
    typename Cfg::Regs ra, rb;
    auto fetch = [&](typename Cfg::Regs& R, int g) {
      const int si = seg_of_chunk(segs, t, g);
      const SegDesc sg = segs[t.seg0 + si];
      Cfg::load(R, sg, t, g - sg.ch0, si, sh, dense, psi, lane);
    };
    int g = wave;
    fetch(ra, g);
    for (;;) {
      const int g2 = g + kW;
      if (g2 < t.nchunk) fetch(rb, g2);
      Cfg::mma(acc, ra);
      if (g2 >= t.nchunk) break;
      const int g3 = g2 + kW;
      if (g3 < t.nchunk) fetch(ra, g3);
      Cfg::mma(acc, rb);
      if (g3 >= t.nchunk) break;
      g = g3;
    }
#pragma unroll
    for (int r = 0; r < Cfg::kRegs; ++r) {
      int row, col;
      Cfg::coords(lane, r, row, col);
      red[wave][row * kTile + col] = Cfg::value(acc, r);
    }
  }
  __syncthreads();

  // phase 2: fixed-order sum, elementwise terms, y
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int el = threadIdx.x + e * kT;
    const int m = t.m0 + el / kTile, n = t.n0 + el % kTile;
    double v = 0.0;
    for (int w = 0; w < nw; ++w) v += (double)red[w][el];
    v += gg[e];
    for (int q = kMaxGG; q < ngg; ++q) v += gg_term(segs[t.seg0 + t.ngemm + q], t, m, n, gsrc, gscale, psi);
    if (m < t.a && n < t.b) {
      const int64_t idx = t.y_off + (int64_t)m * t.ldy + n;
      y[idx] = beta == 0.0 ? alpha * v : alpha * v + beta * y[idx];
    }
  }
}

// ---------------------------------------------------------------------------
// Per-term inner products <G, c_k^{-1} * term_k tile> for grad_c:
// each wave takes whole segments of the tile; partial[blockIdx.x * stride + s].
// The segment's own coefficient is divided out by computing with c = 1.
// ---------------------------------------------------------------------------
template <class Cfg>
__global__ __launch_bounds__(256) void term_dots(const TileDesc* __restrict__ tiles,
                                                 const SegDesc* __restrict__ segs,
                                                 const typename Cfg::op_t* __restrict__ dense,
                                                 const int32_t* __restrict__ gsrc,
                                                 const double* __restrict__ gscale,
                                                 const double* __restrict__ psi,
                                                 const double* __restrict__ g,
                                                 double* __restrict__ partial, int stride) {
  const TileDesc t = tiles[blockIdx.x];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int s = wave; s < t.nseg; s += 4) {
    SegDesc sg = segs[t.seg0 + s];
    sg.c = 1.0;
    double sum = 0.0;
    if (sg.kind == SEG_GG) {
      for (int e = lane; e < kTile * kTile; e += 64) {
        const int m = t.m0 + e / kTile, n = t.n0 + e % kTile;
        if (m < t.a && n < t.b)
          sum += g[t.y_off + (int64_t)m * t.b + n] * gg_term(sg, t, m, n, gsrc, gscale, psi);
      }
    } else {
      typename Cfg::Acc acc;
      Cfg::zero(acc);
      Cfg::seg(acc, sg, t, 0, 1, dense, gsrc, gscale, psi, lane);
#pragma unroll
      for (int r = 0; r < Cfg::kRegs; ++r) {
        int row, col;
        Cfg::coords(lane, r, row, col);
        const int m = t.m0 + row, n = t.n0 + col;
        if (m < t.a && n < t.b) sum += g[t.y_off + (int64_t)m * t.b + n] * Cfg::value(acc, r);
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    if (lane == 0) partial[(int64_t)blockIdx.x * stride + s] = sum;
  }
}

// ---------------------------------------------------------------------------
// The plain FP64 baseline: y *= beta, then one launch per (term, target
// block), each a 16 x 16 LDS-tiled FMA product or an elementwise pass.
// ---------------------------------------------------------------------------
__global__ void scale_vec(double* __restrict__ y, int64_t n, double beta) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = beta == 0.0 ? 0.0 : beta * y[i];
}

__global__ __launch_bounds__(256) void plain_segment(SegDesc sg, TileDesc t,
                                                     const double* __restrict__ dense,
                                                     const int32_t* __restrict__ gsrc,
                                                     const double* __restrict__ gscale,
                                                     const double* __restrict__ psi,
                                                     double* __restrict__ y, double alpha) {
  __shared__ double As[16][17], Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m = blockIdx.y * 16 + ty, n = blockIdx.x * 16 + tx;
  const double* P = psi + sg.psi_off;
  double acc = 0.0;
  if (sg.kind == SEG_GG) {
    if (m < t.a && n < t.b) acc = gg_term(sg, t, m, n, gsrc, gscale, psi);
  } else {
    for (int k0 = 0; k0 < sg.K; k0 += 16) {
      // A tile rows m (block rows), columns k; B tile rows k, columns n
      {
        const int mm = blockIdx.y * 16 + ty, kk = k0 + tx;
        double v = 0.0;
        if (mm < t.a && kk < sg.K) {
          if (sg.kind == SEG_KN) {
            v = dense[sg.op_off + (int64_t)kk * sg.op_ld + mm];
          } else {
            GatherLane ga = gather_at(gsrc, gscale, sg.gA, mm, t.a);
            if (ga.ok) v = ga.s * P[(int64_t)ga.src * sg.psi_ld + kk];
          }
        }
        As[ty][tx] = v;
      }
      {
        const int kk = k0 + ty, nn = blockIdx.x * 16 + tx;
        double v = 0.0;
        if (nn < t.b && kk < sg.K) {
          if (sg.kind == SEG_KN) {
            GatherLane gb = gather_at(gsrc, gscale, sg.gB, nn, t.b);
            if (gb.ok) v = gb.s * P[(int64_t)kk * sg.psi_ld + gb.src];
          } else {
            v = dense[sg.op_off + (int64_t)nn * sg.op_ld + kk];
          }
        }
        Bs[ty][tx] = v;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 16; ++k) acc += As[ty][k] * Bs[k][tx];
      __syncthreads();
    }
    acc *= sg.c;
  }
  if (m < t.a && n < t.b) y[t.y_off + (int64_t)m * t.b + n] += alpha * acc;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_hpsi(int prec, int nslots, const int32_t* order, const TileDesc* tiles,
                       const SegDesc* segs, const void* dense, const int32_t* gsrc,
                       const double* gscale, const double* psi, double* y, double alpha,
                       double beta, hipStream_t stream) {
  if (nslots <= 0) return hipSuccess;
  if (prec == kPrecF32) {
    hipLaunchKernelGGL(hpsi_grouped<F32Tile>, dim3(nslots), dim3(F32Tile::kWaves * 64), 0, stream,
                       order, tiles, segs, (const float*)dense, gsrc, gscale, psi, y, alpha, beta);
  } else if (prec == kPrecBF16X3) {
    hipLaunchKernelGGL(hpsi_grouped<BF16Tile>, dim3(nslots), dim3(BF16Tile::kWaves * 64), 0,
                       stream, order, tiles, segs, (const float*)dense, gsrc, gscale, psi, y, alpha,
                       beta);
  } else {
    hipLaunchKernelGGL(hpsi_grouped<F64Tile>, dim3(nslots), dim3(F64Tile::kWaves * 64), 0, stream,
                       order, tiles, segs, (const double*)dense, gsrc, gscale, psi, y, alpha, beta);
  }
  return hipGetLastError();
}

hipError_t launch_term_dots(int prec, int ntiles, const TileDesc* tiles, const SegDesc* segs,
                            const void* dense, const int32_t* gsrc, const double* gscale,
                            const double* psi, const double* g, double* partial, int stride,
                            hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  if (prec == kPrecF32) {
    hipLaunchKernelGGL(term_dots<CfgF32>, dim3(ntiles), dim3(256), 0, stream, tiles, segs,
                       (const float*)dense, gsrc, gscale, psi, g, partial, stride);
  } else {
    hipLaunchKernelGGL(term_dots<CfgF64>, dim3(ntiles), dim3(256), 0, stream, tiles, segs,
                       (const double*)dense, gsrc, gscale, psi, g, partial, stride);
  }
  return hipGetLastError();
}

hipError_t launch_plain(const std::vector<std::pair<SegDesc, TileDesc>>& work, int64_t D,
                        const double* dense, const int32_t* gsrc, const double* gscale,
                        const double* psi, double* y, double alpha, double beta,
                        hipStream_t stream) {
  hipLaunchKernelGGL(scale_vec, dim3((unsigned)((D + 255) / 256)), dim3(256), 0, stream, y, D, beta);
  for (const auto& w : work) {
    const TileDesc& t = w.second;
    dim3 grid((t.b + 15) / 16, (t.a + 15) / 16);
    hipLaunchKernelGGL(plain_segment, grid, dim3(256), 0, stream, w.first, t, dense, gsrc, gscale,
                       psi, y, alpha);
  }
  return hipGetLastError();
}

}  // namespace dmrg
