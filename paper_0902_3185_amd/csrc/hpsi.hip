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
#include <hip/hip_ext.h>

#include "kernels.h"

namespace dmrg {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

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
// y = alpha * H psi + beta * y.  Workgroup slot b owns the 32 x 32 output
// tile described by image b (see plan.h): the host orders the slots so that
// the blocks of one target pair share an XCD.
//
// Phase 0  the image is copied into LDS (one coalesced read).
// Phase 1  the tile's contraction chunks (all matrix-core segments, in
//          order) are dealt round-robin to the waves.  A chunk's operands
//          are loaded raw into registers two chunks ahead and converted,
//          scaled and masked only when the chunk goes to the matrix cores,
//          so no load is waited for at issue.  Out-of-range rows, columns
//          and contraction indices load from clamped in-range addresses and
//          are zeroed at conversion.  The elementwise terms' psi entries are
//          loaded together with the first chunks and summed in FP64.
// Phase 2  the waves' 32x32 partial tiles are summed through LDS in wave
//          order (FP64), the elementwise terms added, and y written.
//
// Contraction index of element s of a lane's chunk registers: FP32 and
// BF16 k = 8*(lane/32) + s, FP64 k = 4*(lane/16) + s (A and B agree, so the
// order inside a chunk is immaterial).
// ---------------------------------------------------------------------------
constexpr int kMaxGG = 8;     // elementwise segments whose operands are loaded early

__device__ inline int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ inline const ImgHeader& img_header(const uint32_t* img) {
  return *reinterpret_cast<const ImgHeader*>(img);
}
__device__ inline const ImgSeg& img_seg(const uint32_t* img, int s) {
  return *reinterpret_cast<const ImgSeg*>(img + kHdrWords + s * kSegWords);
}
__device__ inline const ImgGG& img_gg(const uint32_t* img, int ngemm, int q) {
  return *reinterpret_cast<const ImgGG*>(img + kHdrWords + ngemm * kSegWords + q * kGGWords);
}

// Tile geometry, uniform over the workgroup.
struct TileGeo {
  int a, b, m0, n0;
};

// FP32 matrix cores, v_mfma_f32_32x32x2f32: A[i][k] from lane i + 32k,
// B[k][j] from lane j + 32k; D[i][j] in lane j + 32*((i/4)%2), register
// (i%4) + 4*(i/8).  One chunk is 8 instructions; element s of lane half h
// carries k = 8h + s.
struct F32Tile {
  using op_t = float;
  using red_t = float;
  static constexpr int kWaves = 16;
  struct Acc {
    f32x16 d;
  };
  struct Raw {
    float f[8];    // SEG_KN: A;  SEG_MK: B
    double d[8];   // SEG_KN: B;  SEG_MK: A  (psi)
  };
  __device__ static void zero(Acc& a) {
#pragma unroll
    for (int r = 0; r < 16; ++r) a.d[r] = 0.f;
  }
  template <bool kStage>
  __device__ static void load(Raw& R, const ImgSeg& sg, int kind, int K, int ch, const TileGeo& g,
                              const op_t* dense, const double* psi, int lane) {
    const int i = lane & 31, kb = ch * kChunk + 8 * (lane >> 5);
    if (kind == SEG_KN) {
      const op_t* At = dense + sg.op_off + min(g.m0 + i, g.a - 1);
      const int64_t lda = sg.op_ld;
      const double* P = psi + sg.psi_off + max(sg.src[i], 0);
      const int64_t ldp = sg.psi_ld;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int64_t k = min(kb + s, K - 1);
        R.f[s] = At[k * lda];
        R.d[s] = P[k * ldp];
      }
    } else if (!kStage) {
      // each lane walks its own row along k with 16-byte loads (rows are
      // only element-aligned, which the memory system takes for vector loads)
      const double* Arow = psi + sg.psi_off + (int64_t)max(sg.src[i], 0) * sg.psi_ld;
      const op_t* Brow = dense + sg.op_off + (int64_t)min(g.n0 + i, g.b - 1) * sg.op_ld;
      if (K - (ch + 1) * kChunk >= 0) {   // whole chunk in range (uniform)
#pragma unroll
        for (int s = 0; s < 8; s += 2) {
          d2 t;
          __builtin_memcpy(&t, Arow + kb + s, sizeof(t));
          R.d[s] = t.x;
          R.d[s + 1] = t.y;
        }
#pragma unroll
        for (int s = 0; s < 8; s += 4) {
          f4 t;
          __builtin_memcpy(&t, Brow + kb + s, sizeof(t));
          R.f[s] = t.x;
          R.f[s + 1] = t.y;
          R.f[s + 2] = t.z;
          R.f[s + 3] = t.w;
        }
      } else {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int k = min(kb + s, K - 1);
          R.d[s] = Arow[k];
          R.f[s] = Brow[k];
        }
      }
    } else {
      // whole rows per group of lanes, so that each load instruction covers
      // few cache lines: A rows are 16 doubles, 8 lanes x 16 bytes per row,
      // 8 rows per instruction; B rows are 16 floats, 4 lanes x 16 bytes, 16
      // rows per instruction.  operands() transposes them through LDS.
      const int q8 = lane & 7, r8 = lane >> 3, q4 = lane & 3, r4 = lane >> 2;
      const int kc = ch * kChunk;
      const bool full = K - (ch + 1) * kChunk >= 0;   // whole chunk in range (uniform)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double* Arow = psi + sg.psi_off + (int64_t)max(sg.src[8 * j + r8], 0) * sg.psi_ld;
        if (full) {
          d2 t;
          __builtin_memcpy(&t, Arow + kc + 2 * q8, sizeof(t));
          R.d[2 * j] = t.x;
          R.d[2 * j + 1] = t.y;
        } else {
          R.d[2 * j] = Arow[min(kc + 2 * q8, K - 1)];
          R.d[2 * j + 1] = Arow[min(kc + 2 * q8 + 1, K - 1)];
        }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const op_t* Brow = dense + sg.op_off + (int64_t)min(g.n0 + 16 * j + r4, g.b - 1) * sg.op_ld;
        if (full) {
          f4 t;
          __builtin_memcpy(&t, Brow + kc + 4 * q4, sizeof(t));
          R.f[4 * j] = t.x;
          R.f[4 * j + 1] = t.y;
          R.f[4 * j + 2] = t.z;
          R.f[4 * j + 3] = t.w;
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) R.f[4 * j + t] = Brow[min(kc + 4 * q4 + t, K - 1)];
        }
      }
    }
  }
  // LDS staging of one wave's row-walking chunk: A and B as [row][k] floats,
  // rows padded to kStageLd (16-byte aligned rows).
  static constexpr int kStageLd = 20;
  static constexpr int kStageFloats = 2 * kTile * kStageLd;   // per wave
  // operands of one chunk in FP32, scaled and masked
  template <bool kStage>
  __device__ static void operands(const Raw& R, const ImgSeg& sg, int kind, int K, int ch,
                                  const TileGeo& g, int lane, float* stage, float (&a)[8],
                                  float (&b)[8]) {
    const int i = lane & 31, kh = lane >> 5, kv = K - ch * kChunk - 8 * kh;
    const int src = sg.src[i];
    if (kind == SEG_KN) {
      const float cA = g.m0 + i < g.a ? (float)sg.c : 0.f;
      const float sB = src >= 0 ? (float)sg.scl[i] : 0.f;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        a[s] = s < kv ? cA * R.f[s] : 0.f;
        b[s] = s < kv ? sB * (float)R.d[s] : 0.f;
      }
    } else if (!kStage) {
      const float cA = src >= 0 ? (float)(sg.c * sg.scl[i]) : 0.f;
      const float sB = g.n0 + i < g.b ? 1.f : 0.f;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        a[s] = s < kv ? cA * (float)R.d[s] : 0.f;
        b[s] = s < kv ? sB * R.f[s] : 0.f;
      }
    } else {
      // transpose through the wave's LDS stage: rows as loaded, then each
      // lane reads its own row's 8 contraction elements (the wave's LDS
      // operations complete in order)
      float* As = stage;
      float* Bs = stage + kTile * kStageLd;
      const int q8 = lane & 7, r8 = lane >> 3, q4 = lane & 3, r4 = lane >> 2;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float2 t;
        t.x = (float)R.d[2 * j];
        t.y = (float)R.d[2 * j + 1];
        *reinterpret_cast<float2*>(As + (8 * j + r8) * kStageLd + 2 * q8) = t;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        float4 t;
        t.x = R.f[4 * j];
        t.y = R.f[4 * j + 1];
        t.z = R.f[4 * j + 2];
        t.w = R.f[4 * j + 3];
        *reinterpret_cast<float4*>(Bs + (16 * j + r4) * kStageLd + 4 * q4) = t;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const float4 a0 = *reinterpret_cast<const float4*>(As + i * kStageLd + 8 * kh);
      const float4 a1 = *reinterpret_cast<const float4*>(As + i * kStageLd + 8 * kh + 4);
      const float4 b0 = *reinterpret_cast<const float4*>(Bs + i * kStageLd + 8 * kh);
      const float4 b1 = *reinterpret_cast<const float4*>(Bs + i * kStageLd + 8 * kh + 4);
      const float ar[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
      const float br[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
      const float cA = src >= 0 ? (float)(sg.c * sg.scl[i]) : 0.f;
      const float sB = g.n0 + i < g.b ? 1.f : 0.f;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        a[s] = s < kv ? cA * ar[s] : 0.f;
        b[s] = s < kv ? sB * br[s] : 0.f;
      }
      // the stage is rewritten by the wave's next chunk only after these reads
      __builtin_amdgcn_wave_barrier();
    }
  }
  template <bool kStage>
  __device__ static void mma(Acc& acc, const Raw& R, const ImgSeg& sg, int kind, int K, int ch,
                             const TileGeo& g, int lane, float* stage) {
    float a[8], b[8];
    operands<kStage>(R, sg, kind, K, ch, g, lane, stage, a, b);
#pragma unroll
    for (int s = 0; s < 8; ++s) acc.d = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], b[s], acc.d, 0, 0, 0);
  }
  static constexpr int kRegs = 16;
  __device__ static float value(const Acc& a, int r) { return a.d[r]; }
  __device__ static void coords(int lane, int r, int& row, int& col) {
    row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    col = lane & 31;
  }
};

// BF16 hi/lo split on the matrix cores: v_mfma_f32_32x32x16_bf16, A[i][k]
// from lane i + 32*(k/8), element k%8 (B likewise with column j); D as in the
// FP32 32x32 layout.  Every FP32 operand x is split into hi = bf16(x) and
// lo = bf16(x - hi); a product is hi*hi + hi*lo + lo*hi (the lo*lo term and
// the rounding of lo leave a relative error of about 2^-16), accumulated in
// FP32.  Raw loads and masking are those of the FP32 tile.
struct BF16Tile {
  using op_t = float;
  using red_t = float;
  static constexpr int kWaves = 16;
  using Acc = F32Tile::Acc;
  using Raw = F32Tile::Raw;
  __device__ static void zero(Acc& a) { F32Tile::zero(a); }
  template <bool kStage>
  __device__ static void load(Raw& R, const ImgSeg& sg, int kind, int K, int ch, const TileGeo& g,
                              const op_t* dense, const double* psi, int lane) {
    F32Tile::load<kStage>(R, sg, kind, K, ch, g, dense, psi, lane);
  }
  __device__ static void split(const float (&x)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const __bf16 h = (__bf16)x[j];
      hi[j] = h;
      lo[j] = (__bf16)(x[j] - (float)h);
    }
  }
  static constexpr int kStageFloats = F32Tile::kStageFloats;
  template <bool kStage>
  __device__ static void mma(Acc& acc, const Raw& R, const ImgSeg& sg, int kind, int K, int ch,
                             const TileGeo& g, int lane, float* stage) {
    float a[8], b[8];
    F32Tile::operands<kStage>(R, sg, kind, K, ch, g, lane, stage, a, b);
    bf16x8 ah, al, bh, bl;
    split(a, ah, al);
    split(b, bh, bl);
    acc.d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc.d, 0, 0, 0);
    acc.d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc.d, 0, 0, 0);
    acc.d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc.d, 0, 0, 0);
  }
  static constexpr int kRegs = 16;
  __device__ static float value(const Acc& a, int r) { return a.d[r]; }
  __device__ static void coords(int lane, int r, int& row, int& col) { F32Tile::coords(lane, r, row, col); }
};

// FP64 matrix cores, v_mfma_f64_16x16x4f64 on the four 16x16 quarters of the
// tile: A[i][k] from lane i + 16k, B[k][j] from lane j + 16k; D row
// 4*reg + lane/16, column lane%16.  Element s of lane group q = lane/16
// carries k = 4q + s.
struct F64Tile {
  using op_t = double;
  using red_t = double;
  static constexpr int kWaves = 8;
  struct Acc {
    f64x4 d[4];
  };
  struct Raw {
    double a0[4], a1[4], b0[4], b1[4];
  };
  __device__ static void zero(Acc& a) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) a.d[q][r] = 0.0;
  }
  template <bool kStage>
  __device__ static void load(Raw& R, const ImgSeg& sg, int kind, int K, int ch, const TileGeo& g,
                              const op_t* dense, const double* psi, int lane) {
    const int i = lane & 15, kb = ch * kChunk + 4 * (lane >> 4);
    if (kind == SEG_KN) {
      const op_t* A0 = dense + sg.op_off + min(g.m0 + i, g.a - 1);
      const op_t* A1 = dense + sg.op_off + min(g.m0 + 16 + i, g.a - 1);
      const int64_t lda = sg.op_ld;
      const double* P0 = psi + sg.psi_off + max(sg.src[i], 0);
      const double* P1 = psi + sg.psi_off + max(sg.src[16 + i], 0);
      const int64_t ldp = sg.psi_ld;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t k = min(kb + s, K - 1);
        R.a0[s] = A0[k * lda];
        R.a1[s] = A1[k * lda];
        R.b0[s] = P0[k * ldp];
        R.b1[s] = P1[k * ldp];
      }
    } else {
      const double* A0 = psi + sg.psi_off + (int64_t)max(sg.src[i], 0) * sg.psi_ld;
      const double* A1 = psi + sg.psi_off + (int64_t)max(sg.src[16 + i], 0) * sg.psi_ld;
      const op_t* B0 = dense + sg.op_off + (int64_t)min(g.n0 + i, g.b - 1) * sg.op_ld;
      const op_t* B1 = dense + sg.op_off + (int64_t)min(g.n0 + 16 + i, g.b - 1) * sg.op_ld;
      if (K - (ch + 1) * kChunk >= 0) {   // whole chunk in range (uniform): 16-byte row loads
#pragma unroll
        for (int s = 0; s < 4; s += 2) {
          d2 t;
          __builtin_memcpy(&t, A0 + kb + s, sizeof(t));
          R.a0[s] = t.x;
          R.a0[s + 1] = t.y;
          __builtin_memcpy(&t, A1 + kb + s, sizeof(t));
          R.a1[s] = t.x;
          R.a1[s + 1] = t.y;
          __builtin_memcpy(&t, B0 + kb + s, sizeof(t));
          R.b0[s] = t.x;
          R.b0[s + 1] = t.y;
          __builtin_memcpy(&t, B1 + kb + s, sizeof(t));
          R.b1[s] = t.x;
          R.b1[s + 1] = t.y;
        }
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = min(kb + s, K - 1);
          R.a0[s] = A0[k];
          R.a1[s] = A1[k];
          R.b0[s] = B0[k];
          R.b1[s] = B1[k];
        }
      }
    }
  }
  static constexpr int kStageFloats = 0;   // rows are read per lane, no LDS stage
  template <bool kStage>
  __device__ static void mma(Acc& acc, const Raw& R, const ImgSeg& sg, int kind, int K, int ch,
                             const TileGeo& g, int lane, float* /*stage*/) {
    const int i = lane & 15, kv = K - ch * kChunk - 4 * (lane >> 4);
    const int src0 = sg.src[i], src1 = sg.src[16 + i];
    double cA0, cA1, sB0, sB1;
    if (kind == SEG_KN) {
      cA0 = g.m0 + i < g.a ? sg.c : 0.0;
      cA1 = g.m0 + 16 + i < g.a ? sg.c : 0.0;
      sB0 = src0 >= 0 ? sg.scl[i] : 0.0;
      sB1 = src1 >= 0 ? sg.scl[16 + i] : 0.0;
    } else {
      cA0 = src0 >= 0 ? sg.c * sg.scl[i] : 0.0;
      cA1 = src1 >= 0 ? sg.c * sg.scl[16 + i] : 0.0;
      sB0 = g.n0 + i < g.b ? 1.0 : 0.0;
      sB1 = g.n0 + 16 + i < g.b ? 1.0 : 0.0;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool v = s < kv;
      const double a0 = v ? cA0 * R.a0[s] : 0.0, a1 = v ? cA1 * R.a1[s] : 0.0;
      const double b0 = v ? sB0 * R.b0[s] : 0.0, b1 = v ? sB1 * R.b1[s] : 0.0;
      acc.d[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc.d[0], 0, 0, 0);
      acc.d[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc.d[1], 0, 0, 0);
      acc.d[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc.d[2], 0, 0, 0);
      acc.d[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc.d[3], 0, 0, 0);
    }
  }
  static constexpr int kRegs = 16;
  __device__ static double value(const Acc& a, int r) { return a.d[r >> 2][r & 3]; }
  __device__ static void coords(int lane, int r, int& row, int& col) {
    const int q = r >> 2, qi = q >> 1, qj = q & 1;
    row = 16 * qi + 4 * (r & 3) + (lane >> 4);
    col = 16 * qj + (lane & 15);
  }
};

// Elementwise term at local element (mi, nj): c * rs * cs * psi[row + col].
// A zero row or column has scale 0 in the image; its load is clamped to
// psi[0] and dropped by that scale, so loads need no branch and the loads
// of several terms go out together.
__device__ inline double img_gg_load(const ImgGG& G, int mi, int nj, const double* psi) {
  const int64_t row = G.row[mi];
  const int32_t col = G.col[nj];
  return psi[(row < 0 ? 0 : row) + (col < 0 ? 0 : col)];
}
__device__ inline double img_gg_coef(const ImgGG& G, int mi, int nj) {
  return G.c * G.rs[mi] * G.cs[nj];
}
__device__ inline double img_gg_term(const ImgGG& G, int mi, int nj, const double* psi) {
  const double v = img_gg_load(G, mi, nj, psi);
  return img_gg_coef(G, mi, nj) * v;
}

template <class Cfg, bool kStage>
__global__ __launch_bounds__(Cfg::kWaves * 64) void hpsi_tiles(
    const uint32_t* __restrict__ images, int32_t stride,
    const typename Cfg::op_t* __restrict__ dense, const double* __restrict__ psi,
    double* __restrict__ y, double alpha, double beta) {
  constexpr int kW = Cfg::kWaves;
  constexpr int kT = kW * 64;
  constexpr int kPer = kTile * kTile / kT;   // output elements per thread
  __shared__ __align__(16) uint32_t img[kImgWords];
  // the waves' partial tiles (phase 2) share LDS with their chunk stages (phase 1)
  using red_t = typename Cfg::red_t;
  constexpr size_t kRedBytes = sizeof(red_t) * kW * kTile * kTile;
  constexpr size_t kStageBytes = kStage ? sizeof(float) * kW * Cfg::kStageFloats : 0;
  __shared__ __align__(16) char pool[kRedBytes > kStageBytes ? kRedBytes : kStageBytes];
  auto red = reinterpret_cast<red_t(*)[kTile * kTile]>(pool);

  // phase 0: the slot's image into LDS
  {
    const uint4* src = reinterpret_cast<const uint4*>(images + (int64_t)blockIdx.x * stride);
    uint4* dst = reinterpret_cast<uint4*>(img);
    for (int x = threadIdx.x; x < stride / 4; x += kT) dst[x] = src[x];
  }
  __syncthreads();
  const ImgHeader& H = img_header(img);
  TileGeo g;
  g.a = rfl(H.a);
  if (g.a == 0) return;   // idle slot
  g.b = rfl(H.b);
  g.m0 = rfl(H.m0);
  g.n0 = rfl(H.n0);
  const int ngemm = rfl(H.ngemm), ngg = rfl(H.ngg), nchunk = rfl(H.nchunk);
  // the wave index is uniform in a wave: say so, so that chunk and segment
  // bookkeeping stays in scalar registers
  const int wave = rfl(threadIdx.x >> 6), lane = threadIdx.x & 63;

  // phase 1
  typename Cfg::Acc acc;
  Cfg::zero(acc);
  double ggv[kPer];
#pragma unroll
  for (int e = 0; e < kPer; ++e) ggv[e] = 0.0;
  // elementwise terms: their loads go out before the first chunks' (terms
  // beyond ngg re-read term 0's), the FP64 sum in term order comes after
  double ggt[kPer][kMaxGG];
  auto gg_issue = [&]() {
    if (ngg == 0) return;
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int el = threadIdx.x + e * kT;
#pragma unroll
      for (int q = 0; q < kMaxGG; ++q)
        ggt[e][q] = img_gg_load(img_gg(img, ngemm, q < ngg ? q : 0), el / kTile, el % kTile, psi);
    }
  };
  auto gg_sum = [&]() {
    if (ngg == 0) return;
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int el = threadIdx.x + e * kT;
#pragma unroll
      for (int q = 0; q < kMaxGG; ++q)
        if (q < ngg) ggv[e] += img_gg_coef(img_gg(img, ngemm, q), el / kTile, el % kTile) * ggt[e][q];
    }
  };
  if (wave < nchunk) {
    typename Cfg::Raw ra, rb;
    int si = 0;   // segment of the latest chunk handed out (chunks come in increasing order)
    auto seg_for = [&](int gc) {
      while (si + 1 < ngemm && gc >= rfl(img_seg(img, si + 1).ch0)) ++si;
      return si;
    };
    auto fetch = [&](typename Cfg::Raw& R, int gc, int s) {
      const ImgSeg& sg = img_seg(img, s);
      Cfg::template load<kStage>(R, sg, rfl(sg.kind), rfl(sg.K), gc - rfl(sg.ch0), g, dense, psi, lane);
    };
    float* stage = reinterpret_cast<float*>(pool) + wave * Cfg::kStageFloats;
    auto run = [&](const typename Cfg::Raw& R, int gc, int s) {
      const ImgSeg& sg = img_seg(img, s);
      Cfg::template mma<kStage>(acc, R, sg, rfl(sg.kind), rfl(sg.K), gc - rfl(sg.ch0), g, lane, stage);
    };
    int gA = wave, sA = seg_for(gA);
    gg_issue();
    fetch(ra, gA, sA);
    int gB = gA + kW, sB = 0;
    if (gB < nchunk) {
      sB = seg_for(gB);
      fetch(rb, gB, sB);
    }
    // keep the scheduler from hoisting the sum (and its wait) above the
    // second chunk's loads
    __builtin_amdgcn_sched_barrier(0);
    gg_sum();
    for (;;) {
      run(ra, gA, sA);
      if (gB >= nchunk) break;
      gA = gB + kW;
      if (gA < nchunk) {
        sA = seg_for(gA);
        fetch(ra, gA, sA);
      }
      run(rb, gB, sB);
      if (gA >= nchunk) break;
      gB = gA + kW;
      if (gB < nchunk) {
        sB = seg_for(gB);
        fetch(rb, gB, sB);
      }
    }
  } else {
    gg_issue();
    gg_sum();
  }
  __syncthreads();   // every wave is done with its chunk stage
  if (wave < nchunk) {
#pragma unroll
    for (int r = 0; r < Cfg::kRegs; ++r) {
      int row, col;
      Cfg::coords(lane, r, row, col);
      red[wave][row * kTile + col] = Cfg::value(acc, r);
    }
  }
  __syncthreads();

  // phase 2: fixed-order sum, elementwise terms, y
  const int nw = nchunk < kW ? nchunk : kW;   // waves that wrote a partial tile
  const int ldy = rfl(H.ldy);
  const int64_t y_off = H.y_off;
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int el = threadIdx.x + e * kT;
    const int mi = el / kTile, nj = el % kTile;
    double v = 0.0;
    for (int w = 0; w < nw; ++w) v += (double)red[w][el];
    v += ggv[e];
    for (int q = kMaxGG; q < ngg; ++q) v += img_gg_term(img_gg(img, ngemm, q), mi, nj, psi);
    const int m = g.m0 + mi, n = g.n0 + nj;
    if (m < g.a && n < g.b) {
      const int64_t idx = y_off + (int64_t)m * ldy + n;
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
template <class Cfg, bool kStage>
void launch_tiles(int nslots, const uint32_t* images, int32_t stride, const void* dense,
                  const double* psi, double* y, double alpha, double beta, hipStream_t stream,
                  hipEvent_t t0, hipEvent_t t1) {
  // hipExtLaunchKernelGGL records t0/t1 (when given) at the dispatch's own
  // start and end, so the interval is the kernel alone
  hipExtLaunchKernelGGL(hpsi_tiles<Cfg, kStage>, dim3(nslots), dim3(Cfg::kWaves * 64), 0, stream, t0,
                        t1, 0, images, stride, (const typename Cfg::op_t*)dense, psi, y, alpha, beta);
}

hipError_t launch_hpsi(int prec, int variant, int nslots, const uint32_t* images, int32_t stride,
                       const void* dense, const double* psi, double* y, double alpha, double beta,
                       hipStream_t stream, hipEvent_t t0, hipEvent_t t1) {
  if (nslots <= 0) return hipSuccess;
  const bool stage = variant == kVariantStagedRows;
  if (prec == kPrecF32) {
    if (stage)
      launch_tiles<F32Tile, true>(nslots, images, stride, dense, psi, y, alpha, beta, stream, t0, t1);
    else
      launch_tiles<F32Tile, false>(nslots, images, stride, dense, psi, y, alpha, beta, stream, t0, t1);
  } else if (prec == kPrecBF16X3) {
    if (stage)
      launch_tiles<BF16Tile, true>(nslots, images, stride, dense, psi, y, alpha, beta, stream, t0, t1);
    else
      launch_tiles<BF16Tile, false>(nslots, images, stride, dense, psi, y, alpha, beta, stream, t0, t1);
  } else {
    launch_tiles<F64Tile, false>(nslots, images, stride, dense, psi, y, alpha, beta, stream, t0, t1);
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
