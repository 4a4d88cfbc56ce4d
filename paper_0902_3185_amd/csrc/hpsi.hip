// Superblock product kernels for gfx950 (CDNA4).
//
// A workgroup owns one 32 x 32 output tile of one target block Y_q at a time
// and reduces every term that writes it (Y_q += c A Psi_q' B^T; paper Sec.
// 3.3, blocking by effective symmetry); a persistent launch gives each
// workgroup a list of tiles, and a list of two small tiles runs both at
// once on the two halves of the waves.  The dense products run on the
// matrix cores: the waves of a tile (16 for FP32 and the BF16 split, 8 for
// FP64) split the contraction chunks of all of its terms, and their partial
// tiles are summed in LDS in a fixed order, so the result does not depend
// on scheduling.  Terms with identity or gather operators on both
// sides are elementwise and are added in FP64 afterwards.  No atomics are
// used on y.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>

#include "kernels.h"

namespace dmrg {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
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
      // the FP32 pool holds A-side blocks row-major (a x K)
      const op_t* A = dense + sg.op_off;
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
          av[s] = (mok && kok) ? cs * A[(int64_t)m * sg.K + k] : 0.f;
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

// FP32 and BF16 products with each wave's contraction chunk staged in LDS.
//
// A chunk is 16 positions of one segment's contraction.  Its two operand
// panels -- A (32 output rows x 16 k) and B (16 k x 32 output columns) --
// are read with 16-byte buffer loads along the direction the data is
// contiguous in (rows of psi and of the row-major operator blocks along k;
// rows of Psi' along the output columns for SEG_KN, over a 32-column window
// that holds every gathered column of the tile), scaled, and written to the
// wave's own LDS area: A as [m][k], B as [k][w] (the window) for SEG_KN and
// as [n][k] for SEG_MK.  The matrix-core operands are then read from LDS in
// the layout of v_mfma_f32_16x16x4f32 on the tile's four 16 x 16 quarters:
// A[i][k] from lane i + 16k, B[k][j] from lane j + 16k, D[i][j] in lane
// j + 16*(i/4), register i%4; lane group kk = lane/16 takes chunk positions
// 4kk .. 4kk + 3, instruction s position 4kk + s.  The BF16 form splits each
// FP32 operand x into hi = bf16(x) and lo = bf16(x - hi) and issues
// hi*hi + hi*lo + lo*hi with v_mfma_f32_16x16x16bf16_1k (A[i][k] from lane
// i + 16*(k/4), element k%4: the same four positions per lane), FP32
// accumulate.
//
// Each lane's byte offsets and scales depend only on the segment, so they
// are formed once per segment; a chunk then costs four loads (one add each)
// and a few multiplies.  Loads past a block's rows or columns read
// neighbouring data (zeroed by the scales) or, past the buffer, zeros: the
// buffer resources carry each buffer's size, which the hardware checks.  A
// chunk that ends past the contraction length is masked element by element.

typedef short s16x4 __attribute__((ext_vector_type(4)));

__device__ inline f4 buf16(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, 0, 0));
}
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
constexpr uint32_t kNoRead = 0x80000000u;   // an offset past every buffer: reads zeros, no traffic

template <bool kBF16>
struct F32S {
  using op_t = float;
  using psi_t = float;
  using red_t = float;
  static constexpr int kWaves = 16;
  // waves per SIMD the register budget must allow (one workgroup of
  // sixteen waves per compute unit)
  static constexpr int kMinWavesPerEU = 4;
  // a workgroup whose list holds two tiles of at most kWaves / 2 chunks
  // each runs them at once, half of the waves on each
  static constexpr bool kPair = true;
  // the next fetch goes out before a chunk's matrix instructions (contract)
  static constexpr bool kEarlyFetch = !kBF16;
  static constexpr int kLdn = 36;                      // [k][w] window row stride (floats)
  static constexpr int kAFloats = kTile * kChunk;      // A panel [m][k]
  static constexpr int kBFloats = kChunk * kLdn;       // B panel ([k][w]; [n][k] uses 512)
  static constexpr int kStageFloats = kAFloats + kBFloats;
  struct Acc {
    f32x4 d[4];   // quarter (qi, qj) at d[2*qi + qj]
  };
  // one chunk in registers: operator panel (rows lane/4 + 16j, positions
  // 4*(lane%4) .. +3) and psi panel (SEG_KN: window row lane/8 + 8j,
  // columns 4*(lane%8) .. +3; SEG_MK: gathered row lane/4 + 16j, positions
  // 4*(lane%4) .. +3)
  struct Raw {
    f4 o[2], p[2];
  };
  // a segment's per-lane byte offsets of its chunk 0 and bytes per chunk
  struct Fetch {
    int seg;
    uint32_t op[2], ps[2];
    uint32_t dop, dps;
  };
  // a segment's per-lane scales: sa (A panel rows), sb (SEG_KN: column
  // scale at use, w the column's place in the window; SEG_MK: B rows)
  struct Use {
    int seg;
    float sa[2], sb[2];
    int w[2];
  };
  __device__ static void zero(Acc& a) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) a.d[q][r] = 0.f;
  }
  __device__ static void setup_fetch(Fetch& f, int s, const ImgSeg& sg, int kind, int K, const TileGeo& g,
                                     int lane) {
    f.seg = s;
    const int64_t ldp = sg.psi_ld;
    if (kind == SEG_KN) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        f.op[j] = (uint32_t)(4 * (sg.op_off + (int64_t)(g.m0 + lane / 4 + 16 * j) * K + (lane & 3) * 4));
        f.ps[j] = (uint32_t)(4 * (sg.psi_off + (int64_t)(lane / 8 + 8 * j) * ldp + sg.pad + (lane & 7) * 4));
      }
      f.dop = 4 * kChunk;
      f.dps = (uint32_t)(4 * kChunk * ldp);
    } else {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = max(sg.src[lane / 4 + 16 * j], 0);
        f.op[j] = (uint32_t)(4 * (sg.op_off + (int64_t)(g.n0 + lane / 4 + 16 * j) * sg.op_ld + (lane & 3) * 4));
        f.ps[j] = (uint32_t)(4 * (sg.psi_off + (int64_t)r * ldp + (lane & 3) * 4));
      }
      f.dop = 4 * kChunk;
      f.dps = 4 * kChunk;
    }
  }
  __device__ static void setup_use(Use& u, int s, const ImgSeg& sg, int kind, const TileGeo& g, int lane) {
    u.seg = s;
    const int i = lane & 15;
    if (kind == SEG_KN) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        u.sa[j] = g.m0 + lane / 4 + 16 * j < g.a ? (float)sg.c : 0.f;
        const int src = sg.src[16 * j + i];
        u.w[j] = src >= 0 ? src - sg.pad : 0;
        u.sb[j] = src >= 0 ? (float)sg.scl[16 * j + i] : 0.f;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = lane / 4 + 16 * j;
        u.sa[j] = sg.src[r] >= 0 ? (float)(sg.c * sg.scl[r]) : 0.f;
        u.sb[j] = g.n0 + r < g.b ? 1.f : 0.f;
        u.w[j] = 0;
      }
    }
  }
  __device__ static void load(Raw& R, const Fetch& f, int ch, bool live, __amdgpu_buffer_rsrc_t rd,
                              __amdgpu_buffer_rsrc_t rp) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      R.o[j] = buf16(rd, live ? f.op[j] + ch * f.dop : kNoRead);
      R.p[j] = buf16(rp, live ? f.ps[j] + ch * f.dps : kNoRead);
    }
  }
  // raw registers -> scaled FP32 panels in the wave's LDS area
  __device__ static void stage(const Raw& R, const Use& u, int kind, int K, int ch, int lane, float* As,
                               float* Bs) {
    const int kc = ch * kChunk;
    const bool full = kc + kChunk <= K;   // uniform
    f4 v[4];
    if (kind == SEG_KN) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        v[j] = u.sa[j] * R.o[j];   // A[m][k] = c op[m][k]
        v[2 + j] = R.p[j];         // window rows
      }
      if (!full) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (kc + (lane & 3) * 4 + e >= K) v[j][e] = 0.f;
          if (kc + lane / 8 + 8 * j >= K) v[2 + j] = f4{0.f, 0.f, 0.f, 0.f};
        }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        *reinterpret_cast<f4*>(As + (lane / 4 + 16 * j) * kChunk + (lane & 3) * 4) = v[j];
        *reinterpret_cast<f4*>(Bs + (lane / 8 + 8 * j) * kLdn + (lane & 7) * 4) = v[2 + j];
      }
    } else {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        v[j] = u.sa[j] * R.p[j];       // A[m][k] = c scl[m] Psi'[src m][k]
        v[2 + j] = u.sb[j] * R.o[j];   // B^T[n][k] = op[n][k]
      }
      if (!full) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (kc + (lane & 3) * 4 + e >= K) v[j][e] = 0.f;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        *reinterpret_cast<f4*>(As + (lane / 4 + 16 * j) * kChunk + (lane & 3) * 4) = v[j];
        *reinterpret_cast<f4*>(Bs + (lane / 4 + 16 * j) * kChunk + (lane & 3) * 4) = v[2 + j];
      }
    }
  }
  __device__ static void split(const f4& x, s16x4& hi, s16x4& lo) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const __bf16 h = (__bf16)x[j];
      const __bf16 l = (__bf16)(x[j] - (float)h);
      hi[j] = __builtin_bit_cast(short, h);
      lo[j] = __builtin_bit_cast(short, l);
    }
  }
  // a chunk's raw registers -> its panels in the wave's LDS area; the
  // registers are free for the next fetch once this has been issued
  __device__ static void put(const Raw& R, const Use& u, int kind, int K, int ch, int lane, float* stage_area) {
    // the previous chunk's reads of this area were issued before this point
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    stage(R, u, kind, K, ch, lane, stage_area, stage_area + kAFloats);
  }
  // the staged chunk through the matrix cores
  __device__ static void mma(Acc& acc, const Use& u, int kind, int lane, const float* stage_area) {
    const float* As = stage_area;
    const float* Bs = stage_area + kAFloats;
    // the wave's LDS operations complete in order: its reads below see the
    // writes of put
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int i = lane & 15, kk = lane >> 4;
    f4 a[2], b[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) a[h] = *reinterpret_cast<const f4*>(As + (16 * h + i) * kChunk + 4 * kk);
    if (kind == SEG_KN) {   // B[k][n] = scl[n] W[k][src n - base]
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int s = 0; s < 4; ++s) b[h][s] = u.sb[h] * Bs[(4 * kk + s) * kLdn + u.w[h]];
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h) b[h] = *reinterpret_cast<const f4*>(Bs + (16 * h + i) * kChunk + 4 * kk);
    }
    if constexpr (kBF16) {
      s16x4 ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        split(a[h], ah[h], al[h]);
        split(b[h], bh[h], bl[h]);
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
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int qi = 0; qi < 2; ++qi)
#pragma unroll
          for (int qj = 0; qj < 2; ++qj)
            acc.d[2 * qi + qj] =
                __builtin_amdgcn_mfma_f32_16x16x4f32(a[qi][s], b[qj][s], acc.d[2 * qi + qj], 0, 0, 0);
    }
  }
  // The wave's chunks are wave, wave + kW, ... of the tile's chunk
  // sequence; two are in flight ahead of the one on the matrix cores.  In
  // the FP32 form a chunk's registers are refilled with the fetch two
  // chunks ahead as soon as the chunk is staged in LDS, before its matrix
  // instructions, which may wait for the other waves of the SIMD; the BF16
  // form fetches after them (its split operands leave no registers for the
  // fetch while they are live).  Fetches are unconditional (one past the
  // wave's last chunk reads nothing), so that every step issues the same
  // loads and the compiler keeps them ahead of the work.
  // stride: the waves sharing the tile (wave is the index among them)
  __device__ static void contract(Acc& acc, const uint32_t* img, int ngemm, int nchunk, const TileGeo& g,
                                  int wave, int lane, const float* dense, const float* psi, int64_t ndense,
                                  int64_t npsi, float* stage_area, int stride = kWaves) {
    const __amdgpu_buffer_rsrc_t rd = buf_rsrc(dense, 4 * ndense), rp = buf_rsrc(psi, 4 * npsi);
    const int nmy = (nchunk - wave + stride - 1) / stride;
    int si = 0;   // segment of the latest chunk fetched (chunks come in increasing order)
    Fetch f;
    f.seg = -1;
    Use u;
    u.seg = -1;
    auto fetch = [&](Raw& R, int i, int& gc, int& s) {
      const bool live = i < nmy;
      gc = wave + stride * (live ? i : nmy - 1);
      while (si + 1 < ngemm && gc >= rfl(img_seg(img, si + 1).ch0)) ++si;
      s = si;
      const ImgSeg& sg = img_seg(img, s);
      if (s != f.seg) setup_fetch(f, s, sg, rfl(sg.kind), rfl(sg.K), g, lane);
      load(R, f, gc - rfl(sg.ch0), live, rd, rp);
    };
    // stage chunk gc (segment s) from R; returns the segment's kind
    auto stage_chunk = [&](const Raw& R, int gc, int s) {
      const ImgSeg& sg = img_seg(img, s);
      const int kind = rfl(sg.kind);
      if (s != u.seg) setup_use(u, s, sg, kind, g, lane);
      put(R, u, kind, rfl(sg.K), gc - rfl(sg.ch0), lane, stage_area);
      return kind;
    };
    Raw ra, rb;
    int gA, sA, gB, sB;
    fetch(ra, 0, gA, sA);
    fetch(rb, 1, gB, sB);
    __builtin_amdgcn_sched_barrier(0);
    for (int i = 0; i < nmy; i += 2) {
      int kind = stage_chunk(ra, gA, sA);
      if constexpr (kEarlyFetch) fetch(ra, i + 2, gA, sA);
      mma(acc, u, kind, lane, stage_area);
      if constexpr (!kEarlyFetch) fetch(ra, i + 2, gA, sA);
      __builtin_amdgcn_sched_barrier(0);
      if (i + 1 < nmy) {
        kind = stage_chunk(rb, gB, sB);
        if constexpr (kEarlyFetch) fetch(rb, i + 3, gB, sB);
        mma(acc, u, kind, lane, stage_area);
        if constexpr (!kEarlyFetch) fetch(rb, i + 3, gB, sB);
      } else {
        fetch(rb, i + 3, gB, sB);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  static constexpr int kRegs = 16;
  __device__ static float value(const Acc& a, int r) { return a.d[r >> 2][r & 3]; }
  __device__ static void coords(int lane, int r, int& row, int& col) {
    const int q = r >> 2;
    row = 16 * (q >> 1) + 4 * (lane >> 4) + (r & 3);
    col = 16 * (q & 1) + (lane & 15);
  }
};

// FP64 matrix cores, v_mfma_f64_16x16x4f64 on the four 16x16 quarters of the
// tile: A[i][k] from lane i + 16k, B[k][j] from lane j + 16k; D row
// 4*reg + lane/16, column lane%16.  Element s of lane group q = lane/16
// carries k = 4q + s.
struct F64Tile {
  using op_t = double;
  using psi_t = double;
  using red_t = double;
  static constexpr int kWaves = 8;
  static constexpr int kMinWavesPerEU = 2;   // one workgroup per compute unit
  static constexpr bool kPair = false;
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
                              const op_t* dense, const double* psi, int lane, int64_t /*ndense*/,
                              int64_t /*npsi*/, bool /*live*/ = true) {
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
                             const TileGeo& g, int lane, float* /*stage*/, const double* /*psi*/) {
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
  // The wave's chunks are wave, wave + kW, ...; their operands are loaded
  // two chunks ahead of the matrix cores.
  __device__ static void contract(Acc& acc, const uint32_t* img, int ngemm, int nchunk, const TileGeo& g,
                                  int wave, int lane, const double* dense, const double* psi,
                                  int64_t /*ndense*/, int64_t /*npsi*/, float* /*stage_area*/) {
    Raw ra, rb;
    int si = 0;   // segment of the latest chunk handed out (chunks come in increasing order)
    auto seg_for = [&](int gc) {
      while (si + 1 < ngemm && gc >= rfl(img_seg(img, si + 1).ch0)) ++si;
      return si;
    };
    auto fetch = [&](Raw& R, int gc, int s) {
      const ImgSeg& sg = img_seg(img, s);
      load<false>(R, sg, rfl(sg.kind), rfl(sg.K), gc - rfl(sg.ch0), g, dense, psi, lane, 0, 0);
    };
    auto run = [&](const Raw& R, int gc, int s) {
      const ImgSeg& sg = img_seg(img, s);
      mma<false>(acc, R, sg, rfl(sg.kind), rfl(sg.K), gc - rfl(sg.ch0), g, lane, nullptr, psi);
    };
    int gA = wave, sA = seg_for(gA);
    fetch(ra, gA, sA);
    int gB = gA + kWaves, sB = 0;
    if (gB < nchunk) {
      sB = seg_for(gB);
      fetch(rb, gB, sB);
    }
    for (;;) {
      run(ra, gA, sA);
      if (gB >= nchunk) break;
      gA = gB + kWaves;
      if (gA < nchunk) {
        sA = seg_for(gA);
        fetch(ra, gA, sA);
      }
      run(rb, gB, sB);
      if (gA >= nchunk) break;
      gB = gA + kWaves;
      if (gB < nchunk) {
        sB = seg_for(gB);
        fetch(rb, gB, sB);
      }
    }
  }
};

// Elementwise terms, c * rs[mi] * cs[nj] * psi[row(mi) + col(nj)].  Threads
// 0 .. 255 take four consecutive columns of one tile row each; the loads of
// the first kGGEarly terms go out before the contraction chunks' and are
// summed after them (terms beyond re-read term 0's entries, dropped at the
// sum).  A zero row or column has scale 0 in the image and reads psi[0], so
// the loads need no branch.
constexpr int kGGEarly = 4;
constexpr int kGGThreads = kTile * kTile / 4;

template <class PsiT>
__device__ inline void gg_load4(const ImgGG& G, int mi, int nj4, const PsiT* psi, PsiT (&v)[4]) {
  const int64_t row = G.row[mi] < 0 ? 0 : G.row[mi];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int32_t col = G.col[nj4 + e];
    v[e] = psi[row + (col < 0 ? 0 : col)];
  }
}
__device__ inline double img_gg_coef(const ImgGG& G, int mi, int nj) {
  return G.c * G.rs[mi] * G.cs[nj];
}

// Two tiles at once (configurations with kPair): a workgroup whose list
// holds two tiles of at most kWaves / 2 chunks each gives the first half of
// its waves the first tile and the other half the second, each half with
// its own image, chunk stages, partial tiles and elementwise sums.  Every
// wave then holds at most one chunk, as it does when the tiles run one
// after the other, and the sums keep their order, so the results are the
// same bits.  Returns false, having done nothing but read the two images,
// when the tiles do not both qualify.
template <class Cfg>
__device__ bool pair_tiles(const uint32_t* __restrict__ images, int32_t stride, int slot,
                           const typename Cfg::op_t* __restrict__ dense,
                           const typename Cfg::psi_t* __restrict__ psi, double* __restrict__ y, double alpha,
                           double beta, int64_t ndense, int64_t npsi, uint32_t* img, uint32_t* img2,
                           char* pool, double* ggs, double* ggs2) {
  using psi_t = typename Cfg::psi_t;
  using red_t = typename Cfg::red_t;
  constexpr int kW = Cfg::kWaves, kH = kW / 2;
  static_assert(kW * 64 == kTile * kTile, "one output element per thread and tile");
  for (int t = 0; t < 2; ++t) {
    const uint4* src = reinterpret_cast<const uint4*>(images + (int64_t)(slot + t) * stride);
    uint4* dst = reinterpret_cast<uint4*>(t ? img2 : img);
    for (int x = threadIdx.x; x < stride / 4; x += kW * 64) dst[x] = src[x];
  }
  __syncthreads();
  {
    const ImgHeader& HA = img_header(img);
    const ImgHeader& HB = img_header(img2);
    const bool both = rfl(HA.a) != 0 && rfl(HB.a) != 0 && rfl(HA.nchunk) <= kH && rfl(HB.nchunk) <= kH;
    if (!both) {
      __syncthreads();   // every thread has read the headers before the images are rewritten
      return false;
    }
  }
  const int wave = rfl((int)threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int grp = wave >= kH ? 1 : 0;   // uniform per wave
  const int gw = wave - grp * kH;       // the wave's index among its tile's waves
  const uint32_t* im = grp ? img2 : img;
  double* gs = grp ? ggs2 : ggs;
  const ImgHeader& H = img_header(im);
  TileGeo g;
  g.a = rfl(H.a);
  g.b = rfl(H.b);
  g.m0 = rfl(H.m0);
  g.n0 = rfl(H.n0);
  const int ngemm = rfl(H.ngemm), ngg = rfl(H.ngg), nchunk = rfl(H.nchunk);
  int tid = (int)threadIdx.x - grp * kH * 64;   // the thread's index among its tile's threads
  asm volatile("" : "+v"(tid));
  const bool gg_thread = ngg > 0 && gw < kGGThreads / 64;
  const int gmi = tid >> 3, gnj = (tid & 7) * 4;
  typename Cfg::Acc acc;
  Cfg::zero(acc);
  if (gw < nchunk)
    Cfg::contract(acc, im, ngemm, nchunk, g, gw, lane, dense, psi, ndense, npsi,
                  reinterpret_cast<float*>(pool) + wave * Cfg::kStageFloats, kH);
  psi_t gr[kGGEarly][4];
  if (gg_thread) {
#pragma unroll
    for (int q = 0; q < kGGEarly; ++q) gg_load4(img_gg(im, ngemm, q < ngg ? q : 0), gmi, gnj, psi, gr[q]);
  }
  __syncthreads();   // every wave is done with its chunk stage
  auto red = reinterpret_cast<red_t(*)[kTile * kTile]>(pool);
  if (gw < nchunk) {
#pragma unroll
    for (int r = 0; r < Cfg::kRegs; ++r) {
      int row, col;
      Cfg::coords(lane, r, row, col);
      red[wave][row * kTile + col] = Cfg::value(acc, r);
    }
  }
  if (gg_thread) {
#pragma unroll
    for (int q = 0; q < kGGEarly; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) asm volatile("" : "+v"(gr[q][e]));
    double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < kGGEarly; ++q)
      if (q < ngg) {
        const ImgGG& G = img_gg(im, ngemm, q);
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] += img_gg_coef(G, gmi, gnj + e) * (double)gr[q][e];
      }
    for (int q = kGGEarly; q < ngg; ++q) {
      const ImgGG& G = img_gg(im, ngemm, q);
      psi_t t[4];
      gg_load4(G, gmi, gnj, psi, t);
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] += img_gg_coef(G, gmi, gnj + e) * (double)t[e];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) gs[gmi * kTile + gnj + e] = v[e];
  }
  __syncthreads();
  // one element of each tile per thread: the waves' partial tiles in wave
  // order, the elementwise terms, y
  const int el = threadIdx.x;
  const int mi = el / kTile, nj = el % kTile;
  for (int t = 0; t < 2; ++t) {
    const ImgHeader& Ht = img_header(t ? img2 : img);
    const int nw = rfl(Ht.nchunk), ngt = rfl(Ht.ngg);
    double v = 0.0;
    for (int w = 0; w < nw; ++w) v += (double)red[t * kH + w][el];
    if (ngt > 0) v += (t ? ggs2 : ggs)[el];
    const int m = rfl(Ht.m0) + mi, n = rfl(Ht.n0) + nj;
    if (m < rfl(Ht.a) && n < rfl(Ht.b)) {
      const int64_t idx = Ht.y_off + (int64_t)m * rfl(Ht.ldy) + n;
      y[idx] = beta == 0.0 ? alpha * v : alpha * v + beta * y[idx];
    }
  }
  return true;
}

template <class Cfg, bool kStage>
__global__ __launch_bounds__(Cfg::kWaves * 64, Cfg::kMinWavesPerEU) void hpsi_tiles(
    const uint32_t* __restrict__ images, int32_t stride,
    const typename Cfg::op_t* __restrict__ dense, const typename Cfg::psi_t* __restrict__ psi,
    double* __restrict__ y, double alpha, double beta, int64_t ndense, int64_t npsi,
    const int32_t* __restrict__ wg_start) {
  using psi_t = typename Cfg::psi_t;
  constexpr int kW = Cfg::kWaves;
  constexpr int kT = kW * 64;
  constexpr int kPer = kTile * kTile / kT;   // output elements per thread
  __shared__ __align__(16) uint32_t img[kImgWords];
  // the waves' partial tiles (phase 2) share LDS with their chunk stages (phase 1)
  using red_t = typename Cfg::red_t;
  constexpr size_t kRedBytes = sizeof(red_t) * kW * kTile * kTile;
  constexpr size_t kStageBytes = kStage ? sizeof(float) * kW * Cfg::kStageFloats : 0;
  __shared__ __align__(16) char pool[kRedBytes > kStageBytes ? kRedBytes : kStageBytes];
  __shared__ double ggs[kTile * kTile];   // elementwise terms' sum per tile element
  // the second tile of a pair run at once (pair_tiles)
  __shared__ __align__(16) uint32_t img2[Cfg::kPair ? kImgWords : 4];
  __shared__ double ggs2[Cfg::kPair ? kTile * kTile : 1];
  auto red = reinterpret_cast<red_t(*)[kTile * kTile]>(pool);

  // the workgroup's slots: a list (persistent launch) or its own index
  const int slot0 = wg_start ? wg_start[blockIdx.x] : (int)blockIdx.x;
  const int slot1 = wg_start ? wg_start[blockIdx.x + 1] : (int)blockIdx.x + 1;
  int first = slot0;
  if constexpr (Cfg::kPair) {
    if (slot1 - slot0 == 2 &&
        pair_tiles<Cfg>(images, stride, slot0, dense, psi, y, alpha, beta, ndense, npsi, img, img2, pool, ggs,
                        ggs2))
      first = slot1;
  }
  for (int slot = first; slot < slot1; ++slot) {
  // phase 0: the slot's image into LDS
  if (slot > slot0) __syncthreads();   // the previous tile is done with LDS
  {
    const uint4* src = reinterpret_cast<const uint4*>(images + (int64_t)slot * stride);
    uint4* dst = reinterpret_cast<uint4*>(img);
    for (int x = threadIdx.x; x < stride / 4; x += kT) dst[x] = src[x];
  }
  __syncthreads();
  const ImgHeader& H = img_header(img);
  TileGeo g;
  g.a = rfl(H.a);
  if (g.a == 0) continue;   // idle slot
  g.b = rfl(H.b);
  g.m0 = rfl(H.m0);
  g.n0 = rfl(H.n0);
  const int ngemm = rfl(H.ngemm), ngg = rfl(H.ngg), nchunk = rfl(H.nchunk);
  // The thread index as a fresh value in every tile: the lane offsets
  // derived from it are formed again per tile instead of being held across
  // the tile loop, where they would not fit the register budget and would
  // be spilled (and their reloads wait for the first operand loads).
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  // the wave index is uniform in a wave: say so, so that chunk and segment
  // bookkeeping stays in scalar registers
  const int wave = rfl(tid >> 6), lane = tid & 63;

  // phase 1
  const bool gg_thread = ngg > 0 && wave < kGGThreads / 64;   // uniform per wave
  const int gmi = tid >> 3, gnj = (tid & 7) * 4;
  typename Cfg::Acc acc;
  Cfg::zero(acc);
  if (wave < nchunk)
    Cfg::contract(acc, img, ngemm, nchunk, g, wave, lane, dense, psi, ndense, npsi,
                  reinterpret_cast<float*>(pool) + wave * Cfg::kStageFloats);
  // the elementwise terms' loads go out now (their latency overlaps the
  // wait for the other waves and the partial tiles' store)
  psi_t gr[kGGEarly][4];
  if (gg_thread) {
#pragma unroll
    for (int q = 0; q < kGGEarly; ++q) gg_load4(img_gg(img, ngemm, q < ngg ? q : 0), gmi, gnj, psi, gr[q]);
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
  if (gg_thread) {   // FP64 sum over the terms in order
    // the raw values stay as loaded until here (the compiler would otherwise
    // widen them next to their loads: an early wait and twice the registers)
#pragma unroll
    for (int q = 0; q < kGGEarly; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) asm volatile("" : "+v"(gr[q][e]));
    double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < kGGEarly; ++q)
      if (q < ngg) {
        const ImgGG& G = img_gg(img, ngemm, q);
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] += img_gg_coef(G, gmi, gnj + e) * (double)gr[q][e];
      }
    for (int q = kGGEarly; q < ngg; ++q) {
      const ImgGG& G = img_gg(img, ngemm, q);
      psi_t t[4];
      gg_load4(G, gmi, gnj, psi, t);
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] += img_gg_coef(G, gmi, gnj + e) * (double)t[e];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) ggs[gmi * kTile + gnj + e] = v[e];
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
    if (ngg > 0) v += ggs[el];
    const int m = g.m0 + mi, n = g.n0 + nj;
    if (m < g.a && n < g.b) {
      const int64_t idx = y_off + (int64_t)m * ldy + n;
      y[idx] = beta == 0.0 ? alpha * v : alpha * v + beta * y[idx];
    }
  }
  }   // slots
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

// psi in FP32 for the products that read an FP32 copy (one pass), and
// kPoolPad zeros after it: the products' masked vector loads may reach
// them, and a zero scale must not meet a NaN left in the buffer.
// A thread converts four consecutive elements with two 16-byte loads and one
// 16-byte store (x 16-byte aligned); the last partial group and the padding
// element by element.
__global__ __launch_bounds__(256) void psi_to_f32(const double* __restrict__ x, float* __restrict__ out,
                                                  int64_t n) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const int64_t i = 4 * ((int64_t)blockIdx.x * 256 + threadIdx.x);
  if (i + 4 <= n) {
    const d2 a = *reinterpret_cast<const d2*>(x + i);
    const d2 b = *reinterpret_cast<const d2*>(x + i + 2);
    *reinterpret_cast<f4*>(out + i) = f4{(float)a[0], (float)a[1], (float)b[0], (float)b[1]};
    return;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t j = i + e;
    if (j < n) out[j] = (float)x[j];
    else if (j < n + kPoolPad) out[j] = 0.f;
  }
}
// the same, one element per thread, for an x that is not 16-byte aligned
__global__ __launch_bounds__(256) void psi_to_f32_unaligned(const double* __restrict__ x,
                                                            float* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = (float)x[i];
  else if (i < n + kPoolPad) out[i] = 0.f;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <class Cfg, bool kStage>
void launch_tiles(int nslots, const uint32_t* images, int32_t stride, const void* dense,
                  const void* psi, double* y, double alpha, double beta, hipStream_t stream,
                  hipEvent_t t0, hipEvent_t t1, int64_t ndense, int64_t npsi, const int32_t* wg_start,
                  int nwg) {
  // hipExtLaunchKernelGGL records t0/t1 (when given) at the dispatch's own
  // start and end, so the interval is the kernel alone
  hipExtLaunchKernelGGL(hpsi_tiles<Cfg, kStage>, dim3(wg_start ? nwg : nslots), dim3(Cfg::kWaves * 64), 0,
                        stream, t0, t1, 0, images, stride, (const typename Cfg::op_t*)dense,
                        (const typename Cfg::psi_t*)psi, y, alpha, beta, ndense, npsi, wg_start);
}

struct CoefBatch {
  double v[kCoefBatch];
  int32_t t0;
};

__global__ __launch_bounds__(256) void patch_coeffs(char* __restrict__ base,
                                                    const CoefRef* __restrict__ refs, int64_t n,
                                                    CoefBatch c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const CoefRef r = refs[i];
  const int32_t t = r.term - c.t0;
  if (t >= 0 && t < kCoefBatch) *reinterpret_cast<double*>(base + r.off) = c.v[t];
}

hipError_t launch_patch_coeffs(void* base, const CoefRef* refs, int64_t n, const double* c,
                               int32_t nterms, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  if (!base || !refs || !c || nterms < 0) return hipErrorInvalidValue;
  for (int32_t t0 = 0; t0 < nterms; t0 += kCoefBatch) {
    CoefBatch b{};
    b.t0 = t0;
    for (int32_t k = 0; k < kCoefBatch && t0 + k < nterms; ++k) b.v[k] = c[t0 + k];
    hipLaunchKernelGGL(patch_coeffs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       static_cast<char*>(base), refs, n, b);
  }
  return hipGetLastError();
}

hipError_t launch_psi_to_f32(const double* psi, float* out, int64_t n, hipStream_t stream) {
  if (n < 0) return hipErrorInvalidValue;
  const int64_t m = n + kPoolPad;
  if ((reinterpret_cast<uintptr_t>(psi) & 15) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0)
    hipLaunchKernelGGL(psi_to_f32, dim3((unsigned)((m + 1023) / 1024)), dim3(256), 0, stream, psi, out, n);
  else
    hipLaunchKernelGGL(psi_to_f32_unaligned, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream, psi,
                       out, n);
  return hipGetLastError();
}

hipError_t launch_hpsi(int prec, int variant, int nslots, const uint32_t* images, int32_t stride,
                       const void* dense, const double* psi, double* y, double alpha, double beta,
                       hipStream_t stream, hipEvent_t t0, hipEvent_t t1, const float* psi32,
                       int64_t ndense, int64_t npsi, const int32_t* wg_start, int nwg) {
  if (nslots <= 0) return hipSuccess;
  if (wg_start && nwg <= 0) return hipErrorInvalidValue;
  if (prec == kPrecF32 || prec == kPrecBF16X3) {
    if (!psi32 || npsi < 4 || ndense < 4) return hipErrorInvalidValue;
    (void)variant;   // variant 1 (the macro-tile kernel) is launched by launch_hpsi_macro
    if (prec == kPrecBF16X3)
      launch_tiles<F32S<true>, true>(nslots, images, stride, dense, psi32, y, alpha, beta, stream, t0, t1,
                                     ndense, npsi, wg_start, nwg);
    else
      launch_tiles<F32S<false>, true>(nslots, images, stride, dense, psi32, y, alpha, beta, stream, t0, t1,
                                      ndense, npsi, wg_start, nwg);
  } else {
    launch_tiles<F64Tile, false>(nslots, images, stride, dense, psi, y, alpha, beta, stream, t0, t1, 0, 0,
                                 wg_start, nwg);
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
