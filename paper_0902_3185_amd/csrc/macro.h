// Macro-tile plan of the FP32 / BF16 product for superblocks with large
// blocks: 64 x 64 output tiles whose contraction is cut into stages of 32
// positions, the stages of all tiles laid end to end and dealt out in equal
// contiguous shares to the workgroups of one persistent launch (a tile may
// thus be shared by consecutive workgroups, each summing part of its
// contraction).  Every share of a shared tile stores its partial 64 x 64 sum
// and a second kernel adds them in share order, so the result does not
// depend on timing.  Host-only code (no HIP calls).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "plan.h"

namespace dmrg {

constexpr int kMac = 64;         // output tile edge
constexpr int kMacStage = 32;    // contraction positions per stage
constexpr int kMacThreads = 256; // four waves, one 32 x 32 quarter each
constexpr int kMacWGsPerCU = 3;  // persistent workgroups per compute unit
constexpr int kMacSegLds = 24;   // segments of one item held in LDS (items are cut to fit)

struct MacTile {
  int64_t y_off;
  int32_t a, b, m0, n0, ldy;
  int32_t seg0, nseg;   // matrix-core segments (MacSeg records)
  int32_t gg0, ngg;     // elementwise segments (MacGG records)
  int32_t nstage;       // stages over all of the tile's segments
  int32_t nsplit;       // pieces of the tile (1: not shared)
  int32_t part0;        // first partial-tile slot of a shared tile
};
struct MacSeg {
  int32_t kind, K, psi_ld, op_ld;   // op_ld: row stride of the padded operator block
  int64_t psi_off, op_off;          // op_off: in MacroPlan::dense
  double c;
  int32_t st0, nst;     // first stage of the segment in the tile, stage count
  int32_t src[kMac];    // gathered side (SEG_KN: columns, SEG_MK: rows), -1 = zero
  float scl[kMac];      // and its scale
};
struct MacGG {
  double c;
  int64_t row[kMac];    // psi_off + srcA(m0 + i) * psi_ld, -1 = zero row
  int32_t col[kMac];    // srcB(n0 + j), -1 = zero column
  double rs[kMac], cs[kMac];
};
// One workgroup's part of one tile: stages [s0, s1) of the tile, share
// `split` of its tile's nsplit, spanning the tile's segments g0 .. g0 + ng - 1
// (ng <= kMacSegLds).
struct MacItem {
  int32_t tile, split, s0, s1;
  int32_t g0, ng, pad[2];
};
static_assert(sizeof(MacTile) % 8 == 0 && sizeof(MacSeg) % 8 == 0 && sizeof(MacGG) % 8 == 0,
              "macro records keep 8-byte alignment");

struct MacroPlan {
  std::vector<MacTile> tiles;
  std::vector<MacSeg> segs;
  std::vector<MacGG> ggs;
  std::vector<MacItem> items;     // workgroup w: items wg_start[w] .. wg_start[w + 1] - 1
  std::vector<int32_t> wg_start;
  std::vector<int32_t> shared;    // tiles split between workgroups
  int32_t nparts = 0;             // partial tiles (kMac * kMac floats each)
  int64_t stages = 0;             // stages over all tiles
  std::vector<CoefRef> coef_seg, coef_gg;   // coefficient fields in segs / ggs
  // the operator blocks the segments read, FP32, row-major with rows padded
  // with zeros to a whole number of stages (so that a stage never needs a
  // mask: past a segment's end the operator side reads zeros), plus
  // kPoolPad zeros at the end
  std::vector<float> dense;
};

// Builds the macro plan of a product plan for at most max_wgs workgroups
// (fewer when there are not min_stages stages per workgroup); pool32 is the
// plan's FP32 operator pool (dense_f32).
void build_macro(const Plan& p, const std::vector<float>& pool32, int max_wgs, int min_stages,
                 MacroPlan& mp);

}  // namespace dmrg
