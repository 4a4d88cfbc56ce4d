// Host-side plan of one superblock product (no HIP calls; builds with any
// C++17 compiler).
//
// The plan is the integer part of H*psi: which S' sector pairs with which E'
// sector (effective q adds, Sec. 3.2: q_S + q_E = q_target), where each block
// of psi starts, and, for every output block and term, which source block
// and operator blocks feed it (Y_q += c A[q<-q'] Psi_q' B^T).  Operator
// blocks whose rows hold at most one nonzero are turned into gathers
// (index + scale); the rest stay dense.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dmrg.h"

namespace dmrg {

// Kinds of per-block work.
enum SegKind : int32_t {
  SEG_KN = 0,   // Y += c * Aop * (Psi' G_B^T): dense A (stored k-major), B side identity/gather
  SEG_MK = 1,   // Y += c * (G_A Psi') * Bop^T: A side identity/gather, dense B (stored row-major)
  SEG_GG = 2    // Y += c * (G_A Psi' G_B^T): elementwise, both sides identity/gather
};

// One (term, output block) contribution.  Offsets are in elements.
struct SegDesc {
  int32_t kind;
  int32_t K;          // contraction length (SEG_KN: a', SEG_MK: b'); 0 for SEG_GG
  double c;           // term coefficient
  int64_t psi_off;    // source block Psi' offset
  int32_t psi_ld;     // columns of Psi' (b')
  int32_t psi_rows;   // rows of Psi' (a')
  int64_t op_off;     // dense pool offset of the operator block (-1: none)
  int32_t op_ld;      // leading dimension of the stored operator block
  int32_t gA;         // gather pool offset for output rows (-1: identity)
  int32_t gB;         // gather pool offset for output columns (-1: identity)
  int32_t term;       // term index k
  int32_t ch0;        // index of this segment's first chunk in its block's chunk sequence
};

// One 32 x 32 output tile of one target block.
struct TileDesc {
  int64_t y_off;      // output block offset
  int32_t a, b;       // output block rows, columns
  int32_t m0, n0;     // tile origin inside the block
  int32_t seg0, nseg; // the block's segments
  int32_t nchunk;     // contraction chunks over all of the block's matrix-core segments
  int32_t ngemm;      // segments [seg0, seg0 + ngemm) are matrix-core ones, the rest elementwise
  int32_t ldy;        // row stride of the output block (b for psi blocks)
  int32_t pad;
};

constexpr int kXcds = 8;     // MI355X: 8 XCDs; workgroup b runs on XCD b % 8
constexpr int kPersistentWGs = 256;   // one workgroup per compute unit

constexpr int kTile = 32;    // output tile edge
constexpr int kChunk = 16;   // contraction chunk

// ---------------------------------------------------------------------------
// Tile images: for every workgroup slot of the fused product, one contiguous
// record of everything its 32 x 32 output tile needs, so that the workgroup
// fetches it into LDS with a single coalesced read and no later lookup
// depends on another load.  Layout (32-bit words, 8-byte aligned records):
//   ImgHeader, then ngemm ImgSeg (matrix-core segments, in chunk order),
//   then ngg ImgGG (elementwise segments).  An image with a == 0 is an idle
//   slot.
// ---------------------------------------------------------------------------
struct ImgHeader {
  int64_t y_off;
  int32_t a, b, m0, n0, ldy;
  int32_t ngemm, ngg, nchunk;
  int32_t pad[6];
};
struct ImgSeg {
  int32_t kind, K, psi_ld, op_ld;
  int64_t psi_off, op_off;
  double c;
  int32_t ch0, pad;   // SEG_KN: first source column of the segment's 32-column window
  int32_t src[kTile];   // gathered side (SEG_KN: columns, SEG_MK: rows): source index, -1 = zero
  double scl[kTile];    // and its scale
};
struct ImgGG {
  double c;
  int64_t row[kTile];   // psi_off + srcA(m0 + i) * psi_ld, -1 = zero row
  int32_t col[kTile];   // srcB(n0 + j), -1 = zero column
  double rs[kTile], cs[kTile];
};
constexpr int kHdrWords = (int)(sizeof(ImgHeader) / 4);
constexpr int kSegWords = (int)(sizeof(ImgSeg) / 4);
constexpr int kGGWords = (int)(sizeof(ImgGG) / 4);
constexpr int kImgWords = 6144;   // LDS room for one image (24 KiB)
static_assert(sizeof(ImgHeader) == 64 && sizeof(ImgSeg) % 8 == 0 && sizeof(ImgGG) % 8 == 0,
              "image records must keep 8-byte alignment");

// Where a term coefficient sits in a device buffer (byte offset of a double),
// so that new coefficients can be written in place by a kernel.
struct CoefRef {
  int64_t off;
  int32_t term;
  int32_t pad;
};

// Images of the given tiles in launch order (order[slot] = tile, -1 idle; an
// empty order means slot = tile).  stride (words, a multiple of 4) is the
// largest image.  Returns false with err set if an image exceeds kImgWords.
// coefs, if given, receives the byte offset and term of every coefficient
// field in out.
bool build_images(const std::vector<TileDesc>& tiles, const std::vector<SegDesc>& segs,
                  const std::vector<int32_t>& order, const std::vector<int32_t>& gsrc,
                  const std::vector<double>& gscale, std::vector<uint32_t>& out,
                  int32_t& stride, std::string& err, std::vector<CoefRef>* coefs = nullptr);

struct Plan {
  // bases
  std::vector<int64_t> qS, qE;
  std::vector<int32_t> dS, dE;
  int64_t q_target = 0;
  // target pairs (ordered by S' sector)
  std::vector<int32_t> pair_s, pair_e;
  std::vector<int64_t> pair_off;
  int64_t D = 0;
  int64_t q_in = 0;               // input sector (== q_target for a Hamiltonian)
  int64_t D_in = 0;
  // terms
  int32_t nterms = 0;
  std::vector<double> coeff;
  // work
  std::vector<SegDesc> segs;      // grouped by output pair
  std::vector<int32_t> pair_seg0, pair_nseg;
  std::vector<TileDesc> tiles;    // sorted by decreasing cost
  // The fused product runs one workgroup per compute unit over lists of
  // tiles: workgroup w takes slots wg_start[w] .. wg_start[w + 1] - 1, slot s
  // being tile order[s].
  std::vector<int32_t> order;
  std::vector<int32_t> wg_start;
  // staged operator data (FP64; converted at upload)
  std::vector<double> dense;      // dense pool
  // A-side blocks of the pool, stored k-major (element (m, k) at off + k * rows + m);
  // the FP32 pool holds them row-major (off + m * cols + k)
  std::vector<int64_t> kmajor_off;
  std::vector<int32_t> kmajor_rows, kmajor_cols;
  std::vector<int32_t> gsrc;      // gather pool: source index (-1: zero row)
  std::vector<double> gscale;     // gather pool: scale
  // statistics of one product
  double flops_alg = 0, flops_exec = 0, bytes_dense = 0;
  int64_t gemm_elems = 0;         // sum of padded K over tiles (for reporting)
};

// Builds `plan` (and, with transpose=true, the plan of H^T = sum c A^T (x) B^T).
// Returns DMRG_OK or an error code with `err` set.
dmrg_status build_plan(const dmrg_basis* S, const dmrg_basis* E, int64_t q_target,
                       int32_t nterms, const dmrg_term* terms, bool transpose, Plan& plan,
                       std::string& err);

// Plan of an operator between two target sectors: input vectors live in the
// q_in sector, outputs in q_out; every term must shift q by q_out - q_in.
dmrg_status build_plan_between(const dmrg_basis* S, const dmrg_basis* E, int64_t q_in,
                               int64_t q_out, int32_t nterms, const dmrg_term* terms,
                               bool transpose, Plan& plan, std::string& err);

// Recomputes statistics for an element size of the staged operators.
double plan_bytes_alg(const Plan& p, int elem_bytes);

// The FP32 operator pool of a plan: the FP64 pool rounded, with the A-side
// blocks row-major, plus kPoolPad zero elements at the end.
constexpr int kPoolPad = 16;
void dense_f32(const Plan& p, std::vector<float>& out);

}  // namespace dmrg
