// Host plan of one superblock product: sector matching, psi layout, block
// classification, segment lists and the cost-sorted tile schedule.
#include "plan.h"

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstring>
#include <numeric>
#include <sstream>

namespace dmrg {

namespace {

struct SideBlock {
  int32_t src_sec = -1;   // source sector (column sector of the block)
  bool dense = false;
  bool empty = false;
  int64_t op_off = -1;    // dense pool offset
  int32_t op_ld = 0;
  int32_t g_off = -1;     // gather pool offset
};

dmrg_status check_basis(const dmrg_basis* b, const char* name, std::string& err) {
  std::ostringstream os;
  if (b == nullptr || b->q == nullptr || b->dim == nullptr || b->nsec < 1) {
    os << name << ": null or empty basis";
    err = os.str();
    return DMRG_E_ARG;
  }
  for (int32_t s = 0; s < b->nsec; ++s) {
    if (b->dim[s] < 1) {
      os << name << ": sector " << s << " has dimension " << b->dim[s];
      err = os.str();
      return DMRG_E_SHAPE;
    }
    if (s > 0 && b->q[s] <= b->q[s - 1]) {
      os << name << ": quantum numbers not strictly increasing at sector " << s;
      err = os.str();
      return DMRG_E_QN;
    }
  }
  return DMRG_OK;
}

// Element (r, c) of block `k` of `op`, transposed if requested.
inline double elem(const dmrg_op* op, int k, int32_t ncols_stored, bool tr, int32_t r,
                   int32_t c) {
  return tr ? op->blk[k][(int64_t)c * ncols_stored + r] : op->blk[k][(int64_t)r * ncols_stored + c];
}

// Validates one side's operator and stages its blocks.  For the A side the
// dense blocks are stored k-major (column-major of the block) for SEG_KN; for
// the B side row-major for SEG_MK.
dmrg_status stage_side(const dmrg_op* op, const dmrg_basis* b, bool a_side, bool tr,
                       const char* name, int term, std::vector<SideBlock>& by_row, Plan& plan,
                       std::string& err) {
  std::ostringstream os;
  by_row.assign(b->nsec, SideBlock());
  if (op == nullptr) return DMRG_OK;
  if (op->nblk < 0 || (op->nblk > 0 && (op->row_sec == nullptr || op->col_sec == nullptr ||
                                        op->blk == nullptr))) {
    os << "term " << term << " " << name << ": null block arrays";
    err = os.str();
    return DMRG_E_ARG;
  }
  std::vector<char> seen(b->nsec, 0);
  for (int32_t k = 0; k < op->nblk; ++k) {
    int32_t r0 = op->row_sec[k], c0 = op->col_sec[k];
    if (r0 < 0 || r0 >= b->nsec || c0 < 0 || c0 >= b->nsec) {
      os << "term " << term << " " << name << ": block " << k << " sector out of range";
      err = os.str();
      return DMRG_E_ARG;
    }
    if (op->blk[k] == nullptr) {
      os << "term " << term << " " << name << ": block " << k << " is null";
      err = os.str();
      return DMRG_E_ARG;
    }
    if (b->q[r0] - b->q[c0] != op->delta) {
      os << "term " << term << " " << name << ": block " << k << " maps q=" << b->q[c0]
         << " to q=" << b->q[r0] << " but the operator's shift is " << op->delta;
      err = os.str();
      return DMRG_E_QN;
    }
    // logical block after the optional transpose
    int32_t r = tr ? c0 : r0, c = tr ? r0 : c0;
    if (seen[r]) {
      os << "term " << term << " " << name << ": two blocks in row sector " << r;
      err = os.str();
      return DMRG_E_QN;
    }
    seen[r] = 1;
    const int32_t rows = b->dim[r], cols = b->dim[c];
    const int32_t stored_cols = b->dim[c0];
    bool gather = true, empty = true;
    for (int32_t i = 0; i < rows && gather; ++i) {
      int nz = 0;
      for (int32_t j = 0; j < cols; ++j)
        if (elem(op, k, stored_cols, tr, i, j) != 0.0) ++nz;
      if (nz > 1) gather = false;
      if (nz > 0) empty = false;
    }
    SideBlock sb;
    sb.src_sec = c;
    if (empty) {
      sb.empty = true;
    } else if (gather) {
      sb.g_off = (int32_t)plan.gsrc.size();
      for (int32_t i = 0; i < rows; ++i) {
        int32_t src = -1;
        double v = 0.0;
        for (int32_t j = 0; j < cols; ++j) {
          double x = elem(op, k, stored_cols, tr, i, j);
          if (x != 0.0) {
            src = j;
            v = x;
          }
        }
        plan.gsrc.push_back(src);
        plan.gscale.push_back(v);
      }
    } else {
      sb.dense = true;
      sb.op_off = (int64_t)plan.dense.size();
      if (a_side) {
        // k-major: element (m, kk) of the block at [kk * rows + m]
        sb.op_ld = rows;
        plan.kmajor_off.push_back(sb.op_off);
        plan.kmajor_rows.push_back(rows);
        plan.kmajor_cols.push_back(cols);
        plan.dense.resize(plan.dense.size() + (size_t)rows * cols);
        double* dst = plan.dense.data() + sb.op_off;
        for (int32_t i = 0; i < rows; ++i)
          for (int32_t j = 0; j < cols; ++j) dst[(int64_t)j * rows + i] = elem(op, k, stored_cols, tr, i, j);
      } else {
        // row-major: element (n, kk) at [n * cols + kk]
        sb.op_ld = cols;
        plan.dense.resize(plan.dense.size() + (size_t)rows * cols);
        double* dst = plan.dense.data() + sb.op_off;
        for (int32_t i = 0; i < rows; ++i)
          for (int32_t j = 0; j < cols; ++j) dst[(int64_t)i * cols + j] = elem(op, k, stored_cols, tr, i, j);
      }
    }
    by_row[r] = sb;
  }
  return DMRG_OK;
}

}  // namespace

dmrg_status build_plan(const dmrg_basis* S, const dmrg_basis* E, int64_t q_target,
                       int32_t nterms, const dmrg_term* terms, bool transpose, Plan& plan,
                       std::string& err) {
  return build_plan_between(S, E, q_target, q_target, nterms, terms, transpose, plan, err);
}

dmrg_status build_plan_between(const dmrg_basis* S, const dmrg_basis* E, int64_t q_in,
                               int64_t q_out, int32_t nterms, const dmrg_term* terms,
                               bool transpose, Plan& plan, std::string& err) {
  // a transposed operator maps q_out back to q_in
  if (transpose) std::swap(q_in, q_out);
  const int64_t q_target = q_out;
  dmrg_status st;
  if ((st = check_basis(S, "S'", err)) != DMRG_OK) return st;
  if ((st = check_basis(E, "E'", err)) != DMRG_OK) return st;
  if (nterms < 0 || (nterms > 0 && terms == nullptr)) {
    err = "null or negative term list";
    return DMRG_E_ARG;
  }
  plan = Plan();
  plan.qS.assign(S->q, S->q + S->nsec);
  plan.qE.assign(E->q, E->q + E->nsec);
  plan.dS.assign(S->dim, S->dim + S->nsec);
  plan.dE.assign(E->dim, E->dim + E->nsec);
  plan.q_target = q_target;
  plan.nterms = nterms;

  // target pairs: S' sector i with the E' sector of q = q_target - q_i
  std::vector<int32_t> pair_of_s(S->nsec, -1);
  int64_t off = 0;
  for (int32_t i = 0; i < S->nsec; ++i) {
    const int64_t want = q_target - S->q[i];
    const int64_t* it = std::lower_bound(E->q, E->q + E->nsec, want);
    if (it != E->q + E->nsec && *it == want) {
      pair_of_s[i] = (int32_t)plan.pair_s.size();
      plan.pair_s.push_back(i);
      plan.pair_e.push_back((int32_t)(it - E->q));
      plan.pair_off.push_back(off);
      off += (int64_t)S->dim[i] * E->dim[it - E->q];
    }
  }
  if (plan.pair_s.empty()) {
    err = "no S'/E' sector pair reaches the target quantum number";
    return DMRG_E_QN;
  }
  plan.D = off;
  const int32_t npairs = (int32_t)plan.pair_s.size();
  // input layout (the same rule, for q_in)
  std::vector<int32_t> in_pair_e(S->nsec, -1);
  std::vector<int64_t> in_off(S->nsec, -1);
  int64_t off_in = 0;
  for (int32_t i = 0; i < S->nsec; ++i) {
    const int64_t want = q_in - S->q[i];
    const int64_t* it = std::lower_bound(E->q, E->q + E->nsec, want);
    if (it != E->q + E->nsec && *it == want) {
      in_pair_e[i] = (int32_t)(it - E->q);
      in_off[i] = off_in;
      off_in += (int64_t)S->dim[i] * E->dim[it - E->q];
    }
  }
  if (off_in == 0) {
    err = "no S'/E' sector pair reaches the input quantum number";
    return DMRG_E_QN;
  }
  plan.q_in = q_in;
  plan.D_in = off_in;

  // stage operators
  std::vector<std::vector<SideBlock>> Aside(nterms), Bside(nterms);
  for (int32_t k = 0; k < nterms; ++k) {
    const dmrg_term& t = terms[k];
    int64_t dA = t.A ? t.A->delta : 0, dB = t.B ? t.B->delta : 0;
    if (transpose) {
      dA = -dA;
      dB = -dB;
    }
    if (dA + dB != q_out - q_in) {
      std::ostringstream os;
      os << "term " << k << " changes the total quantum number by " << dA + dB << ", not by "
         << q_out - q_in;
      err = os.str();
      return DMRG_E_QN;
    }
    if ((st = stage_side(t.A, S, true, transpose, "A", k, Aside[k], plan, err)) != DMRG_OK) return st;
    if ((st = stage_side(t.B, E, false, transpose, "B", k, Bside[k], plan, err)) != DMRG_OK) return st;
    plan.coeff.push_back(t.c);
  }

  // segments per output pair
  plan.pair_seg0.resize(npairs);
  plan.pair_nseg.resize(npairs);
  for (int32_t p = 0; p < npairs; ++p) {
    const int32_t i = plan.pair_s[p], j = plan.pair_e[p];
    plan.pair_seg0[p] = (int32_t)plan.segs.size();
    for (int32_t k = 0; k < nterms; ++k) {
      SideBlock a, b;
      if (terms[k].A) {
        a = Aside[k][i];
        if (a.src_sec < 0 || a.empty) continue;
      } else {
        a.src_sec = i;
      }
      if (terms[k].B) {
        b = Bside[k][j];
        if (b.src_sec < 0 || b.empty) continue;
      } else {
        b.src_sec = j;
      }
      if (in_pair_e[a.src_sec] != b.src_sec) continue;   // source block outside the input sector
      SegDesc sg{};
      sg.c = terms[k].c;
      sg.term = k;
      sg.psi_off = in_off[a.src_sec];
      sg.psi_ld = plan.dE[b.src_sec];
      sg.psi_rows = plan.dS[a.src_sec];
      sg.op_off = -1;
      sg.op_ld = 0;
      sg.gA = a.g_off;
      sg.gB = b.g_off;
      if (a.dense && b.dense) {
        std::ostringstream os;
        os << "term " << k << " has dense blocks on both sides (not supported by the fused kernel)";
        err = os.str();
        return DMRG_E_UNSUPPORTED;
      } else if (a.dense) {
        sg.kind = SEG_KN;
        sg.K = plan.dS[a.src_sec];
        sg.op_off = a.op_off;
        sg.op_ld = a.op_ld;
        sg.gA = -1;
      } else if (b.dense) {
        sg.kind = SEG_MK;
        sg.K = plan.dE[b.src_sec];
        sg.op_off = b.op_off;
        sg.op_ld = b.op_ld;
        sg.gB = -1;
      } else {
        sg.kind = SEG_GG;
        sg.K = 0;
      }
      plan.segs.push_back(sg);
    }
    plan.pair_nseg[p] = (int32_t)plan.segs.size() - plan.pair_seg0[p];
    // matrix-core segments first, elementwise ones after (stable)
    std::stable_partition(plan.segs.begin() + plan.pair_seg0[p], plan.segs.end(),
                          [](const SegDesc& sg) { return sg.kind != SEG_GG; });
    if (plan.pair_nseg[p] > 32) {
      std::ostringstream os;
      os << "target block " << p << " receives " << plan.pair_nseg[p]
         << " terms; the fused kernel takes at most 32 per block";
      err = os.str();
      return DMRG_E_UNSUPPORTED;
    }
  }

  // tiles; each block's segments know where their chunks start
  std::vector<int64_t> tile_cost;
  std::vector<int32_t> tile_pair;
  for (int32_t p = 0; p < npairs; ++p) {
    const int32_t a = plan.dS[plan.pair_s[p]], b = plan.dE[plan.pair_e[p]];
    int64_t cost = 0, kpad = 0;
    int32_t nch = 0, ngemm = 0;
    for (int32_t s = 0; s < plan.pair_nseg[p]; ++s) {
      SegDesc& sg = plan.segs[plan.pair_seg0[p] + s];
      const double c2 = 2.0 * a * b;
      sg.ch0 = nch;
      if (sg.kind == SEG_GG) {
        cost += 2;
        plan.flops_alg += c2;
      } else {
        const int32_t c = (sg.K + kChunk - 1) / kChunk;
        nch += c;
        ++ngemm;
        kpad += (int64_t)c * kChunk;
        cost += 4 * c;
        plan.flops_alg += c2 * sg.K;
        const int32_t gathered = sg.kind == SEG_KN ? (sg.gB >= 0) : (sg.gA >= 0);
        if (gathered) plan.flops_alg += 2.0 * sg.K * (sg.kind == SEG_KN ? b : a);
      }
    }
    // a tile's time: a fixed part (image, first loads, reduction and stores,
    // about as long as 25 contraction chunks) and its chunks and elementwise
    // terms
    const int64_t tcost = 100 + cost;
    for (int32_t m0 = 0; m0 < a; m0 += kTile)
      for (int32_t n0 = 0; n0 < b; n0 += kTile) {
        TileDesc t{};
        t.y_off = plan.pair_off[p];
        t.a = a;
        t.b = b;
        t.m0 = m0;
        t.n0 = n0;
        t.seg0 = plan.pair_seg0[p];
        t.nseg = plan.pair_nseg[p];
        t.nchunk = nch;
        t.ngemm = ngemm;
        t.ldy = b;
        plan.tiles.push_back(t);
        tile_cost.push_back(tcost);
        tile_pair.push_back(p);
        plan.flops_exec += 2.0 * kTile * kTile * (double)kpad;
        plan.gemm_elems += kpad;
      }
  }
  // Work lists of the persistent launch: min(kPersistentWGs, tiles)
  // workgroups, one per compute unit, each taking a list of tiles.  Tiles go
  // to the lists by LPT on their estimated cost (longest first, each to the
  // least loaded list), so that every compute unit ends at about the same
  // time even when a few large blocks hold most of the work; a tile stays
  // on the XCD (workgroup w runs on XCD w % kXcds) of the previous tile of
  // its block when a list there is about as lightly loaded as the least
  // loaded one (within a quarter of the tile's cost), so that a block's
  // operators and psi rows are fetched into few L2s without stacking tiles
  // on one compute unit while another idles.  Within a list the most
  // expensive tile runs first.
  {
    const int ntiles = (int)plan.tiles.size();
    const int nwg = std::max(1, std::min(kPersistentWGs, ntiles));
    std::vector<int32_t> tidx(ntiles);
    for (int t = 0; t < ntiles; ++t) tidx[t] = t;
    std::stable_sort(tidx.begin(), tidx.end(),
                     [&](int32_t x, int32_t y) { return tile_cost[x] > tile_cost[y]; });
    std::vector<int64_t> load(nwg, 0);
    std::vector<int32_t> last_xcd(npairs, -1);
    std::vector<std::vector<int32_t>> lists(nwg);
    for (int32_t t : tidx) {
      int best = 0;
      for (int w = 1; w < nwg; ++w)
        if (load[w] < load[best]) best = w;
      const int pref = last_xcd[tile_pair[t]];
      if (pref >= 0 && best % kXcds != pref) {
        int alt = -1;
        for (int w = pref; w < nwg; w += kXcds)
          if (alt < 0 || load[w] < load[alt]) alt = w;
        if (alt >= 0 && 4 * load[alt] <= 4 * load[best] + tile_cost[t]) best = alt;
      }
      lists[best].push_back(t);
      load[best] += tile_cost[t];
      last_xcd[tile_pair[t]] = best % kXcds;
    }
    plan.order.clear();
    plan.wg_start.assign(1, 0);
    for (auto& l : lists) {
      for (int32_t t : l) plan.order.push_back(t);
      plan.wg_start.push_back((int32_t)plan.order.size());
    }
  }
  plan.bytes_dense = 8.0 * plan.dense.size();
  return DMRG_OK;
}

bool build_images(const std::vector<TileDesc>& tiles, const std::vector<SegDesc>& segs,
                  const std::vector<int32_t>& order, const std::vector<int32_t>& gsrc,
                  const std::vector<double>& gscale, std::vector<uint32_t>& out,
                  int32_t& stride, std::string& err, std::vector<CoefRef>* coefs) {
  const size_t nslots = order.empty() ? tiles.size() : order.size();
  auto tile_of = [&](size_t slot) { return order.empty() ? (int32_t)slot : order[slot]; };
  // gather entry of output index idx (< limit) through pool offset g (-1: identity)
  auto gather = [&](int32_t g, int32_t idx, int32_t limit, int32_t& src, double& scl) {
    src = -1;
    scl = 0.0;
    if (idx >= limit) return;
    if (g < 0) {
      src = idx;
      scl = 1.0;
    } else {
      src = gsrc[g + idx];
      scl = src >= 0 ? gscale[g + idx] : 0.0;
    }
  };
  // A SEG_KN segment reads Psi' through a window of 32 consecutive source
  // columns; a tile whose gathered columns span more is given one image
  // segment per window (each keeps only its own columns), all with the
  // segment's coefficient and contraction.
  auto windows = [&](const SegDesc& sg, const TileDesc& t) {
    std::vector<std::pair<int32_t, std::vector<int32_t>>> w;   // (base column, tile columns)
    std::vector<std::pair<int32_t, int32_t>> cols;             // (source column, tile column)
    for (int32_t i = 0; i < kTile; ++i) {
      int32_t src;
      double scl;
      gather(sg.gB, t.n0 + i, t.b, src, scl);
      if (src >= 0) cols.push_back({src, i});
    }
    std::sort(cols.begin(), cols.end());
    for (const auto& c : cols) {
      if (w.empty() || c.first >= w.back().first + kTile) w.push_back({c.first, {}});
      w.back().second.push_back(c.second);
    }
    return w;
  };
  auto image_segs = [&](const TileDesc& t) {
    int32_t n = 0;
    for (int32_t s = 0; s < t.ngemm; ++s) {
      const SegDesc& sg = segs[t.seg0 + s];
      n += sg.kind == SEG_KN ? (int32_t)windows(sg, t).size() : 1;
    }
    return n;
  };
  int32_t words = kHdrWords;
  for (size_t slot = 0; slot < nslots; ++slot) {
    const int32_t ti = tile_of(slot);
    if (ti < 0) continue;
    const TileDesc& t = tiles[ti];
    words = std::max(words, kHdrWords + image_segs(t) * kSegWords + (t.nseg - t.ngemm) * kGGWords);
  }
  if (words > kImgWords) {
    std::ostringstream os;
    os << "a target block's terms need a " << 4 * words << "-byte tile image; the fused kernel holds "
       << 4 * kImgWords;
    err = os.str();
    return false;
  }
  stride = (words + 3) / 4 * 4;
  out.assign(nslots * (size_t)stride, 0u);
  if (coefs) coefs->clear();
  auto note = [&](const uint32_t* rec, size_t field, int32_t term) {
    if (coefs)
      coefs->push_back({(int64_t)((rec - out.data()) * sizeof(uint32_t) + field), term, 0});
  };
  for (size_t slot = 0; slot < nslots; ++slot) {
    const int32_t ti = tile_of(slot);
    uint32_t* img = out.data() + slot * (size_t)stride;
    ImgHeader h{};
    if (ti >= 0) {
      const TileDesc& t = tiles[ti];
      h.y_off = t.y_off;
      h.a = t.a;
      h.b = t.b;
      h.m0 = t.m0;
      h.n0 = t.n0;
      h.ldy = t.ldy;
      h.ngg = t.nseg - t.ngemm;
      int32_t nrec = 0, nch = 0;
      for (int32_t s = 0; s < t.ngemm; ++s) {
        const SegDesc& sg = segs[t.seg0 + s];
        ImgSeg r{};
        r.kind = sg.kind;
        r.K = sg.K;
        r.psi_ld = sg.psi_ld;
        r.op_ld = sg.op_ld;
        r.psi_off = sg.psi_off;
        r.op_off = sg.op_off;
        r.c = sg.c;
        const int32_t c = (sg.K + kChunk - 1) / kChunk;
        if (sg.kind == SEG_KN) {
          for (const auto& win : windows(sg, t)) {
            ImgSeg w = r;
            for (int32_t i = 0; i < kTile; ++i) {
              w.src[i] = -1;
              w.scl[i] = 0.0;
            }
            for (int32_t i : win.second) gather(sg.gB, t.n0 + i, t.b, w.src[i], w.scl[i]);
            w.pad = win.first;
            w.ch0 = nch;
            nch += c;
            note(img + kHdrWords + nrec * kSegWords, offsetof(ImgSeg, c), sg.term);
            std::memcpy(img + kHdrWords + nrec++ * kSegWords, &w, sizeof(w));
          }
        } else {
          for (int32_t i = 0; i < kTile; ++i) gather(sg.gA, t.m0 + i, t.a, r.src[i], r.scl[i]);
          r.ch0 = nch;
          nch += c;
          note(img + kHdrWords + nrec * kSegWords, offsetof(ImgSeg, c), sg.term);
          std::memcpy(img + kHdrWords + nrec++ * kSegWords, &r, sizeof(r));
        }
      }
      h.ngemm = nrec;
      h.nchunk = nch;
      for (int32_t q = 0; q < t.nseg - t.ngemm; ++q) {
        const SegDesc& sg = segs[t.seg0 + t.ngemm + q];
        ImgGG r{};
        r.c = sg.c;
        for (int32_t i = 0; i < kTile; ++i) {
          int32_t src;
          double scl;
          gather(sg.gA, t.m0 + i, t.a, src, scl);
          r.row[i] = src >= 0 ? sg.psi_off + (int64_t)src * sg.psi_ld : -1;
          r.rs[i] = scl;
          gather(sg.gB, t.n0 + i, t.b, src, scl);
          r.col[i] = src;
          r.cs[i] = scl;
        }
        note(img + kHdrWords + nrec * kSegWords + q * kGGWords, offsetof(ImgGG, c), sg.term);
        std::memcpy(img + kHdrWords + nrec * kSegWords + q * kGGWords, &r, sizeof(r));
      }
    }
    std::memcpy(img, &h, sizeof(h));
  }
  return true;
}

void dense_f32(const Plan& p, std::vector<float>& out) {
  out.assign(p.dense.size() + kPoolPad, 0.f);
  for (size_t i = 0; i < p.dense.size(); ++i) out[i] = (float)p.dense[i];
  for (size_t b = 0; b < p.kmajor_off.size(); ++b) {
    const int64_t off = p.kmajor_off[b];
    const int32_t rows = p.kmajor_rows[b], cols = p.kmajor_cols[b];
    for (int32_t m = 0; m < rows; ++m)
      for (int32_t k = 0; k < cols; ++k)
        out[off + (int64_t)m * cols + k] = (float)p.dense[off + (int64_t)k * rows + m];
  }
}

double plan_bytes_alg(const Plan& p, int elem_bytes) {
  // operators once, gather entries once, psi read once and y written once
  return (double)elem_bytes * p.dense.size() + 12.0 * p.gsrc.size() + 8.0 * (p.D_in + p.D);
}

}  // namespace dmrg
