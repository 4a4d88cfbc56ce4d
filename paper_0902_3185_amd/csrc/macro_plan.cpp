// Macro-tile plan (see macro.h): 64 x 64 tiles, stages of 32 contraction
// positions, equal contiguous shares of all stages per workgroup.
#include "macro.h"

#include <algorithm>
#include <cstddef>
#include <map>

namespace dmrg {

void build_macro(const Plan& p, const std::vector<float>& pool32, int max_wgs, int min_stages,
                 MacroPlan& mp) {
  mp = MacroPlan{};
  // operator block at FP32-pool offset off (rows x K row-major there) ->
  // offset of its padded copy
  std::map<int64_t, int64_t> placed;
  auto place = [&](int64_t off, int32_t rows, int32_t K) {
    auto it = placed.find(off);
    if (it != placed.end()) return it->second;
    const int32_t ld = (K + kMacStage - 1) / kMacStage * kMacStage;
    const int64_t at = (int64_t)mp.dense.size();
    mp.dense.resize(mp.dense.size() + (size_t)rows * ld, 0.f);
    for (int32_t r = 0; r < rows; ++r)
      for (int32_t k = 0; k < K; ++k) mp.dense[at + (int64_t)r * ld + k] = pool32[off + (int64_t)r * K + k];
    placed[off] = at;
    return at;
  };
  // gather entry of output index idx (< limit) through pool offset g (-1: identity)
  auto gather = [&](int32_t g, int32_t idx, int32_t limit, int32_t& src, double& scl) {
    src = -1;
    scl = 0.0;
    if (idx >= limit) return;
    if (g < 0) {
      src = idx;
      scl = 1.0;
    } else {
      src = p.gsrc[g + idx];
      scl = src >= 0 ? p.gscale[g + idx] : 0.0;
    }
  };
  // tiles block by block (pairs in plan order), row-major inside a block, so
  // that a block's tiles take consecutive shares
  for (size_t q = 0; q < p.pair_s.size(); ++q) {
    const int32_t a = p.dS[p.pair_s[q]], b = p.dE[p.pair_e[q]];
    const int32_t s0 = p.pair_seg0[q], ns = p.pair_nseg[q];
    for (int32_t m0 = 0; m0 < a; m0 += kMac)
      for (int32_t n0 = 0; n0 < b; n0 += kMac) {
        MacTile t{};
        t.y_off = p.pair_off[q];
        t.a = a;
        t.b = b;
        t.m0 = m0;
        t.n0 = n0;
        t.ldy = b;
        t.seg0 = (int32_t)mp.segs.size();
        t.gg0 = (int32_t)mp.ggs.size();
        int32_t st = 0;
        for (int32_t s = 0; s < ns; ++s) {
          const SegDesc& sg = p.segs[s0 + s];
          if (sg.kind == SEG_GG) {
            MacGG r{};
            r.c = sg.c;
            for (int32_t i = 0; i < kMac; ++i) {
              int32_t src;
              double scl;
              gather(sg.gA, m0 + i, a, src, scl);
              r.row[i] = src >= 0 ? sg.psi_off + (int64_t)src * sg.psi_ld : -1;
              r.rs[i] = scl;
              gather(sg.gB, n0 + i, b, src, scl);
              r.col[i] = src;
              r.cs[i] = scl;
            }
            mp.coef_gg.push_back({(int64_t)(mp.ggs.size() * sizeof(MacGG) + offsetof(MacGG, c)), sg.term, 0});
            mp.ggs.push_back(r);
            continue;
          }
          MacSeg r{};
          r.kind = sg.kind;
          r.K = sg.K;
          r.psi_ld = sg.psi_ld;
          // the FP32 pool holds both kinds' operator blocks row-major, rows x K
          // (SEG_KN: a rows; SEG_MK: b rows)
          r.op_ld = (sg.K + kMacStage - 1) / kMacStage * kMacStage;
          r.psi_off = sg.psi_off;
          r.op_off = place(sg.op_off, sg.kind == SEG_KN ? a : b, sg.K);
          r.c = sg.c;
          r.st0 = st;
          r.nst = (sg.K + kMacStage - 1) / kMacStage;
          st += r.nst;
          for (int32_t i = 0; i < kMac; ++i) {
            int32_t src;
            double scl;
            if (sg.kind == SEG_KN)
              gather(sg.gB, n0 + i, b, src, scl);
            else
              gather(sg.gA, m0 + i, a, src, scl);
            r.src[i] = src;
            r.scl[i] = (float)scl;
          }
          mp.coef_seg.push_back({(int64_t)(mp.segs.size() * sizeof(MacSeg) + offsetof(MacSeg, c)), sg.term, 0});
          mp.segs.push_back(r);
        }
        t.nseg = (int32_t)mp.segs.size() - t.seg0;
        t.ngg = (int32_t)mp.ggs.size() - t.gg0;
        t.nstage = st;
        t.nsplit = 1;
        t.part0 = -1;
        mp.stages += st;
        mp.tiles.push_back(t);
      }
  }
  mp.dense.resize(mp.dense.size() + kPoolPad, 0.f);
  // equal shares of the stage sequence
  const int64_t total = mp.stages;
  int nwg = (int)std::min<int64_t>(max_wgs, std::max<int64_t>(1, (total + min_stages - 1) / min_stages));
  if (nwg >= kXcds) nwg -= nwg % kXcds;
  const int64_t per = std::max<int64_t>(1, (total + nwg - 1) / nwg);
  std::vector<std::vector<MacItem>> share(nwg);
  int64_t G = 0;
  for (size_t ti = 0; ti < mp.tiles.size(); ++ti) {
    MacTile& t = mp.tiles[ti];
    if (t.nstage == 0) {   // elementwise terms only: one item, no contraction
      const int j = (int)std::min<int64_t>(G / per, nwg - 1);
      share[j].push_back({(int32_t)ti, 0, 0, 0, 0, 0, {0, 0}});
      continue;
    }
    const int64_t g0 = G, g1 = G + t.nstage;
    const int j0 = (int)(g0 / per), j1 = (int)((g1 - 1) / per);
    // the pieces of the tile: one per share it meets, each cut further so
    // that it spans at most kMacSegLds segments
    std::vector<std::pair<int, MacItem>> pieces;
    for (int j = j0; j <= j1; ++j) {
      int32_t a0 = (int32_t)(std::max<int64_t>(g0, (int64_t)j * per) - g0);
      const int32_t a1 = (int32_t)(std::min<int64_t>(g1, (int64_t)(j + 1) * per) - g0);
      while (a0 < a1) {
        int g = 0;
        while (g + 1 < t.nseg && a0 >= mp.segs[t.seg0 + g + 1].st0) ++g;
        const int gl = std::min(g + kMacSegLds, t.nseg);   // first segment not in the piece
        const int32_t cut = gl < t.nseg ? std::min(a1, mp.segs[t.seg0 + gl].st0) : a1;
        int ge = g;   // last segment the piece reaches
        while (ge + 1 < t.nseg && cut - 1 >= mp.segs[t.seg0 + ge + 1].st0) ++ge;
        pieces.push_back({j, {(int32_t)ti, 0, a0, cut, g, ge - g + 1, {0, 0}}});
        a0 = cut;
      }
    }
    t.nsplit = (int32_t)pieces.size();
    if (t.nsplit > 1) {
      t.part0 = mp.nparts;
      mp.nparts += t.nsplit;
      mp.shared.push_back((int32_t)ti);
    }
    for (size_t k = 0; k < pieces.size(); ++k) {
      pieces[k].second.split = (int32_t)k;
      share[pieces[k].first].push_back(pieces[k].second);
    }
    G = g1;
  }
  // share j runs on workgroup b(j): consecutive shares on one XCD (workgroup
  // b runs on XCD b % kXcds), so that a block's tiles meet in one L2
  std::vector<int> share_of(nwg);
  if (nwg % kXcds == 0) {
    const int per_xcd = nwg / kXcds;
    for (int j = 0; j < nwg; ++j) share_of[(j % per_xcd) * kXcds + j / per_xcd] = j;
  } else {
    for (int j = 0; j < nwg; ++j) share_of[j] = j;
  }
  mp.wg_start.assign(1, 0);
  for (int w = 0; w < nwg; ++w) {
    for (const MacItem& it : share[share_of[w]]) mp.items.push_back(it);
    mp.wg_start.push_back((int32_t)mp.items.size());
  }
}

}  // namespace dmrg
