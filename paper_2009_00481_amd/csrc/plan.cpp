// Planner: rows -> BDD shapes, incidence J_i, dependency waves and the HBM layout.
//
// Waves. Alg. "Min-marginal averaging" visits variables one at a time in the processing order.
// Visiting i touches, in each row j of J_i, only level l_j(i): the forward step there reads the
// forward messages of level l-1 and lambda^j of the previous variable of row j, the min-marginals
// read the backward messages of level l+1, and the update couples the rows of J_i through their
// sum. So i may run as soon as the previous variable of each of its rows has run:
//   wave_f(i) = 1 + max_j wave_f(prev_j(i))   (0 if i opens all its rows),
// and the backward pass mirrors this with the next variable of each row. Variables of one wave
// share no row, and every value a variable reads was written in an earlier wave, so running the
// waves in order performs the sequential algorithm's arithmetic exactly (the argument of the
// proof of Prop. "correctness", applied to all rows at once).
//
// Layout. Layers (one per incidence = one BDD level) are stored forward-wave-major: by forward
// wave, then by the variable's processing rank, then ascending row. A variable's layers are
// therefore one contiguous segment, and each wave is one contiguous layer range. Node arrays
// follow the layer order. Arcs are packed as two 16-bit child codes per node.
#include <algorithm>
#include <mutex>
#include <exception>
#include <thread>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <tuple>
#include <unordered_map>

#include "internal.h"

namespace bddmp {

void greedy_colour_order(const Problem &p, std::vector<int32_t> &order) {
  const int32_t n = p.n;
  const int64_t m = int64_t(p.row_ptr.size()) - 1;
  std::vector<int64_t> vptr(size_t(n) + 1, 0);
  for (int32_t c : p.col) vptr[c + 1]++;
  for (int32_t i = 0; i < n; ++i) vptr[i + 1] += vptr[i];
  std::vector<int64_t> vrows(p.col.size());
  std::vector<int64_t> fill(vptr.begin(), vptr.end() - 1);
  for (int64_t j = 0; j < m; ++j)
    for (int64_t q = p.row_ptr[j]; q < p.row_ptr[j + 1]; ++q) vrows[fill[p.col[q]]++] = j;
  std::vector<int32_t> colour(size_t(n), -1);
  std::vector<int32_t> mark;
  int32_t ncol = 0;
  for (int32_t v = 0; v < n; ++v) {
    for (int64_t q = vptr[v]; q < vptr[v + 1]; ++q) {
      const int64_t j = vrows[q];
      for (int64_t t = p.row_ptr[j]; t < p.row_ptr[j + 1]; ++t) {
        const int32_t cu = colour[p.col[t]];
        if (cu >= 0) {
          if (cu >= int32_t(mark.size())) mark.resize(size_t(cu) + 1, -1);
          mark[cu] = v;
        }
      }
    }
    int32_t c = 0;
    while (c < int32_t(mark.size()) && mark[c] == v) ++c;
    colour[v] = c;
    ncol = std::max(ncol, c + 1);
  }
  order.resize(size_t(n));
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return colour[x] < colour[y]; });
}

bool gsel_code(int32_t lanes, uint32_t &code) {
  if (lanes == 0) {
    code = kGselFlat;
    return true;
  }
  if (lanes < 1 || lanes > 64 || (lanes & (lanes - 1))) return false;
  code = 0;
  while ((1 << code) < lanes) ++code;
  return true;
}

bool parse_groups(const char *s, uint32_t &gsel) {
  uint32_t out = 0;
  int k = 0;
  const char *p = s;
  while (k < kWidthClasses) {
    char *e = nullptr;
    const long v = std::strtol(p, &e, 10);
    uint32_t code = 0;
    if (e == p || v > 64 || !gsel_code(int32_t(v), code)) return false;
    out |= code << (4 * k);
    ++k;
    p = e;
    if (k < kWidthClasses) {
      if (*p != ',') return false;
      ++p;
    }
  }
  if (*p) return false;
  gsel = out;
  return true;
}

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// f(begin, end) over [0, n) in contiguous chunks on up to 16 host threads (one for small n); an
// exception thrown in any chunk is rethrown here once every chunk has ended
template <class F>
void parallel_for(int64_t n, F &&f) {
  constexpr int64_t kMinChunk = int64_t(1) << 16;
  const unsigned hw = std::thread::hardware_concurrency();
  const int64_t nt = std::min<int64_t>({int64_t(hw ? hw : 1), 16, (n + kMinChunk - 1) / kMinChunk});
  if (nt <= 1) {
    if (n > 0) f(int64_t(0), n);
    return;
  }
  const int64_t chunk = (n + nt - 1) / nt;
  std::vector<std::exception_ptr> err(static_cast<size_t>(nt));
  auto run = [&](int64_t k) {
    try {
      if (k * chunk < n) f(k * chunk, std::min(n, (k + 1) * chunk));
    } catch (...) {
      err[size_t(k)] = std::current_exception();
    }
  };
  std::vector<std::thread> th;
  int64_t k = 1;
  try {
    for (; k < nt; ++k) th.emplace_back(run, k);
  } catch (...) {
    for (; k < nt; ++k) run(k);  // no more threads: the remaining chunks here
  }
  run(0);
  for (auto &t : th) t.join();
  for (auto &e : err)
    if (e) std::rethrow_exception(e);
}

// Greedy tiling of a pass: consecutive variables share a tile while their layers fit kTile, their
// general levels hold at most cap nodes (wwork: per variable) and they belong to the same group of
// instances (grp); a variable with more rows than kTile gets a big tile of its own. Tiles are
// (start, end) pairs.
void tile_pass(const std::vector<int32_t> &vars, const std::vector<int32_t> &nj, const std::vector<int64_t> &wwork,
               const std::vector<int32_t> &grp, int64_t cap, int64_t pos0, std::vector<int32_t> &tiles,
               std::vector<int32_t> &big, WaveRange &wr) {
  wr.tile_begin = int32_t(tiles.size() / 2);
  wr.big_begin = int32_t(big.size() / 2);
  int64_t pos = pos0, start = pos0, work = 0;
  int32_t cnt = 0, g = -1;
  for (int32_t i : vars) {
    const int32_t c = nj[i];
    if (c > kTile) {
      if (cnt) { tiles.push_back(int32_t(start)); tiles.push_back(int32_t(pos)); }
      big.push_back(int32_t(pos));
      big.push_back(int32_t(pos + c));
      pos += c;
      start = pos;
      cnt = 0;
      work = 0;
      continue;
    }
    if (cnt + c > kTile || (cnt && work + wwork[i] > cap) || (cnt && grp[i] != g)) {
      tiles.push_back(int32_t(start));
      tiles.push_back(int32_t(pos));
      start = pos;
      cnt = 0;
      work = 0;
    }
    pos += c;
    cnt += c;
    work += wwork[i];
    g = grp[i];
  }
  if (cnt) { tiles.push_back(int32_t(start)); tiles.push_back(int32_t(pos)); }
  wr.tile_end = int32_t(tiles.size() / 2);
  wr.big_end = int32_t(big.size() / 2);
}

// Checks every index the wave, bound and output kernels read or write against the array it
// addresses, that narrow records decode to the same arcs as the general array, and that tiles hold
// whole variable segments and cover every layer once per pass. Returns an empty string when sound.
std::string validate_layout(const Plan &P, const std::vector<int32_t> &ownw, const std::vector<int32_t> &childw,
                            const std::vector<int32_t> &level, const std::vector<uint8_t> &exit_cut,
                            const std::vector<uint8_t> &root_cut) {
  const int64_t I = P.I, S = P.S;
  if (int64_t(P.meta.size()) != I || int64_t(P.child.size()) != I || int64_t(P.parent.size()) != I ||
      int64_t(P.garcs.size()) != S)
    return "array sizes";
  // one layer's checks (seen0 / seen1: its arcs met in the in-arc lists), nullptr when sound
  auto check_layer = [&](int64_t L, std::vector<int32_t> &seen0, std::vector<int32_t> &seen1) -> const char * {
    const int64_t os = P.own_slot[L];
    const int32_t w = ownw[L], wc = childw[L];
    if (w <= 0 || w > kMaxWidth || os < 0 || os + w > S) return "own slots";
    if (w <= 2 && os != 2 * L) return "narrow slot";
    const int64_t cs = P.cslot[L];
    if (cs < 0 || cs + wc > P.Sc || (wc <= 2 && cs != 2 * L)) return "child slots";
    const int32_t cl = P.child[L];
    const uint32_t meta = P.meta[L];
    if (exit_cut[L] ? (cl >= 0 || wc != 2 * w) : ((cl < 0) != (wc == 0))) return "child layer";
    if (cl >= 0 && (cl >= I || P.canon_of[cl] != P.canon_of[L] + 1 || ownw[cl] != wc || P.parent[cl] != L))
      return "child layer";
    const int32_t pl = P.parent[L];
    if ((pl < 0) != (level[L] == 0 || root_cut[L])) return "parent layer";
    if (pl >= 0 && (pl >= I || P.child[pl] != L || childw[pl] != w)) return "parent layer";
    for (int32_t u = 0; u < w; ++u) {
      const uint32_t a = P.garcs[size_t(os + u)];
      for (uint32_t ch : {a & 0xFFFFu, a >> 16}) {
        if (ch == kBot) continue;
        if (ch == kTop) {
          if (cl >= 0 || exit_cut[L]) return "TOP before the last level";
          continue;
        }
        if ((cl < 0 && !exit_cut[L]) || int32_t(ch) >= wc) return "child index outside the next level";
        if (exit_cut[L] && (ch >> 1) != uint32_t(u)) return "virtual child of a cut";
      }
    }
    const uint32_t w2 = (meta >> kMetaWidthShift) & 3u;
    const bool narrow = w <= 2 && wc <= 2;
    if (narrow != (w2 != 0) || (narrow && int32_t(w2) != w)) return "narrow flag";
    if (narrow) {
      for (int32_t u = 0; u < 2; ++u) {
        const uint32_t a = u < w ? P.garcs[size_t(os + u)] : (kBot | (kBot << 16));
        for (int beta = 0; beta < 2; ++beta) {
          const uint32_t c16 = beta ? a >> 16 : a & 0xFFFFu;
          const uint32_t c2 = (meta >> (4 * u + 2 * beta)) & 3u;
          const uint32_t want = c16 == kBot ? kC2Bot : (c16 == kTop ? kC2Top : c16);
          if (c2 != want) return "narrow arcs";
        }
      }
    } else {
      if (P.grec.empty()) return "general record missing";
      const int32_t *g = &P.grec[4 * size_t(L)];
      if (g[0] != os || g[1] != cs || g[2] != (w | (wc << 16))) return "general record";
      if (P.gnb[2 * size_t(L)] != (cl >= 0 ? P.own_slot[cl] : -1) || P.gnb[2 * size_t(L) + 1] != (pl >= 0 ? P.cslot[pl] : -1))
        return "neighbour slots";
      // the child level's in-arc lists hold exactly this level's arcs into it
      if (wc > 0 && !exit_cut[L]) {
        const int64_t rb = g[3];
        if (rb < 0 || rb + wc >= int64_t(P.rbeg.size())) return "in-arc base";
        seen0.assign(size_t(w), 0);
        seen1.assign(size_t(w), 0);
        int64_t cnt = 0;
        if (P.rin.size() != P.rbeg.size()) return "packed in-arcs";
        for (int32_t v = 0; v < wc; ++v) {
          const int64_t b0 = P.rbeg[size_t(rb + v)], b1 = P.rbeg[size_t(rb + v + 1)];
          if (b0 < 0 || b1 < b0 || b1 > int64_t(P.rarc.size())) return "in-arc range";
          const uint32_t pk = P.rin[size_t(rb + v)];
          if (b1 - b0 > 2 || b1 == b0) {
            if (pk != kManyInArcs) return "packed in-arcs";
          } else if ((pk & 0xFFFFu) != P.rarc[size_t(b0)] ||
                     (pk >> 16) != (b1 - b0 > 1 ? uint32_t(P.rarc[size_t(b0 + 1)]) : kNoArc16)) {
            return "packed in-arcs";
          }
          for (int64_t q = b0; q < b1; ++q) {
            const uint32_t a = P.rarc[size_t(q)];
            const int32_t u = int32_t(a & (kInArcHi - 1u));
            if (u >= w) return "in-arc source";
            const uint32_t code = P.garcs[size_t(os + u)];
            const uint32_t ch = (a & kInArcHi) ? code >> 16 : code & 0xFFFFu;
            if (int32_t(ch) != v) return "in-arc target";
            if (((a & kInArcHi) ? seen1 : seen0)[u]++) return "in-arc repeated";
            ++cnt;
          }
        }
        int64_t live = 0;
        for (int32_t u = 0; u < w; ++u) {
          const uint32_t code = P.garcs[size_t(os + u)];
          live += ((code & 0xFFFFu) < kTop) + ((code >> 16) < kTop);
        }
        if (cnt != live) return "in-arc count";
      } else if (g[3] != -1) {
        return "in-arc base";
      }
    }
    if (((meta & kMetaRootBit) != 0) != (level[L] == 0)) return "root flag";
    const uint32_t pos = (meta >> kMetaPosShift) & kMetaField, len = (meta >> kMetaLenShift) & kMetaField;
    const int32_t nj = P.var_nj[P.layer_var[L]];
    if (len == 0 || pos >= len || int32_t(len) != std::min<int32_t>(nj, int32_t(kMetaField))) return "segment";
    if (P.layer_of[P.canon_of[L]] != L) return "canon_of / layer_of";
    return nullptr;
  };
  // the layers on several threads; the first failing layer's message
  {
    std::mutex mu;
    int64_t bad_at = I;
    const char *bad = nullptr;
    parallel_for(I, [&](int64_t L0, int64_t L1) {
      std::vector<int32_t> seen0, seen1;
      for (int64_t L = L0; L < L1; ++L)
        if (const char *e = check_layer(L, seen0, seen1)) {
          std::lock_guard<std::mutex> lk(mu);
          if (L < bad_at) {
            bad_at = L;
            bad = e;
          }
          return;
        }
    });
    if (bad) return bad;
  }
  // every layer is visited exactly once per pass; a normal tile holds whole segments of variables
  // with at most kTile rows, a big tile exactly one variable
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<uint8_t> seen(size_t(I), 0);
    const auto &waves = pass ? P.bwd_waves : P.fwd_waves;
    for (const WaveRange &wr : waves)
      for (int big = 0; big < 2; ++big) {
        const auto &tiles = pass ? (big ? P.bwd_big : P.bwd_tiles) : (big ? P.fwd_big : P.fwd_tiles);
        for (int32_t t = big ? wr.big_begin : wr.tile_begin; t < (big ? wr.big_end : wr.tile_end); ++t) {
          const uint32_t w0 = uint32_t(tiles[2 * size_t(t)]);
          const int64_t p0 = big ? int64_t(w0) : int64_t(w0 & kTilePosMask);
          const int64_t p1 = uint32_t(tiles[2 * size_t(t) + 1]) & ~kTileRootBit;
          if (big && (p0 >> kTileClsShift)) return "big tile start";
          const int64_t cap = big ? kBigMax : kTile;
          if (p1 <= p0 || p1 - p0 > cap || p0 < 0 || p1 > I) return "tile bounds";
          for (int64_t p = p0; p < p1; ++p) {
            const int64_t L = (pass && wr.list) ? P.bwd_list[size_t(p)] : p;
            if (L < 0 || L >= I) return "tile layer";
            if (seen[L]++) return "layer visited twice in a pass";
            const int32_t nj = P.var_nj[P.layer_var[L]];
            if (big) {
              if (nj != p1 - p0 || P.layer_var[L] != P.layer_var[(pass && wr.list) ? P.bwd_list[size_t(p0)] : p0])
                return "big tile is not one variable";
              continue;
            }
            const uint32_t meta = P.meta[L];
            if (wr.narrow_only && ((meta >> kMetaWidthShift) & 3u) == 0u) return "narrow-only wave holds a wide level";
            if (((meta >> kMetaWidthShift) & 3u) == 0u) {
              const int32_t mw = std::max(ownw[L], childw[L]);
              const uint32_t need = mw <= 8 ? 0u : (mw <= 32 ? 1u : (mw <= 128 ? 2u : 3u));
              if ((w0 >> kTileClsShift) < need) return "tile width class";
            }
            const int64_t head = p - int64_t((meta >> kMetaPosShift) & kMetaField);
            if (nj > kTile || head < p0 || head + nj > p1) return "segment leaves its tile";
          }
        }
      }
    for (int64_t L = 0; L < I; ++L)
      if (!seen[L]) return "layer missing from a pass";
  }
  // dataflow launch: every dependency tile has a smaller index than the tile waiting for it (so it
  // was taken by a running workgroup before, and the wait ends), and covers the writer of each
  // message the tile reads
  if (P.pers_ok) {
    for (int pass = 0; pass < 2; ++pass) {
      const auto &tiles = pass ? P.bwd_tiles : P.fwd_tiles;
      const auto &waves = pass ? P.bwd_waves : P.fwd_waves;
      const auto &ptr = pass ? P.bdep_ptr : P.fdep_ptr;
      const auto &lst = pass ? P.bdep_list : P.fdep_list;
      const auto &info = pass ? P.btinfo : P.ftinfo;
      const size_t nt = tiles.size() / 2;
      if (ptr.size() != nt + 1 || info.size() != nt || ptr[0] != 0 || size_t(ptr[nt]) != lst.size()) return "dependency arrays";
      std::vector<int32_t> tile_of(size_t(I), -1);
      for (const WaveRange &wr : waves)
        for (int32_t t = wr.tile_begin; t < wr.tile_end; ++t) {
          if (((info[size_t(t)] >> 1) & 1u) != uint32_t(pass && wr.list)) return "tile info list bit";
          const int64_t p0 = uint32_t(tiles[2 * size_t(t)]) & kTilePosMask;
          const int64_t p1 = uint32_t(tiles[2 * size_t(t) + 1]) & ~kTileRootBit;
          for (int64_t q = p0; q < p1; ++q) tile_of[size_t((pass && wr.list) ? P.bwd_list[size_t(q)] : q)] = t;
        }
      for (const WaveRange &wr : waves)
        for (int32_t t = wr.tile_begin; t < wr.tile_end; ++t) {
          const int32_t d0 = ptr[size_t(t)], d1 = ptr[size_t(t) + 1];
          if (d1 < d0) return "dependency offsets";
          for (int32_t q = d0; q < d1; ++q)
            if (lst[size_t(q)] < 0 || lst[size_t(q)] >= t || (q > d0 && lst[size_t(q)] <= lst[size_t(q) - 1]))
              return "dependency tile not smaller than its waiter";
          const int64_t p0 = uint32_t(tiles[2 * size_t(t)]) & kTilePosMask;
          const int64_t p1 = uint32_t(tiles[2 * size_t(t) + 1]) & ~kTileRootBit;
          bool narrow = true;
          for (int64_t q = p0; q < p1; ++q) {
            const int64_t L = (pass && wr.list) ? P.bwd_list[size_t(q)] : q;
            narrow = narrow && ((P.meta[size_t(L)] >> kMetaWidthShift) & 3u) != 0u;
            const int32_t nb = pass ? P.child[size_t(L)] : P.parent[size_t(L)];
            if (nb >= 0 && !std::binary_search(lst.begin() + d0, lst.begin() + d1, tile_of[size_t(nb)]))
              return "missing dependency";
          }
          if ((info[size_t(t)] & 1u) != (narrow ? 1u : 0u)) return "tile info narrow bit";
          const auto &rec = pass ? P.btrec : P.ftrec;
          const int32_t *r = rec.data() + 8 * size_t(t);
          const int32_t nd = d1 - d0;
          if (rec.size() != 8 * nt || r[0] != tiles[2 * size_t(t)] || r[1] != tiles[2 * size_t(t) + 1] ||
              uint32_t(r[2]) != (info[size_t(t)] | (uint32_t(nd) << 8)) || r[3] != d0 || nd >= 512)
            return "tile record";
          for (int32_t q = 0; q < 4; ++q)
            if (r[4 + q] != (q < nd ? lst[size_t(d0 + q)] : -1)) return "tile record dependencies";
        }
      // queues: every tile in exactly one, ascending; a tile's layers and its dependencies all in the
      // queue's group
      const auto &qptr = pass ? P.bqptr : P.fqptr;
      const auto &qtile = pass ? P.bqtile : P.fqtile;
      if (P.n_groups < 1 || P.n_groups > kPassQueues || qptr.size() != size_t(P.n_groups) + 1 || qptr[0] != 0 ||
          size_t(qptr.back()) != nt || qtile.size() != nt)
        return "queue arrays";
      std::vector<int32_t> tq(nt, -1);
      for (int32_t g = 0; g < P.n_groups; ++g)
        for (int32_t k = qptr[size_t(g)]; k < qptr[size_t(g) + 1]; ++k) {
          const int32_t t = qtile[size_t(k)];
          if (t < 0 || size_t(t) >= nt || tq[size_t(t)] >= 0 || (k > qptr[size_t(g)] && t <= qtile[size_t(k) - 1]))
            return "queue tiles";
          tq[size_t(t)] = g;
        }
      for (const WaveRange &wr : waves)
        for (int32_t t = wr.tile_begin; t < wr.tile_end; ++t) {
          const int64_t p0 = uint32_t(tiles[2 * size_t(t)]) & kTilePosMask;
          const int64_t p1 = uint32_t(tiles[2 * size_t(t) + 1]) & ~kTileRootBit;
          for (int64_t q = p0; q < p1; ++q)
            if (P.var_group[size_t(P.layer_var[size_t((pass && wr.list) ? P.bwd_list[size_t(q)] : q)])] != tq[size_t(t)])
              return "tile spans groups";
          for (int32_t q = ptr[size_t(t)]; q < ptr[size_t(t) + 1]; ++q)
            if (tq[size_t(lst[size_t(q)])] != tq[size_t(t)]) return "dependency across groups";
        }
      // two-branch split: an A tile depends on A tiles of earlier waves only; a B tile on B tiles of
      // earlier waves or A tiles of waves up to its wave's b_wait
      const auto &split = pass ? P.bsplit : P.fsplit;
      if (split.size() != waves.size()) return "wave split arrays";
      std::vector<int32_t> wave_of(nt, -1);
      for (size_t w = 0; w < waves.size(); ++w) {
        const WaveRange &wr = waves[w];
        const Plan::WaveSplit &s = split[w];
        if (s.mid < wr.tile_begin || s.mid > wr.tile_end || 2 * (s.mid - wr.tile_begin) > wr.tile_end - wr.tile_begin + 1 ||
            s.b_wait < -1 || s.b_wait >= int32_t(w))
          return "wave split";
        for (int32_t t = wr.tile_begin; t < wr.tile_end; ++t) {
          wave_of[size_t(t)] = int32_t(w);
          for (int32_t q = ptr[size_t(t)]; q < ptr[size_t(t) + 1]; ++q) {
            const int32_t u = lst[size_t(q)], wu = wave_of[size_t(u)];
            if (wu < 0 || wu >= int32_t(w)) return "dependency not in an earlier wave";
            const bool u_in_a = u < split[size_t(wu)].mid;
            if (t < s.mid ? !u_in_a : (u_in_a && wu > s.b_wait)) return "wave split dependency";
          }
        }
      }
    }
  }
  // node maps of the flat path: each tile's general layers in position order, their own nodes
  // then their child nodes, each mapped to the layer's rank; only tiles within the flat stage; each
  // tile's maps at a multiple of 16 bytes, padded to one
  for (int pass = 0; pass < 2; ++pass) {
    const auto &tiles = pass ? P.bwd_tiles : P.fwd_tiles;
    const auto &waves = pass ? P.bwd_waves : P.fwd_waves;
    const auto &gt = pass ? P.bgt : P.fgt;
    const auto &gm = pass ? P.bgm : P.fgm;
    if (gt.size() != tiles.size() || gm.size() % 16) return "node map records";
    size_t used = 0;
    for (const WaveRange &wr : waves)
      for (int32_t t = wr.tile_begin; t < wr.tile_end; ++t) {
        const int64_t p0 = uint32_t(tiles[2 * size_t(t)]) & kTilePosMask;
        const int64_t p1 = uint32_t(tiles[2 * size_t(t) + 1]) & ~kTileRootBit;
        std::vector<int32_t> own, chl;
        int32_t k = 0;
        for (int64_t q = p0; q < p1; ++q) {
          const int64_t L = (pass && wr.list) ? P.bwd_list[size_t(q)] : q;
          if (((P.meta[size_t(L)] >> kMetaWidthShift) & 3u) != 0u) continue;
          own.insert(own.end(), size_t(ownw[size_t(L)]), k);
          chl.insert(chl.end(), size_t(childw[size_t(L)]), k);
          ++k;
        }
        const bool flat = k > 0 && own.size() <= size_t(kFlatCap) && chl.size() <= size_t(kFlatCap);
        const int32_t off = gt[2 * size_t(t)], sizes = gt[2 * size_t(t) + 1];
        if (!flat) {
          if (off != -1) return "node map of a tile outside the flat stage";
          continue;
        }
        const size_t len = (own.size() + chl.size() + 15) / 16 * 16;
        if (off < 0 || off % 16 || size_t(off) != used || sizes != int32_t(own.size() | (chl.size() << 16)) ||
            size_t(off) + len > gm.size())
          return "node map record";
        for (size_t q = 0; q < own.size(); ++q)
          if (gm[size_t(off) + q] != own[q]) return "own node map";
        for (size_t q = 0; q < chl.size(); ++q)
          if (gm[size_t(off) + own.size() + q] != chl[q]) return "child node map";
        used += len;
      }
    if (used != gm.size()) return "node map size";
  }
  for (int32_t j = 0; j < P.m; ++j)
    if (P.root_slot[j] >= S || P.bdd_canon_off[j + 1] < P.bdd_canon_off[j]) return "roots";
  for (int32_t i = 0; i < P.n; ++i)
    if (P.var_nj[i] && (P.var_first[i] < 0 || P.var_first[i] + P.var_nj[i] > I)) return "var_first";
  // cut tables: each cut names an exit layer and the root layer after it, with their slots and
  // arc ranges inside the arrays
  const int64_t nc = P.n_cuts;
  if (int64_t(P.cuts.size()) != 4 * nc || int64_t(P.cut_slots.size()) != 4 * nc || int64_t(P.cut_live.size()) != nc ||
      int64_t(P.cut_rb.size()) != nc || int64_t(P.cut_arc.size()) != P.n_arcs_cut || P.n_cut_narrow > nc)
    return "cut arrays";
  std::vector<uint8_t> arc_seen(size_t(P.n_arcs_cut), 0), live_seen(size_t(P.n_copy), 0);
  for (int64_t c = 0; c < nc; ++c) {
    const int32_t *k = &P.cuts[4 * size_t(c)], *sl = &P.cut_slots[4 * size_t(c)];
    const int32_t Lx = k[0], Lr = k[1], wx = k[3] & 0xFFFF, wr = int32_t(uint32_t(k[3]) >> 16);
    if (Lx < 0 || Lx >= I || Lr < 0 || Lr >= I || !exit_cut[Lx] || !root_cut[Lr] || P.canon_of[Lr] != P.canon_of[Lx] + 1)
      return "cut layers";
    if (wx != ownw[Lx] || wr != ownw[Lr] || k[2] < 0 || k[2] + 2 * wx > P.n_arcs_cut) return "cut record";
    if ((c < P.n_cut_narrow) != (wx <= 2 && wr <= 2)) return "cut class";
    if (sl[0] != P.own_slot[Lx] || sl[1] != P.cslot[Lx] || sl[2] != P.own_slot[Lr] || sl[3] != P.cslot[Lr]) return "cut slots";
    int64_t live = P.cut_live[size_t(c)];
    std::vector<int32_t> into(size_t(wr), 0);
    for (int32_t q = 0; q < 2 * wx; ++q) {
      if (arc_seen[size_t(k[2] + q)]++) return "cut arcs overlap";
      const uint32_t a = P.cut_arc[size_t(k[2] + q)];
      if (a == kBot) continue;
      if (int32_t(a) >= wr) return "cut arc";
      into[a]++;
      if (live < 0 || live >= P.n_copy || live_seen[size_t(live)]++) return "copy pairs";
      ++live;
    }
    const int32_t rb = P.cut_rb[size_t(c)];
    if (c < P.n_cut_narrow) {
      if (rb != -1) return "cut in-arcs";
      continue;
    }
    // the root level's in-arc lists hold exactly the cut's live arcs into each node
    if (rb < 0 || int64_t(rb) + wr >= int64_t(P.rbeg.size()) || P.rin.size() != P.rbeg.size()) return "cut in-arcs";
    for (int32_t v = 0; v < wr; ++v) {
      const int64_t b0 = P.rbeg[size_t(rb + v)], b1 = P.rbeg[size_t(rb + v + 1)];
      if (b0 < 0 || b1 < b0 || b1 > int64_t(P.rarc.size()) || b1 - b0 != into[v]) return "cut in-arcs";
      const uint32_t pk = P.rin[size_t(rb + v)];
      if (b1 - b0 > 2 || b1 == b0 ? pk != kManyInArcs
                                  : ((pk & 0xFFFFu) != P.rarc[size_t(b0)] ||
                                     (pk >> 16) != (b1 - b0 > 1 ? uint32_t(P.rarc[size_t(b0 + 1)]) : kNoArc16)))
        return "cut packed in-arcs";
      for (int64_t q = b0; q < b1; ++q) {
        const uint32_t a = P.rarc[size_t(q)];
        const int32_t u = int32_t(a & (kInArcHi - 1u));
        if (u >= wx || P.cut_arc[size_t(k[2] + 2 * u + ((a & kInArcHi) ? 1 : 0))] != uint32_t(v)) return "cut in-arc target";
      }
    }
  }
  for (uint8_t f : arc_seen)
    if (!f) return "cut arcs not covered";
  for (uint8_t f : live_seen)
    if (!f) return "copy pairs not covered";
  // exit layers name their cut records
  if (nc) {
    if (int64_t(P.exit_rec.size()) != I) return "exit records";
    int64_t nexit = 0;
    for (int64_t L = 0; L < I; ++L) {
      const int32_t r = P.exit_rec[size_t(L)];
      if (r < -1 || r >= nc || (r >= 0) != bool(exit_cut[L]) || (r >= 0 && P.cuts[4 * size_t(r)] != L)) return "exit records";
      nexit += r >= 0;
    }
    if (nexit != nc) return "exit records";
  }
  // instance cut lists: every record once, inside its row's instance, canonical order
  if (P.inst_cut.size() != P.inst_row32.size() || int64_t(P.inst_cut_idx.size()) != nc) return "instance cuts";
  {
    std::vector<uint8_t> seen(static_cast<size_t>(nc), 0);
    for (size_t k = 0; k + 1 < P.inst_cut.size(); ++k) {
      if (P.inst_cut[k + 1] < P.inst_cut[k]) return "instance cuts";
      for (int32_t q = P.inst_cut[k]; q < P.inst_cut[k + 1]; ++q) {
        const int32_t c = P.inst_cut_idx[size_t(q)];
        if (c < 0 || c >= nc || seen[size_t(c)]++) return "instance cut index";
        const int32_t row = P.cut_row[size_t(c)];
        if (row < P.inst_row32[k] || row >= P.inst_row32[k + 1]) return "instance cut row";
        if (q > P.inst_cut[k] && P.canon_of[P.cuts[4 * size_t(c)]] <= P.canon_of[P.cuts[4 * size_t(P.inst_cut_idx[size_t(q - 1)])]])
          return "instance cut order";
      }
    }
  }
  // instance row ranges: from 0 to m, non-decreasing (the bound kernel reads rows inside them)
  const size_t ni = P.inst_row32.size();
  if (ni < 2 || P.inst_row32[0] != 0 || P.inst_row32[ni - 1] != P.m || P.inst_lb_const.size() != ni - 1)
    return "instances";
  for (size_t k = 0; k + 1 < ni; ++k)
    if (P.inst_row32[k + 1] < P.inst_row32[k]) return "instances";
  return "";
}

}  // namespace

int32_t make_plan(const Problem &p, const bddmp_options &opt, Plan &P) {
  P = Plan{};
  const int32_t n = p.n;
  const int64_t m64 = int64_t(p.row_ptr.size()) - 1;
  if (m64 > INT32_MAX - 1) return set_error(BDDMP_INVALID_ARG, "too many rows");
  const int32_t m = int32_t(m64);
  P.n = n;
  P.m = m;
  P.hist_cap = opt.hist_cap > 0 ? opt.hist_cap : 4096;
  if (opt.tile_work < 0) return set_error(BDDMP_INVALID_ARG, "negative tile_work");
  if (opt.tile_work > 0) P.tile_work = opt.tile_work;
  if (opt.n_intervals < 0) return set_error(BDDMP_INVALID_ARG, "negative n_intervals");
  if (!(opt.split_gamma == 0.0f || (opt.split_gamma > 0.0f && opt.split_gamma <= 1.0f)))
    return set_error(BDDMP_INVALID_ARG, "split_gamma must lie in (0, 1] (0: default)");
  if (opt.wave_align != 0 && opt.wave_align != 1) return set_error(BDDMP_INVALID_ARG, "wave_align must be 0 or 1");
  P.split_k = opt.n_intervals > 1 ? opt.n_intervals : 0;
  P.split_gamma = opt.split_gamma > 0.0f ? opt.split_gamma : 0.5f;
  if (opt.tiling && !parse_groups(opt.tiling, P.gsel))
    return set_error(BDDMP_INVALID_ARG, "tiling must be four values, each 0 or a power of two up to 64, e.g. \"0,16,64,64\"");
  P.cost = p.cost;

  // processing order
  if (opt.order_mode == 1) {
    greedy_colour_order(p, P.order);
  } else if (opt.order_mode == 0) {
    if (p.order.empty()) {
      P.order.resize(size_t(n));
      std::iota(P.order.begin(), P.order.end(), 0);
    } else {
      P.order = p.order;
    }
  } else {
    return set_error(BDDMP_INVALID_ARG, "order_mode must be 0 or 1");
  }
  P.rank.assign(size_t(n), -1);
  for (int32_t r = 0; r < n; ++r) P.rank[P.order[r]] = r;

  // rows -> shapes (rows with the same coefficient sequence, sense and rhs share a shape)
  std::unordered_map<std::string, int32_t> memo;
  std::vector<int32_t> stamp(size_t(n), -1);
  std::vector<std::pair<int32_t, int32_t>> items;  // (rank, nnz index)
  std::vector<int64_t> coefs;
  std::string key, err;
  P.row_shape.assign(size_t(m), -1);
  P.canon_off.assign(size_t(m) + 1, 0);
  P.canon_node.assign(size_t(m) + 1, 0);
  std::vector<int32_t> inc_row;
  for (int32_t j = 0; j < m; ++j) {
    const int64_t a0 = p.row_ptr[j], a1 = p.row_ptr[j + 1];
    items.clear();
    for (int64_t q = a0; q < a1; ++q) {
      const int32_t v = p.col[q];
      if (stamp[v] == j) return set_error(BDDMP_INVALID_ARG, "row " + std::to_string(j) + ": repeated column " + std::to_string(v));
      stamp[v] = j;
      if (p.coef[q] != 0) items.emplace_back(P.rank[v], int32_t(q));
    }
    std::sort(items.begin(), items.end());
    const int32_t k = int32_t(items.size());
    coefs.resize(size_t(k));
    for (int32_t t = 0; t < k; ++t) coefs[t] = p.coef[items[t].second];
    key.assign(1 + 8 + 8 * size_t(k), '\0');
    key[0] = char(p.sense[j]);
    std::memcpy(&key[1], &p.rhs[j], 8);
    if (k) std::memcpy(&key[9], coefs.data(), 8 * size_t(k));
    auto it = memo.find(key);
    int32_t sid;
    if (it == memo.end()) {
      Shape sh;
      const int32_t rc = build_shape(coefs.data(), k, p.sense[j], p.rhs[j], opt.node_budget, sh, err);
      if (rc != BDDMP_OK) return set_error(rc, "row " + std::to_string(j) + ": " + err);
      sid = int32_t(P.shapes.size());
      P.shapes.push_back(std::move(sh));
      memo.emplace(key, sid);
    } else {
      sid = it->second;
    }
    const Shape &sh = P.shapes[sid];
    P.row_shape[j] = k ? sid : -1;
    P.canon_off[j + 1] = P.canon_off[j] + k;
    P.canon_node[j + 1] = P.canon_node[j] + sh.first[k];
    for (int32_t t = 0; t < k; ++t) {
      P.inc_var.push_back(p.col[items[t].second]);
      inc_row.push_back(j);
    }
    P.max_width = std::max(P.max_width, sh.max_width);
  }
  P.I = P.canon_off[m];
  P.N = P.canon_node[m];
  if (opt.node_budget > 0 && P.N > opt.node_budget)
    return set_error(BDDMP_BDD_TOO_LARGE, "total nodes " + std::to_string(P.N) + " exceed the node budget");
  if (P.N >= INT32_MAX || P.I >= int64_t(kTilePosMask))
    return set_error(BDDMP_BDD_TOO_LARGE, "more than 2^31 nodes or 2^29 incidences");
  const int64_t I = P.I;
  for (int32_t j = 0; j < m; ++j) {
    if (P.row_shape[j] < 0) continue;
    const Shape &sh = P.shapes[P.row_shape[j]];
    for (size_t u = 0; u < sh.lo.size(); ++u) {
      P.live += (sh.lo[u] != -1) + (sh.hi[u] != -1);
      P.bot += (sh.lo[u] == -1) + (sh.hi[u] == -1);
    }
  }

  // J_i in ascending row order
  P.var_nj.assign(size_t(n), 0);
  for (int64_t c = 0; c < I; ++c) P.var_nj[P.inc_var[c]]++;
  std::vector<int64_t> iptr(size_t(n) + 1, 0);
  for (int32_t i = 0; i < n; ++i) iptr[i + 1] = iptr[i] + P.var_nj[i];
  std::vector<int32_t> ilist(static_cast<size_t>(I));
  {
    std::vector<int64_t> fill(iptr.begin(), iptr.end() - 1);
    for (int64_t c = 0; c < I; ++c) ilist[fill[P.inc_var[c]]++] = int32_t(c);
  }
  for (int32_t i = 0; i < n; ++i) P.max_j = std::max(P.max_j, P.var_nj[i]);
  if (P.max_j > kBigMax)
    return set_error(BDDMP_INVALID_ARG, "a variable appears in more than " + std::to_string(kBigMax) + " rows");

  // statically forced variables: a level with no live 1-arc forces 0, none with a live 0-arc forces 1
  for (int32_t i = 0; i < n; ++i) {
    bool f0 = false, f1 = false;
    for (int64_t q = iptr[i]; q < iptr[i + 1]; ++q) {
      const int64_t c = ilist[q];
      const int32_t j = inc_row[c];
      const Shape &sh = P.shapes[P.row_shape[j]];
      const int32_t l = int32_t(c - P.canon_off[j]);
      bool live0 = false, live1 = false;
      for (int32_t u = sh.first[l]; u < sh.first[l + 1]; ++u) {
        live0 |= sh.lo[u] != -1;
        live1 |= sh.hi[u] != -1;
      }
      f0 |= !live1;
      f1 |= !live0;
    }
    if (f0 && f1) return set_error(BDDMP_CONFLICT, "rows force variable " + std::to_string(i) + " to both 0 and 1");
  }

  // Sec. 6 split: per instance, its variables in processing order form split_k intervals of about
  // equal node count (a variable counts the nodes of its levels over all its rows; the variable
  // with c nodes before it among N lies in interval floor(split_k c / N)), and each row is cut
  // between consecutive levels whose variables lie in different intervals
  std::vector<uint8_t> cut_after(static_cast<size_t>(I), 0);
  if (P.split_k) {
    std::vector<int64_t> iv = p.inst_var.empty() ? std::vector<int64_t>{0, n} : p.inst_var;
    std::vector<int32_t> inst_of(size_t(n), 0);
    for (size_t x = 0; x + 1 < iv.size(); ++x)
      for (int64_t i = iv[x]; i < iv[x + 1]; ++i) inst_of[size_t(i)] = int32_t(x);
    std::vector<int64_t> vn(size_t(n), 0), tot(iv.size(), 0), cum(iv.size(), 0);
    for (int64_t c = 0; c < I; ++c) {
      const int32_t j = inc_row[c];
      const Shape &sh = P.shapes[P.row_shape[j]];
      const int32_t l = int32_t(c - P.canon_off[j]);
      vn[P.inc_var[c]] += sh.first[l + 1] - sh.first[l];
    }
    for (int32_t i = 0; i < n; ++i) tot[inst_of[i]] += vn[i];
    P.var_interval.assign(size_t(n), 0);
    for (int32_t r = 0; r < n; ++r) {
      const int32_t i = P.order[r], x = inst_of[i];
      P.var_interval[i] = tot[x] ? int32_t(int64_t(P.split_k) * cum[x] / tot[x]) : 0;
      cum[x] += vn[i];
    }
    for (int32_t j = 0; j < m; ++j)
      for (int64_t c = P.canon_off[j]; c + 1 < P.canon_off[j + 1]; ++c)
        if (P.var_interval[P.inc_var[c]] != P.var_interval[P.inc_var[c + 1]]) {
          cut_after[c] = 1;
          P.n_cuts++;
        }
  }

  // dependency waves (a cut ends the chain: the levels after it start a sub-BDD of their own)
  P.wave_f.assign(size_t(n), 0);
  P.wave_b.assign(size_t(n), 0);
  for (int32_t r = 0; r < n; ++r) {
    const int32_t i = P.order[r];
    if (!P.var_nj[i]) continue;
    int32_t t = 0;
    for (int64_t q = iptr[i]; q < iptr[i + 1]; ++q) {
      const int64_t c = ilist[q];
      if (c > P.canon_off[inc_row[c]] && !cut_after[c - 1]) t = std::max(t, P.wave_f[P.inc_var[c - 1]]);
    }
    P.wave_f[i] = t + 1;
    P.Df = std::max(P.Df, t + 1);
  }
  for (int32_t r = n - 1; r >= 0; --r) {
    const int32_t i = P.order[r];
    if (!P.var_nj[i]) continue;
    int32_t t = 0;
    for (int64_t q = iptr[i]; q < iptr[i + 1]; ++q) {
      const int64_t c = ilist[q];
      if (c + 1 < P.canon_off[inc_row[c] + 1] && !cut_after[c]) t = std::max(t, P.wave_b[P.inc_var[c + 1]]);
    }
    P.wave_b[i] = t + 1;
    P.Db = std::max(P.Db, t + 1);
  }
  // latest waves: a variable whose longest chain of row successors (its earliest backward wave)
  // has length h can run as late as forward wave D + 1 - h, D the longest chain (Df = Db); a
  // predecessor's chain is longer, so its wave is earlier. The same holds for the backward pass.
  if (P.Df != P.Db) return set_error(BDDMP_INVALID_ARG, "internal: forward and backward chain lengths differ");
  if (opt.wave_align == 1) {
    const int32_t D = P.Df;
    for (int32_t i = 0; i < n; ++i)
      if (P.var_nj[i]) {
        const int32_t f = P.wave_f[i];
        P.wave_f[i] = D + 1 - P.wave_b[i];
        P.wave_b[i] = D + 1 - f;
      }
  }

  // Groups of instances for the dataflow launch: instances never share a row, so a tile whose
  // layers all belong to one group depends only on tiles of that group; each group gets a ticket
  // queue of its own. Up to kPassQueues groups of about equal node counts (largest instance first
  // into the lightest group); a single instance is one group.
  P.var_group.assign(size_t(n), 0);
  P.n_groups = 1;
  if (p.inst_var.size() > 2) {
    const size_t ni = p.inst_var.size() - 1;
    std::vector<int64_t> inst_nodes(ni, 0);
    for (size_t k = 0; k < ni; ++k)
      for (int64_t j = p.inst_row[k]; j < p.inst_row[k + 1]; ++j)
        if (P.row_shape[size_t(j)] >= 0) inst_nodes[k] += int64_t(P.shapes[size_t(P.row_shape[size_t(j)])].lo.size());
    std::vector<int32_t> by_size(ni);
    std::iota(by_size.begin(), by_size.end(), 0);
    std::stable_sort(by_size.begin(), by_size.end(), [&](int32_t a, int32_t b) { return inst_nodes[size_t(a)] > inst_nodes[size_t(b)]; });
    P.n_groups = int32_t(std::min<size_t>(ni, size_t(kPassQueues)));
    std::vector<int64_t> load(size_t(P.n_groups), 0);
    for (int32_t k : by_size) {
      const int32_t g = int32_t(std::min_element(load.begin(), load.end()) - load.begin());
      load[size_t(g)] += inst_nodes[size_t(k)];
      for (int64_t i = p.inst_var[size_t(k)]; i < p.inst_var[size_t(k) + 1]; ++i) P.var_group[size_t(i)] = g;
    }
  }

  // Storage order. Each forward wave sorts its variables by group of instances, then by backward wave, then by the storage
  // position of their earliest parent layer (the previous level of one of their rows), ties and
  // parentless variables by processing order. A workgroup's layers then push to and read from
  // next-level slots that sit together, instead of cache lines shared with other workgroups (and
  // other XCDs), and a backward wave reads runs of neighbouring layers.
  std::vector<std::vector<int32_t>> fw(size_t(P.Df) + 1), bw(size_t(P.Db) + 1);
  for (int32_t r = 0; r < n; ++r) {
    const int32_t i = P.order[r];
    if (P.var_nj[i]) {
      fw[P.wave_f[i]].push_back(i);
      bw[P.wave_b[i]].push_back(i);
    }
  }
  P.canon_of.assign(size_t(I), 0);
  P.layer_of.assign(size_t(I), -1);
  P.layer_var.assign(size_t(I), 0);
  P.var_first.assign(size_t(n), -1);
  std::vector<uint32_t> segpos(size_t(I), 0);
  int64_t L = 0;
  std::vector<std::tuple<int32_t, int64_t, int32_t>> keyed;
  for (int32_t t = 1; t <= P.Df; ++t) {
    keyed.clear();
    for (int32_t i : fw[t]) {
      int64_t key = INT64_MAX;
      for (int64_t q = iptr[i]; q < iptr[i + 1]; ++q) {
        const int32_t c = ilist[q];
        if (c > P.canon_off[inc_row[c]] && !cut_after[c - 1]) key = std::min<int64_t>(key, P.layer_of[c - 1]);
      }
      // first by backward wave, so that each backward wave's members sit in runs inside each forward
      // wave (the backward pass gathers them through the index list with fewer partial cache lines)
      keyed.emplace_back(P.var_group[size_t(i)], (int64_t(P.wave_b[i]) << 40) + (key == INT64_MAX ? (int64_t(1) << 40) - 1 : key),
                         P.rank[i]);
    }
    std::sort(keyed.begin(), keyed.end());
    for (size_t q0 = 0; q0 < keyed.size(); ++q0) fw[t][q0] = P.order[std::get<2>(keyed[q0])];
    for (int32_t i : fw[t]) {
      P.var_first[i] = int32_t(L);
      for (int64_t q = iptr[i]; q < iptr[i + 1]; ++q, ++L) {
        const int32_t c = ilist[q];
        P.canon_of[L] = c;
        P.layer_of[c] = int32_t(L);
        P.layer_var[L] = i;
        segpos[L] = uint32_t(q - iptr[i]);
      }
    }
  }
  // a backward wave lists its variables by group, then in storage order, so that a backward wave
  // holding the same variables as a forward wave is one contiguous layer range (one group) and a
  // group's variables sit together in its tiles
  for (int32_t t = 1; t <= P.Db; ++t)
    std::sort(bw[t].begin(), bw[t].end(), [&](int32_t x, int32_t y) {
      return P.var_group[size_t(x)] != P.var_group[size_t(y)] ? P.var_group[size_t(x)] < P.var_group[size_t(y)]
                                                              : P.var_first[x] < P.var_first[y];
    });

  // node slots: a level of at most 2 nodes sits at slots 2L, 2L+1 (the second one padding when it
  // has one node); wider levels follow after 2I, in layer order
  const size_t In0 = static_cast<size_t>(I);
  std::vector<int32_t> ownw(In0), childw(In0, 0), child_layer(In0, -1), level(In0);
  std::vector<uint8_t> exit_cut(In0, 0), root_cut(In0, 0);
  for (int64_t Lq = 0; Lq < I; ++Lq) {
    const int32_t c = P.canon_of[Lq];
    const int32_t j = inc_row[c];
    const Shape &sh = P.shapes[P.row_shape[j]];
    const int32_t l = int32_t(c - P.canon_off[j]);
    level[Lq] = l;
    ownw[Lq] = sh.first[l + 1] - sh.first[l];
    if (l + 1 < sh.k) {
      if (cut_after[c]) {
        exit_cut[Lq] = 1;
        root_cut[P.layer_of[c + 1]] = 1;
      } else {
        childw[Lq] = sh.first[l + 2] - sh.first[l + 1];
        child_layer[Lq] = P.layer_of[c + 1];
      }
    }
  }
  // an exit layer's virtual child level: one slot per arc
  for (int64_t Lq = 0; Lq < I; ++Lq)
    if (exit_cut[Lq]) childw[Lq] = 2 * ownw[Lq];
  // Forward messages of a layer's own level sit at its own slots; the backward messages of its
  // child level are kept in a second slot space at its child slots, written there by the child
  // layer's backward step. Both spaces put levels of at most 2 nodes at 2L, 2L+1.
  P.own_slot.assign(size_t(I), 0);
  P.cslot.assign(size_t(I), 0);
  int64_t wide = 0, cwide = 0;
  for (int64_t Lq = 0; Lq < I; ++Lq) {
    if (ownw[Lq] <= 2) {
      P.own_slot[Lq] = 2 * Lq;
    } else {
      P.own_slot[Lq] = 2 * I + wide;
      wide += ownw[Lq];
    }
    if (childw[Lq] <= 2) {
      P.cslot[Lq] = 2 * Lq;
    } else {
      P.cslot[Lq] = 2 * I + cwide;
      cwide += childw[Lq];
    }
  }
  P.S = 2 * I + wide;
  P.Sc = 2 * I + cwide;
  if (P.S >= INT32_MAX || P.Sc >= INT32_MAX) return set_error(BDDMP_BDD_TOO_LARGE, "more than 2^31 node slots");
  auto code16 = [](int32_t c) -> uint32_t { return c == -1 ? kBot : (c == -2 ? kTop : uint32_t(c)); };
  auto code2 = [](int32_t c) -> uint32_t { return c == -1 ? kC2Bot : (c == -2 ? kC2Top : uint32_t(c)); };
  P.garcs.assign(size_t(P.S), kBot | (kBot << 16));
  P.meta.assign(size_t(I), 0);
  P.child.assign(size_t(I), -1);
  P.parent.assign(size_t(I), -1);
  for (int64_t Lq = 0; Lq < I; ++Lq) {
    P.child[Lq] = child_layer[Lq];
    if (child_layer[Lq] >= 0) P.parent[child_layer[Lq]] = int32_t(Lq);
  }
  // each layer writes only its own arcs and meta word: on several threads, general layers counted
  // per chunk
  std::vector<int64_t> n_gen_chunk;
  std::mutex n_gen_mu;
  parallel_for(I, [&](int64_t L0, int64_t L1) {
    int64_t n_gen = 0;
    for (int64_t Lq = L0; Lq < L1; ++Lq) {
      const int32_t c = P.canon_of[Lq];
      const int32_t j = inc_row[c];
      const Shape &sh = P.shapes[P.row_shape[j]];
      const int32_t l = level[Lq];
      const bool narrow = ownw[Lq] <= 2 && childw[Lq] <= 2;
      uint32_t meta = 0;
      // child of arc (u, beta): a node of the next level, or at a cut the arc's own virtual slot
      auto arc_child = [&](int32_t u, int beta) -> int32_t {
        const int32_t ch = beta ? sh.hi[sh.first[l] + u] : sh.lo[sh.first[l] + u];
        return (exit_cut[Lq] && ch >= 0) ? 2 * u + beta : ch;
      };
      for (int32_t u = 0; u < ownw[Lq]; ++u)
        P.garcs[size_t(P.own_slot[Lq] + u)] = code16(arc_child(u, 0)) | (code16(arc_child(u, 1)) << 16);
      if (narrow) {
        for (int32_t u = 0; u < 2; ++u) {
          const uint32_t lo = u < ownw[Lq] ? code2(arc_child(u, 0)) : kC2Bot;
          const uint32_t hi = u < ownw[Lq] ? code2(arc_child(u, 1)) : kC2Bot;
          meta |= (lo | (hi << 2)) << (4 * u);
        }
        meta |= uint32_t(ownw[Lq]) << kMetaWidthShift;
      } else {
        ++n_gen;
      }
      if (l == 0) meta |= kMetaRootBit;
      const uint32_t len = uint32_t(std::min<int32_t>(P.var_nj[P.layer_var[Lq]], int32_t(kMetaField)));
      meta |= (std::min<uint32_t>(segpos[Lq], kMetaField) << kMetaPosShift) | (len << kMetaLenShift);
      P.meta[Lq] = meta;
    }
    std::lock_guard<std::mutex> lk(n_gen_mu);
    n_gen_chunk.push_back(n_gen);
  });
  P.n_general = 0;
  for (int64_t v : n_gen_chunk) P.n_general += v;
  if (P.n_general) {
    // general records for every layer (a general level's neighbours read them too), and for each
    // general layer with a child level the in-arc lists of that child level: the pull form of the
    // forward step (Alg. "Forward BDD update step" takes the minimum over in-arcs)
    P.grec.assign(4 * size_t(I), 0);
    P.gnb.assign(2 * size_t(I), -1);
    for (int64_t Lq = 0; Lq < I; ++Lq) {
      if (P.child[Lq] >= 0) P.gnb[2 * size_t(Lq)] = int32_t(P.own_slot[P.child[Lq]]);
      if (P.parent[Lq] >= 0) P.gnb[2 * size_t(Lq) + 1] = int32_t(P.cslot[P.parent[Lq]]);
    }
    // per child node its in-arcs in ascending source order (the 0-arc before the 1-arc of one
    // source), by a counting sort into the flat arrays (sized beforehand)
    {
      size_t nb = 0, na = 0;
      for (int64_t Lq = 0; Lq < I; ++Lq)
        if (((P.meta[Lq] >> kMetaWidthShift) & 3u) == 0u && childw[Lq] > 0 && !exit_cut[Lq]) {
          nb += size_t(childw[Lq]) + 1;
          na += 2 * size_t(ownw[Lq]);
        }
      P.rbeg.reserve(nb);
      P.rin.reserve(nb);
      P.rarc.reserve(na);
    }
    std::vector<int64_t> at;
    for (int64_t Lq = 0; Lq < I; ++Lq) {
      int32_t *g = &P.grec[4 * size_t(Lq)];
      g[0] = int32_t(P.own_slot[Lq]);
      g[1] = int32_t(P.cslot[Lq]);
      g[2] = ownw[Lq] | (childw[Lq] << 16);
      g[3] = -1;
      const bool narrow = ((P.meta[Lq] >> kMetaWidthShift) & 3u) != 0u;
      if (narrow || childw[Lq] == 0 || exit_cut[Lq]) continue;
      g[3] = int32_t(P.rbeg.size());
      const int32_t wc = childw[Lq];
      const uint32_t *arcs = &P.garcs[size_t(P.own_slot[Lq])];
      at.assign(size_t(wc) + 1, 0);
      for (int32_t u = 0; u < ownw[Lq]; ++u) {
        if ((arcs[u] & 0xFFFFu) < kTop) ++at[(arcs[u] & 0xFFFFu) + 1];
        if ((arcs[u] >> 16) < kTop) ++at[(arcs[u] >> 16) + 1];
      }
      const int64_t base = int64_t(P.rarc.size());
      for (int32_t v = 0; v < wc; ++v) at[size_t(v) + 1] += at[size_t(v)];
      for (int32_t v = 0; v <= wc; ++v) P.rbeg.push_back(int32_t(base + at[size_t(v)]));
      P.rarc.resize(size_t(base + at[size_t(wc)]));
      for (int32_t u = 0; u < ownw[Lq]; ++u) {
        if ((arcs[u] & 0xFFFFu) < kTop) P.rarc[size_t(base + at[arcs[u] & 0xFFFFu]++)] = uint16_t(u);
        if ((arcs[u] >> 16) < kTop) P.rarc[size_t(base + at[arcs[u] >> 16]++)] = uint16_t(uint32_t(u) | kInArcHi);
      }
      // at[v] is now the end of v's list, rbeg (just appended) its start
      const int32_t *beg = &P.rbeg[P.rbeg.size() - size_t(wc) - 1];
      for (int32_t v = 0; v < wc; ++v) {
        const int64_t b0 = beg[v], k = int64_t(beg[v + 1]) - b0;
        P.rin.push_back(k > 2 ? kManyInArcs
                              : (k > 0 ? P.rarc[size_t(b0)] : kNoArc16) | ((k > 1 ? P.rarc[size_t(b0) + 1] : kNoArc16) << 16));
      }
      P.rin.push_back(kManyInArcs);
      if (P.rarc.size() >= size_t(INT32_MAX)) return set_error(BDDMP_BDD_TOO_LARGE, "too many in-arcs");
    }
  }
  // general-level work per variable (own plus child nodes of its general layers), for the tiler
  std::vector<int64_t> wwork(size_t(n), 0);
  for (int64_t Lq = 0; Lq < I; ++Lq)
    if (((P.meta[Lq] >> kMetaWidthShift) & 3u) == 0u) wwork[P.layer_var[Lq]] += ownw[Lq] + childw[Lq];
  P.root_slot.assign(size_t(m), -1);
  P.bdd_canon_off.assign(size_t(m) + 1, 0);
  for (int32_t j = 0; j < m; ++j) {
    P.bdd_canon_off[j + 1] = int32_t(P.canon_off[j + 1]);
    if (P.canon_off[j + 1] > P.canon_off[j]) P.root_slot[j] = int32_t(P.own_slot[P.layer_of[P.canon_off[j]]]);
  }

  // cut tables: arcs and live pairs numbered in canonical (row, level) order; the cut records list
  // the narrow cuts (both levels at most 2 nodes, one lane each) first, then the wide ones (one
  // wavefront each, with in-arc lists of the root level for its forward messages)
  for (int pass = 0; pass < 2; ++pass) {
    int64_t base = 0, live = 0;
    for (int32_t j = 0; j < m; ++j)
      for (int64_t c = P.canon_off[j]; c + 1 < P.canon_off[j + 1]; ++c) {
        if (!cut_after[c]) continue;
        const int32_t Lx = P.layer_of[c], Lr = P.layer_of[c + 1];
        const Shape &sh = P.shapes[P.row_shape[j]];
        const int32_t l = int32_t(c - P.canon_off[j]);
        const bool narrow = ownw[Lx] <= 2 && ownw[Lr] <= 2;
        int32_t nlive = 0;
        for (int32_t u = 0; u < ownw[Lx]; ++u)
          nlive += (sh.lo[sh.first[l] + u] >= 0) + (sh.hi[sh.first[l] + u] >= 0);
        if (narrow == (pass == 0)) {
          int32_t rb = -1;
          if (!narrow) {
            rb = int32_t(P.rbeg.size());
            std::vector<std::vector<uint16_t>> lists(static_cast<size_t>(ownw[Lr]));
            for (int32_t u = 0; u < ownw[Lx]; ++u) {
              if (sh.lo[sh.first[l] + u] >= 0) lists[sh.lo[sh.first[l] + u]].push_back(uint16_t(u));
              if (sh.hi[sh.first[l] + u] >= 0) lists[sh.hi[sh.first[l] + u]].push_back(uint16_t(uint32_t(u) | kInArcHi));
            }
            for (const auto &li : lists) {
              P.rbeg.push_back(int32_t(P.rarc.size()));
              P.rarc.insert(P.rarc.end(), li.begin(), li.end());
              P.rin.push_back(li.size() > 2 ? kManyInArcs
                                            : (li.size() > 0 ? li[0] : kNoArc16) | ((li.size() > 1 ? li[1] : kNoArc16) << 16));
            }
            P.rbeg.push_back(int32_t(P.rarc.size()));
            P.rin.push_back(kManyInArcs);
          }
          P.cuts.insert(P.cuts.end(), {Lx, Lr, int32_t(base), ownw[Lx] | (ownw[Lr] << 16)});
          P.cut_slots.insert(P.cut_slots.end(), {int32_t(P.own_slot[Lx]), int32_t(P.cslot[Lx]),
                                                 int32_t(P.own_slot[Lr]), int32_t(P.cslot[Lr])});
          P.cut_live.push_back(int32_t(live));
          P.cut_rb.push_back(rb);
          P.cut_row.push_back(j);
          P.n_cut_narrow += narrow;
        }
        if (pass == 0) {
          for (int32_t u = 0; u < ownw[Lx]; ++u)
            for (int beta = 0; beta < 2; ++beta)
              P.cut_arc.push_back(uint16_t(code16(beta ? sh.hi[sh.first[l] + u] : sh.lo[sh.first[l] + u])));
          P.n_arcs_cut += 2 * ownw[Lx];
          P.n_copy += nlive;
        }
        base += 2 * ownw[Lx];
        live += nlive;
      }
  }
  if (P.n_cuts >= INT32_MAX || P.n_arcs_cut >= INT32_MAX || P.rarc.size() >= size_t(INT32_MAX))
    return set_error(BDDMP_BDD_TOO_LARGE, "too many cuts or copy arcs");
  P.n_cut_parts = (P.n_cut_narrow + kTile - 1) / kTile + (P.n_cuts - P.n_cut_narrow + kCutsPerBlock - 1) / kCutsPerBlock;

  // forward tiles: positions are storage layers
  int64_t pos = 0;
  P.fwd_waves.resize(size_t(P.Df));
  auto wave_work = [&](const std::vector<int32_t> &vars, WaveRange &wr) {
    wr.nodes = 0;
    wr.layers = 0;
    wr.narrow_only = true;
    for (int32_t i : vars)
      for (int32_t q = 0; q < P.var_nj[i]; ++q) {
        const int32_t Lq = P.var_first[i] + q;
        wr.nodes += ownw[Lq];
        wr.layers += 1;
        wr.narrow_only = wr.narrow_only && ((P.meta[Lq] >> kMetaWidthShift) & 3u) != 0u;
      }
  };
  for (int32_t t = 1; t <= P.Df; ++t) {
    tile_pass(fw[t], P.var_nj, wwork, P.var_group, P.tile_work, pos, P.fwd_tiles, P.fwd_big, P.fwd_waves[t - 1]);
    P.fwd_waves[t - 1].list = 0;
    wave_work(fw[t], P.fwd_waves[t - 1]);
    for (int32_t i : fw[t]) pos += P.var_nj[i];
  }
  // backward order (wave_b, rank); a wave whose variables sit back to back in storage uses
  // storage positions directly, otherwise positions go through bwd_list
  P.bwd_list.assign(size_t(I), 0);
  P.bwd_waves.resize(size_t(P.Db));
  pos = 0;
  for (int32_t t = 1; t <= P.Db; ++t) {
    const int64_t w0 = pos;
    bool contig = true;
    for (int32_t i : bw[t])
      for (int32_t q = 0; q < P.var_nj[i]; ++q, ++pos) {
        P.bwd_list[pos] = P.var_first[i] + q;
        if (P.bwd_list[pos] != P.bwd_list[w0] + (pos - w0)) contig = false;
      }
    WaveRange &wr = P.bwd_waves[t - 1];
    tile_pass(bw[t], P.var_nj, wwork, P.var_group, P.tile_work, contig ? P.bwd_list[w0] : w0, P.bwd_tiles, P.bwd_big,
              wr);
    wr.list = contig ? 0 : 1;
    wave_work(bw[t], wr);
    P.bwd_contiguous = P.bwd_contiguous && contig;
  }
  if (P.bwd_contiguous) P.bwd_list.clear();
  // flag backward tiles holding a root level; bound partials: one per wavefront of a normal tile,
  // one per big tile
  for (const WaveRange &wr : P.bwd_waves)
    for (int32_t t = wr.tile_begin; t < wr.tile_end; ++t) {
      bool roots = false;
      for (int64_t q = P.bwd_tiles[2 * size_t(t)]; q < P.bwd_tiles[2 * size_t(t) + 1]; ++q) {
        const int64_t Lq = wr.list ? P.bwd_list[size_t(q)] : q;
        roots = roots || level[Lq] == 0;
      }
      if (roots) P.bwd_tiles[2 * size_t(t) + 1] = int32_t(uint32_t(P.bwd_tiles[2 * size_t(t) + 1]) | kTileRootBit);
    }
  P.n_lbpart = int64_t(kTile / 64) * int64_t(P.bwd_tiles.size() / 2) + int64_t(P.bwd_big.size() / 2);
  // turnaround: a variable of the last forward wave is last in each of its rows, so its backward
  // wave is the first; when the first backward wave holds exactly those layers, tiled alike, the
  // backward pass's first step on them can follow the forward pass's last one inside one launch
  P.fuse_turn = false;
  if (P.Df > 0 && P.Db > 0 && P.n_cuts == 0) {
    const WaveRange &F = P.fwd_waves.back(), &Bw = P.bwd_waves.front();
    bool same = F.narrow_only && Bw.narrow_only && !Bw.list && F.big_begin == F.big_end &&
                Bw.big_begin == Bw.big_end && F.tile_end - F.tile_begin == Bw.tile_end - Bw.tile_begin &&
                F.tile_end > F.tile_begin;
    for (int32_t k = 0; same && k < F.tile_end - F.tile_begin; ++k) {
      const size_t f = 2 * size_t(F.tile_begin + k), b = 2 * size_t(Bw.tile_begin + k);
      const int64_t f0 = int64_t(uint32_t(P.fwd_tiles[f]) & kTilePosMask), f1 = P.fwd_tiles[f + 1];
      const int64_t b0 = int64_t(uint32_t(P.bwd_tiles[b]) & kTilePosMask);
      const int64_t b1 = int64_t(uint32_t(P.bwd_tiles[b + 1]) & ~kTileRootBit);
      same = f0 == b0 && f1 == b1;
      for (int64_t L = f0; same && L < f1; ++L) same = P.child[size_t(L)] < 0;
    }
    P.fuse_turn = same;
  }
  // wrap-around: a variable of the first forward wave is first in each of its rows, so its backward
  // wave is the last; when that wave holds exactly those layers, tiled alike, the last backward step
  // of one iteration and the first forward step of the next can share a launch
  P.fuse_wrap = false;
  if (P.Df > 1 && P.Db > 1 && P.n_cuts == 0) {
    const WaveRange &F = P.fwd_waves.front(), &Bw = P.bwd_waves.back();
    bool same = F.narrow_only && Bw.narrow_only && !Bw.list && F.big_begin == F.big_end &&
                Bw.big_begin == Bw.big_end && F.tile_end - F.tile_begin == Bw.tile_end - Bw.tile_begin &&
                F.tile_end > F.tile_begin;
    for (int32_t k = 0; same && k < F.tile_end - F.tile_begin; ++k) {
      const size_t f = 2 * size_t(F.tile_begin + k), b = 2 * size_t(Bw.tile_begin + k);
      const int64_t f0 = int64_t(uint32_t(P.fwd_tiles[f]) & kTilePosMask), f1 = P.fwd_tiles[f + 1];
      const int64_t b0 = int64_t(uint32_t(P.bwd_tiles[b]) & kTilePosMask);
      const int64_t b1 = int64_t(uint32_t(P.bwd_tiles[b + 1]) & ~kTileRootBit);
      same = f0 == b0 && f1 == b1;
      for (int64_t L = f0; same && L < f1; ++L) same = P.parent[size_t(L)] < 0;
    }
    P.fuse_wrap = same;
  }
  // width class of each normal tile in the top bits of its start
  for (int pass = 0; pass < 2; ++pass) {
    auto &tiles = pass ? P.bwd_tiles : P.fwd_tiles;
    const auto &waves = pass ? P.bwd_waves : P.fwd_waves;
    for (const WaveRange &wr : waves)
      for (int32_t t = wr.tile_begin; t < wr.tile_end; ++t) {
        int32_t mw = 0;
        const int64_t p1 = int64_t(uint32_t(tiles[2 * size_t(t) + 1]) & ~kTileRootBit);
        for (int64_t q = tiles[2 * size_t(t)]; q < p1; ++q) {
          const int64_t Lq = (pass && wr.list) ? P.bwd_list[size_t(q)] : q;
          if (((P.meta[Lq] >> kMetaWidthShift) & 3u) == 0u) mw = std::max({mw, ownw[Lq], childw[Lq]});
        }
        const uint32_t cls = mw <= 8 ? 0u : (mw <= 32 ? 1u : (mw <= 128 ? 2u : 3u));
        tiles[2 * size_t(t)] = int32_t(uint32_t(tiles[2 * size_t(t)]) | (cls << kTileClsShift));
        if (mw > 0) P.class_tiles[cls]++;
      }
  }

  // node maps of the flat path: the layer rank of every own and child node a tile stages, so that
  // the kernel reads it from LDS instead of searching the level offsets
  for (int pass = 0; pass < 2; ++pass) {
    const auto &tiles = pass ? P.bwd_tiles : P.fwd_tiles;
    const auto &waves = pass ? P.bwd_waves : P.fwd_waves;
    auto &gt = pass ? P.bgt : P.fgt;
    auto &gm = pass ? P.bgm : P.fgm;
    gt.assign(tiles.size(), 0);
    gm.clear();
    std::vector<int64_t> gen;
    for (const WaveRange &wr : waves)
      for (int32_t t = wr.tile_begin; t < wr.tile_end; ++t) {
        gt[2 * size_t(t)] = -1;
        gen.clear();
        const int64_t p0 = uint32_t(tiles[2 * size_t(t)]) & kTilePosMask;
        const int64_t p1 = uint32_t(tiles[2 * size_t(t) + 1]) & ~kTileRootBit;
        int64_t tw = 0, tc = 0;
        for (int64_t q = p0; q < p1; ++q) {
          const int64_t Lq = (pass && wr.list) ? P.bwd_list[size_t(q)] : q;
          if (((P.meta[size_t(Lq)] >> kMetaWidthShift) & 3u) != 0u) continue;
          gen.push_back(Lq);
          tw += ownw[size_t(Lq)];
          tc += childw[size_t(Lq)];
        }
        if (gen.empty() || tw > kFlatCap || tc > kFlatCap) continue;
        gt[2 * size_t(t)] = int32_t(gm.size());
        gt[2 * size_t(t) + 1] = int32_t(tw | (tc << 16));
        for (int part = 0; part < 2; ++part)
          for (size_t k = 0; k < gen.size(); ++k)
            gm.insert(gm.end(), size_t(part ? childw[size_t(gen[k])] : ownw[size_t(gen[k])]), uint8_t(k));
        gm.resize((gm.size() + 15) / 16 * 16, 0);
      }
    if (gm.size() >= size_t(INT32_MAX)) return set_error(BDDMP_BDD_TOO_LARGE, "node maps beyond 2^31 bytes");
  }

  // dataflow launch: each tile waits only for the tiles that write what it reads. In the forward
  // pass a layer reads its own level's forward messages, pushed by its parent layer; in the
  // backward pass its child level's backward messages, written by its child layer's backward step.
  // Everything else a tile reads (multipliers of its own layers, the other pass's messages, the
  // structure) is written before the pass begins.
  P.pers_ok = P.fwd_big.empty() && P.bwd_big.empty();
  P.fdep_ptr.clear();
  P.fdep_list.clear();
  P.bdep_ptr.clear();
  P.bdep_list.clear();
  P.ftinfo.clear();
  P.btinfo.clear();
  P.fsplit.clear();
  P.bsplit.clear();
  if (P.pers_ok) {
    std::vector<int32_t> tile_of(In0, -1), d;
    for (int pass = 0; pass < 2; ++pass) {
      const auto &tiles = pass ? P.bwd_tiles : P.fwd_tiles;
      const auto &waves = pass ? P.bwd_waves : P.fwd_waves;
      auto &ptr = pass ? P.bdep_ptr : P.fdep_ptr;
      auto &lst = pass ? P.bdep_list : P.fdep_list;
      auto &info = pass ? P.btinfo : P.ftinfo;
      const size_t nt = tiles.size() / 2;
      auto layer_at = [&](const WaveRange &wr, int64_t q) { return (pass && wr.list) ? int64_t(P.bwd_list[size_t(q)]) : q; };
      auto span = [&](int32_t t) {
        return std::make_pair(int64_t(uint32_t(tiles[2 * size_t(t)]) & kTilePosMask),
                              int64_t(uint32_t(tiles[2 * size_t(t) + 1]) & ~kTileRootBit));
      };
      for (const WaveRange &wr : waves)
        for (int32_t t = wr.tile_begin; t < wr.tile_end; ++t)
          for (int64_t q = span(t).first; q < span(t).second; ++q) tile_of[size_t(layer_at(wr, q))] = t;
      ptr.assign(nt + 1, 0);
      info.assign(nt, 0u);
      for (const WaveRange &wr : waves)
        for (int32_t t = wr.tile_begin; t < wr.tile_end; ++t) {
          d.clear();
          bool narrow = true;
          for (int64_t q = span(t).first; q < span(t).second; ++q) {
            const int64_t Lq = layer_at(wr, q);
            const int32_t nb = pass ? P.child[size_t(Lq)] : P.parent[size_t(Lq)];
            if (nb >= 0) d.push_back(tile_of[size_t(nb)]);
            narrow = narrow && ((P.meta[size_t(Lq)] >> kMetaWidthShift) & 3u) != 0u;
          }
          std::sort(d.begin(), d.end());
          d.erase(std::unique(d.begin(), d.end()), d.end());
          lst.insert(lst.end(), d.begin(), d.end());
          ptr[size_t(t) + 1] = int32_t(lst.size());
          info[size_t(t)] = (narrow ? 1u : 0u) | (wr.list ? 2u : 0u);
        }
      // issue priority from the slack of each tile on the pass's dependency graph: the longest chain
      // of tiles through it against the longest chain of the pass. Tiles on (or near) the longest
      // chains run at a higher wave priority, so their latency, which sets the pass's length, is
      // less inflated by the other workgroups sharing their compute unit.
      std::vector<int32_t> depth(nt, 1), height(nt, 1);
      for (size_t t = 0; t < nt; ++t)
        for (int32_t q = ptr[t]; q < ptr[t + 1]; ++q) depth[t] = std::max(depth[t], depth[size_t(lst[size_t(q)])] + 1);
      for (size_t t = nt; t-- > 0;)
        for (int32_t q = ptr[t]; q < ptr[t + 1]; ++q)
          height[size_t(lst[size_t(q)])] = std::max(height[size_t(lst[size_t(q)])], height[t] + 1);
      int32_t longest = 0;
      for (size_t t = 0; t < nt; ++t) longest = std::max(longest, depth[t] + height[t] - 1);
      for (size_t t = 0; t < nt; ++t) {
        const int32_t slack = longest - (depth[t] + height[t] - 1);
        const uint32_t prio = slack <= 1 ? 3u : (slack <= 4 ? 2u : (slack <= 16 ? 1u : 0u));
        info[t] |= prio << 2;
      }
      // the group's queue: its tiles in pass order
      auto &qptr = pass ? P.bqptr : P.fqptr;
      auto &qtile = pass ? P.bqtile : P.fqtile;
      std::vector<int32_t> tgroup(nt, 0);
      for (const WaveRange &wr : waves)
        for (int32_t t = wr.tile_begin; t < wr.tile_end; ++t)
          tgroup[size_t(t)] = P.var_group[size_t(P.layer_var[size_t(layer_at(wr, span(t).first))])];
      qptr.assign(size_t(P.n_groups) + 1, 0);
      for (size_t t = 0; t < nt; ++t) qptr[size_t(tgroup[t]) + 1]++;
      for (int32_t g = 0; g < P.n_groups; ++g) qptr[size_t(g) + 1] += qptr[size_t(g)];
      qtile.assign(nt, 0);
      std::vector<int32_t> fill(qptr.begin(), qptr.end() - 1);
      for (size_t t = 0; t < nt; ++t) qtile[size_t(fill[size_t(tgroup[t])]++)] = int32_t(t);
      auto &rec = pass ? P.btrec : P.ftrec;
      rec.assign(8 * nt, -1);
      for (size_t t = 0; t < nt; ++t) {
        const int32_t nd = ptr[t + 1] - ptr[t];
        rec[8 * t] = tiles[2 * t];
        rec[8 * t + 1] = tiles[2 * t + 1];
        rec[8 * t + 2] = int32_t(info[t] | (uint32_t(nd) << 8));
        rec[8 * t + 3] = ptr[t];
        for (int32_t q = 0; q < std::min(nd, 4); ++q) rec[8 * t + 4 + q] = lst[size_t(ptr[t] + q)];
      }
      // two-branch split of each wave: the longest prefix whose dependencies all lie in earlier
      // prefixes, cut at half the wave; the rest waits for the latest prefix it reads from
      auto &split = pass ? P.bsplit : P.fsplit;
      split.assign(waves.size(), Plan::WaveSplit{0, -1});
      std::vector<int32_t> wave_of(nt, 0);
      for (size_t w = 0; w < waves.size(); ++w) {
        const WaveRange &wr = waves[w];
        for (int32_t t = wr.tile_begin; t < wr.tile_end; ++t) wave_of[size_t(t)] = int32_t(w);
        const int32_t cap = wr.tile_begin + (wr.tile_end - wr.tile_begin + 1) / 2;
        int32_t mid = wr.tile_begin;
        auto in_a = [&](int32_t u) { return u < split[size_t(wave_of[size_t(u)])].mid; };
        for (; mid < cap; ++mid) {
          bool ok = true;
          for (int32_t q = ptr[size_t(mid)]; ok && q < ptr[size_t(mid) + 1]; ++q) ok = in_a(lst[size_t(q)]);
          if (!ok) break;
        }
        int32_t b_wait = -1;
        for (int32_t t = mid; t < wr.tile_end; ++t)
          for (int32_t q = ptr[size_t(t)]; q < ptr[size_t(t) + 1]; ++q)
            if (in_a(lst[size_t(q)])) b_wait = std::max(b_wait, wave_of[size_t(lst[size_t(q)])]);
        split[w] = Plan::WaveSplit{mid, b_wait};
      }
    }
  }

  P.lb_const = 0.0;
  for (int32_t i = 0; i < n; ++i)
    if (!P.var_nj[i] && p.cost[i] < 0) P.lb_const += p.cost[i];

  // instances (one unless the problem concatenates several)
  if (p.inst_var.empty()) {
    P.inst_var = {0, n};
    P.inst_row = {0, m};
  } else {
    P.inst_var = p.inst_var;
    P.inst_row = p.inst_row;
  }
  const size_t n_inst = P.inst_var.size() - 1;
  P.inst_inc.assign(n_inst + 1, 0);
  P.inst_lb_const.assign(n_inst, 0.0);
  P.inst_row32.assign(n_inst + 1, 0);
  for (size_t k = 0; k <= n_inst; ++k) {
    P.inst_inc[k] = P.canon_off[size_t(P.inst_row[k])];
    P.inst_row32[k] = int32_t(P.inst_row[k]);
  }
  for (size_t k = 0; k < n_inst; ++k)
    for (int64_t i = P.inst_var[k]; i < P.inst_var[k + 1]; ++i)
      if (!P.var_nj[size_t(i)] && p.cost[size_t(i)] < 0) P.inst_lb_const[k] += p.cost[size_t(i)];

  // the cut record of each exit layer (the row-violation walk maps its virtual arc codes back)
  if (P.n_cuts) {
    P.exit_rec.assign(static_cast<size_t>(I), -1);
    for (int64_t c = 0; c < P.n_cuts; ++c) P.exit_rec[size_t(P.cuts[4 * size_t(c)])] = int32_t(c);
  }
  // each instance's cut records in canonical (row, level) order
  {
    std::vector<int32_t> order_c(static_cast<size_t>(P.n_cuts));
    std::iota(order_c.begin(), order_c.end(), 0);
    std::stable_sort(order_c.begin(), order_c.end(), [&](int32_t a, int32_t b) {
      return P.canon_of[P.cuts[4 * size_t(a)]] < P.canon_of[P.cuts[4 * size_t(b)]];
    });
    P.inst_cut.assign(n_inst + 1, 0);
    P.inst_cut_idx.clear();
    size_t q = 0;
    for (size_t k = 0; k < n_inst; ++k) {
      P.inst_cut[k] = int32_t(P.inst_cut_idx.size());
      while (q < order_c.size() && P.cut_row[size_t(order_c[q])] < P.inst_row[k + 1]) P.inst_cut_idx.push_back(order_c[q++]);
    }
    P.inst_cut[n_inst] = int32_t(P.inst_cut_idx.size());
  }

  // arena layout
  ArenaLayout &A = P.lay;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t In = size_t(I), nn = size_t(n), mm = size_t(m), S = size_t(P.S);
  A.meta = take(4 * In);
  A.child = take(4 * In);
  A.parent = take(4 * In);
  A.lam = take(4 * In);
  A.mf = take(4 * S + 16);
  A.mbc = take(4 * size_t(P.Sc) + 16);
  A.garcs = take(4 * S);
  A.grec = take(4 * P.grec.size());
  A.gnb = take(4 * P.gnb.size());
  A.rbeg = take(4 * P.rbeg.size());
  A.rin = take(4 * P.rin.size());
  A.rarc = take(2 * P.rarc.size());
  A.canon_of = take(4 * In);
  A.layer_of = take(4 * In);
  A.layer_var = take(4 * In);
  A.root_slot = take(4 * mm);
  A.fwd_tiles = take(4 * P.fwd_tiles.size());
  A.bwd_tiles = take(4 * P.bwd_tiles.size());
  A.bwd_list = take(4 * P.bwd_list.size());
  A.fwd_big = take(4 * P.fwd_big.size());
  A.bwd_big = take(4 * P.bwd_big.size());
  A.bdd_canon_off = take(4 * (mm + 1));
  A.cost = take(8 * nn);
  A.var_first = take(4 * nn);
  A.var_nj = take(4 * nn);
  A.d_fresh = take(4 * In);
  A.mbuf = take(4 * nn);
  A.xbuf = take(nn);
  A.part = take(8 * 2 * size_t(kLbBlocks));
  A.lbpart = take(8 * size_t(P.n_lbpart + P.n_cut_parts + 1));
  A.lb_hist = take(8 * size_t(P.hist_cap));
  A.scal = take(256);
  A.inst_row = take(4 * P.inst_row32.size());
  A.inst_lb = take(8 * P.inst_lb_const.size());
  const size_t na = size_t(P.n_arcs_cut);
  A.cuts = take(4 * P.cuts.size());
  A.cut_slots = take(4 * P.cut_slots.size());
  A.cut_live = take(4 * P.cut_live.size());
  A.cut_rb = take(4 * P.cut_rb.size());
  A.cut_arc = take(2 * na);
  A.mu_in = take(4 * na);
  A.dfw = take(4 * na);
  A.dbw = take(4 * na);
  A.cut_e = take(4 * size_t(P.n_cuts));
  A.inst_cut = take(4 * P.inst_cut.size());
  A.inst_cut_idx = take(4 * P.inst_cut_idx.size());
  A.exit_rec = take(4 * P.exit_rec.size());
  A.fdep_list = take(4 * P.fdep_list.size());
  A.bdep_list = take(4 * P.bdep_list.size());
  A.ftrec = take(4 * P.ftrec.size());
  A.btrec = take(4 * P.btrec.size());
  A.fqptr = take(4 * P.fqptr.size());
  A.fqtile = take(4 * P.fqtile.size());
  A.bqptr = take(4 * P.bqptr.size());
  A.bqtile = take(4 * P.bqtile.size());
  A.fgt = take(4 * P.fgt.size());
  A.bgt = take(4 * P.bgt.size());
  A.fgm = take(P.fgm.size() + 16);
  A.bgm = take(P.bgm.size() + 16);
  A.fflag = take(4 * P.ftinfo.size());
  A.bflag = take(4 * P.btinfo.size());
  A.pctl = take(4 * 2 * size_t(kPassCtlWords));
  A.total = off;
  const std::string bad = validate_layout(P, ownw, childw, level, exit_cut, root_cut);
  if (!bad.empty()) return set_error(BDDMP_INVALID_ARG, "internal layout check failed: " + bad);
  return BDDMP_OK;
}

}  // namespace bddmp
