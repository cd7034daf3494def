// Device code of bddmp: wave kernels for the forward and backward passes, the fp64 bound, and the
// output kernels, with the launch functions declared in kernels.h.
//
// One wave kernel launch runs every layer (one BDD level of one row) whose variable belongs to the
// wave. A workgroup takes a tile of up to 256 consecutive layers; a variable's layers (its rows
// J_i, ascending) never straddle tiles, so the J_i sum is a workgroup-local LDS reduction. One
// lane handles one layer.
//
// Narrow layers (the level and the next one have at most 2 nodes: every MRF, matching and
// tracking row) need a meta word (arcs as 2-bit codes, width, root flag, segment), the child or
// parent layer index, the multiplier, and two float2 message pairs at slot 2L: the own level's
// forward messages and the child level's backward messages. All loads are at the layer's own
// index and issue together; only the two float2 stores scatter. Wider layers read a general
// record and loop over their nodes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "device.h"
#include "kernels.h"

namespace bddmp {

namespace {

// multiplier update of eq. "mma-update"; rows forcing the variable (infinite difference) absorb
// the finite differences of the others
__device__ __forceinline__ float updated(float lam0, float d, float share, int nf) {
  return nf == 0 ? (lam0 - d) + share : (isinf(d) ? lam0 + share : lam0 - d);
}

// One layer's work split around the J_i sum: begin() computes the min-marginals, push() /
// bstep() apply the new multiplier in the forward push or the backward step.
//
// Every load of a layer is at its own index: its meta word, multiplier, the forward messages of its
// level (written there by its parent's push) and the backward messages of its child level (written
// there by its child's backward step), so all of them issue together. Only the stores scatter:
// the forward push goes to the child layer's own slots, the backward step to the parent layer's
// child slots. tgt is that child (forward) or parent (backward) layer, -1 at a row's end.
// NARROW_ONLY instantiations serve waves without wide levels: no per-lane branch, so the compiler
// issues all loads at once instead of sinking the message loads behind the meta word.
// LOOP: a general layer is handled by its own lane, looping over its nodes (big tiles); otherwise
// general layers are left to the lane groups of the wave kernel. COH: messages of this pass are
// read and written coherently (dataflow launch; see msg_ld).
template <int DIR, bool NARROW_ONLY, bool LOOP, bool COH = false>
struct Layer {
  int L;
  int tgt;
  uint32_t meta;
  float lam0;
  float2 f, b;     // narrow: own forward messages, child backward messages
  float m0, m1;

  __device__ __forceinline__ bool narrow() const {
    return NARROW_ONLY || ((meta >> kMetaWidthShift) & 3u) != 0u;
  }

  // begin() in two steps, for launches whose tiles wait for other tiles of the same pass: first the
  // loads no tile of this pass writes (meta word, multiplier, neighbour layer, the other pass's
  // message pair), then, once the tiles it depends on are done, the pair this pass writes (the own
  // level's forward messages in a forward pass, the child level's backward messages in a backward
  // pass) and the narrow min-marginals
  __device__ __forceinline__ void begin_fixed(const Dev &D, int L_) {
    L = L_;
    meta = D.meta[L];
    lam0 = D.lam[L];
    tgt = DIR == kFwd ? D.child[L] : D.parent[L];
    if (DIR == kFwd) b = msg_ld2<false>(D.mbc + 2 * L);
    else f = msg_ld2<false>(D.mf + 2 * L);
  }
  __device__ __forceinline__ void begin_pass(const Dev &D) {
    take_pass(msg_ld2<COH>((DIR == kFwd ? D.mf : D.mbc) + 2 * L));
  }
  // the same with the pair already loaded
  __device__ __forceinline__ void take_pass(float2 pair) {
    if (DIR == kFwd) f = pair;
    else b = pair;
    m0 = INFINITY;
    m1 = INFINITY;
    if (narrow()) narrow_marginals(lam0);
  }

  __device__ __forceinline__ void begin(const Dev &D, int L_) {
    L = L_;
    meta = D.meta[L];
    lam0 = D.lam[L];
    tgt = DIR == kFwd ? D.child[L] : D.parent[L];
    f = msg_ld2<COH && DIR == kFwd>(D.mf + 2 * L);
    b = msg_ld2<COH && DIR == kBwd>(D.mbc + 2 * L);
    // keep the five independent loads ahead of every use, so they are in flight together
    __builtin_amdgcn_sched_barrier(0);
    m0 = INFINITY;
    m1 = INFINITY;
    if (narrow()) {
      narrow_marginals(lam0);
    } else if (LOOP) {
      const GRec g = grec_of(D, L);
      for (int u = 0; u < g.w; ++u) {
        const uint32_t a = D.garcs[g.os + u];
        const float fu = D.mf[g.os + u];
        m0 = fminf(m0, fu + c16val(D.mbc, g.cs, a & 0xFFFFu));
        m1 = fminf(m1, (fu + lam0) + c16val(D.mbc, g.cs, a >> 16));
      }
    }
  }

  // arc-marginals (m_fwd + theta) + m_bwd minimised per arc label (eqs. "arc-marginal",
  // "marginal-aggregation") of a narrow layer under multiplier lam; a padding node's arcs both lead
  // to BOT
  __device__ __forceinline__ void narrow_marginals(float lam) {
    const uint32_t lo0 = meta & 3u, hi0 = (meta >> 2) & 3u, lo1 = (meta >> 4) & 3u, hi1 = (meta >> 6) & 3u;
    m0 = fminf(f.x + c2val(lo0, b), f.y + c2val(lo1, b));
    m1 = fminf((f.x + lam) + c2val(hi0, b), (f.y + lam) + c2val(hi1, b));
  }

  // forward step of the next level (Alg. "Forward BDD update step") pushed from this level: the
  // lane owns the whole next level, so the min over in-arcs needs no synchronisation
  __device__ __forceinline__ void push(const Dev &D, float lam1) const {
    if (tgt < 0) return;
    if (narrow()) {
      // arc values into the next level's node 0 and node 1, selected per child code (no indexing)
      const float a0 = f.x, a1 = f.x + lam1, a2 = f.y, a3 = f.y + lam1;
      const uint32_t k0 = meta & 3u, k1 = (meta >> 2) & 3u, k2 = (meta >> 4) & 3u, k3 = (meta >> 6) & 3u;
      const float c0 = fminf(fminf(k0 == 0u ? a0 : INFINITY, k1 == 0u ? a1 : INFINITY),
                             fminf(k2 == 0u ? a2 : INFINITY, k3 == 0u ? a3 : INFINITY));
      const float c1 = fminf(fminf(k0 == 1u ? a0 : INFINITY, k1 == 1u ? a1 : INFINITY),
                             fminf(k2 == 1u ? a2 : INFINITY, k3 == 1u ? a3 : INFINITY));
      msg_st2<COH>(D.mf + 2 * tgt, make_float2(c0, c1));
    } else if (LOOP) {
      const GRec g = grec_of(D, L);
      const int cs = D.grec[tgt].x;  // the child layer's own slots
      for (int q = 0; q < g.wc; ++q) D.mf[cs + q] = INFINITY;
      for (int u = 0; u < g.w; ++u) {
        const uint32_t a = D.garcs[g.os + u];
        const uint32_t lo = a & 0xFFFFu, hi = a >> 16;
        const float fu = D.mf[g.os + u];
        if (lo < kTop) D.mf[cs + int(lo)] = fminf(D.mf[cs + int(lo)], fu);
        if (hi < kTop) D.mf[cs + int(hi)] = fminf(D.mf[cs + int(hi)], fu + lam1);
      }
    }
  }

  // a narrow root level's new backward message (the backward step's value at node 0) as a bound
  // term, 0 on other levels
  __device__ __forceinline__ double root_value(float lam1) const {
    const float n0 = fminf(c2val(meta & 3u, b), c2val((meta >> 2) & 3u, b) + lam1);
    return (meta & kMetaRootBit) ? double(n0) : 0.0;
  }

  // backward step of this level (Alg. "Backward BDD update step") with the updated multiplier,
  // stored at the parent layer's child slots; returns the root's new backward message (E^j) on a
  // root level, else 0
  __device__ __forceinline__ double bstep(const Dev &D, float lam1) const {
    float r = 0.0f;
    if (narrow()) {
      const float n0 = fminf(c2val(meta & 3u, b), c2val((meta >> 2) & 3u, b) + lam1);
      const float n1 = fminf(c2val((meta >> 4) & 3u, b), c2val((meta >> 6) & 3u, b) + lam1);
      if (tgt >= 0) msg_st2<COH>(D.mbc + 2 * tgt, make_float2(n0, n1));
      r = n0;
    } else if (LOOP) {
      const GRec g = grec_of(D, L);
      const int ps = tgt >= 0 ? D.grec[tgt].y : -1;  // the parent layer's child slots
      for (int u = 0; u < g.w; ++u) {
        const uint32_t a = D.garcs[g.os + u];
        const float v = fminf(c16val(D.mbc, g.cs, a & 0xFFFFu), c16val(D.mbc, g.cs, a >> 16) + lam1);
        if (ps >= 0) D.mbc[ps + u] = v;
        if (u == 0) r = v;
      }
    }
    return (meta & kMetaRootBit) ? double(r) : 0.0;
  }
};

// General layers of a tile. Their records are read once by the layer's own lane and kept in LDS
// by compact index k (the layer's rank among the tile's general layers, in position order).
struct GenTile {
  int os[kTile], cs[kTile], ww[kTile];
  // forward tiles use the child layer's own slot and the in-arc base, backward tiles the parent's
  // child slot and node 0's new backward message (the root value on a root level)
  union {
    int osc[kTile];
    int pcs[kTile];
  };
  union {
    int rb[kTile];
    float e[kTile];
  };
  int wo[kTile + 1], co[kTile + 1];  // exclusive prefix sums of own / child level widths
  float lam[kTile];
  unsigned m0[kTile], m1[kTile];     // min-marginals as order-preserving integers
};

// float <-> unsigned with the same order (for integer min in LDS; a bijection, so exact)
__device__ __forceinline__ unsigned ord_of(float f) {
  const unsigned b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float float_of(unsigned u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

// Forward step of next-level node v of a general layer (pull form of Alg. "Forward BDD update
// step"): the minimum over its in-arcs of (source forward message + lam on a 1-arc). fu_of(u)
// gives the forward message of this level's node u.
template <class F>
__device__ __forceinline__ float pull_min_pk(const Dev &D, uint32_t pk, int rb, int v, float lam, F fu_of) {
  if (pk != kManyInArcs) {
    const uint32_t a0 = pk & 0xFFFFu, a1 = pk >> 16;
    const float f0 = fu_of(int(a0 & (kInArcHi - 1u)));
    float val = (a0 & kInArcHi) ? f0 + lam : f0;
    if (a1 != kNoArc16) {
      const float f1 = fu_of(int(a1 & (kInArcHi - 1u)));
      val = fminf(val, (a1 & kInArcHi) ? f1 + lam : f1);
    }
    return val;
  }
  const int b0 = D.rbeg[rb + v], b1 = D.rbeg[rb + v + 1];
  float val = INFINITY;
  for (int q = b0; q < b1; ++q) {
    const uint32_t a = D.rarc[q];
    const float fu = fu_of(int(a & (kInArcHi - 1u)));
    val = fminf(val, (a & kInArcHi) ? fu + lam : fu);
  }
  return val;
}
template <class F>
__device__ __forceinline__ float pull_min(const Dev &D, int rb, int v, float lam, F fu_of) {
  return pull_min_pk(D, D.rin[rb + v], rb, v, lam, fu_of);
}

// Group path: one general layer per group of G lanes (G a power of two up to 64; groups are
// aligned inside a wavefront, so a group's shuffles stay among its own lanes, which share their
// control flow). gl is the lane's index in its group.

// min-marginals: each lane minimises over its nodes, then a butterfly min over the group (min is
// exact, so the result does not depend on how nodes are split among lanes)
template <int DIR, bool COH>
__device__ __forceinline__ float2 group_mm(const Dev &D, const GenTile &T, int k, int gl, int G) {
  const int os = T.os[k], cs = T.cs[k], w = T.ww[k] & 0xFFFF;
  const float lam0 = T.lam[k];
  float m0 = INFINITY, m1 = INFINITY;
  for (int u = gl; u < w; u += G) {
    const uint32_t a = D.garcs[os + u];
    const float fu = msg_ld<COH && DIR == kFwd>(D.mf + os + u);
    m0 = fminf(m0, fu + c16val<COH && DIR == kBwd>(D.mbc, cs, a & 0xFFFFu));
    m1 = fminf(m1, (fu + lam0) + c16val<COH && DIR == kBwd>(D.mbc, cs, a >> 16));
  }
  for (int o = G >> 1; o > 0; o >>= 1) {
    m0 = fminf(m0, __shfl_xor(m0, o, 64));
    m1 = fminf(m1, __shfl_xor(m1, o, 64));
  }
  return make_float2(m0, m1);
}

// forward step of the next level in pull form: each lane takes next-level nodes and minimises
// over their in-arcs (Alg. "Forward BDD update step"), so no two lanes write one slot
template <bool COH>
__device__ __forceinline__ void group_push(const Dev &D, const GenTile &T, int k, int gl, int G) {
  const int osc = T.osc[k];
  if (osc < 0) return;
  const int os = T.os[k], wc = int(unsigned(T.ww[k]) >> 16), rb = T.rb[k];
  const float lam1 = T.lam[k];
  for (int v = gl; v < wc; v += G)
    msg_st<COH>(D.mf + osc + v, pull_min(D, rb, v, lam1, [&](int u) { return msg_ld<COH>(D.mf + os + u); }));
}

// backward step of this level, one node per lane; returns node 0's new message in lane 0
template <bool COH>
__device__ __forceinline__ float group_bstep(const Dev &D, const GenTile &T, int k, int gl, int G) {
  const int os = T.os[k], cs = T.cs[k], w = T.ww[k] & 0xFFFF, ps = T.pcs[k];
  const float lam1 = T.lam[k];
  float r = 0.0f;
  for (int u = gl; u < w; u += G) {
    const uint32_t a = D.garcs[os + u];
    const float v = fminf(c16val<COH>(D.mbc, cs, a & 0xFFFFu), c16val<COH>(D.mbc, cs, a >> 16) + lam1);
    if (ps >= 0) msg_st<COH>(D.mbc + ps + u, v);
    if (u == 0) r = v;
  }
  return r;
}

// Flat path: the tile's general nodes spread over all lanes (node t of the concatenated own
// levels, kFlatR per lane), with the child levels' backward messages and the own levels' forward
// messages staged in LDS. A layer's min-marginals are integer minima in LDS (exact).
constexpr int kFlatR = kFlatCap / kTile;   // nodes per lane

// Minimum of v over the lanes j - back .. j of the wavefront (the lanes of lane j's run so far;
// back <= lane), by DPP moves: shifts by 1, 2, 4 and 8 inside each row of 16 lanes, then the last
// lane of rows 0 and 2 into rows 1 and 3, then lane 31 into rows 2 and 3. A lane takes a moved
// value only when its source lies in its run. All 64 lanes must be active.
__device__ __forceinline__ unsigned run_min_up(unsigned v, int back, int lane) {
  constexpr int kNone = int(0xFFFFFFFFu);  // what a lane without a source receives; min identity
  unsigned w;
  w = unsigned(__builtin_amdgcn_update_dpp(kNone, int(v), 0x111, 0xF, 0xF, false));  // row_shr:1
  if (back >= 1) v = min(v, w);
  w = unsigned(__builtin_amdgcn_update_dpp(kNone, int(v), 0x112, 0xF, 0xF, false));  // row_shr:2
  if (back >= 2) v = min(v, w);
  w = unsigned(__builtin_amdgcn_update_dpp(kNone, int(v), 0x114, 0xF, 0xF, false));  // row_shr:4
  if (back >= 4) v = min(v, w);
  w = unsigned(__builtin_amdgcn_update_dpp(kNone, int(v), 0x118, 0xF, 0xF, false));  // row_shr:8
  if (back >= 8) v = min(v, w);
  w = unsigned(__builtin_amdgcn_update_dpp(kNone, int(v), 0x142, 0xA, 0xF, false));  // row_bcast:15
  if ((lane & 16) && back > (lane & 15)) v = min(v, w);
  w = unsigned(__builtin_amdgcn_update_dpp(kNone, int(v), 0x143, 0xC, 0xF, false));  // row_bcast:31
  if (lane >= 32 && back >= lane - 31) v = min(v, w);
  return v;
}

__device__ __forceinline__ float staged(const float *cb, int c0, uint32_t c) {
  return c < kTop ? cb[c0 + int(c)] : (c == kTop ? 0.0f : INFINITY);
}

// LDS of one tile of a wave kernel (narrow-only tiles need only the first members' storage)
template <bool NARROW_ONLY>
struct WaveLds {
  float d[kTile];
  int wcnt[kTile / 64];
  // general-layer paths (one element in narrow-only instantiations)
  std::conditional_t<NARROW_ONLY, int, GenTile> g;
  // J_i shares and forced-row counts; with general layers they reuse the min-marginal words, which
  // are read before the update begins (fewer LDS bytes per workgroup, more workgroups per CU)
  float share_n[NARROW_ONLY ? kTile : 1];
  int nf_n[NARROW_ONLY ? kTile : 1];
  // flat path: first the tile's node maps, then the next levels' backward messages; in a forward
  // tile, once the min-marginals are taken, the own levels' forward messages for the pull (one
  // array serves all three, so that more workgroups fit a CU's LDS)
  alignas(16) float cb[NARROW_ONLY ? 1 : kFlatCap];
};

// One tile of a wave: tix indexes the pass's tile list (dir DIR), btix the backward tile of the same
// levels (kWrap) or tix.
// LIST: backward positions go through bwd_list (a wave that is not one contiguous layer range).
// Narrow layers run one per lane. General layers (a level or its child level wider than 2) are
// collected per tile and run either node-parallel over the whole tile (flat path) or by groups of
// G lanes, as the tile's width class selects.
// w0, end: the tile's start and end words (positions with the width class and root bits).
// list: with LIST, whether this tile's positions go through bwd_list (callers that decide per tile
// instantiate LIST true and pass the tile's flag; the wave launches leave it true).
// COH: messages of this pass are read and written coherently (dataflow launch; see msg_ld).
// No wait inside a tile (wave launches, and tiles whose launch waited before the tile).
struct NoWait {
  __device__ __forceinline__ void operator()() const {}
};

template <int DIR, int MODE, bool NARROW_ONLY, bool LIST, bool COH = false, class Wait = NoWait>
__device__ __forceinline__ void wave_tile(const Dev &D, WaveLds<NARROW_ONLY> &sh, const int tix, const int btix,
                                          const uint32_t w0, const uint32_t end, const bool list = true,
                                          const Wait &wait = Wait{}) {
  // with a wait (a tile of a launch that also runs the tiles it depends on), the loads no tile of
  // this pass writes (and, in general tiles, the width scan) come first, then the wait, then the
  // messages this pass writes
  constexpr bool kDeferred = !std::is_same_v<Wait, NoWait>;
  static_assert(!kDeferred || MODE == kUpdate, "deferred waits: update mode");
  float *const s_d = sh.d;
  int *const s_wcnt = sh.wcnt;
  auto &s_g = sh.g;
  float *s_share;
  int *s_nf;
  if constexpr (NARROW_ONLY) {
    s_share = sh.share_n;
    s_nf = sh.nf_n;
  } else {
    s_share = reinterpret_cast<float *>(s_g.m0);
    s_nf = reinterpret_cast<int *>(s_g.m1);
  }
  float *const s_cb = sh.cb;
  float *const s_fu = s_cb;
  const int p0 = int(w0 & kTilePosMask);
  // a backward tile's end carries bit 31 when the tile holds a root level
  // kWrap: btix is the same levels' backward tile (its root flag and bound partials)
  const bool roots = (DIR == kBwd && (end & kTileRootBit) != 0u) ||
                     (MODE == kWrap && (uint32_t(D.bwd_tiles[2 * btix + 1]) & kTileRootBit) != 0u);
  const int cnt = int(end & ~kTileRootBit) - p0;
  const int s = int(threadIdx.x);
  const bool active = s < cnt;

  Layer<DIR, NARROW_ONLY, false, COH> ly;
  ly.meta = 0;
  ly.lam0 = 0.0f;
  ly.m0 = ly.m1 = 0.0f;
  ly.tgt = -1;
  int4 grec = make_int4(0, 0, 0, 0);
  int2 gnb = make_int2(-1, -1);
  // flat path (the tile's width class selects it and the tile has node maps, i.e. its general
  // levels fit the stage): the tile's node maps, 16 bytes per lane, loaded with the layer records
  const int mode = NARROW_ONLY ? 0 : int((D.gsel >> (4 * (w0 >> kTileClsShift))) & 0xFu);
  int2 gtr = make_int2(-1, 0);
  if constexpr (!NARROW_ONLY) {
    // every tile has a map record, so it is read whatever the width class, in flight together with
    // the caller's read of the tile's start and end words rather than after it
    gtr = (DIR == kFwd ? D.fgt : D.bgt)[tix];
    if (mode != int(kFlat)) gtr.x = -1;
  }
  const bool flat = !NARROW_ONLY && gtr.x >= 0;
  const bool map_lane = flat && 16 * s < (gtr.y & 0xFFFF) + int(uint32_t(gtr.y) >> 16);
  uint4 gmp = make_uint4(0u, 0u, 0u, 0u);
  if constexpr (!NARROW_ONLY)
    if (map_lane) gmp = *reinterpret_cast<const uint4 *>((DIR == kFwd ? D.fgm : D.bgm) + gtr.x + 16 * s);
  if (active) {
    const int L = (DIR == kBwd && LIST && list) ? D.bwd_list[p0 + s] : p0 + s;
    if (!NARROW_ONLY) {
      grec = D.grec[L];
      gnb = D.gnb[L];
    }
    if constexpr (kDeferred) ly.begin_fixed(D, L);
    else ly.begin(D, L);
  }
  if constexpr (kDeferred && NARROW_ONLY) {
    wait();
    if (active) ly.begin_pass(D);
  }
  // the maps into the stage (free until the staging below; the width scan's barriers publish them)
  if constexpr (!NARROW_ONLY)
    if (map_lane) reinterpret_cast<uint4 *>(s_cb)[s] = gmp;

  bool gen = false;
  int ngen = 0, myk = 0, G = 1, TW = 0, TC = 0;
  float2 pass_pair = make_float2(0.0f, 0.0f);
  uint32_t ar[NARROW_ONLY ? 1 : kFlatR];
  float fr[NARROW_ONLY ? 1 : kFlatR];
  int kr[NARROW_ONLY ? 1 : kFlatR];
  int ur[NARROW_ONLY ? 1 : kFlatR];  // flat path: a staged own node's index in its level
  // flat path, forward: layer of each staged next-level node and its packed in-arcs, loaded with
  // the node's backward message so that the pull needs no further round trip
  int kc[NARROW_ONLY ? 1 : kFlatR];
  uint32_t pkc[NARROW_ONLY ? 1 : kFlatR];
  if constexpr (!NARROW_ONLY) {
    GenTile &T = s_g;
    // compact index of the tile's general layers (ballot prefix per wavefront), and exclusive
    // prefix sums of their own and child widths (scan over the tile in position order)
    gen = active && !ly.narrow();
    const uint64_t mask = __ballot(gen);
    const int lane = s & 63, wv = s >> 6;
    const int w = gen ? (grec.z & 0xFFFF) : 0, wc = gen ? int(unsigned(grec.z) >> 16) : 0;
    int iw = w, ic = wc;
    for (int o = 1; o < 64; o <<= 1) {
      const int tw = __shfl_up(iw, o, 64), tc = __shfl_up(ic, o, 64);
      if (lane >= o) {
        iw += tw;
        ic += tc;
      }
    }
    if (lane == 63) {
      s_wcnt[wv] = __popcll(mask);
      s_d[wv] = __int_as_float(iw);
      s_share[wv] = __int_as_float(ic);
    }
    __syncthreads();
    int koff = 0, woff = 0, coff = 0;
    for (int q = 0; q < kTile / 64; ++q) {
      if (q < wv) {
        koff += s_wcnt[q];
        woff += __float_as_int(s_d[q]);
        coff += __float_as_int(s_share[q]);
      }
      ngen += s_wcnt[q];
      TW += __float_as_int(s_d[q]);
      TC += __float_as_int(s_share[q]);
    }
    __syncthreads();
    if (gen) {
      myk = koff + __popcll(mask & ((1ull << lane) - 1ull));
      T.os[myk] = grec.x;
      T.cs[myk] = grec.y;
      T.ww[myk] = grec.z;
      if (DIR == kFwd) {
        T.rb[myk] = grec.w;
        T.osc[myk] = gnb.x;
      } else {
        T.pcs[myk] = gnb.y;
      }
      T.wo[myk] = woff + iw - w;
      T.co[myk] = coff + ic - wc;
      T.lam[myk] = ly.lam0;
      T.m0[myk] = T.m1[myk] = ord_of(INFINITY);
    }
    G = mode == int(kFlat) ? 64 : (1 << mode);
    __syncthreads();
    if constexpr (kDeferred) {
      wait();
      // the pair of messages this pass writes, for every lane (a lane past the tile's layers reads
      // the first position's pair), issued before the node staging's loads and used after them: a
      // narrow layer's min-marginals are taken once the general layers' are
      pass_pair = msg_ld2<COH>((DIR == kFwd ? D.mf : D.mbc) + 2 * (active ? ly.L : p0));
    }
    if (flat) {
      // own nodes: arcs and forward messages; child nodes: backward messages into LDS. Node
      // t = s + r * kTile, its layer's rank from the node maps in the stage. Every lane issues
      // every load (a slot past the tile's nodes reads slot 2 p0, which exists in every slot
      // array, and is marked unused): with a branch per slot the compiler waited for one slot's
      // loads before issuing the next slot's.
      const uint8_t *maps = reinterpret_cast<const uint8_t *>(s_cb);
      int ks[kFlatR], kcs[kFlatR];
#pragma unroll
      for (int r = 0; r < kFlatR; ++r) {
        const int t = s + r * kTile;
        ks[r] = t < TW ? int(maps[t]) : 0;
        kcs[r] = t < TC ? int(maps[TW + t]) : 0;
      }
#pragma unroll
      for (int r = 0; r < kFlatR; ++r) {
        const int t = s + r * kTile;
        const bool ok = r * kTile < TW && t < TW;
        const int k = ks[r];
        const int u = ok ? t - T.wo[k] : 0;
        const int q = ok ? T.os[k] + u : 2 * p0;
        kr[r] = ok ? k : -1;
        ur[r] = u;
        ar[r] = D.garcs[q];
        fr[r] = msg_ld<COH && DIR == kFwd>(D.mf + q);
      }
      // all loads of the lane first, then the LDS stores: a store right after its load would wait
      // for that load before the next one issues
      float cbr[kFlatR];
#pragma unroll
      for (int r = 0; r < kFlatR; ++r) {
        const int t = s + r * kTile;
        const bool ok = r * kTile < TC && t < TC;
        const int k = kcs[r];
        kc[r] = ok ? k : -1;
        cbr[r] = msg_ld<COH && DIR == kBwd>(D.mbc + (ok ? T.cs[k] + (t - T.co[k]) : 2 * p0));
      }
      // the packed in-arcs (no slot of that array exists in every plan, so these stay conditional
      // and go last)
#pragma unroll
      for (int r = 0; r < kFlatR; ++r) {
        pkc[r] = kManyInArcs;
        const int k = kc[r];
        if (DIR == kFwd && k >= 0 && T.osc[k] >= 0) pkc[r] = D.rin[T.rb[k] + (s + r * kTile - T.co[k])];
      }
      // every lane has read its ranks before the stage takes the backward messages
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kFlatR; ++r)
        if (kc[r] >= 0) s_cb[s + r * kTile] = cbr[r];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kFlatR; ++r) {
        if (r * kTile >= TW) break;
        const int k = kr[r];
        unsigned o0 = ord_of(INFINITY), o1 = o0;
        int rest = 0, back = 0;  // nodes of the same level on the following / preceding lanes
        if (k >= 0) {
          const int c0 = T.co[k];
          const float lam0 = T.lam[k];
          rest = (T.ww[k] & 0xFFFF) - 1 - ur[r];
          back = min(ur[r], lane);
          o0 = ord_of(fr[r] + staged(s_cb, c0, ar[r] & 0xFFFFu));
          o1 = ord_of((fr[r] + lam0) + staged(s_cb, c0, ar[r] >> 16));
        }
        // segmented minimum over the runs of one level in the wavefront (a level's nodes sit on
        // consecutive lanes), gathered at each run's last lane, then one LDS atomic per run instead
        // of one per node; integer min of the order-preserving codes is exact
        o0 = run_min_up(o0, back, lane);
        o1 = run_min_up(o1, back, lane);
        if (k >= 0 && (lane == 63 || rest == 0)) {
          atomicMin(&T.m0[k], o0);
          atomicMin(&T.m1[k], o1);
        }
      }
    } else {
      const int grp = s / G, gl = s % G, ngrp = kTile / G;
      for (int k = grp; k < ngen; k += ngrp) {
        const float2 mm = group_mm<DIR, COH>(D, T, k, gl, G);
        if (gl == 0) {
          T.m0[k] = ord_of(mm.x);
          T.m1[k] = ord_of(mm.y);
        }
      }
    }
    __syncthreads();
    if (gen) {
      ly.m0 = float_of(T.m0[myk]);
      ly.m1 = float_of(T.m1[myk]);
    }
    if constexpr (kDeferred)
      if (active && !gen) ly.take_pass(pass_pair);
    if (DIR == kFwd && flat) {
#pragma unroll
      for (int r = 0; r < kFlatR; ++r)
        if (kr[r] >= 0) s_fu[s + r * kTile] = fr[r];
      // the pull below reads them after the barrier that publishes the new multipliers
    }
  }

  float d = ly.m1 - ly.m0;
  float lam1 = ly.lam0;
  if (MODE == kUpdate || MODE == kTurn || MODE == kWrap) {
    static_assert(MODE != kTurn || (DIR == kBwd && NARROW_ONLY && !LIST), "turnaround launch form");
    static_assert(MODE != kWrap || (DIR == kFwd && NARROW_ONLY && !LIST), "wrap-around launch form");
    const int pos = int((ly.meta >> kMetaPosShift) & kMetaField);
    const int len = int((ly.meta >> kMetaLenShift) & kMetaField);
    // kTurn: these levels are the last of their rows, so the forward pass's update of them is
    // followed at once by the backward pass's, with the new multipliers (the forward step below them
    // has nothing to push; their own forward messages and the terminal children are unchanged).
    // kWrap: these levels are the roots of their rows; the backward pass's update of them (its last
    // wave) is followed by the next iteration's forward update (nothing is stored between the two:
    // a root has no parent level, and its forward message and children stay as they are).
#pragma unroll
    for (int round = 0; round < (MODE == kTurn || MODE == kWrap ? 2 : 1); ++round) {
      if (round == 1) {
        ly.narrow_marginals(lam1);
        d = ly.m1 - ly.m0;
      }
      // the previous round's readers of s_d and s_share are past the barriers that follow
      s_d[s] = d;
      __syncthreads();
      if (active && pos == 0) {
        // J_i sum in ascending row order (the segment is sorted by row)
        float sum = 0.0f;
        int nf = 0;
        for (int q = 0; q < len; ++q) {
          const float dq = s_d[s + q];
          if (isinf(dq)) ++nf;
          else sum += dq;
        }
        s_share[s] = nf ? sum / float(nf) : sum / float(len);
        s_nf[s] = nf;
      }
      __syncthreads();
      if (active) {
        const int h = s - pos;
        lam1 = updated(lam1, d, s_share[h], s_nf[h]);
      }
      if constexpr (MODE == kWrap) {
        if (round == 0 && roots) {
          // the backward step at the roots with the updated multipliers: E^j of each row, summed per
          // wavefront into the backward tile's bound partials
          const double v = wave_sum(active ? ly.root_value(lam1) : 0.0);
          if ((threadIdx.x & 63) == 0) D.lbpart[kTile / 64 * btix + (int(threadIdx.x) >> 6)] = v;
        }
      }
    }
    if (active) D.lam[ly.L] = lam1;
  }
  if (MODE == kExtract && active) {
    const int c = D.canon_of[ly.L];
    if (D.out0) D.out0[c] = ly.m0;
    if (D.out1) D.out1[c] = ly.m1;
    D.d_fresh[ly.L] = d;
  }
  if constexpr (!NARROW_ONLY) {
    GenTile &T = s_g;
    if (gen) T.lam[myk] = lam1;
    __syncthreads();
    if (flat) {
      if (DIR == kFwd) {
        // next-level nodes over all lanes, each the minimum over its in-arcs (pull form of Alg.
        // "Forward BDD update step"), reading this level's forward messages from LDS
#pragma unroll
        for (int r = 0; r < kFlatR; ++r) {
          const int k = kc[r];
          if (k >= 0) {
            const int osc = T.osc[k];
            if (osc >= 0) {
              const int v = s + r * kTile - T.co[k], f0 = T.wo[k];
              msg_st<COH>(D.mf + osc + v, pull_min_pk(D, pkc[r], T.rb[k], v, T.lam[k], [&](int u) { return s_fu[f0 + u]; }));
            }
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < kFlatR; ++r) {
          if (r * kTile >= TW) break;
          const int k = kr[r];
          if (k >= 0) {
            const int u = s + r * kTile - T.wo[k], c0 = T.co[k], ps = T.pcs[k];
            const float v = fminf(staged(s_cb, c0, ar[r] & 0xFFFFu), staged(s_cb, c0, ar[r] >> 16) + T.lam[k]);
            if (ps >= 0) msg_st<COH>(D.mbc + ps + u, v);
            if (u == 0) T.e[k] = v;
          }
        }
      }
    } else {
      const int grp = s / G, gl = s % G, ngrp = kTile / G;
      for (int k = grp; k < ngen; k += ngrp) {
        if (DIR == kFwd) {
          group_push<COH>(D, T, k, gl, G);
        } else {
          const float r = group_bstep<COH>(D, T, k, gl, G);
          if (gl == 0) T.e[k] = r;
        }
      }
    }
    if (DIR == kBwd) __syncthreads();
  }
  if (DIR == kFwd) {
    if (active && !gen) ly.push(D, lam1);
  } else {
    double e = 0.0;
    if (active && !gen) e = ly.bstep(D, lam1);
    if constexpr (!NARROW_ONLY)
      if (gen && (ly.meta & kMetaRootBit)) e = double(s_g.e[myk]);
    // bound partial per wavefront: a fixed-shape wavefront sum, only in tiles holding root levels
    // (the branch is uniform over the workgroup); the partials of other tiles stay at the zero the
    // solver's reset stored
    if (roots) {
      const double v = wave_sum(e);
      if ((threadIdx.x & 63) == 0) D.lbpart[kTile / 64 * tix + (int(threadIdx.x) >> 6)] = v;
    }
  }
}

// One wave: a workgroup per tile, tiles tile0 .. tile0 + gridDim.x - 1 (XCD-aware order).
template <int DIR, int MODE, bool NARROW_ONLY, bool LIST>
__global__ __launch_bounds__(kTile) void wave_kernel(const Dev D, const int tile0, const int bwd_tile0) {
  __shared__ WaveLds<NARROW_ONLY> sh;
  const int k = xcd_tile(int(blockIdx.x), int(gridDim.x));
  const int tix = tile0 + k;
  const int32_t *tiles = DIR == kFwd ? D.fwd_tiles : D.bwd_tiles;
  wave_tile<DIR, MODE, NARROW_ONLY, LIST>(D, sh, tix, MODE == kWrap ? bwd_tile0 + k : tix, uint32_t(tiles[2 * tix]),
                                          uint32_t(tiles[2 * tix + 1]));
}

// LDS of the dataflow pass kernel: the general layout when the plan has general layers (its narrow
// tiles use the narrow layout in the same storage), else only the narrow one
union WaveLdsMixed {
  WaveLds<true> n;
  WaveLds<false> g;
};

// Dataflow launch of one pass in update mode (Alg. "Min-marginal averaging", the forward or the
// backward pass). Workgroups stay resident and take tiles in the pass's order (waves ascending); a
// tile waits only for the tiles that write the messages it reads (the plan's dependency lists), not
// for the whole previous wave, so independent rows and instances move on at their own pace.
//
// Tickets: the plan groups the instances (independent subproblems; one group for a single
// instance) and every tile belongs to one group, as do the tiles it waits for. Each group's tiles
// form a queue with a ticket counter of its own that hands out chunks of A.chunk consecutive tiles
// of the queue in order (one counter for all would serialise every draw on one address).
// Workgroup b starts at queue b mod n_queues and moves to the next queue when one runs dry; it
// leaves when it has found every queue dry. Progress: within a queue, a tile waits only for
// smaller tiles of the same queue, and when a chunk is drawn every smaller chunk of its queue has
// been drawn, by a workgroup that runs. So the smallest unfinished tile of a queue either runs (all
// it waits for is done, tiles of its own chunk before it included) or is still to be drawn while
// every drawn chunk of its queue is done; then the queue's workgroups are free, or left for other
// queues and come back, or others arrive as their own queues run dry. The waits thus end whatever
// the residency. Each wait is bounded all the same: past spin_limit polls the workgroup sets the
// error word and goes on, so the kernel always exits.
//
// Publication, per tile: the messages other tiles read are written and read with coherent
// agent-scope accesses (msg_ld / msg_st), so no cache holds a stale copy of them and no cache
// write-back or invalidation is needed. The workgroup waits until its own stores are complete
// (vmcnt 0), then one lane stores the launch's generation to the tile's flag; a waiting workgroup
// polls the flags with coherent loads, and its lanes read the messages only after the barrier that
// follows the polls. Flags hold the generation of the launch that finished them (never reset, so a
// launch never mistakes an older launch's flag for its own); the last workgroup to leave resets the
// counters and advances the generation for the next launch of the pass.
//
// Tile records (32 bytes each): start word, end word, info (bit 0 narrow, bit 1 listed, bits 2-3
// priority, bits 8-16 dependency count), offset of the dependency list, then up to four
// dependencies inline (a tile with more reads them from the list).

// wave issue priority 0..3 (s_setprio takes an immediate)
__device__ __forceinline__ void set_priority(uint32_t p) {
  switch (p) {
    case 0: __builtin_amdgcn_s_setprio(0); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    default: __builtin_amdgcn_s_setprio(3); break;
  }
}

// Wait until the flags of the tiles tile record (ra, rb) depends on hold gen: the first wavefront's
// lanes poll them with coherent loads, each at most spin_limit times (past it the error word is set
// and the wait ends); then the workgroup's barrier, after which its lanes read the messages with
// coherent loads (no cache holds a stale copy for them to hit).
// one wavefront polls a tile's dependencies (lane: its lane index): each lane waits for every 64th
// flag until it holds gen, or sets the error word past spin_limit polls of one flag
__device__ __forceinline__ void poll_deps(const int4 ra, const int4 rb, const int32_t *dep_list, const uint32_t *flags,
                                          uint32_t gen, uint32_t spin_limit, uint32_t *err, int lane) {
  const int nd = int((uint32_t(ra.z) >> 8) & 0x1FFu);
  for (int e = lane; e < nd; e += 64) {
    const int u = nd <= 4 ? (e == 0 ? rb.x : (e == 1 ? rb.y : (e == 2 ? rb.z : rb.w))) : dep_list[ra.w + e];
    const uint32_t *f = flags + u;
    uint32_t spins = 0u;
    while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != gen) {
      if (++spins > spin_limit) {
        atomicOr(err, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
}

__device__ __forceinline__ void wait_deps(const int4 ra, const int4 rb, const int32_t *dep_list, const uint32_t *flags,
                                          uint32_t gen, uint32_t spin_limit, uint32_t *err) {
  const int nd = int((uint32_t(ra.z) >> 8) & 0x1FFu);
  if (!nd) return;
  const int s = int(threadIdx.x);
  if (s < 64) poll_deps(ra, rb, dep_list, flags, gen, spin_limit, err, s);
  __syncthreads();
}

// wait_deps for one tile as a callable (on: whether the tile waits at all)
struct DepWait {
  int4 ra, rb;
  const int32_t *dep_list;
  const uint32_t *flags;
  uint32_t gen, spin_limit;
  uint32_t *err;
  bool on;
  __device__ __forceinline__ void operator()() const {
    if (on) wait_deps(ra, rb, dep_list, flags, gen, spin_limit, err);
  }
};

template <int DIR, bool NARROW_PLAN>
__global__ __launch_bounds__(kTile) __attribute__((amdgpu_waves_per_eu(NARROW_PLAN ? 8 : 6)))
void pass_kernel(const Dev D, const PassArgs A) {
  __shared__ std::conditional_t<NARROW_PLAN, WaveLds<true>, WaveLdsMixed> sh;
  __shared__ int s_next;
  const int s = int(threadIdx.x);
  const uint32_t gen = A.ctl[kPassGen] + 1u;
  int q = int(blockIdx.x) % A.n_queues, tried = 1;
  auto counter = [&](int qq) { return A.ctl + kPassQueue0 + kPassQueueStride * qq; };
  if (s == 0) s_next = int(atomicAdd(counter(q), 1u));
  __syncthreads();
  int k = s_next;
  for (;;) {
    int q0 = A.qptr[q], qn = A.qptr[q + 1] - q0;
    // a dry queue: move on to the next one, leave once every queue was found dry
    while (k * A.chunk >= qn) {
      if (tried == A.n_queues) break;
      q = q + 1 == A.n_queues ? 0 : q + 1;
      ++tried;
      __syncthreads();
      if (s == 0) s_next = int(atomicAdd(counter(q), 1u));
      __syncthreads();
      k = s_next;
      q0 = A.qptr[q];
      qn = A.qptr[q + 1] - q0;
    }
    if (k * A.chunk >= qn) break;
    // the next chunk of this queue is drawn now and read after this one (both drawn in order, so
    // the argument above still holds)
    int nxt = 0;
    if (s == 0) nxt = int(atomicAdd(counter(q), 1u));
    const int j1 = min(qn, (k + 1) * A.chunk);
    for (int j = k * A.chunk; j < j1; ++j) {
      const int t = A.qtile[q0 + j];
      const int4 ra = A.trec[2 * t], rb = A.trec[2 * t + 1];
      const uint32_t info = uint32_t(ra.z);
      const bool list = (info & 2u) != 0u;
      set_priority((info >> 2) & 3u);
      const DepWait dw{ra, rb, A.dep_list, A.flags, gen, A.spin_limit, A.ctl + kPassErr, true};
      if constexpr (NARROW_PLAN) {
        wave_tile<DIR, kUpdate, true, DIR == kBwd, true>(D, sh, t, t, uint32_t(ra.x), uint32_t(ra.y), list, dw);
      } else if (info & 1u) {
        wave_tile<DIR, kUpdate, true, DIR == kBwd, true>(D, sh.n, t, t, uint32_t(ra.x), uint32_t(ra.y), list, dw);
      } else {
        wave_tile<DIR, kUpdate, false, DIR == kBwd, true>(D, sh.g, t, t, uint32_t(ra.x), uint32_t(ra.y), list, dw);
      }
      // every lane's coherent message stores of the tile complete (vmcnt 0; expcnt and lgkmcnt at
      // their maximum) before one lane stores the tile's flag; the barrier also frees the LDS
      __builtin_amdgcn_s_waitcnt(0x0F70);
      __syncthreads();
      if (s == 0) __hip_atomic_store(A.flags + t, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (s == 0) s_next = nxt;
    __syncthreads();
    k = s_next;
  }
  if (s == 0) {
    const uint32_t gone = __hip_atomic_fetch_add(A.ctl + kPassGone, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (gone == gridDim.x - 1u) {
      for (int qq = 0; qq < A.n_queues; ++qq) __hip_atomic_store(counter(qq), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(A.ctl + kPassGone, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(A.ctl + kPassGen, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Several consecutive waves of an update pass in one launch (Alg. "Min-marginal averaging", part of
// the forward or the backward pass), one workgroup per tile, in pass order: the waves' tiles are
// consecutive, so workgroup b runs tile t0 + b, and consecutive tiles go to consecutive XCDs (every
// XCD takes each wave's tiles from its start; measured faster here than the contiguous runs per XCD
// of the wave launches). The tiles of the launch's first wave read only what earlier launches
// wrote; those of a later wave first wait for the flags of the tiles they read from (the plan's
// dependency lists).
//
// Progress: each XCD receives every eighth workgroup and dispatches its workgroups in block order,
// so on every XCD all workgroups of a wave are dispatched before any of the next wave. A workgroup
// waits only for tiles of earlier waves. By induction over the launch's waves: the first wave never
// waits; when every tile of waves before i finishes, a workgroup of wave i either runs or waits for
// one of them, and an XCD whose compute units are full of waiting workgroups of wave i has
// dispatched all of its own earlier-wave workgroups, which finish. Each wait is bounded all the same
// (error word, then the workgroup goes on), so the kernel always exits.
//
// Publication: a tile's messages are written and read with coherent agent-scope accesses (msg_ld /
// msg_st). A tile of a wave that later waves of the launch may read waits until its stores are
// complete (vmcnt 0) before one lane stores the flag; a tile of the launch's last wave stores its
// flag at once (its readers run in later launches, after this one has ended).
template <int DIR, bool NARROW_PLAN>
__global__ __launch_bounds__(kTile) __attribute__((amdgpu_waves_per_eu(NARROW_PLAN ? 8 : 6)))
void group_kernel(const Dev D, const GroupArgs A) {
  __shared__ std::conditional_t<NARROW_PLAN, WaveLds<true>, WaveLdsMixed> sh;
  const int s = int(threadIdx.x);
  const int t = A.t0 + int(blockIdx.x);
  const uint32_t gen = uint32_t(*D.hist_n) | 0x80000000u;
  const int4 ra = A.trec[2 * t], rb = A.trec[2 * t + 1];
  const uint32_t info = uint32_t(ra.z);
  const bool list = (info & 2u) != 0u;
  // the tile issues what no tile of this pass writes (and scans its widths) before it waits
  const DepWait dw{ra, rb, A.dep_list, A.flags, gen, A.spin_limit, A.ctl + kPassErr, t >= A.t_first};
  if constexpr (NARROW_PLAN) {
    wave_tile<DIR, kUpdate, true, DIR == kBwd, true>(D, sh, t, t, uint32_t(ra.x), uint32_t(ra.y), list, dw);
  } else if (info & 1u) {
    wave_tile<DIR, kUpdate, true, DIR == kBwd, true>(D, sh.n, t, t, uint32_t(ra.x), uint32_t(ra.y), list, dw);
  } else {
    wave_tile<DIR, kUpdate, false, DIR == kBwd, true>(D, sh.g, t, t, uint32_t(ra.x), uint32_t(ra.y), list, dw);
  }
  if (t < A.t_last) {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
  }
  if (s == 0) __hip_atomic_store(A.flags + t, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-group launch of a plan whose layers are all narrow, two tiles per workgroup: tiles
// a = t0 + 2 * block and a + 1 (when inside the launch), lane s holding layer s of both, so that
// both tiles' fixed loads, dependency polls and message loads are in flight together and a
// workgroup keeps twice the loads of the one-tile form outstanding. Each layer's arithmetic is that
// of the one-tile form (the same J_i sum order, update, forward push or backward step, bound
// partials per tile and wavefront), so the results are bitwise the same.
//
// When tile a + 1 reads messages tile a writes (the two lie in consecutive waves, and a is then the
// last of its ascending dependency list), the workgroup runs tile a, publishes it, then runs tile
// a + 1, each in the one-tile form. Progress as for group_kernel: the workgroups take the pairs in
// pass order, and a pair waits only for tiles of earlier pairs, or for its own first tile once that
// tile is published.
template <int DIR>
__global__ __launch_bounds__(kTile) __attribute__((amdgpu_waves_per_eu(8)))
void group_pair_kernel(const Dev D, const GroupArgs A) {
  __shared__ WaveLds<true> sh;
  __shared__ float p_d[2][kTile], p_share[2][kTile];
  __shared__ int p_nf[2][kTile];
  const int s = int(threadIdx.x);
  const int ta = A.t0 + 2 * int(blockIdx.x);
  const bool two = ta + 1 < A.t_end;
  const int tb = two ? ta + 1 : ta;
  const uint32_t gen = uint32_t(*D.hist_n) | 0x80000000u;
  const int4 ra[2] = {A.trec[2 * ta], A.trec[2 * tb]};
  const int4 rb[2] = {A.trec[2 * ta + 1], A.trec[2 * tb + 1]};
  const int ndb = int((uint32_t(ra[1].z) >> 8) & 0x1FFu);
  int last_b = -1;
  if (two && tb >= A.t_first && ndb > 0)
    last_b = ndb <= 4 ? (ndb == 1 ? rb[1].x : (ndb == 2 ? rb[1].y : (ndb == 3 ? rb[1].z : rb[1].w)))
                      : A.dep_list[ra[1].w + ndb - 1];
  if (last_b == ta) {
    // tile a + 1 waits for tile a: one after the other (tile a lies before the launch's last wave,
    // so its publication below ends with the barrier that also frees the LDS for tile a + 1)
    for (int k = 0; k < 2; ++k) {
      const int t = ta + k;
      const DepWait dw{ra[k], rb[k], A.dep_list, A.flags, gen, A.spin_limit, A.ctl + kPassErr, t >= A.t_first};
      wave_tile<DIR, kUpdate, true, DIR == kBwd, true>(D, sh, t, t, uint32_t(ra[k].x), uint32_t(ra[k].y),
                                                       (uint32_t(ra[k].z) & 2u) != 0u, dw);
      if (t < A.t_last) {
        __builtin_amdgcn_s_waitcnt(0x0F70);
        __syncthreads();
      }
      if (s == 0) __hip_atomic_store(A.flags + t, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  Layer<DIR, true, false, true> ly[2];
  bool act[2], roots[2];
  int lay[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const uint32_t w0 = uint32_t(ra[k].x), end = uint32_t(ra[k].y);
    const int p0 = int(w0 & kTilePosMask);
    const bool real = k == 0 || two;
    roots[k] = real && DIR == kBwd && (end & kTileRootBit) != 0u;
    act[k] = real && s < int(end & ~kTileRootBit) - p0;
    // every lane loads (a lane past the tile's layers reads its first one and keeps nothing), so
    // no branch separates the two tiles' loads
    const int q = p0 + (act[k] ? s : 0);
    const bool list = (uint32_t(ra[k].z) & 2u) != 0u;
    lay[k] = (DIR == kBwd && list) ? D.bwd_list[q] : q;
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) ly[k].begin_fixed(D, lay[k]);
  // wavefront 0 polls tile a's dependencies, wavefront 1 tile a + 1's, then one barrier
  {
    const int k = s >> 6;
    if (k < 2 && (k == 0 || two) && ta + k >= A.t_first)
      poll_deps(k ? ra[1] : ra[0], k ? rb[1] : rb[0], A.dep_list, A.flags, gen, A.spin_limit, A.ctl + kPassErr, s & 63);
    __syncthreads();
  }
  // both tiles' messages of this pass in flight together, then their min-marginals
  float2 pm[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) pm[k] = msg_ld2<true>((DIR == kFwd ? D.mf : D.mbc) + 2 * ly[k].L);
  float d[2], lam1[2];
  int pos[2], len[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (DIR == kFwd) ly[k].f = pm[k];
    else ly[k].b = pm[k];
    ly[k].narrow_marginals(ly[k].lam0);
    d[k] = act[k] ? ly[k].m1 - ly[k].m0 : 0.0f;
    lam1[k] = ly[k].lam0;
    pos[k] = int((ly[k].meta >> kMetaPosShift) & kMetaField);
    len[k] = int((ly[k].meta >> kMetaLenShift) & kMetaField);
    p_d[k][s] = d[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 2; ++k)
    if (act[k] && pos[k] == 0) {
      // J_i sum in ascending row order (the segment is sorted by row)
      float sum = 0.0f;
      int nf = 0;
      for (int q = 0; q < len[k]; ++q) {
        const float dq = p_d[k][s + q];
        if (isinf(dq)) ++nf;
        else sum += dq;
      }
      p_share[k][s] = nf ? sum / float(nf) : sum / float(len[k]);
      p_nf[k][s] = nf;
    }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (act[k]) {
      const int h = s - pos[k];
      lam1[k] = updated(lam1[k], d[k], p_share[k][h], p_nf[k][h]);
      D.lam[ly[k].L] = lam1[k];
    }
    if (DIR == kFwd) {
      if (act[k]) ly[k].push(D, lam1[k]);
    } else {
      const double e = act[k] ? ly[k].bstep(D, lam1[k]) : 0.0;
      if (roots[k]) {
        const double v = wave_sum(e);
        if ((s & 63) == 0) D.lbpart[kTile / 64 * (ta + k) + (s >> 6)] = v;
      }
    }
  }
  if (ta < A.t_last) {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
  }
  if (s == 0) {
    __hip_atomic_store(A.flags + ta, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (two) __hip_atomic_store(A.flags + tb, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One variable with more than kTile rows per workgroup (its layers are the whole tile).
template <int DIR, int MODE, bool LIST>
__global__ __launch_bounds__(kTile) void wave_big_kernel(const Dev D, const int big0) {
  __shared__ float s_d[kBigMax];
  __shared__ float s_share;
  __shared__ int s_nf;
  __shared__ double s_red[kTile / 64];
  const int32_t *big = DIR == kFwd ? D.fwd_big : D.bwd_big;
  const int b = big0 + int(blockIdx.x);
  const int p0 = big[2 * b];
  const int cnt = big[2 * b + 1] - p0;
  for (int s = int(threadIdx.x); s < cnt; s += kTile) {
    Layer<DIR, false, true> ly;
    ly.begin(D, (DIR == kBwd && LIST) ? D.bwd_list[p0 + s] : p0 + s);
    s_d[s] = ly.m1 - ly.m0;
    if (MODE == kExtract) {
      const int c = D.canon_of[ly.L];
      if (D.out0) D.out0[c] = ly.m0;
      if (D.out1) D.out1[c] = ly.m1;
      D.d_fresh[ly.L] = ly.m1 - ly.m0;
    }
  }
  if (MODE == kUpdate) {
    __syncthreads();
    if (threadIdx.x == 0) {
      float sum = 0.0f;
      int nf = 0;
      for (int q = 0; q < cnt; ++q) {
        if (isinf(s_d[q])) ++nf;
        else sum += s_d[q];
      }
      s_share = nf ? sum / float(nf) : sum / float(cnt);
      s_nf = nf;
    }
    __syncthreads();
  }
  double e = 0.0;
  for (int s = int(threadIdx.x); s < cnt; s += kTile) {
    Layer<DIR, false, true> ly;
    ly.begin(D, (DIR == kBwd && LIST) ? D.bwd_list[p0 + s] : p0 + s);
    float lam1 = ly.lam0;
    if (MODE == kUpdate) {
      lam1 = updated(lam1, s_d[s], s_share, s_nf);
      D.lam[ly.L] = lam1;
    }
    if (DIR == kFwd) ly.push(D, lam1);
    else e += ly.bstep(D, lam1);
  }
  if (DIR == kBwd) {
    const double t = block_sum(e, s_red);
    if (threadIdx.x == 0) D.lbpart[kTile / 64 * D.n_bwd_tiles + b] = t;
  }
}

__global__ void fill_kernel(float *p, float v, int n) {
  const int i = int(blockIdx.x) * blockDim.x + int(threadIdx.x);
  if (i < n) p[i] = v;
}

__global__ void init_lambda_kernel(const Dev D, int I) {
  const int L = int(blockIdx.x) * blockDim.x + int(threadIdx.x);
  if (L >= I) return;
  const int v = D.layer_var[L];
  D.lam[L] = float(D.cost[v] / double(D.var_nj[v]));
}

__global__ void root_zero_kernel(const Dev D, int m) {
  const int j = int(blockIdx.x) * blockDim.x + int(threadIdx.x);
  if (j >= m) return;
  const int r = D.root_slot[j];
  if (r >= 0) D.mf[r] = 0.0f;
}

__global__ void lambda_out_kernel(const Dev D, float *out, int I) {
  const int L = int(blockIdx.x) * blockDim.x + int(threadIdx.x);
  if (L < I) out[D.canon_of[L]] = D.lam[L];
}

__global__ void lambda_in_kernel(const Dev D, const float *in, int I) {
  const int L = int(blockIdx.x) * blockDim.x + int(threadIdx.x);
  if (L < I) D.lam[L] = in[D.canon_of[L]];
}

__global__ void flag_clear_kernel(const Dev D) {
  if (threadIdx.x == 0) *D.flag = 0u;
}

template <class T>
__global__ __launch_bounds__(256) void nonfinite_kernel(const Dev D, const T *p, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * 256;
  bool bad = false;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) bad |= !isfinite(p[i]);
  if (bad) atomicOr(D.flag, 1u);
}

// LB = sum_j E^j (problem (D)) from the per-tile partials of the backward sweep: kLbStage blocks
// each sum one fixed contiguous chunk, then one block sums the chunk totals; fixed order throughout
__global__ __launch_bounds__(256) void lb_stage_kernel(const Dev D, int nparts) {
  __shared__ double sh[4];
  const int chunk = (nparts + kLbStage - 1) / kLbStage;
  const int q0 = int(blockIdx.x) * chunk, q1 = min(nparts, q0 + chunk);
  // four independent running sums per lane (loads in flight together), then combined in order
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int q = q0 + int(threadIdx.x);
  for (; q + 3 * 256 < q1; q += 4 * 256) {
    a0 += D.lbpart[q];
    a1 += D.lbpart[q + 256];
    a2 += D.lbpart[q + 2 * 256];
    a3 += D.lbpart[q + 3 * 256];
  }
  for (; q < q1; q += 256) a0 += D.lbpart[q];
  const double s = block_sum((a0 + a1) + (a2 + a3), sh);
  if (threadIdx.x == 0) D.part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kLbStage) void lb_final_kernel(const Dev D, int which) {
  __shared__ double sh[kLbStage / 64];
  const long long n = *D.hist_n;
  const double c = D.lbc[which];
  const double s = block_sum(D.part[threadIdx.x], sh);
  if (threadIdx.x == 0) {
    D.lb_hist[n % D.hist_cap] = s + c;
    *D.hist_n = n + 1;
  }
}

__global__ void set_counter_kernel(const Dev D, long long value) {
  if (threadIdx.x == 0) *D.hist_n = value;
}

// E^j of each row from the state a backward sweep leaves: the root level's backward message
// (Alg. "Backward BDD update step" at the root, the same operations as in the sweep, so the value
// is bitwise the one the sweep produced). One workgroup per instance sums its rows in a fixed shape.
__global__ __launch_bounds__(256) void instance_bound_kernel(const Dev D) {
  __shared__ double sh[4];
  const int k = int(blockIdx.x);
  const int j0 = D.inst_row[k], j1 = D.inst_row[k + 1];
  double acc = 0.0;
  for (int j = j0 + int(threadIdx.x); j < j1; j += 256) {
    const int c0 = D.bdd_canon_off[j];
    if (c0 == D.bdd_canon_off[j + 1]) continue;
    const int L = D.layer_of[c0];
    const uint32_t meta = D.meta[L];
    const float lam = D.lam[L];
    float e;
    if (((meta >> kMetaWidthShift) & 3u) != 0u) {
      const float2 b = reinterpret_cast<const float2 *>(D.mbc)[L];
      e = fminf(c2val(meta & 3u, b), c2val((meta >> 2) & 3u, b) + lam);
    } else {
      const int4 g = D.grec[L];
      const uint32_t a = D.garcs[g.x];
      e = fminf(c16val(D.mbc, g.y, a & 0xFFFFu), c16val(D.mbc, g.y, a >> 16) + lam);
    }
    acc += double(e);
  }
  // the sub-BDDs after the instance's cuts (Sec. 6), as the last backward copy update left them
  for (int q = D.inst_cut[k] + int(threadIdx.x); q < D.inst_cut[k + 1]; q += 256) acc += double(D.cut_e[D.inst_cut_idx[q]]);
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) D.inst_lb[k] = t;
}

// per variable: g_i = c_i - sum_j lambda^j_i; partial max |g| and sum of min(0, g)
__global__ __launch_bounds__(256) void residual_partial_kernel(const Dev D, int n) {
  __shared__ double sh[4];
  __shared__ double smax[256];
  const int chunk = (n + kLbBlocks - 1) / kLbBlocks;
  const int i0 = int(blockIdx.x) * chunk, i1 = min(n, i0 + chunk);
  double mx = 0.0, corr = 0.0;
  for (int i = i0 + int(threadIdx.x); i < i1; i += 256) {
    const int nj = D.var_nj[i];
    if (!nj) continue;
    const int f0 = D.var_first[i];
    double s = 0.0;
    for (int q = 0; q < nj; ++q) s += double(D.lam[f0 + q]);
    const double g = D.cost[i] - s;
    mx = fmax(mx, fabs(g));
    corr += fmin(0.0, g);
  }
  smax[threadIdx.x] = mx;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + st]);
    __syncthreads();
  }
  const double b = block_sum(corr, sh);
  if (threadIdx.x == 0) {
    D.part[blockIdx.x] = smax[0];
    D.part[kLbBlocks + blockIdx.x] = b;
  }
}

__global__ __launch_bounds__(kLbBlocks) void residual_final_kernel(const Dev D) {
  __shared__ double sa[kLbBlocks];
  __shared__ double sh[kLbBlocks / 64];
  const int t = int(threadIdx.x);
  sa[t] = D.part[t];
  __syncthreads();
  for (int st = kLbBlocks / 2; st > 0; st >>= 1) {
    if (t < st) sa[t] = fmax(sa[t], sa[t + st]);
    __syncthreads();
  }
  const double b = block_sum(D.part[kLbBlocks + t], sh);
  if (t == 0) {
    D.scal[0] = sa[0];
    D.scal[1] = b;
  }
}

// M_i = sum_j (m1 - m0) in ascending row order (Sec. 4), x_i = [M_i <= 0]; c^T x partials
__global__ __launch_bounds__(256) void round_var_kernel(const Dev D, int n) {
  __shared__ double sh[4];
  const int chunk = (n + kLbBlocks - 1) / kLbBlocks;
  const int i0 = int(blockIdx.x) * chunk, i1 = min(n, i0 + chunk);
  double obj = 0.0;
  for (int i = i0 + int(threadIdx.x); i < i1; i += 256) {
    const int nj = D.var_nj[i];
    float M = 0.0f;
    int8_t x;
    if (nj) {
      const int f0 = D.var_first[i];
      for (int q = 0; q < nj; ++q) M += D.d_fresh[f0 + q];
      x = M <= 0.0f ? 1 : 0;
    } else {
      x = D.cost[i] < 0.0 ? 1 : 0;
    }
    D.mbuf[i] = M;
    D.xbuf[i] = x;
    if (x) obj += D.cost[i];
  }
  const double s = block_sum(obj, sh);
  if (threadIdx.x == 0) D.part[blockIdx.x] = s;
}

// a row holds at x iff x's path through its BDD ends in the true terminal (Prop. "Canonicity")
__global__ __launch_bounds__(256) void violation_kernel(const Dev D, int m) {
  __shared__ double sh[4];
  const int chunk = (m + kLbBlocks - 1) / kLbBlocks;
  const int j0 = int(blockIdx.x) * chunk, j1 = min(m, j0 + chunk);
  double bad = 0.0;
  for (int j = j0 + int(threadIdx.x); j < j1; j += 256) {
    const int c0 = D.bdd_canon_off[j], c1 = D.bdd_canon_off[j + 1];
    int slot = D.root_slot[j];
    for (int c = c0; c < c1; ++c) {
      const int L = D.layer_of[c];
      const uint32_t a = D.garcs[slot];
      uint32_t ch = D.xbuf[D.layer_var[L]] ? (a >> 16) : (a & 0xFFFFu);
      // an exit layer of a split codes its live arcs by their copy-arc slot: back to the child
      if (D.exit_rec && ch < kTop) {
        const int r = D.exit_rec[L];
        if (r >= 0) ch = D.cut_arc[D.cuts[r].z + int(ch)];
      }
      if (ch == kBot) {
        bad += 1.0;
        break;
      }
      if (ch == kTop) break;
      const int Lc = D.layer_of[c + 1];
      slot = (D.grec ? D.grec[Lc].x : 2 * Lc) + int(ch);
    }
  }
  const double s = block_sum(bad, sh);
  if (threadIdx.x == 0) D.part[kLbBlocks + blockIdx.x] = s;
}

__global__ __launch_bounds__(kLbBlocks) void round_final_kernel(const Dev D) {
  __shared__ double sh[kLbBlocks / 64];
  const int t = int(threadIdx.x);
  const double a = block_sum(D.part[t], sh);
  const double b = block_sum(D.part[kLbBlocks + t], sh);
  if (t == 0) {
    D.scal[2] = a;
    D.scal[3] = b;
  }
}

int blocks_for(int64_t count, int per) { return int((count + per - 1) / per); }

}  // namespace

// ---------------------------------------------------------------------------------------------
// launch functions
// ---------------------------------------------------------------------------------------------

template <int DIR, int MODE>
static hipError_t wave_dispatch(bool narrow_only, bool list, int nt, int tile0, const Dev &D, hipStream_t s) {
  if (narrow_only && !list)
    hipLaunchKernelGGL((wave_kernel<DIR, MODE, true, false>), dim3(nt), dim3(kTile), 0, s, D, tile0, 0);
  else if (narrow_only)
    hipLaunchKernelGGL((wave_kernel<DIR, MODE, true, true>), dim3(nt), dim3(kTile), 0, s, D, tile0, 0);
  else if (!list)
    hipLaunchKernelGGL((wave_kernel<DIR, MODE, false, false>), dim3(nt), dim3(kTile), 0, s, D, tile0, 0);
  else
    hipLaunchKernelGGL((wave_kernel<DIR, MODE, false, true>), dim3(nt), dim3(kTile), 0, s, D, tile0, 0);
  return hipGetLastError();
}

hipError_t launch_wave(int dir, int mode, bool narrow_only, bool list, int nt, int tile0, const Dev &D,
                       hipStream_t s, int bwd_tile0) {
  if (dir == kFwd && mode == kUpdate) return wave_dispatch<kFwd, kUpdate>(narrow_only, false, nt, tile0, D, s);
  if (dir == kFwd && mode == kExtract) return wave_dispatch<kFwd, kExtract>(narrow_only, false, nt, tile0, D, s);
  if (dir == kBwd && mode == kUpdate) return wave_dispatch<kBwd, kUpdate>(narrow_only, list, nt, tile0, D, s);
  if (dir == kBwd && mode == kNoUpdate) return wave_dispatch<kBwd, kNoUpdate>(narrow_only, list, nt, tile0, D, s);
  if (dir == kBwd && mode == kTurn) {
    if (!narrow_only || list) return hipErrorInvalidValue;
    hipLaunchKernelGGL((wave_kernel<kBwd, kTurn, true, false>), dim3(nt), dim3(kTile), 0, s, D, tile0, 0);
    return hipGetLastError();
  }
  if (dir == kFwd && mode == kWrap) {
    if (!narrow_only || list) return hipErrorInvalidValue;
    hipLaunchKernelGGL((wave_kernel<kFwd, kWrap, true, false>), dim3(nt), dim3(kTile), 0, s, D, tile0, bwd_tile0);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

template <int DIR, bool NARROW_PLAN>
static hipError_t pass_dispatch(int grid, const Dev &D, const PassArgs &A, hipStream_t s) {
  hipLaunchKernelGGL((pass_kernel<DIR, NARROW_PLAN>), dim3(grid), dim3(kTile), 0, s, D, A);
  return hipGetLastError();
}

hipError_t launch_pass(int dir, bool narrow_plan, int grid, const Dev &D, const PassArgs &A, hipStream_t s) {
  if (grid <= 0 || A.n_tiles <= 0) return hipSuccess;
  if (dir == kFwd) return narrow_plan ? pass_dispatch<kFwd, true>(grid, D, A, s) : pass_dispatch<kFwd, false>(grid, D, A, s);
  return narrow_plan ? pass_dispatch<kBwd, true>(grid, D, A, s) : pass_dispatch<kBwd, false>(grid, D, A, s);
}

hipError_t pass_blocks_per_cu(int dir, bool narrow_plan, int *blocks) {
  const void *fn = dir == kFwd ? (narrow_plan ? reinterpret_cast<const void *>(pass_kernel<kFwd, true>)
                                              : reinterpret_cast<const void *>(pass_kernel<kFwd, false>))
                               : (narrow_plan ? reinterpret_cast<const void *>(pass_kernel<kBwd, true>)
                                              : reinterpret_cast<const void *>(pass_kernel<kBwd, false>));
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, kTile, 0);
}

template <int DIR, bool NARROW_PLAN>
static hipError_t group_dispatch(const Dev &D, const GroupArgs &A, hipStream_t s) {
  hipLaunchKernelGGL((group_kernel<DIR, NARROW_PLAN>), dim3(A.t_end - A.t0), dim3(kTile), 0, s, D, A);
  return hipGetLastError();
}

template <int DIR>
static hipError_t group_pair_dispatch(const Dev &D, const GroupArgs &A, hipStream_t s) {
  hipLaunchKernelGGL((group_pair_kernel<DIR>), dim3((A.t_end - A.t0 + 1) / 2), dim3(kTile), 0, s, D, A);
  return hipGetLastError();
}

hipError_t launch_group(int dir, bool narrow_plan, bool pairs, const Dev &D, const GroupArgs &A, hipStream_t s) {
  // t0 <= t_first <= t_end and t0 <= t_last <= t_end (t_last = t0 when the launch holds one wave);
  // two tiles per workgroup only where every layer is narrow
  if (A.t0 < 0 || A.t_first < A.t0 || A.t_end < A.t_first || A.t_last < A.t0 || A.t_end < A.t_last ||
      (pairs && !narrow_plan))
    return hipErrorInvalidValue;
  if (A.t_end <= A.t0) return hipSuccess;
  if (pairs) return dir == kFwd ? group_pair_dispatch<kFwd>(D, A, s) : group_pair_dispatch<kBwd>(D, A, s);
  if (dir == kFwd) return narrow_plan ? group_dispatch<kFwd, true>(D, A, s) : group_dispatch<kFwd, false>(D, A, s);
  return narrow_plan ? group_dispatch<kBwd, true>(D, A, s) : group_dispatch<kBwd, false>(D, A, s);
}

template <int DIR, int MODE>
static hipError_t big_dispatch(bool list, int nb, int big0, const Dev &D, hipStream_t s) {
  if (list)
    hipLaunchKernelGGL((wave_big_kernel<DIR, MODE, true>), dim3(nb), dim3(kTile), 0, s, D, big0);
  else
    hipLaunchKernelGGL((wave_big_kernel<DIR, MODE, false>), dim3(nb), dim3(kTile), 0, s, D, big0);
  return hipGetLastError();
}

hipError_t launch_wave_big(int dir, int mode, bool list, int nb, int big0, const Dev &D, hipStream_t s) {
  if (dir == kFwd && mode == kUpdate) return big_dispatch<kFwd, kUpdate>(false, nb, big0, D, s);
  if (dir == kFwd && mode == kExtract) return big_dispatch<kFwd, kExtract>(false, nb, big0, D, s);
  if (dir == kBwd && mode == kUpdate) return big_dispatch<kBwd, kUpdate>(list, nb, big0, D, s);
  if (dir == kBwd && mode == kNoUpdate) return big_dispatch<kBwd, kNoUpdate>(list, nb, big0, D, s);
  return hipErrorInvalidValue;
}

hipError_t launch_fill(float *p, float v, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_init_lambda(const Dev &D, int I, hipStream_t s) {
  if (I <= 0) return hipSuccess;
  hipLaunchKernelGGL(init_lambda_kernel, dim3(blocks_for(I, 256)), dim3(256), 0, s, D, I);
  return hipGetLastError();
}

hipError_t launch_root_zero(const Dev &D, int m, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(root_zero_kernel, dim3(blocks_for(m, 256)), dim3(256), 0, s, D, m);
  return hipGetLastError();
}

hipError_t launch_lambda_out(const Dev &D, float *out, int I, hipStream_t s) {
  if (I <= 0) return hipSuccess;
  hipLaunchKernelGGL(lambda_out_kernel, dim3(blocks_for(I, 256)), dim3(256), 0, s, D, out, I);
  return hipGetLastError();
}

hipError_t launch_lambda_in(const Dev &D, const float *in, int I, hipStream_t s) {
  if (I <= 0) return hipSuccess;
  hipLaunchKernelGGL(lambda_in_kernel, dim3(blocks_for(I, 256)), dim3(256), 0, s, D, in, I);
  return hipGetLastError();
}

hipError_t launch_flag_clear(const Dev &D, hipStream_t s) {
  hipLaunchKernelGGL(flag_clear_kernel, dim3(1), dim3(64), 0, s, D);
  return hipGetLastError();
}

template <class T>
static hipError_t nonfinite_dispatch(const Dev &D, const T *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = int(std::min<int64_t>((n + 255) / 256, 4096));
  hipLaunchKernelGGL(nonfinite_kernel<T>, dim3(blocks), dim3(256), 0, s, D, p, n);
  return hipGetLastError();
}
hipError_t launch_nonfinite(const Dev &D, const float *p, int64_t n, hipStream_t s) {
  return nonfinite_dispatch(D, p, n, s);
}
hipError_t launch_nonfinite(const Dev &D, const double *p, int64_t n, hipStream_t s) {
  return nonfinite_dispatch(D, p, n, s);
}

hipError_t launch_lb(const Dev &D, int nparts, int which, hipStream_t s) {
  hipLaunchKernelGGL(lb_stage_kernel, dim3(kLbStage), dim3(256), 0, s, D, nparts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lb_final_kernel, dim3(1), dim3(kLbStage), 0, s, D, which);
  return hipGetLastError();
}

hipError_t launch_set_counter(const Dev &D, long long value, hipStream_t s) {
  hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(64), 0, s, D, value);
  return hipGetLastError();
}

hipError_t launch_instance_bounds(const Dev &D, int n_inst, hipStream_t s) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(instance_bound_kernel, dim3(n_inst), dim3(256), 0, s, D);
  return hipGetLastError();
}

hipError_t launch_residual(const Dev &D, int n, hipStream_t s) {
  hipLaunchKernelGGL(residual_partial_kernel, dim3(kLbBlocks), dim3(256), 0, s, D, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(residual_final_kernel, dim3(1), dim3(kLbBlocks), 0, s, D);
  return hipGetLastError();
}

// both partial kernels write every partial slot, also for empty inputs
hipError_t launch_round(const Dev &D, int n, int m, hipStream_t s) {
  hipLaunchKernelGGL(round_var_kernel, dim3(kLbBlocks), dim3(256), 0, s, D, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(violation_kernel, dim3(kLbBlocks), dim3(256), 0, s, D, m);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(round_final_kernel, dim3(1), dim3(kLbBlocks), 0, s, D);
  return hipGetLastError();
}

}  // namespace bddmp
