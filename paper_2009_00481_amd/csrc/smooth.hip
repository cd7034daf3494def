// Smoothed variant (App. "Smoothing") of the wave kernels, and the adjoint kernels that give the
// derivative of the smoothed bound with respect to the costs.
//
// The smoothed passes run the same schedule as the min-plus ones with min replaced by the soft
// minimum smin(a, b) = -alpha log(exp(-a/alpha) + exp(-b/alpha)) in every forward step, backward
// step and marginal (the marginal log-sum-exp algebra of Table "algebras" in the log domain). One
// lane handles one layer; general layers loop over their nodes. Several arguments fold left in the
// order node 0, 1, ... and 0-arc before 1-arc.
//
// The adjoint kernels undo one pass, wave by wave in reverse order. They recompute every value
// the pass produced from the values it read (bitwise the same operations), and pass adjoints back
// through the soft-minimum weights exp(-(argument - result)/alpha), the derivatives of smin.
// Adjoint arrays: glam per layer, gmf in the forward-message slot space, gmb in the child slot
// space. Each slot's adjoint is consumed (read and cleared) by the one layer that produced the
// slot's value, after every reader of that value has added its part: readers run later in the
// pass, so earlier in its reverse.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.h"
#include "kernels.h"

namespace bddmp {

namespace {

__device__ __forceinline__ float smin(float a, float b, float alpha) {
  const float lo = fminf(a, b), hi = fmaxf(a, b);
  if (isinf(hi)) return lo;
  return lo - alpha * log1pf(expf(-(hi - lo) / alpha));
}

// derivative of s = smin(..., a, ...) with respect to argument a
__device__ __forceinline__ float sweight(float a, float s, float alpha) {
  return (isinf(a) || isinf(s)) ? 0.0f : expf(-(a - s) / alpha);
}

// child code of a narrow layer's arc: node index 0 / 1, or -1 for a terminal
__device__ __forceinline__ int c2node(uint32_t code) { return (code & 2u) ? -1 : int(code & 1u); }

// The smoothed update: eq. "mma-update" on the marginal log-sum-exp differences. With rows that
// force the variable (infinite difference), only the rows whose move raises the smoothed bound
// hand their difference to the forced rows (those with d > 0 when a row forces x_i = 1, d < 0 when
// a row forces x_i = 0); the forced rows share the sum.
__device__ __forceinline__ bool moving(float d, bool neg) { return !isinf(d) && (neg ? d > 0.0f : d < 0.0f); }
__device__ __forceinline__ float s_updated(float lam0, float d, float share, int nf, bool neg) {
  if (nf == 0) return (lam0 - d) + share;
  if (isinf(d)) return lam0 + share;
  return moving(d, neg) ? lam0 - d : lam0;
}

// smoothed min-marginals of one layer (eq. "marginal-log-sum-exp" through arc values)
struct SMarg {
  float m0, m1;
};
__device__ __forceinline__ SMarg s_marg_narrow(uint32_t meta, float2 f, float2 b, float lam, float alpha) {
  const uint32_t lo0 = meta & 3u, hi0 = (meta >> 2) & 3u, lo1 = (meta >> 4) & 3u, hi1 = (meta >> 6) & 3u;
  SMarg r;
  r.m0 = smin(f.x + c2val(lo0, b), f.y + c2val(lo1, b), alpha);
  r.m1 = smin((f.x + lam) + c2val(hi0, b), (f.y + lam) + c2val(hi1, b), alpha);
  return r;
}
__device__ __forceinline__ SMarg s_marg_general(const Dev &D, const GRec &g, const float *mb, float lam, float alpha) {
  SMarg r{INFINITY, INFINITY};
  for (int u = 0; u < g.w; ++u) {
    const uint32_t a = D.garcs[g.os + u];
    const float fu = D.mf[g.os + u];
    r.m0 = smin(r.m0, fu + c16val(mb, g.cs, a & 0xFFFFu), alpha);
    r.m1 = smin(r.m1, (fu + lam) + c16val(mb, g.cs, a >> 16), alpha);
  }
  return r;
}

// next-level forward messages pushed from a narrow level (fold over node 0 lo, hi, node 1 lo, hi)
__device__ __forceinline__ float2 s_push_narrow(uint32_t meta, float2 f, float lam, float alpha) {
  const float a[4] = {f.x, f.x + lam, f.y, f.y + lam};
  float c0 = INFINITY, c1 = INFINITY;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t k = (meta >> (2 * q)) & 3u;
    c0 = smin(c0, k == 0u ? a[q] : INFINITY, alpha);
    c1 = smin(c1, k == 1u ? a[q] : INFINITY, alpha);
  }
  return make_float2(c0, c1);
}

struct Seg {
  float share;
  int nf;
  bool neg;
};

// J_i sums of a tile's segments: the head lane of each variable reads its rows' differences in
// ascending row order and leaves the share, the forced count and the forced sign for its lanes
__device__ __forceinline__ Seg seg_update(float d, uint32_t meta, bool active, float *s_d, float *s_share, int *s_nf) {
  const int s = int(threadIdx.x);
  s_d[s] = d;
  __syncthreads();
  const int pos = int((meta >> kMetaPosShift) & kMetaField);
  const int len = int((meta >> kMetaLenShift) & kMetaField);
  if (active && pos == 0) {
    float sum = 0.0f, moved = 0.0f;
    int nf = 0, neg = 0;
    for (int q = 0; q < len; ++q) {
      const float dq = s_d[s + q];
      if (isinf(dq)) {
        ++nf;
        if (dq < 0.0f) neg = 1;
      } else {
        sum += dq;
      }
    }
    if (nf)
      for (int q = 0; q < len; ++q) {
        const float dq = s_d[s + q];
        if (moving(dq, neg)) moved += dq;
      }
    s_share[s] = nf ? moved / float(nf) : sum / float(len);
    s_nf[s] = nf | (neg << 30);
  }
  __syncthreads();
  const int h = s - pos;
  Seg r;
  r.share = s_share[h];
  r.nf = s_nf[h] & ~(1 << 30);
  r.neg = (s_nf[h] >> 30) & 1;
  return r;
}

// Smoothed forward (DIR kFwd) or backward (kBwd) wave; MODE kUpdate or kNoUpdate (initial sweep).
template <int DIR, int MODE, bool LIST>
__global__ __launch_bounds__(kTile) void smooth_wave_kernel(const Dev D, const SmoothArgs A, const int tile0) {
  __shared__ float s_d[kTile];
  __shared__ float s_share[kTile];
  __shared__ int s_nf[kTile];
  const int32_t *tiles = DIR == kFwd ? D.fwd_tiles : D.bwd_tiles;
  const int tix = tile0 + xcd_tile(int(blockIdx.x), int(gridDim.x));
  const int p0 = int(uint32_t(tiles[2 * tix]) & kTilePosMask);
  const uint32_t end = uint32_t(tiles[2 * tix + 1]);
  const bool roots = DIR == kBwd && (end & kTileRootBit) != 0u;
  const int cnt = int(end & ~kTileRootBit) - p0;
  const int s = int(threadIdx.x);
  const bool active = s < cnt;
  const float alpha = A.alpha;

  int L = 0, tgt = -1;
  uint32_t meta = 0;
  float lam0 = 0.0f;
  float2 f = make_float2(0.0f, 0.0f), b = f;
  if (active) {
    L = (DIR == kBwd && LIST) ? D.bwd_list[p0 + s] : p0 + s;
    meta = D.meta[L];
    lam0 = D.lam[L];
    tgt = DIR == kFwd ? D.child[L] : D.parent[L];
    f = reinterpret_cast<const float2 *>(D.mf)[L];
    b = reinterpret_cast<const float2 *>(D.mbc)[L];
  }
  const bool narrow = ((meta >> kMetaWidthShift) & 3u) != 0u;
  float lam1 = lam0;
  if (MODE == kUpdate) {
    SMarg m{0.0f, 0.0f};
    if (active) m = narrow ? s_marg_narrow(meta, f, b, lam0, alpha) : s_marg_general(D, grec_of(D, L), D.mbc, lam0, alpha);
    const float d = m.m1 - m.m0;
    const Seg g = seg_update(d, meta, active, s_d, s_share, s_nf);
    if (active) {
      lam1 = s_updated(lam0, d, g.share, g.nf, g.neg);
      D.lam[L] = lam1;
    }
  }
  if (DIR == kFwd) {
    if (active && tgt >= 0) {
      if (narrow) {
        reinterpret_cast<float2 *>(D.mf)[tgt] = s_push_narrow(meta, f, lam1, alpha);
      } else {
        const GRec g = grec_of(D, L);
        const int cs = D.grec[tgt].x;
        for (int q = 0; q < g.wc; ++q) D.mf[cs + q] = INFINITY;
        for (int u = 0; u < g.w; ++u) {
          const uint32_t a = D.garcs[g.os + u];
          const float fu = D.mf[g.os + u];
          if ((a & 0xFFFFu) < kTop) D.mf[cs + int(a & 0xFFFFu)] = smin(D.mf[cs + int(a & 0xFFFFu)], fu, alpha);
          if ((a >> 16) < kTop) D.mf[cs + int(a >> 16)] = smin(D.mf[cs + int(a >> 16)], fu + lam1, alpha);
        }
      }
    }
  } else {
    float r = 0.0f;
    if (active) {
      if (narrow) {
        const float n0 = smin(c2val(meta & 3u, b), c2val((meta >> 2) & 3u, b) + lam1, alpha);
        const float n1 = smin(c2val((meta >> 4) & 3u, b), c2val((meta >> 6) & 3u, b) + lam1, alpha);
        if (tgt >= 0) reinterpret_cast<float2 *>(D.mbc)[tgt] = make_float2(n0, n1);
        r = n0;
      } else {
        const GRec g = grec_of(D, L);
        const int ps = tgt >= 0 ? D.grec[tgt].y : -1;
        for (int u = 0; u < g.w; ++u) {
          const uint32_t a = D.garcs[g.os + u];
          const float v = smin(c16val(D.mbc, g.cs, a & 0xFFFFu), c16val(D.mbc, g.cs, a >> 16) + lam1, alpha);
          if (ps >= 0) D.mbc[ps + u] = v;
          if (u == 0) r = v;
        }
      }
    }
    const double e = (active && (meta & kMetaRootBit)) ? double(r) : 0.0;
    if (roots) {
      const double v = wave_sum(e);
      if ((threadIdx.x & 63) == 0) D.lbpart[kTile / 64 * tix + (int(threadIdx.x) >> 6)] = v;
    }
  }
}

// Adjoint of the J_i update: given the adjoints of the updated multipliers (gl1), the adjoints of
// the differences. Forced rows: no derivative through their infinite difference.
__device__ __forceinline__ float seg_adjoint(float d, float gl1, uint32_t meta, bool active, float *s_d, float *s_g,
                                             float *s_a, int *s_nf) {
  const int s = int(threadIdx.x);
  s_d[s] = d;
  s_g[s] = gl1;
  __syncthreads();
  const int pos = int((meta >> kMetaPosShift) & kMetaField);
  const int len = int((meta >> kMetaLenShift) & kMetaField);
  if (active && pos == 0) {
    float gsum = 0.0f, gforced = 0.0f;
    int nf = 0, neg = 0;
    for (int q = 0; q < len; ++q) {
      const float dq = s_d[s + q];
      if (isinf(dq)) {
        ++nf;
        gforced += s_g[s + q];
        if (dq < 0.0f) neg = 1;
      }
      gsum += s_g[s + q];
    }
    s_a[s] = nf ? gforced / float(nf) : gsum / float(len);
    s_nf[s] = nf | (neg << 30);
  }
  __syncthreads();
  const int h = s - pos;
  const float avg = s_a[h];
  const int nf = s_nf[h] & ~(1 << 30);
  const bool neg = (s_nf[h] >> 30) & 1;
  if (nf == 0) return -gl1 + avg;
  return moving(d, neg) ? -gl1 + avg : 0.0f;
}

// Adjoint of one wave of a smoothed pass. DIR kBwd, MODE kUpdate: the backward pass (multipliers
// A.lam_prev before, D.lam after; forward messages D.mf; backward messages D.mbc as the pass left
// them). DIR kFwd, MODE kUpdate: the forward pass (A.lam_prev before, A.lam_upd after; D.mf as the
// pass left them; backward messages A.mbt as the pass read them). DIR kBwd, MODE kNoUpdate: the
// initial sweep (D.lam, D.mbc). Three phases, each lane on its own layer: undo the step that
// follows the update (backward step or push), exchange the J_i adjoints (every lane of the
// workgroup takes part), undo the min-marginals.
template <int DIR, int MODE, bool LIST>
__global__ __launch_bounds__(kTile) void smooth_adjoint_kernel(const Dev D, const SmoothArgs A, const int tile0) {
  __shared__ float s_d[kTile];
  __shared__ float s_g[kTile];
  __shared__ float s_a[kTile];
  __shared__ int s_nf[kTile];
  const int32_t *tiles = DIR == kFwd ? D.fwd_tiles : D.bwd_tiles;
  const int tix = tile0 + xcd_tile(int(blockIdx.x), int(gridDim.x));
  const int p0 = int(uint32_t(tiles[2 * tix]) & kTilePosMask);
  const uint32_t end = uint32_t(tiles[2 * tix + 1]);
  const int cnt = int(end & ~kTileRootBit) - p0;
  const int s = int(threadIdx.x);
  const bool active = s < cnt;
  const float alpha = A.alpha;
  float2 *gmf2 = reinterpret_cast<float2 *>(A.gmf);
  float2 *gmb2 = reinterpret_cast<float2 *>(A.gmb);
  // backward messages of the child level as the pass read them
  const float *mbr = (DIR == kFwd) ? A.mbt : D.mbc;

  int L = 0, child = -1, parent = -1;
  uint32_t meta = 0;
  float lam0 = 0.0f, lam1 = 0.0f, gl = 0.0f;
  float2 f = make_float2(0.0f, 0.0f), b = f;
  GRec g{};
  if (active) {
    L = (DIR == kBwd && LIST) ? D.bwd_list[p0 + s] : p0 + s;
    meta = D.meta[L];
    child = D.child[L];
    parent = D.parent[L];
    if (DIR == kBwd) {
      lam1 = D.lam[L];
      lam0 = MODE == kUpdate ? A.lam_prev[L] : lam1;
    } else {
      lam0 = A.lam_prev[L];
      lam1 = A.lam_upd[L];
    }
    gl = A.glam[L];
    f = reinterpret_cast<const float2 *>(D.mf)[L];
    b = reinterpret_cast<const float2 *>(mbr)[L];
  }
  const bool narrow = ((meta >> kMetaWidthShift) & 3u) != 0u;
  const bool root = (meta & kMetaRootBit) != 0u;
  if (active && !narrow) g = grec_of(D, L);
  float gf0 = 0.0f, gf1 = 0.0f, gc0 = 0.0f, gc1 = 0.0f;  // narrow: own / child level adjoints

  // phase 1: the step after the update
  if (active && DIR == kBwd) {
    if (narrow) {
      float2 gn = make_float2(0.0f, 0.0f);
      if (parent >= 0) {
        gn = gmb2[parent];
        gmb2[parent] = make_float2(0.0f, 0.0f);
      } else if (root) {
        gn.x = A.root_seed;
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const uint32_t klo = (meta >> (4 * u)) & 3u, khi = (meta >> (4 * u + 2)) & 3u;
        const float x0 = c2val(klo, b), x1 = c2val(khi, b) + lam1;
        const float n = smin(x0, x1, alpha);
        const float gu = u ? gn.y : gn.x;
        const float w0 = sweight(x0, n, alpha) * gu, w1 = sweight(x1, n, alpha) * gu;
        const int c0 = c2node(klo), c1 = c2node(khi);
        if (c0 == 0) gc0 += w0;
        if (c0 == 1) gc1 += w0;
        if (c1 == 0) gc0 += w1;
        if (c1 == 1) gc1 += w1;
        gl += w1;
      }
    } else {
      const int ps = parent >= 0 ? D.grec[parent].y : -1;
      for (int u = 0; u < g.w; ++u) {
        float gn = 0.0f;
        if (ps >= 0) {
          gn = A.gmb[ps + u];
          A.gmb[ps + u] = 0.0f;
        } else if (root && u == 0) {
          gn = A.root_seed;
        }
        if (gn == 0.0f) continue;
        const uint32_t a = D.garcs[g.os + u];
        const float x0 = c16val(D.mbc, g.cs, a & 0xFFFFu), x1 = c16val(D.mbc, g.cs, a >> 16) + lam1;
        const float n = smin(x0, x1, alpha);
        const float w0 = sweight(x0, n, alpha) * gn, w1 = sweight(x1, n, alpha) * gn;
        if ((a & 0xFFFFu) < kTop) A.gmb[g.cs + int(a & 0xFFFFu)] += w0;
        if ((a >> 16) < kTop) A.gmb[g.cs + int(a >> 16)] += w1;
        gl += w1;
      }
    }
  }
  if (active && DIR == kFwd && child >= 0) {
    if (narrow) {
      const float2 gv = gmf2[child];
      gmf2[child] = make_float2(0.0f, 0.0f);
      const float2 cv = s_push_narrow(meta, f, lam1, alpha);
      const float av[4] = {f.x, f.x + lam1, f.y, f.y + lam1};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t kk = (meta >> (2 * q)) & 3u;
        if (kk > 1u) continue;
        const float w = sweight(av[q], kk == 0u ? cv.x : cv.y, alpha) * (kk == 0u ? gv.x : gv.y);
        if (q < 2) gf0 += w;
        else gf1 += w;
        if (q & 1) gl += w;
      }
    } else {
      const int osc = D.grec[child].x;
      // next-level values recomputed in the pass's fold order, then the adjoints of the in-arcs
      for (int v = 0; v < g.wc; ++v) {
        const float gv = A.gmf[osc + v];
        if (gv == 0.0f) continue;
        float cv = INFINITY;
        for (int u = 0; u < g.w; ++u) {
          const uint32_t a = D.garcs[g.os + u];
          const float fu = D.mf[g.os + u];
          if (int(a & 0xFFFFu) == v) cv = smin(cv, fu, alpha);
          if (int(a >> 16) == v) cv = smin(cv, fu + lam1, alpha);
        }
        for (int u = 0; u < g.w; ++u) {
          const uint32_t a = D.garcs[g.os + u];
          const float fu = D.mf[g.os + u];
          if (int(a & 0xFFFFu) == v) A.gmf[g.os + u] += gv * sweight(fu, cv, alpha);
          if (int(a >> 16) == v) {
            const float w = gv * sweight(fu + lam1, cv, alpha);
            A.gmf[g.os + u] += w;
            gl += w;
          }
        }
      }
      for (int v = 0; v < g.wc; ++v) A.gmf[osc + v] = 0.0f;
    }
  }

  if (MODE == kUpdate) {
    // phase 2: adjoints of the differences (all lanes)
    SMarg m{0.0f, 0.0f};
    if (active) m = narrow ? s_marg_narrow(meta, f, b, lam0, alpha) : s_marg_general(D, g, mbr, lam0, alpha);
    const float d = m.m1 - m.m0;
    const float gd = seg_adjoint(d, gl, meta, active, s_d, s_g, s_a, s_nf);
    // phase 3: the min-marginals
    if (active && !isinf(d) && gd != 0.0f) {
      if (narrow) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const uint32_t klo = (meta >> (4 * u)) & 3u, khi = (meta >> (4 * u + 2)) & 3u;
          const float fu = u ? f.y : f.x;
          const float a0 = fu + c2val(klo, b), a1 = (fu + lam0) + c2val(khi, b);
          const float w0 = -gd * sweight(a0, m.m0, alpha), w1 = gd * sweight(a1, m.m1, alpha);
          if (u) gf1 += w0 + w1;
          else gf0 += w0 + w1;
          const int c0 = c2node(klo), c1 = c2node(khi);
          if (c0 == 0) gc0 += w0;
          if (c0 == 1) gc1 += w0;
          if (c1 == 0) gc0 += w1;
          if (c1 == 1) gc1 += w1;
          gl += w1;
        }
      } else {
        for (int u = 0; u < g.w; ++u) {
          const uint32_t a = D.garcs[g.os + u];
          const float fu = D.mf[g.os + u];
          const float a0 = fu + c16val(mbr, g.cs, a & 0xFFFFu), a1 = (fu + lam0) + c16val(mbr, g.cs, a >> 16);
          const float w0 = -gd * sweight(a0, m.m0, alpha), w1 = gd * sweight(a1, m.m1, alpha);
          A.gmf[g.os + u] += w0 + w1;
          if ((a & 0xFFFFu) < kTop) A.gmb[g.cs + int(a & 0xFFFFu)] += w0;
          if ((a >> 16) < kTop) A.gmb[g.cs + int(a >> 16)] += w1;
          gl += w1;
        }
      }
    }
  }
  if (!active) return;
  A.glam[L] = gl;
  if (narrow) {
    if (gc0 != 0.0f || gc1 != 0.0f) {
      const float2 o = gmb2[L];
      gmb2[L] = make_float2(o.x + gc0, o.y + gc1);
    }
    if (MODE == kUpdate && DIR == kFwd && root) {
      gmf2[L] = make_float2(0.0f, 0.0f);  // the root's forward message is the constant 0
    } else if (gf0 != 0.0f || gf1 != 0.0f) {
      const float2 o = gmf2[L];
      gmf2[L] = make_float2(o.x + gf0, o.y + gf1);
    }
  } else if (MODE == kUpdate && DIR == kFwd && root) {
    for (int u = 0; u < g.w; ++u) A.gmf[g.os + u] = 0.0f;
  }
}

// free-variable constants of the bound: sum of min(0, c_i) and of smin(0, c_i) over variables in
// no row (fixed-shape partial sums, then one workgroup)
__global__ __launch_bounds__(256) void free_const_partial_kernel(const Dev D, int n, float alpha) {
  __shared__ double sh[4];
  const int chunk = (n + kLbBlocks - 1) / kLbBlocks;
  const int i0 = int(blockIdx.x) * chunk, i1 = min(n, i0 + chunk);
  double a = 0.0, b = 0.0;
  for (int i = i0 + int(threadIdx.x); i < i1; i += 256)
    if (D.var_nj[i] == 0) {
      const double c = D.cost[i];
      a += c < 0.0 ? c : 0.0;
      b += double(smin(0.0f, float(c), alpha));
    }
  const double sa = block_sum(a, sh);
  const double sb = block_sum(b, sh);
  if (threadIdx.x == 0) {
    D.part[blockIdx.x] = sa;
    D.part[kLbBlocks + blockIdx.x] = sb;
  }
}

__global__ __launch_bounds__(kLbBlocks) void free_const_final_kernel(const Dev D) {
  __shared__ double sh[kLbBlocks / 64];
  const int t = int(threadIdx.x);
  const double a = block_sum(D.part[t], sh);
  const double b = block_sum(D.part[kLbBlocks + t], sh);
  if (t == 0) {
    D.lbc[0] = a;
    D.lbc[1] = b;
  }
}

// d LB / d c_i: sum over the variable's layers of the multiplier adjoints / |J_i| (lambda_0 =
// c_i / |J_i|); a variable in no row: the weight of c_i in smin(0, c_i)
__global__ void smooth_grad_kernel(const Dev D, const SmoothArgs A, int n, float scale, float *grad) {
  const int i = int(blockIdx.x) * blockDim.x + int(threadIdx.x);
  if (i >= n) return;
  const int nj = D.var_nj[i];
  if (nj == 0) {
    const float c = float(D.cost[i]);
    grad[i] = scale * sweight(c, smin(0.0f, c, A.alpha), A.alpha);
    return;
  }
  const int f0 = D.var_first[i];
  float s = 0.0f;
  for (int q = 0; q < nj; ++q) s += A.glam[f0 + q];
  grad[i] = s / float(nj);
}

__global__ void cost_in_kernel(const Dev D, const double *c, int n) {
  const int i = int(blockIdx.x) * blockDim.x + int(threadIdx.x);
  if (i < n) const_cast<double *>(D.cost)[i] = c[i];
}

int blocks_of(int64_t count, int per) { return int((count + per - 1) / per); }

template <int DIR, int MODE>
hipError_t smooth_dispatch(bool adjoint, bool list, int nt, int tile0, const Dev &D, const SmoothArgs &A, hipStream_t s) {
  if (adjoint) {
    if (list)
      hipLaunchKernelGGL((smooth_adjoint_kernel<DIR, MODE, true>), dim3(nt), dim3(kTile), 0, s, D, A, tile0);
    else
      hipLaunchKernelGGL((smooth_adjoint_kernel<DIR, MODE, false>), dim3(nt), dim3(kTile), 0, s, D, A, tile0);
  } else {
    if (list)
      hipLaunchKernelGGL((smooth_wave_kernel<DIR, MODE, true>), dim3(nt), dim3(kTile), 0, s, D, A, tile0);
    else
      hipLaunchKernelGGL((smooth_wave_kernel<DIR, MODE, false>), dim3(nt), dim3(kTile), 0, s, D, A, tile0);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_smooth_wave(int dir, int mode, bool adjoint, bool list, int nt, int tile0, const Dev &D,
                              const SmoothArgs &A, hipStream_t s) {
  if (nt <= 0) return hipSuccess;
  if (dir == kFwd && mode == kUpdate) return smooth_dispatch<kFwd, kUpdate>(adjoint, false, nt, tile0, D, A, s);
  if (dir == kBwd && mode == kUpdate) return smooth_dispatch<kBwd, kUpdate>(adjoint, list, nt, tile0, D, A, s);
  if (dir == kBwd && mode == kNoUpdate) return smooth_dispatch<kBwd, kNoUpdate>(adjoint, list, nt, tile0, D, A, s);
  return hipErrorInvalidValue;
}

hipError_t launch_free_const(const Dev &D, int n, float alpha, hipStream_t s) {
  hipLaunchKernelGGL(free_const_partial_kernel, dim3(kLbBlocks), dim3(256), 0, s, D, n, alpha);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(free_const_final_kernel, dim3(1), dim3(kLbBlocks), 0, s, D);
  return hipGetLastError();
}

hipError_t launch_smooth_grad(const Dev &D, const SmoothArgs &A, int n, float scale, float *grad, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(smooth_grad_kernel, dim3(blocks_of(n, 256)), dim3(256), 0, s, D, A, n, scale, grad);
  return hipGetLastError();
}

hipError_t launch_cost_in(const Dev &D, const double *c, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(cost_in_kernel, dim3(blocks_of(n, 256)), dim3(256), 0, s, D, c, n);
  return hipGetLastError();
}

}  // namespace bddmp
