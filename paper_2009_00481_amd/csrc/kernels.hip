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

#include <cmath>

#include "kernels.h"

namespace bddmp {

namespace {

// backward message behind a 2-bit child code of a narrow layer
__device__ __forceinline__ float c2val(uint32_t code, float2 b) {
  // codes 0, 1: node of the next level; 2 (kC2Bot): +inf; 3 (kC2Top): 0. Selects, no branches.
  const float node = (code & 1u) ? b.y : b.x;
  const float term = (code & 1u) ? 0.0f : INFINITY;
  return (code & 2u) ? term : node;
}

// backward message behind a 16-bit child code of a general layer
__device__ __forceinline__ float c16val(const float *__restrict__ mb, int cs, uint32_t c) {
  return c < kTop ? mb[cs + int(c)] : (c == kTop ? 0.0f : INFINITY);
}

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
template <int DIR, bool NARROW_ONLY>
struct Layer {
  int L;
  int tgt;
  uint32_t meta;
  float lam0;
  float2 f, b;     // narrow: own forward messages, child backward messages
  int4 g;          // general: own slot, own width, child slot, child width
  float m0, m1;

  __device__ __forceinline__ bool narrow() const {
    return NARROW_ONLY || ((meta >> kMetaWidthShift) & 3u) != 0u;
  }

  __device__ __forceinline__ void begin(const Dev &D, int L_) {
    L = L_;
    meta = D.meta[L];
    lam0 = D.lam[L];
    tgt = DIR == kFwd ? D.child[L] : D.parent[L];
    f = reinterpret_cast<const float2 *>(D.mf)[L];
    b = reinterpret_cast<const float2 *>(D.mbc)[L];
    // keep the five independent loads ahead of every use, so they are in flight together
    __builtin_amdgcn_sched_barrier(0);
    m0 = INFINITY;
    m1 = INFINITY;
    if (narrow()) {
      // arc-marginals (m_fwd + theta) + m_bwd minimised per arc label (eqs. "arc-marginal",
      // "marginal-aggregation"); a padding node's arcs both lead to BOT
      const uint32_t lo0 = meta & 3u, hi0 = (meta >> 2) & 3u, lo1 = (meta >> 4) & 3u, hi1 = (meta >> 6) & 3u;
      m0 = fminf(f.x + c2val(lo0, b), f.y + c2val(lo1, b));
      m1 = fminf((f.x + lam0) + c2val(hi0, b), (f.y + lam0) + c2val(hi1, b));
    } else {
      g = D.grec[L];
      for (int u = 0; u < g.y; ++u) {
        const uint32_t a = D.garcs[g.x + u];
        const float fu = D.mf[g.x + u];
        m0 = fminf(m0, fu + c16val(D.mbc, g.z, a & 0xFFFFu));
        m1 = fminf(m1, (fu + lam0) + c16val(D.mbc, g.z, a >> 16));
      }
    }
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
      reinterpret_cast<float2 *>(D.mf)[tgt] = make_float2(c0, c1);
    } else {
      const int cs = D.grec[tgt].x;  // the child layer's own slots
      for (int q = 0; q < g.w; ++q) D.mf[cs + q] = INFINITY;
      for (int u = 0; u < g.y; ++u) {
        const uint32_t a = D.garcs[g.x + u];
        const uint32_t lo = a & 0xFFFFu, hi = a >> 16;
        const float fu = D.mf[g.x + u];
        if (lo < kTop) D.mf[cs + int(lo)] = fminf(D.mf[cs + int(lo)], fu);
        if (hi < kTop) D.mf[cs + int(hi)] = fminf(D.mf[cs + int(hi)], fu + lam1);
      }
    }
  }

  // backward step of this level (Alg. "Backward BDD update step") with the updated multiplier,
  // stored at the parent layer's child slots; returns the root's new backward message (E^j) on a
  // root level, else 0
  __device__ __forceinline__ double bstep(const Dev &D, float lam1) const {
    float r;
    if (narrow()) {
      const float n0 = fminf(c2val(meta & 3u, b), c2val((meta >> 2) & 3u, b) + lam1);
      const float n1 = fminf(c2val((meta >> 4) & 3u, b), c2val((meta >> 6) & 3u, b) + lam1);
      if (tgt >= 0) reinterpret_cast<float2 *>(D.mbc)[tgt] = make_float2(n0, n1);
      r = n0;
    } else {
      r = 0.0f;
      const int ps = tgt >= 0 ? D.grec[tgt].z : -1;  // the parent layer's child slots
      for (int u = 0; u < g.y; ++u) {
        const uint32_t a = D.garcs[g.x + u];
        const float v = fminf(c16val(D.mbc, g.z, a & 0xFFFFu), c16val(D.mbc, g.z, a >> 16) + lam1);
        if (ps >= 0) D.mbc[ps + u] = v;
        if (u == 0) r = v;
      }
    }
    return (meta & kMetaRootBit) ? double(r) : 0.0;
  }
};

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b runs on XCD b % 8, each XCD
// with its own L2). Remap so that XCD x takes one contiguous run of the launch's tiles: lines at a
// boundary between neighbouring tiles are then shared inside one L2 instead of across XCDs.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int q = n / kXcds, r = n % kXcds;
  const int x = b % kXcds, k = b / kXcds;
  return x * q + min(x, r) + k;
}

// Sum of one double per lane over the workgroup in a fixed shape (butterfly inside each
// wavefront, then the wavefront totals in order), so the result does not depend on timing.
__device__ __forceinline__ double block_sum(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = int(threadIdx.x) >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = int(blockDim.x) >> 6;
  for (int q = 0; q < nw; ++q) s += sh[q];
  __syncthreads();
  return s;
}

// LIST: backward positions go through bwd_list (a wave that is not one contiguous layer range).
template <int DIR, int MODE, bool NARROW_ONLY, bool LIST>
__global__ __launch_bounds__(kTile) void wave_kernel(const Dev D, const int tile0) {
  __shared__ float s_d[kTile];
  __shared__ float s_share[kTile];
  __shared__ int s_nf[kTile];
  __shared__ double s_red[kTile / 64];
  const int32_t *tiles = DIR == kFwd ? D.fwd_tiles : D.bwd_tiles;
  const int tix = tile0 + xcd_tile(int(blockIdx.x), int(gridDim.x));
  const int p0 = tiles[2 * tix];
  // a backward tile's end carries bit 31 when the tile holds a root level
  const uint32_t end = uint32_t(tiles[2 * tix + 1]);
  const bool roots = DIR == kBwd && (end & kTileRootBit) != 0u;
  const int cnt = int(end & ~kTileRootBit) - p0;
  const int s = int(threadIdx.x);
  const bool active = s < cnt;

  Layer<DIR, NARROW_ONLY> ly;
  ly.meta = 0;
  ly.lam0 = 0.0f;
  ly.m0 = ly.m1 = 0.0f;
  if (active) ly.begin(D, (DIR == kBwd && LIST) ? D.bwd_list[p0 + s] : p0 + s);
  const float d = ly.m1 - ly.m0;
  float lam1 = ly.lam0;
  if (MODE == kUpdate) {
    s_d[s] = d;
    __syncthreads();
    const int pos = int((ly.meta >> kMetaPosShift) & kMetaField);
    const int len = int((ly.meta >> kMetaLenShift) & kMetaField);
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
      lam1 = updated(ly.lam0, d, s_share[h], s_nf[h]);
      D.lam[ly.L] = lam1;
    }
  }
  if (MODE == kExtract && active) {
    const int c = D.canon_of[ly.L];
    if (D.out0) D.out0[c] = ly.m0;
    if (D.out1) D.out1[c] = ly.m1;
    D.d_fresh[ly.L] = d;
  }
  if (DIR == kFwd) {
    if (active) ly.push(D, lam1);
  } else {
    const double e = active ? ly.bstep(D, lam1) : 0.0;
    // bound partial per wavefront: a fixed butterfly, only in tiles holding root levels (the
    // branch is uniform over the workgroup)
    double v = 0.0;
    if (roots) {
      v = e;
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    }
    if ((threadIdx.x & 63) == 0) D.lbpart[kTile / 64 * tix + (int(threadIdx.x) >> 6)] = v;
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
    Layer<DIR, false> ly;
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
    Layer<DIR, false> ly;
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

// LB = sum_j E^j (problem (D)) from the per-tile partials of the backward sweep: kLbStage blocks
// each sum one fixed contiguous chunk, then one block sums the chunk totals; fixed order throughout
__global__ __launch_bounds__(256) void lb_stage_kernel(const Dev D, int nparts) {
  __shared__ double sh[4];
  const int chunk = (nparts + kLbStage - 1) / kLbStage;
  const int q0 = int(blockIdx.x) * chunk, q1 = min(nparts, q0 + chunk);
  double acc = 0.0;
  for (int q = q0 + int(threadIdx.x); q < q1; q += 256) acc += D.lbpart[q];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) D.part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kLbStage) void lb_final_kernel(const Dev D, double lb_const, int slot) {
  __shared__ double sh[kLbStage / 64];
  const double s = block_sum(D.part[threadIdx.x], sh);
  if (threadIdx.x == 0) D.lb_hist[slot] = s + lb_const;
}

// per variable: g_i = c_i - sum_j lambda^j_i; partial max |g| and sum of min(0, g)
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
      e = fminf(c16val(D.mbc, g.z, a & 0xFFFFu), c16val(D.mbc, g.z, a >> 16) + lam);
    }
    acc += double(e);
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) D.inst_lb[k] = t;
}

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
      const uint32_t ch = D.xbuf[D.layer_var[L]] ? (a >> 16) : (a & 0xFFFFu);
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
    hipLaunchKernelGGL((wave_kernel<DIR, MODE, true, false>), dim3(nt), dim3(kTile), 0, s, D, tile0);
  else if (narrow_only)
    hipLaunchKernelGGL((wave_kernel<DIR, MODE, true, true>), dim3(nt), dim3(kTile), 0, s, D, tile0);
  else if (!list)
    hipLaunchKernelGGL((wave_kernel<DIR, MODE, false, false>), dim3(nt), dim3(kTile), 0, s, D, tile0);
  else
    hipLaunchKernelGGL((wave_kernel<DIR, MODE, false, true>), dim3(nt), dim3(kTile), 0, s, D, tile0);
  return hipGetLastError();
}

hipError_t launch_wave(int dir, int mode, bool narrow_only, bool list, int nt, int tile0, const Dev &D,
                       hipStream_t s) {
  if (dir == kFwd && mode == kUpdate) return wave_dispatch<kFwd, kUpdate>(narrow_only, false, nt, tile0, D, s);
  if (dir == kFwd && mode == kExtract) return wave_dispatch<kFwd, kExtract>(narrow_only, false, nt, tile0, D, s);
  if (dir == kBwd && mode == kUpdate) return wave_dispatch<kBwd, kUpdate>(narrow_only, list, nt, tile0, D, s);
  if (dir == kBwd && mode == kNoUpdate) return wave_dispatch<kBwd, kNoUpdate>(narrow_only, list, nt, tile0, D, s);
  return hipErrorInvalidValue;
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

hipError_t launch_lb(const Dev &D, int nparts, double lb_const, int slot, hipStream_t s) {
  hipLaunchKernelGGL(lb_stage_kernel, dim3(kLbStage), dim3(256), 0, s, D, nparts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lb_final_kernel, dim3(1), dim3(kLbStage), 0, s, D, lb_const, slot);
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
