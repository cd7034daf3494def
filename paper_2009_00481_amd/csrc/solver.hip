// Device side of bddmp: wave kernels for the forward and backward passes, the fp64 bound, and the
// output kernels, plus the solver's host code that enqueues them on the caller's stream.
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
#include <string>
#include <vector>

#include "internal.h"
#include "solver.h"

namespace bddmp {

namespace {

constexpr int kFwd = 0, kBwd = 1;
constexpr int kUpdate = 0;   // min-marginals, J_i sum, multiplier update, then step
constexpr int kNoUpdate = 1; // step only (initial backward sweep)
constexpr int kExtract = 2;  // min-marginals to the outputs, then step with unchanged multipliers

struct Dev {
  const uint32_t *meta;
  const int32_t *child, *parent;
  float *lam;
  float *mf;   // forward messages of each layer's own level (own slots)
  float *mbc;  // backward messages of each layer's child level (child slots)
  const uint32_t *garcs;
  const int4 *grec;
  const int32_t *canon_of, *layer_of, *layer_var, *root_slot;
  const int32_t *fwd_tiles, *bwd_tiles, *bwd_list, *fwd_big, *bwd_big;
  const int32_t *bdd_canon_off;
  const double *cost;
  const int32_t *var_first, *var_nj;
  float *d_fresh, *mbuf;
  int8_t *xbuf;
  double *part, *lbpart;
  double *lb_hist, *scal;
  float *out0, *out1;
  int32_t n_bwd_tiles;  // bound partials of big backward tiles start here
};

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
constexpr int kLbStage = 256;
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
// host side
// ---------------------------------------------------------------------------------------------

struct Solver {
  const Plan *plan = nullptr;
  char *arena = nullptr;
  hipStream_t stream = nullptr;
  Dev D{};
  int64_t n_hist = 0;  // bounds recorded so far
  int64_t iters = 0;
};

namespace {

int32_t hip_fail(hipError_t e, const char *what) {
  return set_error(BDDMP_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

int32_t launched(const char *what) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? BDDMP_OK : hip_fail(e, what);
}

struct EventPair {
  hipEvent_t a, b;
  int cls;
};

// One pass: every wave in order; ev != nullptr records an event pair around each wave's launches.
template <int DIR, int MODE>
int32_t run_pass(Solver &S, std::vector<EventPair> *ev, int cls) {
  const Plan &P = *S.plan;
  const auto &waves = DIR == kFwd ? P.fwd_waves : P.bwd_waves;
  for (const WaveRange &wr : waves) {
    const int nt = wr.tile_end - wr.tile_begin;
    const int nb = wr.big_end - wr.big_begin;
    EventPair e{};
    if (ev) {
      HIP_TRY(hipEventCreate(&e.a), "hipEventCreate");
      HIP_TRY(hipEventCreate(&e.b), "hipEventCreate");
      e.cls = cls;
      HIP_TRY(hipEventRecord(e.a, S.stream), "hipEventRecord");
    }
    if (nt > 0) {
      const bool list = DIR == kBwd && wr.list;
      if (wr.narrow_only && !list)
        hipLaunchKernelGGL((wave_kernel<DIR, MODE, true, false>), dim3(nt), dim3(kTile), 0, S.stream, S.D, wr.tile_begin);
      else if (wr.narrow_only)
        hipLaunchKernelGGL((wave_kernel<DIR, MODE, true, true>), dim3(nt), dim3(kTile), 0, S.stream, S.D, wr.tile_begin);
      else if (!list)
        hipLaunchKernelGGL((wave_kernel<DIR, MODE, false, false>), dim3(nt), dim3(kTile), 0, S.stream, S.D, wr.tile_begin);
      else
        hipLaunchKernelGGL((wave_kernel<DIR, MODE, false, true>), dim3(nt), dim3(kTile), 0, S.stream, S.D, wr.tile_begin);
      if (int32_t rc = launched("wave kernel")) return rc;
    }
    if (nb > 0) {
      if (DIR == kBwd && wr.list)
        hipLaunchKernelGGL((wave_big_kernel<DIR, MODE, true>), dim3(nb), dim3(kTile), 0, S.stream, S.D, wr.big_begin);
      else
        hipLaunchKernelGGL((wave_big_kernel<DIR, MODE, false>), dim3(nb), dim3(kTile), 0, S.stream, S.D, wr.big_begin);
      if (int32_t rc = launched("wave kernel (big)")) return rc;
    }
    if (ev) {
      HIP_TRY(hipEventRecord(e.b, S.stream), "hipEventRecord");
      ev->push_back(e);
    }
  }
  return BDDMP_OK;
}

// the bound of the backward sweep just run, from its per-tile partials
int32_t record_lb(Solver &S, std::vector<EventPair> *ev) {
  const Plan &P = *S.plan;
  EventPair e{};
  if (ev) {
    HIP_TRY(hipEventCreate(&e.a), "hipEventCreate");
    HIP_TRY(hipEventCreate(&e.b), "hipEventCreate");
    e.cls = 2;
    HIP_TRY(hipEventRecord(e.a, S.stream), "hipEventRecord");
  }
  const int slot = int(S.n_hist % P.hist_cap);
  hipLaunchKernelGGL(lb_stage_kernel, dim3(kLbStage), dim3(256), 0, S.stream, S.D, int(P.n_lbpart));
  if (int32_t rc = launched("lb_stage")) return rc;
  hipLaunchKernelGGL(lb_final_kernel, dim3(1), dim3(kLbStage), 0, S.stream, S.D, P.lb_const, slot);
  if (int32_t rc = launched("lb_final")) return rc;
  if (ev) {
    HIP_TRY(hipEventRecord(e.b, S.stream), "hipEventRecord");
    ev->push_back(e);
  }
  S.n_hist++;
  return BDDMP_OK;
}

int32_t initial_sweep(Solver &S) {
  if (int32_t rc = run_pass<kBwd, kNoUpdate>(S, nullptr, 1)) return rc;
  return record_lb(S, nullptr);
}

int32_t one_iteration(Solver &S, std::vector<EventPair> *ev) {
  if (int32_t rc = run_pass<kFwd, kUpdate>(S, ev, 0)) return rc;
  if (int32_t rc = run_pass<kBwd, kUpdate>(S, ev, 1)) return rc;
  return record_lb(S, ev);
}

}  // namespace

int32_t solver_bind(const Plan &P, void *arena, size_t bytes, void *stream, Solver *&out) {
  out = nullptr;
  if (P.lay.total && !arena) return set_error(BDDMP_INVALID_ARG, "null device arena");
  if (bytes < P.lay.total)
    return set_error(BDDMP_INVALID_ARG, "arena too small: need " + std::to_string(P.lay.total) + " bytes");
  if (reinterpret_cast<uintptr_t>(arena) % 256) return set_error(BDDMP_INVALID_ARG, "arena not 256-byte aligned");
  auto *S = new Solver();
  S->plan = &P;
  S->arena = static_cast<char *>(arena);
  S->stream = static_cast<hipStream_t>(stream);
  const ArenaLayout &A = P.lay;
  char *b = S->arena;
  Dev &D = S->D;
  D.meta = reinterpret_cast<const uint32_t *>(b + A.meta);
  D.child = reinterpret_cast<const int32_t *>(b + A.child);
  D.parent = reinterpret_cast<const int32_t *>(b + A.parent);
  D.lam = reinterpret_cast<float *>(b + A.lam);
  D.mf = reinterpret_cast<float *>(b + A.mf);
  D.mbc = reinterpret_cast<float *>(b + A.mbc);
  D.garcs = reinterpret_cast<const uint32_t *>(b + A.garcs);
  D.grec = P.grec.empty() ? nullptr : reinterpret_cast<const int4 *>(b + A.grec);
  D.canon_of = reinterpret_cast<const int32_t *>(b + A.canon_of);
  D.layer_of = reinterpret_cast<const int32_t *>(b + A.layer_of);
  D.layer_var = reinterpret_cast<const int32_t *>(b + A.layer_var);
  D.root_slot = reinterpret_cast<const int32_t *>(b + A.root_slot);
  D.fwd_tiles = reinterpret_cast<const int32_t *>(b + A.fwd_tiles);
  D.bwd_tiles = reinterpret_cast<const int32_t *>(b + A.bwd_tiles);
  D.bwd_list = reinterpret_cast<const int32_t *>(b + A.bwd_list);
  D.fwd_big = reinterpret_cast<const int32_t *>(b + A.fwd_big);
  D.bwd_big = reinterpret_cast<const int32_t *>(b + A.bwd_big);
  D.bdd_canon_off = reinterpret_cast<const int32_t *>(b + A.bdd_canon_off);
  D.cost = reinterpret_cast<const double *>(b + A.cost);
  D.var_first = reinterpret_cast<const int32_t *>(b + A.var_first);
  D.var_nj = reinterpret_cast<const int32_t *>(b + A.var_nj);
  D.d_fresh = reinterpret_cast<float *>(b + A.d_fresh);
  D.mbuf = reinterpret_cast<float *>(b + A.mbuf);
  D.xbuf = reinterpret_cast<int8_t *>(b + A.xbuf);
  D.part = reinterpret_cast<double *>(b + A.part);
  D.lbpart = reinterpret_cast<double *>(b + A.lbpart);
  D.lb_hist = reinterpret_cast<double *>(b + A.lb_hist);
  D.scal = reinterpret_cast<double *>(b + A.scal);
  D.out0 = D.out1 = nullptr;
  D.n_bwd_tiles = int32_t(P.bwd_tiles.size() / 2);

  auto up = [&](size_t off, const void *src, size_t nbytes) -> hipError_t {
    if (!nbytes) return hipSuccess;
    return hipMemcpyAsync(b + off, src, nbytes, hipMemcpyHostToDevice, S->stream);
  };
  const hipError_t errs[] = {
      up(A.meta, P.meta.data(), 4 * P.meta.size()),
      up(A.child, P.child.data(), 4 * P.child.size()),
      up(A.parent, P.parent.data(), 4 * P.parent.size()),
      up(A.garcs, P.garcs.data(), 4 * P.garcs.size()),
      up(A.grec, P.grec.data(), 4 * P.grec.size()),
      up(A.canon_of, P.canon_of.data(), 4 * P.canon_of.size()),
      up(A.layer_of, P.layer_of.data(), 4 * P.layer_of.size()),
      up(A.layer_var, P.layer_var.data(), 4 * P.layer_var.size()),
      up(A.root_slot, P.root_slot.data(), 4 * P.root_slot.size()),
      up(A.fwd_tiles, P.fwd_tiles.data(), 4 * P.fwd_tiles.size()),
      up(A.bwd_tiles, P.bwd_tiles.data(), 4 * P.bwd_tiles.size()),
      up(A.bwd_list, P.bwd_list.data(), 4 * P.bwd_list.size()),
      up(A.fwd_big, P.fwd_big.data(), 4 * P.fwd_big.size()),
      up(A.bwd_big, P.bwd_big.data(), 4 * P.bwd_big.size()),
      up(A.bdd_canon_off, P.bdd_canon_off.data(), 4 * P.bdd_canon_off.size()),
      up(A.cost, P.cost.data(), 8 * P.cost.size()),
      up(A.var_first, P.var_first.data(), 4 * P.var_first.size()),
      up(A.var_nj, P.var_nj.data(), 4 * P.var_nj.size()),
  };
  for (hipError_t e : errs)
    if (e != hipSuccess) {
      delete S;
      return hip_fail(e, "hipMemcpyAsync (upload)");
    }
  if (const int32_t rc = solver_reset(*S)) {
    delete S;
    return rc;
  }
  out = S;
  return BDDMP_OK;
}

// Initialisation of Alg. "Min-marginal averaging": lambda^j_i = c_i / |J_i|, forward messages
// +inf except the roots (0; padding slots stay +inf), and the initial backward sweep that fills
// every backward message.
int32_t solver_reset(Solver &S) {
  const Plan &P = *S.plan;
  const int nslots = int(P.S + 4);
  hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(nslots, 256)), dim3(256), 0, S.stream, S.D.mf, INFINITY, nslots);
  if (int32_t rc = launched("fill")) return rc;
  const int ncslots = int(P.Sc + 4);
  hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(ncslots, 256)), dim3(256), 0, S.stream, S.D.mbc, INFINITY, ncslots);
  if (int32_t rc = launched("fill")) return rc;
  if (P.I > 0) {
    hipLaunchKernelGGL(init_lambda_kernel, dim3(blocks_for(P.I, 256)), dim3(256), 0, S.stream, S.D, int(P.I));
    if (int32_t rc = launched("init_lambda")) return rc;
  }
  if (P.m > 0) {
    hipLaunchKernelGGL(root_zero_kernel, dim3(blocks_for(P.m, 256)), dim3(256), 0, S.stream, S.D, P.m);
    if (int32_t rc = launched("root_zero")) return rc;
  }
  S.iters = 0;
  return initial_sweep(S);
}

int32_t solver_iterate(Solver &S, int32_t n) {
  if (n < 0) return set_error(BDDMP_INVALID_ARG, "negative iteration count");
  for (int32_t t = 0; t < n; ++t) {
    if (int32_t rc = one_iteration(S, nullptr)) return rc;
    S.iters++;
  }
  return BDDMP_OK;
}

int32_t solver_lower_bound(Solver &S, double *lb, double *residual, double *any_lambda_bound) {
  const Plan &P = *S.plan;
  double h = 0.0, sc[2] = {0.0, 0.0};
  const int slot = int((S.n_hist - 1) % P.hist_cap);
  HIP_TRY(hipMemcpyAsync(&h, S.D.lb_hist + slot, 8, hipMemcpyDeviceToHost, S.stream), "hipMemcpyAsync");
  if ((residual || any_lambda_bound) && P.n > 0) {
    hipLaunchKernelGGL(residual_partial_kernel, dim3(kLbBlocks), dim3(256), 0, S.stream, S.D, P.n);
    if (int32_t rc = launched("residual_partial")) return rc;
    hipLaunchKernelGGL(residual_final_kernel, dim3(1), dim3(kLbBlocks), 0, S.stream, S.D);
    if (int32_t rc = launched("residual_final")) return rc;
    HIP_TRY(hipMemcpyAsync(sc, S.D.scal, 16, hipMemcpyDeviceToHost, S.stream), "hipMemcpyAsync");
  }
  HIP_TRY(hipStreamSynchronize(S.stream), "hipStreamSynchronize");
  if (lb) *lb = h;
  if (residual) *residual = sc[0];
  if (any_lambda_bound) *any_lambda_bound = h + sc[1];
  if (std::isnan(h)) return set_error(BDDMP_NONFINITE, "lower bound is NaN");
  return BDDMP_OK;
}

int32_t solver_lb_history(Solver &S, double *out, int32_t cap, int32_t *n_out) {
  const Plan &P = *S.plan;
  const int64_t have = std::min<int64_t>(S.n_hist, P.hist_cap);
  const int64_t cnt = std::min<int64_t>(have, cap);
  std::vector<double> ring(size_t(P.hist_cap));
  HIP_TRY(hipMemcpyAsync(ring.data(), S.D.lb_hist, 8 * size_t(P.hist_cap), hipMemcpyDeviceToHost, S.stream),
          "hipMemcpyAsync");
  HIP_TRY(hipStreamSynchronize(S.stream), "hipStreamSynchronize");
  for (int64_t q = 0; q < cnt; ++q) {
    const int64_t idx = S.n_hist - cnt + q;
    out[q] = ring[size_t(idx % P.hist_cap)];
  }
  if (n_out) *n_out = int32_t(cnt);
  return BDDMP_OK;
}

int32_t solver_min_marginals(Solver &S, float *m0, float *m1) {
  S.D.out0 = m0;
  S.D.out1 = m1;
  const int32_t rc = run_pass<kFwd, kExtract>(S, nullptr, 0);
  S.D.out0 = S.D.out1 = nullptr;
  return rc;
}

int32_t solver_get_lambda(Solver &S, float *lam) {
  const Plan &P = *S.plan;
  if (P.I == 0) return BDDMP_OK;
  hipLaunchKernelGGL(lambda_out_kernel, dim3(blocks_for(P.I, 256)), dim3(256), 0, S.stream, S.D, lam, int(P.I));
  return launched("lambda_out");
}

int32_t solver_set_lambda(Solver &S, const float *lam) {
  const Plan &P = *S.plan;
  if (P.I > 0) {
    hipLaunchKernelGGL(lambda_in_kernel, dim3(blocks_for(P.I, 256)), dim3(256), 0, S.stream, S.D, lam, int(P.I));
    if (int32_t rc = launched("lambda_in")) return rc;
  }
  return initial_sweep(S);
}

int32_t solver_round_primal(Solver &S, float *M_dev, int8_t *x_host, double *obj, int64_t *nviol) {
  const Plan &P = *S.plan;
  if (int32_t rc = solver_min_marginals(S, nullptr, nullptr)) return rc;
  double sc[2] = {0.0, 0.0};
  // both partial kernels write every partial slot, also for empty inputs
  hipLaunchKernelGGL(round_var_kernel, dim3(kLbBlocks), dim3(256), 0, S.stream, S.D, P.n);
  if (int32_t rc = launched("round_var")) return rc;
  hipLaunchKernelGGL(violation_kernel, dim3(kLbBlocks), dim3(256), 0, S.stream, S.D, P.m);
  if (int32_t rc = launched("violation")) return rc;
  hipLaunchKernelGGL(round_final_kernel, dim3(1), dim3(kLbBlocks), 0, S.stream, S.D);
  if (int32_t rc = launched("round_final")) return rc;
  if (M_dev && P.n)
    HIP_TRY(hipMemcpyAsync(M_dev, S.D.mbuf, 4 * size_t(P.n), hipMemcpyDeviceToDevice, S.stream), "hipMemcpyAsync");
  if (x_host && P.n)
    HIP_TRY(hipMemcpyAsync(x_host, S.D.xbuf, size_t(P.n), hipMemcpyDeviceToHost, S.stream), "hipMemcpyAsync");
  HIP_TRY(hipMemcpyAsync(sc, S.D.scal + 2, 16, hipMemcpyDeviceToHost, S.stream), "hipMemcpyAsync");
  HIP_TRY(hipStreamSynchronize(S.stream), "hipStreamSynchronize");
  if (obj) *obj = sc[0];
  if (nviol) *nviol = int64_t(sc[1]);
  return BDDMP_OK;
}

int32_t solver_time_kernels(Solver &S, int32_t n, bddmp_kernel_times *out) {
  const Plan &P = *S.plan;
  std::vector<EventPair> ev;
  ev.reserve(size_t(n) * (P.fwd_waves.size() + P.bwd_waves.size() + 1));
  int32_t rc = BDDMP_OK;
  for (int32_t t = 0; t < n && !rc; ++t) {
    rc = one_iteration(S, &ev);
    S.iters++;
  }
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (!rc) {
    HIP_TRY(hipEventCreate(&t0), "hipEventCreate");
    HIP_TRY(hipEventCreate(&t1), "hipEventCreate");
    HIP_TRY(hipEventRecord(t0, S.stream), "hipEventRecord");
    for (int32_t t = 0; t < n && !rc; ++t) {
      rc = one_iteration(S, nullptr);
      S.iters++;
    }
    HIP_TRY(hipEventRecord(t1, S.stream), "hipEventRecord");
  }
  const hipError_t se = hipStreamSynchronize(S.stream);
  bddmp_kernel_times r{};
  for (const EventPair &e : ev) {
    float ms = 0.0f;
    if (!rc && se == hipSuccess) hipEventElapsedTime(&ms, e.a, e.b);
    if (e.cls == 0) {
      r.fwd_ms += ms;
      r.fwd_launches++;
    } else if (e.cls == 1) {
      r.bwd_ms += ms;
      r.bwd_launches++;
    } else {
      r.lb_ms += ms;
      r.lb_launches++;
    }
    hipEventDestroy(e.a);
    hipEventDestroy(e.b);
  }
  if (!rc && se == hipSuccess && t0) {
    float ms = 0.0f;
    hipEventElapsedTime(&ms, t0, t1);
    r.iter_ms = n ? ms / n : 0.0;
  }
  if (t0) hipEventDestroy(t0);
  if (t1) hipEventDestroy(t1);
  if (rc) return rc;
  if (se != hipSuccess) return hip_fail(se, "hipStreamSynchronize");
  const double pass_bytes = 20.0 * double(P.N) + 8.0 * double(P.I);
  r.fwd_bytes = pass_bytes * n;
  r.bwd_bytes = pass_bytes * n;
  *out = r;
  return BDDMP_OK;
}

void solver_destroy(Solver *S) { delete S; }

}  // namespace bddmp
