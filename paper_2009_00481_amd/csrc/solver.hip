// Device side of bddmp: wave kernels for the forward and backward passes, the fp64 bound, and the
// output kernels, plus the solver's host code that enqueues them on the caller's stream.
//
// One wave kernel launch runs every layer (one BDD level of one row) whose variable belongs to the
// wave. A workgroup takes a tile of up to 256 consecutive layers; a variable's layers (its rows
// J_i, ascending) never straddle tiles, so the J_i sum is a workgroup-local LDS reduction. One
// lane handles one layer: narrow levels (<= 4 nodes, the MRF / matching / tracking shapes) keep
// their nodes in registers; wider ones loop over nodes. Loads are coalesced because consecutive
// lanes own consecutive layers, whose nodes are consecutive in the forward-wave-major layout.
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
  const uint32_t *arcs;
  float *mf, *mb;
  const int32_t *node_off, *child_off;
  float *lam;
  const uint32_t *seg;
  const int32_t *canon_of, *layer_of, *layer_var;
  const int32_t *fwd_tiles, *bwd_tiles, *bwd_list, *fwd_big, *bwd_big;
  const int32_t *root_node, *bdd_canon_off;
  const double *cost;
  const int32_t *var_first, *var_nj;
  float *d_fresh, *mbuf;
  int8_t *xbuf;
  double *part;
  long long *ipart;
  double *lb_hist, *scal;
  float *out0, *out1;
};

// backward message of a child: its value, 0 for the true terminal, +inf for the false terminal
__device__ __forceinline__ float child_val(const float *__restrict__ mb, int co, uint32_t c) {
  return c < kTop ? mb[co + int(c)] : (c == kTop ? 0.0f : INFINITY);
}

// arc-marginals of one level, minimised per arc label (eqs. "arc-marginal", "marginal-aggregation")
__device__ __forceinline__ void level_mm_loop(const Dev &D, int no, int w, int co, float lam0, float &m0, float &m1) {
  for (int u = 0; u < w; ++u) {
    const uint32_t a = D.arcs[no + u];
    const float f = D.mf[no + u];
    m0 = fminf(m0, f + child_val(D.mb, co, a & 0xFFFFu));
    m1 = fminf(m1, (f + lam0) + child_val(D.mb, co, a >> 16));
  }
}

// forward step of the next level (Alg. "Forward BDD update step"), pushed from this level: the
// lane owns the whole child level, so the min over in-arcs needs no synchronisation
__device__ __noinline__ void push_loop(const Dev &D, int no, int w, int co, float lam1) {
  int wc = 0;
  for (int u = 0; u < w; ++u) {
    const uint32_t a = D.arcs[no + u];
    const uint32_t lo = a & 0xFFFFu, hi = a >> 16;
    if (lo < kTop) wc = max(wc, int(lo) + 1);
    if (hi < kTop) wc = max(wc, int(hi) + 1);
  }
  for (int q = 0; q < wc; ++q) D.mf[co + q] = INFINITY;
  for (int u = 0; u < w; ++u) {
    const uint32_t a = D.arcs[no + u];
    const uint32_t lo = a & 0xFFFFu, hi = a >> 16;
    const float f = D.mf[no + u];
    if (lo < kTop) D.mf[co + int(lo)] = fminf(D.mf[co + int(lo)], f);
    if (hi < kTop) D.mf[co + int(hi)] = fminf(D.mf[co + int(hi)], f + lam1);
  }
}

// backward step of this level (Alg. "Backward BDD update step") with the updated multiplier
__device__ __noinline__ void bwd_step_loop(const Dev &D, int no, int w, int co, float lam1) {
  for (int u = 0; u < w; ++u) {
    const uint32_t a = D.arcs[no + u];
    D.mb[no + u] = fminf(child_val(D.mb, co, a & 0xFFFFu), child_val(D.mb, co, a >> 16) + lam1);
  }
}

// multiplier update of eq. "mma-update"; rows forcing the variable (infinite difference) absorb
// the finite differences of the others
__device__ __forceinline__ float updated(float lam0, float d, float share, int nf) {
  return nf == 0 ? (lam0 - d) + share : (isinf(d) ? lam0 + share : lam0 - d);
}

template <int DIR, int MODE>
__global__ __launch_bounds__(kTile) void wave_kernel(const Dev D, const int tile0, const int use_list) {
  __shared__ float s_d[kTile];
  __shared__ float s_share[kTile];
  __shared__ int s_nf[kTile];
  const int32_t *tiles = DIR == kFwd ? D.fwd_tiles : D.bwd_tiles;
  const int tix = tile0 + int(blockIdx.x);
  const int p0 = tiles[2 * tix];
  const int cnt = tiles[2 * tix + 1] - p0;
  const int s = int(threadIdx.x);
  const bool active = s < cnt;

  int L = 0, no = 0, w = 0, co = -1;
  float lam0 = 0.0f;
  uint32_t sg = 0;
  uint32_t ar[4] = {kBot, kBot, kBot, kBot};
  float f[4] = {0.f, 0.f, 0.f, 0.f}, b0[4] = {0.f, 0.f, 0.f, 0.f}, b1[4] = {0.f, 0.f, 0.f, 0.f};
  float m0 = INFINITY, m1 = INFINITY;
  if (active) {
    L = (DIR == kBwd && use_list) ? D.bwd_list[p0 + s] : p0 + s;
    no = D.node_off[L];
    w = D.node_off[L + 1] - no;
    co = D.child_off[L];
    lam0 = D.lam[L];
    if (MODE == kUpdate) sg = D.seg[L];
    if (w <= 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (u < w) {
          ar[u] = D.arcs[no + u];
          f[u] = D.mf[no + u];
          b0[u] = child_val(D.mb, co, ar[u] & 0xFFFFu);
          b1[u] = child_val(D.mb, co, ar[u] >> 16);
          m0 = fminf(m0, f[u] + b0[u]);
          m1 = fminf(m1, (f[u] + lam0) + b1[u]);
        }
      }
    } else {
      level_mm_loop(D, no, w, co, lam0, m0, m1);
    }
  }
  const float d = m1 - m0;
  float lam1 = lam0;
  if (MODE == kUpdate) {
    s_d[s] = d;
    __syncthreads();
    const int pos = int(sg & 0xFFFFu), len = int(sg >> 16);
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
      lam1 = updated(lam0, d, s_share[h], s_nf[h]);
      D.lam[L] = lam1;
    }
  }
  if (!active) return;
  if (MODE == kExtract) {
    const int c = D.canon_of[L];
    if (D.out0) D.out0[c] = m0;
    if (D.out1) D.out1[c] = m1;
    D.d_fresh[L] = d;
  }
  if (DIR == kFwd) {
    if (co < 0) return;
    if (w <= 4) {
      float c[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
      int wc = 0;
      bool fits = true;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (u < w) {
          const uint32_t lo = ar[u] & 0xFFFFu, hi = ar[u] >> 16;
          const float v0 = f[u], v1 = f[u] + lam1;
          if (lo < kTop) {
            wc = max(wc, int(lo) + 1);
            fits = fits && lo < 4u;
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (lo == uint32_t(q)) c[q] = fminf(c[q], v0);
          }
          if (hi < kTop) {
            wc = max(wc, int(hi) + 1);
            fits = fits && hi < 4u;
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (hi == uint32_t(q)) c[q] = fminf(c[q], v1);
          }
        }
      }
      if (fits) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q < wc) D.mf[co + q] = c[q];
      } else {
        push_loop(D, no, w, co, lam1);
      }
    } else {
      push_loop(D, no, w, co, lam1);
    }
  } else {
    if (w <= 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (u < w) D.mb[no + u] = fminf(b0[u], b1[u] + lam1);
    } else {
      bwd_step_loop(D, no, w, co, lam1);
    }
  }
}

// One variable with more than kTile rows per workgroup (its layers are the whole tile).
template <int DIR, int MODE>
__global__ __launch_bounds__(kTile) void wave_big_kernel(const Dev D, const int big0, const int use_list) {
  __shared__ float s_d[kBigMax];
  __shared__ float s_share;
  __shared__ int s_nf;
  const int32_t *big = DIR == kFwd ? D.fwd_big : D.bwd_big;
  const int b = big0 + int(blockIdx.x);
  const int p0 = big[2 * b];
  const int cnt = big[2 * b + 1] - p0;
  for (int s = int(threadIdx.x); s < cnt; s += kTile) {
    const int L = (DIR == kBwd && use_list) ? D.bwd_list[p0 + s] : p0 + s;
    const int no = D.node_off[L], w = D.node_off[L + 1] - no, co = D.child_off[L];
    float m0 = INFINITY, m1 = INFINITY;
    level_mm_loop(D, no, w, co, D.lam[L], m0, m1);
    s_d[s] = m1 - m0;
    if (MODE == kExtract) {
      const int c = D.canon_of[L];
      if (D.out0) D.out0[c] = m0;
      if (D.out1) D.out1[c] = m1;
      D.d_fresh[L] = m1 - m0;
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
  for (int s = int(threadIdx.x); s < cnt; s += kTile) {
    const int L = (DIR == kBwd && use_list) ? D.bwd_list[p0 + s] : p0 + s;
    const int no = D.node_off[L], w = D.node_off[L + 1] - no, co = D.child_off[L];
    float lam1 = D.lam[L];
    if (MODE == kUpdate) {
      lam1 = updated(lam1, s_d[s], s_share, s_nf);
      D.lam[L] = lam1;
    }
    if (DIR == kFwd) {
      if (co >= 0) push_loop(D, no, w, co, lam1);
    } else {
      bwd_step_loop(D, no, w, co, lam1);
    }
  }
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
  const int r = D.root_node[j];
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

// fixed-shape block tree sum of 256 doubles
__device__ __forceinline__ double block_sum256(double v, double *sh) {
  const int t = int(threadIdx.x);
  sh[t] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_max256(double v, double *sh) {
  const int t = int(threadIdx.x);
  sh[t] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// LB = sum_j E^j, E^j = backward message of the root (problem (D)); fixed partition and tree
__global__ __launch_bounds__(256) void lb_partial_kernel(const Dev D, int m) {
  __shared__ double sh[256];
  const int chunk = (m + kLbBlocks - 1) / kLbBlocks;
  const int j0 = int(blockIdx.x) * chunk, j1 = min(m, j0 + chunk);
  double acc = 0.0;
  for (int j = j0 + int(threadIdx.x); j < j1; j += 256) {
    const int r = D.root_node[j];
    if (r >= 0) acc += double(D.mb[r]);
  }
  const double s = block_sum256(acc, sh);
  if (threadIdx.x == 0) D.part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kLbBlocks) void lb_final_kernel(const Dev D, double lb_const, int slot) {
  __shared__ double sh[kLbBlocks];
  const int t = int(threadIdx.x);
  sh[t] = D.part[t];
  __syncthreads();
  for (int s = kLbBlocks / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  if (t == 0) D.lb_hist[slot] = sh[0] + lb_const;
}

// per variable: g_i = c_i - sum_j lambda^j_i; partial max |g| and sum of min(0, g)
__global__ __launch_bounds__(256) void residual_partial_kernel(const Dev D, int n) {
  __shared__ double sh[256];
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
  const double a = block_max256(mx, sh);
  const double b = block_sum256(corr, sh);
  if (threadIdx.x == 0) {
    D.part[blockIdx.x] = a;
    D.part[kLbBlocks + blockIdx.x] = b;
  }
}

__global__ __launch_bounds__(kLbBlocks) void residual_final_kernel(const Dev D) {
  __shared__ double sa[kLbBlocks], sb[kLbBlocks];
  const int t = int(threadIdx.x);
  sa[t] = D.part[t];
  sb[t] = D.part[kLbBlocks + t];
  __syncthreads();
  for (int s = kLbBlocks / 2; s > 0; s >>= 1) {
    if (t < s) {
      sa[t] = fmax(sa[t], sa[t + s]);
      sb[t] += sb[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    D.scal[0] = sa[0];
    D.scal[1] = sb[0];
  }
}

// M_i = sum_j (m1 - m0) in ascending row order (Sec. 4), x_i = [M_i <= 0]; c^T x partials
__global__ __launch_bounds__(256) void round_var_kernel(const Dev D, int n) {
  __shared__ double sh[256];
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
  const double s = block_sum256(obj, sh);
  if (threadIdx.x == 0) D.part[blockIdx.x] = s;
}

// a row holds at x iff x's path through its BDD ends in the true terminal (Prop. "Canonicity")
__global__ __launch_bounds__(256) void violation_kernel(const Dev D, int m) {
  __shared__ double sh[256];
  const int chunk = (m + kLbBlocks - 1) / kLbBlocks;
  const int j0 = int(blockIdx.x) * chunk, j1 = min(m, j0 + chunk);
  double bad = 0.0;
  for (int j = j0 + int(threadIdx.x); j < j1; j += 256) {
    const int c0 = D.bdd_canon_off[j], c1 = D.bdd_canon_off[j + 1];
    int cur = 0;
    for (int c = c0; c < c1; ++c) {
      const int L = D.layer_of[c];
      const uint32_t a = D.arcs[D.node_off[L] + cur];
      const uint32_t ch = D.xbuf[D.layer_var[L]] ? (a >> 16) : (a & 0xFFFFu);
      if (ch == kBot) {
        bad += 1.0;
        break;
      }
      cur = ch == kTop ? 0 : int(ch);
    }
  }
  const double s = block_sum256(bad, sh);
  if (threadIdx.x == 0) D.part[kLbBlocks + blockIdx.x] = s;
}

__global__ __launch_bounds__(kLbBlocks) void round_final_kernel(const Dev D) {
  __shared__ double sa[kLbBlocks], sb[kLbBlocks];
  const int t = int(threadIdx.x);
  sa[t] = D.part[t];
  sb[t] = D.part[kLbBlocks + t];
  __syncthreads();
  for (int s = kLbBlocks / 2; s > 0; s >>= 1) {
    if (t < s) {
      sa[t] += sa[t + s];
      sb[t] += sb[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    D.scal[2] = sa[0];
    D.scal[3] = sb[0];
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

#define HIP_TRY(expr, what)                 \
  do {                                      \
    hipError_t e_ = (expr);                 \
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

// One pass: every wave in order; ev != nullptr records an event pair around each launch.
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
      hipLaunchKernelGGL((wave_kernel<DIR, MODE>), dim3(nt), dim3(kTile), 0, S.stream, S.D, wr.tile_begin, wr.list);
      if (int32_t rc = launched("wave kernel")) return rc;
    }
    if (nb > 0) {
      hipLaunchKernelGGL((wave_big_kernel<DIR, MODE>), dim3(nb), dim3(kTile), 0, S.stream, S.D, wr.big_begin, wr.list);
      if (int32_t rc = launched("wave kernel (big)")) return rc;
    }
    if (ev) {
      HIP_TRY(hipEventRecord(e.b, S.stream), "hipEventRecord");
      ev->push_back(e);
    }
  }
  return BDDMP_OK;
}

int32_t record_lb(Solver &S, std::vector<EventPair> *ev) {
  const Plan &P = *S.plan;
  EventPair e{};
  if (ev) {
    HIP_TRY(hipEventCreate(&e.a), "hipEventCreate");
    HIP_TRY(hipEventCreate(&e.b), "hipEventCreate");
    e.cls = 2;
    HIP_TRY(hipEventRecord(e.a, S.stream), "hipEventRecord");
  }
  hipLaunchKernelGGL(lb_partial_kernel, dim3(kLbBlocks), dim3(256), 0, S.stream, S.D, P.m);
  if (int32_t rc = launched("lb_partial")) return rc;
  const int slot = int(S.n_hist % P.hist_cap);
  hipLaunchKernelGGL(lb_final_kernel, dim3(1), dim3(kLbBlocks), 0, S.stream, S.D, P.lb_const, slot);
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
  D.arcs = reinterpret_cast<const uint32_t *>(b + A.arcs);
  D.mf = reinterpret_cast<float *>(b + A.mf);
  D.mb = reinterpret_cast<float *>(b + A.mb);
  D.node_off = reinterpret_cast<const int32_t *>(b + A.node_off);
  D.child_off = reinterpret_cast<const int32_t *>(b + A.child_off);
  D.lam = reinterpret_cast<float *>(b + A.lam);
  D.seg = reinterpret_cast<const uint32_t *>(b + A.seg);
  D.canon_of = reinterpret_cast<const int32_t *>(b + A.canon_of);
  D.layer_of = reinterpret_cast<const int32_t *>(b + A.layer_of);
  D.layer_var = reinterpret_cast<const int32_t *>(b + A.layer_var);
  D.fwd_tiles = reinterpret_cast<const int32_t *>(b + A.fwd_tiles);
  D.bwd_tiles = reinterpret_cast<const int32_t *>(b + A.bwd_tiles);
  D.bwd_list = reinterpret_cast<const int32_t *>(b + A.bwd_list);
  D.fwd_big = reinterpret_cast<const int32_t *>(b + A.fwd_big);
  D.bwd_big = reinterpret_cast<const int32_t *>(b + A.bwd_big);
  D.root_node = reinterpret_cast<const int32_t *>(b + A.root_node);
  D.bdd_canon_off = reinterpret_cast<const int32_t *>(b + A.bdd_canon_off);
  D.cost = reinterpret_cast<const double *>(b + A.cost);
  D.var_first = reinterpret_cast<const int32_t *>(b + A.var_first);
  D.var_nj = reinterpret_cast<const int32_t *>(b + A.var_nj);
  D.d_fresh = reinterpret_cast<float *>(b + A.d_fresh);
  D.mbuf = reinterpret_cast<float *>(b + A.mbuf);
  D.xbuf = reinterpret_cast<int8_t *>(b + A.xbuf);
  D.part = reinterpret_cast<double *>(b + A.part);
  D.ipart = reinterpret_cast<long long *>(b + A.ipart);
  D.lb_hist = reinterpret_cast<double *>(b + A.lb_hist);
  D.scal = reinterpret_cast<double *>(b + A.scal);
  D.out0 = D.out1 = nullptr;

  auto up = [&](size_t off, const void *src, size_t nbytes) -> hipError_t {
    if (!nbytes) return hipSuccess;
    return hipMemcpyAsync(b + off, src, nbytes, hipMemcpyHostToDevice, S->stream);
  };
  const hipError_t errs[] = {
      up(A.arcs, P.arcs.data(), 4 * P.arcs.size()),
      up(A.node_off, P.node_off.data(), 4 * P.node_off.size()),
      up(A.child_off, P.child_off.data(), 4 * P.child_off.size()),
      up(A.seg, P.seg.data(), 4 * P.seg.size()),
      up(A.canon_of, P.canon_of.data(), 4 * P.canon_of.size()),
      up(A.layer_of, P.layer_of.data(), 4 * P.layer_of.size()),
      up(A.layer_var, P.layer_var.data(), 4 * P.layer_var.size()),
      up(A.fwd_tiles, P.fwd_tiles.data(), 4 * P.fwd_tiles.size()),
      up(A.bwd_tiles, P.bwd_tiles.data(), 4 * P.bwd_tiles.size()),
      up(A.bwd_list, P.bwd_list.data(), 4 * P.bwd_list.size()),
      up(A.fwd_big, P.fwd_big.data(), 4 * P.fwd_big.size()),
      up(A.bwd_big, P.bwd_big.data(), 4 * P.bwd_big.size()),
      up(A.root_node, P.root_node.data(), 4 * P.root_node.size()),
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

// Initialisation of Alg. "Min-marginal averaging": lambda^j_i = c_i / |J_i|, forward messages of
// the roots = 0, and the initial backward sweep that fills every backward message.
int32_t solver_reset(Solver &S) {
  const Plan &P = *S.plan;
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
  if (residual || any_lambda_bound) {
    if (P.n > 0) {
      hipLaunchKernelGGL(residual_partial_kernel, dim3(kLbBlocks), dim3(256), 0, S.stream, S.D, P.n);
      if (int32_t rc = launched("residual_partial")) return rc;
      hipLaunchKernelGGL(residual_final_kernel, dim3(1), dim3(kLbBlocks), 0, S.stream, S.D);
      if (int32_t rc = launched("residual_final")) return rc;
      HIP_TRY(hipMemcpyAsync(sc, S.D.scal, 16, hipMemcpyDeviceToHost, S.stream), "hipMemcpyAsync");
    }
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
    if (e.cls == 0) { r.fwd_ms += ms; r.fwd_launches++; }
    else if (e.cls == 1) { r.bwd_ms += ms; r.bwd_launches++; }
    else { r.lb_ms += ms; r.lb_launches++; }
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
