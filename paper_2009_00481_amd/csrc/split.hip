// Copy-arc kernels of the sub-BDD split (Sec. 6, Def. "Sub-BDD", Def. "Copy-arc", Alg. "Parallel
// min-marginal averaging"). The wave kernels run every sub-BDD like a whole diagram: an exit layer
// reads the duals mu_bar of its copy-arcs (arcs into TOP) from its virtual child slots, and a cut
// root level holds the forward messages that the arc duals mu give it. Between the passes, these
// kernels update both duals: a narrow cut (both levels at most 2 nodes) per lane, a wide cut per
// wavefront. Arc q of a cut is arc (q / 2, q % 2) of its exit level.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.h"
#include "kernels.h"

namespace bddmp {

namespace {

// backward message of node v of a cut root level with the level's current multiplier (Alg.
// "Backward BDD update step", the operations of the wave kernels' step)
__device__ __forceinline__ float root_bwd(const Dev &D, int os, int cs, float lam, int v) {
  const uint32_t a = D.garcs[os + v];
  return fminf(c16val(D.mbc, cs, a & 0xFFFFu), c16val(D.mbc, cs, a >> 16) + lam);
}

__global__ __launch_bounds__(256) void copy_init_kernel(const Dev D, int nc) {
  const int c = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (c >= nc) return;
  const int4 k = D.cuts[c], sl = D.cut_slots[c];
  const int w2 = 2 * (k.w & 0xFFFF);
  for (int q = 0; q < w2; ++q) {
    D.mu_in[k.z + q] = 0.0f;
    D.dfw[k.z + q] = 0.0f;
    D.dbw[k.z + q] = 0.0f;
    D.mbc[sl.y + q] = 0.0f;
  }
}

// Forward copy-arc update (after the forward pass): each copy-arc's marginal in the sub-BDD it
// closes, (m_fwd(u) + theta) + mu_bar (theta with the exit level's updated multiplier), minus the
// smallest over the cut gives delta_fwd >= 0; mu_bar <- (mu_bar - gamma delta_fwd) + gamma delta_bwd
// (the last backward update).
//
// Narrow cuts (at most 4 arcs): one lane each, arcs unrolled.
__global__ __launch_bounds__(256) void copy_fwd_narrow_kernel(const Dev D, int nn) {
#pragma clang fp contract(off)
  const int c = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (c >= nn) return;
  const int4 k = D.cuts[c], sl = D.cut_slots[c];
  const int w2 = 2 * (k.w & 0xFFFF), base = k.z;
  const float lam = D.lam[k.x], g = D.gamma;
  float m[4];
  bool live[4];
  float mn = INFINITY;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    live[q] = q < w2 && D.cut_arc[base + q] != kBot;
    m[q] = INFINITY;
    if (live[q]) {
      const float th = (q & 1) ? lam : 0.0f;
      m[q] = (D.mf[sl.x + (q >> 1)] + th) + D.mbc[sl.y + q];
    }
    mn = fminf(mn, m[q]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (!live[q]) continue;
    const float d = m[q] - mn;
    D.dfw[base + q] = d;
    D.mbc[sl.y + q] = (D.mbc[sl.y + q] - g * d) + g * D.dbw[base + q];
  }
}

// Wide cuts: one wavefront each (kCutsPerBlock per workgroup), lanes over the arcs, the minimum
// by a butterfly over the wavefront (min is exact, so the split among lanes does not matter).
__global__ __launch_bounds__(256) void copy_fwd_wide_kernel(const Dev D, int nn, int nc) {
#pragma clang fp contract(off)
  const int lane = int(threadIdx.x) & 63;
  const int c = nn + int(blockIdx.x) * kCutsPerBlock + (int(threadIdx.x) >> 6);
  if (c >= nc) return;  // uniform over the wavefront
  const int4 k = D.cuts[c], sl = D.cut_slots[c];
  const int w2 = 2 * (k.w & 0xFFFF), base = k.z;
  const float lam = D.lam[k.x], g = D.gamma;
  float mn = INFINITY;
  for (int q = lane; q < w2; q += 64) {
    if (D.cut_arc[base + q] == kBot) continue;
    const float th = (q & 1) ? lam : 0.0f;
    mn = fminf(mn, (D.mf[sl.x + (q >> 1)] + th) + D.mbc[sl.y + q]);
  }
  for (int o = 32; o > 0; o >>= 1) mn = fminf(mn, __shfl_xor(mn, o, 64));
  for (int q = lane; q < w2; q += 64) {
    if (D.cut_arc[base + q] == kBot) continue;
    const float th = (q & 1) ? lam : 0.0f;
    const float mb = D.mbc[sl.y + q];
    const float d = ((D.mf[sl.x + (q >> 1)] + th) + mb) - mn;
    D.dfw[base + q] = d;
    D.mbc[sl.y + q] = (mb - g * d) + g * D.dbw[base + q];
  }
}

// Backward copy-arc update (after the backward pass): each arc's marginal in the sub-BDD it opens,
// mu + m_bwd(v), minus the smallest over the cut gives delta_bwd >= 0; mu <- (mu - gamma delta_bwd)
// + gamma delta_fwd (this iteration's forward update). Then the root level's forward messages (the
// minimum of mu over each node's in-arcs) and the sub-BDD's E (the minimum over its nodes of
// m_fwd + m_bwd, which is the minimum over the arcs of mu + m_bwd(v)) for the bound, one
// fixed-shape sum per workgroup into lbpart. update = 0 skips the dual update.
__global__ __launch_bounds__(256) void copy_bwd_narrow_kernel(const Dev D, int nn, int update, int part0) {
#pragma clang fp contract(off)
  __shared__ double sh[4];
  const int c = int(blockIdx.x) * 256 + int(threadIdx.x);
  double e = 0.0;
  if (c < nn) {
    const int4 k = D.cuts[c], sl = D.cut_slots[c];
    const int w2 = 2 * (k.w & 0xFFFF), wr = int(uint32_t(k.w) >> 16), base = k.z;
    const float lam = D.lam[k.y], g = D.gamma;
    const float n0 = root_bwd(D, sl.z, sl.w, lam, 0);
    const float n1 = wr > 1 ? root_bwd(D, sl.z, sl.w, lam, 1) : INFINITY;
    float mu[4], nv[4];
    uint32_t v[4];
    float mn = INFINITY;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q] = q < w2 ? uint32_t(D.cut_arc[base + q]) : kBot;
      mu[q] = INFINITY;
      nv[q] = v[q] ? n1 : n0;
      if (v[q] != kBot) {
        mu[q] = D.mu_in[base + q];
        mn = fminf(mn, mu[q] + nv[q]);
      }
    }
    if (update) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (v[q] == kBot) continue;
        const float d = (mu[q] + nv[q]) - mn;
        D.dbw[base + q] = d;
        mu[q] = (mu[q] - g * d) + g * D.dfw[base + q];
        D.mu_in[base + q] = mu[q];
      }
    }
    float f0 = INFINITY, f1 = INFINITY;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (v[q] == 0u) f0 = fminf(f0, mu[q]);
      if (v[q] == 1u) f1 = fminf(f1, mu[q]);
    }
    D.mf[sl.z] = f0;
    if (wr > 1) D.mf[sl.z + 1] = f1;
    const float en = fminf(f0 + n0, f1 + n1);
    D.cut_e[c] = en;
    e = double(en);
  }
  const double t = block_sum(e, sh);
  if (threadIdx.x == 0) D.lbpart[part0 + int(blockIdx.x)] = t;
}

__global__ __launch_bounds__(256) void copy_bwd_wide_kernel(const Dev D, int nn, int nc, int update, int part0) {
#pragma clang fp contract(off)
  __shared__ double sh[4];
  const int lane = int(threadIdx.x) & 63;
  const int c = nn + int(blockIdx.x) * kCutsPerBlock + (int(threadIdx.x) >> 6);
  const bool on = c < nc;  // uniform over the wavefront; every lane reaches the barriers
  int4 k = make_int4(0, 0, 0, 0), sl = make_int4(0, 0, 0, 0);
  float lam = 0.0f;
  if (on) {
    k = D.cuts[c];
    sl = D.cut_slots[c];
    lam = D.lam[k.y];
  }
  const int w2 = 2 * (k.w & 0xFFFF), wr = int(uint32_t(k.w) >> 16), base = k.z;
  if (update) {
    const float g = D.gamma;
    float mn = INFINITY;
    for (int q = lane; q < w2; q += 64) {
      const uint32_t v = D.cut_arc[base + q];
      if (v == kBot) continue;
      mn = fminf(mn, D.mu_in[base + q] + root_bwd(D, sl.z, sl.w, lam, int(v)));
    }
    for (int o = 32; o > 0; o >>= 1) mn = fminf(mn, __shfl_xor(mn, o, 64));
    for (int q = lane; q < w2; q += 64) {
      const uint32_t v = D.cut_arc[base + q];
      if (v == kBot) continue;
      const float mu = D.mu_in[base + q];
      const float d = (mu + root_bwd(D, sl.z, sl.w, lam, int(v))) - mn;
      D.dbw[base + q] = d;
      D.mu_in[base + q] = (mu - g * d) + g * D.dfw[base + q];
    }
  }
  __syncthreads();  // the new duals of every lane before the in-arc minima read them
  float en = INFINITY;
  if (on) {
    const int rb = D.cut_rb[c];
    for (int v = lane; v < wr; v += 64) {
      // forward message of root node v: the minimum of mu over its in-arcs (arc index 2u + label)
      float f = INFINITY;
      const uint32_t pk = D.rin[rb + v];
      if (pk != kManyInArcs) {
        const uint32_t a0 = pk & 0xFFFFu, a1 = pk >> 16;
        f = D.mu_in[base + 2 * int(a0 & (kInArcHi - 1u)) + ((a0 & kInArcHi) ? 1 : 0)];
        if (a1 != kNoArc16) f = fminf(f, D.mu_in[base + 2 * int(a1 & (kInArcHi - 1u)) + ((a1 & kInArcHi) ? 1 : 0)]);
      } else {
        for (int q = D.rbeg[rb + v]; q < D.rbeg[rb + v + 1]; ++q) {
          const uint32_t a = D.rarc[q];
          f = fminf(f, D.mu_in[base + 2 * int(a & (kInArcHi - 1u)) + ((a & kInArcHi) ? 1 : 0)]);
        }
      }
      D.mf[sl.z + v] = f;
      en = fminf(en, f + root_bwd(D, sl.z, sl.w, lam, v));
    }
  }
  for (int o = 32; o > 0; o >>= 1) en = fminf(en, __shfl_xor(en, o, 64));
  if (on && lane == 0) D.cut_e[c] = en;
  const double t = block_sum((on && lane == 0) ? double(en) : 0.0, sh);
  if (threadIdx.x == 0) D.lbpart[part0 + int(blockIdx.x)] = t;
}

// copy state per live pair in canonical order (cuts by row and level, then arc index)
__global__ __launch_bounds__(256) void copy_io_kernel(const Dev D, int nc, int out, float *mub, float *mu, float *df,
                                                      float *db) {
  const int c = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (c >= nc) return;
  const int4 k = D.cuts[c], sl = D.cut_slots[c];
  const int w2 = 2 * (k.w & 0xFFFF), base = k.z;
  int p = D.cut_live[c];
  for (int q = 0; q < w2; ++q) {
    if (D.cut_arc[base + q] == kBot) continue;
    if (out) {
      if (mub) mub[p] = D.mbc[sl.y + q];
      if (mu) mu[p] = D.mu_in[base + q];
      if (df) df[p] = D.dfw[base + q];
      if (db) db[p] = D.dbw[base + q];
    } else {
      D.mbc[sl.y + q] = mub[p];
      D.mu_in[base + q] = mu[p];
      D.dfw[base + q] = df[p];
      D.dbw[base + q] = db[p];
    }
    ++p;
  }
}

int blocks_of(int n) { return (n + 255) / 256; }

}  // namespace

hipError_t launch_copy_init(const Dev &D, int n_cuts, hipStream_t s) {
  if (n_cuts <= 0) return hipSuccess;
  copy_init_kernel<<<blocks_of(n_cuts), 256, 0, s>>>(D, n_cuts);
  return hipGetLastError();
}

hipError_t launch_copy_fwd(const Dev &D, int n_cuts, int n_narrow, hipStream_t s) {
  if (n_narrow > 0) copy_fwd_narrow_kernel<<<blocks_of(n_narrow), 256, 0, s>>>(D, n_narrow);
  const int nw = n_cuts - n_narrow;
  if (nw > 0) copy_fwd_wide_kernel<<<(nw + kCutsPerBlock - 1) / kCutsPerBlock, 256, 0, s>>>(D, n_narrow, n_cuts);
  return hipGetLastError();
}

// bound partials: one per narrow workgroup from part0, then one per wide workgroup
hipError_t launch_copy_bwd(const Dev &D, int n_cuts, int n_narrow, int update, int part0, hipStream_t s) {
  if (n_narrow > 0) copy_bwd_narrow_kernel<<<blocks_of(n_narrow), 256, 0, s>>>(D, n_narrow, update, part0);
  const int nw = n_cuts - n_narrow;
  if (nw > 0)
    copy_bwd_wide_kernel<<<(nw + kCutsPerBlock - 1) / kCutsPerBlock, 256, 0, s>>>(D, n_narrow, n_cuts, update,
                                                                                   part0 + blocks_of(n_narrow));
  return hipGetLastError();
}

hipError_t launch_copy_io(const Dev &D, int n_cuts, bool out, float *mu_bar, float *mu, float *dfw, float *dbw,
                          hipStream_t s) {
  if (n_cuts <= 0) return hipSuccess;
  copy_io_kernel<<<blocks_of(n_cuts), 256, 0, s>>>(D, n_cuts, out ? 1 : 0, mu_bar, mu, dfw, dbw);
  return hipGetLastError();
}

}  // namespace bddmp
