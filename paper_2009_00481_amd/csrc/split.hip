// Copy-arc kernels of the sub-BDD split (Sec. 6, Def. "Sub-BDD", Def. "Copy-arc", Alg. "Parallel
// min-marginal averaging"). The wave kernels run every sub-BDD like a whole diagram: an exit layer
// reads the duals mu_bar of its copy-arcs (arcs into TOP) from its virtual child slots, and a cut
// root level holds the forward messages that the arc duals mu give it. Between the passes, these
// kernels update both duals, one lane per cut (a cut has at most 2 x 32767 arcs; the workloads'
// cuts have a few). Arc q of a cut is arc (q / 2, q % 2) of its exit level.
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

// After the forward pass: each copy-arc's marginal in the sub-BDD it closes, (m_fwd(u) + theta) +
// mu_bar (theta with the exit level's updated multiplier), minus the smallest over the cut gives
// delta_fwd >= 0; mu_bar <- (mu_bar - gamma delta_fwd) + gamma delta_bwd (last backward update).
__global__ __launch_bounds__(256) void copy_fwd_kernel(const Dev D, int nc) {
#pragma clang fp contract(off)
  const int c = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (c >= nc) return;
  const int4 k = D.cuts[c], sl = D.cut_slots[c];
  const int w2 = 2 * (k.w & 0xFFFF), base = k.z;
  const float lam = D.lam[k.x], g = D.gamma;
  float mn = INFINITY;
  for (int q = 0; q < w2; ++q) {
    if (D.cut_arc[base + q] == kBot) continue;
    const float th = (q & 1) ? lam : 0.0f;
    mn = fminf(mn, (D.mf[sl.x + (q >> 1)] + th) + D.mbc[sl.y + q]);
  }
  for (int q = 0; q < w2; ++q) {
    if (D.cut_arc[base + q] == kBot) continue;
    const float th = (q & 1) ? lam : 0.0f;
    const float mb = D.mbc[sl.y + q];
    const float d = ((D.mf[sl.x + (q >> 1)] + th) + mb) - mn;
    D.dfw[base + q] = d;
    D.mbc[sl.y + q] = (mb - g * d) + g * D.dbw[base + q];
  }
}

// After the backward pass: each arc's marginal in the sub-BDD it opens, mu + m_bwd(v), minus the
// smallest over the cut gives delta_bwd >= 0; mu <- (mu - gamma delta_bwd) + gamma delta_fwd (this
// iteration's forward update). Then the root level's forward messages (minimum of mu over each
// node's in-arcs) and the sub-BDD's E (minimum over the arcs of mu + m_bwd(v)) for the bound: one
// fixed-shape sum per workgroup at lbpart[part0 + block]. update = 0 skips the dual update.
__global__ __launch_bounds__(256) void copy_bwd_kernel(const Dev D, int nc, int update, int part0) {
#pragma clang fp contract(off)
  __shared__ double sh[4];
  const int c = int(blockIdx.x) * 256 + int(threadIdx.x);
  double e = 0.0;
  if (c < nc) {
    const int4 k = D.cuts[c], sl = D.cut_slots[c];
    const int w2 = 2 * (k.w & 0xFFFF), wr = int(uint32_t(k.w) >> 16), base = k.z;
    const float lam = D.lam[k.y], g = D.gamma;
    if (update) {
      float mn = INFINITY;
      for (int q = 0; q < w2; ++q) {
        const uint32_t v = D.cut_arc[base + q];
        if (v == kBot) continue;
        mn = fminf(mn, D.mu_in[base + q] + root_bwd(D, sl.z, sl.w, lam, int(v)));
      }
      for (int q = 0; q < w2; ++q) {
        const uint32_t v = D.cut_arc[base + q];
        if (v == kBot) continue;
        const float mu = D.mu_in[base + q];
        const float d = (mu + root_bwd(D, sl.z, sl.w, lam, int(v))) - mn;
        D.dbw[base + q] = d;
        D.mu_in[base + q] = (mu - g * d) + g * D.dfw[base + q];
      }
    }
    for (int v = 0; v < wr; ++v) D.mf[sl.z + v] = INFINITY;
    float en = INFINITY;
    for (int q = 0; q < w2; ++q) {
      const uint32_t v = D.cut_arc[base + q];
      if (v == kBot) continue;
      const float mu = D.mu_in[base + q];
      D.mf[sl.z + int(v)] = fminf(D.mf[sl.z + int(v)], mu);
      en = fminf(en, mu + root_bwd(D, sl.z, sl.w, lam, int(v)));
    }
    e = double(en);
  }
  const double t = block_sum(e, sh);
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

hipError_t launch_copy_fwd(const Dev &D, int n_cuts, hipStream_t s) {
  if (n_cuts <= 0) return hipSuccess;
  copy_fwd_kernel<<<blocks_of(n_cuts), 256, 0, s>>>(D, n_cuts);
  return hipGetLastError();
}

hipError_t launch_copy_bwd(const Dev &D, int n_cuts, int update, int part0, hipStream_t s) {
  if (n_cuts <= 0) return hipSuccess;
  copy_bwd_kernel<<<blocks_of(n_cuts), 256, 0, s>>>(D, n_cuts, update, part0);
  return hipGetLastError();
}

hipError_t launch_copy_io(const Dev &D, int n_cuts, bool out, float *mu_bar, float *mu, float *dfw, float *dbw,
                          hipStream_t s) {
  if (n_cuts <= 0) return hipSuccess;
  copy_io_kernel<<<blocks_of(n_cuts), 256, 0, s>>>(D, n_cuts, out ? 1 : 0, mu_bar, mu, dfw, dbw);
  return hipGetLastError();
}

}  // namespace bddmp
