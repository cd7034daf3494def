// Device helpers shared by the wave kernels (kernels.hip) and the smoothed kernels (smooth.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace bddmp {

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

// General record of a layer: own slot, child slot, own width, child width, base of the child
// level's in-arc offsets (-1 without child level).
struct GRec {
  int os, cs, w, wc, rb;
};
__device__ __forceinline__ GRec grec_of(const Dev &D, int L) {
  const int4 g = D.grec[L];
  return {g.x, g.y, g.z & 0xFFFF, int(uint32_t(g.z) >> 16), g.w};
}

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

}  // namespace bddmp
