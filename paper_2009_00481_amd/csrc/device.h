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

// Message accesses. In the dataflow launch (pass_kernel) a tile reads messages that other tiles of
// the same launch wrote, possibly on another XCD with its own L2. With COH those loads and stores
// are relaxed atomics at agent scope, which the hardware keeps coherent across the device without
// write-back or invalidation of the caches; the wave launches use plain accesses (the kernel
// boundary between waves orders them).
template <bool COH>
__device__ __forceinline__ float msg_ld(const float *p) {
  if constexpr (COH) return __hip_atomic_load(const_cast<float *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return *p;
}
// the float pair at p (8-byte aligned)
template <bool COH>
__device__ __forceinline__ float2 msg_ld2(const float *p) {
  if constexpr (COH) {
    const unsigned long long v = __hip_atomic_load(reinterpret_cast<unsigned long long *>(const_cast<float *>(p)),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_float2(__uint_as_float(unsigned(v)), __uint_as_float(unsigned(v >> 32)));
  } else {
    return *reinterpret_cast<const float2 *>(p);
  }
}
template <bool COH>
__device__ __forceinline__ void msg_st(float *p, float v) {
  if constexpr (COH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else *p = v;
}
template <bool COH>
__device__ __forceinline__ void msg_st2(float *p, float2 v) {
  if constexpr (COH) {
    const unsigned long long w =
        (static_cast<unsigned long long>(__float_as_uint(v.y)) << 32) | static_cast<unsigned long long>(__float_as_uint(v.x));
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    *reinterpret_cast<float2 *>(p) = v;
  }
}

// backward message behind a 16-bit child code of a general layer
template <bool COH = false>
__device__ __forceinline__ float c16val(const float *__restrict__ mb, int cs, uint32_t c) {
  return c < kTop ? msg_ld<COH>(mb + cs + int(c)) : (c == kTop ? 0.0f : INFINITY);
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

// A double moved across lanes by a DPP control (both 32-bit halves; sources stay inside a row of
// 16 lanes for the controls used here).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned lo = unsigned(__builtin_amdgcn_update_dpp(0, int(unsigned(b)), CTRL, 0xF, 0xF, false));
  const unsigned hi = unsigned(__builtin_amdgcn_update_dpp(0, int(unsigned(b >> 32)), CTRL, 0xF, 0xF, false));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

__device__ __forceinline__ double lane_value(double v, int lane) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(unsigned(b)), lane));
  const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(unsigned(b >> 32)), lane));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// Sum of one double per lane over a wavefront in a fixed shape, returned to every lane: lane pairs,
// quads, half rows and rows of 16 lanes by DPP moves (every lane of a row ends with the same row
// sum, since each step adds two equal partial sums in either order), then the four row sums in
// order. All 64 lanes must be active.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Sum of one double per lane over the workgroup in a fixed shape (wave_sum inside each
// wavefront, then the wavefront totals in order), so the result does not depend on timing.
__device__ __forceinline__ double block_sum(double v, double *sh) {
  v = wave_sum(v);
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
