// Wavefront reductions on AMD DPP (data-parallel primitives) for the
// kernels that give a group of lanes to one cell.
#pragma once

#include <hip/hip_runtime.h>

namespace vofpc {

// Group reductions.  Within a row of 16 lanes they use DPP butterflies
// (xor 1 and xor 2 inside quads, then the half-row and row mirrors), which
// stay inside groups of 8 and 16 lanes and avoid the LDS permute latency;
// wider groups finish with cross-row shuffles.  Every lane of the group ends
// with the same, bitwise identical, result (IEEE addition is commutative).
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  int lo = __builtin_bit_cast(int2, v).x, hi = __builtin_bit_cast(int2, v).y;
  int2 r;
  r.x = dpp_i<CTRL>(lo);
  r.y = dpp_i<CTRL>(hi);
  return __builtin_bit_cast(double, r);
}
constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E, kHalfMirror = 0x141, kRowMirror = 0x140;

template <int W>
__device__ __forceinline__ double gsum(double v) {
  static_assert(W == 8 || W == 16 || W == 32 || W == 64, "group width");
  v += dpp_d<kQuadXor1>(v);
  v += dpp_d<kQuadXor2>(v);
  v += dpp_d<kHalfMirror>(v);
  if (W >= 16) v += dpp_d<kRowMirror>(v);
  if (W >= 32) v += __shfl_xor(v, 16, W);
  if (W >= 64) v += __shfl_xor(v, 32, W);
  return v;
}
template <int W>
__device__ __forceinline__ int gsum_i(int v) {
  v += dpp_i<kQuadXor1>(v);
  v += dpp_i<kQuadXor2>(v);
  v += dpp_i<kHalfMirror>(v);
  if (W >= 16) v += dpp_i<kRowMirror>(v);
  if (W >= 32) v += __shfl_xor(v, 16, W);
  if (W >= 64) v += __shfl_xor(v, 32, W);
  return v;
}
template <int W>
__device__ __forceinline__ int gmin_i(int v) {
  v = min(v, dpp_i<kQuadXor1>(v));
  v = min(v, dpp_i<kQuadXor2>(v));
  v = min(v, dpp_i<kHalfMirror>(v));
  if (W >= 16) v = min(v, dpp_i<kRowMirror>(v));
  if (W >= 32) v = min(v, __shfl_xor(v, 16, W));
  if (W >= 64) v = min(v, __shfl_xor(v, 32, W));
  return v;
}
template <int W>
__device__ __forceinline__ double gmin(double v) {
  v = fmin(v, dpp_d<kQuadXor1>(v));
  v = fmin(v, dpp_d<kQuadXor2>(v));
  v = fmin(v, dpp_d<kHalfMirror>(v));
  if (W >= 16) v = fmin(v, dpp_d<kRowMirror>(v));
  if (W >= 32) v = fmin(v, __shfl_xor(v, 16, W));
  if (W >= 64) v = fmin(v, __shfl_xor(v, 32, W));
  return v;
}
template <int W>
__device__ __forceinline__ double gmax(double v) {
  v = fmax(v, dpp_d<kQuadXor1>(v));
  v = fmax(v, dpp_d<kQuadXor2>(v));
  v = fmax(v, dpp_d<kHalfMirror>(v));
  if (W >= 16) v = fmax(v, dpp_d<kRowMirror>(v));
  if (W >= 32) v = fmax(v, __shfl_xor(v, 16, W));
  if (W >= 64) v = fmax(v, __shfl_xor(v, 32, W));
  return v;
}
// value of lane l (uniform l) on every lane
__device__ __forceinline__ double readlane_d(double v, int l) {
  int2 t = __builtin_bit_cast(int2, v);
  t.x = __builtin_amdgcn_readlane(t.x, l);
  t.y = __builtin_amdgcn_readlane(t.y, l);
  return __builtin_bit_cast(double, t);
}

}  // namespace vofpc
