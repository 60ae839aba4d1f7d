// Wavefront reductions on AMD DPP (data-parallel primitives) for the
// kernels that give a group of lanes to one cell.
#pragma once

#include <hip/hip_runtime.h>

namespace vofpc {

// Set bits of a wave-wide lane mask below the calling lane (the lane's
// rank among the set lanes), by the hardware bit counts v_mbcnt_lo/hi.
__device__ __forceinline__ int lanes_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Group reductions.  Within a row of 16 lanes they use DPP butterflies
// (xor 1 and xor 2 inside quads, then the half-row and row mirrors), which
// stay inside groups of 8 and 16 lanes and avoid the LDS permute latency;
// wider groups finish with the cross-row lane swaps.  Every lane of the group ends
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

// The values of lanes l & ~16 and l | 16 (Z = 16), or l & ~32 and l | 32
// (Z = 32), on every lane l, by the gfx950 lane swaps (registers only, no
// LDS permute): the two operands of a cross-row step, in the same order on
// both partners, so a sum, min or max of them is the same on both.
template <int Z>
__device__ __forceinline__ void pair_i(int v, int &lo, int &hi) {
  static_assert(Z == 16 || Z == 32, "swap distance");
  if constexpr (Z == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    lo = r[0];
    hi = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    lo = r[0];
    hi = r[1];
  }
}
template <int Z>
__device__ __forceinline__ void pair_d(double v, double &lo, double &hi) {
  int a0, a1, b0, b1;
  pair_i<Z>(__builtin_bit_cast(int2, v).x, a0, a1);
  pair_i<Z>(__builtin_bit_cast(int2, v).y, b0, b1);
  lo = __builtin_bit_cast(double, make_int2(a0, b0));
  hi = __builtin_bit_cast(double, make_int2(a1, b1));
}

template <int W>
__device__ __forceinline__ double gsum(double v) {
  static_assert(W == 4 || W == 8 || W == 16 || W == 32 || W == 64, "group width");
  v += dpp_d<kQuadXor1>(v);
  v += dpp_d<kQuadXor2>(v);
  if constexpr (W >= 8) v += dpp_d<kHalfMirror>(v);
  if constexpr (W >= 16) v += dpp_d<kRowMirror>(v);
  if constexpr (W >= 32) { double lo, hi; pair_d<16>(v, lo, hi); v = lo + hi; }
  if constexpr (W >= 64) { double lo, hi; pair_d<32>(v, lo, hi); v = lo + hi; }
  return v;
}
template <int W>
__device__ __forceinline__ int gsum_i(int v) {
  static_assert(W == 4 || W == 8 || W == 16 || W == 32 || W == 64, "group width");
  v += dpp_i<kQuadXor1>(v);
  v += dpp_i<kQuadXor2>(v);
  if constexpr (W >= 8) v += dpp_i<kHalfMirror>(v);
  if constexpr (W >= 16) v += dpp_i<kRowMirror>(v);
  if constexpr (W >= 32) { int lo, hi; pair_i<16>(v, lo, hi); v = lo + hi; }
  if constexpr (W >= 64) { int lo, hi; pair_i<32>(v, lo, hi); v = lo + hi; }
  return v;
}
template <int W>
__device__ __forceinline__ int gmin_i(int v) {
  static_assert(W == 4 || W == 8 || W == 16 || W == 32 || W == 64, "group width");
  v = min(v, dpp_i<kQuadXor1>(v));
  v = min(v, dpp_i<kQuadXor2>(v));
  if constexpr (W >= 8) v = min(v, dpp_i<kHalfMirror>(v));
  if constexpr (W >= 16) v = min(v, dpp_i<kRowMirror>(v));
  if constexpr (W >= 32) { int lo, hi; pair_i<16>(v, lo, hi); v = min(lo, hi); }
  if constexpr (W >= 64) { int lo, hi; pair_i<32>(v, lo, hi); v = min(lo, hi); }
  return v;
}
template <int W>
__device__ __forceinline__ double gmin(double v) {
  static_assert(W == 4 || W == 8 || W == 16 || W == 32 || W == 64, "group width");
  v = fmin(v, dpp_d<kQuadXor1>(v));
  v = fmin(v, dpp_d<kQuadXor2>(v));
  if constexpr (W >= 8) v = fmin(v, dpp_d<kHalfMirror>(v));
  if constexpr (W >= 16) v = fmin(v, dpp_d<kRowMirror>(v));
  if constexpr (W >= 32) { double lo, hi; pair_d<16>(v, lo, hi); v = fmin(lo, hi); }
  if constexpr (W >= 64) { double lo, hi; pair_d<32>(v, lo, hi); v = fmin(lo, hi); }
  return v;
}
template <int W>
__device__ __forceinline__ double gmax(double v) {
  static_assert(W == 4 || W == 8 || W == 16 || W == 32 || W == 64, "group width");
  v = fmax(v, dpp_d<kQuadXor1>(v));
  v = fmax(v, dpp_d<kQuadXor2>(v));
  if constexpr (W >= 8) v = fmax(v, dpp_d<kHalfMirror>(v));
  if constexpr (W >= 16) v = fmax(v, dpp_d<kRowMirror>(v));
  if constexpr (W >= 32) { double lo, hi; pair_d<16>(v, lo, hi); v = fmax(lo, hi); }
  if constexpr (W >= 64) { double lo, hi; pair_d<32>(v, lo, hi); v = fmax(lo, hi); }
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
