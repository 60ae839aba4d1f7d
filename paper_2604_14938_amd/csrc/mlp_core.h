// Bracket network: parameter layout, BF16 helpers, the MFMA building blocks
// of the batched kernels, the single-row forward pass run inside the
// reconstruction wave, and the
// assembly of the 32 input features from per-cell sums (shared by the
// features kernel and the reconstruction kernel so both feed the network the
// same numbers).
//
// MFMA tiles: v_mfma_f32_16x16x16_bf16 on one wavefront.  Lane l holds
// A[l%16][4(l/16)+j], B[4(l/16)+j][l%16] and D[4(l/16)+j][l%16], j = 0..3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vofpc {
namespace net {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// 32 -> 64 -> 64 -> 4, tanh hidden layers; row-major W[out][in]
constexpr int kIn = 32, kHid = 64, kOut = 4;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kOut * kHid, kParams = oB3 + kOut;

__device__ __forceinline__ uint16_t to_bf16(float x) {
  uint32_t b = __float_as_uint(x);
  if ((b & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((b >> 16) | 0x40);  // NaN stays NaN
  b += 0x7fffu + ((b >> 16) & 1u);  // round to nearest even
  return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Hidden-layer activation.  For |x| >= 1/8 the identity
// tanh x = 1 - 2 / (e^{2x} + 1) on |x| (hardware base-2 exponential and
// reciprocal; e^{2|x|} overflowing to infinity gives 1), the sign restored;
// below, the Taylor series x - x^3/3 + 2x^5/15 - 17x^7/315 (truncation error
// under 2e-10 there).  Errors of a few 1e-7, far below the BF16 rounding the
// activations get next.
__device__ __forceinline__ float act_tanh(float x) {
  const float ax = fabsf(x);
  if (ax < 0.125f) {
    const float x2 = x * x;
    return x * (1.0f + x2 * (-1.0f / 3.0f + x2 * (2.0f / 15.0f + x2 * (-17.0f / 315.0f))));
  }
  const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * ax);   // 2 log2(e) |x|
  return copysignf(1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f), x);
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// B operand from a row-major weight matrix W[n][k] (B[k][n] = W[n][k]);
// columns n >= nmax are zero.  The four values of a lane are contiguous and
// 8-byte aligned (every matrix offset and row length is a multiple of 4), so
// they come in one load.
__device__ __forceinline__ bf16x4 b_weightT(const uint16_t *W, int ldk, int lane, int n0, int k0, int nmax) {
  const int n = n0 + (lane & 15), k = k0 + 4 * (lane >> 4);
  bf16x4 v = {0, 0, 0, 0};
  if (n < nmax) v = *reinterpret_cast<const bf16x4 *>(W + n * ldk + k);
  return v;
}

// v[l & ~Z] + v[l | Z] on every lane l (Z = 16 or 32) by the gfx950 lane
// swaps: the same two operands, in the same order, on both partners
template <int Z>
__device__ __forceinline__ float cross_sum_f(float v) {
  const int b = __builtin_bit_cast(int, v);
  int lo, hi;
  if constexpr (Z == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(b, b, false, false);
    lo = r[0];
    hi = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(b, b, false, false);
    lo = r[0];
    hi = r[1];
  }
  return __builtin_bit_cast(float, lo) + __builtin_bit_cast(float, hi);
}

// Sum of a float over the 64 lanes of a wavefront, the same on every lane
// (DPP inside rows of 16, then the cross-row lane swaps).
__device__ __forceinline__ float wave_sum_f(float v) {
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x141, 0xF, 0xF, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x140, 0xF, 0xF, false));
  v = cross_sum_f<16>(v);
  v = cross_sum_f<32>(v);
  return v;
}

// dot product of 8 BF16 weights (one 16-byte word) with 8 BF16 inputs
__device__ __forceinline__ float dot8(uint4 w, uint4 x, float acc) {
  const uint32_t wv[4] = {w.x, w.y, w.z, w.w}, xv[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    acc += __uint_as_float(wv[i] << 16) * __uint_as_float(xv[i] << 16);
    acc += __uint_as_float(wv[i] & 0xffff0000u) * __uint_as_float(xv[i] & 0xffff0000u);
  }
  return acc;
}

// Forward pass of one input row by a whole wavefront, one hidden unit per
// lane (a single row is a matrix-vector product: FP32 FMAs on the BF16
// weights and activations, no matrix-core tile).  x: kIn BF16 inputs in LDS
// (16-byte aligned); h1, h2: kHid BF16 LDS scratch (16-byte aligned).
// Returns output component 0 (the normalised isovalue) on every lane; `sync`
// orders LDS traffic within the wave.
template <class Sync>
__device__ __forceinline__ float row_forward(const uint16_t *wb, const float *master, const uint16_t *x, uint16_t *h1,
                                             uint16_t *h2, int lane, Sync sync) {
  static_assert(kHid == 64 && kIn % 8 == 0, "one hidden unit per lane");
  const uint4 *w1 = reinterpret_cast<const uint4 *>(wb + oW1 + lane * kIn);
  const uint4 *w2 = reinterpret_cast<const uint4 *>(wb + oW2 + lane * kHid);
  uint4 r1[kIn / 8];
#pragma unroll
  for (int i = 0; i < kIn / 8; ++i) r1[i] = w1[i];
  const float b1 = master[oB1 + lane], b2 = master[oB2 + lane];
  const float w3 = __uint_as_float((uint32_t)wb[oW3 + lane] << 16), b3 = master[oB3];
  const uint4 *xv = reinterpret_cast<const uint4 *>(x);
  float z = 0.f;
#pragma unroll
  for (int i = 0; i < kIn / 8; ++i) z = dot8(r1[i], xv[i], z);
  h1[lane] = to_bf16(act_tanh(z + b1));
  sync();
  const uint4 *hv = reinterpret_cast<const uint4 *>(h1);
  z = 0.f;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    uint4 r2[kHid / 16];
#pragma unroll
    for (int i = 0; i < kHid / 16; ++i) r2[i] = w2[half * (kHid / 16) + i];
#pragma unroll
    for (int i = 0; i < kHid / 16; ++i) z = dot8(r2[i], hv[half * (kHid / 16) + i], z);
  }
  const float h2v = from_bf16(to_bf16(act_tanh(z + b2)));
  (void)h2;
  return wave_sum_f(w3 * h2v) + b3;
}

// The 32 inputs of one mixed cell (see the features entry point for their
// meaning) from its vertex values sorted ascending (`sorted(i)`), their sum,
// and the face sums
//   s[0] sum A_f, s[1..3] sum A_f da n_f, s[4..9] sum A_f da n_f n_f^T,
//   s[10..15] sum A_f n_f n_f^T, s[16] sum alpha_Q, s[17] interior count,
// da = alpha_Q - alpha_P (xx yy zz xy xz yz order for the tensors).
template <class Sorted>
__device__ __forceinline__ float feature(int i, double aP, Sorted sorted, int nvv, double lsum, double pmin, double Wd,
                                         const double *s, double amin, double amax, int nf) {
  const double iW = Wd > 0 ? 1.0 / Wd : 0.0;
  double v;
  if (i >= 1 && i <= 7) {
    // vertex-value quantile i/8, linear between order statistics
    const double t = i / 8.0 * (nvv - 1);
    const int j = (int)floor(t);
    const double fr = t - j;
    const double lo = sorted(j);
    const double val = (j + 1 >= nvv) ? lo : lo + fr * (sorted(j + 1) - lo);
    v = (val - pmin) * iW;
  } else if (i >= 10 && i <= 24) {
    v = s[i - 9] * (1.0 / s[0]);   // area-weighted face moments
  } else {
    const bool nb = s[17] > 0;
    v = i == 0 ? aP
      : i == 8 ? (lsum / nvv - pmin) * iW
      : i == 9 ? Wd
      : i == 25 ? nf / 32.0
      : i == 26 ? (nb ? s[16] / s[17] : aP)
      : i == 27 ? (nb ? amin : aP)
      : i == 28 ? (nb ? amax : aP)
      : 0.0;
  }
  return (float)v;
}

}  // namespace net
}  // namespace vofpc
