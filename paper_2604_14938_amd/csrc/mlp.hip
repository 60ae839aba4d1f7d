// Bracket network: per-cell features, a 32 -> 64 -> 64 -> 4 tanh perceptron
// on BF16 MFMA with FP32 accumulation (forward, backward, Adam on FP32 master
// weights), and the decoding of its output into a narrowed bisection bracket.
//
// The network predicts u = (s* - phi_min)/W (and a normal); the bracket is
// [phi_min + clamp(u,0,1) W - delta, ... + delta] with delta = k_sigma sigma W.
// The reconstruction checks the bracket and falls back, so the network only
// changes how many volume evaluations a cell needs, never its result.
//
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <vector>

#include "vofpc_internal.h"
#include "mlp_core.h"

namespace vofpc {

using namespace net;
constexpr float kNormalWeight = 0.1f;
constexpr int kTilesPerBlock = 4;  // 64 rows per training block

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct TileMem {
  uint16_t x[16][kIn];    // BF16 inputs
  uint16_t h1[16][kHid];  // BF16 activations
  uint16_t h2[16][kHid];
  uint16_t dz2[16][kHid]; // BF16 back-propagated pre-activation gradients
  uint16_t dz1[16][kHid];
  float y[16][kOut];
  float dy[16][kOut];
};

// A operand from a row-major BF16 tile: rows 0..15, columns k0 + 4(l/16) + j
template <int LD>
__device__ __forceinline__ bf16x4 a_rows(const uint16_t (*t)[LD], int lane, int k0) {
  const int r = lane & 15, k = k0 + 4 * (lane >> 4);
  bf16x4 v;
  v[0] = (short)t[r][k]; v[1] = (short)t[r][k + 1]; v[2] = (short)t[r][k + 2]; v[3] = (short)t[r][k + 3];
  return v;
}
// Forward pass of one 16-row tile (rows past nrows are zero inputs).
__device__ void tile_forward(TileMem &T, const float *X, int64_t row0, int nrows, const uint16_t *wb,
                             const float *master, int lane) {
  for (int i = lane; i < 16 * kIn; i += 64) {
    const int r = i / kIn, c = i % kIn;
    T.x[r][c] = (r < nrows) ? to_bf16(X[(row0 + r) * kIn + c]) : (uint16_t)0;
  }
  wsync();
  const int col = lane & 15, rq = 4 * (lane >> 4);
  // layer 1: h1 = tanh(x W1^T + b1)
  for (int nt = 0; nt < kHid / 16; ++nt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < kIn / 16; ++kt)
      acc = mfma16(a_rows<kIn>(T.x, lane, kt * 16), b_weightT(wb + oW1, kIn, lane, nt * 16, kt * 16, kHid), acc);
    const float b = master[oB1 + nt * 16 + col];
    for (int j = 0; j < 4; ++j) T.h1[rq + j][nt * 16 + col] = to_bf16(act_tanh(acc[j] + b));
  }
  wsync();
  // layer 2
  for (int nt = 0; nt < kHid / 16; ++nt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < kHid / 16; ++kt)
      acc = mfma16(a_rows<kHid>(T.h1, lane, kt * 16), b_weightT(wb + oW2, kHid, lane, nt * 16, kt * 16, kHid), acc);
    const float b = master[oB2 + nt * 16 + col];
    for (int j = 0; j < 4; ++j) T.h2[rq + j][nt * 16 + col] = to_bf16(act_tanh(acc[j] + b));
  }
  wsync();
  // layer 3 (4 outputs, padded to a 16-wide tile)
  {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < kHid / 16; ++kt)
      acc = mfma16(a_rows<kHid>(T.h2, lane, kt * 16), b_weightT(wb + oW3, kHid, lane, 0, kt * 16, kOut), acc);
    if (col < kOut) {
      const float b = master[oB3 + col];
      for (int j = 0; j < 4; ++j) T.y[rq + j][col] = acc[j] + b;
    }
  }
  wsync();
}

__global__ __launch_bounds__(64) void mlp_forward_kernel(const float *X, int64_t n, const uint16_t *wb,
                                                         const float *master, float *Y) {
  __shared__ TileMem T;
  const int lane = threadIdx.x;
  const int64_t tiles = (n + 15) / 16;
  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int64_t r0 = t * 16;
    const int nr = (int)((n - r0) < 16 ? (n - r0) : 16);
    tile_forward(T, X, r0, nr, wb, master, lane);
    for (int i = lane; i < 16 * kOut; i += 64) {
      const int r = i / kOut, c = i % kOut;
      if (r < nr) Y[(r0 + r) * kOut + c] = T.y[r][c];
    }
    wsync();
  }
}

// Forward, loss and backward of the rows of one block; writes the block's
// partial gradient and loss (no atomics: a fixed-order reduction follows).
__global__ __launch_bounds__(64) void mlp_grad_partial_kernel(const float *X, const float *Tg, int64_t n,
                                                              const uint16_t *wb, const float *master,
                                                              float *partial) {
  __shared__ TileMem T;
  __shared__ float red[64];
  const int lane = threadIdx.x;
  const int col = lane & 15, rq = 4 * (lane >> 4);
  const float inv_n = 1.0f / (float)n;
  f32x4 gW2[4][4], gW1[4][2];
  for (int a = 0; a < 4; ++a) {
    for (int b = 0; b < 4; ++b) gW2[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int b = 0; b < 2; ++b) gW1[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
  }
  float gW3[kOut] = {0.f, 0.f, 0.f, 0.f};  // lane = hidden unit
  float gb3 = 0.f, gb2 = 0.f, gb1 = 0.f;     // lane-indexed (gb3 for lane < 4)
  float lsum = 0.f;
  const int64_t tiles = (n + 15) / 16;
  const int64_t t0 = (int64_t)blockIdx.x * kTilesPerBlock;
  for (int64_t t = t0; t < t0 + kTilesPerBlock && t < tiles; ++t) {
    const int64_t r0 = t * 16;
    const int nr = (int)((n - r0) < 16 ? (n - r0) : 16);
    tile_forward(T, X, r0, nr, wb, master, lane);
    // output gradient of the mean loss
    if (lane < 16 * kOut) {
      const int r = lane / kOut, c = lane % kOut;
      float d = 0.f;
      if (r < nr) {
        const float e = T.y[r][c] - Tg[(r0 + r) * kOut + c];
        const float w = (c == 0) ? 1.0f : kNormalWeight;
        d = 2.0f * w * e * inv_n;
        lsum += w * e * e;
      }
      T.dy[r][c] = d;
    }
    wsync();
    // dW3 = dy^T h2, db3, dz2 = (dy W3) * (1 - h2^2)   (FP32, K = 4)
    for (int r = 0; r < 16; ++r) {
      const float h = from_bf16(T.h2[r][lane]);
      float dh = 0.f;
      for (int c = 0; c < kOut; ++c) {
        const float d = T.dy[r][c];
        gW3[c] += d * h;
        dh += d * from_bf16(wb[oW3 + c * kHid + lane]);
      }
      T.dz2[r][lane] = to_bf16(dh * (1.0f - h * h));
    }
    if (lane < kOut)
      for (int r = 0; r < 16; ++r) gb3 += T.dy[r][lane];
    wsync();
    // dz1 = (dz2 W2) * (1 - h1^2): A = dz2 (rows), B[k][n] = W2[k][n]
    for (int nt = 0; nt < kHid / 16; ++nt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int kt = 0; kt < kHid / 16; ++kt) {
        bf16x4 bv;
        const int n = nt * 16 + col, k = kt * 16 + 4 * (lane >> 4);
        for (int j = 0; j < 4; ++j) bv[j] = (short)wb[oW2 + (k + j) * kHid + n];
        acc = mfma16(a_rows<kHid>(T.dz2, lane, kt * 16), bv, acc);
      }
      for (int j = 0; j < 4; ++j) {
        const float h = from_bf16(T.h1[rq + j][nt * 16 + col]);
        T.dz1[rq + j][nt * 16 + col] = to_bf16(acc[j] * (1.0f - h * h));
      }
    }
    wsync();
    // dW2 += dz2^T h1, dW1 += dz1^T x: A[m][k] = dz[k][m], B[k][n] = act[k][n]
    for (int mt = 0; mt < 4; ++mt) {
      bf16x4 a2, a1;
      for (int j = 0; j < 4; ++j) {
        a2[j] = (short)T.dz2[rq + j][mt * 16 + col];
        a1[j] = (short)T.dz1[rq + j][mt * 16 + col];
      }
      for (int nt = 0; nt < 4; ++nt) {
        bf16x4 bv;
        for (int j = 0; j < 4; ++j) bv[j] = (short)T.h1[rq + j][nt * 16 + col];
        gW2[mt][nt] = mfma16(a2, bv, gW2[mt][nt]);
      }
      for (int nt = 0; nt < 2; ++nt) {
        bf16x4 bv;
        for (int j = 0; j < 4; ++j) bv[j] = (short)T.x[rq + j][nt * 16 + col];
        gW1[mt][nt] = mfma16(a1, bv, gW1[mt][nt]);
      }
    }
    for (int r = 0; r < 16; ++r) {
      gb2 += from_bf16(T.dz2[r][lane]);
      gb1 += from_bf16(T.dz1[r][lane]);
    }
    wsync();
  }
  float *out = partial + (int64_t)blockIdx.x * (kParams + 1);
  for (int mt = 0; mt < 4; ++mt) {
    for (int nt = 0; nt < 4; ++nt)
      for (int j = 0; j < 4; ++j) out[oW2 + (mt * 16 + rq + j) * kHid + nt * 16 + col] = gW2[mt][nt][j];
    for (int nt = 0; nt < 2; ++nt)
      for (int j = 0; j < 4; ++j) out[oW1 + (mt * 16 + rq + j) * kIn + nt * 16 + col] = gW1[mt][nt][j];
  }
  for (int c = 0; c < kOut; ++c) out[oW3 + c * kHid + lane] = gW3[c];
  out[oB2 + lane] = gb2;
  out[oB1 + lane] = gb1;
  if (lane < kOut) out[oB3 + lane] = gb3;
  red[lane] = lsum;
  wsync();
  if (lane == 0) {
    float s = 0.f;
    for (int i = 0; i < 64; ++i) s += red[i];
    out[kParams] = s * inv_n;
  }
}

// Fixed-order sum of the block partials.
__global__ void mlp_reduce_kernel(const float *partial, int nblk, float *grad, float *loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > kParams) return;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * (kParams + 1) + i];
  if (i < kParams) grad[i] = s;
  else if (loss) *loss = s;
}

__global__ void adam_kernel(float *master, uint16_t *wb, float *m, float *v, const float *g, float lr, float b1,
                            float b2, float eps, float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kParams) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float w = master[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  master[i] = w;
  wb[i] = to_bf16(w);
}

__global__ void to_bf16_kernel(const float *src, uint16_t *dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = to_bf16(src[i]);
}

// Decode the network output into a bracket per mixed entry.
__global__ __launch_bounds__(64) void mlp_bracket_kernel(const float *X, const double *prange, const int32_t *counts,
                                                         int64_t cap, const uint16_t *wb, const float *master,
                                                         double ksig, double *hlo, double *hhi) {
  __shared__ TileMem T;
  const int lane = threadIdx.x;
  int64_t n = counts[0];
  if (n > cap) n = cap;
  const int64_t tiles = (n + 15) / 16;
  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int64_t r0 = t * 16;
    const int nr = (int)((n - r0) < 16 ? (n - r0) : 16);
    tile_forward(T, X, r0, nr, wb, master, lane);
    if (lane < nr) {
      const int64_t k = r0 + lane;
      const double lo = prange[2 * k], W = prange[2 * k + 1];
      double u = (double)T.y[lane][0];
      u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
      const double sh = lo + u * W, d = ksig * W;
      if (W > 0 && !isnan(u)) {
        hlo[k] = sh - d;
        hhi[k] = sh + d;
      } else {
        hlo[k] = __builtin_nan("");
        hhi[k] = __builtin_nan("");
      }
    }
    wsync();
  }
}

// ----------------------------------------------------------------- features
template <int W>
__device__ __forceinline__ double fsum(double v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}

struct FeatMem {
  double phi[256];
  double sorted[256];
};

// 16 lanes per mixed cell, 4 cells per block.  Definitions: see the header.
__global__ __launch_bounds__(64) void features_kernel(DevMesh m, const double *alpha, const int32_t *mixed,
                                                      const int32_t *counts, int64_t cap, const double *phi_override,
                                                      int vertex_mode, float *feat, double *prange) {
  constexpr int W = 16, G = 4;
  __shared__ FeatMem F[G];
  const int g = threadIdx.x / W, lane = threadIdx.x % W;
  FeatMem &L = F[g];
  int64_t count = counts[0];
  if (count > cap) count = cap;
  for (int64_t k = (int64_t)blockIdx.x * G + g; k < count; k += (int64_t)gridDim.x * G) {
    const int P = mixed[k];
    const double aP = alpha[P];
    const int64_t v0 = m.cv_off[P];
    const int nv = (int)(m.cv_off[P + 1] - v0);
    const int nvv = nv < 256 ? nv : 256;
    for (int i = lane; i < nvv; i += W) {
      const int gv = m.cv_gid[v0 + i];
      double ph;
      if (phi_override) {
        ph = phi_override[gv];
      } else {
        const double *w = vertex_mode ? m.vc_wmean : m.vc_w;
        ph = 0.0;
        for (int64_t j = m.vc_off[gv]; j < m.vc_off[gv + 1]; ++j) ph += w[j] * alpha[m.vc_cell[j]];
      }
      L.phi[i] = ph;
    }
    wsync();
    // ranks -> sorted values
    double lmin = __builtin_inf(), lmax = -__builtin_inf(), lsum = 0;
    for (int i = lane; i < nvv; i += W) {
      const double v = L.phi[i];
      int r = 0;
      for (int j = 0; j < nvv; ++j) {
        const double u = L.phi[j];
        r += (u < v) || (u == v && j < i);
      }
      L.sorted[r] = v;
      lmin = fmin(lmin, v);
      lmax = fmax(lmax, v);
      lsum += v;
    }
    for (int o = W / 2; o > 0; o >>= 1) {
      lmin = fmin(lmin, __shfl_xor(lmin, o, W));
      lmax = fmax(lmax, __shfl_xor(lmax, o, W));
    }
    lsum = fsum<W>(lsum);
    wsync();
    const double pmin = lmin, Wd = lmax - lmin;
    // faces: area-weighted moments, shape tensor, neighbour alpha
    const int64_t f0 = m.cell_face_off[P];
    const int nf = (int)(m.cell_face_off[P + 1] - f0);
    double s[20];
    for (int q = 0; q < 20; ++q) s[q] = 0.0;
    double amin = __builtin_inf(), amax = -__builtin_inf();
    for (int f = lane; f < nf; f += W) {
      const double *Sv = m.cf_S + 3 * (f0 + f);
      const double S0 = Sv[0], S1 = Sv[1], S2 = Sv[2];
      const double A = sqrt(S0 * S0 + S1 * S1 + S2 * S2);
      const double n0 = S0 / A, n1 = S1 / A, n2 = S2 / A;
      const int q = m.cf_nbr[f0 + f];
      const double aQ = (q >= 0) ? alpha[q] : aP;
      const double da = A * (aQ - aP);
      const double o[6] = {n0 * n0, n1 * n1, n2 * n2, n0 * n1, n0 * n2, n1 * n2};
      s[0] += A;
      s[1] += da * n0; s[2] += da * n1; s[3] += da * n2;
      for (int c = 0; c < 6; ++c) {
        s[4 + c] += da * o[c];
        s[10 + c] += A * o[c];
      }
      if (q >= 0) {
        s[16] += aQ;
        s[17] += 1.0;
        amin = fmin(amin, aQ);
        amax = fmax(amax, aQ);
      }
    }
    for (int q = 0; q < 18; ++q) s[q] = fsum<W>(s[q]);
    for (int o = W / 2; o > 0; o >>= 1) {
      amin = fmin(amin, __shfl_xor(amin, o, W));
      amax = fmax(amax, __shfl_xor(amax, o, W));
    }
    if (lane == 0) {
      float *out = feat + k * 32;
      auto sorted = [&](int j) { return L.sorted[j]; };
      for (int i = 0; i < 32; ++i) out[i] = feature(i, aP, sorted, nvv, lsum, pmin, Wd, s, amin, amax, nf);
      prange[2 * k] = pmin;
      prange[2 * k + 1] = Wd;
    }
    wsync();
  }
}

}  // namespace vofpc

using namespace vofpc;

struct vofpc_mlp_s {
  vofpc_ctx ctx;
  float *master = nullptr;
  uint16_t *wb = nullptr;
  float *m = nullptr, *v = nullptr;
  float *grad = nullptr;
  float *partial = nullptr;
  float *loss = nullptr;
  int max_blocks = 0;
  int64_t t = 0;
};

extern "C" vofpc_status vofpc_mlp_destroy(vofpc_mlp M);

extern "C" int vofpc_mlp_param_count(void) { return kParams; }

extern "C" vofpc_status vofpc_mlp_create(vofpc_ctx ctx, int64_t max_batch, vofpc_mlp *out) {
  clear_error();
  VOFPC_REQUIRE(ctx && out && max_batch > 0, VOFPC_E_INVALID_ARG, "mlp_create: bad argument");
  *out = nullptr;
  VOFPC_HIP(hipSetDevice(ctx->device));
  vofpc_mlp M = new (std::nothrow) vofpc_mlp_s();
  VOFPC_REQUIRE(M, VOFPC_E_OOM, "mlp_create: host allocation failed");
  M->ctx = ctx;
  M->max_blocks = (int)((max_batch + 16 * kTilesPerBlock - 1) / (16 * kTilesPerBlock));
  if (hipMalloc(&M->master, sizeof(float) * kParams) != hipSuccess ||
      hipMalloc(&M->m, sizeof(float) * kParams) != hipSuccess ||
      hipMalloc(&M->v, sizeof(float) * kParams) != hipSuccess ||
      hipMalloc(&M->grad, sizeof(float) * kParams) != hipSuccess ||
      hipMalloc(&M->loss, sizeof(float)) != hipSuccess ||
      hipMalloc(&M->wb, sizeof(uint16_t) * kParams) != hipSuccess ||
      hipMalloc(&M->partial, sizeof(float) * (size_t)M->max_blocks * (kParams + 1)) != hipSuccess) {
    vofpc_mlp_destroy(M);
    set_error("mlp_create: hipMalloc failed");
    return VOFPC_E_OOM;
  }
  VOFPC_HIP(hipMemset(M->master, 0, sizeof(float) * kParams));
  VOFPC_HIP(hipMemset(M->wb, 0, sizeof(uint16_t) * kParams));
  VOFPC_HIP(hipMemset(M->m, 0, sizeof(float) * kParams));
  VOFPC_HIP(hipMemset(M->v, 0, sizeof(float) * kParams));
  M->t = 0;
  *out = M;
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_mlp_destroy(vofpc_mlp M) {
  clear_error();
  if (!M) return VOFPC_OK;
  (void)hipSetDevice(M->ctx->device);
  (void)hipFree(M->master); (void)hipFree(M->wb); (void)hipFree(M->m); (void)hipFree(M->v);
  (void)hipFree(M->grad); (void)hipFree(M->partial); (void)hipFree(M->loss);
  delete M;
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_mlp_set_params(vofpc_mlp M, const float *host, int64_t n) {
  clear_error();
  VOFPC_REQUIRE(M && host && n == kParams, VOFPC_E_INVALID_ARG, "mlp_set_params: need all parameters");
  VOFPC_HIP(hipSetDevice(M->ctx->device));
  VOFPC_HIP(hipMemcpy(M->master, host, sizeof(float) * kParams, hipMemcpyHostToDevice));
  VOFPC_HIP(hipMemset(M->m, 0, sizeof(float) * kParams));
  VOFPC_HIP(hipMemset(M->v, 0, sizeof(float) * kParams));
  to_bf16_kernel<<<(kParams + 255) / 256, 256, 0, M->ctx->stream>>>(M->master, M->wb, kParams);
  VOFPC_HIP(hipGetLastError());
  VOFPC_HIP(hipStreamSynchronize(M->ctx->stream));
  M->t = 0;
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_mlp_get_params(vofpc_mlp M, float *host, int64_t n) {
  clear_error();
  VOFPC_REQUIRE(M && host && n == kParams, VOFPC_E_INVALID_ARG, "mlp_get_params: need all parameters");
  VOFPC_HIP(hipSetDevice(M->ctx->device));
  VOFPC_HIP(hipStreamSynchronize(M->ctx->stream));
  VOFPC_HIP(hipMemcpy(host, M->master, sizeof(float) * kParams, hipMemcpyDeviceToHost));
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_mlp_forward(vofpc_ctx ctx, vofpc_mlp M, const float *X, int64_t n, float *Y) {
  clear_error();
  VOFPC_REQUIRE(ctx && M && X && Y && n > 0, VOFPC_E_INVALID_ARG, "mlp_forward: bad argument");
  VOFPC_HIP(hipSetDevice(ctx->device));
  int64_t grid = (n + 15) / 16;
  if (grid > ctx->n_cu * 8) grid = ctx->n_cu * 8;
  mlp_forward_kernel<<<(unsigned)grid, 64, 0, ctx->stream>>>(X, n, M->wb, M->master, Y);
  VOFPC_HIP(hipGetLastError());
  return VOFPC_OK;
}

static vofpc_status mlp_gradient(vofpc_ctx ctx, vofpc_mlp M, const float *X, const float *T, int64_t n) {
  const int nblk = (int)((n + 16 * kTilesPerBlock - 1) / (16 * kTilesPerBlock));
  VOFPC_REQUIRE(nblk <= M->max_blocks, VOFPC_E_INVALID_ARG, "mlp: batch larger than max_batch");
  mlp_grad_partial_kernel<<<nblk, 64, 0, ctx->stream>>>(X, T, n, M->wb, M->master, M->partial);
  mlp_reduce_kernel<<<(kParams + 1 + 255) / 256, 256, 0, ctx->stream>>>(M->partial, nblk, M->grad, M->loss);
  VOFPC_HIP(hipGetLastError());
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_mlp_gradient(vofpc_ctx ctx, vofpc_mlp M, const float *X, const float *T, int64_t n,
                                           float *grad, float *loss) {
  clear_error();
  VOFPC_REQUIRE(ctx && M && X && T && n > 0, VOFPC_E_INVALID_ARG, "mlp_gradient: bad argument");
  VOFPC_HIP(hipSetDevice(ctx->device));
  vofpc_status s = mlp_gradient(ctx, M, X, T, n);
  if (s) return s;
  if (grad) VOFPC_HIP(hipMemcpyAsync(grad, M->grad, sizeof(float) * kParams, hipMemcpyDeviceToDevice, ctx->stream));
  if (loss) VOFPC_HIP(hipMemcpyAsync(loss, M->loss, sizeof(float), hipMemcpyDeviceToDevice, ctx->stream));
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_mlp_train_step(vofpc_ctx ctx, vofpc_mlp M, const float *X, const float *T, int64_t n,
                                             float lr, float *loss) {
  clear_error();
  VOFPC_REQUIRE(ctx && M && X && T && n > 0 && lr > 0, VOFPC_E_INVALID_ARG, "mlp_train_step: bad argument");
  VOFPC_HIP(hipSetDevice(ctx->device));
  vofpc_status s = mlp_gradient(ctx, M, X, T, n);
  if (s) return s;
  M->t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = 1.0f - powf(b1, (float)M->t), bc2 = 1.0f - powf(b2, (float)M->t);
  adam_kernel<<<(kParams + 255) / 256, 256, 0, ctx->stream>>>(M->master, M->wb, M->m, M->v, M->grad, lr, b1, b2,
                                                              1e-8f, bc1, bc2);
  VOFPC_HIP(hipGetLastError());
  if (loss) VOFPC_HIP(hipMemcpyAsync(loss, M->loss, sizeof(float), hipMemcpyDeviceToDevice, ctx->stream));
  return VOFPC_OK;
}

namespace vofpc {
const uint16_t *mlp_weights_bf16(vofpc_mlp M) { return M->wb; }
const float *mlp_params_f32(vofpc_mlp M) { return M->master; }
int mlp_device(vofpc_mlp M) { return M->ctx->device; }

vofpc_status launch_features(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha, const int32_t *mixed,
                             const int32_t *counts, int64_t cap, const vofpc_recon_opts *o, float *feat,
                             double *prange) {
  VOFPC_REQUIRE(alpha && mixed && counts && feat && prange && cap > 0, VOFPC_E_INVALID_ARG,
                "features: bad argument");
  VOFPC_REQUIRE(mesh->max_nv <= 256, VOFPC_E_MESH, "features: cells with more than 256 vertices");
  int64_t grid = (std::min<int64_t>(cap, mesh->d.n_cells) + 3) / 4;
  if (grid > ctx->n_cu * 16) grid = ctx->n_cu * 16;
  if (grid < 1) grid = 1;
  features_kernel<<<(unsigned)grid, 64, 0, ctx->stream>>>(mesh->d, alpha, mixed, counts, cap,
                                                          o ? o->phi_vertex : nullptr, o ? o->vertex_mode : 0, feat,
                                                          prange);
  VOFPC_HIP(hipGetLastError());
  return VOFPC_OK;
}

vofpc_status launch_bracket(vofpc_ctx ctx, vofpc_mlp M, const float *feat, const double *prange,
                            const int32_t *counts, int64_t cap, double ksig, double *hlo, double *hhi) {
  VOFPC_REQUIRE(M && feat && prange && counts && hlo && hhi && cap > 0, VOFPC_E_INVALID_ARG,
                "mlp_bracket: bad argument");
  int64_t grid = (cap + 15) / 16;
  if (grid > ctx->n_cu * 8) grid = ctx->n_cu * 8;
  mlp_bracket_kernel<<<(unsigned)grid, 64, 0, ctx->stream>>>(feat, prange, counts, cap, M->wb, M->master, ksig, hlo,
                                                             hhi);
  VOFPC_HIP(hipGetLastError());
  return VOFPC_OK;
}
}  // namespace vofpc

extern "C" vofpc_status vofpc_features(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha, const int32_t *mixed_idx,
                                       const int32_t *counts, const vofpc_recon_opts *opts, float *features,
                                       double *phi_range, int64_t cap) {
  clear_error();
  VOFPC_REQUIRE(ctx && mesh, VOFPC_E_INVALID_ARG, "features: null context or mesh");
  VOFPC_HIP(hipSetDevice(ctx->device));
  return launch_features(ctx, mesh, alpha, mixed_idx, counts, cap, opts, features, phi_range);
}

extern "C" vofpc_status vofpc_mlp_bracket(vofpc_ctx ctx, vofpc_mlp M, const float *features, const double *phi_range,
                                          const int32_t *counts, int64_t cap, double delta_scale, double *hint_lo,
                                          double *hint_hi) {
  clear_error();
  VOFPC_REQUIRE(ctx, VOFPC_E_INVALID_ARG, "mlp_bracket: null context");
  VOFPC_HIP(hipSetDevice(ctx->device));
  return launch_bracket(ctx, M, features, phi_range, counts, cap, delta_scale, hint_lo, hint_hi);
}
