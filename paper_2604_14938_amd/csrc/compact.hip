// Mixed-cell and gradient-band compaction: wavefront ballots, a block scan and
// a scan of the block totals, giving stable (ascending) index lists and their
// lengths in device memory.
#include <hip/hip_runtime.h>

#include "vofpc_internal.h"

namespace vofpc {

constexpr int kCompactBlock = kCompactBlockCells;
constexpr int kWaves = kCompactBlock / 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Per cell: bit 0 mixed (eps < alpha < 1-eps), bit 1 band (mixed, or a face
// neighbour on the other side of alpha = 1/2).  Block totals of both.
__global__ __launch_bounds__(kCompactBlock) void compact_flags_kernel(DevMesh m, const double *alpha, double eps,
                                                                      uint8_t *flags, int32_t *blk_cnt,
                                                                      int64_t n_blk) {
  __shared__ int32_t wsum[2][kWaves];
  const int64_t P = blockIdx.x * (int64_t)kCompactBlock + threadIdx.x;
  bool mixed = false, band = false;
  if (P < m.n_cells) {
    double a = alpha[P];
    mixed = (a > eps) && (a < 1.0 - eps);
    band = mixed;
    if (!band) {
      double ha = a - 0.5;
      for (int64_t i = m.cell_face_off[P]; i < m.cell_face_off[P + 1]; ++i) {
        int q = m.cf_nbr[i];
        if (q >= 0 && ha * (alpha[q] - 0.5) < 0.0) { band = true; break; }
      }
    }
    flags[P] = (uint8_t)((mixed ? 1 : 0) | (band ? 2 : 0));
  }
  uint64_t bm = __ballot(mixed), bb = __ballot(band);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    wsum[0][w] = __popcll(bm);
    wsum[1][w] = __popcll(bb);
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    int32_t t = 0;
    for (int i = 0; i < kWaves; ++i) t += wsum[threadIdx.x][i];
    blk_cnt[threadIdx.x * n_blk + blockIdx.x] = t;
  }
}

// Exclusive scan of the block totals of both lists (one block) and the list
// lengths.
__global__ __launch_bounds__(1024) void compact_scan_kernel(const int32_t *blk_cnt, int32_t *blk_off, int64_t n_blk,
                                                            int32_t *counts) {
  __shared__ int32_t part[1024];
  for (int list = 0; list < 2; ++list) {
    const int32_t *c = blk_cnt + list * n_blk;
    int32_t *o = blk_off + list * n_blk;
    const int64_t per = (n_blk + 1023) / 1024;
    const int64_t b = threadIdx.x * per, e = (b + per < n_blk) ? b + per : n_blk;
    int32_t s = 0;
    for (int64_t i = b; i < e; ++i) s += c[i];
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 1024 partial sums
    for (int d = 1; d < 1024; d <<= 1) {
      int32_t t = (threadIdx.x >= (unsigned)d) ? part[threadIdx.x - d] : 0;
      __syncthreads();
      part[threadIdx.x] += t;
      __syncthreads();
    }
    int32_t run = part[threadIdx.x] - s;
    for (int64_t i = b; i < e; ++i) {
      o[i] = run;
      run += c[i];
    }
    if (threadIdx.x == 1023) counts[list] = part[1023];
    __syncthreads();
  }
}

// Scatter the cell ids into both lists in ascending order.
__global__ __launch_bounds__(kCompactBlock) void compact_scatter_kernel(int64_t n_cells, const uint8_t *flags,
                                                                        const int32_t *blk_off, int64_t n_blk,
                                                                        int32_t *mixed_idx, int32_t *band_idx) {
  __shared__ int32_t wbase[2][kWaves];
  const int64_t P = blockIdx.x * (int64_t)kCompactBlock + threadIdx.x;
  uint8_t f = (P < n_cells) ? flags[P] : 0;
  bool mixed = f & 1, band = f & 2;
  uint64_t bm = __ballot(mixed), bb = __ballot(band);
  const int w = threadIdx.x >> 6, l = lane_id();
  const uint64_t below = (l == 0) ? 0ull : (~0ull >> (64 - l));
  if (l == 0) {
    wbase[0][w] = __popcll(bm);
    wbase[1][w] = __popcll(bb);
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    int32_t run = blk_off[threadIdx.x * n_blk + blockIdx.x];
    for (int i = 0; i < kWaves; ++i) {
      int32_t t = wbase[threadIdx.x][i];
      wbase[threadIdx.x][i] = run;
      run += t;
    }
  }
  __syncthreads();
  if (mixed) mixed_idx[wbase[0][w] + __popcll(bm & below)] = (int32_t)P;
  if (band) band_idx[wbase[1][w] + __popcll(bb & below)] = (int32_t)P;
}

vofpc_status launch_compact(vofpc_ctx ctx, vofpc_mesh M, const double *alpha, double eps, int32_t *mixed,
                            int32_t *band, int32_t *counts) {
  VOFPC_REQUIRE(alpha && mixed && band && counts, VOFPC_E_INVALID_ARG, "compact: null pointer");
  VOFPC_REQUIRE(eps >= 0 && eps < 0.5, VOFPC_E_INVALID_ARG, "compact: eps_mixed must be in [0, 0.5)");
  const int64_t nb = M->n_blk;
  hipStream_t s = ctx->stream;
  compact_flags_kernel<<<(unsigned)nb, kCompactBlock, 0, s>>>(M->d, alpha, eps, M->flags, M->blk_cnt, nb);
  compact_scan_kernel<<<1, 1024, 0, s>>>(M->blk_cnt, M->blk_off, nb, counts);
  compact_scatter_kernel<<<(unsigned)nb, kCompactBlock, 0, s>>>(M->d.n_cells, M->flags, M->blk_off, nb, mixed,
                                                                  band);
  VOFPC_HIP(hipGetLastError());
  return VOFPC_OK;
}

}  // namespace vofpc
