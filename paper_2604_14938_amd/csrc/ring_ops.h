// Cell domains grown by rings of interior face neighbours, and their lists:
// the extrapolation and the curvature chain both work on the cells within a
// few rings of the interface.
#pragma once

#include <hip/hip_runtime.h>

#include "vofpc_internal.h"
#include "wave_ops.h"

namespace vofpc {

constexpr int kRingBlock = 256;

// grow the domain by one ring: neighbours of layer l-1 cells enter at layer l
// (mark: layer of each cell, -1 outside)
static __global__ __launch_bounds__(kRingBlock) void ring_grow_kernel(DevMesh m, int8_t *mark, int l) {
  const int64_t f = blockIdx.x * (int64_t)kRingBlock + threadIdx.x;
  if (f >= m.n_faces) return;
  const int q = m.face_neigh[f];
  if (q < 0) return;
  const int o = m.face_owner[f];
  const int mo = mark[o], mq = mark[q];
  if (mo == l - 1 && mq < 0) mark[q] = (int8_t)l;
  if (mq == l - 1 && mo < 0) mark[o] = (int8_t)l;
}

// list of the marked cells (in the order of the claims: users must not
// depend on it); one atomic per block on the length in *len
static __global__ __launch_bounds__(kRingBlock) void ring_list_kernel(int64_t n, const int8_t *mark, int32_t *list,
                                                                      int32_t *len) {
  __shared__ int wave_cnt[kRingBlock / 64];
  __shared__ int base;
  const int64_t P = blockIdx.x * (int64_t)kRingBlock + threadIdx.x;
  const bool in = P < n && mark[P] >= 0;
  const uint64_t bm = __ballot(in);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wave_cnt[wave] = __popcll(bm);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < kRingBlock / 64; ++w) tot += wave_cnt[w];
    base = tot ? atomicAdd(len, tot) : 0;
  }
  __syncthreads();
  if (!in) return;
  int off = base;
  for (int w = 0; w < wave; ++w) off += wave_cnt[w];
  list[off + lanes_below(bm)] = (int32_t)P;
}

}  // namespace vofpc
