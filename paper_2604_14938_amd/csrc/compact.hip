// Mixed-cell and gradient-band compaction: a side-bit pass and a face pass
// for the band test (meshes with cells of at most eight faces test it in the
// cell pass), a
// cell pass with wavefront ballots and block totals, the exclusive prefix of
// the block totals, and a scatter, giving stable (ascending) index lists and
// their lengths in device memory.  Up to kScanBlocks blocks each scatter
// block sums the totals before it itself (no extra launch); beyond that a
// one-block scan kernel computes the prefix once, so the work stays linear
// in the number of blocks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "vofpc_internal.h"
#include "wave_ops.h"

namespace vofpc {

constexpr int kCompactBlock = kCompactBlockCells;
constexpr int kWaves = kCompactBlock / 64;
constexpr int64_t kScanBlocks = 4096;   // above this many blocks the prefix is scanned once
constexpr int kScanThreads = 1024;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// The side of alpha = 1/2 of every cell as two bits, above (alpha > 1/2)
// and below (alpha < 1/2; a NaN is neither): side[2w] and side[2w + 1] hold
// the two bits of cells 64w .. 64w + 63, so the face pass gathers from
// n_cells / 4 bytes (held in L2) instead of the 8-byte alphas.
__global__ __launch_bounds__(kCompactBlock) void compact_side_kernel(int64_t n, const double *alpha,
                                                                     uint64_t *side) {
  const int64_t P = blockIdx.x * (int64_t)kCompactBlock + threadIdx.x;
  const double a = P < n ? alpha[P] : 0.5;
  const uint64_t above = __ballot(a > 0.5), below = __ballot(a < 0.5);
  // lane 0 holds the wavefront's first cell: only wavefronts that start
  // inside the mesh have a word (the array holds ceil(n / 64) of them)
  if (lane_id() == 0 && P < n) {
    const int64_t w = P >> 6;
    side[2 * w] = above;
    side[2 * w + 1] = below;
  }
}

// Faces whose two cells lie strictly on opposite sides of alpha = 1/2 (the
// product of their alpha - 1/2 is negative) put both cells in the band
// (interior faces only).  `cross` is a per-cell byte array that the cell
// pass reads and clears again, so the next step starts from zeros.  Each
// thread takes kFaceRun consecutive faces: their owners and neighbours in
// two 16-byte loads, then every side word they need in flight together.
constexpr int kFaceRun = 4;   // a multiple of 4
static_assert(kFaceRun % 4 == 0, "whole 16-byte loads");
__global__ __launch_bounds__(kCompactBlock) void compact_faces_kernel(DevMesh m, const uint64_t *side,
                                                                      uint8_t *cross) {
  const int64_t f0 = (blockIdx.x * (int64_t)kCompactBlock + threadIdx.x) * kFaceRun;
  const int64_t nf = m.n_faces;
  if (f0 >= nf) return;
  int o[kFaceRun], q[kFaceRun];
  if (f0 + kFaceRun <= nf) {
#pragma unroll
    for (int h = 0; h < kFaceRun; h += 4) {
      const int4 ov = *reinterpret_cast<const int4 *>(m.face_owner + f0 + h);
      const int4 qv = *reinterpret_cast<const int4 *>(m.face_neigh + f0 + h);
      o[h] = ov.x; o[h + 1] = ov.y; o[h + 2] = ov.z; o[h + 3] = ov.w;
      q[h] = qv.x; q[h + 1] = qv.y; q[h + 2] = qv.z; q[h + 3] = qv.w;
    }
  } else {
#pragma unroll
    for (int t = 0; t < kFaceRun; ++t) {
      o[t] = f0 + t < nf ? m.face_owner[f0 + t] : 0;
      q[t] = f0 + t < nf ? m.face_neigh[f0 + t] : -1;
    }
  }
  const ulonglong2 *sw = reinterpret_cast<const ulonglong2 *>(side);
  ulonglong2 so[kFaceRun], sq[kFaceRun];
#pragma unroll
  for (int t = 0; t < kFaceRun; ++t) {
    so[t] = sw[o[t] >> 6];
    sq[t] = q[t] >= 0 ? sw[q[t] >> 6] : ulonglong2{0ull, 0ull};
  }
#pragma unroll
  for (int t = 0; t < kFaceRun; ++t) {
    if (q[t] < 0) continue;
    const int bo = o[t] & 63, bq = q[t] & 63;
    const uint64_t cr = ((so[t].x >> bo) & (sq[t].y >> bq)) | ((so[t].y >> bo) & (sq[t].x >> bq));
    if (cr & 1ull) {
      cross[o[t]] = 1;
      cross[q[t]] = 1;
    }
  }
}

// Per cell: bit 0 mixed (eps < alpha < 1-eps), bit 1 band (mixed, or a face
// neighbour on the other side of alpha = 1/2).  Block totals of both.
__global__ __launch_bounds__(kCompactBlock) void compact_flags_kernel(DevMesh m, const double *alpha, double eps,
                                                                      uint8_t *cross, uint8_t *flags,
                                                                      int32_t *blk_cnt, int64_t n_blk) {
  __shared__ int32_t wsum[2][kWaves];
  const int64_t P = blockIdx.x * (int64_t)kCompactBlock + threadIdx.x;
  bool mixed = false, band = false;
  if (P < m.n_cells) {
    const double a = alpha[P];
    mixed = (a > eps) && (a < 1.0 - eps);
    const uint8_t cr = cross[P];
    band = mixed || cr;
    if (cr) cross[P] = 0;
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

// The same flags and totals without the face pass, for meshes whose cells
// have at most eight faces (hexahedra): each cell tests the band over its own
// face neighbours, the eight slots' loads in flight together.  With more
// faces per cell these reads scatter and the face pass is faster.
__global__ __launch_bounds__(kCompactBlock) void compact_cells_kernel(DevMesh m, const double *alpha, double eps,
                                                                      uint8_t *flags, int32_t *blk_cnt,
                                                                      int64_t n_blk) {
  __shared__ int32_t wsum[2][kWaves];
  const int64_t P = blockIdx.x * (int64_t)kCompactBlock + threadIdx.x;
  bool mixed = false, band = false;
  if (P < m.n_cells) {
    const double a = alpha[P];
    mixed = (a > eps) && (a < 1.0 - eps);
    band = mixed;
    const int64_t i0 = m.cell_face_off[P], i1 = m.cell_face_off[P + 1];
    int q[8];
    double aq[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) q[t] = (i0 + t < i1) ? m.cf_nbr[i0 + t] : -1;
#pragma unroll
    for (int t = 0; t < 8; ++t) aq[t] = q[t] >= 0 ? alpha[q[t]] : 0.5;
#pragma unroll
    for (int t = 0; t < 8; ++t) band = band || ((a - 0.5) * (aq[t] - 0.5) < 0.0);
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

// Exclusive prefix of both rows of block totals, in place, by one block, a
// tile of kScanTile totals per row at a time: coalesced loads (the next
// tile's issued before the current one is scanned) staged through LDS, each
// thread scans kScanPer consecutive totals, the thread sums are scanned
// within each wavefront by shuffles and then across the wavefronts, and a
// carry per row runs from tile to tile.  Writes the list lengths.
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanThreads * kScanPer;
__global__ __launch_bounds__(kScanThreads) void compact_scan_kernel(int32_t *blk_cnt, int64_t n_blk,
                                                                    int32_t *counts) {
  constexpr int kW = kScanThreads / 64;
  __shared__ int32_t tile[2][kScanTile];
  __shared__ int32_t wtot[2][kW];
  const int t = threadIdx.x, w = t >> 6, l = lane_id();
  int32_t cur[2][kScanPer];
  auto load = [&](int64_t t0) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < kScanPer; ++j) {
        const int64_t g = t0 + j * kScanThreads + t;
        cur[r][j] = g < n_blk ? blk_cnt[r * n_blk + g] : 0;
      }
  };
  int32_t carry[2] = {0, 0};
  load(0);
  for (int64_t t0 = 0; t0 < n_blk; t0 += kScanTile) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < kScanPer; ++j) tile[r][j * kScanThreads + t] = cur[r][j];
    if (t0 + kScanTile < n_blk) load(t0 + kScanTile);
    __syncthreads();
    int32_t v[2][kScanPer], ex[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      int32_t s = 0;
#pragma unroll
      for (int j = 0; j < kScanPer; ++j) {
        v[r][j] = tile[r][t * kScanPer + j];
        s += v[r][j];
      }
      int32_t inc = s;
      for (int d = 1; d < 64; d <<= 1) {
        const int32_t u = __shfl_up(inc, d);
        if (l >= d) inc += u;
      }
      ex[r] = inc - s;
      if (l == 63) wtot[r][w] = inc;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      int32_t base = 0, all = 0;
      for (int i = 0; i < kW; ++i) {
        base += (i < w) ? wtot[r][i] : 0;
        all += wtot[r][i];
      }
      int32_t run = carry[r] + base + ex[r];
#pragma unroll
      for (int j = 0; j < kScanPer; ++j) {
        tile[r][t * kScanPer + j] = run;
        run += v[r][j];
      }
      carry[r] += all;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < kScanPer; ++j) {
        const int64_t g = t0 + j * kScanThreads + t;
        if (g < n_blk) blk_cnt[r * n_blk + g] = tile[r][j * kScanThreads + t];
      }
    __syncthreads();
  }
  if (t < 2) counts[t] = carry[t];
}

// Scatter the cell ids into both lists in ascending order.  With `scanned`
// the block totals already hold their exclusive prefix; otherwise each block
// sums the totals of the blocks before it and the last block writes the list
// lengths.
__global__ __launch_bounds__(kCompactBlock) void compact_scatter_kernel(int64_t n_cells, const uint8_t *flags,
                                                                        const int32_t *blk_cnt, int64_t n_blk,
                                                                        int scanned, int32_t *mixed_idx,
                                                                        int32_t *band_idx, int32_t *counts) {
  __shared__ int32_t wbase[2][kWaves];
  __shared__ int32_t part[2][kWaves];
  const int64_t b = blockIdx.x;
  const int w = threadIdx.x >> 6, l = lane_id();
  if (scanned) {
    if (threadIdx.x < 2) {
      part[threadIdx.x][0] = blk_cnt[threadIdx.x * n_blk + b];
      for (int i = 1; i < kWaves; ++i) part[threadIdx.x][i] = 0;
    }
  } else {
    // exclusive prefix of the block totals
    int32_t s0 = 0, s1 = 0;
    for (int64_t i = threadIdx.x; i < b; i += kCompactBlock) {
      s0 += blk_cnt[i];
      s1 += blk_cnt[n_blk + i];
    }
    for (int o = 32; o > 0; o >>= 1) {
      s0 += __shfl_xor(s0, o);
      s1 += __shfl_xor(s1, o);
    }
    if (l == 0) {
      part[0][w] = s0;
      part[1][w] = s1;
    }
  }
  const int64_t P = b * kCompactBlock + threadIdx.x;
  uint8_t f = (P < n_cells) ? flags[P] : 0;
  bool mixed = f & 1, band = f & 2;
  uint64_t bm = __ballot(mixed), bb = __ballot(band);
  if (l == 0) {
    wbase[0][w] = __popcll(bm);
    wbase[1][w] = __popcll(bb);
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    int32_t run = 0;
    for (int i = 0; i < kWaves; ++i) run += part[threadIdx.x][i];
    for (int i = 0; i < kWaves; ++i) {
      int32_t t = wbase[threadIdx.x][i];
      wbase[threadIdx.x][i] = run;
      run += t;
    }
    if (!scanned && b == n_blk - 1) counts[threadIdx.x] = run;
  }
  __syncthreads();
  if (mixed) mixed_idx[wbase[0][w] + lanes_below(bm)] = (int32_t)P;
  if (band) band_idx[wbase[1][w] + lanes_below(bb)] = (int32_t)P;
}

// The compaction on the given scratch: flags [n_cells] bytes, cross
// [n_cells] bytes (zero on entry; the cell pass clears what the face pass
// set), blk_cnt [2][n_blk] and side [2][ceil(n_cells / 64)] words (16-byte
// aligned; written before it is read).
static vofpc_status compact_on(vofpc_ctx ctx, vofpc_mesh M, const double *alpha, double eps, int32_t *mixed,
                               int32_t *band, int32_t *counts, uint8_t *flags, uint8_t *cross, int32_t *blk_cnt,
                               uint64_t *side) {
  VOFPC_REQUIRE(alpha && mixed && band && counts, VOFPC_E_INVALID_ARG, "compact: null pointer");
  VOFPC_REQUIRE(eps >= 0 && eps < 0.5, VOFPC_E_INVALID_ARG, "compact: eps_mixed must be in [0, 0.5)");
  const int64_t nb = M->n_blk;
  hipStream_t s = ctx->stream;
  if (M->max_nf <= 8) {
    compact_cells_kernel<<<(unsigned)nb, kCompactBlock, 0, s>>>(M->d, alpha, eps, flags, blk_cnt, nb);
  } else {
    compact_side_kernel<<<(unsigned)nb, kCompactBlock, 0, s>>>(M->d.n_cells, alpha, side);
    const int64_t per = (int64_t)kCompactBlock * kFaceRun;
    const int64_t nfb = (M->d.n_faces + per - 1) / per;
    compact_faces_kernel<<<(unsigned)std::max<int64_t>(nfb, 1), kCompactBlock, 0, s>>>(M->d, side, cross);
    compact_flags_kernel<<<(unsigned)nb, kCompactBlock, 0, s>>>(M->d, alpha, eps, cross, flags, blk_cnt, nb);
  }
  const int scanned = nb > kScanBlocks ? 1 : 0;
  if (scanned) compact_scan_kernel<<<1, kScanThreads, 0, s>>>(blk_cnt, nb, counts);
  compact_scatter_kernel<<<(unsigned)nb, kCompactBlock, 0, s>>>(M->d.n_cells, flags, blk_cnt, nb, scanned, mixed,
                                                                  band, counts);
  VOFPC_HIP(hipGetLastError());
  return VOFPC_OK;
}

vofpc_status launch_compact(vofpc_ctx ctx, vofpc_mesh M, const double *alpha, double eps, int32_t *mixed,
                            int32_t *band, int32_t *counts) {
  return compact_on(ctx, M, alpha, eps, mixed, band, counts, M->flags, M->cross, M->blk_cnt, M->side);
}

// ---------------------------------------------------------------- no allocation
// The compaction's scratch for callers that cannot allocate: one file-scope
// device array per GPU, held until the process ends, laid out as flags
// [kNoAllocMaxCells] bytes, band marks [kNoAllocMaxCells] bytes, block
// totals [2][kNoAllocMaxBlocks] int32 and side bits [2][kNoAllocMaxCells /
// 64] words.  In host code the array's name is not
// a device address: each device's address comes from hipGetSymbolAddress
// (once per device, with that device current) and only that address is used.
constexpr int64_t kNoAllocMaxCells = int64_t(1) << 23;   // 8,388,608 cells
constexpr int64_t kNoAllocMaxBlocks = kNoAllocMaxCells / kCompactBlock;
constexpr int64_t kNoAllocSideOffset = 2 * kNoAllocMaxCells + 2 * kNoAllocMaxBlocks * (int64_t)sizeof(int32_t);
constexpr int64_t kNoAllocBytes = kNoAllocSideOffset + 2 * (kNoAllocMaxCells / 64) * (int64_t)sizeof(uint64_t);
static_assert(kNoAllocSideOffset % 16 == 0, "side words 16-byte aligned");
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_scratch_mu;
static uint8_t *g_scratch_ptr[kNoAllocMaxDevices] = {};

__global__ __launch_bounds__(kCompactBlock) void zero_bytes_kernel(uint8_t *p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)kCompactBlock + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace vofpc

extern "C" vofpc_status vofpc_compact_noalloc(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha, double eps,
                                              int32_t *mixed_idx, int32_t *band_idx, int32_t *counts) {
  using namespace vofpc;
  clear_error();
  VOFPC_REQUIRE(ctx && mesh, VOFPC_E_INVALID_ARG, "compact_noalloc: null context or mesh");
  VOFPC_REQUIRE(mesh->ctx && mesh->ctx->device == ctx->device, VOFPC_E_STATE,
                "compact_noalloc: mesh on another device");
  const int64_t N = mesh->d.n_cells;
  VOFPC_REQUIRE(N <= kNoAllocMaxCells && mesh->n_blk <= kNoAllocMaxBlocks, VOFPC_E_INVALID_ARG,
                "compact_noalloc: meshes of more than 8,388,608 cells exceed its fixed scratch (use vofpc_compact)");
  VOFPC_REQUIRE(ctx->device >= 0 && ctx->device < kNoAllocMaxDevices, VOFPC_E_STATE,
                "compact_noalloc: device index beyond the scratch table");
  VOFPC_HIP(hipSetDevice(ctx->device));
  uint8_t *base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[ctx->device]) {
      void *ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) {
        set_error(std::string("compact_noalloc: hipGetSymbolAddress of the scratch array failed: ") +
                  hipGetErrorString(e));
        return VOFPC_E_HIP;
      }
      g_scratch_ptr[ctx->device] = (uint8_t *)ptr;
    }
    base = g_scratch_ptr[ctx->device];
  }
  uint8_t *flags = base, *cross = base + kNoAllocMaxCells;
  int32_t *blk_cnt = reinterpret_cast<int32_t *>(base + 2 * kNoAllocMaxCells);
  uint64_t *side = reinterpret_cast<uint64_t *>(base + kNoAllocSideOffset);
  // the band marks must start at zero: the array keeps the last call's
  // contents (a call that stopped early may have left marks)
  zero_bytes_kernel<<<(unsigned)((N + kCompactBlock - 1) / kCompactBlock), kCompactBlock, 0, ctx->stream>>>(cross, N);
  VOFPC_HIP(hipGetLastError());
  return compact_on(ctx, mesh, alpha, eps, mixed_idx, band_idx, counts, flags, cross, blk_cnt, side);
}
