// Interface heat-transfer coefficients of the implicit energy coupling
// (Eq. interface_htc, Sec. 2.4.4 "Heat source/sink").  An interior face whose
// two cells lie on opposite sides of alpha = 1/2 is detached from the
// diffusion operator; each of its cells C is tied to T_sat instead with
//   a_f,C = k_C A_int,f / d_f,C,
// k_C the conductivity of C's phase (liquid when alpha_C >= 1/2), d_f,C the
// distance from x_C to the alpha-interpolated crossing point x_f of the
// gradient stencil (Eq. front_interpolation, read as x_P + t (x_Q - x_P),
// t = (a_P - 1/2)/(a_P - a_Q)) measured along the face normal, and A_int,f the
// face-normal projection of the two cells' interface area vectors A n.
//
// Three small kernels: the mixed list is scattered into a per-mesh map
// cell -> entry (so a face can find both cells' interfaces), a row of 16
// lanes per band entry (one face per lane) sums its side of every detached
// face and the owner side appends the face record, and the map is cleared
// again (it stays -1 between calls).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "vofpc_internal.h"
#include "wave_ops.h"

namespace vofpc {

constexpr int kRbBlock = 256;
constexpr int kRbLanes = 16;   // lanes per band cell (one DPP row)

__global__ __launch_bounds__(256) void robin_map_kernel(const int32_t *mixed, const int32_t *counts, int64_t cap,
                                                        int32_t *entry, int32_t value_is_index, int32_t *n_face) {
  int64_t n = counts[0];
  if (n > cap) n = cap;
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) entry[mixed[k]] = value_is_index ? (int32_t)k : -1;
  if (n_face && k == 0) *n_face = 0;
}

struct RobinParams {
  DevMesh m;
  const double *alpha;
  const int32_t *band;
  const int32_t *counts;
  const int32_t *entry;
  vofpc_interface itf;
  double k_l, k_v;
  double *a_diag;
  int64_t face_cap;
  int32_t *face_idx;
  double *face_a, *face_d, *face_area;
  int32_t *n_face;
};

// interface area vector A n of a cell (zero without an interface)
__device__ __forceinline__ void area_vector(const RobinParams &p, int C, double *s) {
  const int e = p.entry[C];
  if (e < 0) {
    s[0] = s[1] = s[2] = 0.0;
    return;
  }
  const int64_t cap = p.itf.cap;
  const double A = p.itf.A[e];
  s[0] = A * p.itf.n[e];
  s[1] = A * p.itf.n[cap + e];
  s[2] = A * p.itf.n[2 * cap + e];
}

// One interior slot of band cell C: whether the face is detached (its two
// cells on opposite sides of alpha = 1/2), whether C owns it, and its record.
struct FaceRec {
  int f;
  double cP, cQ, dP, dQ, area;
};

__device__ __forceinline__ bool face_coupling(const RobinParams &p, int C, double aC, const double *xC,
                                              const double *sC, int64_t i, FaceRec &r, bool &cown) {
  const DevMesh &m = p.m;
  const int64_t N = m.n_cells, NF = m.n_faces;
  const int Qn = m.cf_nbr[i];
  const int f = m.cell_face[i];
  if (Qn < 0) return false;
  // every load of the face is made before the crossing test (they depend
  // only on the slot and its two cells) and the arithmetic runs on every
  // face: a detached face waits for three rounds of dependent loads, not six
  const int own = m.face_owner[f];
  const double aN = p.alpha[Qn];
  const double S0 = m.Sf[f], S1 = m.Sf[NF + f], S2 = m.Sf[2 * NF + f];
  const double xN0 = m.xc[Qn], xN1 = m.xc[N + Qn], xN2 = m.xc[2 * N + Qn];
  double sN[3];
  area_vector(p, Qn, sN);
  const bool cross = (aC - 0.5) * (aN - 0.5) < 0.0;
  // the face's owner P and neighbour Q
  cown = own == C;
  const double aP = cown ? aC : aN, aQ = cown ? aN : aC;
  const double xP0 = cown ? xC[0] : xN0, xP1 = cown ? xC[1] : xN1, xP2 = cown ? xC[2] : xN2;
  const double xQ0 = cown ? xN0 : xC[0], xQ1 = cown ? xN1 : xC[1], xQ2 = cown ? xN2 : xC[2];
  const double mag = sqrt(S0 * S0 + S1 * S1 + S2 * S2);
  const double n0 = S0 / mag, n1 = S1 / mag, n2 = S2 / mag;
  const double t = (aP - 0.5) / (aP - aQ);
  const double xf0 = xP0 + t * (xQ0 - xP0), xf1 = xP1 + t * (xQ1 - xP1), xf2 = xP2 + t * (xQ2 - xP2);
  const double sp0 = cown ? sC[0] : sN[0], sp1 = cown ? sC[1] : sN[1], sp2 = cown ? sC[2] : sN[2];
  const double sq0 = cown ? sN[0] : sC[0], sq1 = cown ? sN[1] : sC[1], sq2 = cown ? sN[2] : sC[2];
  r.f = f;
  r.area = fabs(n0 * (sp0 + sq0) + n1 * (sp1 + sq1) + n2 * (sp2 + sq2));
  r.dP = fabs(n0 * (xf0 - xP0) + n1 * (xf1 - xP1) + n2 * (xf2 - xP2));
  r.dQ = fabs(n0 * (xf0 - xQ0) + n1 * (xf1 - xQ1) + n2 * (xf2 - xQ2));
  const double kP = aP >= 0.5 ? p.k_l : p.k_v, kQ = aQ >= 0.5 ? p.k_l : p.k_v;
  r.cP = r.dP > 0.0 ? kP * r.area / r.dP : 0.0;
  r.cQ = r.dQ > 0.0 ? kQ * r.area / r.dQ : 0.0;
  return cross;
}

__device__ __forceinline__ void write_record(const RobinParams &p, int64_t j, const FaceRec &r) {
  if (j >= p.face_cap) return;
  const int64_t fc = p.face_cap;
  if (p.face_idx) p.face_idx[j] = r.f;
  if (p.face_a) { p.face_a[j] = r.cP; p.face_a[fc + j] = r.cQ; }
  if (p.face_d) { p.face_d[j] = r.dP; p.face_d[fc + j] = r.dQ; }
  if (p.face_area) p.face_area[j] = r.area;
}

__global__ __launch_bounds__(kRbBlock) void robin_kernel(RobinParams p) {
  constexpr int kCells = kRbBlock / kRbLanes;
  constexpr int kWaves = kRbBlock / 64;
  __shared__ int wsum[kWaves];
  __shared__ int bbase;
  const DevMesh &m = p.m;
  const int64_t N = m.n_cells;
  const int64_t nb = p.counts[1];
  const int lane = threadIdx.x % kRbLanes;
  const int wl = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // a row of 16 lanes per band cell, one face per lane; the block walks the
  // band in steps of 16 cells together (the face records are claimed once
  // per block and step)
  for (int64_t k0 = blockIdx.x * (int64_t)kCells; k0 < nb; k0 += (int64_t)gridDim.x * kCells) {
    const int64_t k = k0 + threadIdx.x / kRbLanes;
    int C = -1, cnt = 0;
    double aC = 0.0, xC[3] = {0.0, 0.0, 0.0}, sC[3] = {0.0, 0.0, 0.0};
    FaceRec last{0, 0.0, 0.0, 0.0, 0.0, 0.0};   // the lane's last detached face it owns
    if (k < nb) {
      C = p.band[k];
      aC = p.alpha[C];
      xC[0] = m.xc[C]; xC[1] = m.xc[N + C]; xC[2] = m.xc[2 * N + C];
      area_vector(p, C, sC);
      double sum = 0.0;
      for (int64_t i = m.cell_face_off[C] + lane; i < m.cell_face_off[C + 1]; i += kRbLanes) {
        FaceRec r;
        bool cown;
        if (!face_coupling(p, C, aC, xC, sC, i, r, cown)) continue;
        sum += cown ? r.cP : r.cQ;
        if (cown) { last = r; ++cnt; }
      }
      sum = gsum<kRbLanes>(sum);
      if (lane == 0 && p.a_diag) p.a_diag[k] = sum;
    }
    if (!p.n_face) continue;
    // records: the owner side appends each detached face; offsets from a
    // block-wide prefix of the lanes' counts and one counter claim
    int incl = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int t = __shfl_up(incl, d);
      if (wl >= d) incl += t;
    }
    if (wl == 63) wsum[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < kWaves; ++w) {
        const int t = wsum[w];
        wsum[w] = tot;
        tot += t;
      }
      bbase = tot ? atomicAdd(p.n_face, tot) : 0;
    }
    __syncthreads();
    int64_t j = (int64_t)bbase + wsum[wave] + (incl - cnt);
    if (cnt == 1) {
      write_record(p, j, last);
    } else if (cnt > 1) {
      // more than one owned detached face on this lane (cells with more
      // than 16 faces): walk the lane's faces again in the same order
      for (int64_t i = m.cell_face_off[C] + lane; i < m.cell_face_off[C + 1]; i += kRbLanes) {
        FaceRec r;
        bool cown;
        if (face_coupling(p, C, aC, xC, sC, i, r, cown) && cown) write_record(p, j++, r);
      }
    }
    __syncthreads();   // wsum and bbase are rewritten by the next step
  }
}

}  // namespace vofpc

using namespace vofpc;

extern "C" vofpc_status vofpc_robin(vofpc_ctx ctx, vofpc_mesh M, const double *alpha, const int32_t *mixed_idx,
                                    const int32_t *band_idx, const int32_t *counts, const vofpc_interface *itf,
                                    double k_l, double k_v, double *a_diag, int64_t face_cap, int32_t *face_idx,
                                    double *face_a, double *face_d, double *face_area, int32_t *n_face) {
  clear_error();
  VOFPC_REQUIRE(ctx && M && alpha && mixed_idx && band_idx && counts && itf, VOFPC_E_INVALID_ARG,
                "robin: null argument");
  VOFPC_REQUIRE(M->ctx && M->ctx->device == ctx->device, VOFPC_E_STATE, "robin: mesh on another device");
  VOFPC_REQUIRE(itf->n && itf->A && itf->cap > 0, VOFPC_E_INVALID_ARG, "robin: interface record incomplete");
  VOFPC_REQUIRE(face_cap >= 0, VOFPC_E_INVALID_ARG, "robin: negative face capacity");
  VOFPC_REQUIRE(!(face_idx || face_a || face_d || face_area) || n_face, VOFPC_E_INVALID_ARG,
                "robin: face records need the n_face counter");
  VOFPC_HIP(hipSetDevice(ctx->device));
  const int64_t N = M->d.n_cells;
  hipStream_t s = ctx->stream;
  if (!M->rb_entry) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    VOFPC_HIP(hipStreamIsCapturing(s, &cs));
    VOFPC_REQUIRE(cs == hipStreamCaptureStatusNone, VOFPC_E_STATE,
                  "robin: the first call on a mesh sets up its buffers and must not be captured");
    void *a = nullptr;
    vofpc_status st = mesh_scratch_alloc(M, 4 * (size_t)N, &a);
    if (st) return st;
    VOFPC_HIP(hipMemset(a, 0xff, 4 * (size_t)N));   // -1: no entry
    M->rb_entry = (int32_t *)a;
  }
  const int64_t cap = std::min<int64_t>(itf->cap, N);
  const unsigned gM = (unsigned)std::max<int64_t>(1, (cap + 255) / 256);
  robin_map_kernel<<<gM, 256, 0, s>>>(mixed_idx, counts, itf->cap, M->rb_entry, 1, n_face);
  RobinParams p;
  p.m = M->d;
  p.alpha = alpha;
  p.band = band_idx;
  p.counts = counts;
  p.entry = M->rb_entry;
  p.itf = *itf;
  p.k_l = k_l;
  p.k_v = k_v;
  p.a_diag = a_diag;
  p.face_cap = face_cap;
  p.face_idx = face_idx;
  p.face_a = face_a;
  p.face_d = face_d;
  p.face_area = face_area;
  p.n_face = n_face;
  const int64_t cells_per_block = kRbBlock / kRbLanes;
  const unsigned gB = (unsigned)std::max<int64_t>(
      1, std::min<int64_t>((N + cells_per_block - 1) / cells_per_block, (int64_t)ctx->n_cu * 4));
  robin_kernel<<<gB, kRbBlock, 0, s>>>(p);
  robin_map_kernel<<<gM, 256, 0, s>>>(mixed_idx, counts, itf->cap, M->rb_entry, 0, nullptr);
  VOFPC_HIP(hipGetLastError());
  return VOFPC_OK;
}
