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

__global__ __launch_bounds__(kRbBlock) void robin_kernel(RobinParams p) {
  const DevMesh &m = p.m;
  const int64_t N = m.n_cells, NF = m.n_faces;
  const int64_t nb = p.counts[1];
  constexpr int kCells = kRbBlock / kRbLanes;
  const int lane = threadIdx.x % kRbLanes;
  // a row of 16 lanes per band cell, one face per lane
  for (int64_t k = blockIdx.x * (int64_t)kCells + threadIdx.x / kRbLanes; k < nb; k += (int64_t)gridDim.x * kCells) {
    const int C = p.band[k];
    const double aC = p.alpha[C];
    double sum = 0.0;
    for (int64_t i = m.cell_face_off[C] + lane; i < m.cell_face_off[C + 1]; i += kRbLanes) {
      const int Qn = m.cf_nbr[i];
      if (Qn < 0) continue;
      if (!((aC - 0.5) * (p.alpha[Qn] - 0.5) < 0.0)) continue;
      const int f = m.cell_face[i];
      const int P = m.face_owner[f], Q = m.face_neigh[f];
      const double aP = p.alpha[P], aQ = p.alpha[Q];
      const double S0 = m.Sf[f], S1 = m.Sf[NF + f], S2 = m.Sf[2 * NF + f];
      const double mag = sqrt(S0 * S0 + S1 * S1 + S2 * S2);
      const double n0 = S0 / mag, n1 = S1 / mag, n2 = S2 / mag;
      const double t = (aP - 0.5) / (aP - aQ);
      const double xP0 = m.xc[P], xP1 = m.xc[N + P], xP2 = m.xc[2 * N + P];
      const double xQ0 = m.xc[Q], xQ1 = m.xc[N + Q], xQ2 = m.xc[2 * N + Q];
      const double xf0 = xP0 + t * (xQ0 - xP0), xf1 = xP1 + t * (xQ1 - xP1), xf2 = xP2 + t * (xQ2 - xP2);
      double sp[3], sq[3];
      area_vector(p, P, sp);
      area_vector(p, Q, sq);
      const double area = fabs(n0 * (sp[0] + sq[0]) + n1 * (sp[1] + sq[1]) + n2 * (sp[2] + sq[2]));
      const double dP = fabs(n0 * (xf0 - xP0) + n1 * (xf1 - xP1) + n2 * (xf2 - xP2));
      const double dQ = fabs(n0 * (xf0 - xQ0) + n1 * (xf1 - xQ1) + n2 * (xf2 - xQ2));
      const double kP = aP >= 0.5 ? p.k_l : p.k_v, kQ = aQ >= 0.5 ? p.k_l : p.k_v;
      const double cP = dP > 0.0 ? kP * area / dP : 0.0;
      const double cQ = dQ > 0.0 ? kQ * area / dQ : 0.0;
      sum += (C == P) ? cP : cQ;
      // the owner side appends the face record: one counter claim per
      // wave for all its active lanes that append
      const bool app = C == P && p.n_face;
      const uint64_t bm = __ballot(app);
      const int wl = threadIdx.x & 63;
      const int leader = bm ? __ffsll((long long)bm) - 1 : 0;
      int base = 0;
      if (wl == leader && bm) base = atomicAdd(p.n_face, __popcll(bm));
      base = __shfl(base, leader);
      if (app) {
        const int j = base + __popcll(bm & ((wl == 0) ? 0ull : (~0ull >> (64 - wl))));
        if (j < p.face_cap) {
          const int64_t fc = p.face_cap;
          if (p.face_idx) p.face_idx[j] = f;
          if (p.face_a) { p.face_a[j] = cP; p.face_a[fc + j] = cQ; }
          if (p.face_d) { p.face_d[j] = dP; p.face_d[fc + j] = dQ; }
          if (p.face_area) p.face_area[j] = area;
        }
      }
    }
    sum = gsum<kRbLanes>(sum);
    if (lane == 0 && p.a_diag) p.a_diag[k] = sum;
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
