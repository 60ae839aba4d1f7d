// Surface-tension curvature of the continuum-surface-force term (Sec. 2.4,
// momentum terms, surface tension):
//   smoothing  alpha_hat_P = sum_f alpha_hat_f A_f / sum_f A_f,
//              alpha_hat_f = alpha_P + w_f (alpha_Q - alpha_P), w_f the
//              geometric weight of Q (where the centre connection meets the
//              face plane), boundary faces alpha_P; n_smooth Jacobi sweeps;
//   normal     n = grad(alpha_hat) / (|grad(alpha_hat)| + 1e-15), plain least
//              squares over interior face neighbours (App. B);
//   raw        kappa~ = -div n by the Gauss sum with n_f = n_P + w_f (n_Q - n_P);
//   step 1     kappa* = colour-weighted mean of kappa~ over P and its face
//              neighbours, w = (1 - 2|1/2 - alpha_hat|)^8;
//   step 2     kappa = the same mean of kappa* with each neighbour's weight
//              times |n_P . s_Q|^8 (s_Q the unit centre connection);
//   force      F = sigma kappa grad(alpha), plain least squares of the sharp
//              alpha.
// Every output is exact outside the cells within n_smooth + 3 rings of the
// seed (cells with alpha other than 0 or 1, or with a face neighbour of another
// alpha): a pure cell among equal neighbours keeps alpha_hat = alpha exactly
// (sums of A_f over sums of A_f), so alpha_hat differs from alpha within
// n_smooth - 1 rings, the normal is nonzero one ring further, the raw
// curvature one more, and each smoothing step one more.  The chain therefore
// fills alpha_hat = alpha and zeros everywhere (one streaming pass), lists
// that domain, and runs every stage on the list only, with 16 lanes per cell
// (one face per lane, DPP row sums) like the band gradient.  The geometric
// weight and the area of every cell-face slot depend on the mesh only and are
// built once, by the first call on a mesh.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ring_ops.h"
#include "vofpc_internal.h"
#include "wave_ops.h"

namespace vofpc {

constexpr int kCsfLanes = 16;
constexpr int kCsfBlock = 256;
constexpr int kCsfCells = kCsfBlock / kCsfLanes;
constexpr double kCsfEps = 1e-15;

// geometric weight of the neighbour across face f of cell P
__device__ __forceinline__ double csf_face_weight(const DevMesh &m, int f, int P, int Q) {
  const int64_t N = m.n_cells, NF = m.n_faces;
  const double S0 = m.Sf[f], S1 = m.Sf[NF + f], S2 = m.Sf[2 * NF + f];
  const double a = S0 * (m.xf[f] - m.xc[P]) + S1 * (m.xf[NF + f] - m.xc[N + P]) + S2 * (m.xf[2 * NF + f] - m.xc[2 * N + P]);
  const double b = S0 * (m.xc[Q] - m.xc[P]) + S1 * (m.xc[N + Q] - m.xc[N + P]) + S2 * (m.xc[2 * N + Q] - m.xc[2 * N + P]);
  return a / b;
}

__device__ __forceinline__ double colour_weight(double a) {
  const double w = 1.0 - 2.0 * fabs(0.5 - a);
  const double w2 = w * w, w4 = w2 * w2;
  return w4 * w4;
}

// rows of 16 lanes over the domain list; every lane of a row sees the same
// cell, so the row reductions see all its lanes
#define CSF_CELL_LOOP                                                                                          \
  const int lane = threadIdx.x % kCsfLanes;                                                                    \
  const int64_t nd_ = *len;                                                                                    \
  for (int64_t j_ = blockIdx.x * (int64_t)kCsfCells + threadIdx.x / kCsfLanes; j_ < nd_;                       \
       j_ += (int64_t)gridDim.x * kCsfCells)

// per cell-face slot, once per mesh: the geometric weight of the neighbour
// (as seen from the slot's cell) and the face area
__global__ __launch_bounds__(kCsfBlock) void csf_slot_kernel(DevMesh m, double *slot) {
  const int64_t NF = m.n_faces, NS = m.cell_face_off[m.n_cells];
  const int lane = threadIdx.x % kCsfLanes;
  for (int64_t P = blockIdx.x * (int64_t)kCsfCells + threadIdx.x / kCsfLanes; P < m.n_cells;
       P += (int64_t)gridDim.x * kCsfCells) {
    for (int64_t i = m.cell_face_off[P] + lane; i < m.cell_face_off[P + 1]; i += kCsfLanes) {
      const int f = m.cell_face[i];
      const int Q = m.cf_nbr[i];
      const double S0 = m.Sf[f], S1 = m.Sf[NF + f], S2 = m.Sf[2 * NF + f];
      slot[i] = Q >= 0 ? csf_face_weight(m, f, (int)P, Q) : 0.0;
      slot[NS + i] = sqrt(S0 * S0 + S1 * S1 + S2 * S2);
    }
  }
}

__global__ __launch_bounds__(kCsfBlock) void csf_smooth_kernel(DevMesh m, const double *slot, const int32_t *list,
                                                               const int32_t *len, const double *cur, double *nxt) {
  const int64_t NS = m.cell_face_off[m.n_cells];
  CSF_CELL_LOOP {
    const int P = list[j_];
    const double aP = cur[P];
    double num = 0.0, den = 0.0;
    for (int64_t i = m.cell_face_off[P] + lane; i < m.cell_face_off[P + 1]; i += kCsfLanes) {
      const int Q = m.cf_nbr[i];
      const double A = slot[NS + i];
      const double af = Q >= 0 ? aP + slot[i] * (cur[Q] - aP) : aP;
      num += af * A;
      den += A;
    }
    num = gsum<kCsfLanes>(num);
    den = gsum<kCsfLanes>(den);
    if (lane == 0) nxt[P] = num / den;
  }
}

__global__ __launch_bounds__(kCsfBlock) void csf_seed_faces_kernel(DevMesh m, const double *alpha, int8_t *mark) {
  const int64_t f = blockIdx.x * (int64_t)kCsfBlock + threadIdx.x;
  if (f >= m.n_faces) return;
  const int q = m.face_neigh[f];
  if (q < 0) return;
  const int o = m.face_owner[f];
  if (alpha[o] != alpha[q]) {
    mark[o] = 0;
    mark[q] = 0;
  }
}

// every cell: alpha_hat = alpha (both smoothing buffers) and every other
// output 0, their values outside the domain; and the seed of the domain,
// the cells with alpha other than 0 or 1 (the face pass adds the cells with
// a neighbour of another alpha); the domain length is reset
__global__ __launch_bounds__(kCsfBlock) void csf_fill_kernel(int64_t N, const double *alpha, double *ah, double *tmp,
                                                             double *n, double *kr, double *ks, double *kappa,
                                                             double *F, int8_t *mark, int32_t *len) {
  for (int64_t P = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; P < N; P += (int64_t)gridDim.x * blockDim.x) {
    const double a = alpha[P];
    mark[P] = (a == 0.0 || a == 1.0) ? -1 : 0;
    ah[P] = a;
    tmp[P] = a;
    n[P] = 0.0;
    n[N + P] = 0.0;
    n[2 * N + P] = 0.0;
    kr[P] = 0.0;
    ks[P] = 0.0;
    kappa[P] = 0.0;
    if (F) {
      F[P] = 0.0;
      F[N + P] = 0.0;
      F[2 * N + P] = 0.0;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *len = 0;
}

// n = g / (|g| + eps) in place, on the domain
__global__ __launch_bounds__(kCsfBlock) void csf_normalise_kernel(int64_t N, const int32_t *list, const int32_t *len,
                                                                  double *n) {
  const int64_t nd = *len;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nd; j += (int64_t)gridDim.x * blockDim.x) {
    const int P = list[j];
    const double g0 = n[P], g1 = n[N + P], g2 = n[2 * N + P];
    const double den = sqrt(g0 * g0 + g1 * g1 + g2 * g2) + kCsfEps;
    n[P] = g0 / den;
    n[N + P] = g1 / den;
    n[2 * N + P] = g2 / den;
  }
}

__global__ __launch_bounds__(kCsfBlock) void csf_divergence_kernel(DevMesh m, const double *slot, const int32_t *list,
                                                                   const int32_t *len, const double *n, double *kraw) {
  const int64_t N = m.n_cells, NF = m.n_faces;
  CSF_CELL_LOOP {
    const int P = list[j_];
    const double p0 = n[P], p1 = n[N + P], p2 = n[2 * N + P];
    double div = 0.0;
    for (int64_t i = m.cell_face_off[P] + lane; i < m.cell_face_off[P + 1]; i += kCsfLanes) {
      const int f = m.cell_face[i];
      const int Q = m.cf_nbr[i];
      double f0 = p0, f1 = p1, f2 = p2;
      if (Q >= 0) {
        const double w = slot[i];
        f0 = p0 + w * (n[Q] - p0);
        f1 = p1 + w * (n[N + Q] - p1);
        f2 = p2 + w * (n[2 * N + Q] - p2);
      }
      const double sg = (m.face_owner[f] == P) ? 1.0 : -1.0;
      div += sg * (f0 * m.Sf[f] + f1 * m.Sf[NF + f] + f2 * m.Sf[2 * NF + f]);
    }
    div = gsum<kCsfLanes>(div);
    if (lane == 0) kraw[P] = -div / m.V[P];
  }
}

__global__ __launch_bounds__(kCsfBlock) void csf_step1_kernel(DevMesh m, const int32_t *list, const int32_t *len,
                                                              const double *ah, const double *kraw, double *kstar) {
  CSF_CELL_LOOP {
    const int P = list[j_];
    double num = 0.0, den = 0.0;
    for (int64_t i = m.cell_face_off[P] + lane; i < m.cell_face_off[P + 1]; i += kCsfLanes) {
      const int Q = m.cf_nbr[i];
      if (Q < 0) continue;
      const double wQ = colour_weight(ah[Q]);
      num += kraw[Q] * wQ;
      den += wQ;
    }
    num = gsum<kCsfLanes>(num);
    den = gsum<kCsfLanes>(den);
    if (lane == 0) {
      const double wP = colour_weight(ah[P]);
      kstar[P] = (kraw[P] * wP + num) / (wP + den + kCsfEps);
    }
  }
}

// step 2, and the force where asked: F holds grad(alpha) on entry
__global__ __launch_bounds__(kCsfBlock) void csf_step2_kernel(DevMesh m, const int32_t *list, const int32_t *len,
                                                              const double *ah, const double *n, const double *kstar,
                                                              double *kappa, double sigma, double *F) {
  const int64_t N = m.n_cells;
  CSF_CELL_LOOP {
    const int P = list[j_];
    const double n0 = n[P], n1 = n[N + P], n2 = n[2 * N + P];
    const double x0 = m.xc[P], x1 = m.xc[N + P], x2 = m.xc[2 * N + P];
    double num = 0.0, den = 0.0;
    for (int64_t i = m.cell_face_off[P] + lane; i < m.cell_face_off[P + 1]; i += kCsfLanes) {
      const int Q = m.cf_nbr[i];
      if (Q < 0) continue;
      const double s0 = m.xc[Q] - x0, s1 = m.xc[N + Q] - x1, s2 = m.xc[2 * N + Q] - x2;
      const double len = sqrt(s0 * s0 + s1 * s1 + s2 * s2);
      const double c = fabs((n0 * s0 + n1 * s1 + n2 * s2) / len);
      const double c2 = c * c, c4 = c2 * c2;
      const double w = colour_weight(ah[Q]) * (c4 * c4);
      num += kstar[Q] * w;
      den += w;
    }
    num = gsum<kCsfLanes>(num);
    den = gsum<kCsfLanes>(den);
    if (lane == 0) {
      const double wP = colour_weight(ah[P]);
      const double k = (kstar[P] * wP + num) / (wP + den + kCsfEps);
      kappa[P] = k;
      if (F) {
        const double s = sigma * k;
        F[P] *= s;
        F[N + P] *= s;
        F[2 * N + P] *= s;
      }
    }
  }
}

}  // namespace vofpc

using namespace vofpc;

extern "C" vofpc_status vofpc_csf_opts_default(vofpc_csf_opts *o) {
  clear_error();
  VOFPC_REQUIRE(o, VOFPC_E_INVALID_ARG, "csf_opts_default: null argument");
  o->n_smooth = 2;
  o->sigma = 1.0;
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_curvature(vofpc_ctx ctx, vofpc_mesh M, const double *alpha, const vofpc_csf_opts *opts,
                                        double *alpha_hat, double *n, double *kappa_raw, double *kappa,
                                        double *force) {
  clear_error();
  VOFPC_REQUIRE(ctx && M && alpha && alpha_hat && n && kappa, VOFPC_E_INVALID_ARG, "curvature: null argument");
  VOFPC_REQUIRE(M->ctx && M->ctx->device == ctx->device, VOFPC_E_STATE, "curvature: mesh on another device");
  vofpc_csf_opts o;
  if (opts) o = *opts; else vofpc_csf_opts_default(&o);
  VOFPC_REQUIRE(o.n_smooth >= 0 && o.n_smooth <= 100, VOFPC_E_INVALID_ARG, "curvature: n_smooth out of range");
  VOFPC_HIP(hipSetDevice(ctx->device));
  const int64_t N = M->d.n_cells, NF = M->d.n_faces;
  hipStream_t s = ctx->stream;
  if (!M->csf_buf) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    VOFPC_HIP(hipStreamIsCapturing(s, &cs));
    VOFPC_REQUIRE(cs == hipStreamCaptureStatusNone, VOFPC_E_STATE,
                  "curvature: the first call on a mesh sets up its buffers and must not be captured");
    void *a = nullptr, *b = nullptr, *c = nullptr, *d = nullptr;
    vofpc_status st;
    if ((st = mesh_scratch_alloc(M, 24 * (size_t)N, &a)) || (st = mesh_scratch_alloc(M, (size_t)N, &b)) ||
        (st = mesh_scratch_alloc(M, 4 * (size_t)N, &c)) || (st = mesh_scratch_alloc(M, 16, &d)))
      return st;
    M->csf_buf = (double *)a;
    M->csf_mark = (int8_t *)b;
    M->csf_list = (int32_t *)c;
    M->csf_len = (int32_t *)d;
  }
  if (!M->csf_slot) {
    // per-slot weights and areas: fixed by the geometry, built once
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    VOFPC_HIP(hipStreamIsCapturing(s, &cs));
    VOFPC_REQUIRE(cs == hipStreamCaptureStatusNone, VOFPC_E_STATE,
                  "curvature: the first call on a mesh sets up its buffers and must not be captured");
    void *a = nullptr;
    vofpc_status st = mesh_scratch_alloc(M, 16 * (size_t)std::max<int64_t>(M->ncf, 1), &a);
    if (st) return st;
    M->csf_slot = (double *)a;
    csf_slot_kernel<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>((N + kCsfCells - 1) / kCsfCells,
                                                                       (int64_t)ctx->n_cu * 16)),
                      kCsfBlock, 0, s>>>(M->d, M->csf_slot);
    VOFPC_HIP(hipGetLastError());
  }
  double *tmp = M->csf_buf;                                  // smoothing ping-pong
  double *kr = kappa_raw ? kappa_raw : M->csf_buf + N;       // raw curvature
  double *ks = M->csf_buf + 2 * N;                           // step-1 curvature
  int8_t *mark = M->csf_mark;
  int32_t *list = M->csf_list;
  int32_t *len = M->csf_len + 1;   // [1]: domain length (the gradient reads a band count there)
  const unsigned gN = (unsigned)std::max<int64_t>(1, (N + kCsfBlock - 1) / kCsfBlock);
  const unsigned gF = (unsigned)std::max<int64_t>(1, (NF + kCsfBlock - 1) / kCsfBlock);
  const unsigned gC = (unsigned)std::max<int64_t>(1, std::min<int64_t>((N + kCsfCells - 1) / kCsfCells,
                                                                         (int64_t)ctx->n_cu * 16));
  const unsigned gE = (unsigned)std::max<int64_t>(1, std::min<int64_t>((N + kCsfBlock - 1) / kCsfBlock,
                                                                         (int64_t)ctx->n_cu * 8));
  // the domain: seed, then n_smooth + 3 rings
  csf_fill_kernel<<<gE, kCsfBlock, 0, s>>>(N, alpha, alpha_hat, tmp, n, kr, ks, kappa, force, mark, len);
  csf_seed_faces_kernel<<<gF, kCsfBlock, 0, s>>>(M->d, alpha, mark);
  for (int l = 1; l <= o.n_smooth + 3; ++l) ring_grow_kernel<<<gF, kRingBlock, 0, s>>>(M->d, mark, l);
  ring_list_kernel<<<gN, kRingBlock, 0, s>>>(N, mark, list, len);
  // smoothing: sweep k writes alpha_hat when n_smooth - 1 - k is even, so the
  // last sweep lands there
  const double *src = alpha;
  for (int k = 0; k < o.n_smooth; ++k) {
    double *dst = ((o.n_smooth - 1 - k) % 2 == 0) ? alpha_hat : tmp;
    csf_smooth_kernel<<<gC, kCsfBlock, 0, s>>>(M->d, M->csf_slot, list, len, src, dst);
    src = dst;
  }
  VOFPC_HIP(hipGetLastError());
  // normal from the plain gradient of alpha_hat (interior neighbours only)
  vofpc_status st = launch_grad(ctx, M, alpha_hat, nullptr, 0.0, alpha_hat, list, M->csf_len, VOFPC_SCOPE_BAND,
                                VOFPC_GRAD_STANDARD, n, nullptr);
  if (st) return st;
  csf_normalise_kernel<<<gE, kCsfBlock, 0, s>>>(N, list, len, n);
  csf_divergence_kernel<<<gC, kCsfBlock, 0, s>>>(M->d, M->csf_slot, list, len, n, kr);
  csf_step1_kernel<<<gC, kCsfBlock, 0, s>>>(M->d, list, len, alpha_hat, kr, ks);
  if (force) {
    st = launch_grad(ctx, M, alpha, nullptr, 0.0, alpha, list, M->csf_len, VOFPC_SCOPE_BAND, VOFPC_GRAD_STANDARD,
                     force, nullptr);
    if (st) return st;
  }
  csf_step2_kernel<<<gC, kCsfBlock, 0, s>>>(M->d, list, len, alpha_hat, n, ks, kappa, o.sigma, force);
  VOFPC_HIP(hipGetLastError());
  return VOFPC_OK;
}
