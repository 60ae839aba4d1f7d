// Phase gradients at the interface by pseudo-time extrapolation
// (Eq. extrapolation, Sec. 2.4.4), each gradient component separately:
//   the domain D is the mixed cells and `layers` rings of interior face
//   neighbours around them; on D, G_l = G_v = the interface-modified gradient;
//   a liquid cell (alpha >= 1/2) keeps G_l and advances G_v, a vapour cell
//   keeps G_v and advances G_l, with velocity c = sgn(alpha - 1/2) n (n: the
//   interface normal where the cell has an interface, else the unit plain
//   least-squares gradient of alpha over interior neighbours);
//   first-order upwind, Jacobi: with w_f = -c.S_f over the faces whose
//   neighbour is in D and c.S_f < 0, F_P <- F_P + theta (sum w_f F_Q / w - F_P),
//   theta = min(dtau w / V_P, 1), dtau = the smallest centre distance of two
//   face neighbours; stop at the first sweep whose largest change is below
//   tol, or after max_iter sweeps.
//
// One kernel per sweep: the kernel boundary is the synchronisation.  A grid
// barrier inside one persistent kernel was measured slower on this chip: with
// one block per XCD it lacks memory parallelism, and with many blocks every
// sweep pays device-scope fences that write back and invalidate the per-XCD
// L2 caches.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ring_ops.h"
#include "vofpc_internal.h"
#include "wave_ops.h"

namespace vofpc {

constexpr int kExBlock = 256;
constexpr int kExMaxGrid = 1024;   // blocks of the stencil and sweep kernels at most

__device__ __forceinline__ bool is_mixed(double a, double eps) { return a > eps && a < 1.0 - eps; }

// layer 0: the mixed cells; everything else outside; the list length is reset
__global__ __launch_bounds__(kExBlock) void ex_init_kernel(int64_t n, const double *alpha, double eps, int8_t *mark,
                                                           int32_t *info) {
  const int64_t P = blockIdx.x * (int64_t)kExBlock + threadIdx.x;
  if (P < n) mark[P] = is_mixed(alpha[P], eps) ? 0 : -1;
  if (P == 0) {
    info[1] = 0;
    info[2] = 0;
    info[3] = 0;
    info[4] = 0;
  }
}

// advection direction: unit plain gradient of alpha (computed into nrm by
// the gradient kernel) ...
__global__ __launch_bounds__(kExBlock) void ex_normalise_kernel(int64_t N, const int32_t *list, const int32_t *info,
                                                                double *nrm) {
  const int64_t j = blockIdx.x * (int64_t)kExBlock + threadIdx.x;
  if (j >= info[1]) return;
  const int P = list[j];
  const double g0 = nrm[P], g1 = nrm[N + P], g2 = nrm[2 * N + P];
  const double len = sqrt(g0 * g0 + g1 * g1 + g2 * g2);
  nrm[P] = len > 0 ? g0 / len : 0.0;
  nrm[N + P] = len > 0 ? g1 / len : 0.0;
  nrm[2 * N + P] = len > 0 ? g2 / len : 0.0;
}

// ... replaced by the interface normal where the cell has an interface
__global__ __launch_bounds__(kExBlock) void ex_interface_normal_kernel(int64_t N, const int32_t *mixed,
                                                                       const int32_t *counts, vofpc_interface itf,
                                                                       double *nrm) {
  int64_t n = counts[0];
  if (n > itf.cap) n = itf.cap;
  const int64_t k = blockIdx.x * (int64_t)kExBlock + threadIdx.x;
  if (k >= n) return;
  if (!(itf.A[k] > 0)) return;
  const int P = mixed[k];
  nrm[P] = itf.n[k];
  nrm[N + P] = itf.n[itf.cap + k];
  nrm[2 * N + P] = itf.n[2 * itf.cap + k];
}

struct ExParams {
  DevMesh m;
  const double *alpha;
  const int32_t *list;
  double *wup;      // per cell-face slot: upwind weights w_f / sum w, packed at the front of each cell's slots
  int32_t *upn;     // per cell-face slot: the neighbour of each packed upwind weight
  int2 *upr;        // per domain entry: first slot and number of its packed upwind weights
  double *theta;    // per domain entry: pseudo-time fraction min(dtau sum w / V, 1), 0 without upwind faces
  int32_t *info;
  double *part;     // [2][grid] per-block largest change of the last two sweeps
  const int8_t *mark;
  const double *nrm;
  double *buf;   // [2][N][kExRec]
  double dtau, tol;
  int max_iter;
  double *gl, *gv;
};

constexpr int kExLanes = 8;   // lanes per domain cell in the stencil and sweeps (half a DPP row)
constexpr int kExBlocksPerCu = 4;   // stencil and sweep blocks per CU
// The two iterates of both fields: one 64-byte record per cell and iterate,
// G_l in words 0-2 and G_v in words 3-5, so a neighbour's gathered
// components share one cache line.
constexpr int kExRec = 8;

// Upwind weight of cell-face slot i of cell P for velocity c: w_f = -c.S_f
// (S_f outward from P) when that is positive and the neighbour Q is in the
// domain, else 0.
__device__ __forceinline__ double ex_up_weight(const ExParams &p, int P, double c0, double c1, double c2, int64_t i,
                                               int &Q) {
  const DevMesh &m = p.m;
  const int64_t NF = m.n_faces;
  Q = m.cf_nbr[i];
  if (Q < 0 || p.mark[Q] < 0) return 0.0;
  const int f = m.cell_face[i];
  const double sg = (m.face_owner[f] == P) ? 1.0 : -1.0;
  const double cs = c0 * (sg * m.Sf[f]) + c1 * (sg * m.Sf[NF + f]) + c2 * (sg * m.Sf[2 * NF + f]);
  return cs < 0.0 ? -cs : 0.0;
}

// The upwind stencil of domain entry j, fixed for the whole iteration (and
// the start of both fields, the gradient p.gl, written to both iterates): with
// c = sgn(alpha - 1/2) n, the faces with c.S_f < 0 (S_f outward) whose
// neighbour is in the domain get w_f = -c.S_f; those faces, in slot order,
// are packed at the front of the cell's slot range as (w_f / sum w,
// neighbour), the entry keeps (first slot, count) and
// theta = min(dtau sum w / V_P, 1) (0 when no face is upwind: no update).
__device__ __forceinline__ void ex_stencil(const ExParams &p, int64_t j, int lane) {
  const DevMesh &m = p.m;
  const int64_t N = m.n_cells;
  const int P = p.list[j];
  if (lane < 3) {
    // both fields start from the gradient (each iterate)
    const double g = p.gl[lane * N + P];
    double *rec0 = p.buf + (int64_t)P * kExRec, *rec1 = p.buf + ((int64_t)N + P) * kExRec;
    rec0[lane] = g;
    rec0[3 + lane] = g;
    rec1[lane] = g;
    rec1[3 + lane] = g;
  }
  const double sgn = p.alpha[P] >= 0.5 ? 1.0 : -1.0;
  const double c0 = sgn * p.nrm[P], c1 = sgn * p.nrm[N + P], c2 = sgn * p.nrm[2 * N + P];
  const int64_t i0 = m.cell_face_off[P], i1 = m.cell_face_off[P + 1];
  double w = 0.0;
  for (int64_t i = i0 + lane; i < i1; i += kExLanes) {
    int Q;
    w += ex_up_weight(p, P, c0, c1, c2, i, Q);
  }
  w = gsum<kExLanes>(w);
  // the lanes of a group share the cell, so they run the same rounds; each
  // round packs its upwind slots after those of the rounds before
  const int gl0 = (threadIdx.x & 63) & ~(kExLanes - 1);
  const uint64_t below = (1ull << lane) - 1;
  int n = 0;
  for (int64_t k0 = i0; k0 < i1; k0 += kExLanes) {
    const int64_t i = k0 + lane;
    int Q = -1;
    const double wf = (i < i1 && w > 0.0) ? ex_up_weight(p, P, c0, c1, c2, i, Q) : 0.0;
    const bool up = wf > 0.0;
    const uint64_t gm = (__ballot(up) >> gl0) & ((1ull << kExLanes) - 1);
    if (up) {
      const int64_t o = i0 + n + __popcll(gm & below);
      p.wup[o] = wf / w;
      p.upn[o] = Q;
    }
    n += __popcll(gm);
  }
  if (lane == 0) {
    double th = 0.0;
    if (w > 0.0) {
      th = p.dtau * w / m.V[P];
      if (th > 1.0) th = 1.0;
    }
    p.theta[j] = th;
    p.upr[j] = make_int2((int)i0, n);
  }
}

__global__ __launch_bounds__(kExBlock) void ex_stencil_kernel(ExParams p) {
  constexpr int kCells = kExBlock / kExLanes;
  const int64_t nd = p.info[1];
  const int lane = threadIdx.x % kExLanes;
  for (int64_t j = blockIdx.x * (int64_t)kCells + threadIdx.x / kExLanes; j < nd; j += (int64_t)gridDim.x * kCells)
    ex_stencil(p, j, lane);
}

// Upwind update of domain entry j from iterate cur by a group of kExLanes
// lanes, one packed upwind slot per lane and round: the new values of its three advanced
// components and their largest change (ex_compute), written into the next
// iterate by ex_store.  The kept field was written to both iterates at the
// start and is not touched.
struct ExNew {
  int P, adv;
  double n0, n1, n2, change;
};

__device__ __forceinline__ ExNew ex_compute(const ExParams &p, int64_t j, int lane, const double *cur) {
  const DevMesh &m = p.m;
  const int64_t N = m.n_cells;
  ExNew r;
  r.P = p.list[j];
  r.adv = p.alpha[r.P] >= 0.5 ? 3 : 0;   // G_v advances in liquid, G_l in vapour
  const double *ca = cur + r.adv;
  const int2 ur = p.upr[j];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int k = lane; k < ur.y; k += kExLanes) {
    const double wf = p.wup[ur.x + k];
    const double *q = ca + (int64_t)p.upn[ur.x + k] * kExRec;
    a0 += wf * q[0];
    a1 += wf * q[1];
    a2 += wf * q[2];
  }
  a0 = gsum<kExLanes>(a0);
  a1 = gsum<kExLanes>(a1);
  a2 = gsum<kExLanes>(a2);
  const double th = p.theta[j];
  const int P = r.P;
  const double *o = ca + (int64_t)P * kExRec;
  const double o0 = o[0], o1 = o[1], o2 = o[2];
  r.n0 = o0 + th * (a0 - o0);
  r.n1 = o1 + th * (a1 - o1);
  r.n2 = o2 + th * (a2 - o2);
  r.change = fmax(fabs(r.n0 - o0), fmax(fabs(r.n1 - o1), fabs(r.n2 - o2)));
  return r;
}

__device__ __forceinline__ void ex_store(const ExParams &p, const ExNew &r, double *nxt) {
  const int64_t N = p.m.n_cells;
  double *na = nxt + (int64_t)r.P * kExRec + r.adv;
  na[0] = r.n0;
  na[1] = r.n1;
  na[2] = r.n2;
}

// Sweep `it` (0-based) of the Jacobi iteration.  From the second sweep on it
// first reads the largest change of the previous sweep (complete: it ran in
// the previous kernel): below tol, the iteration has converged after `it`
// sweeps and this and every later sweep kernel return at once.
__global__ __launch_bounds__(kExBlock) void ex_sweep_kernel(ExParams p, int it) {
  __shared__ double red[kExBlock / 64];
  const int converged = p.info[4];
  const int64_t nd = p.info[1];
  if (converged) return;
  const int64_t N = p.m.n_cells;
  const double *cur = p.buf + (int64_t)(it & 1) * kExRec * N;
  double *nxt = p.buf + (int64_t)((it + 1) & 1) * kExRec * N;
  // groups of kExLanes lanes take the domain cells; every lane of a group
  // sees the same cells, so the group reductions see all its lanes.  The
  // group's first cell is computed before the convergence test of the
  // previous sweep (its gathers and that test's reads are in flight
  // together) and stored after.
  constexpr int kCells = kExBlock / kExLanes;
  const int lane = threadIdx.x % kExLanes;
  const int64_t j0 = blockIdx.x * (int64_t)kCells + threadIdx.x / kExLanes;
  const int64_t stride = (int64_t)gridDim.x * kCells;
  ExNew first{0, 0, 0.0, 0.0, 0.0, 0.0};
  if (j0 < nd) first = ex_compute(p, j0, lane, cur);
  if (it > 0) {
    // largest change of the previous sweep: the maximum of its blocks'
    // partial maxima (every block of that kernel wrote its slot)
    const double *part = p.part + (int64_t)((it - 1) & 1) * gridDim.x;
    double prev = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kExBlock) prev = fmax(prev, part[b]);
    for (int o = 32; o > 0; o >>= 1) prev = fmax(prev, __shfl_xor(prev, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = prev;
    __syncthreads();
    prev = red[0];
    for (int i = 1; i < kExBlock / 64; ++i) prev = fmax(prev, red[i]);
    __syncthreads();
    if (prev < p.tol) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.info[4] = 1;
        p.info[2] = it;
      }
      return;
    }
  }
  double change = 0.0;
  if (j0 < nd && lane == 0) {
    ex_store(p, first, nxt);
    change = first.change;
  }
  for (int64_t j = j0 + stride; j < nd; j += stride) {
    const ExNew r = ex_compute(p, j, lane, cur);
    if (lane == 0) {
      ex_store(p, r, nxt);
      change = fmax(change, r.change);
    }
  }
  // this block's largest change into its slot of this sweep's partials
  // (plain stores: the next sweep kernel reads them after the kernel boundary)
  for (int o = 32; o > 0; o >>= 1) change = fmax(change, __shfl_xor(change, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = change;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = red[0];
    for (int i = 1; i < kExBlock / 64; ++i) b = fmax(b, red[i]);
    p.part[(int64_t)(it & 1) * gridDim.x + blockIdx.x] = b;
  }
}

// After the last sweep kernel: the number of sweeps done, and the outputs on
// the domain from the buffer of the newest iterate.
__global__ __launch_bounds__(kExBlock) void ex_finish_kernel(ExParams p) {
  const int64_t N = p.m.n_cells;
  const int64_t nd = p.info[1];
  // converged: the count the first idle sweep kernel recorded; otherwise
  // every sweep ran (the last one counts whether or not it met the tolerance)
  const int sweeps = p.info[4] ? p.info[2] : p.max_iter;
  const double *fin = p.buf + (int64_t)(sweeps & 1) * kExRec * N;
  for (int64_t j = blockIdx.x * (int64_t)kExBlock + threadIdx.x; j < nd; j += (int64_t)gridDim.x * kExBlock) {
    const int P = p.list[j];
    const double *rec = fin + (int64_t)P * kExRec;
    for (int d = 0; d < 3; ++d) {
      p.gl[d * N + P] = rec[d];
      p.gv[d * N + P] = rec[3 + d];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) p.info[2] = sweeps;
}

__global__ void ex_report_kernel(const int32_t *info, int32_t *out) {
  if (threadIdx.x == 0) {
    out[0] = info[2];
    out[1] = info[3];
  }
}

}  // namespace vofpc

using namespace vofpc;

extern "C" vofpc_status vofpc_extrap_opts_default(vofpc_extrap_opts *o) {
  clear_error();
  VOFPC_REQUIRE(o, VOFPC_E_INVALID_ARG, "extrap_opts_default: null argument");
  o->eps_mixed = 1e-8;
  o->layers = 2;
  o->max_iter = 120;
  o->tol = 1e-3;
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_extrapolate(vofpc_ctx ctx, vofpc_mesh M, const double *alpha, const double *T,
                                          const double *T_bface, double T_sat, const int32_t *mixed_idx,
                                          const int32_t *counts, const vofpc_interface *itf,
                                          const vofpc_extrap_opts *opts, double *gradT_l, double *gradT_v,
                                          int32_t *report) {
  clear_error();
  VOFPC_REQUIRE(ctx && M && alpha && T && T_bface && mixed_idx && counts && itf && gradT_l && gradT_v,
                VOFPC_E_INVALID_ARG, "extrapolate: null argument");
  VOFPC_REQUIRE(M->ctx && M->ctx->device == ctx->device, VOFPC_E_STATE, "extrapolate: mesh on another device");
  VOFPC_REQUIRE(itf->n && itf->A && itf->cap > 0, VOFPC_E_INVALID_ARG, "extrapolate: interface record incomplete");
  vofpc_extrap_opts o;
  if (opts) o = *opts; else vofpc_extrap_opts_default(&o);
  VOFPC_REQUIRE(o.layers >= 0 && o.layers <= 100 && o.max_iter >= 0 && o.max_iter <= 100000 && o.tol >= 0 &&
                    o.eps_mixed >= 0 && o.eps_mixed < 0.5,
                VOFPC_E_INVALID_ARG, "extrapolate: options out of range");
  VOFPC_REQUIRE(M->ncf <= INT32_MAX, VOFPC_E_INVALID_ARG, "extrapolate: more than 2^31 - 1 cell-face slots");
  VOFPC_HIP(hipSetDevice(ctx->device));
  const int64_t N = M->d.n_cells, NF = M->d.n_faces;
  hipStream_t s = ctx->stream;
  if (!M->ex_buf) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    VOFPC_HIP(hipStreamIsCapturing(s, &cs));
    VOFPC_REQUIRE(cs == hipStreamCaptureStatusNone, VOFPC_E_STATE,
                  "extrapolate: the first call on a mesh sets up its buffers and must not be captured");
    void *a = nullptr, *b = nullptr, *c = nullptr, *d = nullptr, *e = nullptr, *f = nullptr, *g = nullptr,
         *h = nullptr, *i = nullptr, *j = nullptr;
    vofpc_status st;
    if ((st = mesh_scratch_alloc(M, (size_t)N, &a)) || (st = mesh_scratch_alloc(M, 4 * (size_t)N, &b)) ||
        (st = mesh_scratch_alloc(M, 32, &c)) || (st = mesh_scratch_alloc(M, 16 * kExMaxGrid, &d)) ||
        (st = mesh_scratch_alloc(M, 24 * (size_t)N, &e)) || (st = mesh_scratch_alloc(M, 16 * sizeof(double) * (size_t)N, &f)) ||
        (st = mesh_scratch_alloc(M, 8 * (size_t)M->ncf, &g)) || (st = mesh_scratch_alloc(M, 8 * (size_t)N, &h)) ||
        (st = mesh_scratch_alloc(M, 4 * (size_t)M->ncf, &i)) || (st = mesh_scratch_alloc(M, 8 * (size_t)N, &j)))
      return st;
    M->ex_mark = (int8_t *)a; M->ex_list = (int32_t *)b; M->ex_info = (int32_t *)c; M->ex_part = (double *)d;
    M->ex_nrm = (double *)e; M->ex_buf = (double *)f; M->ex_wup = (double *)g; M->ex_theta = (double *)h;
    M->ex_upn = (int32_t *)i; M->ex_upr = (int2 *)j;
  }
  const unsigned gN = (unsigned)((N + kExBlock - 1) / kExBlock), gF = (unsigned)((NF + kExBlock - 1) / kExBlock);
  ex_init_kernel<<<gN, kExBlock, 0, s>>>(N, alpha, o.eps_mixed, M->ex_mark, M->ex_info);
  for (int l = 1; l <= o.layers; ++l) ring_grow_kernel<<<gF, kRingBlock, 0, s>>>(M->d, M->ex_mark, l);
  ring_list_kernel<<<gN, kRingBlock, 0, s>>>(N, M->ex_mark, M->ex_list, M->ex_info + 1);
  VOFPC_HIP(hipGetLastError());
  // gradient of T (interface-modified) and of alpha (plain, interior
  // neighbours only) on the domain; the domain length sits in ex_info[1],
  // where the gradient kernel reads its band count
  const int32_t *dom_counts = M->ex_info;
  vofpc_status st = launch_grad2(ctx, M, M->ex_list, dom_counts, T, T_bface, T_sat, alpha, VOFPC_GRAD_MODIFIED,
                                 gradT_l, alpha, nullptr, 0.0, alpha, VOFPC_GRAD_STANDARD, M->ex_nrm);
  if (st) return st;
  ex_normalise_kernel<<<gN, kExBlock, 0, s>>>(N, M->ex_list, M->ex_info, M->ex_nrm);
  const unsigned gM = (unsigned)((std::min<int64_t>(itf->cap, N) + kExBlock - 1) / kExBlock);
  ex_interface_normal_kernel<<<gM, kExBlock, 0, s>>>(N, mixed_idx, counts, *itf, M->ex_nrm);
  ExParams p;
  p.m = M->d;
  p.alpha = alpha;
  p.list = M->ex_list;
  p.info = M->ex_info;
  p.part = M->ex_part;
  p.mark = M->ex_mark;
  p.nrm = M->ex_nrm;
  p.buf = M->ex_buf;
  p.wup = M->ex_wup;
  p.upn = M->ex_upn;
  p.upr = M->ex_upr;
  p.theta = M->ex_theta;
  p.dtau = M->min_centre_dist;
  p.tol = o.tol;
  p.max_iter = o.max_iter;
  p.gl = gradT_l;
  p.gv = gradT_v;
  // sweeps: 16 domain cells per block, four blocks per CU (a domain of
  // 16k cells in one pass: each pass is a chain of dependent gathers); the
  // finish kernel one cell per thread
  const unsigned gS = (unsigned)std::max<int64_t>(1, std::min<int64_t>(gN, (int64_t)ctx->n_cu * 2));
  const unsigned gW = (unsigned)std::max<int64_t>(
      1, std::min<int64_t>((N + kExBlock / kExLanes - 1) / (kExBlock / kExLanes),
                           std::min<int64_t>((int64_t)ctx->n_cu * kExBlocksPerCu, kExMaxGrid)));
  // the upwind stencil once; then one kernel per sweep: the kernel boundary
  // orders the sweeps, and once the tolerance is met the remaining sweep
  // kernels return at once
  ex_stencil_kernel<<<gW, kExBlock, 0, s>>>(p);
  for (int it = 0; it < o.max_iter; ++it) ex_sweep_kernel<<<gW, kExBlock, 0, s>>>(p, it);
  ex_finish_kernel<<<gS, kExBlock, 0, s>>>(p);
  if (report) ex_report_kernel<<<1, 64, 0, s>>>(M->ex_info, report);
  VOFPC_HIP(hipGetLastError());
  return VOFPC_OK;
}
