// Interface-modified least-squares temperature gradient (App. B with the
// modification of Sec. 2.4.4) and the mass transfer rate (Eq. mass_transfer,
// Eq. latent_source).
//
// Eight lanes per cell, faces dealt round the lanes.  The gradient gathers, for every
// face of the cell, the neighbour centroid, alpha and T (or the boundary face
// centroid and value), so the least-squares matrix is accumulated from data
// the right-hand side needs anyway; cells without a crossing face may instead
// use the stored inverse (VOFPC_SCOPE_ALL).
#include <hip/hip_runtime.h>

#include "vofpc_internal.h"
#include "wave_ops.h"

namespace vofpc {

struct GradParams {
  DevMesh m;
  const double *T, *Tb, *alpha;
  double T_sat;
  const int32_t *band, *counts;
  int scope, variant;   // base variant (VOFPC_GRAD_MODIFIED/STANDARD/PRINTED)
  int weight;           // 0 uniform, 1 inverse distance, 2 inverse distance squared
  const int64_t *xn_off;   // vertex-neighbour stencil (null: face neighbours)
  const int32_t *xn_cell;
  double *grad;
  int32_t *status;
};

// least-squares sums of one cell: G (6 components) and b
struct LsqSums {
  double xx = 0, yy = 0, zz = 0, xy = 0, xz = 0, yz = 0, b0 = 0, b1 = 0, b2 = 0;
  __device__ __forceinline__ void add(double r0, double r1, double r2, double dv, int weight) {
    double w = 1.0;
    if (weight == 1) w = 1.0 / sqrt(r0 * r0 + r1 * r1 + r2 * r2);
    else if (weight == 2) w = 1.0 / (r0 * r0 + r1 * r1 + r2 * r2);
    const double w0 = w * r0, w1 = w * r1, w2 = w * r2;
    xx += w0 * r0; yy += w1 * r1; zz += w2 * r2; xy += w0 * r1; xz += w0 * r2; yz += w1 * r2;
    b0 += w0 * dv; b1 += w1 * dv; b2 += w2 * dv;
  }
};

constexpr int kGradLanes = 8;   // lanes per cell (half a DPP row)

// Gradient of cell P by a group of kGradLanes lanes: lane j takes faces j,
// j + kGradLanes, ...; the least-squares sums are reduced over the group.
__device__ __forceinline__ void grad_cell(const GradParams &p, int P, int j) {
  const DevMesh &m = p.m;
  const int64_t N = m.n_cells, NF = m.n_faces;
  const double xP0 = m.xc[P], xP1 = m.xc[N + P], xP2 = m.xc[2 * N + P];
  const double aP = p.alpha[P], TP = p.T[P];
  const bool modify = p.variant != VOFPC_GRAD_STANDARD;
  const bool printed = p.variant == VOFPC_GRAD_PRINTED;
  LsqSums L;
  int crossed = 0;
  // an interior neighbour q: the centre connection, shortened to the
  // alpha-interpolated crossing held at T_sat where the interface cuts it
  auto interior = [&](int q) {
    double r0 = m.xc[q] - xP0, r1 = m.xc[N + q] - xP1, r2 = m.xc[2 * N + q] - xP2;
    const double aQ = p.alpha[q];
    double val = p.T[q];
    if (modify && (aP - 0.5) * (aQ - 0.5) < 0.0) {
      const double t = printed ? fabs(aQ - 0.5) / fabs(aP - aQ) : (aP - 0.5) / (aP - aQ);
      r0 *= t; r1 *= t; r2 *= t;
      val = p.T_sat;
      crossed = 1;
    }
    L.add(r0, r1, r2, val - TP, p.weight);
  };
  const int64_t i0 = m.cell_face_off[P], i1 = m.cell_face_off[P + 1];
  if (p.xn_off) {
    for (int64_t i = p.xn_off[P] + j; i < p.xn_off[P + 1]; i += kGradLanes) interior(p.xn_cell[i]);
  }
  for (int64_t i = i0 + j; i < i1; i += kGradLanes) {
    const int q = m.cf_nbr[i];
    if (q >= 0) {
      if (!p.xn_off) interior(q);
    } else if (q == -1 && p.Tb) {   // no boundary values given: interior neighbours only
      const int f = m.cell_face[i];
      L.add(m.xf[f] - xP0, m.xf[NF + f] - xP1, m.xf[2 * NF + f] - xP2, p.Tb[f] - TP, p.weight);
    }
  }
  double xx = L.xx, yy = L.yy, zz = L.zz, xy = L.xy, xz = L.xz, yz = L.yz, b0 = L.b0, b1 = L.b1, b2 = L.b2;
  xx = gsum<kGradLanes>(xx); yy = gsum<kGradLanes>(yy); zz = gsum<kGradLanes>(zz);
  xy = gsum<kGradLanes>(xy); xz = gsum<kGradLanes>(xz); yz = gsum<kGradLanes>(yz);
  b0 = gsum<kGradLanes>(b0); b1 = gsum<kGradLanes>(b1); b2 = gsum<kGradLanes>(b2);
  crossed = gsum_i<kGradLanes>(crossed);
  if (j != 0) return;
  double g0, g1, g2;
  int st = VOFPC_CELL_OK;
  // the stored inverse holds the face stencil with boundary values: usable
  // for the plain variant when boundary values are given
  if (p.scope == VOFPC_SCOPE_ALL && !crossed && p.weight == 0 && !p.xn_off && p.Tb) {
    const double *gi = m.ginv;
    const double ixx = gi[P], iyy = gi[N + P], izz = gi[2 * N + P];
    const double ixy = gi[3 * N + P], ixz = gi[4 * N + P], iyz = gi[5 * N + P];
    g0 = ixx * b0 + ixy * b1 + ixz * b2;
    g1 = ixy * b0 + iyy * b1 + iyz * b2;
    g2 = ixz * b0 + iyz * b1 + izz * b2;
    if (ixx == 0 && iyy == 0 && izz == 0) st = VOFPC_CELL_G_SINGULAR;
  } else {
    const double c00 = yy * zz - yz * yz, c01 = xz * yz - xy * zz, c02 = xy * yz - xz * yy;
    const double c11 = xx * zz - xz * xz, c12 = xy * xz - xx * yz, c22 = xx * yy - xy * xy;
    const double det = xx * c00 + xy * c01 + xz * c02;
    const double tr = (xx + yy + zz) * (1.0 / 3.0);
    if (det > 1e-12 * tr * tr * tr) {
      const double id = 1.0 / det;
      g0 = (c00 * b0 + c01 * b1 + c02 * b2) * id;
      g1 = (c01 * b0 + c11 * b1 + c12 * b2) * id;
      g2 = (c02 * b0 + c12 * b1 + c22 * b2) * id;
    } else {
      g0 = g1 = g2 = 0.0;
      st = VOFPC_CELL_G_SINGULAR;
    }
  }
  p.grad[P] = g0;
  p.grad[N + P] = g1;
  p.grad[2 * N + P] = g2;
  if (p.status) p.status[P] = st;
}

// A block of 256 lanes serves 256 / kGradLanes cells at a time; every lane
// of a group iterates the same cells, so the group's reductions see all its
// lanes.
__global__ __launch_bounds__(256) void grad_kernel(GradParams p) {
  const int64_t n = (p.scope == VOFPC_SCOPE_ALL) ? p.m.n_cells : (int64_t)p.counts[1];
  constexpr int kCellsPerBlock = 256 / kGradLanes;
  const int j = threadIdx.x % kGradLanes;
  const int64_t stride = (int64_t)gridDim.x * kCellsPerBlock;
  for (int64_t k = blockIdx.x * (int64_t)kCellsPerBlock + threadIdx.x / kGradLanes; k < n; k += stride) {
    const int P = (p.scope == VOFPC_SCOPE_ALL) ? (int)k : p.band[k];
    grad_cell(p, P, j);
  }
}

// Two gradients over the same band list in one launch (the group computes
// both for its cell; used where a caller needs two fields' gradients on one
// domain).
__global__ __launch_bounds__(256) void grad2_kernel(GradParams a, GradParams b) {
  const int64_t n = a.counts[1];
  constexpr int kCellsPerBlock = 256 / kGradLanes;
  const int j = threadIdx.x % kGradLanes;
  const int64_t stride = (int64_t)gridDim.x * kCellsPerBlock;
  for (int64_t k = blockIdx.x * (int64_t)kCellsPerBlock + threadIdx.x / kGradLanes; k < n; k += stride) {
    const int P = a.band[k];
    grad_cell(a, P, j);
    grad_cell(b, P, j);
  }
}

static vofpc_status grad_params(vofpc_mesh M, const double *T, const double *Tb, double T_sat, const double *alpha,
                                const int32_t *band, const int32_t *counts, int32_t scope, int32_t variant,
                                double *grad, int32_t *status, GradParams &p) {
  VOFPC_REQUIRE(T && alpha && grad, VOFPC_E_INVALID_ARG, "grad_T: null argument");
  VOFPC_REQUIRE(scope == VOFPC_SCOPE_BAND || scope == VOFPC_SCOPE_ALL, VOFPC_E_INVALID_ARG, "grad_T: unknown scope");
  VOFPC_REQUIRE(scope == VOFPC_SCOPE_ALL || (band && counts), VOFPC_E_INVALID_ARG,
                "grad_T: band scope needs band_idx and counts");
  const int base = variant & 0xf, flags = variant & ~0xf;
  VOFPC_REQUIRE(base >= VOFPC_GRAD_MODIFIED && base <= VOFPC_GRAD_PRINTED &&
                    (flags & ~(VOFPC_GRAD_W_INV_DIST | VOFPC_GRAD_W_INV_DIST2 | VOFPC_GRAD_VERTEX_STENCIL)) == 0 &&
                    (flags & (VOFPC_GRAD_W_INV_DIST | VOFPC_GRAD_W_INV_DIST2)) !=
                        (VOFPC_GRAD_W_INV_DIST | VOFPC_GRAD_W_INV_DIST2),
                VOFPC_E_INVALID_ARG, "grad_T: unknown variant");
  VOFPC_REQUIRE(!(flags & VOFPC_GRAD_VERTEX_STENCIL) || M->xn_off, VOFPC_E_STATE,
                "grad_T: the vertex stencil of this mesh is not built");
  p.m = M->d;
  p.T = T; p.Tb = Tb; p.alpha = alpha; p.T_sat = T_sat;
  p.band = band; p.counts = counts;
  p.scope = scope; p.variant = base;
  p.weight = (flags & VOFPC_GRAD_W_INV_DIST) ? 1 : (flags & VOFPC_GRAD_W_INV_DIST2) ? 2 : 0;
  p.xn_off = (flags & VOFPC_GRAD_VERTEX_STENCIL) ? M->xn_off : nullptr;
  p.xn_cell = (flags & VOFPC_GRAD_VERTEX_STENCIL) ? M->xn_cell : nullptr;
  p.grad = grad; p.status = status;
  return VOFPC_OK;
}

static unsigned grad_grid(vofpc_ctx ctx, vofpc_mesh M) {
  int64_t grid = (M->d.n_cells + 15) / 16;
  const int64_t cap = (int64_t)ctx->n_cu * 16;
  if (grid > cap) grid = cap;
  return (unsigned)(grid > 0 ? grid : 1);
}

vofpc_status launch_grad(vofpc_ctx ctx, vofpc_mesh M, const double *T, const double *Tb, double T_sat,
                         const double *alpha, const int32_t *band, const int32_t *counts, int32_t scope,
                         int32_t variant, double *grad, int32_t *status) {
  GradParams p;
  vofpc_status st = grad_params(M, T, Tb, T_sat, alpha, band, counts, scope, variant, grad, status, p);
  if (st) return st;
  grad_kernel<<<grad_grid(ctx, M), 256, 0, ctx->stream>>>(p);
  VOFPC_HIP(hipGetLastError());
  return VOFPC_OK;
}

vofpc_status launch_grad2(vofpc_ctx ctx, vofpc_mesh M, const int32_t *band, const int32_t *counts, const double *T1,
                          const double *Tb1, double T_sat1, const double *alpha1, int32_t variant1, double *grad1,
                          const double *T2, const double *Tb2, double T_sat2, const double *alpha2, int32_t variant2,
                          double *grad2) {
  GradParams a, b;
  vofpc_status st = grad_params(M, T1, Tb1, T_sat1, alpha1, band, counts, VOFPC_SCOPE_BAND, variant1, grad1, nullptr, a);
  if (st) return st;
  st = grad_params(M, T2, Tb2, T_sat2, alpha2, band, counts, VOFPC_SCOPE_BAND, variant2, grad2, nullptr, b);
  if (st) return st;
  grad2_kernel<<<grad_grid(ctx, M), 256, 0, ctx->stream>>>(a, b);
  VOFPC_HIP(hipGetLastError());
  return VOFPC_OK;
}

// ------------------------------------------------------------ mass transfer
struct MdotParams {
  const double *V, *alpha;
  int64_t n_cells;
  const int32_t *mixed, *counts;
  vofpc_interface itf;
  const double *gradT, *gl, *gv;
  double k_l, k_v, h_lv;
  double *mdot, *Qdot, *mdot_c, *Qdot_c;
};

__global__ __launch_bounds__(256) void fill_zero_kernel(double *a, double *b, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    if (a) a[i] = 0.0;
    if (b) b[i] = 0.0;
  }
}

__global__ __launch_bounds__(256) void mdot_kernel(MdotParams p) {
  int64_t n = p.counts[0];
  if (n > p.itf.cap) n = p.itf.cap;
  const int64_t N = p.n_cells, cap = p.itf.cap;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += stride) {
    const int P = p.mixed[k];
    const double A = p.itf.A[k];
    double md = 0.0;
    if (A > 0.0) {
      const double n0 = p.itf.n[k], n1 = p.itf.n[cap + k], n2 = p.itf.n[2 * cap + k];
      double gl = 0.0, gv = 0.0;  // projections on n
      if (p.gl && p.gv) {
        gl = p.gl[P] * n0 + p.gl[N + P] * n1 + p.gl[2 * N + P] * n2;
        gv = p.gv[P] * n0 + p.gv[N + P] * n1 + p.gv[2 * N + P] * n2;
      } else {
        const double gn = p.gradT[P] * n0 + p.gradT[N + P] * n1 + p.gradT[2 * N + P] * n2;
        if (p.alpha[P] >= 0.5) gl = gn; else gv = gn;
      }
      const double ql = p.k_l * gl * A;
      const double qv = -p.k_v * gv * A;
      md = (ql + qv) / (p.h_lv * p.V[P]);
    }
    p.mdot[k] = md;
    p.Qdot[k] = -md * p.h_lv;
    if (p.mdot_c) p.mdot_c[P] = md;
    if (p.Qdot_c) p.Qdot_c[P] = -md * p.h_lv;
  }
}

vofpc_status launch_mass_transfer(vofpc_ctx ctx, vofpc_mesh M, const double *alpha, const int32_t *mixed,
                                  const int32_t *counts, const vofpc_interface *itf, const double *gradT,
                                  const double *gl, const double *gv, double k_l, double k_v, double h_lv,
                                  double *mdot, double *Qdot, double *mdot_c, double *Qdot_c) {
  VOFPC_REQUIRE(alpha && mixed && counts && itf && mdot && Qdot, VOFPC_E_INVALID_ARG, "mass_transfer: null argument");
  VOFPC_REQUIRE(itf->n && itf->A && itf->cap > 0, VOFPC_E_INVALID_ARG, "mass_transfer: interface record incomplete");
  VOFPC_REQUIRE((gl == nullptr) == (gv == nullptr), VOFPC_E_INVALID_ARG,
                "mass_transfer: give both phase gradients or neither");
  VOFPC_REQUIRE(gradT || gl, VOFPC_E_INVALID_ARG, "mass_transfer: no gradient given");
  VOFPC_REQUIRE(h_lv != 0.0, VOFPC_E_INVALID_ARG, "mass_transfer: h_lv must be nonzero");
  const int64_t N = M->d.n_cells;
  hipStream_t s = ctx->stream;
  if (mdot_c || Qdot_c) {
    int64_t g = (N + 255) / 256;
    if (g > ctx->n_cu * 8) g = ctx->n_cu * 8;
    fill_zero_kernel<<<(unsigned)g, 256, 0, s>>>(mdot_c, Qdot_c, N);
  }
  MdotParams p;
  p.V = M->d.V; p.alpha = alpha; p.n_cells = N;
  p.mixed = mixed; p.counts = counts; p.itf = *itf;
  p.gradT = gradT; p.gl = gl; p.gv = gv;
  p.k_l = k_l; p.k_v = k_v; p.h_lv = h_lv;
  p.mdot = mdot; p.Qdot = Qdot; p.mdot_c = mdot_c; p.Qdot_c = Qdot_c;
  int64_t grid = (std::min<int64_t>(N, itf->cap) + 255) / 256;
  if (grid > ctx->n_cu * 8) grid = ctx->n_cu * 8;
  if (grid < 1) grid = 1;
  mdot_kernel<<<(unsigned)grid, 256, 0, s>>>(p);
  VOFPC_HIP(hipGetLastError());
  return VOFPC_OK;
}

}  // namespace vofpc
