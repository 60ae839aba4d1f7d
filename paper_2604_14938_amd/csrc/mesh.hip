// Mesh upload: host-side validation and packing of the CSR topology, device
// copies, and the per-mesh geometry computed on the GPU (volumes, centroids,
// face area vectors and centroids, stored least-squares inverses, vertex
// weights).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "vofpc_internal.h"

namespace vofpc {

// ------------------------------------------------------------ geometry kernels
// Face area vector (right-hand rule on the stored loop) and area centroid,
// from the fan of triangles around the loop's vertex mean.
// Each cell-face slot's outward area vector (the face's, signed for the
// slot's cell), a cell's slots side by side.
__global__ void slot_area_kernel(DevMesh m, double *cf_S) {
  const int64_t P = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (P >= m.n_cells) return;
  const int64_t NF = m.n_faces;
  for (int64_t i = m.cell_face_off[P]; i < m.cell_face_off[P + 1]; ++i) {
    const int f = m.cell_face[i];
    const double sg = (m.face_owner[f] == P) ? 1.0 : -1.0;
    for (int c = 0; c < 3; ++c) cf_S[3 * i + c] = sg * m.Sf[c * NF + f];
  }
}

__global__ void face_geom_kernel(DevMesh m, double *Sf, double *xf) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= m.n_faces) return;
  const int64_t NV = m.n_verts, NF = m.n_faces;
  const int64_t o = m.face_vert_off[f];
  const int n = (int)(m.face_vert_off[f + 1] - o);
  double c0 = 0, c1 = 0, c2 = 0;
  for (int k = 0; k < n; ++k) {
    int v = m.face_vert[o + k];
    c0 += m.xyz[v]; c1 += m.xyz[NV + v]; c2 += m.xyz[2 * NV + v];
  }
  c0 /= n; c1 /= n; c2 /= n;
  double S0 = 0, S1 = 0, S2 = 0;
  for (int k = 0; k < n; ++k) {
    int va = m.face_vert[o + k], vb = m.face_vert[o + (k + 1 == n ? 0 : k + 1)];
    double a0 = m.xyz[va] - c0, a1 = m.xyz[NV + va] - c1, a2 = m.xyz[2 * NV + va] - c2;
    double b0 = m.xyz[vb] - c0, b1 = m.xyz[NV + vb] - c1, b2 = m.xyz[2 * NV + vb] - c2;
    S0 += 0.5 * (a1 * b2 - a2 * b1);
    S1 += 0.5 * (a2 * b0 - a0 * b2);
    S2 += 0.5 * (a0 * b1 - a1 * b0);
  }
  double Am = sqrt(S0 * S0 + S1 * S1 + S2 * S2);
  double n0 = S0 / Am, n1 = S1 / Am, n2 = S2 / Am;
  double w = 0, x0 = 0, x1 = 0, x2 = 0;
  for (int k = 0; k < n; ++k) {
    int va = m.face_vert[o + k], vb = m.face_vert[o + (k + 1 == n ? 0 : k + 1)];
    double A0 = m.xyz[va], A1 = m.xyz[NV + va], A2 = m.xyz[2 * NV + va];
    double B0 = m.xyz[vb], B1 = m.xyz[NV + vb], B2 = m.xyz[2 * NV + vb];
    double a0 = A0 - c0, a1 = A1 - c1, a2 = A2 - c2, b0 = B0 - c0, b1 = B1 - c1, b2 = B2 - c2;
    double t = 0.5 * (n0 * (a1 * b2 - a2 * b1) + n1 * (a2 * b0 - a0 * b2) + n2 * (a0 * b1 - a1 * b0));
    w += t;
    x0 += t * (c0 + A0 + B0) * (1.0 / 3.0);
    x1 += t * (c1 + A1 + B1) * (1.0 / 3.0);
    x2 += t * (c2 + A2 + B2) * (1.0 / 3.0);
  }
  Sf[f] = S0; Sf[NF + f] = S1; Sf[2 * NF + f] = S2;
  xf[f] = x0 / w; xf[NF + f] = x1 / w; xf[2 * NF + f] = x2 / w;
}

// Cell volume and centroid as a sum of pyramids from an interior point o (the
// mean of the face centroids) over the planar faces: V_f = (x_f - o).S_f / 3
// with the pyramid centroid at o + 3/4 (x_f - o).
__global__ void cell_geom_kernel(DevMesh m, const double *Sf, const double *xf, double *V, double *xc,
                                 int32_t *bad) {
  int64_t P = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (P >= m.n_cells) return;
  const int64_t NF = m.n_faces, N = m.n_cells;
  const int64_t b = m.cell_face_off[P], e = m.cell_face_off[P + 1];
  double o0 = 0, o1 = 0, o2 = 0;
  for (int64_t i = b; i < e; ++i) {
    int f = m.cell_face[i];
    o0 += xf[f]; o1 += xf[NF + f]; o2 += xf[2 * NF + f];
  }
  double inv = 1.0 / (double)(e - b);
  o0 *= inv; o1 *= inv; o2 *= inv;
  double vol = 0, m0 = 0, m1 = 0, m2 = 0;
  for (int64_t i = b; i < e; ++i) {
    int f = m.cell_face[i];
    double sg = (m.face_owner[f] == P) ? 1.0 : -1.0;
    double d0 = xf[f] - o0, d1 = xf[NF + f] - o1, d2 = xf[2 * NF + f] - o2;
    double vp = sg * (d0 * Sf[f] + d1 * Sf[NF + f] + d2 * Sf[2 * NF + f]) * (1.0 / 3.0);
    vol += vp;
    m0 += vp * (o0 + 0.75 * d0);
    m1 += vp * (o1 + 0.75 * d1);
    m2 += vp * (o2 + 0.75 * d2);
  }
  V[P] = vol;
  xc[P] = m0 / vol; xc[N + P] = m1 / vol; xc[2 * N + P] = m2 / vol;
  if (!(vol > 0)) atomicExch(bad, 1);
}

// Stored inverse of the plain least-squares matrix G_P = sum r r^T over face
// neighbours and value-boundary face centroids (App. B), six components.
__global__ void ginv_kernel(DevMesh m, const double *xc, const double *xf, double *ginv) {
  int64_t P = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (P >= m.n_cells) return;
  const int64_t N = m.n_cells, NF = m.n_faces;
  double px = xc[P], py = xc[N + P], pz = xc[2 * N + P];
  double xx = 0, yy = 0, zz = 0, xy = 0, xz = 0, yz = 0;
  for (int64_t i = m.cell_face_off[P]; i < m.cell_face_off[P + 1]; ++i) {
    int q = m.cf_nbr[i];
    double rx, ry, rz;
    if (q >= 0) {
      rx = xc[q] - px; ry = xc[N + q] - py; rz = xc[2 * N + q] - pz;
    } else if (q == -1) {
      int f = m.cell_face[i];
      rx = xf[f] - px; ry = xf[NF + f] - py; rz = xf[2 * NF + f] - pz;
    } else {
      continue;
    }
    xx += rx * rx; yy += ry * ry; zz += rz * rz; xy += rx * ry; xz += rx * rz; yz += ry * rz;
  }
  double c00 = yy * zz - yz * yz, c01 = xz * yz - xy * zz, c02 = xy * yz - xz * yy;
  double c11 = xx * zz - xz * xz, c12 = xy * xz - xx * yz, c22 = xx * yy - xy * xy;
  double det = xx * c00 + xy * c01 + xz * c02;
  double tr = (xx + yy + zz) * (1.0 / 3.0);
  double id = (det > 1e-12 * tr * tr * tr) ? 1.0 / det : 0.0;
  ginv[P] = c00 * id; ginv[N + P] = c11 * id; ginv[2 * N + P] = c22 * id;
  ginv[3 * N + P] = c01 * id; ginv[4 * N + P] = c02 * id; ginv[5 * N + P] = c12 * id;
}

// Normalised inverse-distance weights 1/|x_v - x_c| of the cells sharing a
// vertex, and the plain-mean weights 1/count.
__global__ void vertex_weight_kernel(DevMesh m, const double *xc, double *w, double *wmean) {
  int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= m.n_verts) return;
  const int64_t N = m.n_cells, NV = m.n_verts;
  double x = m.xyz[v], y = m.xyz[NV + v], z = m.xyz[2 * NV + v];
  int64_t b = m.vc_off[v], e = m.vc_off[v + 1];
  double sum = 0;
  for (int64_t j = b; j < e; ++j) {
    int c = m.vc_cell[j];
    double dx = x - xc[c], dy = y - xc[N + c], dz = z - xc[2 * N + c];
    double wi = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    w[j] = wi;
    sum += wi;
  }
  double inv = 1.0 / sum, im = 1.0 / (double)(e - b);
  for (int64_t j = b; j < e; ++j) {
    w[j] *= inv;
    wmean[j] = im;
  }
}

// Smallest |x_Q - x_P| over interior faces: non-negative doubles order like
// their bit patterns, so an unsigned atomic min reduces them.
__global__ void centre_distance_kernel(DevMesh m, const double *xc, uint64_t *dmin) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= m.n_faces) return;
  const int q = m.face_neigh[f];
  if (q < 0) return;
  const int o = m.face_owner[f];
  const int64_t N = m.n_cells;
  const double r0 = xc[q] - xc[o], r1 = xc[N + q] - xc[N + o], r2 = xc[2 * N + q] - xc[2 * N + o];
  const double d = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
  atomicMin((unsigned long long *)dmin, (unsigned long long)__double_as_longlong(d));
}

// -------------------------------------------------------------- host packing
namespace {

template <class T>
vofpc_status dev_copy(vofpc_mesh M, const T *host, size_t n, T **out) {
  void *p = nullptr;
  size_t bytes = std::max<size_t>(n * sizeof(T), 16);
  if (M->n_alloc >= (int)(sizeof(M->alloc) / sizeof(M->alloc[0]))) {
    set_error("mesh: too many device allocations");
    return VOFPC_E_STATE;
  }
  if (hipMalloc(&p, bytes) != hipSuccess) {
    set_error("hipMalloc failed during mesh upload");
    return VOFPC_E_OOM;
  }
  M->alloc[M->n_alloc++] = p;
  M->bytes += (int64_t)bytes;
  if (host && n) VOFPC_HIP(hipMemcpy(p, host, n * sizeof(T), hipMemcpyHostToDevice));
  *out = (T *)p;
  return VOFPC_OK;
}

}  // namespace

vofpc_status mesh_scratch_alloc(vofpc_mesh M, size_t bytes, void **out) {
  uint8_t *p = nullptr;
  vofpc_status st = dev_copy<uint8_t>(M, nullptr, bytes, &p);
  *out = p;
  return st;
}

// Cell -> vertex-neighbour lists (every cell sharing a vertex with the cell,
// itself excluded) for the extended gradient stencil, from the mesh's own
// cell -> vertex and vertex -> cell arrays, built on the host once.
vofpc_status mesh_vertex_stencil(vofpc_mesh M) {
  if (M->xn_off) return VOFPC_OK;
  const int64_t N = M->d.n_cells, NV = M->d.n_verts;
  std::vector<int64_t> cv_off(N + 1), vc_off(NV + 1);
  VOFPC_HIP(hipMemcpy(cv_off.data(), M->d.cv_off, sizeof(int64_t) * (N + 1), hipMemcpyDeviceToHost));
  VOFPC_HIP(hipMemcpy(vc_off.data(), M->d.vc_off, sizeof(int64_t) * (NV + 1), hipMemcpyDeviceToHost));
  std::vector<int32_t> cv(cv_off[N]), vc(vc_off[NV]);
  VOFPC_HIP(hipMemcpy(cv.data(), M->d.cv_gid, sizeof(int32_t) * cv.size(), hipMemcpyDeviceToHost));
  VOFPC_HIP(hipMemcpy(vc.data(), M->d.vc_cell, sizeof(int32_t) * vc.size(), hipMemcpyDeviceToHost));
  std::vector<int64_t> off(N + 1, 0);
  std::vector<int32_t> nb;
  nb.reserve((size_t)N * 32);
  std::vector<int32_t> stamp(N, -1);
  for (int64_t P = 0; P < N; ++P) {
    stamp[P] = (int32_t)P;
    for (int64_t a = cv_off[P]; a < cv_off[P + 1]; ++a) {
      const int32_t v = cv[a];
      for (int64_t j = vc_off[v]; j < vc_off[v + 1]; ++j) {
        const int32_t c = vc[j];
        if (stamp[c] != (int32_t)P) {
          stamp[c] = (int32_t)P;
          nb.push_back(c);
        }
      }
    }
    off[P + 1] = (int64_t)nb.size();
  }
  int64_t *d_off = nullptr;
  int32_t *d_nb = nullptr;
  vofpc_status st = dev_copy<int64_t>(M, off.data(), off.size(), &d_off);
  if (!st) st = dev_copy<int32_t>(M, nb.data(), nb.size(), &d_nb);
  if (st) return st;
  M->xn_off = d_off;
  M->xn_cell = d_nb;
  return VOFPC_OK;
}

// Kernel classes of a mesh: the class of its largest cell, and whether its
// cells spread over several classes, in which case the reconstruction
// buckets its mixed entries by class.  When all but at most 1 % of class 0
// are hexahedral-sized cells the others move to class 1 (mesh_class_of).
static vofpc_status setup_classes(vofpc_mesh M, const ClassStats &cs) {
  const int64_t N = M->d.n_cells;
  M->class_stats = cs;
  int64_t class_cnt[kClasses], cmax[kClasses][4];
  for (int c = 0; c < kClasses; ++c) {
    class_cnt[c] = cs.cnt[c];
    for (int t = 0; t < 4; ++t) cmax[c][t] = cs.max[c][t];
  }
  const int64_t rest = cs.cnt[0] - cs.hex_cnt;
  M->hex0 = rest > 0 && rest * 100 <= cs.cnt[0];
  if (M->hex0) {
    class_cnt[0] = cs.hex_cnt;
    class_cnt[1] += rest;
    for (int t = 0; t < 4; ++t) {
      cmax[0][t] = cs.hex_max[t];
      cmax[1][t] = std::max(cmax[1][t], cs.rest_max[t]);
    }
  }
  int big = 0;
  M->max_class = 0;
  for (int c = 0; c < kClasses; ++c) {
    M->class_cells[c] = class_cnt[c];
    for (int t = 0; t < 4; ++t) M->class_max[c][t] = cmax[c][t];
    M->tune[c] = 3;
    if (class_cnt[c] > 0) M->max_class = c;
    if (class_cnt[c] > 0) ++big;
  }
  M->bucketed = big >= 2;
  M->bucket_lists = nullptr;
  M->bucket_counts = nullptr;
  if (M->bucketed) {
    vofpc_status st = dev_copy<int32_t>(M, nullptr, (size_t)kClasses * N, &M->bucket_lists);
    if (!st) st = dev_copy<int32_t>(M, nullptr, kClasses, &M->bucket_counts);
    if (st) return st;
  }
  return VOFPC_OK;
}

vofpc_status mesh_upload(vofpc_ctx ctx, const vofpc_mesh_desc *d, vofpc_mesh *out) {
  VOFPC_REQUIRE(ctx && d && out, VOFPC_E_INVALID_ARG, "mesh_upload: null argument");
  const int64_t N = d->n_cells, NF = d->n_faces, NV = d->n_verts;
  VOFPC_REQUIRE(N > 0 && NF > 0 && NV > 0, VOFPC_E_INVALID_ARG, "mesh_upload: empty mesh");
  VOFPC_REQUIRE(N < INT32_MAX && NF < INT32_MAX && NV < INT32_MAX, VOFPC_E_INVALID_ARG,
                "mesh_upload: counts must fit in int32");
  VOFPC_REQUIRE(d->cell_face_off && d->cell_face && d->face_vert_off && d->face_vert && d->face_owner &&
                    d->face_neigh && d->face_bc && d->vert_xyz,
                VOFPC_E_INVALID_ARG, "mesh_upload: null array in descriptor");
  const int64_t *cfo = d->cell_face_off, *fvo = d->face_vert_off;
  VOFPC_REQUIRE(cfo[0] == 0 && fvo[0] == 0, VOFPC_E_MESH, "mesh_upload: offsets must start at 0");
  for (int64_t i = 0; i < N; ++i)
    VOFPC_REQUIRE(cfo[i + 1] >= cfo[i] + 4 && cfo[i + 1] - cfo[i] <= 255, VOFPC_E_MESH,
                  "mesh_upload: a cell needs 4..255 faces (cell " + std::to_string(i) + ")");
  for (int64_t f = 0; f < NF; ++f) {
    VOFPC_REQUIRE(fvo[f + 1] >= fvo[f] + 3 && fvo[f + 1] - fvo[f] <= 255, VOFPC_E_MESH,
                  "mesh_upload: a face needs 3..255 vertices (face " + std::to_string(f) + ")");
    int32_t o = d->face_owner[f], q = d->face_neigh[f];
    VOFPC_REQUIRE(o >= 0 && o < N && q >= -1 && q < N && q != o, VOFPC_E_MESH,
                  "mesh_upload: bad owner/neighbour of face " + std::to_string(f));
    VOFPC_REQUIRE(d->face_bc[f] >= 0 && d->face_bc[f] <= 2, VOFPC_E_MESH, "mesh_upload: face_bc must be 0, 1 or 2");
    VOFPC_REQUIRE((q >= 0) == (d->face_bc[f] == 0), VOFPC_E_MESH,
                  "mesh_upload: interior faces need face_bc 0, boundary faces 1 or 2 (face " + std::to_string(f) + ")");
  }
  const int64_t nfv = fvo[NF];
  for (int64_t k = 0; k < nfv; ++k)
    VOFPC_REQUIRE(d->face_vert[k] >= 0 && d->face_vert[k] < NV, VOFPC_E_MESH, "mesh_upload: vertex id out of range");
  // every face listed exactly by its owner and (if interior) its neighbour
  const int64_t ncf = cfo[N];
  std::vector<int32_t> seen(NF, 0);
  for (int64_t P = 0; P < N; ++P)
    for (int64_t i = cfo[P]; i < cfo[P + 1]; ++i) {
      int32_t f = d->cell_face[i];
      VOFPC_REQUIRE(f >= 0 && f < NF, VOFPC_E_MESH, "mesh_upload: face id out of range");
      VOFPC_REQUIRE(d->face_owner[f] == P || d->face_neigh[f] == P, VOFPC_E_MESH,
                    "mesh_upload: cell " + std::to_string(P) + " lists face " + std::to_string(f) +
                        " it does not own or neighbour");
      seen[f]++;
    }
  for (int64_t f = 0; f < NF; ++f)
    VOFPC_REQUIRE(seen[f] == (d->face_neigh[f] >= 0 ? 2 : 1), VOFPC_E_MESH,
                  "mesh_upload: face " + std::to_string(f) + " is not listed by exactly its cells");

  // packed cell-local polyhedra
  std::vector<int64_t> cv_off(N + 1, 0), cl_off(N + 1, 0);
  std::vector<int32_t> cv_gid;
  std::vector<uint8_t> cl_lv;
  std::vector<uint16_t> cl_eid;            // local undirected edge id per loop position
  std::vector<uint32_t> ce;                // per local edge: u, v, face running u -> v, the other face
  std::vector<uint32_t> cl_info;           // face (bits 0-7), index in face (8-15), next position (16-31)
  std::vector<int32_t> edge_stamp(65536, -1), edge_id(65536, 0);
  std::vector<int32_t> cf_nbr(ncf);
  std::vector<uint16_t> cf_loff(ncf);
  std::vector<uint8_t> cf_lsz(ncf);
  cv_gid.reserve(ncf * 2);
  cl_lv.reserve(nfv * 2);
  int64_t max_nf = 0, max_nv = 0, max_fv = 0, max_ne = 0, max_loop = 0;
  ClassStats class_stats;
  std::vector<int32_t> loc;
  std::vector<uint16_t> dedge;
  for (int64_t P = 0; P < N; ++P) {
    loc.clear();
    dedge.clear();
    int64_t lbase = (int64_t)cl_lv.size();
    for (int64_t i = cfo[P]; i < cfo[P + 1]; ++i) {
      int32_t f = d->cell_face[i];
      int64_t o = fvo[f], n = fvo[f + 1] - o;
      bool rev = d->face_owner[f] != P;
      int64_t loff = (int64_t)cl_lv.size() - lbase;
      VOFPC_REQUIRE(loff < 65535, VOFPC_E_MESH, "mesh_upload: cell loops too long");
      cf_loff[i] = (uint16_t)loff;
      cf_lsz[i] = (uint8_t)n;
      const uint32_t fl = (uint32_t)(i - cfo[P]);
      for (int64_t k = 0; k < n; ++k)
        cl_info.push_back(fl | (uint32_t)k << 8 | (uint32_t)(loff + (k + 1 == n ? 0 : k + 1)) << 16);
      int32_t first = -1, prev = -1;
      for (int64_t k = 0; k < n; ++k) {
        int32_t g = d->face_vert[o + (rev ? n - 1 - k : k)];
        int32_t l = -1;
        for (size_t j = 0; j < loc.size(); ++j)
          if (loc[j] == g) { l = (int32_t)j; break; }
        if (l < 0) {
          VOFPC_REQUIRE(loc.size() < 255, VOFPC_E_MESH, "mesh_upload: more than 255 vertices in a cell");
          l = (int32_t)loc.size();
          loc.push_back(g);
        }
        cl_lv.push_back((uint8_t)l);
        if (k == 0) first = l; else dedge.push_back((uint16_t)(prev << 8 | l));
        prev = l;
      }
      dedge.push_back((uint16_t)(prev << 8 | first));
      int32_t q = d->face_owner[f] == P ? d->face_neigh[f] : d->face_owner[f];
      cf_nbr[i] = q >= 0 ? q : (d->face_bc[f] == 2 ? -2 : -1);
      max_fv = std::max(max_fv, n);
    }
    // closed surface: every directed edge once, and its reverse once
    std::sort(dedge.begin(), dedge.end());
    for (size_t j = 0; j < dedge.size(); ++j) {
      VOFPC_REQUIRE(j == 0 || dedge[j] != dedge[j - 1], VOFPC_E_MESH,
                    "mesh_upload: cell " + std::to_string(P) + " repeats a directed edge (bad orientation)");
      uint16_t r = (uint16_t)((dedge[j] & 0xff) << 8 | (dedge[j] >> 8));
      VOFPC_REQUIRE(std::binary_search(dedge.begin(), dedge.end(), r), VOFPC_E_MESH,
                    "mesh_upload: cell " + std::to_string(P) + " is not closed");
    }
    // local edge ids in order of first appearance along the loops
    {
      int32_t ne = 0;
      for (int64_t i = cfo[P]; i < cfo[P + 1]; ++i) {
        int64_t o = lbase + cf_loff[i], n = cf_lsz[i];
        for (int64_t k = 0; k < n; ++k) {
          int a = cl_lv[o + k], b = cl_lv[o + (k + 1 == n ? 0 : k + 1)];
          int key = a < b ? (a << 8 | b) : (b << 8 | a);
          const uint32_t fl = (uint32_t)(i - cfo[P]);
          if (edge_stamp[key] != (int32_t)P) {
            edge_stamp[key] = (int32_t)P;
            edge_id[key] = ne++;
            ce.push_back((uint32_t)a | (uint32_t)b << 8 | fl << 16);
          } else {
            ce[ce.size() - ne + edge_id[key]] |= fl << 24;   // the second face runs b -> a
          }
          cl_eid.push_back((uint16_t)edge_id[key]);
        }
      }
    }
    for (int32_t g : loc) cv_gid.push_back(g);
    cv_off[P + 1] = (int64_t)cv_gid.size();
    cl_off[P + 1] = (int64_t)cl_lv.size();
    max_nf = std::max(max_nf, cfo[P + 1] - cfo[P]);
    max_nv = std::max<int64_t>(max_nv, (int64_t)loc.size());
    max_ne = std::max<int64_t>(max_ne, (int64_t)dedge.size() / 2);
    max_loop = std::max<int64_t>(max_loop, cl_off[P + 1] - cl_off[P]);
    {
      const int64_t sz[4] = {(int64_t)loc.size(), cfo[P + 1] - cfo[P], cl_off[P + 1] - cl_off[P],
                             (int64_t)dedge.size() / 2};
      class_stats.add(sz);
    }
  }
  // vertex -> cell incidence (cells ascending)
  std::vector<int64_t> vc_off(NV + 1, 0);
  for (int32_t g : cv_gid) vc_off[g + 1]++;
  for (int64_t v = 0; v < NV; ++v) vc_off[v + 1] += vc_off[v];
  for (int64_t v = 0; v < NV; ++v)
    VOFPC_REQUIRE(vc_off[v + 1] > vc_off[v], VOFPC_E_MESH, "mesh_upload: vertex " + std::to_string(v) + " is unused");
  std::vector<int32_t> vc_cell(vc_off[NV]);
  {
    std::vector<int64_t> fill(vc_off.begin(), vc_off.end() - 1);
    for (int64_t P = 0; P < N; ++P)
      for (int64_t j = cv_off[P]; j < cv_off[P + 1]; ++j) vc_cell[fill[cv_gid[j]]++] = (int32_t)P;
  }

  VOFPC_HIP(hipSetDevice(ctx->device));
  vofpc_mesh M = new (std::nothrow) vofpc_mesh_s();
  VOFPC_REQUIRE(M, VOFPC_E_OOM, "mesh_upload: host allocation failed");
  M->ctx = ctx;
  DevMesh &m = M->d;
  m.n_cells = N; m.n_faces = NF; m.n_verts = NV;
  vofpc_status st = VOFPC_OK;
#define COPY(field, host, n, T)                                   \
  do {                                                             \
    T *p_ = nullptr;                                               \
    st = dev_copy<T>(M, host, (size_t)(n), &p_);                   \
    if (st) { vofpc_mesh_free(M); return st; }                     \
    m.field = p_;                                                  \
  } while (0)
  COPY(cell_face_off, cfo, N + 1, int64_t);
  COPY(cell_face, d->cell_face, ncf, int32_t);
  COPY(face_vert_off, fvo, NF + 1, int64_t);
  COPY(face_vert, d->face_vert, nfv, int32_t);
  COPY(face_owner, d->face_owner, NF, int32_t);
  COPY(face_neigh, d->face_neigh, NF, int32_t);
  COPY(face_bc, d->face_bc, NF, int8_t);
  COPY(xyz, d->vert_xyz, 3 * NV, double);
  COPY(cf_nbr, cf_nbr.data(), ncf, int32_t);
  COPY(cf_loff, cf_loff.data(), ncf, uint16_t);
  COPY(cf_lsz, cf_lsz.data(), ncf, uint8_t);
  COPY(cv_off, cv_off.data(), N + 1, int64_t);
  COPY(cv_gid, cv_gid.data(), cv_gid.size(), int32_t);
  COPY(cl_off, cl_off.data(), N + 1, int64_t);
  COPY(cl_lv, cl_lv.data(), cl_lv.size(), uint8_t);
  COPY(cl_eid, cl_eid.data(), cl_eid.size(), uint16_t);
  COPY(cl_info, cl_info.data(), cl_info.size(), uint32_t);
  COPY(ce, ce.data(), ce.size(), uint32_t);
  COPY(vc_off, vc_off.data(), NV + 1, int64_t);
  COPY(vc_cell, vc_cell.data(), vc_cell.size(), int32_t);
  COPY(vc_w, (const double *)nullptr, vc_cell.size(), double);
  COPY(vc_wmean, (const double *)nullptr, vc_cell.size(), double);
  COPY(V, (const double *)nullptr, N, double);
  COPY(xc, (const double *)nullptr, 3 * N, double);
  COPY(Sf, (const double *)nullptr, 3 * NF, double);
  COPY(xf, (const double *)nullptr, 3 * NF, double);
  COPY(ginv, (const double *)nullptr, 6 * N, double);
  COPY(cf_S, (const double *)nullptr, 3 * ncf, double);
  M->n_blk = (N + kCompactBlockCells - 1) / kCompactBlockCells;
  {
    uint8_t *fl = nullptr;
    int32_t *bc = nullptr;
    if ((st = dev_copy<uint8_t>(M, nullptr, N, &fl)) || (st = dev_copy<int32_t>(M, nullptr, 2 * M->n_blk, &bc))) {
      vofpc_mesh_free(M);
      return st;
    }
    M->flags = fl; M->blk_cnt = bc;
    uint8_t *cr = nullptr;
    if ((st = dev_copy<uint8_t>(M, nullptr, N, &cr))) {
      vofpc_mesh_free(M);
      return st;
    }
    M->cross = cr;
    VOFPC_HIP(hipMemset(cr, 0, (size_t)std::max<int64_t>(N, 1)));
    uint64_t *sd = nullptr;
    if ((st = dev_copy<uint64_t>(M, nullptr, 2 * ((N + 63) / 64), &sd))) {
      vofpc_mesh_free(M);
      return st;
    }
    M->side = sd;
  }
  int32_t *bad = nullptr;
  if ((st = dev_copy<int32_t>(M, nullptr, 1, &bad))) {
    vofpc_mesh_free(M);
    return st;
  }
#undef COPY
  M->max_nf = max_nf; M->max_nv = max_nv; M->max_fv = max_fv; M->max_ne = max_ne; M->max_loop = max_loop;
  M->ncf = ncf; M->nfv = nfv; M->ncv = (int64_t)cv_gid.size(); M->ncl = (int64_t)cl_lv.size();
  M->nvc = (int64_t)vc_cell.size();
  if ((st = setup_classes(M, class_stats))) {
    vofpc_mesh_free(M);
    return st;
  }

  hipStream_t s = ctx->stream;
  const int B = 256;
  VOFPC_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), s));
  face_geom_kernel<<<(unsigned)((NF + B - 1) / B), B, 0, s>>>(m, (double *)m.Sf, (double *)m.xf);
  cell_geom_kernel<<<(unsigned)((N + B - 1) / B), B, 0, s>>>(m, m.Sf, m.xf, (double *)m.V, (double *)m.xc, bad);
  ginv_kernel<<<(unsigned)((N + B - 1) / B), B, 0, s>>>(m, m.xc, m.xf, (double *)m.ginv);
  slot_area_kernel<<<(unsigned)((N + B - 1) / B), B, 0, s>>>(m, (double *)m.cf_S);
  vertex_weight_kernel<<<(unsigned)((NV + B - 1) / B), B, 0, s>>>(m, m.xc, (double *)m.vc_w, (double *)m.vc_wmean);
  // smallest distance between the centres of two face neighbours (the
  // pseudo-time step of the gradient extrapolation); as ordered bits of a
  // non-negative double, reduced by atomic min
  uint64_t *dmin = nullptr;
  if ((st = dev_copy<uint64_t>(M, nullptr, 1, &dmin))) {
    vofpc_mesh_free(M);
    return st;
  }
  VOFPC_HIP(hipMemsetAsync(dmin, 0x7f, sizeof(uint64_t), s));
  centre_distance_kernel<<<(unsigned)((NF + B - 1) / B), B, 0, s>>>(m, m.xc, dmin);
  VOFPC_HIP(hipGetLastError());
  int32_t hbad = 0;
  uint64_t hmin = 0;
  VOFPC_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  VOFPC_HIP(hipMemcpyAsync(&hmin, dmin, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  VOFPC_HIP(hipStreamSynchronize(s));
  if (hbad) {
    vofpc_mesh_free(M);
    set_error("mesh_upload: a cell has non-positive volume (inverted or open)");
    return VOFPC_E_MESH;
  }
  {
    double d;
    memcpy(&d, &hmin, sizeof d);
    M->min_centre_dist = d;   // huge (0x7f7f...) when the mesh has no interior face
  }
  *out = M;
  return VOFPC_OK;
}

// ------------------------------------------------------------- concatenation
// dst[i] = src[i] + add (mode 1), + add where src >= 0 (mode 2), or a copy (0)
template <class T>
__global__ __launch_bounds__(256) void concat_copy_kernel(T *dst, const T *src, int64_t n, int64_t add, int mode) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const T v = src[i];
    dst[i] = (mode == 1 || (mode == 2 && v >= 0)) ? (T)(v + add) : v;
  }
}

namespace {
template <class T>
vofpc_status concat_copy(hipStream_t s, T *dst, const T *src, int64_t n, int64_t add, int mode) {
  if (n <= 0) return VOFPC_OK;
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  concat_copy_kernel<T><<<(unsigned)g, 256, 0, s>>>(dst, src, n, add, mode);
  VOFPC_HIP(hipGetLastError());
  return VOFPC_OK;
}
}  // namespace

vofpc_status mesh_concat(vofpc_ctx ctx, const vofpc_mesh *ms, int32_t n, vofpc_mesh *out) {
  VOFPC_REQUIRE(ctx && ms && out && n >= 1, VOFPC_E_INVALID_ARG, "mesh_concat: bad argument");
  int64_t N = 0, NF = 0, NV = 0, ncf = 0, nfv = 0, ncv = 0, ncl = 0, nvc = 0;
  int64_t mx[5] = {0, 0, 0, 0, 0};
  for (int i = 0; i < n; ++i) {
    const vofpc_mesh a = ms[i];
    VOFPC_REQUIRE(a, VOFPC_E_INVALID_ARG, "mesh_concat: null mesh in the list");
    VOFPC_REQUIRE(a->ctx && a->ctx->device == ctx->device, VOFPC_E_STATE, "mesh_concat: mesh on another device");
    N += a->d.n_cells; NF += a->d.n_faces; NV += a->d.n_verts;
    ncf += a->ncf; nfv += a->nfv; ncv += a->ncv; ncl += a->ncl; nvc += a->nvc;
    mx[0] = std::max(mx[0], a->max_nf); mx[1] = std::max(mx[1], a->max_nv); mx[2] = std::max(mx[2], a->max_fv);
    mx[3] = std::max(mx[3], a->max_ne); mx[4] = std::max(mx[4], a->max_loop);
  }
  VOFPC_REQUIRE(N < INT32_MAX && NF < INT32_MAX && NV < INT32_MAX && ncf < INT32_MAX && nvc < INT32_MAX,
                VOFPC_E_INVALID_ARG, "mesh_concat: totals must fit in int32");
  VOFPC_HIP(hipSetDevice(ctx->device));
  vofpc_mesh M = new (std::nothrow) vofpc_mesh_s();
  VOFPC_REQUIRE(M, VOFPC_E_OOM, "mesh_concat: host allocation failed");
  M->ctx = ctx;
  DevMesh &m = M->d;
  m.n_cells = N; m.n_faces = NF; m.n_verts = NV;
  vofpc_status st = VOFPC_OK;
#define ALLOC(field, n_, T)                                        \
  do {                                                             \
    T *p_ = nullptr;                                               \
    st = dev_copy<T>(M, (const T *)nullptr, (size_t)(n_), &p_);    \
    if (st) { vofpc_mesh_free(M); return st; }                     \
    m.field = p_;                                                  \
  } while (0)
  ALLOC(cell_face_off, N + 1, int64_t);
  ALLOC(cell_face, ncf, int32_t);
  ALLOC(face_vert_off, NF + 1, int64_t);
  ALLOC(face_vert, nfv, int32_t);
  ALLOC(face_owner, NF, int32_t);
  ALLOC(face_neigh, NF, int32_t);
  ALLOC(face_bc, NF, int8_t);
  ALLOC(xyz, 3 * NV, double);
  ALLOC(cf_nbr, ncf, int32_t);
  ALLOC(cf_loff, ncf, uint16_t);
  ALLOC(cf_lsz, ncf, uint8_t);
  ALLOC(cv_off, N + 1, int64_t);
  ALLOC(cv_gid, ncv, int32_t);
  ALLOC(cl_off, N + 1, int64_t);
  ALLOC(cl_lv, ncl, uint8_t);
  ALLOC(cl_eid, ncl, uint16_t);
  ALLOC(cl_info, ncl, uint32_t);
  ALLOC(ce, ncl / 2, uint32_t);
  ALLOC(vc_off, NV + 1, int64_t);
  ALLOC(vc_cell, nvc, int32_t);
  ALLOC(vc_w, nvc, double);
  ALLOC(vc_wmean, nvc, double);
  ALLOC(V, N, double);
  ALLOC(xc, 3 * N, double);
  ALLOC(Sf, 3 * NF, double);
  ALLOC(xf, 3 * NF, double);
  ALLOC(ginv, 6 * N, double);
  ALLOC(cf_S, 3 * ncf, double);
#undef ALLOC
  M->n_blk = (N + kCompactBlockCells - 1) / kCompactBlockCells;
  {
    uint8_t *fl = nullptr;
    int32_t *bc = nullptr;
    if ((st = dev_copy<uint8_t>(M, nullptr, N, &fl)) || (st = dev_copy<int32_t>(M, nullptr, 2 * M->n_blk, &bc))) {
      vofpc_mesh_free(M);
      return st;
    }
    M->flags = fl; M->blk_cnt = bc;
    uint8_t *cr = nullptr;
    if ((st = dev_copy<uint8_t>(M, nullptr, N, &cr))) {
      vofpc_mesh_free(M);
      return st;
    }
    M->cross = cr;
    VOFPC_HIP(hipMemset(cr, 0, (size_t)std::max<int64_t>(N, 1)));
    uint64_t *sd = nullptr;
    if ((st = dev_copy<uint64_t>(M, nullptr, 2 * ((N + 63) / 64), &sd))) {
      vofpc_mesh_free(M);
      return st;
    }
    M->side = sd;
  }
  M->max_nf = mx[0]; M->max_nv = mx[1]; M->max_fv = mx[2]; M->max_ne = mx[3]; M->max_loop = mx[4];
  M->ncf = ncf; M->nfv = nfv; M->ncv = ncv; M->ncl = ncl; M->nvc = nvc;
  {
    ClassStats cs;
    M->min_centre_dist = ms[0]->min_centre_dist;
    for (int i = 0; i < n; ++i) {
      cs.merge(ms[i]->class_stats);
      M->min_centre_dist = std::min(M->min_centre_dist, ms[i]->min_centre_dist);
    }
    if ((st = setup_classes(M, cs))) {
      vofpc_mesh_free(M);
      return st;
    }
  }
  hipStream_t s = ctx->stream;
  int64_t bN = 0, bF = 0, bV = 0, bcf = 0, bfv = 0, bcv = 0, bcl = 0, bvc = 0;
#define CC(dst, src, cnt, add, mode)                                                        \
  do {                                                                                      \
    st = concat_copy(s, (dst), (src), (cnt), (add), (mode));                                \
    if (st) { vofpc_mesh_free(M); return st; }                                              \
  } while (0)
  for (int i = 0; i < n; ++i) {
    const DevMesh &a = ms[i]->d;
    const vofpc_mesh_s &A = *ms[i];
    const int64_t n_ = a.n_cells, nf_ = a.n_faces, nv_ = a.n_verts;
    // offset arrays (n+1 entries; the last entry of one mesh equals the first of the next)
    CC((int64_t *)m.cell_face_off + bN, a.cell_face_off, n_ + 1, bcf, 1);
    CC((int64_t *)m.face_vert_off + bF, a.face_vert_off, nf_ + 1, bfv, 1);
    CC((int64_t *)m.cv_off + bN, a.cv_off, n_ + 1, bcv, 1);
    CC((int64_t *)m.cl_off + bN, a.cl_off, n_ + 1, bcl, 1);
    CC((int64_t *)m.vc_off + bV, a.vc_off, nv_ + 1, bvc, 1);
    // ids
    CC((int32_t *)m.cell_face + bcf, a.cell_face, A.ncf, bF, 1);
    CC((int32_t *)m.face_vert + bfv, a.face_vert, A.nfv, bV, 1);
    CC((int32_t *)m.face_owner + bF, a.face_owner, nf_, bN, 1);
    CC((int32_t *)m.face_neigh + bF, a.face_neigh, nf_, bN, 2);
    CC((int32_t *)m.cf_nbr + bcf, a.cf_nbr, A.ncf, bN, 2);
    CC((int32_t *)m.cv_gid + bcv, a.cv_gid, A.ncv, bV, 1);
    CC((int32_t *)m.vc_cell + bvc, a.vc_cell, A.nvc, bN, 1);
    // plain copies
    CC((int8_t *)m.face_bc + bF, a.face_bc, nf_, 0, 0);
    CC((uint16_t *)m.cf_loff + bcf, a.cf_loff, A.ncf, 0, 0);
    CC((uint8_t *)m.cf_lsz + bcf, a.cf_lsz, A.ncf, 0, 0);
    CC((uint8_t *)m.cl_lv + bcl, a.cl_lv, A.ncl, 0, 0);
    CC((uint16_t *)m.cl_eid + bcl, a.cl_eid, A.ncl, 0, 0);
    CC((uint32_t *)m.cl_info + bcl, a.cl_info, A.ncl, 0, 0);
    CC((uint32_t *)m.ce + bcl / 2, a.ce, A.ncl / 2, 0, 0);
    CC((double *)m.vc_w + bvc, a.vc_w, A.nvc, 0, 0);
    CC((double *)m.vc_wmean + bvc, a.vc_wmean, A.nvc, 0, 0);
    CC((double *)m.V + bN, a.V, n_, 0, 0);
    CC((double *)m.cf_S + 3 * bcf, a.cf_S, 3 * A.ncf, 0, 0);
    // structure-of-arrays fields, one component at a time
    for (int c = 0; c < 3; ++c) {
      CC((double *)m.xyz + c * NV + bV, a.xyz + c * nv_, nv_, 0, 0);
      CC((double *)m.xc + c * N + bN, a.xc + c * n_, n_, 0, 0);
      CC((double *)m.Sf + c * NF + bF, a.Sf + c * nf_, nf_, 0, 0);
      CC((double *)m.xf + c * NF + bF, a.xf + c * nf_, nf_, 0, 0);
    }
    for (int c = 0; c < 6; ++c) CC((double *)m.ginv + c * N + bN, a.ginv + c * n_, n_, 0, 0);
    bN += n_; bF += nf_; bV += nv_;
    bcf += A.ncf; bfv += A.nfv; bcv += A.ncv; bcl += A.ncl; bvc += A.nvc;
  }
#undef CC
  VOFPC_HIP(hipStreamSynchronize(s));
  *out = M;
  return VOFPC_OK;
}

}  // namespace vofpc

extern "C" vofpc_status vofpc_mesh_concat(vofpc_ctx ctx, const vofpc_mesh *meshes, int32_t n, vofpc_mesh *out) {
  vofpc::clear_error();
  if (out) *out = nullptr;
  return vofpc::mesh_concat(ctx, meshes, n, out);
}

extern "C" vofpc_status vofpc_mesh_upload(vofpc_ctx ctx, const vofpc_mesh_desc *desc, vofpc_mesh *out) {
  vofpc::clear_error();
  if (out) *out = nullptr;
  return vofpc::mesh_upload(ctx, desc, out);
}

extern "C" vofpc_status vofpc_mesh_free(vofpc_mesh mesh) {
  vofpc::clear_error();
  if (!mesh) return VOFPC_OK;
  if (mesh->ctx) (void)hipSetDevice(mesh->ctx->device);
  for (int i = 0; i < mesh->n_alloc; ++i) (void)hipFree(mesh->alloc[i]);
  delete mesh;
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_mesh_info(vofpc_mesh m, int64_t info[8]) {
  vofpc::clear_error();
  VOFPC_REQUIRE(m && info, VOFPC_E_INVALID_ARG, "mesh_info: null argument");
  info[0] = m->d.n_cells; info[1] = m->d.n_faces; info[2] = m->d.n_verts;
  info[3] = m->max_nf; info[4] = m->max_nv; info[5] = m->max_fv; info[6] = m->max_ne; info[7] = m->bytes;
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_mesh_classes(vofpc_mesh m, int64_t cells[4], int32_t tune[4], int32_t *bucketed) {
  vofpc::clear_error();
  VOFPC_REQUIRE(m, VOFPC_E_INVALID_ARG, "mesh_classes: null mesh");
  for (int c = 0; c < vofpc::kClasses; ++c) {
    if (cells) cells[c] = m->class_cells[c];
    if (tune) tune[c] = m->tune[c];
  }
  if (bucketed) *bucketed = m->bucketed ? 1 : 0;
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_mesh_geometry(vofpc_mesh m, double *V, double *xc, double *Sf, double *xf) {
  vofpc::clear_error();
  VOFPC_REQUIRE(m, VOFPC_E_INVALID_ARG, "mesh_geometry: null mesh");
  hipStream_t s = m->ctx->stream;
  VOFPC_HIP(hipSetDevice(m->ctx->device));
  const int64_t N = m->d.n_cells, NF = m->d.n_faces;
  if (V) VOFPC_HIP(hipMemcpyAsync(V, m->d.V, N * 8, hipMemcpyDeviceToDevice, s));
  if (xc) VOFPC_HIP(hipMemcpyAsync(xc, m->d.xc, 3 * N * 8, hipMemcpyDeviceToDevice, s));
  if (Sf) VOFPC_HIP(hipMemcpyAsync(Sf, m->d.Sf, 3 * NF * 8, hipMemcpyDeviceToDevice, s));
  if (xf) VOFPC_HIP(hipMemcpyAsync(xf, m->d.xf, 3 * NF * 8, hipMemcpyDeviceToDevice, s));
  return VOFPC_OK;
}
