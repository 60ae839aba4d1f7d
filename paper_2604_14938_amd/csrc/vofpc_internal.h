// Internal declarations shared by the vofpc translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/vofpc.h"

namespace vofpc {

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
void clear_error();

#define VOFPC_HIP(call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      ::vofpc::set_error(std::string(#call) + ": " + hipGetErrorString(e_));         \
      return VOFPC_E_HIP;                                                            \
    }                                                                                \
  } while (0)

#define VOFPC_REQUIRE(cond, code, msg)                                               \
  do {                                                                               \
    if (!(cond)) {                                                                   \
      ::vofpc::set_error(msg);                                                       \
      return code;                                                                   \
    }                                                                                \
  } while (0)

// ------------------------------------------------------------- device mesh
// Everything a kernel needs about a mesh, as raw device pointers.
struct DevMesh {
  int64_t n_cells, n_faces, n_verts;
  // topology (as uploaded)
  const int64_t *cell_face_off;
  const int32_t *cell_face;
  const int64_t *face_vert_off;
  const int32_t *face_vert;
  const int32_t *face_owner;
  const int32_t *face_neigh;
  const int8_t *face_bc;
  const double *xyz;  // [3][n_verts]
  // per cell-face slot (same indexing as cell_face): neighbour across the
  // face, or -1 (boundary with value) / -2 (symmetry); loop offset and size
  // of the face inside the cell's packed loops
  const int32_t *cf_nbr;
  const uint16_t *cf_loff;
  const uint8_t *cf_lsz;
  const double *cf_S;  // [slot][3]: the face's area vector pointing out of the slot's cell
                       // (Sf or -Sf), a cell's slots contiguous
  // packed cell-local polyhedra: distinct vertices (global ids) and the
  // outward face loops as local vertex ids, faces in cell_face order
  const int64_t *cv_off;
  const int32_t *cv_gid;
  const int64_t *cl_off;
  const uint8_t *cl_lv;
  const uint16_t *cl_eid;  // local undirected edge id of each loop position
  const uint32_t *cl_info; // face within the cell (bits 0-7), index within the face
                           // (8-15) and cell-local next loop position (16-31)
  const uint32_t *ce;      // per cell-local edge (cell P's edges from cl_off[P]/2, in
                           // local edge id order): vertices u (bits 0-7), v (8-15),
                           // the face whose loop runs u -> v (16-23) and the other (24-31)
  // vertex -> cell incidence with normalised inverse-distance weights
  const int64_t *vc_off;
  const int32_t *vc_cell;
  const double *vc_w;
  const double *vc_wmean;  // 1/count per incidence
  // geometry
  const double *V;     // [n_cells]
  const double *xc;    // [3][n_cells]
  const double *Sf;    // [3][n_faces]
  const double *xf;    // [3][n_faces]
  const double *ginv;  // [6][n_cells] xx yy zz xy xz yz of the inverse
};

// cells per block of the compaction kernels (sizes a mesh's block arrays)
constexpr int kCompactBlockCells = 256;
// XCDs of the chip (the hardware hands workgroup b to XCD b % kXcd; a
// schedule built on this only gains or loses locality, never correctness)
// and the spacing of the work-queue counters (one 128-byte line each)
constexpr int kXcd = 8;
constexpr int kQueueStride = 32;
constexpr int kQueueSet = (1 + kXcd) * kQueueStride;   // the counters of one class launch

// Reconstruction kernel classes: the template variants by the largest cell
// they hold (vertices, faces, loop positions, edges): hexahedra and smaller
// cells; the usual Voronoi cells (about 99.5 % of a jittered-BCC mesh's);
// the larger Voronoi cells; anything larger.
constexpr int kClasses = 4;
constexpr int kQueueInts = kClasses * kQueueSet;   // one set per class: class launches may overlap
__host__ __device__ inline int class_of(int64_t nv, int64_t nf, int64_t nl, int64_t ne) {
  if (nv <= 16 && nf <= 8 && nl <= 48 && ne <= 24) return 0;
  if (nv <= 32 && nf <= 20 && nl <= 96 && ne <= 48) return 1;
  if (nv <= 48 && nf <= 32 && nl <= 128 && ne <= 64) return 2;
  return 3;
}
// Cells within the hexahedral caps (vertices, faces, loop positions, edges).
__host__ __device__ inline bool fits_hex(int64_t nv, int64_t nf, int64_t nl, int64_t ne) {
  return nv <= 8 && nf <= 6 && nl <= 24 && ne <= 12;
}
// The class a mesh gives a cell: class_of, except that a mesh whose class 0
// is all but at most 1 % hexahedral-sized cells (hex0) moves the other
// class-0 cells to class 1, so its class 0 runs the hexahedral layout.
__host__ __device__ inline int mesh_class_of(bool hex0, int64_t nv, int64_t nf, int64_t nl, int64_t ne) {
  const int c = class_of(nv, nf, nl, ne);
  return (hex0 && c == 0 && !fits_hex(nv, nf, nl, ne)) ? 1 : c;
}
// Size statistics of a mesh's cells by class_of, kept so that meshes can be
// concatenated: counts and largest sizes per class, and of the class-0 cells
// the number within the hexahedral caps, their largest sizes and those of
// the others.
struct ClassStats {
  int64_t cnt[4] = {0, 0, 0, 0};
  int64_t max[4][4] = {};
  int64_t hex_cnt = 0;
  int64_t hex_max[4] = {0, 0, 0, 0};
  int64_t rest_max[4] = {0, 0, 0, 0};
  void add(const int64_t sz[4]) {
    const int c = class_of(sz[0], sz[1], sz[2], sz[3]);
    ++cnt[c];
    for (int t = 0; t < 4; ++t) max[c][t] = max[c][t] > sz[t] ? max[c][t] : sz[t];
    if (c != 0) return;
    int64_t *m = fits_hex(sz[0], sz[1], sz[2], sz[3]) ? hex_max : rest_max;
    if (m == hex_max) ++hex_cnt;
    for (int t = 0; t < 4; ++t) m[t] = m[t] > sz[t] ? m[t] : sz[t];
  }
  void merge(const ClassStats &o) {
    for (int c = 0; c < 4; ++c) {
      cnt[c] += o.cnt[c];
      for (int t = 0; t < 4; ++t) max[c][t] = max[c][t] > o.max[c][t] ? max[c][t] : o.max[c][t];
    }
    hex_cnt += o.hex_cnt;
    for (int t = 0; t < 4; ++t) {
      hex_max[t] = hex_max[t] > o.hex_max[t] ? hex_max[t] : o.hex_max[t];
      rest_max[t] = rest_max[t] > o.rest_max[t] ? rest_max[t] : o.rest_max[t];
    }
  }
};

}  // namespace vofpc

struct vofpc_ctx_s {
  int device;
  hipStream_t stream;
  int n_cu;
  // claim counters of the reconstruction kernels' work queues, one set of
  // kQueueSet ints per class (the wavefront kernel's at 0, the group
  // kernel's one per XCD after it, kQueueStride ints apart); zero between
  // launches (each launch wraps them back), so calls on one context must not
  // overlap
  int *queue = nullptr;
  // second stream (default priority) for the class kernels that run beside
  // the main class of a bucketed launch, with the fork and join events
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  bool overlap_classes = true;   // use the second stream (vofpc_ctx_overlap_classes)
  // per-class kernel timing of the reconstruction (eager launches only):
  // an event pair around each class kernel of the latest call, and around
  // its bracket pass (learned form) when it has one
  bool time_classes = false;
  hipEvent_t cls_ev[vofpc::kClasses][2] = {};
  bool cls_rec[vofpc::kClasses] = {};
  hipEvent_t pass_ev[vofpc::kClasses][2] = {};
  bool pass_rec[vofpc::kClasses] = {};
};

struct vofpc_mesh_s {
  vofpc_ctx ctx;
  vofpc::DevMesh d;
  int64_t max_nf, max_nv, max_fv, max_ne, max_loop;
  // array lengths: cell_face, face_vert, cv_gid, cl_lv (loop positions), vc_cell
  int64_t ncf, nfv, ncv, ncl, nvc;
  int64_t bytes;
  // scratch for compaction (owned by the mesh; calls on one mesh must not
  // overlap in time)
  uint8_t *flags;
  uint8_t *cross;     // band marks of the face pass (zero between calls)
  int32_t *blk_cnt;   // [2][n_blocks]
  uint64_t *side;     // [2][ceil(n_cells / 64)]: the side of alpha = 1/2 of each cell as bits
  int64_t n_blk;
  // cells per kernel class; the class of the largest cell; bucketed meshes
  // (cells spread over several classes) launch one variant per class over
  // per-class entry lists [kClasses][n_cells] with device counts
  int64_t class_cells[vofpc::kClasses];
  // learned brackets [2][n_cells] of a bracket pass when the caller keeps
  // none (allocated by the first such call, outside capture)
  double *hint_buf = nullptr;
  int64_t class_max[vofpc::kClasses][4];   // largest vertices, faces, loop positions, edges per class
  vofpc::ClassStats class_stats;           // by class_of, before the hex0 move
  bool hex0;                               // class 0 holds only hexahedral-sized cells (mesh_class_of)
  int max_class;
  bool bucketed;
  int32_t *bucket_lists;
  int32_t *bucket_counts;
  // kernel flavour chosen per class (autotuned): 3 or 4 = one cell per
  // wavefront with the register budget of 3 or 4 waves per SIMD; 10 + G =
  // G lanes per cell (G = 1, 2, 4, 8)
  int tune[vofpc::kClasses];
  // smallest centre distance of two face neighbours (extrapolation step)
  double min_centre_dist;
  // gradient-extrapolation scratch, allocated by its first call (outside capture)
  int8_t *ex_mark = nullptr;       // layer of each cell in the domain (-1 outside)
  int32_t *ex_list = nullptr;      // domain cells (any order)
  int32_t *ex_info = nullptr;      // [1] domain size, [2] sweeps done, [3] unused, [4] converged
  double *ex_part = nullptr;       // [2][grid] per-block largest change of the last two sweeps
  double *ex_nrm = nullptr;        // [3][n_cells] advection direction
  double *ex_buf = nullptr;        // [2][n_cells][8]: G_l and G_v per cell, two iterates
  double *ex_wup = nullptr;        // per cell-face slot: normalised upwind weight
  double *ex_theta = nullptr;      // per domain entry: pseudo-time fraction
  int32_t *ex_upn = nullptr;       // per cell-face slot: neighbour of a packed upwind weight
  int2 *ex_upr = nullptr;          // per domain entry: first slot and count of its upwind weights
  // interface coupling: mixed entry of each cell (-1 between calls)
  int32_t *rb_entry = nullptr;
  // curvature scratch: [3][n_cells] (smoothing ping-pong, raw and step-1
  // curvature), the domain marks, list and length ([1])
  double *csf_buf = nullptr;
  int8_t *csf_mark = nullptr;
  int32_t *csf_list = nullptr;
  int32_t *csf_len = nullptr;
  double *csf_slot = nullptr;      // [2][slots]: geometric weight of the neighbour, face area
  // vertex-neighbour gradient stencil (built by its first use): CSR over cells
  int64_t *xn_off = nullptr;
  int32_t *xn_cell = nullptr;
  void *alloc[96];
  int n_alloc;
};

struct vofpc_graph_s {
  vofpc_ctx ctx;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

namespace vofpc {
// launchers (return VOFPC_OK or an error code with the message set)
vofpc_status launch_compact(vofpc_ctx ctx, vofpc_mesh m, const double *alpha, double eps, int32_t *mixed,
                            int32_t *band, int32_t *counts);
// mass transfer finished by the reconstruction (the whole step): the
// one-sided form of vofpc_mass_transfer over the mixed list
struct MdotFuse {
  const double *gradT;
  double k_l, k_v, h_lv;
  double *mdot, *Qdot;
};
// net (optional): bracket network run inside the reconstruction, with
// half-width factor delta; net_lo/net_hi (optional) receive its brackets;
// mf (optional): mass transfer of every entry from the finished gradient
vofpc_status launch_reconstruct(vofpc_ctx ctx, vofpc_mesh m, const double *alpha, const int32_t *mixed,
                                const int32_t *counts, const vofpc_recon_opts *o, const double *hlo,
                                const double *hhi, const vofpc_interface *out, vofpc_mlp net = nullptr,
                                double delta = 0.0, double *net_lo = nullptr, double *net_hi = nullptr,
                                const MdotFuse *mf = nullptr);
// device scratch owned by a mesh (freed with it)
vofpc_status mesh_scratch_alloc(vofpc_mesh M, size_t bytes, void **out);
// build the cell -> vertex-neighbour lists of a mesh (synchronous; no-op once built)
vofpc_status mesh_vertex_stencil(vofpc_mesh M);
// device parameters of a network: BF16 weights and FP32 master copy
const uint16_t *mlp_weights_bf16(vofpc_mlp M);
const float *mlp_params_f32(vofpc_mlp M);
int mlp_device(vofpc_mlp M);
// two band-scope gradients over one list in a single launch
vofpc_status launch_grad2(vofpc_ctx ctx, vofpc_mesh m, const int32_t *band, const int32_t *counts, const double *T1,
                          const double *Tb1, double T_sat1, const double *alpha1, int32_t variant1, double *grad1,
                          const double *T2, const double *Tb2, double T_sat2, const double *alpha2, int32_t variant2,
                          double *grad2);
vofpc_status launch_grad(vofpc_ctx ctx, vofpc_mesh m, const double *T, const double *Tb, double T_sat,
                         const double *alpha, const int32_t *band, const int32_t *counts, int32_t scope,
                         int32_t variant, double *grad, int32_t *status);
vofpc_status launch_features(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha, const int32_t *mixed,
                             const int32_t *counts, int64_t cap, const vofpc_recon_opts *o, float *feat,
                             double *prange);
vofpc_status launch_bracket(vofpc_ctx ctx, vofpc_mlp M, const float *feat, const double *prange,
                            const int32_t *counts, int64_t cap, double ksig, double *hlo, double *hhi);
vofpc_status launch_mass_transfer(vofpc_ctx ctx, vofpc_mesh m, const double *alpha, const int32_t *mixed,
                                  const int32_t *counts, const vofpc_interface *itf, const double *gradT,
                                  const double *gl, const double *gv, double k_l, double k_v, double h_lv,
                                  double *mdot, double *Qdot, double *mdot_c, double *Qdot_c);
}  // namespace vofpc
