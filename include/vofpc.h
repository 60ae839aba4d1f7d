/* vofpc: interface hot path of a sharp-interface phase-change VOF method on
 * unstructured polyhedral meshes, for AMD Instinct MI355X (gfx950).
 *
 * The path, per time step (the method of Kren, Nicheno and Sato, 2026):
 *   1. compaction: the mixed cells (eps < alpha < 1-eps) and the gradient
 *      band (mixed cells and cells owning a face crossed by alpha = 1/2);
 *   2. reconstruction of every mixed cell: alpha is carried to the polyhedron
 *      vertices; the cell is cut by the iso-polygons of that vertex field
 *      (edge intersections by linear interpolation, Eq. edge_intersection,
 *      assembled through the faces into closed polygons, Sec. 2.1); the
 *      paper cuts at a fixed threshold, this library searches the isovalue
 *      until the liquid volume equals alpha V_P (its volume-matched reading
 *      of Sec. 2.1); the result is the interface normal n (vapour -> liquid),
 *      area A_int and centre-to-interface distance d;
 *   3. the interface-modified least-squares temperature gradient (Sec. 2.4.4,
 *      Eq. front_interpolation, App. B): across a face crossed by the
 *      interface the neighbour is replaced by the alpha-interpolated crossing
 *      point held at T_sat;
 *   4. the mass transfer rate mdot = (q_l + q_v)/(h_lv V_P) with
 *      q_l = k_l (grad T_l . n) A_int, q_v = -k_v (grad T_v . n) A_int
 *      (Eq. mass_transfer) and the latent source Qdot = -mdot h_lv
 *      (Eq. latent_source), only where A_int > 0.
 *
 * Conventions of the whole interface:
 *   - Every call returns a vofpc_status (0 = success, negative = error) and
 *     never throws across the boundary; vofpc_last_error() returns a
 *     thread-local message for the last failing call of the calling thread.
 *   - Compute calls are asynchronous on the context's HIP stream; their
 *     device outputs are valid once that stream has been synchronised.
 *   - "device" pointers are HIP device allocations of the context's device
 *     (for example torch tensor data pointers); "host" pointers are ordinary
 *     host memory.  The caller owns every field, list and output buffer; the
 *     library owns uploaded meshes, graphs and its own small scratch.
 *   - Floating point is FP64 throughout.  Vector fields are structure of
 *     arrays: a [3][n] array holds all x, then all y, then all z.
 *   - Per-cell numerical outcomes are reported as VOFPC_CELL_* codes in the
 *     status outputs, not as call errors.
 */
#ifndef VOFPC_H
#define VOFPC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- status codes */
typedef int vofpc_status;
#define VOFPC_OK 0
#define VOFPC_E_INVALID_ARG (-1) /* null or inconsistent argument */
#define VOFPC_E_HIP (-2)         /* a HIP runtime call failed */
#define VOFPC_E_OOM (-3)         /* device or host allocation failed */
#define VOFPC_E_MESH (-4)        /* mesh topology or geometry is invalid */
#define VOFPC_E_STATE (-5)       /* object used with the wrong context/device */

/* per-cell outcome codes (status outputs of reconstruct and grad_T) */
#define VOFPC_CELL_OK 0
#define VOFPC_CELL_NOT_MIXED 1        /* alpha <= eps or >= 1-eps: no interface */
#define VOFPC_CELL_LEARNED_FALLBACK 2 /* the narrowed bracket failed its check */
#define VOFPC_CELL_DEGENERATE 3       /* constant vertex field: linear alpha used */
#define VOFPC_CELL_MAX_ITER 4         /* the isovalue search stopped at max_iter evaluations */
#define VOFPC_CELL_G_SINGULAR 5       /* least-squares matrix singular: grad = 0 */
#define VOFPC_CELL_BAD_INPUT 6        /* alpha NaN or outside [0,1] */
#define VOFPC_CELL_NO_ROOT 7          /* liquid volume jumps across alpha V_P */

typedef struct vofpc_ctx_s *vofpc_ctx;
typedef struct vofpc_mesh_s *vofpc_mesh;
typedef struct vofpc_graph_s *vofpc_graph;
typedef struct vofpc_mlp_s *vofpc_mlp;

/* Thread-local message of the last failed call on this thread ("" if none).
 * The pointer stays valid until the next vofpc call on the same thread. */
const char *vofpc_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int vofpc_version(void);

/* ------------------------------------------------------------------ context */
/* Create a context on HIP device `device`, issuing work on `hip_stream` (a
 * hipStream_t; NULL = the device's null stream).  The stream must stay valid
 * while the context uses it.  The context also creates a second stream of
 * its own (default priority) that a bucketed reconstruction forks to and
 * joins back before returning (vofpc_ctx_overlap_classes), so synchronising
 * the context's stream still covers all of a call's work.  *out receives
 * the handle. */
vofpc_status vofpc_ctx_create(int device, void *hip_stream, vofpc_ctx *out);
/* Change the stream later work is issued on. */
vofpc_status vofpc_ctx_set_stream(vofpc_ctx ctx, void *hip_stream);
/* Destroy a context (after its meshes and graphs).  NULL is accepted. */
vofpc_status vofpc_ctx_destroy(vofpc_ctx ctx);

/* --------------------------------------------------------------------- mesh */
/* A polyhedral mesh in CSR form (finite-volume, cell-centred storage).  All
 * pointers are HOST pointers; the arrays are copied during the upload.
 *   cell_face_off[n_cells+1], cell_face[cell_face_off[n_cells]]: faces of
 *       each cell (each interior face appears in both of its cells);
 *   face_vert_off[n_faces+1], face_vert[...]: vertex loop of each face,
 *       counter-clockwise seen from outside its owner (right-hand normal
 *       points from owner to neighbour);
 *   face_owner[n_faces], face_neigh[n_faces] (-1 on the boundary);
 *   face_bc[n_faces]: 0 interior, 1 boundary with a given value (acts as a
 *       least-squares neighbour at the face centroid), 2 symmetry (skipped);
 *   vert_xyz[3][n_verts]: vertex coordinates.
 * Cells must be closed, convex polyhedra with planar faces; at most 255
 * vertices and 255 faces per cell. */
typedef struct {
  int64_t n_cells, n_faces, n_verts;
  const int64_t *cell_face_off;
  const int32_t *cell_face;
  const int64_t *face_vert_off;
  const int32_t *face_vert;
  const int32_t *face_owner;
  const int32_t *face_neigh;
  const int8_t *face_bc;
  const double *vert_xyz;
} vofpc_mesh_desc;

/* Validate and upload a mesh, then compute its geometry on the device: cell
 * volumes V and centroids x_P, face area vectors S_f and area centroids x_f,
 * the stored inverse least-squares matrix of every cell (six components of
 * the symmetric inverse, App. B) and the inverse-distance weights that carry
 * cell values to vertices.  Synchronises the context stream.  Returns
 * VOFPC_E_MESH for inconsistent topology, open or inverted cells. */
vofpc_status vofpc_mesh_upload(vofpc_ctx ctx, const vofpc_mesh_desc *desc, vofpc_mesh *out);
/* Disjoint union of n uploaded meshes (multi-instance batches, several
 * meshes in one step): cells, faces and vertices of mesh i follow those of
 * meshes 0..i-1 in order, ids and offsets shifted accordingly; geometry is
 * copied, not recomputed.  Fields over the union are the per-mesh fields laid
 * end to end (vector fields per component: [3][total]).  The inputs stay
 * valid and unchanged; all must live on the context's device.  Synchronises
 * the context stream.  Totals must fit in int32. */
vofpc_status vofpc_mesh_concat(vofpc_ctx ctx, const vofpc_mesh *meshes, int32_t n, vofpc_mesh *out);
/* Free a mesh and its device memory.  NULL is accepted. */
vofpc_status vofpc_mesh_free(vofpc_mesh mesh);
/* info[0..7] = n_cells, n_faces, n_verts, max faces per cell, max vertices
 * per cell, max vertices per face, max edges per cell, device bytes held. */
vofpc_status vofpc_mesh_info(vofpc_mesh mesh, int64_t info[8]);
/* Kernel classes of the mesh's cells (HOST outputs, any may be NULL): cells[c]
 * = number of cells whose size (vertices, faces, loop positions, edges) fits
 * class c = 0 (<= 16, 8, 48, 24: hexahedra and smaller), 1 (<= 32, 20, 96,
 * 48: the usual Voronoi cells), 2 (<= 48, 32, 128, 64) or 3 (larger), the
 * smallest that holds it; when all but at most 1 % of a mesh's class-0 cells
 * are within the hexahedral sizes (8, 6, 24, 12), the other class-0 cells
 * are counted in class 1 instead, so that class 0 runs the hexahedral
 * layout (a mixed hexahedral and Voronoi mesh); tune[c]
 * = the reconstruction kernel flavour used for class c (see
 * vofpc_mesh_set_tune); *bucketed = 1 when the cells spread over several
 * classes: then the reconstruction splits the mixed entries by class and
 * launches each class's kernel on its own entries (size buckets), else the
 * one class's kernel runs. */
vofpc_status vofpc_mesh_classes(vofpc_mesh mesh, int64_t cells[4], int32_t tune[4], int32_t *bucketed);
/* Reconstruction kernel flavours (tile shapes) per class:
 *   3, 4   one cell per wavefront (64 lanes over its loop positions), with
 *          the register budget of 3 or 4 waves per SIMD; 3 for every
 *          class, 4 for classes 0 to 2;
 *   10+G   a group of G lanes per cell (the lanes share the cell's edges and
 *          faces), 64/G cells per wavefront: G = 1, 2, 4 for class 0 when
 *          its cells are at most hexahedra (8 vertices, 6 faces), else
 *          G = 2, 4; G = 4, 8, 16 for classes 1 and 2.
 * The learned form runs the network inside the reconstruction for every
 * flavour.  Results of all flavours agree within the parity tolerances. */
#define VOFPC_FLAVOUR_WAVE3 3
#define VOFPC_FLAVOUR_WAVE4 4
#define VOFPC_FLAVOUR_GROUP(G) (10 + (G))
/* Set the flavour of every class (HOST tune[4]); classes without cells
 * accept any value.  VOFPC_E_INVALID_ARG (nothing changed) when a class with
 * cells is given a flavour that has no build for it. */
vofpc_status vofpc_mesh_set_tune(vofpc_mesh mesh, const int32_t tune[4]);
/* Class launches side by side (default on).  A bucketed reconstruction runs
 * the usual Voronoi class (1) and its bracket pass on the context's stream
 * and the other classes beside it on a second stream the context owns
 * (default priority), forked after the bucketing and joined before the call
 * returns, so one class's idle issue slots and tail are filled by another's
 * work.  With enable = 0 every class runs in turn on the context's stream
 * (then each class kernel's time is its own).  Results are the same either
 * way, bit for bit. */
vofpc_status vofpc_ctx_overlap_classes(vofpc_ctx ctx, int32_t enable);
/* Per-class kernel timing of the reconstruction (a measurement aid).  With
 * enable != 0, every later eager reconstruction on this context records a HIP
 * event pair around each class kernel it launches, on the stream the kernel
 * runs on, and around the class's bracket pass when the learned form runs
 * one (none while the stream is being captured); enable = 0 destroys the
 * events.
 * vofpc_ctx_class_ms waits for the latest call's events and writes to HOST
 * ms[8] the duration in milliseconds of each class kernel (ms[0..3]) and of
 * each bracket pass (ms[4..7]), -1 where none ran, then forgets them;
 * VOFPC_E_STATE when timing is off. */
vofpc_status vofpc_ctx_time_classes(vofpc_ctx ctx, int32_t enable);
vofpc_status vofpc_ctx_class_ms(vofpc_ctx ctx, float ms[8]);
/* Copy the computed geometry into caller DEVICE buffers (any may be NULL):
 * V[n_cells], xc[3][n_cells], Sf[3][n_faces], xf[3][n_faces]. */
vofpc_status vofpc_mesh_geometry(vofpc_mesh mesh, double *V, double *xc, double *Sf, double *xf);

/* ------------------------------------------------------------- compaction */
/* Mixed-cell list M (cells with eps_mixed < alpha < 1-eps_mixed, ascending)
 * and band list B (cells that are mixed or own a face with
 * (alpha_P - 1/2)(alpha_Q - 1/2) < 0, ascending): the crossing test of the
 * interface-modified gradient (Sec. 2.4.4) marks the cells whose gradient
 * changes, and with the mixed cells it gives the one-to-two-cell band where
 * the latent source lives (Eq. latent_source).  alpha: DEVICE [n_cells].
 * mixed_idx and band_idx: DEVICE int32 [n_cells] (capacity n_cells);
 * counts: DEVICE int32 [2] receives |M| and |B|.  No host readback. */
vofpc_status vofpc_compact(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha, double eps_mixed,
                           int32_t *mixed_idx, int32_t *band_idx, int32_t *counts);
/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): vofpc_compact with
 * the same arguments and results, its scratch (per-cell flag and band-mark
 * bytes, per-block totals, per-cell side bits) taken from a fixed array the
 * library holds on each GPU until the process ends (about 19 MB) instead of
 * the mesh's; it
 * allocates nothing.  Meshes of at most 8,388,608 cells; larger ones give
 * VOFPC_E_INVALID_ARG.  Every call on one GPU shares that array: calls that
 * overlap in time on one GPU (other streams, other threads) race and give
 * undefined lists. */
vofpc_status vofpc_compact_noalloc(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha, double eps_mixed,
                                   int32_t *mixed_idx, int32_t *band_idx, int32_t *counts);

/* --------------------------------------------------------- reconstruction */
#define VOFPC_BRACKET_PLAIN 0   /* search [phi_min, phi_max] of the cell */
#define VOFPC_BRACKET_HINT 1    /* first guess from hint_lo/hint_hi (see vofpc_reconstruct) */
#define VOFPC_VERTEX_IDW 0      /* vertex value: inverse-distance cell average */
#define VOFPC_VERTEX_MEAN 1     /* vertex value: plain average of the cells */

typedef struct {
  double eps_mixed;   /* mixed when eps < alpha < 1-eps (default 1e-8) */
  double tol_rel;     /* stop when |V/V_P - alpha| <= tol_rel min(alpha,1-alpha) (1e-13) */
  int32_t max_iter;   /* volume evaluations per cell before VOFPC_CELL_MAX_ITER (100) */
  int32_t vertex_mode;/* VOFPC_VERTEX_* */
  int32_t fixed_iso;  /* nonzero: no root-find, cut at `iso` (paper's isoap mode) */
  int32_t bracket;    /* VOFPC_BRACKET_* */
  double iso;         /* isovalue for fixed_iso (0.5) */
  const double *phi_vertex; /* optional DEVICE [n_verts] vertex field override */
} vofpc_recon_opts;

/* Fill *opts with the defaults above. */
vofpc_status vofpc_recon_opts_default(vofpc_recon_opts *opts);

/* Interface record over the mixed list: entry k describes cell mixed_idx[k]
 * (k < counts[0]).  All pointers are DEVICE arrays of `cap` entries (n is
 * [3][cap]); cap must be >= the number of mixed cells (n_cells is always
 * enough).  Entries k >= counts[0] are left untouched. */
typedef struct {
  double *s;          /* isovalue found (NaN when no interface) */
  double *n;          /* [3][cap] unit normal, vapour -> liquid (0 when none) */
  double *A;          /* interface area A_int (0 when none) */
  double *d;          /* n . (x_P - c_int), positive when x_P is in the liquid */
  double *alpha_got;  /* V_liq(s)/V_P */
  int32_t *status;    /* VOFPC_CELL_* */
  int32_t *iters;     /* volume evaluations spent */
  int64_t cap;
} vofpc_interface;

/* Reconstruct the interface in every listed mixed cell.  The cut is the
 * paper's iso-surface of a vertex field (Sec. 2.1: edge intersections by
 * Eq. edge_intersection, assembled through the faces into iso-polygons);
 * the paper takes a fixed threshold, while this library moves the isovalue
 * until the cut liquid volume (divergence theorem) matches alpha V_P, its
 * volume-matched reading of Sec. 2.1.  alpha: DEVICE [n_cells]; mixed_idx/counts from
 * vofpc_compact.
 * The isovalue search keeps a bracket [lo, hi] of [phi_min, phi_max] with
 * V(lo) > alpha V_P > V(hi) and stops at the first isovalue whose residual
 * |V/V_P - alpha| is within tol_rel min(alpha, 1-alpha); when the bracket
 * shrinks to two ulps first, the end nearer to alpha V_P is taken
 * (VOFPC_CELL_NO_ROOT when its residual exceeds 1e-10).  Guesses come from
 * regula falsi / inverse quadratic interpolation with bisection safeguards;
 * between two breakpoints of the cut topology several guesses are evaluated
 * at once.  Any isovalue in the stopping window is a valid result; the
 * oracle's bisection may stop at another one of the same window.
 * hint_lo/hint_hi: DEVICE [cap] per mixed entry, read only when
 * opts->bracket is VOFPC_BRACKET_HINT (NaN entries: plain search, no flag):
 * the bracket, clipped to [phi_min, phi_max], is checked with two cuts, at
 * its centre and at its end on the side of the root that the centre's
 * residual gives.  When that end is past the root the search goes on in
 * the half between them; otherwise it goes on beyond that end and the cell
 * is flagged VOFPC_CELL_LEARNED_FALLBACK.  The flag therefore marks exactly
 * the cells whose root lies outside the clipped bracket (V(s) decreasing),
 * as a cut at both ends would. */
vofpc_status vofpc_reconstruct(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha, const int32_t *mixed_idx,
                               const int32_t *counts, const vofpc_recon_opts *opts, const double *hint_lo,
                               const double *hint_hi, const vofpc_interface *out);

/* Reconstruction with the bracket network run inside the same kernel: each
 * mixed cell's 32 inputs (as vofpc_features defines them) and the forward
 * pass (BF16 MFMA tiles of 16 cells in the group flavours, one FP32 row per
 * wavefront in the wavefront flavours) give the predicted isovalue
 * phi_min + clamp(u,0,1) W and the bracket around it of half-width
 * delta_scale W, checked as with VOFPC_BRACKET_HINT with the first cut at the
 * predicted isovalue.  opts->bracket must be
 * VOFPC_BRACKET_PLAIN.  hint_lo/hint_hi: optional DEVICE double[cap]
 * receiving the network's brackets (both or neither; NaN where the network
 * gives none).  Cells whose vertex field is degenerate skip the network. */
vofpc_status vofpc_reconstruct_learned(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha,
                                       const int32_t *mixed_idx, const int32_t *counts,
                                       const vofpc_recon_opts *opts, vofpc_mlp mlp, double delta_scale,
                                       double *hint_lo, double *hint_hi, const vofpc_interface *out);

/* Autotune the reconstruction of a mesh: for each class with cells and more
 * than one flavour (see vofpc_mesh_set_tune: lanes per cell and register
 * budget), time every flavour on the mixed cells of `alpha` (DEVICE
 * [n_cells]; opts may be NULL) and keep the fastest in the mesh.
 * cache_path (optional, a text file): a line for the same device, CU count,
 * mesh sizes, class counts and options is used without timing
 * (*from_cache = 1); otherwise the choice is appended.  choice: optional
 * HOST int32[4] receiving the flavour per class.  On error the mesh keeps
 * the flavours it had.  Allocates trial buffers and synchronises the context
 * stream (a set-up call, not for capture). */
vofpc_status vofpc_autotune(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha, const vofpc_recon_opts *opts,
                            const char *cache_path, int32_t *choice, int32_t *from_cache);

/* ----------------------------------------------------------------- gradient */
#define VOFPC_SCOPE_BAND 0  /* write grad at band cells only (others untouched) */
#define VOFPC_SCOPE_ALL 1   /* write grad at every cell */
#define VOFPC_GRAD_MODIFIED 0 /* interface-modified stencil (Sec. 2.4.4) */
#define VOFPC_GRAD_STANDARD 1 /* plain least squares, no modification */
#define VOFPC_GRAD_PRINTED 2  /* modified, with the printed mirror weight |a_Q-1/2|/|a_P-a_Q| */
/* Flags or-ed into the variant (App. B, "Weighting" and "Neighbour stencil";
 * the paper runs with neither): the fit minimises sum w (dT - g.r)^2 with
 * w = 1/|r| or 1/|r|^2 of the (possibly shortened) displacement r, and the
 * vertex stencil takes every cell sharing a vertex with P in place of the
 * face neighbours (crossing test and shortening apply to each connection). */
#define VOFPC_GRAD_W_INV_DIST 0x10
#define VOFPC_GRAD_W_INV_DIST2 0x20
#define VOFPC_GRAD_VERTEX_STENCIL 0x40

/* Interface-modified least-squares gradient of T (App. B with Sec. 2.4.4).
 * T: DEVICE [n_cells]; T_bface: DEVICE [n_faces] (values used on faces with
 * face_bc == 1); alpha: DEVICE [n_cells]; band_idx/counts from
 * vofpc_compact (ignored for VOFPC_SCOPE_ALL).  Band cells build their
 * least-squares matrix on the fly; other cells use the stored inverse (plain
 * variants without flags only; with a flag every cell builds its own).
 * variant: VOFPC_GRAD_MODIFIED/STANDARD/PRINTED, optionally or-ed with one
 * weight flag and VOFPC_GRAD_VERTEX_STENCIL; anything else is
 * VOFPC_E_INVALID_ARG.  The first call with the vertex stencil on a mesh
 * builds its cell -> vertex-neighbour lists (mesh-owned, about 4 B per
 * neighbour; host work plus a copy) and must not be captured.
 * grad: DEVICE [3][n_cells]; status: optional DEVICE int32 [n_cells]
 * (VOFPC_CELL_OK or VOFPC_CELL_G_SINGULAR, written where grad is written). */
vofpc_status vofpc_grad_T(vofpc_ctx ctx, vofpc_mesh mesh, const double *T, const double *T_bface, double T_sat,
                          const double *alpha, const int32_t *band_idx, const int32_t *counts, int32_t scope,
                          int32_t variant, double *grad, int32_t *status);

/* ------------------------------------------------------------ mass transfer */
/* mdot and Qdot for every mixed entry k (Eq. mass_transfer, Eq. latent_source):
 * zero where A_int = 0.  gradT: DEVICE [3][n_cells].  gradT_l/gradT_v:
 * optional DEVICE [3][n_cells] phase gradients; when both are NULL the cell's
 * own phase (liquid when alpha >= 1/2) takes gradT and the other phase 0.
 * mdot/Qdot: DEVICE [cap] over the mixed list.  mdot_cells/Qdot_cells:
 * optional DEVICE [n_cells] dense fields, zero-filled then scattered. */
vofpc_status vofpc_mass_transfer(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha, const int32_t *mixed_idx,
                                 const int32_t *counts, const vofpc_interface *itf, const double *gradT,
                                 const double *gradT_l, const double *gradT_v, double k_l, double k_v,
                                 double h_lv, double *mdot, double *Qdot, double *mdot_cells,
                                 double *Qdot_cells);

/* ---------------------------------------------------- phase gradients */
typedef struct {
  double eps_mixed;  /* mixed cells seed the domain (1e-8) */
  int32_t layers;    /* rings of interior face neighbours around them (2) */
  int32_t max_iter;  /* pseudo-time sweeps at most (120) */
  double tol;        /* stop when the largest change of a sweep is below this (1e-3, units of grad T) */
} vofpc_extrap_opts;

/* Fill *opts with the defaults above. */
vofpc_status vofpc_extrap_opts_default(vofpc_extrap_opts *opts);

/* Liquid- and vapour-side temperature gradients at the interface by
 * pseudo-time extrapolation (Eq. extrapolation, Sec. 2.4.4), for the
 * two-sided mass transfer of Eq. mass_transfer (pass them to
 * vofpc_mass_transfer as gradT_l, gradT_v).  On the domain D (mixed cells and
 * opts->layers rings of interior face neighbours) both fields start from the
 * interface-modified gradient of T (computed here); a liquid cell (alpha >=
 * 1/2) keeps gradT_l and advances gradT_v, a vapour cell the reverse, with
 * velocity sgn(alpha - 1/2) n (the interface normal of itf where A > 0, else
 * the unit plain least-squares gradient of alpha over interior neighbours),
 * first-order upwind over the faces to D neighbours, pseudo-time step the
 * smallest centre distance of two face neighbours with the local Courant
 * number clipped at 1, Jacobi sweeps until the largest change falls below
 * opts->tol or opts->max_iter sweeps.
 * alpha, T: DEVICE [n_cells]; T_bface: DEVICE [n_faces]; mixed_idx, counts,
 * itf: the compaction and reconstruction of this alpha; opts may be NULL.
 * gradT_l, gradT_v: DEVICE [3][n_cells], written on D only.  report:
 * optional DEVICE int32[2] = (sweeps done, 0).  Each sweep is one kernel;
 * after convergence the remaining sweep kernels return at once
 * (opts->max_iter kernels are always issued, so a captured graph holds them
 * all; an idle one costs about 1.6 microseconds).  The first
 * call on a mesh allocates its scratch (mesh-owned) and must not be captured;
 * later calls are graph-capturable.  Calls on one mesh must not overlap. */
vofpc_status vofpc_extrapolate(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha, const double *T,
                               const double *T_bface, double T_sat, const int32_t *mixed_idx,
                               const int32_t *counts, const vofpc_interface *itf, const vofpc_extrap_opts *opts,
                               double *gradT_l, double *gradT_v, int32_t *report);

/* ------------------------------------------ interface coupling coefficients */
/* Coefficients of the implicit interface condition of the energy equation
 * (Eq. interface_htc, Sec. 2.4.4 "Heat source/sink").  An interior face f
 * whose cells P (owner) and Q satisfy (alpha_P - 1/2)(alpha_Q - 1/2) < 0 is
 * detached: its diffusive coupling is dropped and each of its cells C is tied
 * to T_sat with a_f,C = k_C A_int,f / d_f,C, added to C's diagonal with
 * a_f,C T_sat on the right-hand side.  Readings: k_C = k_l when alpha_C >= 1/2,
 * else k_v; x_f = x_P + t (x_Q - x_P), t = (alpha_P - 1/2)/(alpha_P - alpha_Q)
 * (the crossing point of the gradient stencil, Eq. front_interpolation);
 * d_f,C = |nf . (x_f - x_C)| with nf the unit face normal; A_int,f =
 * |nf . (A_P n_P + A_Q n_Q)|, the face-normal projection of the interface area
 * vectors of the two cells (zero for a cell that is not in the mixed list).
 * A side with d = 0 (a centre connection parallel to the face) gets a = 0.
 *
 * mixed_idx, band_idx, counts: the lists of vofpc_compact (cells must be
 * valid ids); itf: the reconstruction of the mixed list (entry k <-> cell
 * mixed_idx[k]; A and n are read).  Outputs (DEVICE, caller-owned, each
 * optional):
 *   a_diag     [n_band] compact over the band list: entry k holds the sum of
 *              a_f,C over the detached faces of C = band_idx[k] (0 if none);
 *   face_idx   [face_cap] detached faces, in no particular order;
 *   face_a     [2][face_cap] a_f on the owner side, then on the neighbour side;
 *   face_d     [2][face_cap] d_f on the owner side, then the neighbour side;
 *   face_area  [face_cap] A_int,f;
 *   n_face     int32[1]: the number of detached faces (required when any face
 *              output is given); records beyond face_cap are not written, so
 *              n_face > face_cap means the capacity was too small.
 * The first call on a mesh allocates a mesh-owned map (4 B per cell) and must
 * not be captured; later calls are graph-capturable.  Calls on one mesh must
 * not overlap. */
vofpc_status vofpc_robin(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha, const int32_t *mixed_idx,
                         const int32_t *band_idx, const int32_t *counts, const vofpc_interface *itf, double k_l,
                         double k_v, double *a_diag, int64_t face_cap, int32_t *face_idx, double *face_a,
                         double *face_d, double *face_area, int32_t *n_face);

/* ------------------------------------------------- surface-tension curvature */
/* Curvature of the continuum-surface-force term (Sec. 2.4, momentum terms,
 * surface tension), over every cell:
 *   alpha_hat: n_smooth Jacobi sweeps of the face-area-weighted average of
 *     face values alpha_P + w_f (alpha_Q - alpha_P), w_f the geometric weight
 *     of Q (the fraction of the centre connection P->Q at the face plane),
 *     alpha_P on boundary faces;
 *   n = grad(alpha_hat) / (|grad(alpha_hat)| + 1e-15), the plain least-squares
 *     gradient over interior face neighbours (App. B), vapour -> liquid;
 *   kappa_raw = -div n by the Gauss sum with n_f = n_P + w_f (n_Q - n_P)
 *     (n_P on boundary faces);
 *   kappa* = (k~_P w_P + sum_Q k~_Q w_Q) / (w_P + sum_Q w_Q + 1e-15) over the
 *     face neighbours, w = (1 - 2|1/2 - alpha_hat|)^8;
 *   kappa = (k*_P w_P + sum_Q k*_Q w_Q wn_Q) / (w_P + sum_Q w_Q wn_Q + 1e-15),
 *     wn_Q = |n_P . s_Q|^8, s_Q the unit centre connection (the 1e-15 is
 *     added here too so that pure cells give 0);
 *   force = sigma kappa grad(alpha), the plain gradient of the sharp alpha.
 * A droplet (liquid inside) has positive curvature.
 * alpha: DEVICE [n_cells].  Outputs (DEVICE, caller-owned): alpha_hat [n_cells],
 * n [3][n_cells], kappa [n_cells] required; kappa_raw [n_cells] and force
 * [3][n_cells] optional (NULL skips; without force the gradient of alpha is
 * not computed).  opts NULL: defaults.  The first call on a mesh allocates
 * its scratch (about 29 B per cell plus a table of 16 B per cell-face slot,
 * the neighbour weights and face areas, mesh-owned) and must not be
 * captured; later calls are graph-capturable.  Calls on one mesh must not
 * overlap. */
typedef struct {
  int32_t n_smooth;  /* smoothing sweeps of alpha (2) */
  double sigma;      /* surface tension coefficient for the force (1.0) */
} vofpc_csf_opts;

vofpc_status vofpc_csf_opts_default(vofpc_csf_opts *opts);
vofpc_status vofpc_curvature(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha, const vofpc_csf_opts *opts,
                             double *alpha_hat, double *n, double *kappa_raw, double *kappa, double *force);

/* ---------------------------------------------------------- bracket network */
/* A small network predicts the isovalue of every mixed cell; the
 * reconstruction takes it as the first guess of its bracketed search, whose
 * stopping rule alone decides the result, so the network changes only how
 * many volume evaluations a cell needs.  Architecture: 32 features -> 64 -> 64 -> 4 (tanh hidden layers),
 * BF16 weights and activations on MFMA with FP32 accumulation, FP32 master
 * weights updated by Adam.  Outputs per cell: u, the isovalue normalised to
 * the cell's vertex-value range, (s - phi_min)/(phi_max - phi_min), and a
 * 3-vector for the interface normal.  Loss: mean (u-u*)^2 + 0.1 mean|n-n*|^2.
 * Parameters are one FP32 vector in the order W1[64][32], b1[64],
 * W2[64][64], b2[64], W3[4][64], b3[4]. */

/* Number of network parameters (6532). */
int vofpc_mlp_param_count(void);
/* Create a network on the context's device; `max_batch` bounds the rows of
 * one training call (it sizes the gradient workspace).  Weights start at 0. */
vofpc_status vofpc_mlp_create(vofpc_ctx ctx, int64_t max_batch, vofpc_mlp *out);
/* Destroy a network.  NULL is accepted. */
vofpc_status vofpc_mlp_destroy(vofpc_mlp mlp);
/* Copy all parameters from HOST float[n] (n = vofpc_mlp_param_count()) and
 * reset the Adam state.  Synchronises the context stream. */
vofpc_status vofpc_mlp_set_params(vofpc_mlp mlp, const float *host, int64_t n);
/* Copy the FP32 master parameters to HOST float[n].  Synchronises. */
vofpc_status vofpc_mlp_get_params(vofpc_mlp mlp, float *host, int64_t n);
/* Forward pass: X DEVICE float[n][32] -> Y DEVICE float[n][4]. */
vofpc_status vofpc_mlp_forward(vofpc_ctx ctx, vofpc_mlp mlp, const float *X, int64_t n, float *Y);
/* Loss and gradient of the mean loss over n rows of X with targets T DEVICE
 * float[n][4] (u*, n*): grad DEVICE float[param_count], loss DEVICE float[1]
 * (either may be NULL).  Deterministic (fixed-order reduction). */
vofpc_status vofpc_mlp_gradient(vofpc_ctx ctx, vofpc_mlp mlp, const float *X, const float *T, int64_t n,
                                float *grad, float *loss);
/* One Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8) on the gradient of
 * n rows; loss DEVICE float[1] receives the pre-step loss (may be NULL). */
vofpc_status vofpc_mlp_train_step(vofpc_ctx ctx, vofpc_mlp mlp, const float *X, const float *T, int64_t n,
                                  float lr, float *loss);
/* Network inputs of every listed mixed cell (entry k = cell mixed_idx[k]):
 * features DEVICE float[cap][32], phi_range DEVICE double[cap][2] =
 * (phi_min, phi_max - phi_min) of the cell's vertex field (the vertex rule of
 * opts, which may be NULL for the defaults).  Definitions: 0 alpha_P; 1-7
 * vertex-value quantiles q = 1/8..7/8 normalised to the range; 8 normalised
 * mean; 9 range; 10-12 sum A_f (alpha_Q-alpha_P) n_f / sum A_f; 13-18 the
 * same with n_f n_f^T (xx yy zz xy xz yz); 19-24 sum A_f n_f n_f^T / sum A_f;
 * 25 faces/32; 26-28 mean, min, max of the neighbours' alpha; 29-31 zero. */
vofpc_status vofpc_features(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha, const int32_t *mixed_idx,
                            const int32_t *counts, const vofpc_recon_opts *opts, float *features,
                            double *phi_range, int64_t cap);
/* Narrowed brackets from the network: hint = phi_min + clamp(u,0,1) W +- delta
 * with delta = delta_scale W (DEVICE double[cap] each; NaN where W = 0). */
vofpc_status vofpc_mlp_bracket(vofpc_ctx ctx, vofpc_mlp mlp, const float *features, const double *phi_range,
                               const int32_t *counts, int64_t cap, double delta_scale, double *hint_lo,
                               double *hint_hi);

/* ------------------------------------------------------------- whole step */
/* Every buffer of one step: compaction, reconstruction, band gradient and
 * mass transfer, with the meaning given above.  All pointers DEVICE. */
typedef struct {
  const double *alpha, *T, *T_bface;
  double T_sat, k_l, k_v, h_lv;
  vofpc_recon_opts opts;
  double *hint_lo, *hint_hi; /* read with opts.bracket == VOFPC_BRACKET_HINT; with mlp set:
                              * optional outputs of the network's brackets */
  int32_t *mixed_idx, *band_idx, *counts;
  vofpc_interface itf;
  double *gradT;          /* [3][n_cells], written on the band */
  int32_t *grad_status;   /* optional [n_cells] */
  double *mdot, *Qdot;    /* [cap] over the mixed list */
  /* learned form: with mlp set, the reconstruction runs the network inside
   * its kernel (vofpc_reconstruct_learned with delta_scale) */
  vofpc_mlp mlp;
  double delta_scale;
} vofpc_step_args;

/* Issue one step on the context stream. */
vofpc_status vofpc_step(vofpc_ctx ctx, vofpc_mesh mesh, const vofpc_step_args *args);

/* Capture one step (with the buffers of *args) into a HIP graph on the
 * context stream; replaying it re-runs the step on whatever the buffers hold
 * at replay time.  The mixed and band counts stay on the device, so the
 * graph needs no host readback. */
vofpc_status vofpc_graph_create(vofpc_ctx ctx, vofpc_mesh mesh, const vofpc_step_args *args, vofpc_graph *out);
/* Launch a captured step on the context stream. */
vofpc_status vofpc_graph_launch(vofpc_graph g);
/* Destroy a captured step.  NULL is accepted. */
vofpc_status vofpc_graph_destroy(vofpc_graph g);

#ifdef __cplusplus
}
#endif
#endif /* VOFPC_H */
