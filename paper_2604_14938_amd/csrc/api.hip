// C entry points: contexts, errors, argument checks, the whole-step sequence
// and its HIP-graph capture.
#include <hip/hip_runtime.h>

#include <new>
#include <string>

#include "vofpc_internal.h"

namespace vofpc {
namespace {
thread_local std::string g_err;
}
void set_error(const std::string &msg) { g_err = msg; }
void clear_error() { g_err.clear(); }
}  // namespace vofpc

using namespace vofpc;

extern "C" const char *vofpc_last_error(void) { return g_err.c_str(); }

extern "C" int vofpc_version(void) { return 10000; }

extern "C" vofpc_status vofpc_ctx_create(int device, void *stream, vofpc_ctx *out) {
  clear_error();
  VOFPC_REQUIRE(out, VOFPC_E_INVALID_ARG, "ctx_create: null output");
  *out = nullptr;
  int n = 0;
  VOFPC_HIP(hipGetDeviceCount(&n));
  VOFPC_REQUIRE(device >= 0 && device < n, VOFPC_E_INVALID_ARG, "ctx_create: no such device");
  VOFPC_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  VOFPC_HIP(hipGetDeviceProperties(&prop, device));
  vofpc_ctx c = new (std::nothrow) vofpc_ctx_s();
  VOFPC_REQUIRE(c, VOFPC_E_OOM, "ctx_create: host allocation failed");
  c->device = device;
  c->stream = (hipStream_t)stream;
  c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  if (hipMalloc(&c->queue, kQueueInts * sizeof(int)) != hipSuccess) {
    delete c;
    set_error("ctx_create: hipMalloc of the work-queue counters failed");
    return VOFPC_E_OOM;
  }
  hipError_t e = hipMemset(c->queue, 0, kQueueInts * sizeof(int));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    if (c->side) (void)hipStreamDestroy(c->side);
    (void)hipFree(c->queue);
    delete c;
    set_error(std::string("ctx_create: ") + hipGetErrorString(e));
    return VOFPC_E_HIP;
  }
  *out = c;
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_ctx_set_stream(vofpc_ctx ctx, void *stream) {
  clear_error();
  VOFPC_REQUIRE(ctx, VOFPC_E_INVALID_ARG, "ctx_set_stream: null context");
  ctx->stream = (hipStream_t)stream;
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_ctx_destroy(vofpc_ctx ctx) {
  clear_error();
  if (ctx && ctx->queue) {
    (void)hipSetDevice(ctx->device);
    (void)hipFree(ctx->queue);
  }
  if (ctx) {
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
  }
  if (ctx && ctx->time_classes)
    for (int c = 0; c < vofpc::kClasses; ++c)
      for (int j = 0; j < 2; ++j) {
        (void)hipEventDestroy(ctx->cls_ev[c][j]);
        (void)hipEventDestroy(ctx->pass_ev[c][j]);
      }
  delete ctx;
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_recon_opts_default(vofpc_recon_opts *o) {
  clear_error();
  VOFPC_REQUIRE(o, VOFPC_E_INVALID_ARG, "recon_opts_default: null argument");
  o->eps_mixed = 1e-8;
  o->tol_rel = 1e-13;
  o->max_iter = 100;
  o->vertex_mode = VOFPC_VERTEX_IDW;
  o->fixed_iso = 0;
  o->bracket = VOFPC_BRACKET_PLAIN;
  o->iso = 0.5;
  o->phi_vertex = nullptr;
  return VOFPC_OK;
}

static vofpc_status check_pair(vofpc_ctx ctx, vofpc_mesh mesh) {
  VOFPC_REQUIRE(ctx && mesh, VOFPC_E_INVALID_ARG, "null context or mesh");
  VOFPC_REQUIRE(mesh->ctx && mesh->ctx->device == ctx->device, VOFPC_E_STATE,
                "mesh was uploaded on another device");
  VOFPC_HIP(hipSetDevice(ctx->device));
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_compact(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha, double eps,
                                      int32_t *mixed_idx, int32_t *band_idx, int32_t *counts) {
  clear_error();
  vofpc_status s = check_pair(ctx, mesh);
  if (s) return s;
  return launch_compact(ctx, mesh, alpha, eps, mixed_idx, band_idx, counts);
}

extern "C" vofpc_status vofpc_reconstruct(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha,
                                          const int32_t *mixed_idx, const int32_t *counts,
                                          const vofpc_recon_opts *opts, const double *hint_lo,
                                          const double *hint_hi, const vofpc_interface *out) {
  clear_error();
  vofpc_status s = check_pair(ctx, mesh);
  if (s) return s;
  return launch_reconstruct(ctx, mesh, alpha, mixed_idx, counts, opts, hint_lo, hint_hi, out);
}

extern "C" vofpc_status vofpc_reconstruct_learned(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha,
                                                  const int32_t *mixed_idx, const int32_t *counts,
                                                  const vofpc_recon_opts *opts, vofpc_mlp mlp, double delta_scale,
                                                  double *hint_lo, double *hint_hi, const vofpc_interface *out) {
  clear_error();
  vofpc_status s = check_pair(ctx, mesh);
  if (s) return s;
  VOFPC_REQUIRE(mlp, VOFPC_E_INVALID_ARG, "reconstruct_learned: null network");
  VOFPC_REQUIRE((hint_lo == nullptr) == (hint_hi == nullptr), VOFPC_E_INVALID_ARG,
                "reconstruct_learned: give both bracket outputs or neither");
  return launch_reconstruct(ctx, mesh, alpha, mixed_idx, counts, opts, nullptr, nullptr, out, mlp, delta_scale,
                            hint_lo, hint_hi);
}

extern "C" vofpc_status vofpc_grad_T(vofpc_ctx ctx, vofpc_mesh mesh, const double *T, const double *T_bface,
                                     double T_sat, const double *alpha, const int32_t *band_idx,
                                     const int32_t *counts, int32_t scope, int32_t variant, double *grad,
                                     int32_t *status) {
  clear_error();
  vofpc_status s = check_pair(ctx, mesh);
  if (s) return s;
  VOFPC_REQUIRE(T_bface, VOFPC_E_INVALID_ARG, "grad_T: null T_bface");
  if ((variant & VOFPC_GRAD_VERTEX_STENCIL) && !mesh->xn_off) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    VOFPC_HIP(hipStreamIsCapturing(ctx->stream, &cs));
    VOFPC_REQUIRE(cs == hipStreamCaptureStatusNone, VOFPC_E_STATE,
                  "grad_T: the first vertex-stencil call on a mesh builds its lists and must not be captured");
    s = mesh_vertex_stencil(mesh);
    if (s) return s;
  }
  return launch_grad(ctx, mesh, T, T_bface, T_sat, alpha, band_idx, counts, scope, variant, grad, status);
}

extern "C" vofpc_status vofpc_mass_transfer(vofpc_ctx ctx, vofpc_mesh mesh, const double *alpha,
                                            const int32_t *mixed_idx, const int32_t *counts,
                                            const vofpc_interface *itf, const double *gradT,
                                            const double *gradT_l, const double *gradT_v, double k_l,
                                            double k_v, double h_lv, double *mdot, double *Qdot,
                                            double *mdot_cells, double *Qdot_cells) {
  clear_error();
  vofpc_status s = check_pair(ctx, mesh);
  if (s) return s;
  return launch_mass_transfer(ctx, mesh, alpha, mixed_idx, counts, itf, gradT, gradT_l, gradT_v, k_l, k_v, h_lv,
                              mdot, Qdot, mdot_cells, Qdot_cells);
}

static vofpc_status issue_step(vofpc_ctx ctx, vofpc_mesh mesh, const vofpc_step_args *a) {
  VOFPC_REQUIRE(a, VOFPC_E_INVALID_ARG, "step: null arguments");
  VOFPC_REQUIRE(a->mdot && a->Qdot && a->gradT, VOFPC_E_INVALID_ARG, "step: null gradient or mass-transfer output");
  VOFPC_REQUIRE(a->h_lv != 0.0, VOFPC_E_INVALID_ARG, "step: h_lv must be nonzero");
  vofpc_status s = launch_compact(ctx, mesh, a->alpha, a->opts.eps_mixed, a->mixed_idx, a->band_idx, a->counts);
  if (s) return s;
  // the band gradient first (it needs only the lists), so the reconstruction
  // can finish every mixed cell with its mass transfer (Eq. mass_transfer)
  s = launch_grad(ctx, mesh, a->T, a->T_bface, a->T_sat, a->alpha, a->band_idx, a->counts, VOFPC_SCOPE_BAND,
                  VOFPC_GRAD_MODIFIED, a->gradT, a->grad_status);
  if (s) return s;
  MdotFuse mf{a->gradT, a->k_l, a->k_v, a->h_lv, a->mdot, a->Qdot};
  if (a->mlp) {
    // learned form: the network runs inside the reconstruction kernel
    VOFPC_REQUIRE(a->opts.bracket == VOFPC_BRACKET_PLAIN, VOFPC_E_INVALID_ARG,
                  "step: the learned form takes opts.bracket = VOFPC_BRACKET_PLAIN");
    VOFPC_REQUIRE((a->hint_lo == nullptr) == (a->hint_hi == nullptr), VOFPC_E_INVALID_ARG,
                  "step: give both hint_lo and hint_hi or neither");
    return launch_reconstruct(ctx, mesh, a->alpha, a->mixed_idx, a->counts, &a->opts, nullptr, nullptr, &a->itf,
                              a->mlp, a->delta_scale, a->hint_lo, a->hint_hi, &mf);
  }
  return launch_reconstruct(ctx, mesh, a->alpha, a->mixed_idx, a->counts, &a->opts, a->hint_lo, a->hint_hi, &a->itf,
                            nullptr, 0.0, nullptr, nullptr, &mf);
}

extern "C" vofpc_status vofpc_step(vofpc_ctx ctx, vofpc_mesh mesh, const vofpc_step_args *args) {
  clear_error();
  vofpc_status s = check_pair(ctx, mesh);
  if (s) return s;
  return issue_step(ctx, mesh, args);
}

extern "C" vofpc_status vofpc_graph_create(vofpc_ctx ctx, vofpc_mesh mesh, const vofpc_step_args *args,
                                           vofpc_graph *out) {
  clear_error();
  VOFPC_REQUIRE(out, VOFPC_E_INVALID_ARG, "graph_create: null output");
  *out = nullptr;
  vofpc_status s = check_pair(ctx, mesh);
  if (s) return s;
  VOFPC_REQUIRE(ctx->stream != nullptr, VOFPC_E_STATE, "graph_create: capture needs a non-null stream");
  hipGraph_t g = nullptr;
  VOFPC_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  s = issue_step(ctx, mesh, args);
  hipError_t e = hipStreamEndCapture(ctx->stream, &g);
  if (s) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) {
    set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    return VOFPC_E_HIP;
  }
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return VOFPC_E_HIP;
  }
  vofpc_graph G = new (std::nothrow) vofpc_graph_s();
  if (!G) {
    (void)hipGraphExecDestroy(x);
    (void)hipGraphDestroy(g);
    set_error("graph_create: host allocation failed");
    return VOFPC_E_OOM;
  }
  G->ctx = ctx;
  G->graph = g;
  G->exec = x;
  *out = G;
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_graph_launch(vofpc_graph g) {
  clear_error();
  VOFPC_REQUIRE(g, VOFPC_E_INVALID_ARG, "graph_launch: null graph");
  VOFPC_HIP(hipSetDevice(g->ctx->device));
  VOFPC_HIP(hipGraphLaunch(g->exec, g->ctx->stream));
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_graph_destroy(vofpc_graph g) {
  clear_error();
  if (!g) return VOFPC_OK;
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  delete g;
  return VOFPC_OK;
}
