// Declarations shared by the two reconstruction kernels: the wavefront
// kernel (one cell per wavefront, recon.hip) and the group kernel (G lanes
// per cell, recon_thin.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "vofpc_internal.h"
#include "wave_ops.h"

namespace vofpc {

// Order LDS traffic between the lanes of one wavefront (no hardware barrier:
// the groups of a wave run independent loops).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double det3(double a0, double a1, double a2, double b0, double b1, double b2, double c0,
                                       double c1, double c2) {
  return a0 * (b1 * c2 - b2 * c1) + a1 * (b2 * c0 - b0 * c2) + a2 * (b0 * c1 - b1 * c0);
}

struct CutRes {
  double V, S0, S1, S2, A, c0, c1, c2;
  int nch;
  bool err;
};

struct ReconParams {
  DevMesh m;
  const double *alpha;
  const int32_t *mixed;
  const int32_t *counts;
  const double *phi_override;
  const double *hint_lo, *hint_hi;
  double eps, tol_rel, iso;
  int max_iter, vertex_mode, fixed_iso, use_hint;
  int *queue;   // claim counters: the wavefront kernel's (cells beyond the first grid-size ones) at 0, then
                // one per XCD for the group kernel (kQueueStride ints apart)
  // optional entry list of this launch (a face-count bucket): entries[j] for
  // j < *entry_count instead of every mixed entry
  const int32_t *entries;
  const int32_t *entry_count;
  // bracket network run inside the kernel (null: none): BF16 weights, FP32
  // parameters, half-width factor, optional outputs of the bracket
  const uint16_t *net_wb;
  const float *net_master;
  double net_delta;
  double *net_lo, *net_hi;
  // mass transfer written with the interface (null gradT: not fused)
  MdotFuse mf;
  vofpc_interface out;
};

// The batches of a group-kernel launch in runs of kRun consecutive batches,
// run r to XCD r % kXcd: consecutive mixed entries are mostly neighbouring
// cells, which share vertices and faces, so a run is staged through one L2
// instead of being spread over all of them.  xcd_count: the batches of XCD
// x; xcd_batch: its i-th batch (runs in order, then batches within a run).
template <int kRun>
__device__ __forceinline__ int64_t xcd_count(int64_t nbatch, int x) {
  const int64_t nrun = nbatch / kRun, rem = nbatch % kRun;
  const int64_t full = nrun / kXcd + (x < nrun % kXcd ? 1 : 0);
  return full * kRun + (x == nrun % kXcd ? rem : 0);
}
template <int kRun>
__device__ __forceinline__ int64_t xcd_batch(int64_t i, int x) {
  return ((i / kRun) * kXcd + x) * kRun + i % kRun;
}
// cells per run
constexpr int kRunCells = 256;

// Spacing of the doubles above |x|: the bit patterns of non-negative
// doubles are ordered as their values, so the next double up is the pattern
// plus one (+inf gives NaN, as nextafter(inf, inf) - inf does).
__device__ __forceinline__ double ulp_of(double x) {
  const double a = fabs(x);
  return __longlong_as_double(__double_as_longlong(a) + 1) - a;
}

// The next double toward +inf (nextafter(x, +inf) for every x).
__device__ __forceinline__ double next_up(double x) {
  if (x == 0.0) return __longlong_as_double(1ll);   // either zero: the smallest subnormal
  if (!(x < __builtin_inf())) return x;              // +inf and NaN stay
  const long long b = __double_as_longlong(x);
  return __longlong_as_double(x > 0.0 ? b + 1 : b - 1);
}

// Root of the inverse quadratic through three (isovalue, residual) points;
// NaN or infinite when two residuals coincide.
__device__ __forceinline__ double iqi(double x0, double f0, double x1, double f1, double x2, double f2) {
  return x0 * f1 * f2 / ((f0 - f1) * (f0 - f2)) + x1 * f0 * f2 / ((f1 - f0) * (f1 - f2)) +
         x2 * f0 * f1 / ((f2 - f0) * (f2 - f1));
}

// A face of the cell as the bracket network sees it: the area vector
// oriented out of the cell and the neighbour's volume fraction.
struct NetFace {
  double S0, S1, S2, aQ;
  bool inner;
};

__device__ __forceinline__ NetFace load_net_face(const ReconParams &p, int P, double aP, int64_t slot) {
  const DevMesh &m = p.m;
  const int q = m.cf_nbr[slot];
  NetFace r;
  r.S0 = m.cf_S[3 * slot];
  r.S1 = m.cf_S[3 * slot + 1];
  r.S2 = m.cf_S[3 * slot + 2];
  r.inner = q >= 0;
  r.aQ = r.inner ? p.alpha[q] : aP;
  return r;
}

// Launch the group kernel with G lanes per cell on the entries of class c
// (the class's largest cell sizes in cmax = vertices, faces, loop positions,
// edges pick the LDS layout).  Returns VOFPC_E_INVALID_ARG when no build of
// the kernel holds that class.
vofpc_status launch_thin(vofpc_ctx ctx, const ReconParams &p, int64_t n_entries, int c, int G,
                         const int64_t cmax[4]);
// Whether launch_thin has a build for class c with these sizes and G.
bool thin_available(int c, int G, const int64_t cmax[4]);
// The learned brackets of the entries of class c (1 or 2) in a pass of their
// own: 16 cells per wavefront; writes hlo/hhi[k] per mixed entry k (NaN
// where the cell gets no network).  p carries the network and delta.
vofpc_status launch_bracket_pass(vofpc_ctx ctx, const ReconParams &p, int64_t n_entries, int c, double *hlo,
                                 double *hhi);

}  // namespace vofpc
