// Volume-matched iso-polygon reconstruction of the mixed cells.
//
// One cell per group of W lanes (W divides 64; a block is one wavefront, so a
// block holds 64/W cells).  The cell's polyhedron is staged in LDS: vertex
// positions relative to the centroid, the vertex field, the outward face
// loops as local vertex ids.  A volume evaluation at isovalue s spreads the
// faces over the lanes:
//   - each face lane walks its loop: liquid edges and the liquid parts of the
//     cut edges add to the divergence-theorem sum; exits (liquid -> vapour)
//     and entries (vapour -> liquid) are kept as bit masks over loop
//     positions; each exit is paired with an entry (the next one in loop
//     order when the face-mean value is >= s or the face has two crossings,
//     else the previous one), giving a chord exit -> entry that closes the
//     face's liquid polygon;
//   - chords are linked into iso-loops (the loop continues in the face whose
//     entry edge is this chord's exit edge) and labelled by pointer jumping;
//   - each loop is fanned from its length-weighted polyline centroid, which
//     adds its volume share, its area vector and its centre.
// Crossing points follow Eq. edge_intersection, computed from the liquid end
// of the edge so both faces sharing an edge get the same point.
//
// The isovalue is bisected until |V/V_P - alpha| <= tol_rel min(alpha,1-alpha);
// when the bracket collapses first, the end nearer to alpha V_P is kept.
#include <hip/hip_runtime.h>

#include "vofpc_internal.h"

namespace vofpc {

// Order LDS traffic between the lanes of one wavefront (no hardware barrier:
// the groups of a wave run independent loops).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int W>
__device__ __forceinline__ double gsum(double v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}
template <int W>
__device__ __forceinline__ int gmin_i(int v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, W));
  return v;
}
template <int W>
__device__ __forceinline__ int gsum_i(int v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}
template <int W>
__device__ __forceinline__ double gmin(double v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, W));
  return v;
}
template <int W>
__device__ __forceinline__ double gmax(double v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, W));
  return v;
}
// exclusive prefix sum over the group
template <int W>
__device__ __forceinline__ int gscan_excl(int v, int lane) {
  int inc = v;
#pragma unroll
  for (int d = 1; d < W; d <<= 1) {
    int t = __shfl_up(inc, d, W);
    if (lane >= d) inc += t;
  }
  return inc - v;
}

__device__ __forceinline__ double det3(double a0, double a1, double a2, double b0, double b1, double b2, double c0,
                                       double c1, double c2) {
  return a0 * (b1 * c2 - b2 * c1) + a1 * (b2 * c0 - b0 * c2) + a2 * (b0 * c1 - b1 * c0);
}

template <int NV, int NF, int NL, int NCH>
struct GroupMem {
  double X[3][NV];
  double phi[NV];
  double cf[3][NF];
  double fmean[NF];
  double ps[3][NCH];
  uint16_t floff[NF];
  uint16_t xkey[NCH];
  uint16_t nkey[NCH];
  uint16_t nxt[NCH];
  uint16_t lab[2][NCH];
  uint16_t jmp[2][NCH];
  uint8_t fsz[NF];
  uint8_t lv[NL];
};

struct CutRes {
  double V, S0, S1, S2, A, c0, c1, c2;
  int nloops;
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
  vofpc_interface out;
};

// crossing point of the edge (a, b) at isovalue s, from its liquid end
template <class GM>
__device__ __forceinline__ void crossing(const GM &L, int a, int b, double s, double &p0, double &p1, double &p2) {
  int i = (L.phi[a] >= s) ? a : b;
  int j = (i == a) ? b : a;
  double lam = (s - L.phi[i]) / (L.phi[j] - L.phi[i]);
  p0 = L.X[0][i] + lam * (L.X[0][j] - L.X[0][i]);
  p1 = L.X[1][i] + lam * (L.X[1][j] - L.X[1][i]);
  p2 = L.X[2][i] + lam * (L.X[2][j] - L.X[2][i]);
}

__device__ __forceinline__ int next_bit_after(uint64_t mask, int q) {
  uint64_t hi = (q >= 63) ? 0ull : (mask & (~0ull << (q + 1)));
  return hi ? __ffsll((long long)hi) - 1 : __ffsll((long long)mask) - 1;
}
__device__ __forceinline__ int prev_bit_before(uint64_t mask, int q) {
  uint64_t lo = (q == 0) ? 0ull : (mask & (~0ull >> (64 - q)));
  return lo ? 63 - __clzll((long long)lo) : 63 - __clzll((long long)mask);
}

// One volume evaluation of the staged cell at isovalue s.
template <int W, int NV, int NF, int NL, int NCH>
__device__ CutRes cut_eval(GroupMem<NV, NF, NL, NCH> &L, int lane, int nf, double s) {
  CutRes R;
  R.err = false;
  double vf = 0.0;
  int nch = 0;
  bool err = false;
  // ---- faces: liquid parts and chords
  for (int base = 0; base < nf; base += W) {
    const int f = base + lane;
    uint64_t ex = 0, en = 0;
    int m = 0, o = 0;
    double c0 = 0, c1 = 0, c2 = 0;
    if (f < nf) {
      m = L.fsz[f];
      o = L.floff[f];
      c0 = L.cf[0][f]; c1 = L.cf[1][f]; c2 = L.cf[2][f];
      if (m > 64) err = true;
      int a = L.lv[o];
      bool la = L.phi[a] >= s;
      for (int k = 0; k < m && k < 64; ++k) {
        int b = L.lv[o + (k + 1 == m ? 0 : k + 1)];
        bool lb = L.phi[b] >= s;
        if (la && lb) {
          vf += det3(c0, c1, c2, L.X[0][a], L.X[1][a], L.X[2][a], L.X[0][b], L.X[1][b], L.X[2][b]);
        } else if (la != lb) {
          double p0, p1, p2;
          crossing(L, a, b, s, p0, p1, p2);
          if (la) {  // exit: liquid part from a to the crossing
            vf += det3(c0, c1, c2, L.X[0][a], L.X[1][a], L.X[2][a], p0, p1, p2);
            ex |= 1ull << k;
          } else {   // entry: liquid part from the crossing to b
            vf += det3(c0, c1, c2, p0, p1, p2, L.X[0][b], L.X[1][b], L.X[2][b]);
            en |= 1ull << k;
          }
        }
        a = b;
        la = lb;
      }
    }
    int my = __popcll(ex);
    if (my && (en == 0 || __popcll(en) != my)) {  // a closed loop alternates exits and entries
      err = true;
      my = 0;
    }
    const int slot = nch + gscan_excl<W>(my, lane);
    if (my) {
      const int nx = my + __popcll(en);
      const bool liquid_connected = (nx == 2) || (L.fmean[f] >= s);
      uint64_t rem = ex;
      int j = 0;
      while (rem) {
        const int q = __ffsll((long long)rem) - 1;
        rem &= rem - 1;
        const int r = liquid_connected ? next_bit_after(en, q) : prev_bit_before(en, q);
        const int xa = L.lv[o + q], xb = L.lv[o + (q + 1 == m ? 0 : q + 1)];
        const int na = L.lv[o + r], nb = L.lv[o + (r + 1 == m ? 0 : r + 1)];
        double s0, s1, s2, e0, e1, e2;
        crossing(L, xa, xb, s, s0, s1, s2);
        crossing(L, na, nb, s, e0, e1, e2);
        vf += det3(c0, c1, c2, s0, s1, s2, e0, e1, e2);
        const int c = slot + j++;
        if (c < NCH) {
          L.ps[0][c] = s0; L.ps[1][c] = s1; L.ps[2][c] = s2;
          L.xkey[c] = (uint16_t)(xa < xb ? (xa << 8 | xb) : (xb << 8 | xa));
          L.nkey[c] = (uint16_t)(na < nb ? (na << 8 | nb) : (nb << 8 | na));
        } else {
          err = true;
        }
      }
    }
    nch += gsum_i<W>(my);
  }
  wave_sync();
  if (nch > NCH) nch = NCH;
  // ---- link chords: next = the chord whose entry edge is this chord's exit edge
  for (int c = lane; c < nch; c += W) {
    const uint16_t key = L.xkey[c];
    int nx = -1;
    for (int j = 0; j < nch; ++j)
      if (L.nkey[j] == key) { nx = j; break; }
    if (nx < 0) { err = true; nx = c; }
    L.nxt[c] = (uint16_t)nx;
    L.lab[0][c] = (uint16_t)c;
    L.jmp[0][c] = (uint16_t)nx;
  }
  wave_sync();
  // ---- loop labels: minimum chord index on each cycle, by pointer jumping
  int cur = 0;
  for (int span = 1; span < nch; span <<= 1) {
    for (int c = lane; c < nch; c += W) {
      const int j = L.jmp[cur][c];
      const int a = L.lab[cur][c], b = L.lab[cur][j];
      L.lab[cur ^ 1][c] = (uint16_t)(a < b ? a : b);
      L.jmp[cur ^ 1][c] = L.jmp[cur][j];
    }
    wave_sync();
    cur ^= 1;
  }
  // ---- loops: centroid, fan volume, area vector
  double Vi = 0, S0 = 0, S1 = 0, S2 = 0, Asum = 0, cw0 = 0, cw1 = 0, cw2 = 0;
  int nloops = 0, prev = -1;
  while (true) {
    int cand = 0x7fffffff;
    for (int c = lane; c < nch; c += W)
      if (L.lab[cur][c] == c && c > prev && c < cand) cand = c;
    cand = gmin_i<W>(cand);
    if (cand == 0x7fffffff) break;
    double l = 0, m0 = 0, m1 = 0, m2 = 0;
    for (int c = lane; c < nch; c += W) {
      if (L.lab[cur][c] != cand) continue;
      const int n = L.nxt[c];
      const double a0 = L.ps[0][c], a1 = L.ps[1][c], a2 = L.ps[2][c];
      const double b0 = L.ps[0][n], b1 = L.ps[1][n], b2 = L.ps[2][n];
      const double d0 = b0 - a0, d1 = b1 - a1, d2 = b2 - a2;
      const double len = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      l += len;
      m0 += len * (a0 + b0) * 0.5;
      m1 += len * (a1 + b1) * 0.5;
      m2 += len * (a2 + b2) * 0.5;
    }
    l = gsum<W>(l); m0 = gsum<W>(m0); m1 = gsum<W>(m1); m2 = gsum<W>(m2);
    double k0, k1, k2;
    if (l > 0) {
      k0 = m0 / l; k1 = m1 / l; k2 = m2 / l;
    } else {
      k0 = L.ps[0][cand]; k1 = L.ps[1][cand]; k2 = L.ps[2][cand];
    }
    double vi = 0, t0 = 0, t1 = 0, t2 = 0;
    for (int c = lane; c < nch; c += W) {
      if (L.lab[cur][c] != cand) continue;
      const int n = L.nxt[c];
      const double a0 = L.ps[0][c], a1 = L.ps[1][c], a2 = L.ps[2][c];
      const double b0 = L.ps[0][n], b1 = L.ps[1][n], b2 = L.ps[2][n];
      vi += det3(k0, k1, k2, a0, a1, a2, b0, b1, b2);
      const double u0 = a0 - k0, u1 = a1 - k1, u2 = a2 - k2;
      const double w0 = b0 - k0, w1 = b1 - k1, w2 = b2 - k2;
      // the fan is oriented out of the liquid; the normal is the opposite
      t0 -= 0.5 * (u1 * w2 - u2 * w1);
      t1 -= 0.5 * (u2 * w0 - u0 * w2);
      t2 -= 0.5 * (u0 * w1 - u1 * w0);
    }
    vi = gsum<W>(vi); t0 = gsum<W>(t0); t1 = gsum<W>(t1); t2 = gsum<W>(t2);
    const double Ak = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
    Vi += vi;
    S0 += t0; S1 += t1; S2 += t2;
    Asum += Ak;
    cw0 += Ak * k0; cw1 += Ak * k1; cw2 += Ak * k2;
    ++nloops;
    prev = cand;
  }
  vf = gsum<W>(vf);
  R.V = (vf + Vi) * (1.0 / 6.0);
  R.S0 = S0; R.S1 = S1; R.S2 = S2;
  R.A = Asum;
  if (Asum > 0) {
    R.c0 = cw0 / Asum; R.c1 = cw1 / Asum; R.c2 = cw2 / Asum;
  } else {
    R.c0 = R.c1 = R.c2 = 0;
  }
  R.nloops = nloops;
  R.err = gsum_i<W>(err ? 1 : 0) != 0;
  wave_sync();
  return R;
}

__device__ __forceinline__ double ulp_of(double x) {
  x = fabs(x);
  return nextafter(x, __builtin_inf()) - x;
}

template <int W, int NV, int NF, int NL, int NCH>
__global__ __launch_bounds__(64) void recon_kernel(ReconParams p) {
  constexpr int G = 64 / W;
  __shared__ GroupMem<NV, NF, NL, NCH> mem[G];
  const int g = threadIdx.x / W, lane = threadIdx.x % W;
  GroupMem<NV, NF, NL, NCH> &L = mem[g];
  const DevMesh &m = p.m;
  const int64_t N = m.n_cells;
  const int64_t cap = p.out.cap;
  int64_t count = p.counts[0];
  if (count > cap) count = cap;
  const int64_t stride = (int64_t)gridDim.x * G;
  for (int64_t k = (int64_t)blockIdx.x * G + g; k < count; k += stride) {
    const int P = p.mixed[k];
    const double a = p.alpha[P];
    double s_out = __builtin_nan(""), A_out = 0, d_out = 0, n0 = 0, n1 = 0, n2 = 0, ag = a;
    int st = VOFPC_CELL_OK, it = 0;
    const int64_t f0 = m.cell_face_off[P];
    const int nf = (int)(m.cell_face_off[P + 1] - f0);
    const int64_t v0 = m.cv_off[P];
    const int nv = (int)(m.cv_off[P + 1] - v0);
    const int64_t l0 = m.cl_off[P];
    const int nl = (int)(m.cl_off[P + 1] - l0);
    if (!(a >= 0.0 && a <= 1.0)) {
      st = VOFPC_CELL_BAD_INPUT;
    } else if (!(a > p.eps && a < 1.0 - p.eps)) {
      st = VOFPC_CELL_NOT_MIXED;
    } else if (nv > NV || nf > NF || nl > NL) {
      st = VOFPC_CELL_BAD_INPUT;  // cannot happen: the launcher sizes the caps
    } else {
      const double xP0 = m.xc[P], xP1 = m.xc[N + P], xP2 = m.xc[2 * N + P];
      const double VP = m.V[P];
      // ---- stage the polyhedron
      for (int i = lane; i < nv; i += W) {
        const int gv = m.cv_gid[v0 + i];
        L.X[0][i] = m.xyz[gv] - xP0;
        L.X[1][i] = m.xyz[m.n_verts + gv] - xP1;
        L.X[2][i] = m.xyz[2 * m.n_verts + gv] - xP2;
        double ph;
        if (p.phi_override) {
          ph = p.phi_override[gv];
        } else {
          const double *w = p.vertex_mode ? m.vc_wmean : m.vc_w;
          ph = 0.0;
          for (int64_t j = m.vc_off[gv]; j < m.vc_off[gv + 1]; ++j) ph += w[j] * p.alpha[m.vc_cell[j]];
        }
        L.phi[i] = ph;
      }
      for (int i = lane; i < nl; i += W) L.lv[i] = m.cl_lv[l0 + i];
      for (int f = lane; f < nf; f += W) {
        L.floff[f] = m.cf_loff[f0 + f];
        L.fsz[f] = m.cf_lsz[f0 + f];
      }
      wave_sync();
      double lo_phi = __builtin_inf(), hi_phi = -__builtin_inf();
      for (int i = lane; i < nv; i += W) {
        lo_phi = fmin(lo_phi, L.phi[i]);
        hi_phi = fmax(hi_phi, L.phi[i]);
      }
      double pmin = gmin<W>(lo_phi), pmax = gmax<W>(hi_phi);
      bool have_field = true;
      if (pmax - pmin <= 1e-12) {
        // degenerate vertex field: linear alpha from the plain least-squares
        // gradient over the interior face neighbours
        st = VOFPC_CELL_DEGENERATE;
        double gxx = 0, gyy = 0, gzz = 0, gxy = 0, gxz = 0, gyz = 0, b0 = 0, b1 = 0, b2 = 0;
        for (int f = lane; f < nf; f += W) {
          const int q = m.cf_nbr[f0 + f];
          if (q < 0) continue;
          const double r0 = m.xc[q] - xP0, r1 = m.xc[N + q] - xP1, r2 = m.xc[2 * N + q] - xP2;
          const double dv = p.alpha[q] - a;
          gxx += r0 * r0; gyy += r1 * r1; gzz += r2 * r2; gxy += r0 * r1; gxz += r0 * r2; gyz += r1 * r2;
          b0 += r0 * dv; b1 += r1 * dv; b2 += r2 * dv;
        }
        gxx = gsum<W>(gxx); gyy = gsum<W>(gyy); gzz = gsum<W>(gzz);
        gxy = gsum<W>(gxy); gxz = gsum<W>(gxz); gyz = gsum<W>(gyz);
        b0 = gsum<W>(b0); b1 = gsum<W>(b1); b2 = gsum<W>(b2);
        const double c00 = gyy * gzz - gyz * gyz, c01 = gxz * gyz - gxy * gzz, c02 = gxy * gyz - gxz * gyy;
        const double c11 = gxx * gzz - gxz * gxz, c12 = gxy * gxz - gxx * gyz, c22 = gxx * gyy - gxy * gxy;
        const double det = gxx * c00 + gxy * c01 + gxz * c02;
        const double tr = (gxx + gyy + gzz) / 3.0;
        double g0 = 0, g1 = 0, g2 = 0;
        if (det > 1e-12 * tr * tr * tr) {
          g0 = (c00 * b0 + c01 * b1 + c02 * b2) / det;
          g1 = (c01 * b0 + c11 * b1 + c12 * b2) / det;
          g2 = (c02 * b0 + c12 * b1 + c22 * b2) / det;
        }
        wave_sync();
        lo_phi = __builtin_inf();
        hi_phi = -__builtin_inf();
        for (int i = lane; i < nv; i += W) {
          const double ph = a + (g0 * L.X[0][i] + g1 * L.X[1][i] + g2 * L.X[2][i]);
          L.phi[i] = ph;
          lo_phi = fmin(lo_phi, ph);
          hi_phi = fmax(hi_phi, ph);
        }
        pmin = gmin<W>(lo_phi);
        pmax = gmax<W>(hi_phi);
        if (pmax - pmin <= 1e-12) have_field = false;
      }
      if (have_field) {
        // face vertex means (fan centres of the planar faces) and face-mean
        // vertex values (pairing rule of faces with four or more crossings)
        for (int f = lane; f < nf; f += W) {
          const int o = L.floff[f], n = L.fsz[f];
          double c0 = 0, c1 = 0, c2 = 0, fm = 0;
          for (int k2 = 0; k2 < n; ++k2) {
            const int v = L.lv[o + k2];
            c0 += L.X[0][v]; c1 += L.X[1][v]; c2 += L.X[2][v];
            fm += L.phi[v];
          }
          L.cf[0][f] = c0 / n; L.cf[1][f] = c1 / n; L.cf[2][f] = c2 / n;
          L.fmean[f] = fm / n;
        }
        wave_sync();
        CutRes c;
        c.err = false;
        double s = __builtin_nan("");
        bool cut_ok = false;
        if (p.fixed_iso) {
          s = p.iso;
          c = cut_eval<W>(L, lane, nf, s);
          it = 1;
          cut_ok = true;
        } else {
          double lo = pmin, hi = pmax, rlo = 1.0 - a, rhi = -a;
          const double tol = p.tol_rel * (a < 1.0 - a ? a : 1.0 - a);
          CutRes clo, chi;
          bool have_lo = false, have_hi = false, done = false, collapsed = false;
          if (p.use_hint) {
            const double hl = p.hint_lo[k], hh = p.hint_hi[k];
            if (!isnan(hl) && !isnan(hh)) {
              double l2 = hl > pmin ? hl : pmin;
              double h2 = hh < pmax ? hh : pmax;
              if (l2 > h2) { l2 = pmin; h2 = pmax; }
              const CutRes cl = cut_eval<W>(L, lane, nf, l2);
              const CutRes chh = cut_eval<W>(L, lane, nf, h2);
              it += 2;
              const double rl = cl.V / VP - a, rh = chh.V / VP - a;
              if (fabs(rl) <= tol) { s = l2; c = cl; done = true; }
              else if (fabs(rh) <= tol) { s = h2; c = chh; done = true; }
              else if (rl > 0 && rh < 0) {
                lo = l2; rlo = rl; clo = cl; have_lo = true;
                hi = h2; rhi = rh; chi = chh; have_hi = true;
              } else if (rl <= 0) {
                hi = l2; rhi = rl; chi = cl; have_hi = true;
                if (st == VOFPC_CELL_OK) st = VOFPC_CELL_LEARNED_FALLBACK;
              } else {
                lo = h2; rlo = rh; clo = chh; have_lo = true;
                if (st == VOFPC_CELL_OK) st = VOFPC_CELL_LEARNED_FALLBACK;
              }
              if (done) cut_ok = true;
            }
          }
          while (!done) {
            if (it >= p.max_iter) { st = VOFPC_CELL_MAX_ITER; break; }
            s = lo + (hi - lo) / 2.0;
            c = cut_eval<W>(L, lane, nf, s);
            ++it;
            cut_ok = true;
            const double r = c.V / VP - a;
            if (fabs(r) <= tol) break;
            if (r > 0) { lo = s; rlo = r; clo = c; have_lo = true; }
            else { hi = s; rhi = r; chi = c; have_hi = true; }
            const double big = fabs(lo) > fabs(hi) ? fabs(lo) : fabs(hi);
            if (hi - lo <= 2.0 * ulp_of(big)) { collapsed = true; break; }
          }
          if (collapsed) {
            const bool take_lo = fabs(rlo) <= fabs(rhi);
            s = take_lo ? lo : hi;
            if (take_lo ? have_lo : have_hi) {
              c = take_lo ? clo : chi;
            } else {
              c = cut_eval<W>(L, lane, nf, s);
              ++it;
            }
            if (fabs(take_lo ? rlo : rhi) > 1e-10 && st != VOFPC_CELL_MAX_ITER) st = VOFPC_CELL_NO_ROOT;
          }
        }
        if (cut_ok && c.err) {
          st = VOFPC_CELL_BAD_INPUT;
        } else if (cut_ok) {
          s_out = s;
          ag = c.V / VP;
          A_out = c.A;
          const double Sm = sqrt(c.S0 * c.S0 + c.S1 * c.S1 + c.S2 * c.S2);
          if (Sm > 0) {
            n0 = c.S0 / Sm; n1 = c.S1 / Sm; n2 = c.S2 / Sm;
            d_out = -(n0 * c.c0 + n1 * c.c1 + n2 * c.c2);
          }
        }
      }
    }
    if (lane == 0) {
      p.out.s[k] = s_out;
      p.out.n[k] = n0; p.out.n[cap + k] = n1; p.out.n[2 * cap + k] = n2;
      p.out.A[k] = A_out;
      p.out.d[k] = d_out;
      p.out.alpha_got[k] = ag;
      p.out.status[k] = st;
      p.out.iters[k] = it;
    }
    wave_sync();
  }
}

namespace {
template <int W, int NV, int NF, int NL, int NCH>
vofpc_status launch_t(vofpc_ctx ctx, const ReconParams &p, int64_t n_cells) {
  constexpr int G = 64 / W;
  int64_t need = (n_cells + G - 1) / G;
  int blocks_per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks_per_cu, recon_kernel<W, NV, NF, NL, NCH>, 64, 0);
  if (e != hipSuccess || blocks_per_cu <= 0) blocks_per_cu = 4;
  int64_t grid = (int64_t)ctx->n_cu * blocks_per_cu * 4;
  if (grid > need) grid = need;
  if (grid < 1) grid = 1;
  recon_kernel<W, NV, NF, NL, NCH><<<(unsigned)grid, 64, 0, ctx->stream>>>(p);
  VOFPC_HIP(hipGetLastError());
  return VOFPC_OK;
}
}  // namespace

vofpc_status launch_reconstruct(vofpc_ctx ctx, vofpc_mesh M, const double *alpha, const int32_t *mixed,
                                const int32_t *counts, const vofpc_recon_opts *o, const double *hlo,
                                const double *hhi, const vofpc_interface *out) {
  VOFPC_REQUIRE(alpha && mixed && counts && o && out, VOFPC_E_INVALID_ARG, "reconstruct: null argument");
  VOFPC_REQUIRE(out->s && out->n && out->A && out->d && out->alpha_got && out->status && out->iters,
                VOFPC_E_INVALID_ARG, "reconstruct: null output array");
  VOFPC_REQUIRE(out->cap > 0, VOFPC_E_INVALID_ARG, "reconstruct: output capacity must be positive");
  VOFPC_REQUIRE(o->eps_mixed >= 0 && o->eps_mixed < 0.5, VOFPC_E_INVALID_ARG, "reconstruct: eps_mixed in [0, 0.5)");
  VOFPC_REQUIRE(o->tol_rel >= 0 && o->max_iter >= 1 && o->max_iter <= 10000, VOFPC_E_INVALID_ARG,
                "reconstruct: tol_rel >= 0 and 1 <= max_iter <= 10000");
  VOFPC_REQUIRE(o->vertex_mode == VOFPC_VERTEX_IDW || o->vertex_mode == VOFPC_VERTEX_MEAN, VOFPC_E_INVALID_ARG,
                "reconstruct: unknown vertex_mode");
  VOFPC_REQUIRE(o->bracket == VOFPC_BRACKET_PLAIN || o->bracket == VOFPC_BRACKET_HINT, VOFPC_E_INVALID_ARG,
                "reconstruct: unknown bracket");
  VOFPC_REQUIRE(o->bracket != VOFPC_BRACKET_HINT || (hlo && hhi), VOFPC_E_INVALID_ARG,
                "reconstruct: hint bracket needs hint_lo and hint_hi");
  ReconParams p;
  p.m = M->d;
  p.alpha = alpha;
  p.mixed = mixed;
  p.counts = counts;
  p.phi_override = o->phi_vertex;
  p.hint_lo = hlo;
  p.hint_hi = hhi;
  p.eps = o->eps_mixed;
  p.tol_rel = o->tol_rel;
  p.iso = o->iso;
  p.max_iter = o->max_iter;
  p.vertex_mode = o->vertex_mode;
  p.fixed_iso = o->fixed_iso ? 1 : 0;
  p.use_hint = (o->bracket == VOFPC_BRACKET_HINT) ? 1 : 0;
  p.out = *out;
  const int64_t nf = M->max_nf, nv = M->max_nv, nl = M->max_loop, ne = M->max_ne, fv = M->max_fv;
  VOFPC_REQUIRE(fv <= 64, VOFPC_E_MESH, "reconstruct: faces with more than 64 vertices are not supported");
  const int64_t N = M->d.n_cells;
  if (nv <= 16 && nf <= 8 && nl <= 48 && ne <= 24) return launch_t<8, 16, 8, 48, 24>(ctx, p, N);
  if (nv <= 64 && nf <= 32 && nl <= 256 && ne <= 96) return launch_t<16, 64, 32, 256, 96>(ctx, p, N);
  if (nv <= 128 && nf <= 64 && nl <= 512 && ne <= 192) return launch_t<32, 128, 64, 512, 192>(ctx, p, N);
  return launch_t<64, 255, 255, 1536, 768>(ctx, p, N);
}

}  // namespace vofpc
