// Volume-matched iso-polygon reconstruction with a group of G lanes per mixed
// cell (G = 1 to 16) and 64/G cells per wavefront.
//
// The one-cell-per-wavefront kernel (recon.hip) spreads a cell's loop
// positions over 64 lanes, so most lanes idle on hexahedra and on the search
// control.  Here a group of G lanes shares a cell's edges and faces, combines
// its lanes' sums by DPP butterflies, and a wavefront works on 64/G cells at
// once, staged side by side in LDS (arrays indexed [item][cell slot], so the
// cells of a wavefront read different banks).
//
// One volume evaluation at isovalue s (divergence theorem, each face's
// liquid polygon fanned from a point of its plane, here its first vertex):
//   - per edge: the two faces' terms of the whole edge, D_e = det(c1, u, v) +
//     det(c2, v, u), are fixed per cell; an evaluation adds D_e times the
//     edge's liquid fraction (1, 0, or for a cut edge the fraction from its
//     liquid end, which scales both faces' liquid pieces of the edge alike),
//     and registers a cut edge with the face the iso-curve leaves through it
//     and the face it enters through it;
//   - per face: a face with two crossings has one chord, exit -> entry; a
//     face with four or more pairs each exit with the next entry in loop
//     order when the face-mean vertex value is >= s, else with the previous
//     one (the oracle's rule); the chord closes the face's liquid polygon;
//     crossing points follow Eq. edge_intersection from the liquid end of
//     the edge, computed once per edge, so both faces get the same point;
//   - per chord, the terms of its iso-loop: a loop is the chain of chords
//     (the chord entering through edge e follows the chord leaving through
//     e), and fanning a loop from its length-weighted polyline centroid k
//     gives volume k . Y / 6 and area vector -Y / 2 with Y = sum over its
//     chords of (entry point x exit point), the centroid from sum l and
//     sum l (entry + exit): chord-local sums, taken about a reference
//     vertex of the cell.  A single loop (the usual case, found by walking
//     the chord links once) needs nothing else; several loops are labelled
//     through LDS and their sums gathered loop by loop in a second pass over
//     the faces.
//
// Search: Brent's method (Brent 1973, ch. 4) on r(s) = V(s)/V_P - alpha
// over a bracket of [phi_min, phi_max] whose ends straddle the root: inverse
// quadratic interpolation or the secant, the midpoint when the estimate
// leaves the quarter of the bracket next to its better end or does not
// shrink fast enough; one evaluation per step, the stopping rule of the
// wavefront kernel.  A narrowed bracket [h_lo, h_hi] is first checked with
// two evaluations: at its centre (the network's predicted isovalue), whose
// residual gives the side of the root, and at its end on that side.  The
// half on the root's side starts the method when that end is past the root;
// otherwise the part of the full bracket beyond that end does (status
// LEARNED_FALLBACK: the root is outside the bracket).
//
// Scheduling: a wavefront takes 64/G consecutive mixed entries (a batch),
// stages them together, runs their searches side by side until the last one
// stops, writes them out and claims the next batch.  The batches go to the
// XCDs in runs of consecutive batches (neighbouring cells share an L2), and
// each XCD's wavefronts claim its batches from a counter of its own that
// wraps back to zero after the XCD's last claim.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "recon_common.h"
#include "mlp_core.h"

namespace vofpc {
namespace {

// ---------------------------------------------------------- group reductions
// Sums, minima and maxima over the G consecutive lanes of a group by DPP quad,
// half-row and row butterflies; every lane of the group ends with the same
// bits.
template <int G>
__device__ __forceinline__ double tsum(double v) {
  if constexpr (G >= 2) v += dpp_d<kQuadXor1>(v);
  if constexpr (G >= 4) v += dpp_d<kQuadXor2>(v);
  if constexpr (G >= 8) v += dpp_d<kHalfMirror>(v);
  if constexpr (G >= 16) v += dpp_d<kRowMirror>(v);
  return v;
}
template <int G>
__device__ __forceinline__ int tsum_i(int v) {
  if constexpr (G >= 2) v += dpp_i<kQuadXor1>(v);
  if constexpr (G >= 4) v += dpp_i<kQuadXor2>(v);
  if constexpr (G >= 8) v += dpp_i<kHalfMirror>(v);
  if constexpr (G >= 16) v += dpp_i<kRowMirror>(v);
  return v;
}
template <int G>
__device__ __forceinline__ int tmin_i(int v) {
  if constexpr (G >= 2) v = min(v, dpp_i<kQuadXor1>(v));
  if constexpr (G >= 4) v = min(v, dpp_i<kQuadXor2>(v));
  if constexpr (G >= 8) v = min(v, dpp_i<kHalfMirror>(v));
  if constexpr (G >= 16) v = min(v, dpp_i<kRowMirror>(v));
  return v;
}
template <int G>
__device__ __forceinline__ double tmin(double v) {
  if constexpr (G >= 2) v = fmin(v, dpp_d<kQuadXor1>(v));
  if constexpr (G >= 4) v = fmin(v, dpp_d<kQuadXor2>(v));
  if constexpr (G >= 8) v = fmin(v, dpp_d<kHalfMirror>(v));
  if constexpr (G >= 16) v = fmin(v, dpp_d<kRowMirror>(v));
  return v;
}
template <int G>
__device__ __forceinline__ double tmax(double v) {
  if constexpr (G >= 2) v = fmax(v, dpp_d<kQuadXor1>(v));
  if constexpr (G >= 4) v = fmax(v, dpp_d<kQuadXor2>(v));
  if constexpr (G >= 8) v = fmax(v, dpp_d<kHalfMirror>(v));
  if constexpr (G >= 16) v = fmax(v, dpp_d<kRowMirror>(v));
  return v;
}

// ------------------------------------------------------------ fast division
// Quotient a/b from the hardware reciprocal, refined by two Newton steps and
// one residual correction (within an ulp of the rounded quotient; b finite
// and nonzero): a few instructions instead of the IEEE division sequence.
__device__ __forceinline__ double qdiv(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(fma(-b, r, 1.0), r, r);
  r = fma(fma(-b, r, 1.0), r, r);
  const double q = a * r;
  return fma(fma(-b, q, a), r, q);
}
// Square root of x >= 0 from the hardware reciprocal square root, refined by
// two Newton steps and one residual correction (0 for x = 0).
__device__ __forceinline__ double qsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  y = y * fma(-0.5 * x * y, y, 1.5);
  const double t = x * y;
  return x > 0.0 ? fma(fma(-t, t, x), 0.5 * y, t) : 0.0;
}
// Root of the inverse quadratic through three (isovalue, residual) points,
// about x0 over one common denominator; NaN or infinite when two residuals
// coincide.
__device__ __forceinline__ double iqi1(double x0, double f0, double x1, double f1, double x2, double f2) {
  const double d01 = f0 - f1, d02 = f0 - f2, d12 = f1 - f2;
  return x0 + qdiv((x2 - x0) * f0 * f1 * d01 - (x1 - x0) * f0 * f2 * d02, d01 * d02 * d12);
}

// ----------------------------------------------------------------- LDS layout
// The staged cells of one wavefront, item-major and cell-slot-minor; the
// 4- and 8-byte arrays have an odd slot stride CP, so the lanes of a group,
// which read different items of one cell, spread over the LDS banks.
// Network scratch of a wavefront (learned form): one BF16 input row per cell
// slot (16 rows at least: a tile), one 16-row tile of hidden activations and
// the first output per slot.
template <int C>
struct ThinNet {
  static constexpr int R = C < 16 ? 16 : C;
  alignas(16) uint16_t x[R][net::kIn];
  alignas(16) uint16_t h[16][net::kHid];
  float u[R];
};

template <int C, int NV, int NF, int NL, int NE>
struct ThinMem {
  static constexpr int CP = C | 1;
  double X[3][NV][CP];  // vertex positions relative to the cell centroid
  double phi[NV][CP];   // vertex field
  double D[NE][CP];     // volume term of an edge taken whole by both of its faces
  // scratch of one evaluation; outside evaluations (the network phase of the
  // learned form) the same bytes hold the network's rows
  union {
    struct {
      double fr[NE][CP];    // liquid fraction of each cut edge (this evaluation)
      int32_t cnt[NF][CP];  // crossings of each face (this evaluation)
    };
    ThinNet<C> net;
  };
  uint8_t eu[NE][C], ev[NE][C];    // end vertices of each edge
  uint8_t ef1[NE][C], ef2[NE][C];  // face whose loop runs eu -> ev, and the other face
  uint8_t fx[NF][C], fn[NF][C];    // exit and entry edge of a face with two crossings
  uint8_t lv[NL][C];    // local vertex of each loop position
  uint8_t eid[NL][C];   // local edge of each loop position
  uint8_t foff[NF][C];  // first loop position of each face
  uint8_t fsz[NF][C];   // positions of each face
  uint8_t link[NE][C];  // exit edge of the chord entering through edge e (0xff: e not cut)
  uint8_t lab[NE][C];   // loop of each cut edge (evaluations with several loops)
};

// per-lane sums of the chords of one loop (or of all loops)
struct ChordAcc {
  double L, M0, M1, M2, Y0, Y1, Y2;
};

template <int G>
__device__ __forceinline__ void reduce_acc(ChordAcc &a) {
  a.L = tsum<G>(a.L);
  a.M0 = tsum<G>(a.M0); a.M1 = tsum<G>(a.M1); a.M2 = tsum<G>(a.M2);
  a.Y0 = tsum<G>(a.Y0); a.Y1 = tsum<G>(a.Y1); a.Y2 = tsum<G>(a.Y2);
}

// Crossing point of cut edge e at isovalue s: Eq. edge_intersection from
// the edge's liquid end, with the liquid fraction of this evaluation, so
// both faces of the edge get the same point.
template <class TM>
__device__ __forceinline__ void edge_point(const TM &M, int sl, int e, double s, double &p0, double &p1, double &p2) {
  const int u = M.eu[e][sl], v = M.ev[e][sl];
  const bool ul = M.phi[u][sl] >= s;
  const int i = ul ? u : v, j = ul ? v : u;
  const double lam = M.fr[e][sl];
  p0 = M.X[0][i][sl] + lam * (M.X[0][j][sl] - M.X[0][i][sl]);
  p1 = M.X[1][i][sl] + lam * (M.X[1][j][sl] - M.X[1][i][sl]);
  p2 = M.X[2][i][sl] + lam * (M.X[2][j][sl] - M.X[2][i][sl]);
}

// One chord from exit point x to entry point e (edges ex, en) of a face with
// fan point c.  mode 0: the face volume term, the link and the chord sums;
// mode 1: only the sums, and only when the chord lies on loop `loop`.
template <class TM>
__device__ __forceinline__ void add_chord(TM &M, int sl, int mode, int loop, const double *r, double c0, double c1,
                                          double c2, double x0, double x1, double x2, double e0, double e1, double e2,
                                          int ex, int en, double &vf, ChordAcc &acc, int &nch, int &estart) {
  if (mode == 0) {
    vf += det3(c0, c1, c2, x0, x1, x2, e0, e1, e2);
    M.link[en][sl] = (uint8_t)ex;
    estart = en < estart ? en : estart;
    ++nch;
  } else if (M.lab[en][sl] != loop) {
    return;
  }
  // the chord as a loop segment, from its entry point u to its exit point w,
  // both relative to the cell's reference point r (near a small cut piece,
  // so the cross products of a small loop do not cancel)
  const double u0 = e0 - r[0], u1 = e1 - r[1], u2 = e2 - r[2];
  const double w0 = x0 - r[0], w1 = x1 - r[1], w2 = x2 - r[2];
  const double d0 = w0 - u0, d1 = w1 - u1, d2 = w2 - u2;
  const double l = qsqrt(d0 * d0 + d1 * d1 + d2 * d2);
  acc.L += l;
  acc.M0 += l * (u0 + w0);
  acc.M1 += l * (u1 + w1);
  acc.M2 += l * (u2 + w2);
  acc.Y0 += u1 * w2 - u2 * w1;
  acc.Y1 += u2 * w0 - u0 * w2;
  acc.Y2 += u0 * w1 - u1 * w0;
}

// The chords of face f at isovalue s (see add_chord for mode): one chord,
// exit -> entry, for a face with two crossings; with four or more, each exit
// pairs with the next entry in loop order when the face-mean vertex value is
// >= s, else with the previous one.  The fan point is the face's first
// vertex.
template <class TM>
__device__ void chords_of_face(TM &M, int sl, int f, double s, int mode, int loop, const double *r, double &vf,
                               ChordAcc &acc, int &nch, int &estart, bool &err) {
  const int c = M.cnt[f][sl];
  if (c == 0) return;
  const int o = M.foff[f][sl];
  const int a0 = M.lv[o][sl];
  const double c0 = M.X[0][a0][sl], c1 = M.X[1][a0][sl], c2 = M.X[2][a0][sl];
  if (c == 2) {
    const int ex = M.fx[f][sl], en = M.fn[f][sl];
    double x0, x1, x2, e0, e1, e2;
    edge_point(M, sl, ex, s, x0, x1, x2);
    edge_point(M, sl, en, s, e0, e1, e2);
    add_chord(M, sl, mode, loop, r, c0, c1, c2, x0, x1, x2, e0, e1, e2, ex, en, vf, acc, nch, estart);
    return;
  }
  if (c & 1) {
    err = true;   // a closed loop alternates exits and entries
    return;
  }
  const int n = M.fsz[f][sl];
  double fm = 0.0;
  for (int k = 0; k < n; ++k) fm += M.phi[M.lv[o + k][sl]][sl];
  const bool conn = fm / (double)n >= s;
  for (int k = 0; k < n; ++k) {
    const int u = M.lv[o + k][sl], v = M.lv[o + ((k + 1 == n) ? 0 : k + 1)][sl];
    if (!(M.phi[u][sl] >= s) || M.phi[v][sl] >= s) continue;   // not an exit
    int rr = k;
    bool found = false;
    for (int t = 0; t < n && !found; ++t) {
      rr = conn ? ((rr + 1 == n) ? 0 : rr + 1) : ((rr == 0) ? n - 1 : rr - 1);
      const int ru = M.lv[o + rr][sl], rv = M.lv[o + ((rr + 1 == n) ? 0 : rr + 1)][sl];
      found = !(M.phi[ru][sl] >= s) && M.phi[rv][sl] >= s;
    }
    if (!found) {
      err = true;
      continue;
    }
    const int ex = M.eid[o + k][sl], en = M.eid[o + rr][sl];
    double x0, x1, x2, e0, e1, e2;
    edge_point(M, sl, ex, s, x0, x1, x2);
    edge_point(M, sl, en, s, e0, e1, e2);
    add_chord(M, sl, mode, loop, r, c0, c1, c2, x0, x1, x2, e0, e1, e2, ex, en, vf, acc, nch, estart);
  }
}

// Add one loop's fan: centroid k = r + M/(2L) from the length sums (relative
// to r), volume k . Y, area vector -Y/2.
__device__ __forceinline__ void finish_loop(const ChordAcc &a, const double *r, double &Vi, double &S0, double &S1,
                                            double &S2, double &A, double &cw0, double &cw1, double &cw2) {
  double k0 = r[0], k1 = r[1], k2 = r[2];   // a loop of zero length has zero area: its centre does not matter
  if (a.L > 0) {
    const double h = qdiv(0.5, a.L);
    k0 += a.M0 * h; k1 += a.M1 * h; k2 += a.M2 * h;
  }
  Vi += k0 * a.Y0 + k1 * a.Y1 + k2 * a.Y2;
  const double t0 = -0.5 * a.Y0, t1 = -0.5 * a.Y1, t2 = -0.5 * a.Y2;
  const double Ak = qsqrt(t0 * t0 + t1 * t1 + t2 * t2);
  S0 += t0; S1 += t1; S2 += t2;
  A += Ak;
  cw0 += Ak * k0; cw1 += Ak * k1; cw2 += Ak * k2;
}

// One volume evaluation of the cell in slot sl at isovalue s by its group.
template <int G, class TM>
__device__ CutRes thin_eval(TM &M, int sl, int q, int nf, int ne, double s, const double *r) {
  for (int e = q; e < ne; e += G) M.link[e][sl] = 0xff;
  for (int f = q; f < nf; f += G) M.cnt[f][sl] = 0;
  wave_sync();
  // edges: the liquid parts of the faces (an edge's term times its liquid
  // fraction: 1, 0, or, for a cut edge, the fraction from its liquid end,
  // which scales both faces' pieces alike), and each crossing registered
  // with the face the iso-curve leaves through it and the one it enters
  double vf = 0.0;
  for (int e = q; e < ne; e += G) {
    const int u = M.eu[e][sl], v = M.ev[e][sl];
    const double pu = M.phi[u][sl], pv = M.phi[v][sl];
    const bool lu = pu >= s, lw = pv >= s;
    if (lu && lw) {
      vf += M.D[e][sl];
    } else if (lu != lw) {
      const double pi = lu ? pu : pv, pj = lu ? pv : pu;
      const double lam = qdiv(s - pi, pj - pi);
      M.fr[e][sl] = lam;
      vf += lam * M.D[e][sl];
      const int f1 = M.ef1[e][sl], f2 = M.ef2[e][sl];
      const int fo = lu ? f1 : f2, fi = lu ? f2 : f1;   // face f1 runs u -> v
      M.fx[fo][sl] = (uint8_t)e;
      M.fn[fi][sl] = (uint8_t)e;
      atomicAdd(&M.cnt[fo][sl], 1);
      atomicAdd(&M.cnt[fi][sl], 1);
    }
  }
  wave_sync();
  ChordAcc acc{0, 0, 0, 0, 0, 0, 0};
  int nch = 0, estart = 0xff;
  bool err = false;
  for (int f = q; f < nf; f += G) chords_of_face(M, sl, f, s, 0, 0, r, vf, acc, nch, estart, err);
  vf = tsum<G>(vf);
  reduce_acc<G>(acc);
  nch = tsum_i<G>(nch);
  estart = tmin_i<G>(estart);
  int bad = tsum_i<G>(err ? 1 : 0);
  wave_sync();
  double Vi = 0, S0 = 0, S1 = 0, S2 = 0, A = 0, cw0 = 0, cw1 = 0, cw2 = 0;
  if (nch > 0 && bad == 0) {
    // follow the chord links once from one cut edge: a single loop returns
    // after nch chords
    int e = estart, len = 0;
    do {
      e = M.link[e][sl];
      ++len;
    } while (e != estart && e != 0xff && len <= nch);
    if (e == 0xff) {
      bad = 1;
    } else if (e == estart && len == nch) {
      finish_loop(acc, r, Vi, S0, S1, S2, A, cw0, cw1, cw2);
    } else {
      // several loops: label the cut edges, then gather each loop's chords
      for (int t = 0; t < ne; ++t) M.lab[t][sl] = 0xff;
      int nloop = 0;
      for (int t = 0; t < ne && bad == 0; ++t) {
        if (M.link[t][sl] == 0xff || M.lab[t][sl] != 0xff) continue;
        int u = t, steps = 0;
        do {
          M.lab[u][sl] = (uint8_t)nloop;
          u = M.link[u][sl];
          ++steps;
        } while (u != t && u != 0xff && steps <= nch);
        if (u != t) bad = 1;
        ++nloop;
      }
      wave_sync();
      for (int lp = 0; lp < nloop && bad == 0; ++lp) {
        ChordAcc la{0, 0, 0, 0, 0, 0, 0};
        double dv = 0.0;
        int dn = 0, ds = 0;
        bool derr = false;
        for (int f = q; f < nf; f += G) chords_of_face(M, sl, f, s, 1, lp, r, dv, la, dn, ds, derr);
        reduce_acc<G>(la);
        finish_loop(la, r, Vi, S0, S1, S2, A, cw0, cw1, cw2);
      }
    }
  }
  wave_sync();
  CutRes R;
  R.err = bad != 0;
  R.nch = nch;
  R.V = (vf + Vi) * (1.0 / 6.0);
  R.S0 = S0; R.S1 = S1; R.S2 = S2;
  R.A = A;
  if (A > 0) {
    const double ia = qdiv(1.0, A);
    R.c0 = cw0 * ia; R.c1 = cw1 * ia; R.c2 = cw2 * ia;
  } else {
    R.c0 = R.c1 = R.c2 = 0.0;
  }
  return R;
}



// Forward pass of the wavefront's rows on v_mfma_f32_16x16x16_bf16 tiles, all
// 64 lanes, 16 rows per tile (BF16 weights and activations, FP32
// accumulation, tanh hidden layers); u[r] = output 0 of row r.  Lane l holds
// A[l%16][4(l/16)+j], B[4(l/16)+j][l%16] and D[4(l/16)+j][l%16].
template <int C>
__device__ void net_tiles(ThinNet<C> &T, const uint16_t *wb, const float *master, int lane) {
  using namespace net;
  const int col = lane & 15, rq = 4 * (lane >> 4);
  for (int t0 = 0; t0 < ThinNet<C>::R; t0 += 16) {
    for (int nt = 0; nt < kHid / 16; ++nt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int kt = 0; kt < kIn / 16; ++kt)
        acc = mfma16(*reinterpret_cast<const bf16x4 *>(&T.x[t0 + col][kt * 16 + rq]),
                     b_weightT(wb + oW1, kIn, lane, nt * 16, kt * 16, kHid), acc);
      const float b = master[oB1 + nt * 16 + col];
      for (int j = 0; j < 4; ++j) T.h[rq + j][nt * 16 + col] = to_bf16(act_tanh(acc[j] + b));
    }
    wave_sync();
    f32x4 acc2[kHid / 16];
    for (int nt = 0; nt < kHid / 16; ++nt) {
      acc2[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
      for (int kt = 0; kt < kHid / 16; ++kt)
        acc2[nt] = mfma16(*reinterpret_cast<const bf16x4 *>(&T.h[col][kt * 16 + rq]),
                          b_weightT(wb + oW2, kHid, lane, nt * 16, kt * 16, kHid), acc2[nt]);
    }
    wave_sync();
    for (int nt = 0; nt < kHid / 16; ++nt) {
      const float b = master[oB2 + nt * 16 + col];
      for (int j = 0; j < 4; ++j) T.h[rq + j][nt * 16 + col] = to_bf16(act_tanh(acc2[nt][j] + b));
    }
    wave_sync();
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < kHid / 16; ++kt)
      acc = mfma16(*reinterpret_cast<const bf16x4 *>(&T.h[col][kt * 16 + rq]),
                   b_weightT(wb + oW3, kHid, lane, 0, kt * 16, kOut), acc);
    if (col == 0) {
      const float b = master[oB3];
      for (int j = 0; j < 4; ++j) T.u[t0 + rq + j] = acc[j] + b;
    }
    wave_sync();
  }
}

// The 32 network inputs of the cell in slot sl (the definitions of the
// features entry point) into its BF16 row: face sums over the group's faces,
// the vertex values ordered by rank (ties by index) through M.link.
template <int G, class TM, int C>
__device__ void cell_features(TM &M, ThinNet<C> &T, int sl, int q, const ReconParams &p, int P, double a, int nv,
                              int nf, int64_t f0, double pmin, double Wd) {
  double t[18];
#pragma unroll
  for (int i = 0; i < 18; ++i) t[i] = 0.0;
  double amin = __builtin_inf(), amax = -__builtin_inf();
  for (int f = q; f < nf; f += G) {
    const NetFace g = load_net_face(p, P, a, f0 + f);
    const double A = sqrt(g.S0 * g.S0 + g.S1 * g.S1 + g.S2 * g.S2);
    const double n0 = g.S0 / A, n1 = g.S1 / A, n2 = g.S2 / A;
    const double da = A * (g.aQ - a);
    const double o[6] = {n0 * n0, n1 * n1, n2 * n2, n0 * n1, n0 * n2, n1 * n2};
    t[0] += A;
    t[1] += da * n0; t[2] += da * n1; t[3] += da * n2;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      t[4 + c] += da * o[c];
      t[10 + c] += A * o[c];
    }
    if (g.inner) {
      t[16] += g.aQ;
      t[17] += 1.0;
      amin = fmin(amin, g.aQ);
      amax = fmax(amax, g.aQ);
    }
  }
#pragma unroll
  for (int i = 0; i < 18; ++i) t[i] = tsum<G>(t[i]);
  amin = tmin<G>(amin);
  amax = tmax<G>(amax);
  double lsum = 0.0;
  for (int i = q; i < nv; i += G) {
    const double v = M.phi[i][sl];
    int r = 0;
    for (int jv = 0; jv < nv; ++jv) {
      const double u = M.phi[jv][sl];
      r += (u < v) || (u == v && jv < i);
    }
    M.link[r][sl] = (uint8_t)i;
    lsum += v;
  }
  lsum = tsum<G>(lsum);
  wave_sync();
  auto sorted = [&](int r) { return M.phi[M.link[r][sl]][sl]; };
  if constexpr (sizeof(T.h) >= sizeof(double) * 18 * C) {
    // the sums go through LDS (the hidden-layer tile, not yet in use: 18
    // doubles per cell slot), so each lane computes only its own features
    // with a runtime index
    double *ts = reinterpret_cast<double *>(&T.h[0][0]) + 18 * sl;
    if (q == 0) {
#pragma unroll
      for (int i = 0; i < 18; ++i) ts[i] = t[i];
    }
    wave_sync();
    for (int i = q; i < net::kIn; i += G)
      T.x[sl][i] = net::to_bf16(net::feature(i, a, sorted, nv, lsum, pmin, Wd, ts, amin, amax, nf));
    wave_sync();
  } else {
    // few lanes per cell: every feature index unrolled, each taken by the
    // lane it falls to (the sums stay in registers; a runtime index would
    // put them in scratch)
#pragma unroll
    for (int i = 0; i < net::kIn; ++i)
      if (i % G == q) T.x[sl][i] = net::to_bf16(net::feature(i, a, sorted, nv, lsum, pmin, Wd, t, amin, amax, nf));
  }
}

// The cell's vertices (positions relative to xP, when WANT_X) and their
// inverse-distance vertex field (or the caller's override) into LDS; lane q
// of a group takes vertices q, q + G, ...  Each lane works KV vertices per
// round with the loads of a round issued together level by level (vertex
// ids; positions and incidence ranges; incidences four at a time; neighbour
// alphas) and sums each vertex's incidences in order.  lo/hi: the lane's
// smallest and largest vertex value.
template <int G, int KV, bool WANT_X, class TM>
__device__ __forceinline__ void stage_vertex_field(TM &M, const DevMesh &m, const ReconParams &p, int sl, int q,
                                                   int64_t v0, int nv, double xP0, double xP1, double xP2, double &lo,
                                                   double &hi) {
  const double *w = p.vertex_mode ? m.vc_wmean : m.vc_w;
  for (int i0 = q; i0 < nv; i0 += KV * G) {
    int gv[KV];
    int64_t jb[KV], je[KV];
    double px[KV], py[KV], pz[KV], ph[KV];
#pragma unroll
    for (int t = 0; t < KV; ++t) {
      const int i = i0 + t * G;
      gv[t] = i < nv ? m.cv_gid[v0 + i] : -1;
    }
#pragma unroll
    for (int t = 0; t < KV; ++t) {
      const bool in = gv[t] >= 0;
      if constexpr (WANT_X) {
        px[t] = in ? m.xyz[gv[t]] : 0.0;
        py[t] = in ? m.xyz[m.n_verts + gv[t]] : 0.0;
        pz[t] = in ? m.xyz[2 * m.n_verts + gv[t]] : 0.0;
      }
      ph[t] = 0.0;
      if (p.phi_override) {
        ph[t] = in ? p.phi_override[gv[t]] : 0.0;
        jb[t] = je[t] = 0;
      } else {
        jb[t] = in ? m.vc_off[gv[t]] : 0;
        je[t] = in ? m.vc_off[gv[t] + 1] : 0;
      }
    }
    bool more = true;
    for (int c4 = 0; more; c4 += 4) {
      int cc[KV][4];
      double ww[KV][4], aa[KV][4];
#pragma unroll
      for (int t = 0; t < KV; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t jj = jb[t] + c4 + u;
          const bool in = jj < je[t];
          cc[t][u] = in ? m.vc_cell[jj] : 0;
          ww[t][u] = in ? w[jj] : 0.0;
        }
#pragma unroll
      for (int t = 0; t < KV; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) aa[t][u] = (jb[t] + c4 + u < je[t]) ? p.alpha[cc[t][u]] : 0.0;
      more = false;
#pragma unroll
      for (int t = 0; t < KV; ++t) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (jb[t] + c4 + u < je[t]) ph[t] += ww[t][u] * aa[t][u];
        more = more || jb[t] + c4 + 4 < je[t];
      }
    }
#pragma unroll
    for (int t = 0; t < KV; ++t) {
      const int i = i0 + t * G;
      if (i < nv) {
        if constexpr (WANT_X) {
          M.X[0][i][sl] = px[t] - xP0;
          M.X[1][i][sl] = py[t] - xP1;
          M.X[2][i][sl] = pz[t] - xP2;
        }
        M.phi[i][sl] = ph[t];
        lo = fmin(lo, ph[t]);
        hi = fmax(hi, ph[t]);
      }
    }
  }
}

// Waves per SIMD a build's register budget is sized for: enough for every
// wave its LDS lets a CU hold (rounded up over the four SIMDs), at most 3
// (168 VGPRs: the search state and one face walk fit without spills; a
// 4-wave budget of 128 VGPRs spills).  The learned builds are held to the
// same budget: what does not fit spills in the staging and network phases,
// once per batch, not in the search.
constexpr int thin_occupancy(int bytes) {
  return (160 * 1024) / bytes >= 9 ? 3 : ((160 * 1024) / bytes + 3) / 4;
}

template <int G, int NV, int NF, int NL, int NE, bool NET>
__global__ __launch_bounds__(64, (thin_occupancy((int)sizeof(ThinMem<64 / G, NV, NF, NL, NE>))))
void recon_thin_kernel(ReconParams p) {
  constexpr int C = 64 / G;
  __shared__ ThinMem<C, NV, NF, NL, NE> M;
  ThinNet<C> &T = M.net;
  const int lane = threadIdx.x, sl = lane / G, q = lane % G;
  const DevMesh &m = p.m;
  const int64_t N = m.n_cells;
  const int64_t cap = p.out.cap;
  int64_t count = p.entries ? (int64_t)*p.entry_count : (int64_t)p.counts[0];
  if (count > cap) count = cap;
  const int64_t nbatch = (count + C - 1) / C;
  // this XCD's batches (runs of kRunCells cells): the first one per
  // workgroup by its index, the rest claimed from the XCD's counter
  constexpr int kRun = kRunCells / C;
  const int xcd = (int)(blockIdx.x % kXcd);
  const int64_t nx = xcd_count<kRun>(nbatch, xcd);
  const int64_t wx = ((int64_t)gridDim.x - xcd + kXcd - 1) / kXcd;
  unsigned int *claim = reinterpret_cast<unsigned int *>(p.queue + (1 + xcd) * kQueueStride);
  for (int64_t ix = blockIdx.x / kXcd; ix < nx;) {
    const int64_t bt = xcd_batch<kRun>(ix, xcd);
    const int64_t j = bt * C + sl;
    const bool active = j < count;
    // ---- phase 1, per cell: checks and staging
    int64_t k = 0, f0 = 0;
    int P = 0, nf = 0, nv = 0, nl = 0, ne = 0, st = VOFPC_CELL_OK, it = 0;
    double a = 0.0, VP = 1.0, pmin = 0.0, pmax = 0.0;
    bool have_field = false;
    double s_out = __builtin_nan(""), A_out = 0, d_out = 0, n0 = 0, n1 = 0, n2 = 0, ag = 0.0;
    if (active) {
      k = p.entries ? (int64_t)p.entries[j] : j;
      P = p.mixed[k];
      a = p.alpha[P];
      ag = a;
      f0 = m.cell_face_off[P];
      nf = (int)(m.cell_face_off[P + 1] - f0);
      const int64_t v0 = m.cv_off[P];
      nv = (int)(m.cv_off[P + 1] - v0);
      const int64_t l0 = m.cl_off[P];
      nl = (int)(m.cl_off[P + 1] - l0);
      ne = nl / 2;   // a closed surface uses every edge twice
      if (!(a >= 0.0 && a <= 1.0)) {
        st = VOFPC_CELL_BAD_INPUT;
      } else if (!(a > p.eps && a < 1.0 - p.eps)) {
        st = VOFPC_CELL_NOT_MIXED;
      } else if (nv > NV || nf > NF || nl > NL || ne > NE) {
        st = VOFPC_CELL_BAD_INPUT;   // cannot happen: the launcher sizes the build by the class
      } else {
        const double xP0 = m.xc[P], xP1 = m.xc[N + P], xP2 = m.xc[2 * N + P];
        VP = m.V[P];
        // ---- stage the polyhedron: loop positions, face offsets and edges,
        // and the vertices with the inverse-distance vertex field.  The
        // loads of each part are issued together (topology into registers
        // first, then the vertices level by level: ids, positions and
        // incidence ranges, incidences, neighbour alphas), so their
        // latencies overlap instead of adding up.
        // (builds whose topology takes more than 40 registers per lane store
        // it straight to LDS after the vertices instead)
        constexpr int KL = (NL + G - 1) / G, KF = (NF + G - 1) / G, KE = (NE + G - 1) / G;
        constexpr bool kPre = 2 * KL + 2 * KF + KE <= 40;
        constexpr int KV = (NV + G - 1) / G < 2 ? (NV + G - 1) / G : 2;   // vertices per lane per round
        uint8_t tl[kPre ? KL : 1], te[kPre ? KL : 1], tfo[kPre ? KF : 1], tfs[kPre ? KF : 1];
        uint32_t tw[kPre ? KE : 1];
        if constexpr (kPre) {
#pragma unroll
        for (int t = 0; t < KL; ++t) {
          const int i = q + t * G;
          tl[t] = i < nl ? m.cl_lv[l0 + i] : (uint8_t)0;
          te[t] = i < nl ? (uint8_t)m.cl_eid[l0 + i] : (uint8_t)0;
        }
#pragma unroll
        for (int t = 0; t < KF; ++t) {
          const int f = q + t * G;
          tfo[t] = f < nf ? (uint8_t)m.cf_loff[f0 + f] : (uint8_t)0;
          tfs[t] = f < nf ? m.cf_lsz[f0 + f] : (uint8_t)0;
        }
#pragma unroll
        for (int t = 0; t < KE; ++t) {
          const int e = q + t * G;
          tw[t] = e < ne ? m.ce[(l0 >> 1) + e] : 0u;
        }
        }
        double lo_phi = __builtin_inf(), hi_phi = -__builtin_inf();
        stage_vertex_field<G, KV, true>(M, m, p, sl, q, v0, nv, xP0, xP1, xP2, lo_phi, hi_phi);
        if constexpr (kPre) {
#pragma unroll
          for (int t = 0; t < KL; ++t) {
            const int i = q + t * G;
            if (i < nl) {
              M.lv[i][sl] = tl[t];
              M.eid[i][sl] = te[t];
            }
          }
#pragma unroll
          for (int t = 0; t < KF; ++t) {
            const int f = q + t * G;
            if (f < nf) {
              M.foff[f][sl] = tfo[t];
              M.fsz[f][sl] = tfs[t];
            }
          }
#pragma unroll
          for (int t = 0; t < KE; ++t) {
            const int e = q + t * G;
            if (e < ne) {
              const uint32_t wv = tw[t];
              M.eu[e][sl] = (uint8_t)(wv & 0xffu);
              M.ev[e][sl] = (uint8_t)((wv >> 8) & 0xffu);
              M.ef1[e][sl] = (uint8_t)((wv >> 16) & 0xffu);
              M.ef2[e][sl] = (uint8_t)(wv >> 24);
            }
          }
        } else {
          for (int i = q; i < nl; i += G) {
            M.lv[i][sl] = m.cl_lv[l0 + i];
            M.eid[i][sl] = (uint8_t)m.cl_eid[l0 + i];
          }
          for (int f = q; f < nf; f += G) {
            M.foff[f][sl] = (uint8_t)m.cf_loff[f0 + f];
            M.fsz[f][sl] = m.cf_lsz[f0 + f];
          }
          for (int e = q; e < ne; e += G) {
            const uint32_t wv = m.ce[(l0 >> 1) + e];
            M.eu[e][sl] = (uint8_t)(wv & 0xffu);
            M.ev[e][sl] = (uint8_t)((wv >> 8) & 0xffu);
            M.ef1[e][sl] = (uint8_t)((wv >> 16) & 0xffu);
            M.ef2[e][sl] = (uint8_t)(wv >> 24);
          }
        }
        wave_sync();
        // the whole-edge volume term of each edge: its two faces' fan terms,
        // det(c1, u, v) + det(c2, v, u) with c = the face's first vertex
        for (int e = q; e < ne; e += G) {
          const int u = M.eu[e][sl], v = M.ev[e][sl];
          const int a1 = M.lv[M.foff[M.ef1[e][sl]][sl]][sl], a2 = M.lv[M.foff[M.ef2[e][sl]][sl]][sl];
          const double d0 = M.X[0][a1][sl] - M.X[0][a2][sl], d1 = M.X[1][a1][sl] - M.X[1][a2][sl],
                       d2 = M.X[2][a1][sl] - M.X[2][a2][sl];
          M.D[e][sl] = det3(d0, d1, d2, M.X[0][u][sl], M.X[1][u][sl], M.X[2][u][sl], M.X[0][v][sl], M.X[1][v][sl],
                            M.X[2][v][sl]);
        }
        pmin = tmin<G>(lo_phi);
        pmax = tmax<G>(hi_phi);
        have_field = true;
        wave_sync();
        if (pmax - pmin <= 1e-12) {
          // degenerate vertex field: linear alpha from the plain least-squares
          // gradient over the interior face neighbours
          st = VOFPC_CELL_DEGENERATE;
          double gxx = 0, gyy = 0, gzz = 0, gxy = 0, gxz = 0, gyz = 0, b0 = 0, b1 = 0, b2 = 0;
          for (int f = q; f < nf; f += G) {
            const int qq = m.cf_nbr[f0 + f];
            if (qq < 0) continue;
            const double r0 = m.xc[qq] - xP0, r1 = m.xc[N + qq] - xP1, r2 = m.xc[2 * N + qq] - xP2;
            const double dv = p.alpha[qq] - a;
            gxx += r0 * r0; gyy += r1 * r1; gzz += r2 * r2; gxy += r0 * r1; gxz += r0 * r2; gyz += r1 * r2;
            b0 += r0 * dv; b1 += r1 * dv; b2 += r2 * dv;
          }
          gxx = tsum<G>(gxx); gyy = tsum<G>(gyy); gzz = tsum<G>(gzz);
          gxy = tsum<G>(gxy); gxz = tsum<G>(gxz); gyz = tsum<G>(gyz);
          b0 = tsum<G>(b0); b1 = tsum<G>(b1); b2 = tsum<G>(b2);
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
          lo_phi = __builtin_inf();
          hi_phi = -__builtin_inf();
          for (int i = q; i < nv; i += G) {
            const double ph = a + (g0 * M.X[0][i][sl] + g1 * M.X[1][i][sl] + g2 * M.X[2][i][sl]);
            M.phi[i][sl] = ph;
            lo_phi = fmin(lo_phi, ph);
            hi_phi = fmax(hi_phi, ph);
          }
          pmin = tmin<G>(lo_phi);
          pmax = tmax<G>(hi_phi);
          if (pmax - pmin <= 1e-12) have_field = false;
          wave_sync();
        }
      }
    }
    // ---- phase 2: the narrowed bracket of every cell with a vertex field,
    // from the network (run on the wavefront's cells together) or the caller
    double hl = 0.0, hh = 0.0, hm = 0.0;
    bool hint = false;
    if constexpr (NET) {
      const bool row = active && have_field && st == VOFPC_CELL_OK;   // degenerate fields skip the network
      // rows of a tile beyond the wavefront's cells are zero (the bytes are
      // the evaluations' scratch in between)
      for (int i = lane; i < (ThinNet<C>::R - C) * net::kIn; i += 64) T.x[C + i / net::kIn][i % net::kIn] = 0;
      if (row) {
        cell_features<G>(M, T, sl, q, p, P, a, nv, nf, f0, pmin, pmax - pmin);
      } else {
        for (int i = q; i < net::kIn; i += G) T.x[sl][i] = 0;
      }
      wave_sync();
      net_tiles<C>(T, p.net_wb, p.net_master, lane);
      if (row) {
        const float u = T.u[sl];
        if (!isnan(u)) {
          const double Wd = pmax - pmin;
          const double uc = u < 0.f ? 0.0 : (u > 1.f ? 1.0 : (double)u);
          const double sh = pmin + uc * Wd, dl = p.net_delta * Wd;
          hl = sh - dl;
          hh = sh + dl;
          if (q == 0 && p.net_lo) {
            p.net_lo[k] = hl;
            p.net_hi[k] = hh;
          }
          hl = hl > pmin ? hl : pmin;
          hh = hh < pmax ? hh : pmax;
          if (hl > hh) { hl = pmin; hh = pmax; }
          hm = sh < hl ? hl : (sh > hh ? hh : sh);
          hint = true;
        } else if (q == 0 && p.net_lo) {
          p.net_lo[k] = __builtin_nan("");
          p.net_hi[k] = __builtin_nan("");
        }
      } else if (active && q == 0 && p.net_lo) {
        p.net_lo[k] = __builtin_nan("");
        p.net_hi[k] = __builtin_nan("");
      }
      wave_sync();
    } else {
      if (active && have_field && p.use_hint) {
        hl = p.hint_lo[k];
        hh = p.hint_hi[k];
        if (!isnan(hl) && !isnan(hh)) {
          hl = hl > pmin ? hl : pmin;
          hh = hh < pmax ? hh : pmax;
          if (hl > hh) { hl = pmin; hh = pmax; }
          hm = hl + (hh - hl) / 2.0;
          hint = true;
        }
      }
    }
    // ---- phase 3, per cell: the search and the outputs
    if (active) {
        if (have_field) {
          // reference point of the loop sums: the vertex of largest value when
          // the cell is mostly vapour (a small liquid piece sits at it), else
          // the vertex of smallest value (the smallest index among ties)
          double ref[3];
          {
            const bool top = a < 0.5;
            const double want = top ? pmax : pmin;
            int cand = 0x7fffffff;
            for (int i = q; i < nv; i += G)
              if (M.phi[i][sl] == want && i < cand) cand = i;
            cand = tmin_i<G>(cand);
            ref[0] = M.X[0][cand][sl];
            ref[1] = M.X[1][cand][sl];
            ref[2] = M.X[2][cand][sl];
          }
          // One evaluation site; the phase decides where the next one is:
          // the fixed isovalue, the centre of a narrowed bracket and then its
          // end on the root's side, the search estimate, or the bracket end
          // kept when the search cannot stop.
          enum { kFixed, kHintMid, kHintEnd, kSearch, kFinal };
          CutRes c;
          c.err = false;
          double s = __builtin_nan("");
          double lo = pmin, hi = pmax, rlo = 1.0 - a, rhi = -a, rm = 0.0;
          const double iVP = 1.0 / VP;
          const double tol = p.tol_rel * (a < 1.0 - a ? a : 1.0 - a);
          // Brent's method (Brent 1973, ch. 4) on the residual r(s) = V(s)/V_P - alpha:
          // xb is the bracket end of smaller |r|, xa the other end, xc the
          // previous xb, xd the one before; the estimate is inverse quadratic
          // interpolation through (xa, xb, xc) when the three residuals differ,
          // else the secant through xa and xb, replaced by the midpoint when it
          // falls outside the quarter of the bracket next to xb or does not
          // shrink fast enough against the previous steps.
          double xa = 0, fa = 0, xb = 0, fb = 0, xc = 0, fc = 0, xd = 0;
          bool bis = true, started = false, collapsed = false;
          // a jump of V: where a face with four or more crossings switches its
          // pairing (at its vertex-value mean) or a loop pinches at a vertex
          // (at that vertex's value), V may step over alpha V_P and the search
          // bisects down to two ulps.  From the second bisection step in a row
          // on a bracket narrower than a hundredth of [phi_min, phi_max], such
          // a value inside the bracket (the one nearest the bisection point)
          // is cut instead, then the adjacent double on the root's side: a
          // sign change between the two pins the bracket to one ulp (at most
          // four tries per cell).
          double xj = 0.0, rlast = 0.0;
          int jtries = 0, nbis = 0;
          bool jnext = false;
          int ph = p.fixed_iso ? kFixed : (hint ? kHintMid : kSearch);
          while (true) {
            double se = 0.0;
            if (ph == kSearch) {
              if (!started) {
                // the bracket [lo, hi] (full, or what the narrowed bracket's
                // check left) starts the method
                xa = lo; fa = rlo; xb = hi; fb = rhi;
                if (fabs(fa) < fabs(fb)) {
                  xa = hi; fa = rhi; xb = lo; fb = rlo;
                }
                xc = xa; fc = fa; xd = xa;
                bis = true;
                started = true;
              }
              const double big = fabs(xa) > fabs(xb) ? fabs(xa) : fabs(xb);
              if (fabs(xb - xa) <= 2.0 * ulp_of(big)) {
                collapsed = true;
                ph = kFinal;
              } else if (it >= p.max_iter) {
                st = VOFPC_CELL_MAX_ITER;
                ph = kFinal;
              } else {
                const double blo = xa < xb ? xa : xb, bhi = xa < xb ? xb : xa;
                bool pinned = false;
                if (jnext) {
                  // the double next to the tried face mean, on the root's side
                  jnext = false;
                  const double nb = rlast > 0 ? nextafter(xj, __builtin_inf()) : nextafter(xj, -__builtin_inf());
                  if (nb > blo && nb < bhi) {
                    se = nb;
                    pinned = true;
                  }
                }
                if (!pinned) {
                  if (fa != fc && fb != fc) se = iqi1(xa, fa, xb, fb, xc, fc);
                  else se = xb - fb * qdiv(xb - xa, fb - fa);
                  const double q0 = (3.0 * xa + xb) * 0.25;
                  const bool inside = q0 < xb ? (se > q0 && se < xb) : (se > xb && se < q0);
                  const double du = 4.0 * ulp_of(xb);
                  const double lastd = bis ? fabs(xb - xc) : fabs(xc - xd);
                  if (!inside || fabs(se - xb) >= 0.5 * lastd || lastd < du) {
                    se = xa + (xb - xa) * 0.5;
                    bis = true;
                  } else {
                    bis = false;
                  }
                  nbis = bis ? nbis + 1 : 0;
                  if (nbis >= 2 && it > 0 && jtries < 4 && bhi - blo <= 0.01 * (pmax - pmin)) {
                    // candidates: the means of the faces with four or more
                    // crossings at the last evaluation, and the vertex values
                    const double mid = se;
                    double bd = __builtin_inf(), bv = __builtin_inf();
                    for (int f = q; f < nf; f += G) {
                      if (M.cnt[f][sl] < 4) continue;
                      const int o = M.foff[f][sl], n = M.fsz[f][sl];
                      double fm = 0.0;
                      for (int k2 = 0; k2 < n; ++k2) fm += M.phi[M.lv[o + k2][sl]][sl];
                      const double sj = fm / (double)n;
                      const double d = fabs(sj - mid);
                      if (sj > blo && sj < bhi && sj != xj && (d < bd || (d == bd && sj < bv))) {
                        bd = d;
                        bv = sj;
                      }
                    }
                    for (int i = q; i < nv; i += G) {
                      const double sj = M.phi[i][sl];
                      const double d = fabs(sj - mid);
                      if (sj > blo && sj < bhi && sj != xj && (d < bd || (d == bd && sj < bv))) {
                        bd = d;
                        bv = sj;
                      }
                    }
                    const double bdm = tmin<G>(bd);
                    const double cj = tmin<G>(bd == bdm ? bv : __builtin_inf());
                    if (cj < __builtin_inf()) {
                      se = cj;
                      xj = cj;
                      jnext = true;
                      ++jtries;
                    }
                  }
                }
              }
            }
            if (ph == kFinal) {
              se = xb;
            } else if (ph == kFixed) {
              se = p.iso;
            } else if (ph == kHintMid) {
              se = hm;
            } else if (ph == kHintEnd) {
              se = rm > 0 ? hh : hl;
            }
            const CutRes cf = thin_eval<G>(M, sl, q, nf, ne, se, ref);
            ++it;
            const double r = cf.V * iVP - a;
            if (ph == kFixed || ph == kFinal || fabs(r) <= tol) {
              s = se;
              c = cf;
              if (ph == kFinal && collapsed && fabs(fb) > 1e-10) st = VOFPC_CELL_NO_ROOT;
              break;
            }
            if (ph == kHintMid) {
              // the residual at the centre tells the side of the root: that
              // half of the bracket is checked by a cut at its end
              rm = r;
              if (r > 0) {
                lo = se; rlo = r;
              } else {
                hi = se; rhi = r;
              }
              if ((r > 0 ? hh : hl) == se) {
                // the centre is the end: the root lies beyond it
                if (st == VOFPC_CELL_OK) st = VOFPC_CELL_LEARNED_FALLBACK;
                ph = kSearch;
              } else {
                ph = kHintEnd;
              }
              continue;
            }
            if (ph == kHintEnd) {
              // the bracket holds when its end is past the root; otherwise the
              // root lies beyond that end
              const bool up = rm > 0;
              if (up ? r < 0 : r > 0) {
                if (up) { hi = se; rhi = r; } else { lo = se; rlo = r; }
              } else {
                if (up) { lo = se; rlo = r; } else { hi = se; rhi = r; }
                if (st == VOFPC_CELL_OK) st = VOFPC_CELL_LEARNED_FALLBACK;
              }
              ph = kSearch;
              continue;
            }
            // keep the end across the root from the estimate; xb the end of
            // smaller residual
            rlast = r;
            xd = xc;
            xc = xb; fc = fb;
            if ((fa > 0) != (r > 0)) {
              xb = se; fb = r;
            } else {
              xa = se; fa = r;
            }
            if (fabs(fa) < fabs(fb)) {
              const double tx = xa, tf = fa;
              xa = xb; fa = fb; xb = tx; fb = tf;
            }
          }
          const bool cut_ok = true;
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
      if (q == 0) {
        if (p.mf.gradT) {
          // mass transfer of the entry (one-sided form, as vofpc_mass_transfer)
          double md = 0.0;
          if (A_out > 0.0) {
            const double gn = p.mf.gradT[P] * n0 + p.mf.gradT[N + P] * n1 + p.mf.gradT[2 * N + P] * n2;
            const double gl = (a >= 0.5) ? gn : 0.0, gv = (a >= 0.5) ? 0.0 : gn;
            const double ql = p.mf.k_l * gl * A_out;
            const double qv = -p.mf.k_v * gv * A_out;
            md = (ql + qv) / (p.mf.h_lv * m.V[P]);
          }
          p.mf.mdot[k] = md;
          p.mf.Qdot[k] = -md * p.mf.h_lv;
        }
        p.out.s[k] = s_out;
        p.out.n[k] = n0; p.out.n[cap + k] = n1; p.out.n[2 * cap + k] = n2;
        p.out.A[k] = A_out;
        p.out.d[k] = d_out;
        p.out.alpha_got[k] = ag;
        p.out.status[k] = st;
        p.out.iters[k] = it;
      }
    }
    // next batch: a wrapping increment, so the XCD's nx claims (one per
    // batch done) bring its counter back to zero
    int nb = 0;
    if (lane == 0) nb = (int)atomicInc(claim, (unsigned int)(nx - 1));
    ix = wx + __builtin_amdgcn_readfirstlane(nb);
    wave_sync();
  }
}

// ---- the learned bracket in a pass of its own
// In the builds whose wavefronts hold fewer than 16 cells (G >= 8) the
// network's 16-row tile would run mostly empty inside the reconstruction.
// This pass takes 16 cells per wavefront (4 lanes each), stages only their
// vertex field, computes the features, runs one full tile and writes each
// entry's bracket [sh - d, sh + d] around the predicted isovalue sh (NaN
// where the reconstruction would run no network: not mixed, bad input,
// degenerate field).  The reconstruction then checks it as a caller's
// bracket.
template <int NVM>
struct PassMem {
  double phi[NVM][17];
  uint8_t link[NVM][16];
  ThinNet<16> net;
};

template <int NVM>
__global__ __launch_bounds__(64) void bracket_pass_kernel(ReconParams p, double *hlo, double *hhi) {
  constexpr int G = 4, C = 16;
  __shared__ PassMem<NVM> M;
  ThinNet<C> &T = M.net;
  const int lane = threadIdx.x, sl = lane / G, q = lane % G;
  const DevMesh &m = p.m;
  int64_t count = p.entries ? (int64_t)*p.entry_count : (int64_t)p.counts[0];
  if (count > p.out.cap) count = p.out.cap;
  const int64_t nbatch = (count + C - 1) / C;
  // this XCD's batches (runs of kRunCells cells), a fixed share per workgroup
  constexpr int kRun = kRunCells / C;
  const int xcd = (int)(blockIdx.x % kXcd);
  const int64_t nx = xcd_count<kRun>(nbatch, xcd);
  const int64_t wx = ((int64_t)gridDim.x - xcd + kXcd - 1) / kXcd;
  for (int64_t ix = blockIdx.x / kXcd; ix < nx; ix += wx) {
    const int64_t bt = xcd_batch<kRun>(ix, xcd);
    const int64_t j = bt * C + sl;
    const bool active = j < count;
    int64_t k = 0, f0 = 0;
    int P = 0, nf = 0, nv = 0;
    double a = 0.0, pmin = 0.0, pmax = 0.0;
    bool row = false;
    if (active) {
      k = p.entries ? (int64_t)p.entries[j] : j;
      P = p.mixed[k];
      a = p.alpha[P];
      f0 = m.cell_face_off[P];
      nf = (int)(m.cell_face_off[P + 1] - f0);
      const int64_t v0 = m.cv_off[P];
      nv = (int)(m.cv_off[P + 1] - v0);
      if (a > p.eps && a < 1.0 - p.eps && nv <= NVM) {   // a NaN alpha fails both tests
        double lo = __builtin_inf(), hi = -__builtin_inf();
        stage_vertex_field<G, 2, false>(M, m, p, sl, q, v0, nv, 0.0, 0.0, 0.0, lo, hi);
        pmin = tmin<G>(lo);
        pmax = tmax<G>(hi);
        row = pmax - pmin > 1e-12;
      }
    }
    wave_sync();
    if (row) {
      cell_features<G>(M, T, sl, q, p, P, a, nv, nf, f0, pmin, pmax - pmin);
    } else {
      for (int i = q; i < net::kIn; i += G) T.x[sl][i] = 0;
    }
    wave_sync();
    net_tiles<C>(T, p.net_wb, p.net_master, lane);
    if (active && q == 0) {
      double lo = __builtin_nan(""), hi = __builtin_nan("");
      const float u = T.u[sl];
      if (row && !isnan(u)) {
        const double Wd = pmax - pmin;
        const double uc = u < 0.f ? 0.0 : (u > 1.f ? 1.0 : (double)u);
        const double sh = pmin + uc * Wd, dl = p.net_delta * Wd;
        lo = sh - dl;
        hi = sh + dl;
      }
      hlo[k] = lo;
      hhi[k] = hi;
    }
    wave_sync();
  }
}

template <int NVM>
vofpc_status launch_pass(vofpc_ctx ctx, const ReconParams &p, int64_t n_entries, double *hlo, double *hhi) {
  int blocks_per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks_per_cu, bracket_pass_kernel<NVM>, 64, 0);
  if (e != hipSuccess || blocks_per_cu <= 0) blocks_per_cu = 4;
  int64_t grid = (int64_t)ctx->n_cu * blocks_per_cu;
  const int64_t need = (n_entries + 15) / 16;
  if (grid > need) grid = need;
  if (grid < 1) grid = 1;
  bracket_pass_kernel<NVM><<<(unsigned)grid, 64, 0, ctx->stream>>>(p, hlo, hhi);
  VOFPC_HIP(hipGetLastError());
  return VOFPC_OK;
}

template <int G, int NV, int NF, int NL, int NE, bool NET>
vofpc_status launch_net(vofpc_ctx ctx, const ReconParams &p, int64_t n_entries) {
  constexpr int C = 64 / G;
  int blocks_per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks_per_cu,
                                                              recon_thin_kernel<G, NV, NF, NL, NE, NET>, 64, 0);
  if (e != hipSuccess || blocks_per_cu <= 0) blocks_per_cu = 1;
  int64_t grid = (int64_t)ctx->n_cu * blocks_per_cu;
  const int64_t need = (n_entries + C - 1) / C;
  if (grid > need) grid = need;
  if (grid < 1) grid = 1;
  recon_thin_kernel<G, NV, NF, NL, NE, NET><<<(unsigned)grid, 64, 0, ctx->stream>>>(p);
  VOFPC_HIP(hipGetLastError());
  return VOFPC_OK;
}

// the plain build, or the build that runs the network (learned form)
template <int G, int NV, int NF, int NL, int NE>
vofpc_status launch_t(vofpc_ctx ctx, const ReconParams &p, int64_t n_entries) {
  if (p.net_wb) return launch_net<G, NV, NF, NL, NE, true>(ctx, p, n_entries);
  return launch_net<G, NV, NF, NL, NE, false>(ctx, p, n_entries);
}

// The builds: class 0 in two sizes (hexahedra and smaller: G = 1, 2, 4; the
// class caps: G = 2, 4), class 1 at its caps (G = 4, 8, 16).
struct ThinCaps {
  int nv, nf, nl, ne;
};
constexpr ThinCaps kHex{8, 6, 24, 12}, kC0{16, 8, 48, 24}, kC1{32, 20, 96, 48}, kC2{48, 32, 128, 64};

__host__ bool fits(const ThinCaps &t, const int64_t cmax[4]) {
  return cmax[0] <= t.nv && cmax[1] <= t.nf && cmax[2] <= t.nl && cmax[3] <= t.ne;
}

}  // namespace

bool thin_available(int c, int G, const int64_t cmax[4]) {
  if (c == 0) return fits(kHex, cmax) ? (G == 1 || G == 2 || G == 4) : ((G == 2 || G == 4) && fits(kC0, cmax));
  if (c == 1) return (G == 4 || G == 8 || G == 16) && fits(kC1, cmax);
  if (c == 2) return (G == 4 || G == 8 || G == 16) && fits(kC2, cmax);
  return false;
}

vofpc_status launch_bracket_pass(vofpc_ctx ctx, const ReconParams &p, int64_t n_entries, int c, double *hlo,
                                 double *hhi) {
  VOFPC_REQUIRE(c == 1 || c == 2, VOFPC_E_INVALID_ARG, "reconstruct: no bracket pass for this class");
  return c == 1 ? launch_pass<kC1.nv>(ctx, p, n_entries, hlo, hhi) : launch_pass<kC2.nv>(ctx, p, n_entries, hlo, hhi);
}

vofpc_status launch_thin(vofpc_ctx ctx, const ReconParams &p, int64_t n_entries, int c, int G,
                         const int64_t cmax[4]) {
  VOFPC_REQUIRE(thin_available(c, G, cmax), VOFPC_E_INVALID_ARG, "reconstruct: no group build for this class");
  if (c == 0) {
    if (fits(kHex, cmax)) {
      if (G == 1) return launch_t<1, kHex.nv, kHex.nf, kHex.nl, kHex.ne>(ctx, p, n_entries);
      if (G == 2) return launch_t<2, kHex.nv, kHex.nf, kHex.nl, kHex.ne>(ctx, p, n_entries);
      return launch_t<4, kHex.nv, kHex.nf, kHex.nl, kHex.ne>(ctx, p, n_entries);
    }
    if (G == 2) return launch_t<2, kC0.nv, kC0.nf, kC0.nl, kC0.ne>(ctx, p, n_entries);
    return launch_t<4, kC0.nv, kC0.nf, kC0.nl, kC0.ne>(ctx, p, n_entries);
  }
  if (c == 1) {
    if (G == 4) return launch_t<4, kC1.nv, kC1.nf, kC1.nl, kC1.ne>(ctx, p, n_entries);
    if (G == 8) return launch_t<8, kC1.nv, kC1.nf, kC1.nl, kC1.ne>(ctx, p, n_entries);
    return launch_t<16, kC1.nv, kC1.nf, kC1.nl, kC1.ne>(ctx, p, n_entries);
  }
  if (G == 4) return launch_t<4, kC2.nv, kC2.nf, kC2.nl, kC2.ne>(ctx, p, n_entries);
  if (G == 8) return launch_t<8, kC2.nv, kC2.nf, kC2.nl, kC2.ne>(ctx, p, n_entries);
  return launch_t<16, kC2.nv, kC2.nf, kC2.nl, kC2.ne>(ctx, p, n_entries);
}

}  // namespace vofpc
