// Volume-matched iso-polygon reconstruction of the mixed cells.
//
// One cell per wavefront (a block is one wavefront of 64 lanes).  The cell's
// polyhedron is staged in LDS: vertex
// positions relative to the centroid, the vertex field, the outward face
// loops as local vertex ids with a local edge id and the reciprocal of the
// vertex-value difference for every loop position.
//
// Full volume evaluation at isovalue s (faces spread over the lanes):
//   - each face lane walks its loop: liquid edges and the liquid parts of the
//     cut edges add to the divergence-theorem sum; exits (liquid -> vapour)
//     and entries (vapour -> liquid) are bit masks over loop positions; each
//     exit is paired with an entry (the next one in loop order when the
//     face-mean value is >= s or the face has two crossings, else the
//     previous one), giving a chord exit -> entry that closes the face's
//     liquid polygon;
//   - chords are linked into iso-loops (the loop continues in the face whose
//     entry edge is this chord's exit edge) and labelled by pointer jumping;
//   - each loop is fanned from its length-weighted polyline centroid, which
//     adds its volume share, its area vector and its centre.
// Crossing points follow Eq. edge_intersection, computed from the liquid end
// of the edge so both faces sharing an edge get the same point.
//
// Fixed-topology evaluation: the set of cut edges, their pairing and the
// loops only change when s crosses a vertex value or a face-mean value.  A
// full evaluation records, per chord (one chord per lane), the edge it leaves
// through, its face centre, its neighbours on the loop and the constant sum
// over the fully liquid edges, valid up to the neighbouring breakpoints; an
// isovalue inside that interval then only moves the crossing points along
// their edges and redoes the chord and loop sums.  Two such records are kept,
// so a bracket closing in on a breakpoint from both sides stays on the short
// path.  It evaluates the same volume function (same construction, fewer
// operations) at the same isovalues.
//
// The isovalue search keeps a bracket [lo, hi] with V(lo) > alpha V_P > V(hi)
// and picks its isovalues by regula falsi (Illinois weight) and inverse
// quadratic interpolation, with a bisection step after a slow update, until
// |V/V_P - alpha| <= tol_rel min(alpha,1-alpha); when the bracket collapses
// first, the end nearer to alpha V_P is kept.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>

#include "recon_common.h"
#include "mlp_core.h"

namespace vofpc {


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


// Chord data of a fixed topology, one chord per lane (see the file comment),
// valid for isovalues in (bp_lo, bp_hi].
template <int W>
struct FastSlot {
  double xi[3][W];   // liquid end of the exit edge
  double dx[3][W];   // vapour end minus liquid end
  double phi_i[W];   // value at the liquid end
  double inv[W];     // 1/(phi_vapour - phi_liquid)
  double cf[3][W];   // centre of the chord's face
  double xn[3][W];   // liquid end of the entry edge
  double c_full;     // sum over the fully liquid face edges
  double bp_lo, bp_hi;
  uint8_t prev[W], next[W], lab[W];
  int nch, nloops, valid;
};

constexpr int kSlotChords = 16;   // chords a cached topology can hold

template <int W, int NV, int NF, int NL, int NCH>
struct GroupMem {
  double X[3][NV];
  double phi[NV];
  double cf[3][NF];
  double fmean[NF];
  double inv[NL];         // 1/(phi[next] - phi[this]) of each loop position
  FastSlot<W> fs[2];
  uint16_t ch_xe[NCH];    // chord exit edge id
  uint16_t ch_ne[NCH];    // chord entry edge id
  uint16_t ch_face[NCH];  // chord face
  uint16_t ch_xpos[NCH];  // loop position of the exit edge
  uint16_t by_entry[NCH]; // chord entering through edge e
  uint16_t by_exit[NCH];  // chord leaving through edge e
  uint16_t lab[2][NCH > 64 ? NCH : 1];   // loop labelling through LDS (more chords than lanes)
  uint16_t jmp[2][NCH > 64 ? NCH : 1];
  uint16_t floff[NF];
  uint16_t eid[NL];
  double sp_s[8];                         // isovalues of a parallel round
  double end_res[2][8];                   // cut at the current bracket ends (lo, hi)
  double ept[3][NCH];                     // crossing point of each cut edge (by edge id)
  uint64_t fex[NF], fen[NF];              // exit / entry bit masks of each face
  uint16_t pnext[NL];                     // next loop position of the same face
  uint8_t pface[NL];                      // face of a loop position
  uint8_t pk[NL];                         // index of the position within its face
  uint8_t fsz[NF];
  uint8_t lv[NL];
  // bracket network: face sums, input row and hidden activations
  double nsum[20];
  alignas(16) uint16_t nx[net::kIn];
  alignas(16) uint16_t nh1[net::kHid];
  alignas(16) uint16_t nh2[net::kHid];
};



__device__ __forceinline__ int next_bit_after(uint64_t mask, int q) {
  uint64_t hi = (q >= 63) ? 0ull : (mask & (~0ull << (q + 1)));
  return hi ? __ffsll((long long)hi) - 1 : __ffsll((long long)mask) - 1;
}
__device__ __forceinline__ int prev_bit_before(uint64_t mask, int q) {
  uint64_t lo = (q == 0) ? 0ull : (mask & (~0ull >> (64 - q)));
  return lo ? 63 - __clzll((long long)lo) : 63 - __clzll((long long)mask);
}

// crossing point on loop position `pos` (edge a -> b), from the liquid end
template <class GM>
__device__ __forceinline__ void crossing_at(const GM &L, int pos, int a, int b, double s, double &p0, double &p1,
                                            double &p2) {
  const double iv = L.inv[pos];  // 1/(phi_b - phi_a); from b the reciprocal is -iv
  int i, j;
  double lam;
  if (L.phi[a] >= s) {
    i = a; j = b; lam = (s - L.phi[a]) * iv;
  } else {
    i = b; j = a; lam = (s - L.phi[b]) * (-iv);
  }
  p0 = L.X[0][i] + lam * (L.X[0][j] - L.X[0][i]);
  p1 = L.X[1][i] + lam * (L.X[1][j] - L.X[1][i]);
  p2 = L.X[2][i] + lam * (L.X[2][j] - L.X[2][i]);
}

// Sums of one loop over the lanes selected by `mine`: polyline centroid,
// fan volume, area vector.
template <int W>
__device__ __forceinline__ void one_loop(bool mine, double len, double p0, double p1, double p2, double q0, double q1,
                                         double q2, double first0, double first1, double first2, double &Vi,
                                         double &S0, double &S1, double &S2, double &Asum, double &cw0, double &cw1,
                                         double &cw2) {
  double l = mine ? len : 0.0;
  double m0 = mine ? len * (p0 + q0) : 0.0;
  double m1 = mine ? len * (p1 + q1) : 0.0;
  double m2 = mine ? len * (p2 + q2) : 0.0;
  l = gsum<W>(l); m0 = gsum<W>(m0); m1 = gsum<W>(m1); m2 = gsum<W>(m2);
  double k0, k1, k2;
  if (l > 0) {
    const double h = 0.5 / l;
    k0 = m0 * h; k1 = m1 * h; k2 = m2 * h;
  } else {
    k0 = first0; k1 = first1; k2 = first2;
  }
  double vi = 0, t0 = 0, t1 = 0, t2 = 0;
  if (mine) {
    vi = det3(k0, k1, k2, p0, p1, p2, q0, q1, q2);
    const double u0 = p0 - k0, u1 = p1 - k1, u2 = p2 - k2;
    const double w0 = q0 - k0, w1 = q1 - k1, w2 = q2 - k2;
    // the fan is oriented out of the liquid; the normal is the opposite
    t0 = -0.5 * (u1 * w2 - u2 * w1);
    t1 = -0.5 * (u2 * w0 - u0 * w2);
    t2 = -0.5 * (u0 * w1 - u1 * w0);
  }
  vi = gsum<W>(vi); t0 = gsum<W>(t0); t1 = gsum<W>(t1); t2 = gsum<W>(t2);
  const double Ak = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
  Vi += vi;
  S0 += t0; S1 += t1; S2 += t2;
  Asum += Ak;
  cw0 += Ak * k0; cw1 += Ak * k1; cw2 += Ak * k2;
}

// Loop sums with one chord per lane (nch <= W): lane c holds the loop point
// p (exit point of chord c), the lane of the next point on its loop and its
// loop label (smallest chord index on the loop; idle lanes are not valid).
// nloops is the number of loops when known, else -1.
template <int W>
__device__ __forceinline__ void loops_reg(int lane, bool valid, double p0, double p1, double p2, int next, int lab,
                                          int nloops, CutRes &R) {
  const double q0 = __shfl(p0, next, W), q1 = __shfl(p1, next, W), q2 = __shfl(p2, next, W);
  const double d0 = q0 - p0, d1 = q1 - p1, d2 = q2 - p2;
  const double len = valid ? sqrt(d0 * d0 + d1 * d1 + d2 * d2) : 0.0;
  double Vi = 0, S0 = 0, S1 = 0, S2 = 0, Asum = 0, cw0 = 0, cw1 = 0, cw2 = 0;
  if (nloops < 0) nloops = gsum_i<W>((valid && lab == lane) ? 1 : 0);
  // the loop's first point on every lane of the group: a register read of
  // one lane when the group is the whole wave, a shuffle within a segment
  auto bcast = [&](double v, int src) {
    if constexpr (W == 64) return readlane_d(v, __builtin_amdgcn_readfirstlane(src));
    else return __shfl(v, src, W);
  };
  if (nloops == 1) {
    const double f0 = bcast(p0, 0), f1 = bcast(p1, 0), f2 = bcast(p2, 0);
    one_loop<W>(valid, len, p0, p1, p2, q0, q1, q2, f0, f1, f2, Vi, S0, S1, S2, Asum, cw0, cw1, cw2);
  } else if (nloops > 1) {
    int prev = -1;
    while (true) {
      const int cand = gmin_i<W>((valid && lab == lane && lane > prev) ? lane : 0x7fffffff);
      if (cand == 0x7fffffff) break;
      const double f0 = bcast(p0, cand), f1 = bcast(p1, cand), f2 = bcast(p2, cand);
      one_loop<W>(valid && lab == cand, len, p0, p1, p2, q0, q1, q2, f0, f1, f2, Vi, S0, S1, S2, Asum, cw0, cw1,
                  cw2);
      prev = cand;
    }
  }
  R.V += Vi * (1.0 / 6.0);
  R.S0 = S0; R.S1 = S1; R.S2 = S2;
  R.A = Asum;
  if (Asum > 0) {
    const double ia = 1.0 / Asum;
    R.c0 = cw0 * ia; R.c1 = cw1 * ia; R.c2 = cw2 * ia;
  } else {
    R.c0 = R.c1 = R.c2 = 0;
  }
}

// Loop labels of the chords in registers by pointer jumping.
template <int W>
__device__ __forceinline__ int labels_reg(int lane, bool valid, int next, int nch) {
  int lab = valid ? lane : 0x7fff;
  int j = valid ? next : lane;
  for (int span = 1; span < nch; span <<= 1) {
    const int lj = __shfl(lab, j, W);
    const int jj = __shfl(j, j, W);
    lab = lab < lj ? lab : lj;
    j = jj;
  }
  return lab;
}

// Loop sums for more chords than lanes: labels and sums through LDS.
template <int W, class GM>
__device__ void loops_lds(GM &L, int lane, int nch, CutRes &R) {
  for (int c = lane; c < nch; c += W) {
    L.lab[0][c] = (uint16_t)c;
    L.jmp[0][c] = L.by_entry[L.ch_xe[c]];
  }
  wave_sync();
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
  double Vi = 0, S0 = 0, S1 = 0, S2 = 0, Asum = 0, cw0 = 0, cw1 = 0, cw2 = 0;
  int prev = -1;
  while (true) {
    int cand = 0x7fffffff;
    for (int c = lane; c < nch; c += W)
      if (L.lab[cur][c] == c && c > prev && c < cand) cand = c;
    cand = gmin_i<W>(cand);
    if (cand == 0x7fffffff) break;
    double l = 0, m0 = 0, m1 = 0, m2 = 0;
    for (int c = lane; c < nch; c += W) {
      if (L.lab[cur][c] != cand) continue;
      const int n = L.by_entry[L.ch_xe[c]];
      const int ea = L.ch_xe[c], eb = L.ch_xe[n];
      const double a0 = L.ept[0][ea], a1 = L.ept[1][ea], a2 = L.ept[2][ea];
      const double b0 = L.ept[0][eb], b1 = L.ept[1][eb], b2 = L.ept[2][eb];
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
      const int ec = L.ch_xe[cand];
      k0 = L.ept[0][ec]; k1 = L.ept[1][ec]; k2 = L.ept[2][ec];
    }
    double vi = 0, t0 = 0, t1 = 0, t2 = 0;
    for (int c = lane; c < nch; c += W) {
      if (L.lab[cur][c] != cand) continue;
      const int n = L.by_entry[L.ch_xe[c]];
      const int ea = L.ch_xe[c], eb = L.ch_xe[n];
      const double a0 = L.ept[0][ea], a1 = L.ept[1][ea], a2 = L.ept[2][ea];
      const double b0 = L.ept[0][eb], b1 = L.ept[1][eb], b2 = L.ept[2][eb];
      vi += det3(k0, k1, k2, a0, a1, a2, b0, b1, b2);
      const double u0 = a0 - k0, u1 = a1 - k1, u2 = a2 - k2;
      const double w0 = b0 - k0, w1 = b1 - k1, w2 = b2 - k2;
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
    prev = cand;
  }
  R.V += Vi * (1.0 / 6.0);
  R.S0 = S0; R.S1 = S1; R.S2 = S2;
  R.A = Asum;
  if (Asum > 0) {
    R.c0 = cw0 / Asum; R.c1 = cw1 / Asum; R.c2 = cw2 / Asum;
  } else {
    R.c0 = R.c1 = R.c2 = 0;
  }
}

// Full volume evaluation, faces over the lanes of the wave.  With
// build_slot >= 0 it also records the fixed-topology chord data of this
// isovalue into that cache slot (when the chords fit it).
template <int NV, int NF, int NL, int NCH>
__device__ CutRes cut_full(GroupMem<kSlotChords, NV, NF, NL, NCH> &L, int lane, int nf, int nl, double s,
                           int build_slot) {
  constexpr int W = 64;
  CutRes R;
  R.err = false;
  double vfull = 0.0, vcut = 0.0;
  int nch = 0;
  bool err = false;
  // (1) loop positions over the lanes: liquid edges and liquid parts of cut
  // edges, exit / entry bits of every face, crossing points by edge
  for (int f = lane; f < nf; f += W) {
    L.fex[f] = 0;
    L.fen[f] = 0;
  }
  wave_sync();
  for (int pos = lane; pos < nl; pos += W) {
    const int f = L.pface[pos];
    const int a = L.lv[pos], b = L.lv[L.pnext[pos]];
    const bool la = L.phi[a] >= s, lb = L.phi[b] >= s;
    const double c0 = L.cf[0][f], c1 = L.cf[1][f], c2 = L.cf[2][f];
    if (la && lb) {
      vfull += det3(c0, c1, c2, L.X[0][a], L.X[1][a], L.X[2][a], L.X[0][b], L.X[1][b], L.X[2][b]);
    } else if (la != lb) {
      double p0, p1, p2;
      crossing_at(L, pos, a, b, s, p0, p1, p2);
      const uint64_t bit = 1ull << L.pk[pos];
      if (la) {  // exit: liquid part from a to the crossing
        vcut += det3(c0, c1, c2, L.X[0][a], L.X[1][a], L.X[2][a], p0, p1, p2);
        atomicOr((unsigned long long *)&L.fex[f], (unsigned long long)bit);
        const int e = L.eid[pos];
        L.ept[0][e] = p0; L.ept[1][e] = p1; L.ept[2][e] = p2;
      } else {   // entry: liquid part from the crossing to b
        vcut += det3(c0, c1, c2, p0, p1, p2, L.X[0][b], L.X[1][b], L.X[2][b]);
        atomicOr((unsigned long long *)&L.fen[f], (unsigned long long)bit);
      }
    }
  }
  wave_sync();
  // (2) chords: each exit is paired with an entry of its face (the next one
  // in loop order when the face-mean value is >= s or the face has two
  // crossings, else the previous one); chords are numbered in position order
  for (int base = 0; base < nl; base += W) {
    const int pos = base + lane;
    bool is_exit = false;
    int f = 0, q = 0;
    uint64_t ex = 0, en = 0;
    if (pos < nl) {
      f = L.pface[pos];
      q = L.pk[pos];
      ex = L.fex[f];
      en = L.fen[f];
      is_exit = (ex >> q) & 1ull;
    }
    if (is_exit && __popcll(en) != __popcll(ex)) {  // a closed loop alternates exits and entries
      err = true;
      is_exit = false;
    }
    const uint64_t bal = __ballot(is_exit);
    // rank among the exits (both forms count the same bits; which one the
    // register allocator handles better differs between the kernel variants,
    // measured: the hardware count for the hexahedral variant)
    const int c = nch + (NV <= 16 ? lanes_below(bal) : __popcll(bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane)))));
    if (is_exit) {
      const bool liquid_connected = (__popcll(ex) == 1) || (L.fmean[f] >= s);
      const int r = liquid_connected ? next_bit_after(en, q) : prev_bit_before(en, q);
      const int o = L.floff[f];
      const int xe = L.eid[pos], ne = L.eid[o + r];
      const double s0 = L.ept[0][xe], s1 = L.ept[1][xe], s2 = L.ept[2][xe];
      const double e0 = L.ept[0][ne], e1 = L.ept[1][ne], e2 = L.ept[2][ne];
      vcut += det3(L.cf[0][f], L.cf[1][f], L.cf[2][f], s0, s1, s2, e0, e1, e2);
      if (c < NCH) {
        L.ch_xe[c] = (uint16_t)xe;
        L.ch_ne[c] = (uint16_t)ne;
        L.ch_face[c] = (uint16_t)f;
        L.ch_xpos[c] = (uint16_t)pos;
        L.by_entry[ne] = (uint16_t)c;
        L.by_exit[xe] = (uint16_t)c;
      } else {
        err = true;
      }
    }
    nch += __popcll(bal);
  }
  wave_sync();
  if (nch > NCH) nch = NCH;
  vfull = gsum<W>(vfull);
  vcut = gsum<W>(vcut);
  R.V = (vfull + vcut) * (1.0 / 6.0);
  R.nch = nch;
  if (nch <= W) {
    const bool valid = lane < nch;
    double p0 = 0, p1 = 0, p2 = 0;
    int next = lane;
    if (valid) {
      const int e = L.ch_xe[lane];
      p0 = L.ept[0][e]; p1 = L.ept[1][e]; p2 = L.ept[2][e];
      next = L.by_entry[e];
    }
    int lab, nloops;
    if (nch <= 16) {
      // chords in the first row: row-local shuffles and DPP sums, then the
      // sums of lane 0 go to the whole wave
      lab = labels_reg<16>(lane, valid, next, nch);
      nloops = gsum_i<16>((valid && lab == lane) ? 1 : 0);
      loops_reg<16>(lane, valid, p0, p1, p2, next, lab, nloops, R);
      nloops = __builtin_amdgcn_readfirstlane(nloops);
      R.V = readlane_d(R.V, 0); R.S0 = readlane_d(R.S0, 0); R.S1 = readlane_d(R.S1, 0);
      R.S2 = readlane_d(R.S2, 0); R.A = readlane_d(R.A, 0); R.c0 = readlane_d(R.c0, 0);
      R.c1 = readlane_d(R.c1, 0); R.c2 = readlane_d(R.c2, 0);
    } else {
      lab = labels_reg<W>(lane, valid, next, nch);
      nloops = gsum_i<W>((valid && lab == lane) ? 1 : 0);
      loops_reg<W>(lane, valid, p0, p1, p2, next, lab, nloops, R);
    }
    if (build_slot >= 0 && nch <= kSlotChords) {
      FastSlot<kSlotChords> &F = L.fs[build_slot];
      if (lane == 0) {
        F.nch = nch;
        F.nloops = nloops;
        F.c_full = vfull;
      }
      int prev = lane;
      if (valid) {
        const int pos = L.ch_xpos[lane];
        const int f = L.ch_face[lane];
        const int o = L.floff[f], m = L.fsz[f];
        const int a = L.lv[pos];                                       // liquid end
        const int b = L.lv[(pos + 1 - o == m) ? o : pos + 1];          // vapour end
        F.xi[0][lane] = L.X[0][a]; F.xi[1][lane] = L.X[1][a]; F.xi[2][lane] = L.X[2][a];
        F.dx[0][lane] = L.X[0][b] - L.X[0][a];
        F.dx[1][lane] = L.X[1][b] - L.X[1][a];
        F.dx[2][lane] = L.X[2][b] - L.X[2][a];
        F.phi_i[lane] = L.phi[a];
        F.inv[lane] = L.inv[pos];
        F.cf[0][lane] = L.cf[0][f]; F.cf[1][lane] = L.cf[1][f]; F.cf[2][lane] = L.cf[2][f];
        prev = L.by_exit[L.ch_ne[lane]];
        F.next[lane] = (uint8_t)next;
        F.lab[lane] = (uint8_t)lab;
        F.prev[lane] = (uint8_t)prev;
      }
      wave_sync();
      // liquid end of the entry edge = liquid end of the previous chord's exit edge
      if (valid) {
        F.xn[0][lane] = F.xi[0][prev]; F.xn[1][lane] = F.xi[1][prev]; F.xn[2][lane] = F.xi[2][prev];
      }
    }
  } else {
    if constexpr (NCH > 64) loops_lds<W>(L, lane, nch, R);
  }
  R.err = gsum_i<W>(err ? 1 : 0) != 0;
  wave_sync();
  return R;
}

// Evaluation on a fixed topology by a segment of C lanes, chord c on lane c
// of the segment (see the file comment).
template <int C>
__device__ CutRes cut_fast(const FastSlot<kSlotChords> &F, int c, double s) {
  CutRes R;
  R.err = false;
  const int nch = F.nch;
  R.nch = nch;
  const bool valid = c < nch;
  double p0 = 0, p1 = 0, p2 = 0, v = 0.0;
  int prev = c, next = c, lab = C;
  if (valid) {
    const double lam = (s - F.phi_i[c]) * F.inv[c];
    p0 = F.xi[0][c] + lam * F.dx[0][c];
    p1 = F.xi[1][c] + lam * F.dx[1][c];
    p2 = F.xi[2][c] + lam * F.dx[2][c];
    prev = F.prev[c];
    next = F.next[c];
    lab = F.lab[c];
  }
  // entry point of this chord = exit point of the previous chord on the loop
  const double n0 = __shfl(p0, prev, C), n1 = __shfl(p1, prev, C), n2 = __shfl(p2, prev, C);
  if (valid) {
    const double c0 = F.cf[0][c], c1 = F.cf[1][c], c2 = F.cf[2][c];
    v = det3(c0, c1, c2, F.xi[0][c], F.xi[1][c], F.xi[2][c], p0, p1, p2) +
        det3(c0, c1, c2, p0, p1, p2, n0, n1, n2) +
        det3(c0, c1, c2, n0, n1, n2, F.xn[0][c], F.xn[1][c], F.xn[2][c]);
  }
  v = gsum<C>(v);
  R.V = (F.c_full + v) * (1.0 / 6.0);
  loops_reg<C>(c, valid, p0, p1, p2, next, lab, F.nloops, R);
  return R;
}


// The topology of a cut (which vertices are liquid, how faces with four or
// more crossings pair them) is constant for isovalues between consecutive
// breakpoints, the vertex values and the face-mean values: on (b_i, b_i+1].
// This returns that interval around s.
template <class GM>
__device__ __forceinline__ void breakpoint_interval(const GM &L, int lane, int nv, int nf, double s, double &lo,
                                                    double &hi) {
  double a = -__builtin_inf(), b = __builtin_inf();
  for (int i = lane; i < nv; i += 64) {
    const double v = L.phi[i];
    if (v < s) a = fmax(a, v); else b = fmin(b, v);
  }
  for (int f = lane; f < nf; f += 64) {
    const double v = L.fmean[f];
    if (v < s) a = fmax(a, v); else b = fmin(b, v);
  }
  lo = gmax<64>(a);
  hi = gmin<64>(b);
}

// Full evaluation at s that refreshes the older cache slot.
template <int NV, int NF, int NL, int NCH>
__device__ __forceinline__ CutRes full_step(GroupMem<kSlotChords, NV, NF, NL, NCH> &L, int lane, int nv, int nf,
                                            int nl, double s, int &lru) {
  const int slot = lru;
  CutRes c = cut_full(L, lane, nf, nl, s, slot);
  const bool ok = c.nch <= kSlotChords && !c.err;
  double blo = 0, bhi = 0;
  if (ok) breakpoint_interval(L, lane, nv, nf, s, blo, bhi);
  if (lane == 0) {
    L.fs[slot].valid = ok ? 1 : 0;
    L.fs[slot].bp_lo = blo;
    L.fs[slot].bp_hi = bhi;
  }
  wave_sync();
  lru ^= 1;
  return c;
}

// Evaluate the isovalues L.sp_s[0..npts) on cached slot u, C lanes per
// isovalue (segment j takes point j).  The first lane of each evaluating
// segment returns true with the point and its cut sums.
template <int C, int NV, int NF, int NL, int NCH>
__device__ __forceinline__ bool fast_round(const GroupMem<kSlotChords, NV, NF, NL, NCH> &L, int lane, int u, int npts,
                                           double &x, CutRes &R) {
  const int seg = lane / C, c = lane % C;
  x = 0.0;
  R.V = R.S0 = R.S1 = R.S2 = R.A = R.c0 = R.c1 = R.c2 = 0.0;
  if (seg < npts) {
    x = L.sp_s[seg];
    R = cut_fast<C>(L.fs[u], c, x);
  }
  return seg < npts && c == 0;
}


template <class GM>
__device__ __forceinline__ void store_end(GM &L, int lane, int side, const CutRes &c) {
  if (lane == 0) {
    double *e = L.end_res[side];
    e[0] = c.V; e[1] = c.S0; e[2] = c.S1; e[3] = c.S2; e[4] = c.A; e[5] = c.c0; e[6] = c.c1; e[7] = c.c2;
  }
}


// The bracket network's normalised isovalue for the staged cell: its 32
// inputs from the staged vertex values and the cell's faces, then the
// forward pass of one row, one hidden unit per lane with FP32 FMAs.
template <int NF, class GM>
__device__ float net_guess(GM &L, int lane, const ReconParams &p, int64_t k, int P, double aP, int nv, int nf,
                           int64_t f0, double pmin, double Wd, const NetFace &pf) {
  constexpr int W = 64;
  // face sums (see the feature definitions) into L.nsum
  double amin = __builtin_inf(), amax = -__builtin_inf();
  auto face = [&](const NetFace &g, double &A, double &n0, double &n1, double &n2, double &aQ, bool &inner) {
    A = sqrt(g.S0 * g.S0 + g.S1 * g.S1 + g.S2 * g.S2);
    n0 = g.S0 / A; n1 = g.S1 / A; n2 = g.S2 / A;
    inner = g.inner;
    aQ = g.aQ;
  };
  if constexpr (NF <= W) {
    // one face per lane: each sum is reduced as soon as it is formed
    double A = 0, n0 = 0, n1 = 0, n2 = 0, aQ = aP;
    bool inner = false;
    if (lane < nf) face(pf, A, n0, n1, n2, aQ, inner);   // loaded before the staging
    const double da = A * (aQ - aP);
    if (inner) {
      amin = aQ;
      amax = aQ;
    }
    const bool row = nf <= 16;   // faces within the first row: DPP sums only
    auto red = [&](int i, double v) {
      v = row ? gsum<16>(v) : gsum<W>(v);
      if (lane == 0) L.nsum[i] = v;
    };
    red(0, A);
    red(1, da * n0); red(2, da * n1); red(3, da * n2);
    red(4, da * n0 * n0); red(5, da * n1 * n1); red(6, da * n2 * n2);
    red(7, da * n0 * n1); red(8, da * n0 * n2); red(9, da * n1 * n2);
    red(10, A * n0 * n0); red(11, A * n1 * n1); red(12, A * n2 * n2);
    red(13, A * n0 * n1); red(14, A * n0 * n2); red(15, A * n1 * n2);
    red(16, inner ? aQ : 0.0);
    red(17, inner ? 1.0 : 0.0);
    amin = row ? readlane_d(gmin<16>(amin), 0) : gmin<W>(amin);
    amax = row ? readlane_d(gmax<16>(amax), 0) : gmax<W>(amax);
  } else {
    double t[18];
#pragma unroll
    for (int i = 0; i < 18; ++i) t[i] = 0.0;
    for (int f = lane; f < nf; f += W) {
      double A, n0, n1, n2, aQ;
      bool inner;
      face(load_net_face(p, P, aP, f0 + f), A, n0, n1, n2, aQ, inner);
      const double da = A * (aQ - aP);
      const double o[6] = {n0 * n0, n1 * n1, n2 * n2, n0 * n1, n0 * n2, n1 * n2};
      t[0] += A;
      t[1] += da * n0; t[2] += da * n1; t[3] += da * n2;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        t[4 + c] += da * o[c];
        t[10 + c] += A * o[c];
      }
      if (inner) {
        t[16] += aQ;
        t[17] += 1.0;
        amin = fmin(amin, aQ);
        amax = fmax(amax, aQ);
      }
    }
#pragma unroll
    for (int i = 0; i < 18; ++i) {
      const double v = gsum<W>(t[i]);
      if (lane == 0) L.nsum[i] = v;
    }
    amin = gmin<W>(amin);
    amax = gmax<W>(amax);
  }
  // vertex values sorted by rank (ties by index) into the crossing-point
  // scratch, which holds at least as many values as the cell has vertices
  double *srt = &L.ept[0][0];
  double lsum = 0.0;
  for (int i = lane; i < nv; i += W) {
    const double v = L.phi[i];
    int r = 0;
    for (int j = 0; j < nv; ++j) {
      const double u = L.phi[j];
      r += (u < v) || (u == v && j < i);
    }
    srt[r] = v;
    lsum += v;
  }
  lsum = gsum<W>(lsum);
  wave_sync();
  if (lane < net::kIn) {
    auto sorted = [&](int j) { return srt[j]; };
    const float x = net::feature(lane, aP, sorted, nv, lsum, pmin, Wd, L.nsum, amin, amax, nf);
    L.nx[lane] = net::to_bf16(x);
  }
  wave_sync();
  const float u = net::row_forward(p.net_wb, p.net_master, L.nx, L.nh1, L.nh2, lane, [] { wave_sync(); });
  wave_sync();
  (void)k;
  return u;
}

// One cell per wavefront (block of 64 lanes).
template <int NV, int NF, int NL, int NCH, int OCC>
__global__ __launch_bounds__(64, OCC) void recon_kernel(ReconParams p) {
  constexpr int W = 64;
  __shared__ GroupMem<kSlotChords, NV, NF, NL, NCH> L;
  const int lane = threadIdx.x;
  const DevMesh &m = p.m;
  const int64_t N = m.n_cells;
  const int64_t cap = p.out.cap;
  int64_t count = p.entries ? (int64_t)*p.entry_count : (int64_t)p.counts[0];
  if (count > cap) count = cap;
  // cells go to blocks through a counter: block b starts with entry b and
  // then claims the next unclaimed one, so blocks that meet cheap cells do
  // more of them
  for (int64_t j = blockIdx.x; j < count;) {
    const int64_t k = p.entries ? (int64_t)p.entries[j] : j;
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
      // learned form with one face per lane: the network's face data are
      // loaded first, so their loads are in flight during the staging
      NetFace pf{0.0, 0.0, 0.0, a, false};
      if (NF <= W && p.net_wb && lane < nf) pf = load_net_face(p, P, a, f0 + lane);
      // ---- stage the polyhedron (vertex field by inverse-distance weights;
      // the incidences of a vertex are read four at a time, summed in order)
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
          const int64_t j1 = m.vc_off[gv + 1];
          for (int64_t j = m.vc_off[gv]; j < j1; j += 4) {
            int cc[4];
            double ww[4], aa[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              const bool in = j + t < j1;
              cc[t] = in ? m.vc_cell[j + t] : 0;
              ww[t] = in ? w[j + t] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) aa[t] = (j + t < j1) ? p.alpha[cc[t]] : 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t)
              if (j + t < j1) ph += ww[t] * aa[t];
          }
        }
        L.phi[i] = ph;
      }
      for (int i = lane; i < nl; i += W) {
        const uint32_t info = m.cl_info[l0 + i];
        L.lv[i] = m.cl_lv[l0 + i];
        L.eid[i] = m.cl_eid[l0 + i];
        L.pface[i] = (uint8_t)(info & 0xffu);
        L.pk[i] = (uint8_t)((info >> 8) & 0xffu);
        L.pnext[i] = (uint16_t)(info >> 16);
      }
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
        wave_sync();
        // face vertex means (fan centres of the planar faces), face-mean
        // vertex values (pairing rule of faces with four or more crossings)
        // and the reciprocal value difference of every loop position
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
        for (int i = lane; i < nl; i += W) L.inv[i] = 1.0 / (L.phi[L.lv[L.pnext[i]]] - L.phi[L.lv[i]]);
        if (lane == 0) {
          L.fs[0].valid = 0;
          L.fs[1].valid = 0;
        }
        wave_sync();
        CutRes c;
        c.err = false;
        double s = __builtin_nan("");
        bool cut_ok = false;
        if (p.fixed_iso) {
          s = p.iso;
          c = cut_full(L, lane, nf, nl, s, -1);
          it = 1;
          cut_ok = true;
        } else {
          double lo = pmin, hi = pmax, rlo = 1.0 - a, rhi = -a;
          const double tol = p.tol_rel * (a < 1.0 - a ? a : 1.0 - a);
          bool have_lo = false, have_hi = false, collapsed = false;
          double s3 = 0, r3 = 0;   // third point for inverse quadratic interpolation
          bool have3 = false;
          int kept = 0;            // > 0: lo kept that many updates in a row, < 0: hi
          bool slow = false;       // the last update did not halve the bracket
          int lru = 0, probe = -1;
          // learned bracket [sh - dl, sh + dl]; the status records whether
          // the root fell outside it
          bool hint = false;
          double hl = 0, hh = 0, hm = 0;
          if (p.net_wb && st == VOFPC_CELL_OK) {
            const double Wd = pmax - pmin;
            const float u = net_guess<NF>(L, lane, p, k, P, a, nv, nf, f0, pmin, Wd, pf);
            if (!isnan(u)) {
              const double uc = u < 0.f ? 0.0 : (u > 1.f ? 1.0 : (double)u);
              const double sh = pmin + uc * Wd, dl = p.net_delta * Wd;
              hl = sh - dl;
              hh = sh + dl;
              if (lane == 0 && p.net_lo) {
                p.net_lo[k] = hl;
                p.net_hi[k] = hh;
              }
              hl = hl > pmin ? hl : pmin;
              hh = hh < pmax ? hh : pmax;
              hint = hl <= hh;
              hm = sh < hl ? hl : (sh > hh ? hh : sh);
            } else if (lane == 0 && p.net_lo) {
              p.net_lo[k] = __builtin_nan("");
              p.net_hi[k] = __builtin_nan("");
            }
          } else if (p.net_wb) {
            if (lane == 0 && p.net_lo) {   // no network bracket for this cell
              p.net_lo[k] = __builtin_nan("");
              p.net_hi[k] = __builtin_nan("");
            }
          } else if (p.use_hint) {
            hl = p.hint_lo[k];
            hh = p.hint_hi[k];
            if (!isnan(hl) && !isnan(hh)) {
              hl = hl > pmin ? hl : pmin;
              hh = hh < pmax ? hh : pmax;
              hint = hl <= hh;
              hm = hl + (hh - hl) / 2.0;
            }
          }
          if (hint) {
            // check the narrowed bracket with two cuts: at its centre (the
            // predicted isovalue), whose residual tells the side of the root,
            // and at the bracket end on that side.  The bracket holds when
            // that end is past the root (the half on the root's side is
            // kept); otherwise the root lies beyond it (LEARNED_FALLBACK).
            const CutRes cm = full_step(L, lane, nv, nf, nl, hm, lru);
            ++it;
            const double rm = cm.V / VP - a;
            if (fabs(rm) <= tol) {
              s = hm; c = cm; cut_ok = true;
            } else {
              const bool up = rm > 0;          // the root lies above hm
              const double he = up ? hh : hl;
              if (up) {
                s3 = hi; r3 = rhi;
                lo = hm; rlo = rm; have_lo = true; store_end(L, lane, 0, cm);
              } else {
                s3 = lo; r3 = rlo;
                hi = hm; rhi = rm; have_hi = true; store_end(L, lane, 1, cm);
              }
              have3 = true;
              bool holds = false;
              if (he != hm) {
                wave_sync();
                const CutRes ce = full_step(L, lane, nv, nf, nl, he, lru);
                ++it;
                const double re = ce.V / VP - a;
                if (fabs(re) <= tol) {
                  s = he; c = ce; cut_ok = true;
                  holds = true;
                } else if (up ? re < 0 : re > 0) {
                  holds = true;
                  s3 = up ? hi : lo; r3 = up ? rhi : rlo;
                  if (up) { hi = he; rhi = re; have_hi = true; store_end(L, lane, 1, ce); }
                  else { lo = he; rlo = re; have_lo = true; store_end(L, lane, 0, ce); }
                } else {
                  s3 = hm; r3 = rm;
                  if (up) { lo = he; rlo = re; store_end(L, lane, 0, ce); }
                  else { hi = he; rhi = re; store_end(L, lane, 1, ce); }
                }
              }
              if (!holds && st == VOFPC_CELL_OK) st = VOFPC_CELL_LEARNED_FALLBACK;
            }
            wave_sync();
          }
          while (!cut_ok) {
            const double big = fabs(lo) > fabs(hi) ? fabs(lo) : fabs(hi);
            if (hi - lo <= 2.0 * ulp_of(big)) { collapsed = true; break; }
            if (it >= p.max_iter) { st = VOFPC_CELL_MAX_ITER; break; }
            const double w0 = hi - lo;
            // next estimate: regula falsi with the Illinois weight on an end
            // kept twice, inverse quadratic interpolation when it stays
            // inside the bracket, a bisection step after a slow update
            const double fl = kept >= 2 ? 0.5 * rlo : rlo, fh = kept <= -2 ? 0.5 * rhi : rhi;
            double se = lo + w0 * (fl / (fl - fh));
            double d = 0.125 * w0;
            if (have3 && kept > -2 && kept < 2) {
              const double q = iqi(lo, rlo, hi, rhi, s3, r3);
              if (q > lo && q < hi) {
                d = 4.0 * fabs(q - se);
                se = q;
              }
            }
            if (slow || !(se > lo && se < hi)) {
              se = lo + w0 / 2.0;
              d = 0.125 * w0;
            }
            if (!(se > lo && se < hi)) { collapsed = true; break; }
            const double du = 8.0 * ulp_of(se);
            d = d > du ? d : du;
            d = d < 0.5 * w0 ? d : 0.5 * w0;
            // a slot just built is probed at once; otherwise the slot that
            // covers the estimate, if any
            int u = probe;
            probe = -1;
            if (u < 0) {
              if (L.fs[0].valid && se > L.fs[0].bp_lo && se <= L.fs[0].bp_hi) u = 0;
              else if (L.fs[1].valid && se > L.fs[1].bp_lo && se <= L.fs[1].bp_hi) u = 1;
            }
            if (u < 0) {
              // no cached topology covers the estimate: full evaluation
              const int slot = lru;
              const CutRes cf = full_step(L, lane, nv, nf, nl, se, lru);
              ++it;
              const double r = cf.V / VP - a;
              if (fabs(r) <= tol) {
                s = se; c = cf; cut_ok = true;
                break;
              }
              if (r > 0) {
                s3 = lo; r3 = rlo;
                lo = se; rlo = r; have_lo = true;
                store_end(L, lane, 0, cf);
                kept = kept <= 0 ? kept - 1 : -1;
              } else {
                s3 = hi; r3 = rhi;
                hi = se; rhi = r; have_hi = true;
                store_end(L, lane, 1, cf);
                kept = kept >= 0 ? kept + 1 : 1;
              }
              have3 = true;
              slow = (hi - lo) > 0.5 * w0;
              if (L.fs[slot].valid) probe = slot;
              wave_sync();
              continue;
            }
            // parallel round on the cached topology: the estimate, the ends
            // of the topology interval when the bracket reaches past them,
            // a ladder around the estimate and the bracket midpoint
            const double blo = L.fs[u].bp_lo, bhi = L.fs[u].bp_hi;
            const int nch = L.fs[u].nch;
            const int C = nch <= 8 ? 8 : 16;
            const int K = 64 / C;
            // candidates in lanes 0..7 (estimate, left and right interval
            // ends, ladder -d/16, +d/16, -d, +d, midpoint); the first K that
            // lie inside both the bracket and the interval are evaluated
            double xc;
            bool okc;
            {
              // ladder offsets: lanes 3, 4 at -d/16, +d/16, lanes 5, 6 at -d, +d
              // (selected from d itself, so no per-lane constant is held
              // across the loop; scaling by 1/16 is exact)
              const double dd = lane < 5 ? 0.0625 * d : d;
              xc = (lane >= 3 && lane <= 6) ? ((lane & 1) ? se - dd : se + dd) : se;
              if (lane == 1) xc = next_up(blo);
              if (lane == 2) xc = bhi;
              if (lane == 7) xc = lo + w0 / 2.0;
              okc = lane < 8 && xc > lo && xc < hi && xc > blo && xc <= bhi && (lane != 1 || lo <= blo) &&
                    (lane != 2 || hi > bhi);
            }
            const uint64_t cm = __ballot(okc);
            const int cpos = NV <= 16 ? lanes_below(cm) : __popcll(cm & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
            int np = __popcll(cm);
            np = np < K ? np : K;
            if (okc && cpos < K) L.sp_s[cpos] = xc;
            if (np == 0) continue;   // a probe round with nothing inside the bracket
            wave_sync();
            double xj;
            CutRes Rj;
            bool vj;
            if (C == 8) vj = fast_round<8>(L, lane, u, np, xj, Rj);
            else vj = fast_round<16>(L, lane, u, np, xj, Rj);
            it += np;
            // the point nearest to alpha V_P ends the search; otherwise the
            // tightest sign change becomes the bracket.  Segment j's point and
            // residual move to lane j, reductions run over lanes 0..7.
            const double rj = Rj.V / VP - a;
            const double inf = __builtin_inf();
            (void)vj;
            const int srcl = (lane < 8 ? lane : 0) * C;
            const double x8 = __shfl(xj, srcl), r8 = __shfl(rj, srcl);
            const bool v8 = lane < np;
            const bool fnd = v8 && fabs(r8) <= tol;
            const uint64_t fm = __ballot(fnd);
            if (fm) {
              const double mabs = readlane_d(gmin<8>(fnd ? fabs(r8) : inf), 0);
              const int bj = __ffsll((long long)__ballot(fnd && fabs(r8) == mabs)) - 1;
              const int bl = bj * C;
              s = readlane_d(xj, bl);
              c.V = readlane_d(Rj.V, bl); c.S0 = readlane_d(Rj.S0, bl); c.S1 = readlane_d(Rj.S1, bl);
              c.S2 = readlane_d(Rj.S2, bl); c.A = readlane_d(Rj.A, bl); c.c0 = readlane_d(Rj.c0, bl);
              c.c1 = readlane_d(Rj.c1, bl); c.c2 = readlane_d(Rj.c2, bl);
              c.err = false;
              cut_ok = true;
              break;
            }
            const double olo = lo, orlo = rlo, ohi = hi, orhi = rhi;
            const bool pos = v8 && r8 > 0 && x8 > lo && x8 < hi;
            const double slo = readlane_d(gmax<8>(pos ? x8 : -inf), 0);
            int jl = -1, jh = -1;
            if (slo > lo) {
              jl = __ffsll((long long)__ballot(pos && x8 == slo)) - 1;
              lo = slo;
              rlo = readlane_d(r8, jl);
            }
            const bool neg = v8 && !(r8 > 0) && x8 > lo && x8 < hi;
            const double shi = readlane_d(gmin<8>(neg ? x8 : inf), 0);
            if (shi < hi) {
              jh = __ffsll((long long)__ballot(neg && x8 == shi)) - 1;
              hi = shi;
              rhi = readlane_d(r8, jh);
            }
            if (jl >= 0 && lane == jl * C) {
              double *e = L.end_res[0];
              e[0] = Rj.V; e[1] = Rj.S0; e[2] = Rj.S1; e[3] = Rj.S2; e[4] = Rj.A; e[5] = Rj.c0; e[6] = Rj.c1; e[7] = Rj.c2;
            }
            if (jh >= 0 && lane == jh * C) {
              double *e = L.end_res[1];
              e[0] = Rj.V; e[1] = Rj.S0; e[2] = Rj.S1; e[3] = Rj.S2; e[4] = Rj.A; e[5] = Rj.c0; e[6] = Rj.c1; e[7] = Rj.c2;
            }
            have_lo = have_lo || jl >= 0;
            have_hi = have_hi || jh >= 0;
            // third point: the evaluated point off the bracket nearest the root
            const bool off = v8 && lane != jl && lane != jh;
            const double m3 = readlane_d(gmin<8>(off ? fabs(r8) : inf), 0);
            double b3 = inf;
            if (m3 < inf) {
              const int l3 = __ffsll((long long)__ballot(off && fabs(r8) == m3)) - 1;
              b3 = m3; s3 = readlane_d(x8, l3); r3 = readlane_d(r8, l3);
            }
            if (jl >= 0 && fabs(orlo) < b3) { b3 = fabs(orlo); s3 = olo; r3 = orlo; }
            if (jh >= 0 && fabs(orhi) < b3) { b3 = fabs(orhi); s3 = ohi; r3 = orhi; }
            have3 = have3 || b3 < inf;
            if (jl >= 0 && jh >= 0) kept = 0;
            else if (jl >= 0) kept = kept <= 0 ? kept - 1 : -1;
            else if (jh >= 0) kept = kept >= 0 ? kept + 1 : 1;
            slow = (hi - lo) > 0.5 * w0;
            wave_sync();
          }
          if (collapsed || st == VOFPC_CELL_MAX_ITER) {
            // the bracket end nearer to alpha V_P
            wave_sync();
            const bool take_lo = fabs(rlo) <= fabs(rhi);
            const double se = take_lo ? lo : hi;
            if (take_lo ? have_lo : have_hi) {
              const double *e = L.end_res[take_lo ? 0 : 1];
              c.V = e[0]; c.S0 = e[1]; c.S1 = e[2]; c.S2 = e[3]; c.A = e[4]; c.c0 = e[5]; c.c1 = e[6]; c.c2 = e[7];
              c.err = false;
            } else {
              c = cut_full(L, lane, nf, nl, se, -1);
              ++it;
            }
            s = se;
            cut_ok = true;
            if (collapsed && fabs(take_lo ? rlo : rhi) > 1e-10) st = VOFPC_CELL_NO_ROOT;
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
    int nk = 0;
    if (lane == 0 && p.mf.gradT) {
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
    if (lane == 0) {
      p.out.s[k] = s_out;
      p.out.n[k] = n0; p.out.n[cap + k] = n1; p.out.n[2 * cap + k] = n2;
      p.out.A[k] = A_out;
      p.out.d[k] = d_out;
      p.out.alpha_got[k] = ag;
      p.out.status[k] = st;
      p.out.iters[k] = it;
      // wrapping increment: a launch makes exactly `count` claims (one
      // after each cell; the first one at or past `count` ends a block), so
      // the counter is back at zero when the launch ends
      nk = (int)atomicInc((unsigned int *)p.queue, (unsigned int)(count - 1));
    }
    j = (int64_t)gridDim.x + __builtin_amdgcn_readfirstlane(nk);
    wave_sync();
  }
}

// ----------------------------------------------------------------- buckets
// Kernel class of a cell: the smallest template variant that holds it (with
// the mesh's hexahedral class 0, mesh_class_of).
__device__ __forceinline__ int cell_class(const DevMesh &m, bool hex0, int P) {
  const int64_t nf = m.cell_face_off[P + 1] - m.cell_face_off[P];
  const int64_t nv = m.cv_off[P + 1] - m.cv_off[P];
  const int64_t nl = m.cl_off[P + 1] - m.cl_off[P];
  return mesh_class_of(hex0, nv, nf, nl, nl / 2);
}

__global__ void bucket_zero_kernel(int32_t *c) {
  if (threadIdx.x < kClasses) c[threadIdx.x] = 0;
}

// Split the mixed entries into one list per class (order within a list is
// the order of the claims; results do not depend on it).  Blocks of 1024
// stride over the mixed entries; per tile of 1024 entries, one claim per
// class on the list counter (the waves' counts summed in LDS first).
constexpr int kBucketBlock = 1024;
__global__ __launch_bounds__(kBucketBlock) void bucket_kernel(DevMesh m, int hex0, const int32_t *mixed,
                                                              const int32_t *counts, int64_t cap, int32_t *lists,
                                                              int64_t stride, int32_t *bcount) {
  constexpr int kW = kBucketBlock / 64;
  __shared__ int32_t wcnt[kW][kClasses];
  __shared__ int32_t gbase[kClasses];
  int64_t count = counts[0];
  if (count > cap) count = cap;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t k0 = (int64_t)blockIdx.x * kBucketBlock; k0 < count; k0 += (int64_t)gridDim.x * kBucketBlock) {
    const int64_t k = k0 + threadIdx.x;
    const int c = (k < count) ? cell_class(m, hex0 != 0, mixed[k]) : -1;
    uint64_t mine = 0;
#pragma unroll
    for (int q = 0; q < kClasses; ++q) {
      const uint64_t bm = __ballot(c == q);
      if (c == q) mine = bm;
      if (lane == 0) wcnt[w][q] = __popcll(bm);
    }
    __syncthreads();
    if (threadIdx.x < kClasses) {
      const int q = threadIdx.x;
      int tot = 0;
      for (int i = 0; i < kW; ++i) tot += wcnt[i][q];
      gbase[q] = tot ? atomicAdd(&bcount[q], tot) : 0;
    }
    __syncthreads();
    if (c >= 0) {
      int off = gbase[c] + lanes_below(mine);
      for (int i = 0; i < w; ++i) off += wcnt[i][c];
      lists[c * stride + off] = (int32_t)k;
    }
    __syncthreads();
  }
}

namespace {
template <int NV, int NF, int NL, int NCH, int OCC>
vofpc_status launch_t(vofpc_ctx ctx, const ReconParams &p, int64_t n_cells) {
  int blocks_per_cu = 0;
  hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks_per_cu, recon_kernel<NV, NF, NL, NCH, OCC>, 64, 0);
  if (e != hipSuccess || blocks_per_cu <= 0) blocks_per_cu = 4;
  int64_t grid = (int64_t)ctx->n_cu * blocks_per_cu;
  if (grid > n_cells) grid = n_cells;
  if (grid < 1) grid = 1;
  recon_kernel<NV, NF, NL, NCH, OCC><<<(unsigned)grid, 64, 0, ctx->stream>>>(p);
  VOFPC_HIP(hipGetLastError());
  return VOFPC_OK;
}

// Launch the variant of class c in flavour `flav`: 3 or 4 = one cell per
// wavefront with the register budget of that many waves per SIMD (the two
// common classes have both), 10 + G = G lanes per cell (recon_thin.hip).
vofpc_status launch_class(vofpc_ctx ctx, vofpc_mesh M, const ReconParams &p, int64_t n_cells, int c, int flav) {
  if (flav >= 10) return launch_thin(ctx, p, n_cells, c, flav - 10, M->class_max[c]);
  const int occ = flav == 4 ? 4 : 3;
  switch (c) {
    case 0:
      return occ == 4 ? launch_t<16, 8, 48, 24, 4>(ctx, p, n_cells) : launch_t<16, 8, 48, 24, 3>(ctx, p, n_cells);
    case 1:
      return occ == 4 ? launch_t<32, 20, 96, 48, 4>(ctx, p, n_cells) : launch_t<32, 20, 96, 48, 3>(ctx, p, n_cells);
    case 2:
      return occ == 4 ? launch_t<48, 32, 128, 64, 4>(ctx, p, n_cells) : launch_t<48, 32, 128, 64, 3>(ctx, p, n_cells);
    default:
      return launch_t<255, 255, 1536, 768, 3>(ctx, p, n_cells);
  }
}
}  // namespace

// The class that stays on the context's stream when a bucketed launch runs
// the others beside it.
constexpr int kMainClass = 1;

vofpc_status launch_reconstruct(vofpc_ctx ctx, vofpc_mesh M, const double *alpha, const int32_t *mixed,
                                const int32_t *counts, const vofpc_recon_opts *o, const double *hlo,
                                const double *hhi, const vofpc_interface *out, vofpc_mlp net, double delta,
                                double *net_lo, double *net_hi, const MdotFuse *mf) {
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
  p.queue = ctx->queue;
  p.mf = mf ? *mf : MdotFuse{nullptr, 0.0, 0.0, 0.0, nullptr, nullptr};
  p.net_wb = net ? mlp_weights_bf16(net) : nullptr;
  p.net_master = net ? mlp_params_f32(net) : nullptr;
  p.net_delta = delta;
  p.net_lo = net ? net_lo : nullptr;
  p.net_hi = net ? net_hi : nullptr;
  VOFPC_REQUIRE(!net || mlp_device(net) == ctx->device, VOFPC_E_STATE,
                "reconstruct_learned: the network lives on another device");
  VOFPC_REQUIRE(!net || (delta >= 0 && delta < 1e300), VOFPC_E_INVALID_ARG,
                "reconstruct_learned: delta_scale must be finite and >= 0");
  VOFPC_REQUIRE(!net || !p.use_hint, VOFPC_E_INVALID_ARG,
                "reconstruct_learned: the network replaces hint brackets (use VOFPC_BRACKET_PLAIN)");
  p.out = *out;
  VOFPC_REQUIRE(M->max_fv <= 64, VOFPC_E_MESH, "reconstruct: faces with more than 64 vertices are not supported");
  const int64_t N = M->d.n_cells;
  p.entries = nullptr;
  p.entry_count = nullptr;
  // event pairs around the class kernels when the context times them (not
  // while the stream is being captured)
  bool timed = false;
  if (ctx->time_classes) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    VOFPC_HIP(hipStreamIsCapturing(ctx->stream, &cs));
    timed = cs == hipStreamCaptureStatusNone;
    if (timed)
      for (int c = 0; c < kClasses; ++c) ctx->cls_rec[c] = ctx->pass_rec[c] = false;
  }
  // learned form in a group build whose wavefronts hold fewer than 16 cells
  // (G = 8, 16: classes 1 and 2): the brackets come from a pass of their own
  // with full network tiles, and the class kernel checks them as a caller's
  // brackets (the same check and flag)
  auto pass_first = [&](int c) {
    const int f = M->tune[c];
    return p.net_wb != nullptr && (c == 1 || c == 2) && (f == VOFPC_FLAVOUR_GROUP(8) || f == VOFPC_FLAVOUR_GROUP(16));
  };
  bool any_pass = false;
  for (int c = 0; c < kClasses; ++c)
    any_pass = any_pass || ((M->bucketed ? M->class_cells[c] > 0 : c == M->max_class) && pass_first(c));
  if (any_pass && !p.net_lo && !M->hint_buf) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    VOFPC_HIP(hipStreamIsCapturing(ctx->stream, &cs));
    VOFPC_REQUIRE(cs == hipStreamCaptureStatusNone, VOFPC_E_STATE,
                  "reconstruct_learned: the first call on a mesh without hint_lo/hint_hi sets up its bracket "
                  "buffer and must not be captured");
    void *b = nullptr;
    vofpc_status st = mesh_scratch_alloc(M, 2 * sizeof(double) * (size_t)N, &b);
    if (st) return st;
    M->hint_buf = (double *)b;
  }
  auto run_class = [&](int64_t n_cells, int c) -> vofpc_status {
    vofpc_status st;
    if (pass_first(c)) {
      double *hl = p.net_lo ? p.net_lo : M->hint_buf, *hh = p.net_hi ? p.net_hi : M->hint_buf + N;
      if (timed) VOFPC_HIP(hipEventRecord(ctx->pass_ev[c][0], ctx->stream));
      st = launch_bracket_pass(ctx, p, n_cells, c, hl, hh);
      if (st) return st;
      if (timed) {
        VOFPC_HIP(hipEventRecord(ctx->pass_ev[c][1], ctx->stream));
        ctx->pass_rec[c] = true;
        VOFPC_HIP(hipEventRecord(ctx->cls_ev[c][0], ctx->stream));
      }
      ReconParams q = p;
      q.net_wb = nullptr;
      q.net_master = nullptr;
      q.net_lo = q.net_hi = nullptr;
      q.use_hint = 1;
      q.hint_lo = hl;
      q.hint_hi = hh;
      st = launch_class(ctx, M, q, n_cells, c, M->tune[c]);
    } else {
      if (timed) VOFPC_HIP(hipEventRecord(ctx->cls_ev[c][0], ctx->stream));
      st = launch_class(ctx, M, p, n_cells, c, M->tune[c]);
    }
    if (st) return st;
    if (timed) {
      VOFPC_HIP(hipEventRecord(ctx->cls_ev[c][1], ctx->stream));
      ctx->cls_rec[c] = true;
    }
    return VOFPC_OK;
  };
  if (!M->bucketed) return run_class(N, M->max_class);
  // one launch per class present in the mesh, each over its own entries
  bucket_zero_kernel<<<1, 64, 0, ctx->stream>>>(M->bucket_counts);
  const int64_t span = std::min<int64_t>(out->cap, N);
  const int64_t bgrid = std::min<int64_t>((span + kBucketBlock - 1) / kBucketBlock, (int64_t)ctx->n_cu * 2);
  bucket_kernel<<<(unsigned)std::max<int64_t>(bgrid, 1), kBucketBlock, 0, ctx->stream>>>(
      M->d, M->hex0 ? 1 : 0, mixed, counts, out->cap, M->bucket_lists, N, M->bucket_counts);
  VOFPC_HIP(hipGetLastError());
  // the usual Voronoi class (with its bracket pass) on the context's stream,
  // the other classes beside it on the side stream, forked after the
  // bucketing and joined before the call returns (each class claims from
  // its own counters), so one class's tail overlaps another's work
  bool others = false;
  for (int c = 0; c < kClasses; ++c) others = others || (c != kMainClass && M->class_cells[c] > 0);
  const bool fork = ctx->overlap_classes && ctx->side && others && M->class_cells[kMainClass] > 0;
  hipStream_t main_stream = ctx->stream;
  if (fork) {
    VOFPC_HIP(hipEventRecord(ctx->fork_ev, main_stream));
    VOFPC_HIP(hipStreamWaitEvent(ctx->side, ctx->fork_ev, 0));
  }
  vofpc_status st = VOFPC_OK;
  for (int c = 0; c < kClasses && st == VOFPC_OK; ++c) {
    if (M->class_cells[c] == 0) continue;
    p.entries = M->bucket_lists + (int64_t)c * N;
    p.entry_count = M->bucket_counts + c;
    p.queue = ctx->queue + c * kQueueSet;
    if (fork && c != kMainClass) ctx->stream = ctx->side;
    st = run_class(M->class_cells[c], c);
    ctx->stream = main_stream;
  }
  if (fork) {
    VOFPC_HIP(hipEventRecord(ctx->join_ev, ctx->side));
    VOFPC_HIP(hipStreamWaitEvent(main_stream, ctx->join_ev, 0));
  }
  return st;
}

extern "C" vofpc_status vofpc_ctx_overlap_classes(vofpc_ctx ctx, int32_t enable) {
  using namespace vofpc;
  clear_error();
  VOFPC_REQUIRE(ctx, VOFPC_E_INVALID_ARG, "ctx_overlap_classes: null context");
  ctx->overlap_classes = enable != 0;
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_ctx_time_classes(vofpc_ctx ctx, int32_t enable) {
  using namespace vofpc;
  clear_error();
  VOFPC_REQUIRE(ctx, VOFPC_E_INVALID_ARG, "ctx_time_classes: null context");
  VOFPC_HIP(hipSetDevice(ctx->device));
  if (enable && !ctx->time_classes) {
    for (int c = 0; c < kClasses; ++c)
      for (int j = 0; j < 2; ++j) {
        VOFPC_HIP(hipEventCreate(&ctx->cls_ev[c][j]));
        VOFPC_HIP(hipEventCreate(&ctx->pass_ev[c][j]));
      }
  } else if (!enable && ctx->time_classes) {
    for (int c = 0; c < kClasses; ++c)
      for (int j = 0; j < 2; ++j) {
        (void)hipEventDestroy(ctx->cls_ev[c][j]);
        (void)hipEventDestroy(ctx->pass_ev[c][j]);
        ctx->cls_ev[c][j] = ctx->pass_ev[c][j] = nullptr;
      }
  }
  ctx->time_classes = enable != 0;
  for (int c = 0; c < kClasses; ++c) ctx->cls_rec[c] = ctx->pass_rec[c] = false;
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_ctx_class_ms(vofpc_ctx ctx, float ms[8]) {
  using namespace vofpc;
  clear_error();
  VOFPC_REQUIRE(ctx && ms, VOFPC_E_INVALID_ARG, "ctx_class_ms: null argument");
  VOFPC_REQUIRE(ctx->time_classes, VOFPC_E_STATE, "ctx_class_ms: class timing is not enabled on this context");
  VOFPC_HIP(hipSetDevice(ctx->device));
  for (int c = 0; c < kClasses; ++c) {
    ms[c] = ms[kClasses + c] = -1.0f;
    if (ctx->cls_rec[c]) {
      VOFPC_HIP(hipEventSynchronize(ctx->cls_ev[c][1]));
      VOFPC_HIP(hipEventElapsedTime(&ms[c], ctx->cls_ev[c][0], ctx->cls_ev[c][1]));
      ctx->cls_rec[c] = false;
    }
    if (ctx->pass_rec[c]) {
      VOFPC_HIP(hipEventSynchronize(ctx->pass_ev[c][1]));
      VOFPC_HIP(hipEventElapsedTime(&ms[kClasses + c], ctx->pass_ev[c][0], ctx->pass_ev[c][1]));
      ctx->pass_rec[c] = false;
    }
  }
  return VOFPC_OK;
}


// ---------------------------------------------------------------- autotuner
namespace {
struct TuneBuffers {
  int32_t *mixed = nullptr, *band = nullptr, *counts = nullptr, *status = nullptr, *iters = nullptr;
  double *s = nullptr, *n = nullptr, *A = nullptr, *d = nullptr, *ag = nullptr;
  ~TuneBuffers() {
    (void)hipFree(mixed); (void)hipFree(band); (void)hipFree(counts); (void)hipFree(status); (void)hipFree(iters);
    (void)hipFree(s); (void)hipFree(n); (void)hipFree(A); (void)hipFree(d); (void)hipFree(ag);
  }
};

// Whether class c of mesh M has a build of flavour f.
bool flavour_ok(vofpc_mesh M, int c, int f) {
  if (f == VOFPC_FLAVOUR_WAVE3) return true;
  if (f == VOFPC_FLAVOUR_WAVE4) return c <= 2;
  if (f >= 10 && f <= 26) return thin_available(c, f - 10, M->class_max[c]);
  return false;
}

// The flavours the tuner tries for class c.
int candidates(vofpc_mesh M, int c, int out[8]) {
  int n = 0;
  const int all[] = {VOFPC_FLAVOUR_WAVE3, VOFPC_FLAVOUR_WAVE4, 11, 12, 14, 18, 26};
  for (int f : all)
    if (flavour_ok(M, c, f)) out[n++] = f;
  return n;
}

std::string tune_key(vofpc_ctx ctx, vofpc_mesh M, const vofpc_recon_opts &o) {
  hipDeviceProp_t prop;
  std::string arch = "gpu";
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
  for (char &ch : arch)
    if (ch == ' ' || ch == ':') ch = '_';
  char buf[384];
  snprintf(buf, sizeof buf, "%s cu%d n%lld f%lld v%lld c%lld,%lld,%lld,%lld o%d,%d,%d,%d,%.3g", arch.c_str(),
           ctx->n_cu, (long long)M->d.n_cells, (long long)M->d.n_faces, (long long)M->d.n_verts,
           (long long)M->class_cells[0], (long long)M->class_cells[1], (long long)M->class_cells[2],
           (long long)M->class_cells[3], o.vertex_mode, o.fixed_iso, o.bracket, o.max_iter, o.tol_rel);
  return buf;
}
}  // namespace

}  // namespace vofpc

extern "C" vofpc_status vofpc_mesh_set_tune(vofpc_mesh M, const int32_t tune[4]) {
  using namespace vofpc;
  clear_error();
  VOFPC_REQUIRE(M && tune, VOFPC_E_INVALID_ARG, "mesh_set_tune: null argument");
  for (int c = 0; c < kClasses; ++c)
    VOFPC_REQUIRE(M->class_cells[c] == 0 || flavour_ok(M, c, tune[c]), VOFPC_E_INVALID_ARG,
                  "mesh_set_tune: flavour " + std::to_string(tune[c]) + " has no build for class " +
                      std::to_string(c));
  for (int c = 0; c < kClasses; ++c)
    if (M->class_cells[c] > 0) M->tune[c] = tune[c];
  return VOFPC_OK;
}

extern "C" vofpc_status vofpc_autotune(vofpc_ctx ctx, vofpc_mesh M, const double *alpha, const vofpc_recon_opts *opts,
                                       const char *cache_path, int32_t *choice, int32_t *from_cache) {
  using namespace vofpc;
  clear_error();
  VOFPC_REQUIRE(ctx && M && alpha, VOFPC_E_INVALID_ARG, "autotune: null argument");
  VOFPC_REQUIRE(M->ctx && M->ctx->device == ctx->device, VOFPC_E_STATE, "autotune: mesh on another device");
  VOFPC_HIP(hipSetDevice(ctx->device));
  vofpc_recon_opts o;
  if (opts) o = *opts; else vofpc_recon_opts_default(&o);
  if (from_cache) *from_cache = 0;
  const std::string key = tune_key(ctx, M, o);
  const std::string tag = "vofpc-tune " + key + " :";
  if (cache_path) {
    if (FILE *f = fopen(cache_path, "r")) {
      char line[512];
      int hit[kClasses];
      bool found = false;
      while (fgets(line, sizeof line, f)) {
        if (strncmp(line, tag.c_str(), tag.size()) != 0) continue;
        int t[kClasses];
        if (sscanf(line + tag.size(), "%d %d %d %d", &t[0], &t[1], &t[2], &t[3]) != kClasses) continue;
        bool ok = true;
        for (int c = 0; c < kClasses; ++c) ok = ok && (M->class_cells[c] == 0 || flavour_ok(M, c, t[c]));
        if (!ok) continue;
        for (int c = 0; c < kClasses; ++c) hit[c] = t[c];
        found = true;
      }
      fclose(f);
      if (found) {
        for (int c = 0; c < kClasses; ++c)
          if (M->class_cells[c] > 0) M->tune[c] = hit[c];
        if (from_cache) *from_cache = 1;
        if (choice)
          for (int c = 0; c < kClasses; ++c) choice[c] = M->tune[c];
        return VOFPC_OK;
      }
    }
  }
  // time the flavours on this field (greedy per class, all classes launched)
  const int64_t N = M->d.n_cells;
  int saved[kClasses];
  for (int c = 0; c < kClasses; ++c) saved[c] = M->tune[c];
  TuneBuffers b;
  if (hipMalloc(&b.mixed, 4 * N) || hipMalloc(&b.band, 4 * N) || hipMalloc(&b.counts, 8) ||
      hipMalloc(&b.status, 4 * N) || hipMalloc(&b.iters, 4 * N) || hipMalloc(&b.s, 8 * N) ||
      hipMalloc(&b.n, 24 * N) || hipMalloc(&b.A, 8 * N) || hipMalloc(&b.d, 8 * N) || hipMalloc(&b.ag, 8 * N)) {
    set_error("autotune: hipMalloc of the trial buffers failed");
    return VOFPC_E_OOM;
  }
  vofpc_interface itf;
  itf.s = b.s; itf.n = b.n; itf.A = b.A; itf.d = b.d; itf.alpha_got = b.ag; itf.status = b.status;
  itf.iters = b.iters; itf.cap = N;
  vofpc_status st = launch_compact(ctx, M, alpha, o.eps_mixed, b.mixed, b.band, b.counts);
  if (st) return st;
  hipEvent_t e0, e1;
  VOFPC_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    set_error("autotune: hipEventCreate failed");
    return VOFPC_E_HIP;
  }
  for (int c = 0; c < kClasses && !st; ++c) {
    if (M->class_cells[c] == 0 || (!M->bucketed && c != M->max_class)) continue;
    int cand[8];
    const int nc = candidates(M, c, cand);
    if (nc < 2) continue;
    float best = 0.f;
    int best_f = M->tune[c];
    for (int i = 0; i < nc && !st; ++i) {
      M->tune[c] = cand[i];
      st = launch_reconstruct(ctx, M, alpha, b.mixed, b.counts, &o, nullptr, nullptr, &itf);
      if (st) break;
      if (hipEventRecord(e0, ctx->stream) != hipSuccess) { st = VOFPC_E_HIP; set_error("autotune: event record"); break; }
      for (int r = 0; r < 3 && !st; ++r) st = launch_reconstruct(ctx, M, alpha, b.mixed, b.counts, &o, nullptr, nullptr, &itf);
      if (st) break;
      if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        st = VOFPC_E_HIP;
        set_error("autotune: event wait failed");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (i == 0 || ms < best) { best = ms; best_f = cand[i]; }
    }
    M->tune[c] = best_f;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!st && hipStreamSynchronize(ctx->stream) != hipSuccess) {
    st = VOFPC_E_HIP;
    set_error("autotune: stream synchronisation failed");
  }
  if (st) {
    for (int c = 0; c < kClasses; ++c) M->tune[c] = saved[c];
    return st;
  }
  if (cache_path) {
    if (FILE *f = fopen(cache_path, "a")) {
      fprintf(f, "%s %d %d %d %d\n", tag.c_str(), M->tune[0], M->tune[1], M->tune[2], M->tune[3]);
      fclose(f);
    }
  }
  if (choice)
    for (int c = 0; c < kClasses; ++c) choice[c] = M->tune[c];
  return VOFPC_OK;
}
