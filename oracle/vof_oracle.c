/* Plain single-threaded FP64 CPU oracle for the interface hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the tests, the smoke check and the bench's CPU
 * baseline do.  It shares no code with the HIP library.
 *
 * What it computes, step by step, in the order the method states it:
 *
 *   geometry     face area vectors / centroids, cell volumes / centroids
 *                (finite-volume cell-centred storage, Sec. 5 and App. B);
 *   vertex field alpha at the polyhedron vertices (Sec. 2.1 says the iso-
 *                surface is taken from a field defined at the vertices; the
 *                cell-to-vertex rule is not given: inverse-distance average
 *                of the cells sharing the vertex);
 *   cut          for an isovalue s, edge intersections by linear interpolation
 *                (Eq. edge_intersection), assembled into iso-polygons through
 *                the faces (Sec. 2.1, isopolygon assembly); the liquid volume
 *                by the divergence theorem over the liquid face parts and the
 *                iso-polygons;
 *   root-find    bisection on s until the liquid volume equals alpha V_P
 *                (the volume-matched reading of the reconstruction);
 *   gradient     least squares over face neighbours with the interface
 *                modification (Sec. 2.4.4 "Interface-modified temperature
 *                gradient", Eq. front_interpolation, App. B);
 *   mass rate    q_l, q_v, mdot = (q_l+q_v)/(h_lv V_P) (Eq. mass_transfer),
 *                Qdot = -mdot h_lv (Eq. latent_source), only where A_int > 0.
 *
 * Conventions where the paper is silent (each one is listed with its reason
 * in the design notes of the repository):
 *   - a vertex is liquid when phi >= s;
 *   - a face with 4 or more crossings pairs each exit with the next entry in
 *     loop order when the face-mean phi is >= s (liquid connected), else with
 *     the previous entry;
 *   - each iso-loop is fanned from its length-weighted polyline centroid;
 *   - the interface normal points from vapour to liquid;
 *   - the crossing point of a cell-centre connection is the linear
 *     interpolation of alpha, t = (a_P - 1/2)/(a_P - a_Q) (the printed
 *     Eq. front_interpolation gives the mirror point; a flag selects it).
 *
 * Compiled with -O2 -ffp-contract=off: no fused multiply-add contraction.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXF 256   /* faces per cell */
#define ORC_MAXV 256   /* vertices per cell */
#define ORC_MAXFV 64   /* vertices per face */
#define ORC_MAXX 512   /* crossings per cell */

enum {
  ORC_OK = 0,
  ORC_NOT_MIXED = 1,
  ORC_LEARNED_FALLBACK = 2,
  ORC_DEGENERATE = 3,
  ORC_MAX_ITER = 4,
  ORC_G_SINGULAR = 5,
  ORC_BAD_INPUT = 6,
  ORC_NO_ROOT = 7
};

typedef struct {
  int64_t n_cells, n_faces, n_verts;
  const int64_t *cell_face_off;
  const int32_t *cell_face;
  const int64_t *face_vert_off;
  const int32_t *face_vert;
  const int32_t *face_owner;
  const int32_t *face_neigh;
  const int8_t *face_bc;
  const double *vert_xyz; /* [3][n_verts] */
} orc_mesh;

/* ------------------------------------------------------------------ vectors */
static void v_sub(const double *a, const double *b, double *o) {
  o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static void v_cross(const double *a, const double *b, double *o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static double v_dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double v_det(const double *a, const double *b, const double *c) {
  double t[3];
  v_cross(b, c, t);
  return v_dot(a, t);
}
static void vtx(const orc_mesh *m, int64_t v, double *o) {
  o[0] = m->vert_xyz[v];
  o[1] = m->vert_xyz[m->n_verts + v];
  o[2] = m->vert_xyz[2 * m->n_verts + v];
}

/* ----------------------------------------------------------------- geometry */
/* Face area vector S_f (right-hand rule on the stored loop, i.e. pointing out
 * of the owner) and area centroid x_f, from the fan of triangles around the
 * vertex mean.  Output SoA [3][NF]. */
int orc_face_geometry(const orc_mesh *m, double *Sf, double *xf) {
  for (int64_t f = 0; f < m->n_faces; ++f) {
    int64_t o = m->face_vert_off[f], n = m->face_vert_off[f + 1] - o;
    if (n < 3) return -1;
    double c[3] = {0, 0, 0}, p[3];
    for (int64_t k = 0; k < n; ++k) {
      vtx(m, m->face_vert[o + k], p);
      c[0] += p[0]; c[1] += p[1]; c[2] += p[2];
    }
    c[0] /= (double)n; c[1] /= (double)n; c[2] /= (double)n;
    double S[3] = {0, 0, 0}, xs[3] = {0, 0, 0}, tri[3][3], a[3], b[3], s[3];
    /* first pass: total area vector gives the face normal direction */
    for (int64_t k = 0; k < n; ++k) {
      vtx(m, m->face_vert[o + k], tri[0]);
      vtx(m, m->face_vert[o + (k + 1) % n], tri[1]);
      v_sub(tri[0], c, a);
      v_sub(tri[1], c, b);
      v_cross(a, b, s);
      S[0] += 0.5 * s[0]; S[1] += 0.5 * s[1]; S[2] += 0.5 * s[2];
    }
    double Amag = sqrt(v_dot(S, S));
    if (!(Amag > 0)) return -2;
    double nh[3] = {S[0] / Amag, S[1] / Amag, S[2] / Amag}, wsum = 0;
    for (int64_t k = 0; k < n; ++k) {
      vtx(m, m->face_vert[o + k], tri[0]);
      vtx(m, m->face_vert[o + (k + 1) % n], tri[1]);
      v_sub(tri[0], c, a);
      v_sub(tri[1], c, b);
      v_cross(a, b, s);
      double w = 0.5 * v_dot(s, nh);  /* signed triangle area */
      for (int d = 0; d < 3; ++d) xs[d] += w * (c[d] + tri[0][d] + tri[1][d]) / 3.0;
      wsum += w;
    }
    for (int d = 0; d < 3; ++d) {
      Sf[d * m->n_faces + f] = S[d];
      xf[d * m->n_faces + f] = xs[d] / wsum;
    }
  }
  return 0;
}

/* Cell volume and centroid, from the tetrahedra (o, c_f, v_k, v_k+1) where o
 * is the vertex mean of the cell and c_f the vertex mean of face f (the cell
 * is star-shaped with respect to o).  xc is SoA [3][N]. */
int orc_cell_geometry(const orc_mesh *m, double *V, double *xc) {
  for (int64_t P = 0; P < m->n_cells; ++P) {
    double o[3] = {0, 0, 0}, p[3];
    int64_t cnt = 0;
    for (int64_t i = m->cell_face_off[P]; i < m->cell_face_off[P + 1]; ++i) {
      int32_t f = m->cell_face[i];
      for (int64_t k = m->face_vert_off[f]; k < m->face_vert_off[f + 1]; ++k) {
        vtx(m, m->face_vert[k], p);
        o[0] += p[0]; o[1] += p[1]; o[2] += p[2];
        ++cnt;
      }
    }
    if (cnt == 0) return -1;
    /* mean over face-vertex incidences: still an interior point of a convex cell */
    o[0] /= (double)cnt; o[1] /= (double)cnt; o[2] /= (double)cnt;
    double vol = 0, mom[3] = {0, 0, 0};
    for (int64_t i = m->cell_face_off[P]; i < m->cell_face_off[P + 1]; ++i) {
      int32_t f = m->cell_face[i];
      int64_t fo = m->face_vert_off[f], n = m->face_vert_off[f + 1] - fo;
      double sgn = (m->face_owner[f] == P) ? 1.0 : -1.0;
      double c[3] = {0, 0, 0};
      for (int64_t k = 0; k < n; ++k) {
        vtx(m, m->face_vert[fo + k], p);
        c[0] += p[0]; c[1] += p[1]; c[2] += p[2];
      }
      c[0] /= (double)n; c[1] /= (double)n; c[2] /= (double)n;
      for (int64_t k = 0; k < n; ++k) {
        double a[3], b[3], A[3], B[3], C[3];
        vtx(m, m->face_vert[fo + k], a);
        vtx(m, m->face_vert[fo + (k + 1) % n], b);
        v_sub(c, o, A);
        v_sub(a, o, B);
        v_sub(b, o, C);
        double tv = sgn * v_det(A, B, C) / 6.0;
        vol += tv;
        for (int d = 0; d < 3; ++d) mom[d] += tv * (o[d] + c[d] + a[d] + b[d]) / 4.0;
      }
    }
    if (!(vol > 0)) return -2;
    V[P] = vol;
    for (int d = 0; d < 3; ++d) xc[d * m->n_cells + P] = mom[d] / vol;
  }
  return 0;
}

/* ------------------------------------------------------------- vertex field */
/* phi_v = sum_c w_c alpha_c / sum_c w_c over the cells c sharing vertex v,
 * with w_c = 1/|x_v - x_c| (mode 0, inverse distance) or w_c = 1 (mode 1). */
int orc_vertex_field(const orc_mesh *m, const double *xc, const double *alpha, int mode, double *phi) {
  double *num = calloc((size_t)m->n_verts, sizeof(double));
  double *den = calloc((size_t)m->n_verts, sizeof(double));
  int64_t *last = malloc((size_t)m->n_verts * sizeof(int64_t));
  if (!num || !den || !last) { free(num); free(den); free(last); return -1; }
  for (int64_t v = 0; v < m->n_verts; ++v) last[v] = -1;
  for (int64_t P = 0; P < m->n_cells; ++P) {
    for (int64_t i = m->cell_face_off[P]; i < m->cell_face_off[P + 1]; ++i) {
      int32_t f = m->cell_face[i];
      for (int64_t k = m->face_vert_off[f]; k < m->face_vert_off[f + 1]; ++k) {
        int32_t v = m->face_vert[k];
        if (last[v] == P) continue; /* each cell once per vertex */
        last[v] = P;
        double w = 1.0;
        if (mode == 0) {
          double p[3], c[3] = {xc[P], xc[m->n_cells + P], xc[2 * m->n_cells + P]}, d[3];
          vtx(m, v, p);
          v_sub(p, c, d);
          w = 1.0 / sqrt(v_dot(d, d));
        }
        num[v] += w * alpha[P];
        den[v] += w;
      }
    }
  }
  for (int64_t v = 0; v < m->n_verts; ++v) phi[v] = den[v] > 0 ? num[v] / den[v] : 0.0;
  free(num); free(den); free(last);
  return 0;
}

/* ------------------------------------------------------- cell-local polyhedron */
typedef struct {
  int nf, nv;
  int fo[ORC_MAXF + 1];     /* face offsets into lv */
  int lv[ORC_MAXF * 8 + ORC_MAXFV]; /* local vertex ids, loops outward from the cell */
  double X[ORC_MAXV][3];    /* vertex positions relative to the cell centroid */
  double phi[ORC_MAXV];
  double cf[ORC_MAXF][3];   /* face vertex mean (relative) */
  int32_t gv[ORC_MAXV];     /* global vertex ids */
} poly_t;

static int build_poly(const orc_mesh *m, int64_t P, const double *xP, const double *phi_glob, poly_t *py) {
  py->nf = 0;
  py->nv = 0;
  py->fo[0] = 0;
  int64_t nfc = m->cell_face_off[P + 1] - m->cell_face_off[P];
  if (nfc > ORC_MAXF) return -1;
  for (int64_t i = m->cell_face_off[P]; i < m->cell_face_off[P + 1]; ++i) {
    int32_t f = m->cell_face[i];
    int64_t o = m->face_vert_off[f], n = m->face_vert_off[f + 1] - o;
    if (n > ORC_MAXFV || py->fo[py->nf] + n > (int)(sizeof(py->lv) / sizeof(int))) return -2;
    int rev = (m->face_owner[f] != P);
    for (int64_t k = 0; k < n; ++k) {
      int32_t g = m->face_vert[o + (rev ? (n - 1 - k) : k)];
      int l = -1;
      for (int j = 0; j < py->nv; ++j)
        if (py->gv[j] == g) { l = j; break; }
      if (l < 0) {
        if (py->nv >= ORC_MAXV) return -3;
        l = py->nv++;
        py->gv[l] = g;
        double p[3];
        vtx(m, g, p);
        v_sub(p, xP, py->X[l]);
        py->phi[l] = phi_glob ? phi_glob[g] : 0.0;
      }
      py->lv[py->fo[py->nf] + k] = l;
    }
    py->fo[py->nf + 1] = py->fo[py->nf] + (int)n;
    py->nf++;
  }
  for (int f = 0; f < py->nf; ++f) {
    double c[3] = {0, 0, 0};
    int n = py->fo[f + 1] - py->fo[f];
    for (int k = 0; k < n; ++k)
      for (int d = 0; d < 3; ++d) c[d] += py->X[py->lv[py->fo[f] + k]][d];
    for (int d = 0; d < 3; ++d) py->cf[f][d] = c[d] / (double)n;
  }
  return 0;
}

/* ----------------------------------------------------------------- the cut */
typedef struct {
  double V;        /* liquid volume */
  double S[3];     /* sum of iso-loop area vectors, pointing vapour -> liquid */
  double A;        /* sum of |S_k| */
  double c[3];     /* |S_k|-weighted mean of loop centres (relative) */
  int nloops;
  int ncross;
} cut_t;

/* crossing point on the edge between vertices a and b of the polyhedron, at
 * isovalue s; computed from the liquid end so both faces sharing the edge
 * obtain the same point (Eq. edge_intersection with alpha_iso = s). */
static void crossing(const poly_t *py, int a, int b, double s, double *p) {
  int i = py->phi[a] >= s ? a : b; /* liquid end */
  int j = (i == a) ? b : a;
  double lam = (s - py->phi[i]) / (py->phi[j] - py->phi[i]);
  for (int d = 0; d < 3; ++d) p[d] = py->X[i][d] + lam * (py->X[j][d] - py->X[i][d]);
}

typedef struct {
  int ea, eb;      /* exit edge (start) local vertex pair, as min/max */
  int xa, xb;
  int na, nb;      /* entry edge (end) */
  double ps[3];    /* start point (exit crossing) */
  double pe[3];    /* end point (entry crossing) */
  int next;        /* next chord along the iso-loop */
  int done;
} chord_t;

static int same_edge(int a0, int a1, int b0, int b1) {
  return (a0 == b0 && a1 == b1) || (a0 == b1 && a1 == b0);
}

int orc_cut_poly(const poly_t *py, double s, cut_t *out) {
  static chord_t ch[ORC_MAXX];
  int nch = 0;
  double Vf = 0;
  out->ncross = 0;
  for (int f = 0; f < py->nf; ++f) {
    int o = py->fo[f], n = py->fo[f + 1] - o;
    const double *cf = py->cf[f];
    /* crossings of this face in loop order: position k means edge (k, k+1) */
    int xk[ORC_MAXFV], xexit[ORC_MAXFV], nx = 0;
    double fmean = 0;
    for (int k = 0; k < n; ++k) fmean += py->phi[py->lv[o + k]];
    fmean /= (double)n;
    for (int k = 0; k < n; ++k) {
      int a = py->lv[o + k], b = py->lv[o + (k + 1) % n];
      int la = py->phi[a] >= s, lb = py->phi[b] >= s;
      if (la && lb) {
        Vf += v_det(cf, py->X[a], py->X[b]);
      } else if (la && !lb) {            /* exit: liquid -> vapour */
        double p[3];
        crossing(py, a, b, s, p);
        Vf += v_det(cf, py->X[a], p);
        xk[nx] = k; xexit[nx] = 1; ++nx;
      } else if (!la && lb) {            /* entry: vapour -> liquid */
        double p[3];
        crossing(py, a, b, s, p);
        Vf += v_det(cf, p, py->X[b]);
        xk[nx] = k; xexit[nx] = 0; ++nx;
      }
    }
    out->ncross += nx;
    if (nx == 0) continue;
    /* pair exits with entries; an odd count cannot happen on a closed loop */
    if (nx % 2) return -1;
    int liquid_connected = fmean >= s;
    for (int q = 0; q < nx; ++q) {
      if (!xexit[q]) continue;
      int r;
      if (nx == 2 || liquid_connected) {
        r = q;
        do { r = (r + 1) % nx; } while (xexit[r]);
      } else {
        r = q;
        do { r = (r - 1 + nx) % nx; } while (xexit[r]);
      }
      if (nch >= ORC_MAXX) return -2;
      chord_t *c = &ch[nch++];
      int ka = xk[q], kb = xk[r];
      c->xa = py->lv[o + ka]; c->xb = py->lv[o + (ka + 1) % n];
      c->na = py->lv[o + kb]; c->nb = py->lv[o + (kb + 1) % n];
      crossing(py, c->xa, c->xb, s, c->ps);
      crossing(py, c->na, c->nb, s, c->pe);
      c->done = 0;
      /* the chord closes this face's liquid polygon: exit -> entry */
      Vf += v_det(cf, c->ps, c->pe);
    }
  }
  /* link chords into iso-loops: after chord c (exit edge E), the loop goes on
   * with the chord of the neighbouring face whose entry edge is E */
  for (int i = 0; i < nch; ++i) {
    ch[i].next = -1;
    for (int j = 0; j < nch; ++j)
      if (same_edge(ch[i].xa, ch[i].xb, ch[j].na, ch[j].nb)) { ch[i].next = j; break; }
    if (ch[i].next < 0) return -3;
  }
  double Vi = 0, Ssum[3] = {0, 0, 0}, Asum = 0, cw[3] = {0, 0, 0};
  int nloops = 0;
  for (int i = 0; i < nch; ++i) {
    if (ch[i].done) continue;
    /* loop points: start points of the chords in link order */
    int idx[ORC_MAXX], len = 0, j = i;
    do {
      if (len >= ORC_MAXX) return -4;
      idx[len++] = j;
      ch[j].done = 1;
      j = ch[j].next;
    } while (j != i && !ch[j].done);
    if (j != i) return -5; /* not a permutation cycle */
    /* fan apex: centroid of the loop taken as a polyline (segments weighted
     * by length), which moves continuously when two loop points merge at a
     * polyhedron vertex; the plain mean of the points would jump there */
    double ck[3] = {0, 0, 0}, ltot = 0;
    for (int k = 0; k < len; ++k) {
      const double *a = ch[idx[k]].ps, *b = ch[idx[(k + 1) % len]].ps;
      double e[3];
      v_sub(b, a, e);
      double l = sqrt(v_dot(e, e));
      for (int d = 0; d < 3; ++d) ck[d] += l * (a[d] + b[d]) * 0.5;
      ltot += l;
    }
    if (ltot > 0) {
      for (int d = 0; d < 3; ++d) ck[d] /= ltot;
    } else {
      for (int d = 0; d < 3; ++d) ck[d] = ch[idx[0]].ps[d];
    }
    double Sk[3] = {0, 0, 0};
    for (int k = 0; k < len; ++k) {
      const double *a = ch[idx[k]].ps, *b = ch[idx[(k + 1) % len]].ps;
      double u[3], w[3], t[3];
      Vi += v_det(ck, a, b);
      v_sub(a, ck, u);
      v_sub(b, ck, w);
      v_cross(u, w, t);
      /* the fan is oriented out of the liquid; the interface normal is the
       * opposite (vapour -> liquid) */
      for (int d = 0; d < 3; ++d) Sk[d] -= 0.5 * t[d];
    }
    double Ak = sqrt(v_dot(Sk, Sk));
    for (int d = 0; d < 3; ++d) {
      Ssum[d] += Sk[d];
      cw[d] += Ak * ck[d];
    }
    Asum += Ak;
    ++nloops;
  }
  out->V = (Vf + Vi) / 6.0;
  for (int d = 0; d < 3; ++d) {
    out->S[d] = Ssum[d];
    out->c[d] = Asum > 0 ? cw[d] / Asum : 0.0;
  }
  out->A = Asum;
  out->nloops = nloops;
  return 0;
}

/* One cut of cell P at isovalue s (test entry point). res = {V, S[3], A, c[3]
 * relative to the centroid, nloops}. */
int orc_cut_cell(const orc_mesh *m, int64_t P, const double *xc, const double *phi, double s, double *res) {
  static poly_t py;
  double xP[3] = {xc[P], xc[m->n_cells + P], xc[2 * m->n_cells + P]};
  int e = build_poly(m, P, xP, phi, &py);
  if (e) return e;
  cut_t c;
  e = orc_cut_poly(&py, s, &c);
  if (e) return e - 10;
  res[0] = c.V;
  res[1] = c.S[0]; res[2] = c.S[1]; res[3] = c.S[2];
  res[4] = c.A;
  res[5] = c.c[0]; res[6] = c.c[1]; res[7] = c.c[2];
  res[8] = c.nloops;
  return 0;
}

/* ------------------------------------------------------ least-squares solve */
/* Solve G g = b for symmetric 3x3 G by the explicit inverse (adjugate over
 * determinant, App. B).  Returns 1 when G is singular: det <= 1e-12 (tr/3)^3. */
static int solve_sym3(const double G[6] /* xx yy zz xy xz yz */, const double *b, double *g) {
  double xx = G[0], yy = G[1], zz = G[2], xy = G[3], xz = G[4], yz = G[5];
  double c00 = yy * zz - yz * yz;
  double c01 = xz * yz - xy * zz;
  double c02 = xy * yz - xz * yy;
  double c11 = xx * zz - xz * xz;
  double c12 = xy * xz - xx * yz;
  double c22 = xx * yy - xy * xy;
  double det = xx * c00 + xy * c01 + xz * c02;
  double tr = (xx + yy + zz) / 3.0;
  if (!(det > 1e-12 * tr * tr * tr)) {
    g[0] = g[1] = g[2] = 0.0;
    return 1;
  }
  g[0] = (c00 * b[0] + c01 * b[1] + c02 * b[2]) / det;
  g[1] = (c01 * b[0] + c11 * b[1] + c12 * b[2]) / det;
  g[2] = (c02 * b[0] + c12 * b[1] + c22 * b[2]) / det;
  return 0;
}

/* Cells sharing at least one vertex with each cell (the extended stencil of
 * App. B "Neighbour stencil"), as CSR over cells, P itself excluded, in the
 * order first met walking P's faces and their vertices.  Caller frees. */
static int vertex_neighbours(const orc_mesh *m, int64_t **off_out, int32_t **nb_out) {
  int64_t N = m->n_cells, NV = m->n_verts;
  /* vertex -> cells: each cell once per vertex */
  int64_t *vo = (int64_t *)calloc((size_t)NV + 1, sizeof(int64_t));
  int32_t *last = (int32_t *)malloc(sizeof(int32_t) * (size_t)NV);
  if (!vo || !last) { free(vo); free(last); return 1; }
  for (int pass = 0; pass < 2; ++pass) {
    for (int64_t v = 0; v < NV; ++v) last[v] = -1;
    int64_t *fill = NULL;
    int32_t *vc = NULL;
    if (pass == 1) {
      for (int64_t v = 0; v < NV; ++v) vo[v + 1] += vo[v];
      fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)NV);
      vc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(vo[NV] ? vo[NV] : 1));
      if (!fill || !vc) { free(fill); free(vc); free(vo); free(last); return 1; }
      for (int64_t v = 0; v < NV; ++v) fill[v] = vo[v];
    }
    for (int64_t P = 0; P < N; ++P)
      for (int64_t i = m->cell_face_off[P]; i < m->cell_face_off[P + 1]; ++i) {
        int32_t f = m->cell_face[i];
        for (int64_t k = m->face_vert_off[f]; k < m->face_vert_off[f + 1]; ++k) {
          int32_t v = m->face_vert[k];
          if (last[v] == P) continue;
          last[v] = (int32_t)P;
          if (pass == 0) vo[v + 1]++;
          else vc[fill[v]++] = (int32_t)P;
        }
      }
    if (pass == 1) {
      /* cell -> vertex neighbours */
      int32_t *stamp = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
      int64_t *off = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
      int64_t cap = 0;
      if (!stamp || !off) { free(stamp); free(off); free(fill); free(vc); free(vo); free(last); return 1; }
      for (int64_t P = 0; P < N; ++P) stamp[P] = -1;
      /* count */
      for (int64_t P = 0; P < N; ++P) {
        stamp[P] = (int32_t)P;
        for (int64_t i = m->cell_face_off[P]; i < m->cell_face_off[P + 1]; ++i) {
          int32_t f = m->cell_face[i];
          for (int64_t k = m->face_vert_off[f]; k < m->face_vert_off[f + 1]; ++k) {
            int32_t v = m->face_vert[k];
            for (int64_t j = vo[v]; j < vo[v + 1]; ++j)
              if (stamp[vc[j]] != (int32_t)P) { stamp[vc[j]] = (int32_t)P; off[P + 1]++; }
          }
        }
      }
      for (int64_t P = 0; P < N; ++P) off[P + 1] += off[P];
      cap = off[N];
      int32_t *nb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap ? cap : 1));
      if (!nb) { free(stamp); free(off); free(fill); free(vc); free(vo); free(last); return 1; }
      for (int64_t P = 0; P < N; ++P) stamp[P] = -1;
      for (int64_t P = 0; P < N; ++P) {
        int64_t w = off[P];
        stamp[P] = (int32_t)P;
        for (int64_t i = m->cell_face_off[P]; i < m->cell_face_off[P + 1]; ++i) {
          int32_t f = m->cell_face[i];
          for (int64_t k = m->face_vert_off[f]; k < m->face_vert_off[f + 1]; ++k) {
            int32_t v = m->face_vert[k];
            for (int64_t j = vo[v]; j < vo[v + 1]; ++j)
              if (stamp[vc[j]] != (int32_t)P) { stamp[vc[j]] = (int32_t)P; nb[w++] = vc[j]; }
          }
        }
      }
      free(stamp); free(fill); free(vc);
      *off_out = off;
      *nb_out = nb;
    }
  }
  free(vo); free(last);
  return 0;
}

/* Least-squares gradient of a cell field (App. B; interface modification of
 * Sec. 2.4.4).  modified: replace a crossing neighbour by (x_f, value_sat);
 * printed: use the printed Eq. front_interpolation weight |a_Q-1/2|/|a_P-a_Q|
 * instead of the linear-interpolation weight (a_P-1/2)/(a_P-a_Q).
 * weight (App. B "Weighting"): 0 uniform, 1 inverse distance 1/|r|, 2 inverse
 * distance squared 1/|r|^2, with r the (possibly shortened) displacement;
 * the fit minimises sum w (dphi - g.r)^2, so G = sum w r r^T, b = sum w r dphi.
 * extended (App. B "Neighbour stencil"): the interior neighbours are all
 * cells sharing a vertex with P instead of the face neighbours; the crossing
 * test and shortening apply to each centre connection alike.
 * Boundary faces with bc==1 act as neighbours at the face centroid with the
 * value Tb[f]; bc==2 (symmetry) faces are skipped.  grad is SoA [3][N].
 * only (optional, int8 [N]): compute the cells with only[P] != 0 and give
 * the others status -1 and a NaN gradient (a band is the usual subset). */
static void lsq_add(double *G, double *b, const double *r, double dv, int weight) {
  double w = 1.0;
  if (weight == 1) w = 1.0 / sqrt(v_dot(r, r));
  else if (weight == 2) w = 1.0 / v_dot(r, r);
  G[0] += w * r[0] * r[0]; G[1] += w * r[1] * r[1]; G[2] += w * r[2] * r[2];
  G[3] += w * r[0] * r[1]; G[4] += w * r[0] * r[2]; G[5] += w * r[1] * r[2];
  b[0] += w * r[0] * dv; b[1] += w * r[1] * dv; b[2] += w * r[2] * dv;
}

int orc_grad(const orc_mesh *m, const double *xc, const double *xf, const double *T, const double *Tb,
             double T_sat, const double *alpha, int modified, int printed, int weight, int extended,
             double *grad, int32_t *status, const int8_t *only) {
  int64_t N = m->n_cells;
  int64_t *xoff = NULL;
  int32_t *xnb = NULL;
  if (extended && vertex_neighbours(m, &xoff, &xnb)) return 1;
  for (int64_t P = 0; P < N; ++P) {
    if (only && !only[P]) {
      if (status) status[P] = -1;
      for (int d = 0; d < 3; ++d) grad[d * N + P] = NAN;
      continue;
    }
    double G[6] = {0, 0, 0, 0, 0, 0}, b[3] = {0, 0, 0};
    double xP[3] = {xc[P], xc[N + P], xc[2 * N + P]};
    /* interior neighbours: the face neighbours, or every vertex neighbour */
    int64_t n_in = extended ? xoff[P + 1] - xoff[P] : m->cell_face_off[P + 1] - m->cell_face_off[P];
    for (int64_t j = 0; j < n_in; ++j) {
      int32_t Q;
      if (extended) {
        Q = xnb[xoff[P] + j];
      } else {
        int32_t f = m->cell_face[m->cell_face_off[P] + j];
        Q = (m->face_owner[f] == P) ? m->face_neigh[f] : m->face_owner[f];
        if (Q < 0) continue;
      }
      double xQ[3] = {xc[Q], xc[N + Q], xc[2 * N + Q]};
      double r[3], val = T[Q];
      v_sub(xQ, xP, r);
      if (modified && (alpha[P] - 0.5) * (alpha[Q] - 0.5) < 0.0) {
        double t = printed ? fabs(alpha[Q] - 0.5) / fabs(alpha[P] - alpha[Q])
                           : (alpha[P] - 0.5) / (alpha[P] - alpha[Q]);
        r[0] *= t; r[1] *= t; r[2] *= t;
        val = T_sat;
      }
      lsq_add(G, b, r, val - T[P], weight);
    }
    /* boundary faces with a value: virtual neighbours at the face centroid */
    for (int64_t i = m->cell_face_off[P]; i < m->cell_face_off[P + 1]; ++i) {
      int32_t f = m->cell_face[i];
      if (m->face_neigh[f] >= 0 || m->face_bc[f] != 1) continue;
      double x[3] = {xf[f], xf[m->n_faces + f], xf[2 * m->n_faces + f]}, r[3];
      v_sub(x, xP, r);
      lsq_add(G, b, r, Tb[f] - T[P], weight);
    }
    double g[3];
    int sing = solve_sym3(G, b, g);
    if (status) status[P] = sing ? ORC_G_SINGULAR : ORC_OK;
    for (int d = 0; d < 3; ++d) grad[d * N + P] = g[d];
  }
  free(xoff);
  free(xnb);
  return 0;
}

/* ---------------------------------------------------------- reconstruction */
typedef struct {
  double eps_mixed;   /* mixed when eps < alpha < 1-eps */
  double tol_rel;     /* |V/V_P - alpha| <= tol_rel min(alpha, 1-alpha) */
  int max_iter;
  int vertex_mode;    /* 0 inverse distance, 1 plain mean */
  int fixed_iso;      /* 1: no root-find, cut at iso */
  double iso;
} orc_opts;

static double ulp_of(double x) {
  x = fabs(x);
  return nextafter(x, INFINITY) - x;
}

/* Reconstruct every mixed cell.  Outputs are dense over cells (SoA vectors
 * [3][N]); non-mixed cells get s = NaN, n = 0, A = 0, d = 0, alpha_got =
 * alpha.  phi_in may supply the vertex field (else it is built from alpha);
 * hint_lo/hint_hi may supply a narrowed initial bracket per cell (NaN = none).
 */
/* only (optional, int8 [N]): reconstruct the cells with only[P] != 0 and
 * mark every other cell with status -1 (not processed); NULL: every cell. */
int orc_reconstruct(const orc_mesh *m, const double *V, const double *xc, const double *alpha,
                    const orc_opts *op, const double *phi_in, const double *hint_lo, const double *hint_hi,
                    double *s_out, double *n_out, double *A_out, double *d_out, double *agot,
                    int32_t *status, int32_t *iters, const int8_t *only) {
  int64_t N = m->n_cells;
  double *phi = NULL;
  if (phi_in) {
    phi = (double *)phi_in;
  } else {
    phi = malloc((size_t)m->n_verts * sizeof(double));
    if (!phi) return -1;
    orc_vertex_field(m, xc, alpha, op->vertex_mode, phi);
  }
  static poly_t py;
  int err = 0;
  for (int64_t P = 0; P < N && !err; ++P) {
    double a = alpha[P];
    s_out[P] = NAN;
    A_out[P] = 0; d_out[P] = 0; agot[P] = a; iters[P] = 0;
    for (int d = 0; d < 3; ++d) n_out[d * N + P] = 0;
    if (only && !only[P]) { status[P] = -1; continue; }
    if (!(a >= 0.0 && a <= 1.0)) { status[P] = ORC_BAD_INPUT; continue; }
    if (!(a > op->eps_mixed && a < 1.0 - op->eps_mixed)) { status[P] = ORC_NOT_MIXED; continue; }
    double xP[3] = {xc[P], xc[N + P], xc[2 * N + P]};
    if (build_poly(m, P, xP, phi, &py)) { err = -2; break; }
    int st = ORC_OK;
    double pmin = INFINITY, pmax = -INFINITY;
    for (int v = 0; v < py.nv; ++v) {
      if (py.phi[v] < pmin) pmin = py.phi[v];
      if (py.phi[v] > pmax) pmax = py.phi[v];
    }
    if (pmax - pmin <= 1e-12) {
      /* degenerate vertex field: use the linear field from the plain
       * least-squares gradient of alpha over the interior face neighbours */
      st = ORC_DEGENERATE;
      double G[6] = {0, 0, 0, 0, 0, 0}, b[3] = {0, 0, 0}, g[3];
      for (int64_t i = m->cell_face_off[P]; i < m->cell_face_off[P + 1]; ++i) {
        int32_t f = m->cell_face[i];
        int32_t Q = (m->face_owner[f] == P) ? m->face_neigh[f] : m->face_owner[f];
        if (Q < 0) continue;
        double r[3] = {xc[Q] - xP[0], xc[N + Q] - xP[1], xc[2 * N + Q] - xP[2]};
        double dv = alpha[Q] - a;
        G[0] += r[0] * r[0]; G[1] += r[1] * r[1]; G[2] += r[2] * r[2];
        G[3] += r[0] * r[1]; G[4] += r[0] * r[2]; G[5] += r[1] * r[2];
        b[0] += r[0] * dv; b[1] += r[1] * dv; b[2] += r[2] * dv;
      }
      solve_sym3(G, b, g);
      pmin = INFINITY; pmax = -INFINITY;
      for (int v = 0; v < py.nv; ++v) {
        py.phi[v] = a + v_dot(g, py.X[v]);
        if (py.phi[v] < pmin) pmin = py.phi[v];
        if (py.phi[v] > pmax) pmax = py.phi[v];
      }
      if (pmax - pmin <= 1e-12) { status[P] = st; continue; }
    }
    cut_t c;
    double s;
    int it = 0;
    if (op->fixed_iso) {
      s = op->iso;
      if (orc_cut_poly(&py, s, &c)) { err = -3; break; }
      it = 1;
    } else {
      /* bracket ends and their residuals r = V/V_P - alpha; at phi_min the
       * whole cell is liquid (r = 1 - alpha), at phi_max none of it (r = -alpha) */
      double lo = pmin, hi = pmax, rlo = 1.0 - a, rhi = -a;
      double tol = op->tol_rel * (a < 1.0 - a ? a : 1.0 - a);
      cut_t clo, chi;
      int have_lo = 0, have_hi = 0, done = 0;
      s = NAN;
      if (hint_lo && hint_hi && !isnan(hint_lo[P]) && !isnan(hint_hi[P])) {
        /* narrowed bracket: verify it with two cuts; when it fails keep the
         * part of the full bracket that must hold the root */
        double l2 = hint_lo[P] > pmin ? hint_lo[P] : pmin;
        double h2 = hint_hi[P] < pmax ? hint_hi[P] : pmax;
        if (l2 > h2) { l2 = pmin; h2 = pmax; }
        cut_t cl, chh;
        if (orc_cut_poly(&py, l2, &cl) || orc_cut_poly(&py, h2, &chh)) { err = -3; break; }
        it += 2;
        double rl = cl.V / V[P] - a, rh = chh.V / V[P] - a;
        if (fabs(rl) <= tol) { s = l2; c = cl; done = 1; }
        else if (fabs(rh) <= tol) { s = h2; c = chh; done = 1; }
        else if (rl > 0 && rh < 0) { lo = l2; rlo = rl; clo = cl; have_lo = 1; hi = h2; rhi = rh; chi = chh; have_hi = 1; }
        else if (rl <= 0) { hi = l2; rhi = rl; chi = cl; have_hi = 1; st = st ? st : ORC_LEARNED_FALLBACK; }
        else { lo = h2; rlo = rh; clo = chh; have_lo = 1; st = st ? st : ORC_LEARNED_FALLBACK; }
      }
      int collapsed = 0;
      while (!done) {
        if (it >= op->max_iter) { st = ORC_MAX_ITER; break; }
        s = lo + (hi - lo) / 2.0;
        if (orc_cut_poly(&py, s, &c)) { err = -3; break; }
        ++it;
        double r = c.V / V[P] - a;
        if (fabs(r) <= tol) break;
        if (r > 0) { lo = s; rlo = r; clo = c; have_lo = 1; }
        else { hi = s; rhi = r; chi = c; have_hi = 1; }
        double big = fabs(lo) > fabs(hi) ? fabs(lo) : fabs(hi);
        if (hi - lo <= 2.0 * ulp_of(big)) { collapsed = 1; break; }
      }
      if (err) break;
      if (collapsed) {
        /* no isovalue meets the tolerance: keep the bracket end whose volume
         * is nearer alpha V_P (the volume may jump, e.g. where a face with
         * four crossings changes its pairing) */
        int take_lo = fabs(rlo) <= fabs(rhi);
        s = take_lo ? lo : hi;
        if (take_lo ? have_lo : have_hi) {
          c = take_lo ? clo : chi;
        } else {
          if (orc_cut_poly(&py, s, &c)) { err = -3; break; }
          ++it;
        }
        if (fabs(take_lo ? rlo : rhi) > 1e-10 && st != ORC_MAX_ITER) st = ORC_NO_ROOT;
      }
      if (isnan(s)) { status[P] = st; continue; }
    }
    double Sm = sqrt(v_dot(c.S, c.S));
    s_out[P] = s;
    agot[P] = c.V / V[P];
    iters[P] = it;
    A_out[P] = c.A;
    if (Sm > 0) {
      double nn[3] = {c.S[0] / Sm, c.S[1] / Sm, c.S[2] / Sm};
      for (int d = 0; d < 3; ++d) n_out[d * N + P] = nn[d];
      /* d = n . (x_P - c_int), with x_P the origin of the local frame */
      d_out[P] = -v_dot(nn, c.c);
    }
    status[P] = st;
  }
  if (!phi_in) free(phi);
  return err;
}

/* ------------------------------------------------------------ mass transfer */
/* mdot = (q_l + q_v)/(h_lv V_P), q_l = k_l (gl.n) A, q_v = -k_v (gv.n) A, only
 * where A > 0 (Eq. mass_transfer, Eq. latent_source).  gl/gv NULL selects the
 * one-sided fill from grad: the cell's own phase (liquid when alpha >= 1/2)
 * takes grad, the other phase 0. */
int orc_mass_transfer(int64_t N, const double *V, const double *alpha, const double *n, const double *A,
                      const double *grad, const double *gl, const double *gv, double k_l, double k_v,
                      double h_lv, double *mdot, double *Qdot) {
  for (int64_t P = 0; P < N; ++P) {
    if (!(A[P] > 0)) { mdot[P] = 0; Qdot[P] = 0; continue; }
    double nn[3] = {n[P], n[N + P], n[2 * N + P]};
    double L[3] = {0, 0, 0}, W[3] = {0, 0, 0};
    if (gl && gv) {
      for (int d = 0; d < 3; ++d) { L[d] = gl[d * N + P]; W[d] = gv[d * N + P]; }
    } else if (alpha[P] >= 0.5) {
      for (int d = 0; d < 3; ++d) L[d] = grad[d * N + P];
    } else {
      for (int d = 0; d < 3; ++d) W[d] = grad[d * N + P];
    }
    double ql = k_l * v_dot(L, nn) * A[P];
    double qv = -k_v * v_dot(W, nn) * A[P];
    mdot[P] = (ql + qv) / (h_lv * V[P]);
    Qdot[P] = -mdot[P] * h_lv;
  }
  return 0;
}

/* ------------------------------------------------- gradient extrapolation */
/* Plain least-squares gradient of a cell field over the interior face
 * neighbours of P only (App. B without boundary faces). */
static void lsq_interior(const orc_mesh *m, const double *xc, const double *val, int64_t P, double *g) {
  int64_t N = m->n_cells;
  double G[6] = {0, 0, 0, 0, 0, 0}, b[3] = {0, 0, 0};
  for (int64_t i = m->cell_face_off[P]; i < m->cell_face_off[P + 1]; ++i) {
    int32_t f = m->cell_face[i];
    int32_t Q = (m->face_owner[f] == P) ? m->face_neigh[f] : m->face_owner[f];
    if (Q < 0) continue;
    double r[3] = {xc[Q] - xc[P], xc[N + Q] - xc[N + P], xc[2 * N + Q] - xc[2 * N + P]};
    double dv = val[Q] - val[P];
    G[0] += r[0] * r[0]; G[1] += r[1] * r[1]; G[2] += r[2] * r[2];
    G[3] += r[0] * r[1]; G[4] += r[0] * r[2]; G[5] += r[1] * r[2];
    b[0] += r[0] * dv; b[1] += r[1] * dv; b[2] += r[2] * dv;
  }
  solve_sym3(G, b, g);
}

/* Phase gradients at the interface by pseudo-time extrapolation
 * (Eq. extrapolation, Sec. 2.4.4), applied to each gradient component:
 *   G_l = G_v = grad (the interface-modified gradient) on the domain D, the
 *   cells within `layers` interior-face hops of a mixed cell;
 *   a liquid cell (alpha >= 1/2) keeps G_l and advances G_v, a vapour cell
 *   keeps G_v and advances G_l, with velocity c = sgn(alpha - 1/2) n, where n
 *   is the interface normal of a cell with A > 0 and otherwise the unit plain
 *   least-squares gradient of alpha (no change where that vanishes);
 *   first-order upwind: with w_f = -c.S_f over the faces of P whose
 *   neighbour Q is in D and c.S_f < 0 (S_f outward from P), w = sum w_f,
 *   F_P <- F_P + theta (sum w_f F_Q / w - F_P), theta = min(dtau w / V_P, 1);
 *   Jacobi sweeps, dtau = min |x_Q - x_P| over interior faces;
 *   stop at the first sweep whose largest change is below tol, or after
 *   max_iter sweeps.
 * gl, gv: [3][N] outputs (equal to grad outside D); iters: sweeps done;
 * domain (optional, int8 [N]): 1 on D. */
int orc_extrapolate(const orc_mesh *m, const double *V, const double *xc, const double *Sf, const double *alpha,
                    const double *grad, const double *n_int, const double *A, double eps, int layers, int max_iter,
                    double tol, double *gl, double *gv, int32_t *iters, int8_t *domain) {
  int64_t N = m->n_cells, NF = m->n_faces;
  int *mark = (int *)malloc(sizeof(int) * (size_t)N);
  int *next = (int *)malloc(sizeof(int) * (size_t)N);
  double *nrm = (double *)malloc(sizeof(double) * 3 * (size_t)N);
  double *cur = (double *)malloc(sizeof(double) * 6 * (size_t)N);   /* [field l/v][3][N] */
  double *nxt = (double *)malloc(sizeof(double) * 6 * (size_t)N);
  if (!mark || !next || !nrm || !cur || !nxt) {
    free(mark); free(next); free(nrm); free(cur); free(nxt);
    return 1;
  }
  /* domain: layers of interior face neighbours around the mixed cells */
  for (int64_t P = 0; P < N; ++P) mark[P] = (alpha[P] > eps && alpha[P] < 1.0 - eps) ? 0 : -1;
  for (int l = 1; l <= layers; ++l) {
    memcpy(next, mark, sizeof(int) * (size_t)N);
    for (int64_t f = 0; f < NF; ++f) {
      int32_t o = m->face_owner[f], q = m->face_neigh[f];
      if (q < 0) continue;
      if (mark[o] == l - 1 && mark[q] < 0) next[q] = l;
      if (mark[q] == l - 1 && mark[o] < 0) next[o] = l;
    }
    memcpy(mark, next, sizeof(int) * (size_t)N);
  }
  /* advection direction per domain cell */
  for (int64_t P = 0; P < N; ++P) {
    nrm[P] = nrm[N + P] = nrm[2 * N + P] = 0.0;
    if (mark[P] < 0) continue;
    if (mark[P] == 0 && A[P] > 0) {
      for (int d = 0; d < 3; ++d) nrm[d * N + P] = n_int[d * N + P];
    } else {
      double g[3];
      lsq_interior(m, xc, alpha, P, g);
      double len = sqrt(v_dot(g, g));
      if (len > 0)
        for (int d = 0; d < 3; ++d) nrm[d * N + P] = g[d] / len;
    }
  }
  double dtau = DBL_MAX;
  for (int64_t f = 0; f < NF; ++f) {
    int32_t o = m->face_owner[f], q = m->face_neigh[f];
    if (q < 0) continue;
    double r[3] = {xc[q] - xc[o], xc[N + q] - xc[N + o], xc[2 * N + q] - xc[2 * N + o]};
    double d = sqrt(v_dot(r, r));
    if (d < dtau) dtau = d;
  }
  for (int k = 0; k < 2; ++k)
    for (int d = 0; d < 3; ++d)
      for (int64_t P = 0; P < N; ++P) cur[(k * 3 + d) * N + P] = grad[d * N + P];
  int it = 0;
  while (it < max_iter) {
    memcpy(nxt, cur, sizeof(double) * 6 * (size_t)N);
    double change = 0.0;
    for (int64_t P = 0; P < N; ++P) {
      if (mark[P] < 0) continue;
      int liquid = alpha[P] >= 0.5;
      double s = liquid ? 1.0 : -1.0;
      double c[3] = {s * nrm[P], s * nrm[N + P], s * nrm[2 * N + P]};
      int fld = liquid ? 1 : 0; /* advanced field: G_v in liquid, G_l in vapour */
      double w = 0.0, acc[3] = {0, 0, 0};
      for (int64_t i = m->cell_face_off[P]; i < m->cell_face_off[P + 1]; ++i) {
        int32_t f = m->cell_face[i];
        int32_t Q = (m->face_owner[f] == P) ? m->face_neigh[f] : m->face_owner[f];
        if (Q < 0 || mark[Q] < 0) continue;
        double sg = (m->face_owner[f] == P) ? 1.0 : -1.0;
        double S[3] = {sg * Sf[f], sg * Sf[NF + f], sg * Sf[2 * NF + f]};
        double cs = v_dot(c, S);
        if (!(cs < 0.0)) continue;
        double wf = -cs;
        w += wf;
        for (int d = 0; d < 3; ++d) acc[d] += wf * cur[(fld * 3 + d) * N + Q];
      }
      if (!(w > 0.0)) continue;
      double theta = dtau * w / V[P];
      if (theta > 1.0) theta = 1.0;
      for (int d = 0; d < 3; ++d) {
        double old = cur[(fld * 3 + d) * N + P];
        double val = old + theta * (acc[d] / w - old);
        nxt[(fld * 3 + d) * N + P] = val;
        double ch = fabs(val - old);
        if (ch > change) change = ch;
      }
    }
    double *t = cur; cur = nxt; nxt = t;
    ++it;
    if (change < tol) break;
  }
  for (int d = 0; d < 3; ++d)
    for (int64_t P = 0; P < N; ++P) {
      gl[d * N + P] = cur[d * N + P];
      gv[d * N + P] = cur[(3 + d) * N + P];
    }
  if (iters) *iters = it;
  if (domain)
    for (int64_t P = 0; P < N; ++P) domain[P] = mark[P] >= 0 ? 1 : 0;
  free(mark); free(next); free(nrm); free(cur); free(nxt);
  return 0;
}

/* ------------------------------------------ interface heat transfer (Robin) */
/* Coefficients of the implicit interface coupling of the energy equation
 * (Eq. interface_htc, Sec. 2.4.4 "Heat source/sink"): every interior face
 * whose cells lie on opposite sides of alpha = 1/2 is detached, and each of
 * its two cells C gets a_f,C = k_C A_int,f / d_f,C, where
 *   k_C      = k_l when alpha_C >= 1/2, else k_v (the cell's own phase);
 *   x_f      = the crossing point of the gradient stencil,
 *              x_P + t (x_Q - x_P), t = (a_P - 1/2)/(a_P - a_Q);
 *   d_f,C    = |nf . (x_f - x_C)|, nf = S_f/|S_f| (normal distance);
 *   A_int,f  = |nf . (A_P n_P + A_Q n_Q)|, the face-normal projection of the
 *              interface area vectors of the two cells (0 for a cell without
 *              an interface).
 * A side whose distance is not positive gets a = 0.
 * Outputs (any may be NULL): a_cell [N] = sum of a_f,C over the cell's
 * detached faces; a_face, d_face [2][NF] (owner side, neighbour side),
 * area_face [NF], crossing [NF] (1 on detached faces); the face outputs are 0
 * on faces that are not detached. */
int orc_robin(const orc_mesh *m, const double *xc, const double *Sf, const double *alpha, const double *n,
              const double *A, double k_l, double k_v, double *a_cell, double *a_face, double *d_face,
              double *area_face, int8_t *crossing) {
  int64_t N = m->n_cells, NF = m->n_faces;
  if (a_cell)
    for (int64_t P = 0; P < N; ++P) a_cell[P] = 0.0;
  for (int64_t f = 0; f < NF; ++f) {
    int32_t P = m->face_owner[f], Q = m->face_neigh[f];
    int cross = Q >= 0 && (alpha[P] - 0.5) * (alpha[Q] - 0.5) < 0.0;
    double aP = 0.0, aQ = 0.0, dP = 0.0, dQ = 0.0, area = 0.0;
    if (cross) {
      double S[3] = {Sf[f], Sf[NF + f], Sf[2 * NF + f]};
      double mag = sqrt(v_dot(S, S));
      double nf[3] = {S[0] / mag, S[1] / mag, S[2] / mag};
      double xP[3] = {xc[P], xc[N + P], xc[2 * N + P]};
      double xQ[3] = {xc[Q], xc[N + Q], xc[2 * N + Q]};
      double t = (alpha[P] - 0.5) / (alpha[P] - alpha[Q]);
      double xf[3], r[3];
      for (int d = 0; d < 3; ++d) xf[d] = xP[d] + t * (xQ[d] - xP[d]);
      v_sub(xf, xP, r);
      dP = fabs(v_dot(nf, r));
      v_sub(xf, xQ, r);
      dQ = fabs(v_dot(nf, r));
      double sint[3];
      for (int d = 0; d < 3; ++d) sint[d] = A[P] * n[d * N + P] + A[Q] * n[d * N + Q];
      area = fabs(v_dot(nf, sint));
      double kP = alpha[P] >= 0.5 ? k_l : k_v;
      double kQ = alpha[Q] >= 0.5 ? k_l : k_v;
      if (dP > 0.0) aP = kP * area / dP;
      if (dQ > 0.0) aQ = kQ * area / dQ;
      if (a_cell) {
        a_cell[P] += aP;
        a_cell[Q] += aQ;
      }
    }
    if (a_face) { a_face[f] = aP; a_face[NF + f] = aQ; }
    if (d_face) { d_face[f] = dP; d_face[NF + f] = dQ; }
    if (area_face) area_face[f] = area;
    if (crossing) crossing[f] = (int8_t)cross;
  }
  return 0;
}

/* ------------------------------------------------- CSF curvature chain */
/* Surface-tension curvature of the continuum-surface-force model (Sec. 2.4,
 * momentum terms, surface tension), in the order the method states it:
 *   smoothing  alpha_hat_P = sum_f alpha_hat_f A_f / sum_f A_f over all faces,
 *              alpha_hat_f = alpha_P + w_f (alpha_Q - alpha_P) (the printed
 *              (1 - w_f) alpha_P + w_f alpha_Q, written so that equal values
 *              stay exact), w_f the geometric weight of Q: the fraction of the
 *              centre connection P->Q at which it meets the face plane,
 *              w_f = nf.(x_f - x_P) / nf.(x_Q - x_P); boundary faces take
 *              alpha_hat_P; Jacobi sweeps, n_smooth of them;
 *   normal     n_P = grad(alpha_hat)/(|grad(alpha_hat)| + 1e-15), the plain
 *              least-squares gradient over interior face neighbours (App. B);
 *   raw        kappa~_P = -div n = -(1/V_P) sum_f n_f . S_f (Gauss, S_f
 *              outward), n_f = n_P + w_f (n_Q - n_P), n_P on boundary faces;
 *   step 1     kappa*_P = (kappa~_P w_P + sum_Q kappa~_Q w_Q) /
 *              (w_P + sum_Q w_Q + 1e-15), w_i = (1 - 2|1/2 - alpha_hat_i|)^8,
 *              Q over the face neighbours;
 *   step 2     kappa_P = (kappa*_P w_P + sum_Q kappa*_Q w_Q wn_Q) /
 *              (w_P + sum_Q w_Q wn_Q + 1e-15), wn_Q = |n_P . s_Q|^8, s_Q the
 *              unit centre connection (the 1e-15 of step 1 is added here too:
 *              without it pure cells divide 0 by 0);
 *   force      F_P = sigma kappa_P grad(alpha)_P, the plain least-squares
 *              gradient of the sharp alpha over interior face neighbours.
 * Each stage is its own function so that it can be checked alone.  Arrays are
 * SoA, vectors [3][N]. */
static double face_weight(const orc_mesh *m, const double *xc, const double *Sf, const double *xf, int32_t f,
                          int64_t P, int64_t Q) {
  int64_t N = m->n_cells, NF = m->n_faces;
  double S[3] = {Sf[f], Sf[NF + f], Sf[2 * NF + f]};
  double a = 0.0, b = 0.0;
  for (int d = 0; d < 3; ++d) {
    a += S[d] * (xf[d * NF + f] - xc[d * N + P]);
    b += S[d] * (xc[d * N + Q] - xc[d * N + P]);
  }
  return a / b;
}

int orc_csf_smooth(const orc_mesh *m, const double *xc, const double *Sf, const double *xf, const double *alpha,
                   int n_smooth, double *alpha_hat) {
  int64_t N = m->n_cells, NF = m->n_faces;
  double *cur = (double *)malloc(sizeof(double) * (size_t)N);
  if (!cur) return 1;
  memcpy(alpha_hat, alpha, sizeof(double) * (size_t)N);
  for (int it = 0; it < n_smooth; ++it) {
    memcpy(cur, alpha_hat, sizeof(double) * (size_t)N);
    for (int64_t P = 0; P < N; ++P) {
      double num = 0.0, den = 0.0;
      for (int64_t i = m->cell_face_off[P]; i < m->cell_face_off[P + 1]; ++i) {
        int32_t f = m->cell_face[i];
        int32_t Q = (m->face_owner[f] == P) ? m->face_neigh[f] : m->face_owner[f];
        double A = sqrt(Sf[f] * Sf[f] + Sf[NF + f] * Sf[NF + f] + Sf[2 * NF + f] * Sf[2 * NF + f]);
        double af = cur[P];
        if (Q >= 0) af = cur[P] + face_weight(m, xc, Sf, xf, f, P, Q) * (cur[Q] - cur[P]);
        num += af * A;
        den += A;
      }
      alpha_hat[P] = num / den;
    }
  }
  free(cur);
  return 0;
}

/* plain least-squares gradient over interior face neighbours (App. B) */
int orc_lsq_interior(const orc_mesh *m, const double *xc, const double *val, double *grad) {
  int64_t N = m->n_cells;
  for (int64_t P = 0; P < N; ++P) {
    double g[3];
    lsq_interior(m, xc, val, P, g);
    for (int d = 0; d < 3; ++d) grad[d * N + P] = g[d];
  }
  return 0;
}

int orc_csf_normal(const orc_mesh *m, const double *xc, const double *alpha_hat, double *n) {
  int64_t N = m->n_cells;
  orc_lsq_interior(m, xc, alpha_hat, n);
  for (int64_t P = 0; P < N; ++P) {
    double g[3] = {n[P], n[N + P], n[2 * N + P]};
    double den = sqrt(v_dot(g, g)) + 1e-15;
    for (int d = 0; d < 3; ++d) n[d * N + P] = g[d] / den;
  }
  return 0;
}

int orc_csf_raw_curvature(const orc_mesh *m, const double *V, const double *xc, const double *Sf, const double *xf,
                          const double *n, double *kraw) {
  int64_t N = m->n_cells, NF = m->n_faces;
  for (int64_t P = 0; P < N; ++P) {
    double div = 0.0;
    for (int64_t i = m->cell_face_off[P]; i < m->cell_face_off[P + 1]; ++i) {
      int32_t f = m->cell_face[i];
      int32_t Q = (m->face_owner[f] == P) ? m->face_neigh[f] : m->face_owner[f];
      double sg = (m->face_owner[f] == P) ? 1.0 : -1.0;
      double nf[3];
      for (int d = 0; d < 3; ++d) nf[d] = n[d * N + P];
      if (Q >= 0) {
        double w = face_weight(m, xc, Sf, xf, f, P, Q);
        for (int d = 0; d < 3; ++d) nf[d] = n[d * N + P] + w * (n[d * N + Q] - n[d * N + P]);
      }
      div += sg * (nf[0] * Sf[f] + nf[1] * Sf[NF + f] + nf[2] * Sf[2 * NF + f]);
    }
    kraw[P] = -div / V[P];
  }
  return 0;
}

static double colour_weight(double a) {
  double w = 1.0 - 2.0 * fabs(0.5 - a);
  double w2 = w * w, w4 = w2 * w2;
  return w4 * w4;
}

int orc_csf_smooth_curvature(const orc_mesh *m, const double *xc, const double *alpha_hat, const double *n,
                             const double *kraw, double *kstar, double *kappa) {
  int64_t N = m->n_cells;
  for (int64_t P = 0; P < N; ++P) {
    double wP = colour_weight(alpha_hat[P]);
    double num = kraw[P] * wP, den = wP;
    for (int64_t i = m->cell_face_off[P]; i < m->cell_face_off[P + 1]; ++i) {
      int32_t f = m->cell_face[i];
      int32_t Q = (m->face_owner[f] == P) ? m->face_neigh[f] : m->face_owner[f];
      if (Q < 0) continue;
      double wQ = colour_weight(alpha_hat[Q]);
      num += kraw[Q] * wQ;
      den += wQ;
    }
    kstar[P] = num / (den + 1e-15);
  }
  for (int64_t P = 0; P < N; ++P) {
    double wP = colour_weight(alpha_hat[P]);
    double num = kstar[P] * wP, den = wP;
    double nP[3] = {n[P], n[N + P], n[2 * N + P]};
    for (int64_t i = m->cell_face_off[P]; i < m->cell_face_off[P + 1]; ++i) {
      int32_t f = m->cell_face[i];
      int32_t Q = (m->face_owner[f] == P) ? m->face_neigh[f] : m->face_owner[f];
      if (Q < 0) continue;
      double s[3] = {xc[Q] - xc[P], xc[N + Q] - xc[N + P], xc[2 * N + Q] - xc[2 * N + P]};
      double len = sqrt(v_dot(s, s));
      double c = fabs(v_dot(nP, s) / len);
      double c2 = c * c, c4 = c2 * c2;
      double wn = c4 * c4;
      double wQ = colour_weight(alpha_hat[Q]);
      num += kstar[Q] * wQ * wn;
      den += wQ * wn;
    }
    kappa[P] = num / (den + 1e-15);
  }
  return 0;
}

/* the whole chain; F (optional) = sigma kappa grad(alpha) */
int orc_csf(const orc_mesh *m, const double *V, const double *xc, const double *Sf, const double *xf,
            const double *alpha, int n_smooth, double sigma, double *alpha_hat, double *n, double *kraw,
            double *kstar, double *kappa, double *F) {
  int64_t N = m->n_cells;
  if (orc_csf_smooth(m, xc, Sf, xf, alpha, n_smooth, alpha_hat)) return 1;
  orc_csf_normal(m, xc, alpha_hat, n);
  orc_csf_raw_curvature(m, V, xc, Sf, xf, n, kraw);
  orc_csf_smooth_curvature(m, xc, alpha_hat, n, kraw, kstar, kappa);
  if (F) {
    orc_lsq_interior(m, xc, alpha, F);
    for (int64_t P = 0; P < N; ++P)
      for (int d = 0; d < 3; ++d) F[d * N + P] = sigma * kappa[P] * F[d * N + P];
  }
  return 0;
}
