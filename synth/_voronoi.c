/* Box-clipped Voronoi cells of a seed set (input-generation helper).
 *
 * Cell i is the box [lo, hi] clipped by the bisector half-spaces of the
 * seeds nearest to seed i, in order of distance, until no further seed can
 * cut it (the next seed is farther than twice the cell's largest vertex
 * distance).  Only the cells of seeds marked `keep` are built; every seed
 * still clips its neighbours, so a face between a kept and a dropped cell
 * becomes a boundary face of the kept one (a staircase wall).
 *
 * Every vertex is named by its four generators (seeds and box walls, walls
 * as -1..-6), sorted.  Its position is computed from that name alone (the
 * bisectors of its smallest seed with the others and its walls, solved by
 * Cramer's rule), and a seed m cuts it when m is strictly nearer to it than
 * its smallest seed: both decisions are functions of the name, so the cells
 * sharing a vertex agree on it bit for bit and the cells fit together.  The
 * assembled mesh is checked (every interior face seen from both cells with
 * the same vertices in reverse order) and an inconsistency is reported as an
 * error.
 *
 * Output: the CSR mesh the library and the oracle take (faces ordered by
 * owner, interior faces by neighbour, then boundary faces; loops
 * counter-clockwise seen from outside the owner), vertex coordinates and the
 * half-space n.x <= c of every face on its owner's side.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define VG_MAXV 160   /* vertices of a cell while it is clipped */
#define VG_MAXF 64    /* faces of a cell */
#define VG_MAXFV 40   /* vertices of a face */
#define VG_MAXC 1024  /* candidate seeds of a cell */

typedef struct {
  double x[3];
  int32_t key[4];
  int alive;
} vg_vtx;

typedef struct {
  int32_t gen;   /* the other generator: a seed id or a wall -1..-6 */
  int n;
  int v[VG_MAXFV];
} vg_face;

typedef struct {
  int nv, nf;
  vg_vtx V[VG_MAXV];
  vg_face F[VG_MAXF];
} vg_poly;

/* a finished cell: compact vertices (name, position) and face loops */
typedef struct {
  int nv, nf;
  int32_t *key;    /* [nv][4] */
  double *x;       /* [nv][3] */
  int32_t *gid;    /* [nv] global vertex ids */
  int32_t *fgen;   /* [nf] */
  int32_t *foff;   /* [nf+1] into floop */
  uint8_t *floop;  /* local vertex ids */
  int64_t *fid;    /* [nf] global face ids */
} vg_cell;

typedef struct {
  int64_t N;
  const double *P;   /* [N][3] */
  double lo[3], hi[3];
  const uint8_t *keep;
  /* bucket grid */
  int g[3];
  double bsz[3];
  int64_t *boff;
  int64_t *bseed;
} vg_ctx;

static void wall_plane(const vg_ctx *c, int w, double n[3], double *rhs) {
  /* wall -1: x >= lo_x, -2: x <= hi_x, -3/-4: y, -5/-6: z; as n.x <= rhs */
  int k = (-w - 1) / 2, hi = (-w - 1) % 2;
  n[0] = n[1] = n[2] = 0.0;
  if (hi) { n[k] = 1.0; *rhs = c->hi[k]; }
  else { n[k] = -1.0; *rhs = -c->lo[k]; }
}

static void sort4(int32_t *k) {
  for (int i = 1; i < 4; ++i) {
    int32_t t = k[i];
    int j = i - 1;
    while (j >= 0 && k[j] > t) { k[j + 1] = k[j]; --j; }
    k[j + 1] = t;
  }
}

/* smallest seed of a name (names always hold at least one seed) */
static int32_t first_seed(const int32_t *k) {
  for (int i = 0; i < 4; ++i)
    if (k[i] >= 0) return k[i];
  return -1;
}

/* position of the vertex named k (sorted) */
static int vertex_pos(const vg_ctx *c, const int32_t *k, double x[3]) {
  double A[3][3], b[3];
  int r = 0;
  int32_t s0 = first_seed(k);
  const double *p0 = c->P + 3 * s0;
  for (int i = 0; i < 4; ++i) {
    if (k[i] == s0) continue;
    if (k[i] >= 0) {
      const double *p = c->P + 3 * k[i];
      for (int d = 0; d < 3; ++d) A[r][d] = p[d] - p0[d];
      b[r] = 0.5 * ((p[0] - p0[0]) * (p[0] + p0[0]) + (p[1] - p0[1]) * (p[1] + p0[1]) +
                    (p[2] - p0[2]) * (p[2] + p0[2]));
    } else {
      wall_plane(c, k[i], A[r], &b[r]);
    }
    ++r;
  }
  if (r != 3) return -1;
  double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
               A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
  if (!(fabs(det) > 0)) return -1;
  for (int col = 0; col < 3; ++col) {
    double M[3][3];
    memcpy(M, A, sizeof M);
    for (int row = 0; row < 3; ++row) M[row][col] = b[row];
    double dc = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
    x[col] = dc / det;
  }
  return 0;
}

static double d2(const double *a, const double *b) {
  double u = a[0] - b[0], v = a[1] - b[1], w = a[2] - b[2];
  return u * u + v * v + w * w;
}

/* does seed m cut the vertex (strictly nearer to it than its smallest seed)? */
static int cuts(const vg_ctx *c, const vg_vtx *v, int32_t m) {
  return d2(v->x, c->P + 3 * m) < d2(v->x, c->P + 3 * first_seed(v->key));
}

/* drop dead vertices and renumber the loops (between clips only) */
static void compact(vg_poly *py) {
  int map[VG_MAXV], n = 0;
  for (int i = 0; i < py->nv; ++i) {
    map[i] = py->V[i].alive ? n : -1;
    if (py->V[i].alive) py->V[n++] = py->V[i];
  }
  for (int f = 0; f < py->nf; ++f)
    for (int j = 0; j < py->F[f].n; ++j) py->F[f].v[j] = map[py->F[f].v[j]];
  py->nv = n;
}

static int add_vertex(const vg_ctx *c, vg_poly *py, const int32_t *key) {
  if (py->nv >= VG_MAXV) return -1;
  vg_vtx *v = &py->V[py->nv];
  memcpy(v->key, key, sizeof v->key);
  sort4(v->key);
  if (vertex_pos(c, v->key, v->x)) return -1;
  v->alive = 1;
  return py->nv++;
}

static void init_box(const vg_ctx *c, int32_t i, vg_poly *py) {
  /* vertex (a, b, d) of the box: x from wall -1 - a (lo) or -2 (hi), ... */
  py->nv = 0;
  py->nf = 0;
  for (int z = 0; z < 2; ++z)
    for (int y = 0; y < 2; ++y)
      for (int x = 0; x < 2; ++x) {
        int32_t key[4] = {i, -1 - x, -3 - y, -5 - z};
        add_vertex(c, py, key);
      }
#define VID(x, y, z) ((x) + 2 * (y) + 4 * (z))
  /* faces counter-clockwise seen from outside */
  const int quads[6][4] = {
      {VID(0, 0, 0), VID(0, 0, 1), VID(0, 1, 1), VID(0, 1, 0)},   /* x = lo, gen -1 */
      {VID(1, 0, 0), VID(1, 1, 0), VID(1, 1, 1), VID(1, 0, 1)},   /* x = hi, gen -2 */
      {VID(0, 0, 0), VID(1, 0, 0), VID(1, 0, 1), VID(0, 0, 1)},   /* y = lo, gen -3 */
      {VID(0, 1, 0), VID(0, 1, 1), VID(1, 1, 1), VID(1, 1, 0)},   /* y = hi, gen -4 */
      {VID(0, 0, 0), VID(0, 1, 0), VID(1, 1, 0), VID(1, 0, 0)},   /* z = lo, gen -5 */
      {VID(0, 0, 1), VID(1, 0, 1), VID(1, 1, 1), VID(0, 1, 1)},   /* z = hi, gen -6 */
  };
#undef VID
  for (int f = 0; f < 6; ++f) {
    py->F[f].gen = -1 - f;
    py->F[f].n = 4;
    for (int j = 0; j < 4; ++j) py->F[f].v[j] = quads[f][j];
  }
  py->nf = 6;
}

/* common generators of two vertex names other than `own`: exactly two for
 * the ends of an edge */
static int common2(const int32_t *a, const int32_t *b, int32_t own, int32_t out[2]) {
  int n = 0;
  for (int i = 0; i < 4; ++i) {
    if (a[i] == own) continue;
    for (int j = 0; j < 4; ++j)
      if (a[i] == b[j]) {
        if (n < 2) out[n] = a[i];
        ++n;
        break;
      }
  }
  return n == 2 ? 0 : -1;
}

/* clip cell `own` by the bisector of seed m; returns 0, or -1 on a
 * topology failure */
static int clip(const vg_ctx *c, vg_poly *py, int32_t own, int32_t m) {
  if (py->nv > VG_MAXV / 2) compact(py);
  int out[VG_MAXV], any = 0;
  for (int i = 0; i < py->nv; ++i) {
    out[i] = py->V[i].alive && cuts(c, &py->V[i], m);
    any |= out[i];
  }
  if (!any) return 0;
  /* new vertices by cut edge, and the cap's next pointers */
  int ea[64], eb[64], ev[64], ne = 0;
  int capnext_from[64], capnext_to[64], ncap = 0;
  int nf = 0;
  vg_face nfcs[VG_MAXF];
  for (int f = 0; f < py->nf; ++f) {
    const vg_face *F = &py->F[f];
    vg_face G;
    G.gen = F->gen;
    G.n = 0;
    int A = -1, B = -1;
    for (int j = 0; j < F->n; ++j) {
      int a = F->v[j], b = F->v[(j + 1) % F->n];
      if (!out[a]) {
        if (G.n >= VG_MAXFV) return -1;
        G.v[G.n++] = a;
      }
      if (out[a] != out[b]) {
        int lo = a < b ? a : b, hi = a < b ? b : a, id = -1;
        for (int t = 0; t < ne; ++t)
          if (ea[t] == lo && eb[t] == hi) { id = ev[t]; break; }
        if (id < 0) {
          int32_t cm[2];
          if (common2(py->V[a].key, py->V[b].key, own, cm)) return -1;
          int32_t key[4] = {own, cm[0], cm[1], m};
          id = add_vertex(c, py, key);
          if (id < 0 || ne >= 64) return -1;
          out[id] = 0;
          ea[ne] = lo; eb[ne] = hi; ev[ne] = id; ++ne;
        }
        if (G.n >= VG_MAXFV) return -1;
        G.v[G.n++] = id;
        if (!out[a]) A = id; else B = id;
      }
    }
    if (G.n == 0) continue;            /* the face lies beyond the plane */
    if (A >= 0 || B >= 0) {
      if (A < 0 || B < 0 || ncap >= 64) return -1;
      /* the face runs A -> B along the plane; the cap runs B -> A */
      capnext_from[ncap] = B;
      capnext_to[ncap] = A;
      ++ncap;
    }
    if (nf >= VG_MAXF) return -1;
    nfcs[nf++] = G;
  }
  /* the cap face */
  if (ncap < 3 || nf >= VG_MAXF) return -1;
  vg_face cap;
  cap.gen = m;
  cap.n = 0;
  int start = capnext_from[0], v = start;
  do {
    if (cap.n >= VG_MAXFV) return -1;
    cap.v[cap.n++] = v;
    int nx = -1;
    for (int t = 0; t < ncap; ++t)
      if (capnext_from[t] == v) { nx = capnext_to[t]; break; }
    if (nx < 0) return -1;
    v = nx;
  } while (v != start && cap.n <= ncap);
  if (v != start || cap.n != ncap) return -1;
  nfcs[nf++] = cap;
  for (int i = 0; i < py->nv; ++i)
    if (out[i]) py->V[i].alive = 0;
  memcpy(py->F, nfcs, sizeof(vg_face) * nf);
  py->nf = nf;
  return 0;
}

typedef struct {
  double d;
  int32_t s;
} vg_cand;

static int cand_cmp(const void *a, const void *b) {
  const vg_cand *x = a, *y = b;
  if (x->d < y->d) return -1;
  if (x->d > y->d) return 1;
  return (x->s > y->s) - (x->s < y->s);
}

static int gather(const vg_ctx *c, int32_t i, int R, vg_cand *cd, int *nc, double *cover) {
  const double *p = c->P + 3 * i;
  int b[3];
  *cover = INFINITY;
  for (int d = 0; d < 3; ++d) {
    b[d] = (int)floor((p[d] - c->lo[d]) / c->bsz[d]);
    if (b[d] < 0) b[d] = 0;
    if (b[d] >= c->g[d]) b[d] = c->g[d] - 1;
    /* distance from the seed to the nearest bucket outside the block (the
     * box walls bound the cell where the block reaches them) */
    double left = (b[d] - R > 0) ? p[d] - (c->lo[d] + (b[d] - R) * c->bsz[d]) : INFINITY;
    double right = (b[d] + R + 1 < c->g[d]) ? (c->lo[d] + (b[d] + R + 1) * c->bsz[d]) - p[d] : INFINITY;
    if (left < *cover) *cover = left;
    if (right < *cover) *cover = right;
  }
  int n = 0;
  for (int z = b[2] - R; z <= b[2] + R; ++z) {
    if (z < 0 || z >= c->g[2]) continue;
    for (int y = b[1] - R; y <= b[1] + R; ++y) {
      if (y < 0 || y >= c->g[1]) continue;
      for (int x = b[0] - R; x <= b[0] + R; ++x) {
        if (x < 0 || x >= c->g[0]) continue;
        int64_t bk = x + (int64_t)c->g[0] * (y + (int64_t)c->g[1] * z);
        for (int64_t t = c->boff[bk]; t < c->boff[bk + 1]; ++t) {
          int32_t s = (int32_t)c->bseed[t];
          if (s == i) continue;
          if (n >= VG_MAXC) return -1;
          cd[n].d = d2(p, c->P + 3 * s);
          cd[n].s = s;
          ++n;
        }
      }
    }
  }
  qsort(cd, (size_t)n, sizeof *cd, cand_cmp);
  *nc = n;
  return 0;
}

/* build the cell of seed i */
static int build_cell(const vg_ctx *c, int32_t i, vg_poly *py, vg_cand *cd) {
  init_box(c, i, py);
  const double *p = c->P + 3 * i;
  int32_t done[VG_MAXC];   /* seeds already clipped by (a wider round re-gathers them) */
  int ndone = 0;
  for (int R = 2; R <= 6; ++R) {
    int nc = 0;
    double cover;
    if (gather(c, i, R, cd, &nc, &cover)) return -1;
    double rmax2 = 0;
    for (int v = 0; v < py->nv; ++v)
      if (py->V[v].alive) { double q = d2(py->V[v].x, p); if (q > rmax2) rmax2 = q; }
    for (int t = 0; t < nc; ++t) {
      if (cd[t].d > 4.0 * rmax2) break;   /* no farther seed can cut the cell */
      int seen = 0;
      for (int u = 0; u < ndone && !seen; ++u) seen = done[u] == cd[t].s;
      if (seen) continue;
      if (ndone >= VG_MAXC) return -1;
      done[ndone++] = cd[t].s;
      if (clip(c, py, i, cd[t].s)) return -2;
      rmax2 = 0;
      for (int v = 0; v < py->nv; ++v)
        if (py->V[v].alive) { double q = d2(py->V[v].x, p); if (q > rmax2) rmax2 = q; }
    }
    /* every seed that could still cut lies within 2 sqrt(rmax2) of p */
    if (4.0 * rmax2 < cover * cover) return 0;
  }
  return -3;
}

static int finish_cell(const vg_poly *py, vg_cell *out) {
  int map[VG_MAXV], n = 0, tot = 0;
  for (int v = 0; v < py->nv; ++v) map[v] = py->V[v].alive ? n++ : -1;
  for (int f = 0; f < py->nf; ++f) tot += py->F[f].n;
  if (n > 255) return -1;
  out->nv = n;
  out->nf = py->nf;
  out->key = malloc(sizeof(int32_t) * 4 * n);
  out->x = malloc(sizeof(double) * 3 * n);
  out->gid = malloc(sizeof(int32_t) * n);
  out->fgen = malloc(sizeof(int32_t) * py->nf);
  out->foff = malloc(sizeof(int32_t) * (py->nf + 1));
  out->floop = malloc((size_t)tot);
  out->fid = malloc(sizeof(int64_t) * py->nf);
  if (!out->key || !out->x || !out->gid || !out->fgen || !out->foff || !out->floop || !out->fid) return -1;
  for (int v = 0; v < py->nv; ++v) {
    if (map[v] < 0) continue;
    memcpy(out->key + 4 * map[v], py->V[v].key, sizeof(int32_t) * 4);
    memcpy(out->x + 3 * map[v], py->V[v].x, sizeof(double) * 3);
  }
  int o = 0;
  for (int f = 0; f < py->nf; ++f) {
    out->fgen[f] = py->F[f].gen;
    out->foff[f] = o;
    for (int j = 0; j < py->F[f].n; ++j) {
      int m = map[py->F[f].v[j]];
      if (m < 0) return -1;
      out->floop[o++] = (uint8_t)m;
    }
  }
  out->foff[py->nf] = o;
  return 0;
}

static int key_eq(const int32_t *a, const int32_t *b) {
  return a[0] == b[0] && a[1] == b[1] && a[2] == b[2] && a[3] == b[3];
}

typedef struct {
  int64_t n_cells, n_faces, n_verts, n_fv;
  int64_t *cell_face_off;
  int32_t *cell_face;
  int64_t *face_vert_off;
  int32_t *face_vert;
  int32_t *face_owner, *face_neigh;
  double *vert_xyz;     /* [3][NV] */
  double *face_plane;   /* [NF][4] */
  int32_t *cell_seed;   /* [N] seed of each kept cell */
} vg_result;

void vg_free(vg_result *r) {
  free(r->cell_face_off); free(r->cell_face); free(r->face_vert_off); free(r->face_vert);
  free(r->face_owner); free(r->face_neigh); free(r->vert_xyz); free(r->face_plane); free(r->cell_seed);
  memset(r, 0, sizeof *r);
}

/* face of cell `cl` whose other generator is g, or -1 */
static int face_to(const vg_cell *cl, int32_t g) {
  for (int f = 0; f < cl->nf; ++f)
    if (cl->fgen[f] == g) return f;
  return -1;
}

/* Build the mesh.  Returns 0, or a negative code: -1 memory, -2 a cell
 * failed to build (err_seed receives its seed), -3 the cells do not fit
 * together (err_seed receives a seed of the failing face). */
int vg_build(int64_t N, const double *P, const double *lo, const double *hi, const uint8_t *keep, int nthreads,
             vg_result *res, int64_t *err_seed) {
  memset(res, 0, sizeof *res);
  *err_seed = -1;
  vg_ctx c;
  c.N = N;
  c.P = P;
  c.keep = keep;
  double vol = 1.0;
  for (int d = 0; d < 3; ++d) {
    c.lo[d] = lo[d];
    c.hi[d] = hi[d];
    vol *= hi[d] - lo[d];
  }
  double h = cbrt(vol / (double)N);
  for (int d = 0; d < 3; ++d) {
    c.g[d] = (int)((hi[d] - lo[d]) / h);
    if (c.g[d] < 1) c.g[d] = 1;
    c.bsz[d] = (hi[d] - lo[d]) / c.g[d];
  }
  int64_t nb = (int64_t)c.g[0] * c.g[1] * c.g[2];
  c.boff = calloc((size_t)nb + 1, sizeof(int64_t));
  c.bseed = malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
  int64_t *bk = malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
  if (!c.boff || !c.bseed || !bk) { free(c.boff); free(c.bseed); free(bk); return -1; }
  for (int64_t s = 0; s < N; ++s) {
    int b[3];
    for (int d = 0; d < 3; ++d) {
      b[d] = (int)floor((P[3 * s + d] - lo[d]) / c.bsz[d]);
      if (b[d] < 0) b[d] = 0;
      if (b[d] >= c.g[d]) b[d] = c.g[d] - 1;
    }
    bk[s] = b[0] + (int64_t)c.g[0] * (b[1] + (int64_t)c.g[1] * b[2]);
    c.boff[bk[s] + 1]++;
  }
  for (int64_t t = 0; t < nb; ++t) c.boff[t + 1] += c.boff[t];
  {
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)nb);
    if (!fill) { free(c.boff); free(c.bseed); free(bk); return -1; }
    memcpy(fill, c.boff, sizeof(int64_t) * (size_t)nb);
    for (int64_t s = 0; s < N; ++s) c.bseed[fill[bk[s]]++] = s;
    free(fill);
  }
  free(bk);
  /* kept cells in seed order */
  int64_t *cell_of = malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
  int64_t NC = 0;
  for (int64_t s = 0; s < N; ++s) cell_of[s] = keep[s] ? NC++ : -1;
  vg_cell *cells = calloc((size_t)(NC > 0 ? NC : 1), sizeof(vg_cell));
  int32_t *seed_of = malloc(sizeof(int32_t) * (size_t)(NC > 0 ? NC : 1));
  if (!cell_of || !cells || !seed_of) return -1;
  for (int64_t s = 0; s < N; ++s)
    if (cell_of[s] >= 0) seed_of[cell_of[s]] = (int32_t)s;
  int fail = 0;
  int64_t fail_seed = -1;
#pragma omp parallel num_threads(nthreads)
  {
    vg_poly *py = malloc(sizeof(vg_poly));
    vg_cand *cd = malloc(sizeof(vg_cand) * VG_MAXC);
#pragma omp for schedule(dynamic, 256)
    for (int64_t ci = 0; ci < NC; ++ci) {
      if (fail) continue;
      int32_t s = seed_of[ci];
      if (!py || !cd || build_cell(&c, s, py, cd) || finish_cell(py, &cells[ci])) {
#pragma omp critical
        { fail = 1; fail_seed = s; }
      }
    }
    free(py);
    free(cd);
  }
  int rc = 0;
  if (fail) { rc = -2; *err_seed = fail_seed; goto done; }
  /* global vertex ids: a vertex belongs to the smallest kept seed of its name */
  {
    int64_t *vbase = malloc(sizeof(int64_t) * (size_t)(NC + 1));
    if (!vbase) { rc = -1; goto done; }
    vbase[0] = 0;
    for (int64_t ci = 0; ci < NC; ++ci) {
      int32_t s = seed_of[ci], own = 0;
      const vg_cell *cl = &cells[ci];
      for (int v = 0; v < cl->nv; ++v) {
        const int32_t *k = cl->key + 4 * v;
        int32_t o = -1;
        for (int t = 0; t < 4; ++t)
          if (k[t] >= 0 && keep[k[t]]) { o = k[t]; break; }
        if (o == s) cells[ci].gid[v] = own++;
        else cells[ci].gid[v] = -1;
      }
      vbase[ci + 1] = vbase[ci] + own;
    }
    int64_t NV = vbase[NC];
    res->n_verts = NV;
    res->vert_xyz = malloc(sizeof(double) * 3 * (size_t)(NV > 0 ? NV : 1));
    if (!res->vert_xyz) { free(vbase); rc = -1; goto done; }
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t ci = 0; ci < NC; ++ci) {
      vg_cell *cl = &cells[ci];
      for (int v = 0; v < cl->nv; ++v)
        if (cl->gid[v] >= 0) {
          int64_t g = vbase[ci] + cl->gid[v];
          cl->gid[v] = (int32_t)g;
          for (int d = 0; d < 3; ++d) res->vert_xyz[d * NV + g] = cl->x[3 * v + d];
        }
    }
    /* the other vertices: their owner-local index (the owner's ids are
     * final), stored as -2 - index and resolved below */
    int bad = 0;
    int64_t bad_seed = -1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t ci = 0; ci < NC; ++ci) {
      vg_cell *cl = &cells[ci];
      for (int v = 0; v < cl->nv; ++v) {
        if (cl->gid[v] >= 0) continue;
        const int32_t *k = cl->key + 4 * v;
        int32_t o = -1;
        for (int t = 0; t < 4; ++t)
          if (k[t] >= 0 && keep[k[t]]) { o = k[t]; break; }
        const vg_cell *oc = &cells[cell_of[o]];
        int found = -1;
        for (int u = 0; u < oc->nv; ++u)
          if (key_eq(oc->key + 4 * u, k)) { found = u; break; }
        if (found < 0) {
#pragma omp critical
          { bad = 1; bad_seed = seed_of[ci]; }
          cl->gid[v] = 0;
        } else {
          cl->gid[v] = -2 - found;
        }
      }
    }
    if (bad) { free(vbase); rc = -3; *err_seed = bad_seed; goto done; }
    /* resolve owner-local indices (the owners' ids are final now) */
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t ci = 0; ci < NC; ++ci) {
      vg_cell *cl = &cells[ci];
      for (int v = 0; v < cl->nv; ++v) {
        if (cl->gid[v] > -2) continue;
        const int32_t *k = cl->key + 4 * v;
        int32_t o = -1;
        for (int t = 0; t < 4; ++t)
          if (k[t] >= 0 && keep[k[t]]) { o = k[t]; break; }
        cl->gid[v] = cells[cell_of[o]].gid[-2 - cl->gid[v]];
      }
    }
    free(vbase);
  }
  /* faces: an interior face belongs to its smaller seed's cell */
  {
    int64_t *fbase = malloc(sizeof(int64_t) * (size_t)(NC + 1));
    if (!fbase) { rc = -1; goto done; }
    fbase[0] = 0;
    int64_t fvtot = 0;
    for (int64_t ci = 0; ci < NC; ++ci) {
      const vg_cell *cl = &cells[ci];
      int32_t s = seed_of[ci];
      int own = 0;
      for (int f = 0; f < cl->nf; ++f) {
        int32_t g = cl->fgen[f];
        if (g >= 0 && keep[g] && g < s) continue;
        ++own;
        fvtot += cl->foff[f + 1] - cl->foff[f];
      }
      fbase[ci + 1] = fbase[ci] + own;
    }
    int64_t NF = fbase[NC];
    res->n_faces = NF;
    res->n_fv = fvtot;
    res->face_vert_off = malloc(sizeof(int64_t) * (size_t)(NF + 1));
    res->face_vert = malloc(sizeof(int32_t) * (size_t)(fvtot > 0 ? fvtot : 1));
    res->face_owner = malloc(sizeof(int32_t) * (size_t)(NF > 0 ? NF : 1));
    res->face_neigh = malloc(sizeof(int32_t) * (size_t)(NF > 0 ? NF : 1));
    res->face_plane = malloc(sizeof(double) * 4 * (size_t)(NF > 0 ? NF : 1));
    int64_t *fvbase = malloc(sizeof(int64_t) * (size_t)(NC + 1));
    if (!res->face_vert_off || !res->face_vert || !res->face_owner || !res->face_neigh || !res->face_plane ||
        !fvbase) {
      free(fbase); free(fvbase); rc = -1; goto done;
    }
    fvbase[0] = 0;
    for (int64_t ci = 0; ci < NC; ++ci) {
      const vg_cell *cl = &cells[ci];
      int32_t s = seed_of[ci];
      int64_t t = 0;
      for (int f = 0; f < cl->nf; ++f) {
        int32_t g = cl->fgen[f];
        if (g >= 0 && keep[g] && g < s) continue;
        t += cl->foff[f + 1] - cl->foff[f];
      }
      fvbase[ci + 1] = fvbase[ci] + t;
    }
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t ci = 0; ci < NC; ++ci) {
      vg_cell *cl = &cells[ci];
      int32_t s = seed_of[ci];
      /* owned faces: interior ones by neighbour cell, then the boundary ones */
      int order[VG_MAXF], no = 0;
      for (int pass = 0; pass < 2; ++pass)
        for (int f = 0; f < cl->nf; ++f) {
          int32_t g = cl->fgen[f];
          int interior = g >= 0 && keep[g];
          if (interior && g < s) continue;
          if (pass == 0 && interior) {
            int at = no;   /* insertion by neighbour seed */
            while (at > 0 && cl->fgen[order[at - 1]] > g) { order[at] = order[at - 1]; --at; }
            order[at] = f;
            ++no;
          } else if (pass == 1 && !interior) {
            order[no++] = f;
          }
        }
      int64_t fi = fbase[ci], fv = fvbase[ci];
      const double *p = c.P + 3 * s;
      for (int j = 0; j < no; ++j) {
        int f = order[j];
        int32_t g = cl->fgen[f];
        cl->fid[f] = fi;
        res->face_owner[fi] = (int32_t)ci;
        res->face_neigh[fi] = (g >= 0 && keep[g]) ? (int32_t)cell_of[g] : -1;
        res->face_vert_off[fi] = fv;
        for (int t = cl->foff[f]; t < cl->foff[f + 1]; ++t) res->face_vert[fv++] = cl->gid[cl->floop[t]];
        double *pl = res->face_plane + 4 * fi;
        if (g >= 0) {
          const double *q = c.P + 3 * g;
          for (int d = 0; d < 3; ++d) pl[d] = q[d] - p[d];
          pl[3] = 0.5 * ((q[0] - p[0]) * (q[0] + p[0]) + (q[1] - p[1]) * (q[1] + p[1]) + (q[2] - p[2]) * (q[2] + p[2]));
        } else {
          wall_plane(&c, g, pl, &pl[3]);
        }
        ++fi;
      }
    }
    res->face_vert_off[NF] = fvtot;
    /* faces owned by the other cell, and the check that both cells see the
     * same vertices in reverse order */
    int bad = 0;
    int64_t bad_seed = -1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t ci = 0; ci < NC; ++ci) {
      vg_cell *cl = &cells[ci];
      int32_t s = seed_of[ci];
      for (int f = 0; f < cl->nf; ++f) {
        int32_t g = cl->fgen[f];
        if (!(g >= 0 && keep[g] && g < s)) continue;
        const vg_cell *oc = &cells[cell_of[g]];
        int of = face_to(oc, s);
        int n = cl->foff[f + 1] - cl->foff[f];
        int ok = of >= 0 && (oc->foff[of + 1] - oc->foff[of]) == n;
        if (ok) {
          cl->fid[f] = oc->fid[of];
          /* reverse cyclic order: find the first vertex of mine in theirs */
          const uint8_t *mine = cl->floop + cl->foff[f], *theirs = oc->floop + oc->foff[of];
          int at = -1;
          for (int t = 0; t < n; ++t)
            if (oc->gid[theirs[t]] == cl->gid[mine[0]]) { at = t; break; }
          ok = at >= 0;
          for (int t = 0; t < n && ok; ++t)
            ok = cl->gid[mine[t]] == oc->gid[theirs[((at - t) % n + n) % n]];
        }
        if (!ok) {
#pragma omp critical
          { bad = 1; bad_seed = s; }
        }
      }
    }
    free(fbase);
    free(fvbase);
    if (bad) { rc = -3; *err_seed = bad_seed; goto done; }
  }
  /* cell -> face lists, faces ascending */
  {
    res->n_cells = NC;
    res->cell_face_off = malloc(sizeof(int64_t) * (size_t)(NC + 1));
    res->cell_seed = malloc(sizeof(int32_t) * (size_t)(NC > 0 ? NC : 1));
    if (!res->cell_face_off || !res->cell_seed) { rc = -1; goto done; }
    res->cell_face_off[0] = 0;
    for (int64_t ci = 0; ci < NC; ++ci) {
      res->cell_face_off[ci + 1] = res->cell_face_off[ci] + cells[ci].nf;
      res->cell_seed[ci] = seed_of[ci];
    }
    res->cell_face = malloc(sizeof(int32_t) * (size_t)(res->cell_face_off[NC] > 0 ? res->cell_face_off[NC] : 1));
    if (!res->cell_face) { rc = -1; goto done; }
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t ci = 0; ci < NC; ++ci) {
      const vg_cell *cl = &cells[ci];
      int32_t *dst = res->cell_face + res->cell_face_off[ci];
      for (int f = 0; f < cl->nf; ++f) {
        int64_t id = cl->fid[f];
        int at = f;
        while (at > 0 && dst[at - 1] > id) { dst[at] = dst[at - 1]; --at; }
        dst[at] = (int32_t)id;
      }
    }
  }
done:
  for (int64_t ci = 0; ci < NC; ++ci) {
    free(cells[ci].key); free(cells[ci].x); free(cells[ci].gid); free(cells[ci].fgen);
    free(cells[ci].foff); free(cells[ci].floop); free(cells[ci].fid);
  }
  free(cells);
  free(cell_of);
  free(seed_of);
  free(c.boff);
  free(c.bseed);
  if (rc) vg_free(res);
  return rc;
}
