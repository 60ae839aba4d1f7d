/* Volume fractions of synthetic input fields by sub-point counting.
 *
 * Input-generation helper only: for each requested cell, K^3 sub-points
 * (centres of a regular K^3 grid over the cell's bounding box) are kept when
 * they satisfy every half-space n.x <= c of the cell (bisector planes of a
 * Voronoi cell; none for a hexahedron, whose box is the cell), and counted as
 * liquid when the region predicate says so.  The fraction liquid/kept is the
 * cell's liquid volume fraction.
 *
 * Region kinds:
 *   0  vapour inside any of the listed spheres (x,y,z,r), liquid elsewhere;
 *   1  annular film: liquid where sqrt(x^2+z^2) > R - delta(y), with
 *      delta(y) = d0 (1 + amp sin(2 pi waves y / L)); params (R,d0,amp,waves,L);
 *   2  half-space: liquid where n.x >= c; params (nx, ny, nz, c).
 */
#include <math.h>
#include <stdint.h>

static int liquid_at(int kind, const double *x, int nsph, const double *sph,
                     const double *prm) {
  if (kind == 0) {
    for (int s = 0; s < nsph; ++s) {
      double dx = x[0] - sph[4 * s], dy = x[1] - sph[4 * s + 1], dz = x[2] - sph[4 * s + 2];
      if (dx * dx + dy * dy + dz * dz < sph[4 * s + 3] * sph[4 * s + 3]) return 0;
    }
    return 1;
  }
  if (kind == 2) return prm[0] * x[0] + prm[1] * x[1] + prm[2] * x[2] >= prm[3];
  double r = sqrt(x[0] * x[0] + x[2] * x[2]);
  double delta = prm[1] * (1.0 + prm[2] * sin(2.0 * M_PI * prm[3] * x[1] / prm[4]));
  return r > prm[0] - delta;
}

void synth_subsample(int64_t ncell, const double *bbox /* [ncell][6] */,
                     const int64_t *plane_off, const double *planes /* [.][4] n,c */,
                     const int64_t *sph_off, const double *sph /* [.][4] */,
                     int kind, const double *prm, int K, double *out) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t c = 0; c < ncell; ++c) {
    const double *b = bbox + 6 * c;
    const double *pl = planes + 4 * plane_off[c];
    int np = (int)(plane_off[c + 1] - plane_off[c]);
    const double *sp = sph + 4 * sph_off[c];
    int ns = (int)(sph_off[c + 1] - sph_off[c]);
    int64_t kept = 0, liq = 0;
    double hx = (b[3] - b[0]) / K, hy = (b[4] - b[1]) / K, hz = (b[5] - b[2]) / K;
    for (int k = 0; k < K; ++k)
      for (int j = 0; j < K; ++j)
        for (int i = 0; i < K; ++i) {
          double x[3] = {b[0] + (i + 0.5) * hx, b[1] + (j + 0.5) * hy, b[2] + (k + 0.5) * hz};
          int in = 1;
          for (int p = 0; p < np && in; ++p)
            in = pl[4 * p] * x[0] + pl[4 * p + 1] * x[1] + pl[4 * p + 2] * x[2] <= pl[4 * p + 3];
          if (!in) continue;
          ++kept;
          liq += liquid_at(kind, x, ns, sp, prm);
        }
    out[c] = kept ? (double)liq / (double)kept : -1.0;
  }
}
