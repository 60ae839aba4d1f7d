"""Pins of the oracle's surface-tension curvature chain (Sec. 2.4, the CSF
surface-tension term): each stage against a closed form worked out by hand
on uniform hexahedra, exactness for linear fields, closed cells, phase swap,
and the curvature 2/R of a sphere."""
import numpy as np
import pytest

import oracle
from synth import fields, meshes


@pytest.fixture(scope="module")
def hex6():
    m = meshes.hex_mesh(6)
    return m, oracle.geometry(m)


def _idx(geom, h):
    return np.floor(geom.xc / h).astype(int)


def test_smoothing_of_a_step_matches_the_hand_computed_values(hex6):
    """alpha = 1 for x-index >= 3 on 6^3 hexahedra.  On a uniform mesh w_f = 1/2
    and all faces have the same area, so a cell whose y and z neighbours carry
    its own value gets alpha_hat = (5/6) f_i + (f_{i-1} + f_{i+1})/12, and a
    wall face counts the cell's own value: after one sweep the profile along x
    is 0, 0, 1/12, 11/12, 1, 1; after two 0, 1/144, 21/144, 123/144, 143/144, 1."""
    m, geom = hex6
    ix = _idx(geom, 1 / 6)
    alpha = (ix[0] >= 3).astype(float)
    inner = np.all((ix[1:] >= 1) & (ix[1:] <= 4), axis=0)
    for ns, prof in ((1, [0, 0, 1 / 12, 11 / 12, 1, 1]), (2, [0, 1 / 144, 21 / 144, 123 / 144, 143 / 144, 1])):
        ah = oracle.csf_smooth(m, geom, alpha, ns)
        np.testing.assert_allclose(ah[inner], np.asarray(prof)[ix[0, inner]], rtol=0, atol=1e-15)
    # pure regions stay exactly pure
    ah = oracle.csf_smooth(m, geom, np.ones(m.n_cells), 3)
    assert np.all(ah == 1.0)


def test_linear_fields_pass_the_smoothing_and_give_exact_normals():
    """On uniform hexahedra the face average of a linear field is its cell
    value, so smoothing leaves it unchanged away from the walls, and the
    normal is the unit gradient; a constant field has n = 0 (the 1e-15
    regularisation)."""
    m = meshes.hex_mesh(8)
    geom = oracle.geometry(m)
    ix = _idx(geom, 1 / 8)
    g = np.array([0.3, -0.2, 0.5])
    lin = 0.5 + g @ (geom.xc - 0.5)
    inner = np.all((ix >= 2) & (ix <= 5), axis=0)
    ah = oracle.csf_smooth(m, geom, lin, 2)
    np.testing.assert_allclose(ah[inner], lin[inner], atol=1e-15)
    o = oracle.csf(m, geom, lin, n_smooth=0)
    np.testing.assert_allclose(o["n"][:, inner], np.broadcast_to((g / np.linalg.norm(g))[:, None], (3, inner.sum())),
                               atol=1e-12)
    o = oracle.csf(m, geom, np.full(m.n_cells, 0.3), n_smooth=1)
    assert np.all(o["n"] == 0) and np.all(o["kappa_raw"] == 0)


def test_raw_curvature_divergence():
    """-div n by the Gauss sum: exact (-(a+b+c)) for the linear field
    (a x, b y, c z) on uniform hexahedra, where the face-interpolated value is
    the value at the face centre; zero for a constant field on any closed
    cell (Voronoi included); +2/rho for the inward radial unit field of a
    sphere (second order in h)."""
    m = meshes.hex_mesh(8)
    geom = oracle.geometry(m)
    ix = _idx(geom, 1 / 8)
    inner = np.all((ix >= 1) & (ix <= 6), axis=0)
    a, b, c = 0.7, -1.3, 0.4
    n = np.stack([a * geom.xc[0], b * geom.xc[1], c * geom.xc[2]])
    k = oracle.csf_raw_curvature(m, geom, n)
    np.testing.assert_allclose(k[inner], -(a + b + c), atol=1e-12)
    mv = meshes.voronoi_box_mesh(6, seed=4)
    gv = oracle.geometry(mv)
    k = oracle.csf_raw_curvature(mv, gv, np.broadcast_to(np.array([0.3, 0.9, -0.2])[:, None], (3, mv.n_cells)).copy())
    assert np.abs(k).max() < 1e-11
    m = meshes.hex_mesh(40)
    geom = oracle.geometry(m)
    rel = geom.xc - 0.5
    rho = np.linalg.norm(rel, axis=0)
    k = oracle.csf_raw_curvature(m, geom, -rel / rho)
    sel = (rho > 0.25) & (rho < 0.35)
    np.testing.assert_allclose(k[sel], 2 / rho[sel], rtol=5e-3)


def test_two_step_smoothing_closed_forms(hex6):
    """alpha_hat = 1/2 everywhere (all colour weights 1), raw curvature f(x
    index): step 1 averages the cell and its six face neighbours,
    k*_i = (5 f_i + f_{i-1} + f_{i+1})/7 (ignoring the 1e-15); step 2 with
    n = e_x keeps only the x neighbours, k_i = (k*_{i-1} + k*_i + k*_{i+1})/3,
    and with n = e_y only the y neighbours, whose k* equals the cell's
    away from the walls, so k = k*.  A constant raw curvature passes both steps unchanged."""
    m, geom = hex6
    ix = _idx(geom, 1 / 6)
    inner = np.all((ix >= 1) & (ix <= 4), axis=0)
    f = np.array([0.0, 1.0, -2.0, 5.0, 3.0, 1.5])
    kraw = f[ix[0]]
    ah = np.full(m.n_cells, 0.5)
    ex = np.zeros((3, m.n_cells))
    ex[0] = 1.0
    ks, k = oracle.csf_smooth_curvature(m, geom, ah, ex, kraw)
    fpad = np.concatenate([[np.nan], f, [np.nan]])
    i = ix[0, inner]
    ks_exp = (5 * f[i] + fpad[i] + fpad[i + 2]) / 7
    np.testing.assert_allclose(ks[inner], ks_exp, rtol=1e-14)
    ks_line = np.array([np.nan] + [(5 * f[j] + f[j - 1] + f[j + 1]) / 7 for j in range(1, 5)] + [np.nan])
    inner2 = inner & (ix[0] >= 2) & (ix[0] <= 3)
    j = ix[0, inner2]
    np.testing.assert_allclose(k[inner2], (ks_line[j - 1] + ks_line[j] + ks_line[j + 1]) / 3, rtol=1e-14)
    ey = np.zeros((3, m.n_cells))
    ey[1] = 1.0
    ks2, k2 = oracle.csf_smooth_curvature(m, geom, ah, ey, kraw)
    iny = inner & (ix[1] >= 2) & (ix[1] <= 3)          # y neighbours away from the walls
    np.testing.assert_allclose(k2[iny], ks2[iny], rtol=1e-14)
    ks3, k3 = oracle.csf_smooth_curvature(m, geom, ah, ex, np.full(m.n_cells, 2.5))
    np.testing.assert_allclose(k3, 2.5, rtol=1e-14)
    # pure cells: every weight vanishes and the curvature is 0, not 0/0
    ks4, k4 = oracle.csf_smooth_curvature(m, geom, np.ones(m.n_cells), ex, kraw)
    assert np.all(ks4 == 0) and np.all(k4 == 0)


def test_colour_weight_is_the_eighth_power():
    """One cell at alpha_hat = a among pure neighbours: k* = k~ w / (w + eps)
    with w = (1 - 2|1/2 - a|)^8, so k*/k~ = w/(w + 1e-15)."""
    m = meshes.hex_mesh(4)
    geom = oracle.geometry(m)
    ah = np.zeros(m.n_cells)
    P = 21
    for a in (0.5, 0.4, 0.1, 0.97):
        ah[P] = a
        kraw = np.zeros(m.n_cells)
        kraw[P] = 3.0
        ks, _ = oracle.csf_smooth_curvature(m, geom, ah, np.zeros((3, m.n_cells)), kraw)
        w = (1 - 2 * abs(0.5 - a)) ** 8
        assert ks[P] == pytest.approx(3.0 * w / (w + 1e-15), rel=1e-13)


def test_phase_swap_flips_curvature_and_keeps_the_force():
    m = meshes.voronoi_box_mesh(10, seed=6)
    geom = oracle.geometry(m)
    a = fields.sphere_alpha(m, np.array([[0.45, 0.5, 0.55, 0.28]]), K=8)
    o1 = oracle.csf(m, geom, a, n_smooth=2, sigma=0.07)
    o2 = oracle.csf(m, geom, 1.0 - a, n_smooth=2, sigma=0.07)
    np.testing.assert_allclose(o2["alpha_hat"], 1.0 - o1["alpha_hat"], atol=1e-14)
    sel = np.abs(o1["alpha_hat"] - 0.5) < 0.49
    np.testing.assert_allclose(o2["n"][:, sel], -o1["n"][:, sel], atol=1e-9)
    sk = np.abs(o1["kappa"]).max()
    np.testing.assert_allclose(o2["kappa"], -o1["kappa"], atol=1e-9 * sk)
    np.testing.assert_allclose(o2["F"], o1["F"], atol=1e-9 * np.abs(o1["F"]).max())


@pytest.mark.parametrize("kind", ["hex", "voronoi"])
def test_sphere_curvature_is_two_over_r(kind):
    """A droplet (liquid inside, n pointing inwards) of radius R: the smoothed
    curvature of the cells with |alpha_hat - 1/2| < 1/4 averages 2/R within
    8 %; a bubble gives -2/R."""
    m = meshes.hex_mesh(32) if kind == "hex" else meshes.voronoi_box_mesh(16, 3)
    geom = oracle.geometry(m)
    R = 0.3
    bub = fields.sphere_alpha(m, np.array([[0.5, 0.5, 0.5, R]]), K=12)
    for alpha, sign in ((1.0 - bub, 1.0), (bub, -1.0)):
        o = oracle.csf(m, geom, alpha, n_smooth=2)
        sel = np.abs(o["alpha_hat"] - 0.5) < 0.25
        assert sign * np.mean(o["kappa"][sel]) * R / 2 == pytest.approx(1.0, abs=0.08)


def test_smoothing_weight_on_a_graded_mesh():
    """x stretched so the cells along x have widths dx_i: for the vapour cell
    i next to the liquid column i+1, only its x+ face carries liquid, with
    alpha_hat_f = w = dx_i/(dx_i + dx_{i+1}) (the face splits the centre
    connection in that ratio), so one sweep gives w A_x / sum_f A_f with
    A_x = h^2 and the side faces dx_i h: alpha_hat = w h / (2h + 4 dx_i)."""
    m = meshes.hex_mesh(6)
    xs = np.array([0.0, 0.1, 0.25, 0.45, 0.6, 0.85, 1.0])     # new x of the 7 vertex planes
    xyz = m.vert_xyz.copy()
    k = np.rint(xyz[0] * 6).astype(int)
    xyz[0] = xs[k]
    m = meshes.Mesh(**{**m.__dict__, "vert_xyz": xyz})
    geom = oracle.geometry(m)
    dx = np.diff(xs)
    ix = np.searchsorted(xs, geom.xc[0]) - 1
    h = 1 / 6
    iy = np.floor(geom.xc[1:] / h).astype(int)
    inner = np.all((iy >= 1) & (iy <= 4), axis=0)
    alpha = (ix >= 3).astype(float)
    ah = oracle.csf_smooth(m, geom, alpha, 1)
    cell = inner & (ix == 2)
    w = dx[2] / (dx[2] + dx[3])
    np.testing.assert_allclose(ah[cell], w * h / (2 * h + 4 * dx[2]), rtol=1e-13)
    cell = inner & (ix == 3)                     # liquid side: 1 - (1 - w') * h / (2h + 4 dx_3)
    w3 = dx[3] / (dx[3] + dx[2])                 # weight of the vapour neighbour seen from cell 3
    np.testing.assert_allclose(ah[cell], 1 - w3 * h / (2 * h + 4 * dx[3]), rtol=1e-13)
