"""The angular analysis of the gradient-anisotropy study (Sec. 3.3) and the
finding it reproduces on the oracle: a coherent four-fold mode of |grad T| on
hexahedral meshes that the Voronoi meshes do not show."""
import numpy as np
import pytest

import oracle
from paper_2604_14938_amd import anisotropy as an
from synth import workloads


def test_polar_recovers_a_planted_mode():
    """Values 1 + a cos(m theta + phi) on points around a circle: the binned
    profile's Fourier amplitude of mode m is a (in % of the mean), the other
    modes vanish, and the min/max ratio is that of the bin means."""
    rng = np.random.default_rng(0)
    th = rng.uniform(-np.pi, np.pi, 20000)
    xc = np.stack([0.5 + 0.3 * np.cos(th), 0.5 + 0.3 * np.sin(th), 0.5 + rng.uniform(-0.01, 0.01, th.size)])
    cells = np.arange(th.size)
    for m, a, phi in ((4, 0.12, 0.3), (2, 0.05, -1.0)):
        # value constant inside each bin, so the bin means are exact samples
        n_bins = 48
        k = np.minimum(((th + np.pi) / (2 * np.pi) * n_bins).astype(int), n_bins - 1)
        tc = -np.pi + (k + 0.5) * 2 * np.pi / n_bins
        v = 1.0 + a * np.cos(m * tc + phi)
        P = an.polar(xc, v, cells, (0.5, 0.5, 0.5), 0.02, n_bins=n_bins)
        assert P["modes_pct"][m - 1] == pytest.approx(100 * a, rel=1e-10)
        others = [x for i, x in enumerate(P["modes_pct"]) if i != m - 1]
        assert max(others) < 1e-9
        tb = -np.pi + (np.arange(n_bins) + 0.5) * 2 * np.pi / n_bins
        b = 1.0 + a * np.cos(m * tb + phi)
        assert P["min_max"] == pytest.approx(b.min() / b.max(), rel=1e-12)
    with pytest.raises(ValueError):
        an.polar(xc[:, :3], np.ones(3), np.arange(3), (0.5, 0.5, 0.5), 0.02, n_bins=48)


def test_interface_cells_are_the_liquid_side_of_crossing_faces():
    from synth import meshes
    m = meshes.hex_mesh(6)
    x = m.cell_vertex_mean()[:, 0]
    alpha = np.where(x < 0.5, 0.0, 1.0)
    alpha[(x > 0.5) & (x < 0.67)] = 0.7          # column 3 mixed, liquid side
    cells = an.interface_cells(alpha, m.face_owner, m.face_neigh)
    expect = np.nonzero((x > 0.5) & (x < 0.67))[0]
    np.testing.assert_array_equal(cells, expect)


def test_erf_profile_gradient_is_the_derivative_of_the_profile():
    c = np.array([0.5, 0.5, 0.5])
    pts = np.array([[0.8, 0.5, 0.5], [0.5, 0.1, 0.55]]).T
    g = an.erf_profile_gradient(pts, c, 0.25, 0.05, 1.25)
    from scipy.special import erf
    for i in range(2):
        rho = np.linalg.norm(pts[:, i] - c)
        e = 1e-7
        fd = 1.25 * (erf((rho + e - 0.25) / 0.05) - erf((rho - e - 0.25) / 0.05)) / (2 * e)
        assert g[i] == pytest.approx(fd, rel=1e-6)


def _m4(kind, n, **kw):
    wl = workloads.static_sphere(kind, n)
    geom = oracle.geometry(wl.mesh)
    cells = an.interface_cells(wl.alpha, wl.mesh.face_owner, wl.mesh.face_neigh)
    exact = an.erf_profile_gradient(geom.xc, wl.meta["centre"], wl.meta["r"], wl.meta["width"], wl.meta["dT"])
    g, _ = oracle.grad(wl.mesh, geom, wl.T, wl.T_bface, wl.T_sat, wl.alpha, **kw)
    return an.polar(geom.xc, np.linalg.norm(g, axis=0) / exact, cells, wl.meta["centre"], wl.mesh.h, n_bins=24)


@pytest.mark.parametrize("modified", [True, False])
def test_hexahedral_meshes_show_a_coherent_four_fold_mode(modified):
    """Static sphere, erf profile, the oracle's gradient: on 32^3 hexahedra
    the m = 4 mode of |grad T| dominates every other mode of 1..8 (the
    coherent pattern of the Cartesian stencil); on a Voronoi mesh of similar
    size (2 * 25^3 cells) m = 4 is several times smaller and not dominant."""
    hx = _m4("hex", 32, modified=modified)
    vo = _m4("voronoi", 25, modified=modified)
    m = hx["modes_pct"]
    assert m[3] > 3.0 and m[3] > 4 * max(m[i] for i in range(8) if i != 3)
    assert vo["m4_pct"] < hx["m4_pct"] / 4
    assert vo["m4_pct"] < 2 * np.median(vo["modes_pct"]) + 1.0


def test_vertex_stencil_equals_face_stencil_on_voronoi_meshes():
    """Two Voronoi cells that share a vertex also share a face (a vertex is
    the circumcentre of a Delaunay tetrahedron, whose vertex pairs are
    Delaunay edges), so the extended stencil adds nothing there; on
    hexahedra it adds the edge and corner neighbours."""
    wl = workloads.static_sphere("voronoi", 8)
    geom = oracle.geometry(wl.mesh)
    a, _ = oracle.grad(wl.mesh, geom, wl.T, wl.T_bface, wl.T_sat, wl.alpha)
    b, _ = oracle.grad(wl.mesh, geom, wl.T, wl.T_bface, wl.T_sat, wl.alpha, extended=True)
    np.testing.assert_allclose(b, a, rtol=1e-12, atol=1e-12 * np.abs(a).max())
    wl = workloads.static_sphere("hex", 12)
    geom = oracle.geometry(wl.mesh)
    a, _ = oracle.grad(wl.mesh, geom, wl.T, wl.T_bface, wl.T_sat, wl.alpha)
    b, _ = oracle.grad(wl.mesh, geom, wl.T, wl.T_bface, wl.T_sat, wl.alpha, extended=True)
    assert np.abs(b - a).max() > 1e-3 * np.abs(a).max()
