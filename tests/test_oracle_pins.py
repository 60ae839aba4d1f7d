"""Pins of the CPU oracle against closed forms, invariants and the paper.

Each test fixes part of the oracle with something other than the oracle
itself: analytic plane cuts of a cube and a tetrahedron, independent convex
hull clipping, Monte Carlo counting, symmetry of the construction, exactness
of least squares on linear data, and the one-dimensional relations of App. C.
"""
import numpy as np
import pytest

import oracle
from synth import meshes, workloads
from tests import polytools as pt


def _linear_phi(mesh, g, c0=0.0):
    return mesh.vert_xyz.T @ g + c0


# ------------------------------------------------------------------ plane cuts
def test_unit_cube_plane_cut_matches_closed_form():
    """Vertex-linear field on the unit cube: the iso-cut is the plane, so the
    liquid volume, the interface area, the normal and the centre distance have
    closed forms (edge intersection, Eq. edge_intersection, is exact here)."""
    mesh = meshes.hex_mesh(1)
    om = oracle.OMesh(mesh)
    geom = oracle.geometry(om)
    assert geom.V[0] == pytest.approx(1.0, abs=1e-15)
    rng = np.random.default_rng(11)
    for _ in range(40):
        m = rng.uniform(0.1, 1.0, 3) * rng.choice([-1, 1], 3)
        phi = _linear_phi(mesh, m)
        lo, hi = phi.min(), phi.max()
        s = rng.uniform(lo, hi)
        res = oracle.cut_cell(om, 0, geom.xc, phi, s)
        # map to positive coefficients: x_i -> 1 - x_i for m_i < 0
        mp = np.abs(m)
        shift = np.sum(np.where(m < 0, -m, 0.0))    # m.x = mp.x' - shift
        v_below = pt.below_unit_cube(mp, s + shift)
        assert res["V"] == pytest.approx(1.0 - v_below, abs=1e-14)
        assert res["A"] == pytest.approx(pt.below_unit_cube_area(mp, s + shift), rel=1e-12, abs=1e-14)
        n = res["S"] / np.linalg.norm(res["S"])
        np.testing.assert_allclose(n, m / np.linalg.norm(m), atol=1e-12)
        # signed distance of the centroid to the plane, positive on the liquid side
        d = -np.dot(n, res["c"])
        assert d == pytest.approx((m @ geom.xc[:, 0] - s) / np.linalg.norm(m), abs=1e-13)


def test_tetrahedron_cut_matches_simplex_formula():
    """V_liq/V of a linear field on a tetrahedron equals 1 - sum_i (s-f_i)_+^3 /
    prod_{j!=i}(f_j-f_i) in every case (one, two or three vertices liquid)."""
    rng = np.random.default_rng(5)
    for _ in range(60):
        P = rng.normal(size=(4, 3))
        mesh = pt.tet_mesh(P)
        om = oracle.OMesh(mesh)
        geom = oracle.geometry(om)
        vt = abs(np.linalg.det(np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]]))) / 6.0
        assert geom.V[0] == pytest.approx(vt, rel=1e-13)
        g = rng.normal(size=3)
        phi = _linear_phi(mesh, g)
        s = rng.uniform(phi.min(), phi.max())
        res = oracle.cut_cell(om, 0, geom.xc, phi, s)
        assert res["V"] / vt == pytest.approx(1.0 - pt.tet_fraction_below(phi, s), abs=1e-12)
        np.testing.assert_allclose(res["S"] / np.linalg.norm(res["S"]), g / np.linalg.norm(g), atol=1e-11)
        assert res["nloops"] == 1


def test_convex_hull_cut_matches_independent_clipping():
    """Random convex polyhedra (triangulated hulls), linear field: volume and
    cut area agree with convex-hull clipping done by scipy."""
    rng = np.random.default_rng(3)
    for _ in range(25):
        pts = rng.normal(size=(rng.integers(8, 30), 3))
        mesh = pt.hull_mesh(pts)
        om = oracle.OMesh(mesh)
        geom = oracle.geometry(om)
        from scipy.spatial import ConvexHull
        assert geom.V[0] == pytest.approx(ConvexHull(pts).volume, rel=1e-12)
        g = rng.normal(size=3)
        phi = _linear_phi(mesh, g)
        s = rng.uniform(np.quantile(phi, 0.1), np.quantile(phi, 0.9))
        res = oracle.cut_cell(om, 0, geom.xc, phi, s)
        vol, area = pt.clip_hull_volume_area(mesh.vert_xyz.T, g, s)
        assert res["V"] == pytest.approx(vol, rel=1e-11)
        assert res["A"] == pytest.approx(area, rel=1e-11)


def test_monte_carlo_volume_on_voronoi_cells():
    """Counting 4e5 uniform points in a Voronoi cell (nearest-seed test) on the
    liquid side of a plane agrees with the cut volume within 5 sigma."""
    mesh = meshes.voronoi_box_mesh(5, seed=9)
    om = oracle.OMesh(mesh)
    geom = oracle.geometry(om)
    rng = np.random.default_rng(1)
    off, nb = mesh.face_neighbours()
    for P in rng.choice(mesh.n_cells, 4, replace=False):
        bb = mesh.cell_bbox()[P]
        g = rng.normal(size=3)
        phi = _linear_phi(mesh, g)
        cell_phi = phi[mesh.face_vert[np.concatenate([np.arange(mesh.face_vert_off[f], mesh.face_vert_off[f + 1])
                                                        for f in mesh.cell_face[mesh.cell_face_off[P]:mesh.cell_face_off[P + 1]]])]]
        s = 0.5 * (cell_phi.min() + cell_phi.max())
        nsamp = 400_000
        X = rng.uniform(bb[:3], bb[3:], size=(nsamp, 3))
        p = mesh.seeds[P]
        inside = np.ones(nsamp, bool)
        for q in nb[off[P]:off[P + 1]]:
            qq = mesh.seeds[q]
            inside &= (X @ (qq - p)) <= 0.5 * (qq @ qq - p @ p)
        box_vol = np.prod(bb[3:] - bb[:3])
        v_cell = inside.mean() * box_vol
        liq = inside & (X @ g >= s)
        frac = liq.mean()
        v_mc = frac * box_vol
        sigma = np.sqrt(frac * (1 - frac) / nsamp) * box_vol
        res = oracle.cut_cell(om, P, geom.xc, phi, s)
        assert abs(res["V"] - v_mc) < 5 * sigma + 1e-15
        assert abs(geom.V[P] - v_cell) < 5 * np.sqrt(inside.mean() * (1 - inside.mean()) / nsamp) * box_vol


# ---------------------------------------------------- general (non-linear) fields
def _cell_vertex_ids(mesh, P):
    fs = mesh.cell_face[mesh.cell_face_off[P]:mesh.cell_face_off[P + 1]]
    return np.unique(np.concatenate([mesh.face_vert[mesh.face_vert_off[f]:mesh.face_vert_off[f + 1]] for f in fs]))


def test_liquid_and_vapour_volumes_sum_to_cell_volume():
    """For an arbitrary vertex field the iso-surface seen from the liquid side
    (phi >= s) and from the vapour side (-phi >= -s) is the same surface, so
    the two volumes add up to V_P."""
    mesh = meshes.voronoi_box_mesh(5, seed=4)
    om = oracle.OMesh(mesh)
    geom = oracle.geometry(om)
    rng = np.random.default_rng(2)
    phi = rng.uniform(0, 1, mesh.n_verts)   # rough field: saddles, several loops
    nloops_seen = set()
    for P in range(mesh.n_cells):
        ids = _cell_vertex_ids(mesh, P)
        for s in rng.uniform(phi[ids].min(), phi[ids].max(), 3):
            a = oracle.cut_cell(om, P, geom.xc, phi, s)
            b = oracle.cut_cell(om, P, geom.xc, -phi, -s)
            assert a["V"] + b["V"] == pytest.approx(geom.V[P], rel=1e-13)
            assert a["A"] == pytest.approx(b["A"], rel=1e-12)
            np.testing.assert_allclose(a["S"], -b["S"], atol=1e-14 * geom.V[P] ** (2 / 3))
            nloops_seen.add(a["nloops"])
    assert max(nloops_seen) >= 2   # the rough field exercises multi-loop cells


def test_volume_is_monotone_in_isovalue():
    """V_liq(s) does not increase with s (sampled at 400 isovalues per cell) for
    a smooth inverse-distance vertex field."""
    wl = workloads.voronoi_bubble(n=8, seed=3, r=0.3)
    om = oracle.OMesh(wl.mesh)
    geom = oracle.geometry(om)
    phi = oracle.vertex_field(om, geom.xc, wl.alpha)
    mixed = np.nonzero((wl.alpha > 1e-8) & (wl.alpha < 1 - 1e-8))[0]
    for P in mixed[:20]:
        ids = _cell_vertex_ids(wl.mesh, P)
        ss = np.linspace(phi[ids].min(), phi[ids].max(), 400)
        V = np.array([oracle.cut_cell(om, P, geom.xc, phi, s)["V"] for s in ss])
        assert V[0] == pytest.approx(geom.V[P], rel=1e-13)
        assert V[-1] == pytest.approx(0.0, abs=1e-15 * geom.V[P])
        assert np.all(np.diff(V) <= 1e-14 * geom.V[P])


# ---------------------------------------------------------------- reconstruction
def test_alpha_recovered_on_every_mixed_cell(hex_sphere_wl, small_voronoi_wl):
    for wl in (hex_sphere_wl, small_voronoi_wl):
        om = oracle.OMesh(wl.mesh)
        geom = oracle.geometry(om)
        rec = oracle.reconstruct(om, wl.alpha, geom)
        mixed = rec["status"] != oracle.NOT_MIXED
        assert mixed.sum() == wl.n_mixed
        ok = rec["status"] == oracle.OK
        noroot = rec["status"] == oracle.NO_ROOT
        assert np.all(ok | noroot | ~mixed)
        assert noroot.sum() <= 0.02 * mixed.sum()
        a = wl.alpha[ok]
        err = np.abs(rec["alpha_got"][ok] - a)
        # recovered to 1e-12 absolute; most cells stop on the relative tolerance
        assert err.max() <= 1e-12
        assert np.mean(err <= 1e-13 * np.minimum(a, 1 - a)) > 0.5
        assert np.all(rec["A"][mixed] > 0)
        assert np.all(np.abs(np.linalg.norm(rec["n"][:, mixed], axis=0) - 1) < 1e-14)
        # no-root cells: the volume jumps across alpha at s*, and the side kept
        # is the one nearer to alpha
        phi = oracle.vertex_field(om, geom.xc, wl.alpha)
        for P in np.nonzero(noroot)[0]:
            s = rec["s"][P]
            vm = oracle.cut_cell(om, P, geom.xc, phi, s - 1e-12)["V"] / geom.V[P]
            vp = oracle.cut_cell(om, P, geom.xc, phi, s + 1e-12)["V"] / geom.V[P]
            assert vm > wl.alpha[P] > vp
            assert abs(rec["alpha_got"][P] - wl.alpha[P]) == pytest.approx(
                min(abs(vm - wl.alpha[P]), abs(vp - wl.alpha[P])), abs=1e-9)
        # normal points from vapour (inside the bubble) to liquid (outward)
        c = wl.meta["spheres"][0, :3]
        radial = geom.xc[:, mixed] - c[:, None]
        assert np.mean(np.sum(radial * rec["n"][:, mixed], 0) > 0) > 0.97


def test_total_interface_area_approximates_the_sphere(hex_sphere_wl):
    rec = oracle.reconstruct(hex_sphere_wl.mesh, hex_sphere_wl.alpha)
    assert rec["A"].sum() == pytest.approx(4 * np.pi * 0.3 ** 2, rel=0.01)


def test_rigid_motion_invariance(small_voronoi_wl):
    wl = small_voronoi_wl
    rng = np.random.default_rng(8)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    t = rng.normal(size=3)
    m2 = meshes.Mesh(**{**wl.mesh.__dict__, "vert_xyz": Q @ wl.mesh.vert_xyz + t[:, None]})
    a = oracle.reconstruct(wl.mesh, wl.alpha)
    b = oracle.reconstruct(m2, wl.alpha)
    mixed = (a["status"] == oracle.OK) & (b["status"] == oracle.OK)
    np.testing.assert_allclose(b["A"][mixed], a["A"][mixed], rtol=1e-9)
    np.testing.assert_allclose(b["d"][mixed], a["d"][mixed], atol=1e-9 * wl.mesh.h)
    np.testing.assert_allclose(b["alpha_got"][mixed], a["alpha_got"][mixed], atol=1e-12)
    np.testing.assert_allclose(b["n"][:, mixed], Q @ a["n"][:, mixed], atol=1e-9)


def test_phase_swap_symmetry(small_voronoi_wl):
    """alpha -> 1-alpha: s -> 1-s, n -> -n, same A, d -> -d."""
    wl = small_voronoi_wl
    a = oracle.reconstruct(wl.mesh, wl.alpha)
    b = oracle.reconstruct(wl.mesh, 1.0 - wl.alpha)
    m = (a["status"] == oracle.OK) & (b["status"] == oracle.OK)
    np.testing.assert_allclose(b["A"][m], a["A"][m], rtol=1e-9)
    np.testing.assert_allclose(b["n"][:, m], -a["n"][:, m], atol=1e-9)
    np.testing.assert_allclose(b["d"][m], -a["d"][m], atol=1e-9 * wl.mesh.h)
    np.testing.assert_allclose(b["s"][m], 1.0 - a["s"][m], atol=1e-9)


def test_fixed_isovalue_mode_cuts_at_one_half(hex_sphere_wl):
    wl = hex_sphere_wl
    rec = oracle.reconstruct(wl.mesh, wl.alpha, fixed_iso=True, iso=0.5)
    m = rec["status"] != oracle.NOT_MIXED
    assert np.all(rec["s"][m] == 0.5)
    assert np.all(rec["iters"][m] == 1)


def test_degenerate_vertex_field_falls_back_to_linear_alpha():
    """A uniform alpha gives a constant vertex field: the cell is flagged and,
    with zero alpha gradient, no interface is placed."""
    mesh = meshes.hex_mesh(4)
    alpha = np.full(mesh.n_cells, 0.4)
    rec = oracle.reconstruct(mesh, alpha)
    assert np.all(rec["status"] == oracle.DEGENERATE)
    assert np.all(rec["A"] == 0)
    # a constant field on the vertices but a linear alpha across the cells
    x = oracle.geometry(mesh).xc
    alpha = 0.5 + 0.1 * (x[0] - 0.5)
    phi = np.full(mesh.n_verts, 0.5)
    rec = oracle.reconstruct(mesh, alpha, phi=phi)
    assert np.all(rec["status"] == oracle.DEGENERATE)
    ok = rec["A"] > 0
    assert ok.all()
    np.testing.assert_allclose(rec["n"][0], 1.0, atol=1e-12)
    np.testing.assert_allclose(rec["A"], mesh.h ** 2, rtol=1e-12)


def test_bad_and_pure_cells_are_not_reconstructed():
    mesh = meshes.hex_mesh(3)
    alpha = np.full(mesh.n_cells, 1.0)
    alpha[0] = np.nan
    alpha[1] = -0.2
    alpha[2] = 0.0
    alpha[3] = 1e-9
    rec = oracle.reconstruct(mesh, alpha)
    assert list(rec["status"][:4]) == [oracle.BAD_INPUT, oracle.BAD_INPUT, oracle.NOT_MIXED, oracle.NOT_MIXED]
    assert np.all(rec["status"][4:] == oracle.NOT_MIXED)
    assert np.all(np.isnan(rec["s"]))


def test_narrowed_bracket_gives_the_same_result(small_voronoi_wl):
    """A valid narrowed bracket and a wrong one both end inside the stopping
    window; the wrong one is flagged as a fallback."""
    wl = small_voronoi_wl
    a = oracle.reconstruct(wl.mesh, wl.alpha)
    m = a["status"] == oracle.OK
    s = np.where(m, a["s"], np.nan)
    good = oracle.reconstruct(wl.mesh, wl.alpha, hint_lo=s - 1e-3, hint_hi=s + 1e-3)
    bad = oracle.reconstruct(wl.mesh, wl.alpha, hint_lo=s + 1e-2, hint_hi=s + 2e-2)
    for r in (good, bad):
        np.testing.assert_allclose(r["alpha_got"][m], a["alpha_got"][m], atol=1e-12)
        np.testing.assert_allclose(r["A"][m], a["A"][m], rtol=1e-8, atol=1e-9 * wl.mesh.h ** 2)
    assert np.all(good["status"][m] == oracle.OK)
    assert np.mean(good["iters"][m]) < np.mean(a["iters"][m])
    assert np.all(np.isin(bad["status"][m], [oracle.LEARNED_FALLBACK, oracle.OK]))
    assert np.mean(bad["status"][m] == oracle.LEARNED_FALLBACK) > 0.9


# ------------------------------------------------------------- least squares
def test_least_squares_exact_for_linear_field(small_voronoi_wl):
    wl = small_voronoi_wl
    geom = oracle.geometry(wl.mesh)
    g = np.array([0.3, -1.7, 2.2])
    T = 5.0 + g @ geom.xc
    Tb = 5.0 + g @ geom.xf
    grad, st = oracle.grad(wl.mesh, geom, T, Tb, 0.0, np.ones(wl.mesh.n_cells), modified=True)
    assert np.all(st == oracle.OK)
    np.testing.assert_allclose(grad, np.broadcast_to(g[:, None], grad.shape), rtol=0, atol=1e-11)


@pytest.mark.parametrize("weight,extended", [(0, False), (1, False), (2, True), (0, True)])
def test_modified_stencil_exact_for_planar_interface(weight, extended):
    """alpha = 1/2 + kappa dist(x), T = T_sat + G dist(x) for a plane: the
    alpha-interpolated crossing points lie on the plane where T = T_sat, so the
    interface-modified gradient is exactly G n, for any weights and for the
    vertex-neighbour stencil alike.  The printed mirror weight of
    Eq. front_interpolation does not have this property."""
    wl = workloads.voronoi_bubble(n=8, seed=5, r=0.3)
    mesh = wl.mesh
    geom = oracle.geometry(mesh)
    nrm = np.array([1.0, 2.0, -0.5])
    nrm /= np.linalg.norm(nrm)
    dist = nrm @ (geom.xc - 0.5)
    alpha = 0.5 + 0.6 * dist           # stays inside (0, 1) on the unit box
    assert alpha.min() > 0 and alpha.max() < 1
    T_sat, G = 373.15, 40.0
    T = T_sat + G * dist
    Tb = T_sat + G * (nrm @ (geom.xf - 0.5))
    grad, _ = oracle.grad(mesh, geom, T, Tb, T_sat, alpha, modified=True, weight=weight, extended=extended)
    np.testing.assert_allclose(grad, np.broadcast_to((G * nrm)[:, None], grad.shape), atol=1e-9)
    band = oracle.band_mask(mesh, alpha)
    printed, _ = oracle.grad(mesh, geom, T, Tb, T_sat, alpha, modified=True, printed=True, weight=weight,
                             extended=extended)
    err = np.linalg.norm(printed - (G * nrm)[:, None], axis=0)
    assert err[band & (np.abs(alpha - 0.5) > 0.05)].max() > 1.0


def _one_d_setup(theta_frac, d_over_h, n=8, weight=0, extended=False, full=False):
    """Hex mesh, interface normal to x between two cell columns; returns
    (gradient from the oracle, closed form Eq. g_fm, std ratio)."""
    mesh = meshes.hex_mesh(n)
    geom = oracle.geometry(mesh)
    h = mesh.h
    x = geom.xc[0]
    i_iface = n // 2                       # cells with index >= i_iface are liquid
    xP = (i_iface + 0.5) * h               # first liquid cell centre
    x_int = xP - d_over_h * h              # interface between P and its vapour neighbour
    # alpha linear in x across P and its vapour neighbour Q so that the
    # alpha-interpolated crossing sits at x_int; 0 / 1 further away
    kappa = 0.4 / h
    alpha = np.clip(0.5 + kappa * (x - x_int), 0.0, 1.0)
    T_sat, dT = 373.15, 2.0
    T_far = T_sat + dT
    T = np.where(x > x_int, T_sat + dT * np.clip((x - x_int) / (h * (1 + d_over_h)), 0, 1), T_sat)
    theta = theta_frac * dT
    T = np.where(np.isclose(x, xP), T_sat + theta, T)
    T = np.where(np.isclose(x, xP + h), T_far, T)
    Tb = np.full(mesh.n_faces, T_sat)
    grad, _ = oracle.grad(mesh, geom, T, Tb, T_sat, alpha, modified=True, weight=weight, extended=extended)
    P = np.nonzero(np.isclose(x, xP) & np.isclose(geom.xc[1], (n // 2 + 0.5) * h) &
                   np.isclose(geom.xc[2], (n // 2 + 0.5) * h))[0][0]
    d = d_over_h * h
    g_fm = ((T[P] - T_sat) * d + (T_far - T[P]) * h) / (d * d + h * h)   # Eq. g_fm
    g_std = (T_far - T_sat) / (2 * h)                                     # Eq. g_std
    if full:
        return grad[:, P], dict(T_P=T[P], T_sat=T_sat, T_far=T_far, d=d, h=h, g_fm=g_fm)
    return grad[:, P], g_fm, g_std


@pytest.mark.parametrize("d_over_h", [0.3, 0.5, 0.7])
@pytest.mark.parametrize("theta_frac", [0.0, 0.2])
def test_one_dimensional_modified_gradient_matches_app_c(d_over_h, theta_frac):
    g, g_fm, _ = _one_d_setup(theta_frac, d_over_h)
    assert g[0] == pytest.approx(g_fm, rel=1e-12)
    assert abs(g[1]) < 1e-9 and abs(g[2]) < 1e-9


@pytest.mark.parametrize("d_over_h", [0.3, 0.7])
@pytest.mark.parametrize("theta_frac", [0.0, 0.2])
def test_one_dimensional_weighted_gradients(d_over_h, theta_frac):
    """The same one-dimensional stencil (the interface point at distance d
    with T_sat, the far neighbour at h) under the weights of App. B: with
    w = 1/|r| the fit is the secant from the interface point to the far
    neighbour, (T_far - T_sat)/(d + h); with w = 1/|r|^2 it is the mean of the
    two one-sided slopes.  The vertex-neighbour stencil with uniform weights
    shifts every column by the same y/z offsets and gives Eq. g_fm again."""
    g1, c = _one_d_setup(theta_frac, d_over_h, weight=1, full=True)
    assert g1[0] == pytest.approx((c["T_far"] - c["T_sat"]) / (c["d"] + c["h"]), rel=1e-12)
    g2, c = _one_d_setup(theta_frac, d_over_h, weight=2, full=True)
    mean = 0.5 * ((c["T_P"] - c["T_sat"]) / c["d"] + (c["T_far"] - c["T_P"]) / c["h"])
    assert g2[0] == pytest.approx(mean, rel=1e-12)
    ge, c = _one_d_setup(theta_frac, d_over_h, extended=True, full=True)
    assert ge[0] == pytest.approx(c["g_fm"], rel=1e-12)
    for g in (g1, g2, ge):
        assert abs(g[1]) < 1e-9 and abs(g[2]) < 1e-9


@pytest.mark.parametrize("weight", [0, 1, 2])
def test_vertex_neighbour_stencil_on_a_cubic_field(weight):
    """T = x^2 y on a uniform hex mesh, interior cells at (a, b, .): the face
    stencil gives (2ab, a^2, 0) for any weights (all distances h); the
    26-cell vertex stencil gives (2ab, a^2 + c h^2, 0), where c is the
    w-weighted mean of the squared x offsets (in units of h) over the
    (x, z) offsets of the y-neighbours: sum_w(sx^2) / sum_w(1) over
    sx, sz in {-1, 0, 1} with w = (1 + sx^2 + sz^2)^(-k/2): 2/3 for k = 0,
    (sqrt2 + 4/sqrt3)/(1 + 2 sqrt2 + 4/sqrt3) for k = 1 and 7/13 for k = 2."""
    n = 8
    mesh = meshes.hex_mesh(n)
    geom = oracle.geometry(mesh)
    h = mesh.h
    T = geom.xc[0] ** 2 * geom.xc[1]
    Tb = geom.xf[0] ** 2 * geom.xf[1]
    one = np.ones(mesh.n_cells)
    idx = np.floor(geom.xc / h).astype(int)
    inner = np.all((idx >= 1) & (idx <= n - 2), axis=0)
    a, b = geom.xc[0, inner], geom.xc[1, inner]
    c = {0: 2.0 / 3.0, 1: (np.sqrt(2) + 4 / np.sqrt(3)) / (1 + 2 * np.sqrt(2) + 4 / np.sqrt(3)), 2: 7.0 / 13.0}[weight]
    gf, _ = oracle.grad(mesh, geom, T, Tb, 0.0, one, weight=weight)
    ge, _ = oracle.grad(mesh, geom, T, Tb, 0.0, one, weight=weight, extended=True)
    np.testing.assert_allclose(gf[0, inner], 2 * a * b, atol=1e-12)
    np.testing.assert_allclose(gf[1, inner], a * a, atol=1e-12)
    np.testing.assert_allclose(ge[0, inner], 2 * a * b, atol=1e-12)
    np.testing.assert_allclose(ge[1, inner], a * a + c * h * h, atol=1e-12)
    assert np.abs(gf[2, inner]).max() < 1e-12 and np.abs(ge[2, inner]).max() < 1e-12


def test_boost_ratio_reproduces_printed_values():
    rows = np.loadtxt(__file__.replace("test_oracle_pins.py", "golden/appc_boost_ratio.txt"))
    for d_over_h, printed in rows:
        if d_over_h == 0.0:
            continue
        g, _, g_std = _one_d_setup(0.0, d_over_h)
        assert round(g[0] / g_std, 2) == pytest.approx(printed, abs=0.011)
    # d -> 0: the one-sided difference over h, twice the central one
    g, _, g_std = _one_d_setup(0.0, 1e-6)
    assert g[0] / g_std == pytest.approx(2.0, rel=1e-5)


# ------------------------------------------------------------------ mass rate
def test_mass_transfer_identity_and_sign(hex_sphere_wl):
    wl = hex_sphere_wl
    r = oracle.run_path(wl)
    rec, geom = r["rec"], r["geom"]
    A, n, g = rec["A"], rec["n"], r["grad"]
    has = A > 0
    assert np.all(r["mdot"][~has] == 0) and np.all(r["Qdot"][~has] == 0)
    liq = wl.alpha >= 0.5
    expect = np.where(liq, wl.k_l * np.sum(g * n, 0) * A, -wl.k_v * np.sum(g * n, 0) * A) / (wl.h_lv * geom.V)
    np.testing.assert_allclose(r["mdot"][has], expect[has], rtol=1e-13)
    np.testing.assert_allclose(r["Qdot"], -r["mdot"] * wl.h_lv, rtol=1e-15)
    # superheated liquid around a vapour bubble: evaporation in liquid cells
    assert np.all(r["mdot"][has & liq] > 0)


def test_two_sided_gradients_are_used_when_given(hex_sphere_wl):
    wl = hex_sphere_wl
    r = oracle.run_path(wl)
    rec, geom = r["rec"], r["geom"]
    N = wl.mesh.n_cells
    gl = np.tile([[1.0], [0.0], [0.0]], (1, N))
    gv = np.tile([[0.0], [0.0], [-2.0]], (1, N))
    mdot, _ = oracle.mass_transfer(geom, wl.alpha, rec["n"], rec["A"], r["grad"], 0.5, 0.25, 10.0, gl=gl, gv=gv)
    has = rec["A"] > 0
    ql = 0.5 * rec["n"][0] * rec["A"]
    qv = -0.25 * (-2.0 * rec["n"][2]) * rec["A"]
    np.testing.assert_allclose(mdot[has], ((ql + qv) / (10.0 * geom.V))[has], rtol=1e-13)


# ---------------------------------------------------------------- extrapolation
def _sym_boundary(mesh):
    """A copy of the mesh whose boundary faces are symmetry faces (skipped by
    the gradient stencil)."""
    import copy
    m = copy.copy(mesh)
    m.face_bc = np.where(mesh.face_neigh < 0, 2, 0).astype(np.int8)
    return m


def test_extrapolation_carries_each_phase_slope_across_a_plane():
    """Plane interface, alpha linear in the distance (so the alpha-interpolated
    crossings lie on the plane), T rising with slope G_l in the liquid and G_v
    in the vapour: the interface-modified gradient is G_l n in liquid cells and
    G_v n in vapour cells, and the pseudo-time extrapolation (Eq.
    extrapolation) fills the other phase's field with the other slope, so
    every domain cell ends with G_l n and G_v n."""
    mesh = _sym_boundary(meshes.hex_mesh(8))
    geom = oracle.geometry(mesh)
    nrm = np.array([0.8, 0.5, 0.2])
    nrm /= np.linalg.norm(nrm)
    dist = nrm @ (geom.xc - 0.5)
    alpha = 0.5 + 0.6 * dist
    T_sat, Gl, Gv = 373.15, 40.0, -15.0
    T = T_sat + np.where(dist >= 0, Gl, Gv) * dist
    grad, _ = oracle.grad(mesh, geom, T, np.zeros(mesh.n_faces), T_sat, alpha, modified=True)
    liq = alpha >= 0.5
    np.testing.assert_allclose(grad[:, liq], np.broadcast_to((Gl * nrm)[:, None], grad[:, liq].shape), atol=1e-9)
    np.testing.assert_allclose(grad[:, ~liq], np.broadcast_to((Gv * nrm)[:, None], grad[:, ~liq].shape), atol=1e-9)
    N = mesh.n_cells
    n_int = np.broadcast_to(nrm[:, None], (3, N)).copy()
    gl, gv, sweeps, dom = oracle.extrapolate(mesh, geom, alpha, grad, n_int, np.ones(N), max_iter=2000, tol=1e-13)
    assert dom.all() and sweeps < 2000
    np.testing.assert_allclose(gl, np.broadcast_to((Gl * nrm)[:, None], gl.shape), atol=1e-9)
    np.testing.assert_allclose(gv, np.broadcast_to((Gv * nrm)[:, None], gv.shape), atol=1e-9)


def _rough_extrapolation_case(seed=3):
    wl = workloads.random_bubbles(meshes.voronoi_box_mesh(8, seed=seed), seed=seed, n_max=12, K=8, r_hi_h=3.0)
    geom = oracle.geometry(wl.mesh)
    rec = oracle.reconstruct(wl.mesh, wl.alpha, geom)
    grad, _ = oracle.grad(wl.mesh, geom, wl.T, wl.T_bface, wl.T_sat, wl.alpha)
    rng = np.random.default_rng(seed)
    grad = grad + rng.normal(size=grad.shape) * 5.0      # rough fields: nothing special about them
    return wl, geom, rec, grad


def test_extrapolation_keeps_own_phase_and_obeys_a_maximum_principle():
    """Each cell keeps its own phase's field (G_l in liquid, G_v in vapour)
    and cells outside the domain keep the gradient; the upwind update is a
    convex combination, so every extrapolated value lies within the range of
    the initial field on the domain."""
    wl, geom, rec, grad = _rough_extrapolation_case()
    gl, gv, sweeps, dom = oracle.extrapolate(wl.mesh, geom, wl.alpha, grad, rec["n"], rec["A"])
    liq = wl.alpha >= 0.5
    np.testing.assert_array_equal(gl[:, liq], grad[:, liq])
    np.testing.assert_array_equal(gv[:, ~liq], grad[:, ~liq])
    np.testing.assert_array_equal(gl[:, ~dom], grad[:, ~dom])
    np.testing.assert_array_equal(gv[:, ~dom], grad[:, ~dom])
    for d in range(3):
        lo, hi = grad[d, dom].min(), grad[d, dom].max()
        for g in (gl, gv):
            assert g[d, dom].min() >= lo - 1e-12 and g[d, dom].max() <= hi + 1e-12
    assert 1 <= sweeps <= 120
    # the domain holds the mixed cells and two layers of face neighbours
    mixed = (wl.alpha > 1e-8) & (wl.alpha < 1 - 1e-8)
    assert dom[mixed].all() and dom.sum() > mixed.sum()


def test_extrapolation_phase_swap():
    """alpha -> 1 - alpha flips every normal and swaps the phases, leaving
    the advection velocity sgn(alpha - 1/2) n unchanged: the liquid and vapour
    fields trade places (cells at alpha = 1/2 exactly are excluded by the
    tie rule)."""
    wl, geom, rec, grad = _rough_extrapolation_case(seed=5)
    wl.alpha[wl.alpha == 0.5] += 1e-6          # keep every cell off the tie
    rec = oracle.reconstruct(wl.mesh, wl.alpha, geom)
    gl, gv, s1, dom = oracle.extrapolate(wl.mesh, geom, wl.alpha, grad, rec["n"], rec["A"], tol=1e-9)
    gl2, gv2, s2, dom2 = oracle.extrapolate(wl.mesh, geom, 1.0 - wl.alpha, grad, -rec["n"], rec["A"], tol=1e-9)
    np.testing.assert_array_equal(dom, dom2)
    scale = np.abs(grad).max()
    np.testing.assert_allclose(gl2, gv, atol=1e-9 * scale)
    np.testing.assert_allclose(gv2, gl, atol=1e-9 * scale)


# ------------------------------------------- interface heat transfer (Robin)
def _column_case(axis, frac, liquid_high, shear=0.0):
    """Hex 8^3 with a plane normal to `axis` inside the cells of index 4
    along it, at fraction `frac` of the cell from its low side; liquid above
    the plane when liquid_high.  shear != 0 (axis 1 only) moves every vertex
    by shear*y along x: the cells become parallelepipeds whose y-faces keep
    the normal e_y while the centre connections across them tilt.  Returns
    mesh, geometry, alpha, the cell index along the axis, the exact interface
    arrays (A = h^2, n = +-e_axis in the cut cells) and h."""
    mesh = meshes.hex_mesh(8)
    if shear:
        assert axis == 1
        xyz = mesh.vert_xyz.copy()
        xyz[0] += shear * xyz[1]
        mesh = meshes.Mesh(**{**mesh.__dict__, "vert_xyz": xyz})
    geom = oracle.geometry(mesh)
    h = 1.0 / 8
    idx = np.floor(geom.xc[axis] / h).astype(int)
    a_cut = 1.0 - frac if liquid_high else frac
    alpha = np.where(idx < 4, 0.0 if liquid_high else 1.0, 1.0 if liquid_high else 0.0)
    alpha[idx == 4] = a_cut
    N = mesh.n_cells
    n_int = np.zeros((3, N))
    n_int[axis, idx == 4] = 1.0 if liquid_high else -1.0
    A = np.where(idx == 4, h * h, 0.0)
    return mesh, geom, alpha, idx, n_int, A, h


@pytest.mark.parametrize("axis,frac,liquid_high,shear",
                         [(0, 0.3, True, 0.0), (1, 0.65, False, 0.0), (2, 0.45, True, 0.0), (1, 0.3, True, 0.4)])
def test_robin_coefficients_for_a_plane_parallel_to_the_faces(axis, frac, liquid_high, shear):
    """A plane parallel to the faces through the cells of index 4: the only
    detached faces are the h^2 faces between index 3 and 4 (when the cut
    cell holds more than half of the phase of index 5) or between 4 and 5
    (otherwise); their projected interface area is h^2, and the alpha-
    interpolated crossing lies at 1/(2|alpha_cut - alpha_far|) of the centre
    distance from the far-phase cell, so its normal distance from each centre
    is that fraction of h (on the sheared mesh too, where the centre
    connection is longer than h).  Checked against these closed forms, face
    by face, with the conductivities of each side's phase, for exact
    interface arrays and (unsheared) for the oracle's own reconstruction."""
    mesh, geom, alpha, idx, n_int, A, h = _column_case(axis, frac, liquid_high, shear)
    k_l, k_v = 0.68, 0.025
    a_cut = alpha[idx == 4][0]
    lo_alpha = alpha[idx == 3][0]
    # the detached interface sits between index 3 and 4 when the cut cell is
    # on the other side of 1/2 from index 3, else between 4 and 5
    pair = (3, 4) if (lo_alpha - 0.5) * (a_cut - 0.5) < 0 else (4, 5)
    far = pair[0] if pair[0] != 4 else pair[1]
    a_far = alpha[idx == far][0]
    t_far = 0.5 / abs(a_cut - a_far)          # from the far cell's centre, in units of h
    cases = [(n_int, A, 1e-13)]
    if not shear:
        rec = oracle.reconstruct(mesh, alpha, geom)
        np.testing.assert_allclose(rec["A"][idx == 4], h * h, rtol=1e-12)
        cases.append((rec["n"], rec["A"], 1e-11))
    else:
        # the connection across a y-face is longer than h: a plain distance
        # would differ from the normal distance by this factor
        assert np.sqrt(1 + shear ** 2) > 1.05
    Smag = np.sqrt((geom.Sf ** 2).sum(0))
    along = np.abs(geom.Sf[axis]) > (1 - 1e-12) * Smag      # faces normal to the axis
    for nn, AA, tol in cases:
        r = oracle.robin(mesh, geom, alpha, nn, AA, k_l, k_v)
        o, q = mesh.face_owner, mesh.face_neigh
        io, iq = idx[o], np.where(q >= 0, idx[np.maximum(q, 0)], -1)
        expect = (q >= 0) & along & (np.minimum(io, iq) == pair[0]) & (np.maximum(io, iq) == pair[1])
        np.testing.assert_array_equal(r["crossing"], expect)
        f = np.nonzero(expect)[0]
        assert len(f) == 64
        np.testing.assert_allclose(r["area_face"][f], h * h, rtol=tol)
        for side, cells in ((0, o[f]), (1, q[f])):
            is_far = idx[cells] == far
            d_exp = np.where(is_far, t_far, 1.0 - t_far) * h
            k = np.where(alpha[cells] >= 0.5, k_l, k_v)
            np.testing.assert_allclose(r["d_face"][side, f], d_exp, rtol=1e-12)
            np.testing.assert_allclose(r["a_face"][side, f], k * h * h / d_exp, rtol=tol)
        assert not r["a_face"][:, ~expect].any() and not r["area_face"][~expect].any()
        # per cell: the sum over its detached faces (one each here)
        a_exp = np.zeros(mesh.n_cells)
        np.add.at(a_exp, o[f], r["a_face"][0, f])
        np.add.at(a_exp, q[f], r["a_face"][1, f])
        np.testing.assert_allclose(r["a_cell"], a_exp, rtol=1e-14)


def test_robin_no_face_is_detached_at_alpha_one_half():
    """A cut cell at alpha = 1/2 exactly is on neither side: the crossing
    test is strict, so no face is detached and every coefficient is 0."""
    mesh, geom, alpha, idx, n_int, A, h = _column_case(2, 0.5, True)
    r = oracle.robin(mesh, geom, alpha, n_int, A, 0.68, 0.025)
    assert not r["crossing"].any() and not r["a_cell"].any() and not r["a_face"].any()


def test_robin_coefficients_phase_swap_and_rigid_motion():
    """alpha -> 1-alpha with n -> -n and k_l <-> k_v leaves every
    coefficient unchanged; so does a rotation plus translation of the mesh
    with the normals rotated."""
    wl = workloads.random_bubbles(meshes.voronoi_box_mesh(8, seed=9), seed=9, n_max=12, K=8, r_hi_h=3.0)
    wl.alpha[wl.alpha == 0.5] += 1e-6
    geom = oracle.geometry(wl.mesh)
    rec = oracle.reconstruct(wl.mesh, wl.alpha, geom)
    r0 = oracle.robin(wl.mesh, geom, wl.alpha, rec["n"], rec["A"], 0.68, 0.025)
    assert r0["crossing"].sum() > 50 and (r0["a_face"][:, r0["crossing"]] > 0).mean() > 0.9
    r1 = oracle.robin(wl.mesh, geom, 1.0 - wl.alpha, -rec["n"], rec["A"], 0.025, 0.68)
    np.testing.assert_array_equal(r1["crossing"], r0["crossing"])
    for k in ("a_cell", "a_face", "d_face", "area_face"):
        np.testing.assert_allclose(r1[k], r0[k], rtol=1e-9, atol=0)
    rng = np.random.default_rng(10)
    Qm, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Qm) < 0:
        Qm[:, 0] *= -1
    t = rng.normal(size=3)
    m2 = meshes.Mesh(**{**wl.mesh.__dict__, "vert_xyz": Qm @ wl.mesh.vert_xyz + t[:, None]})
    g2 = oracle.geometry(m2)
    r2 = oracle.robin(m2, g2, wl.alpha, Qm @ rec["n"], rec["A"], 0.68, 0.025)
    np.testing.assert_array_equal(r2["crossing"], r0["crossing"])
    scale = {k: np.abs(r0[k]).max() for k in ("a_cell", "a_face", "d_face", "area_face")}
    for k in scale:
        np.testing.assert_allclose(r2[k], r0[k], atol=1e-9 * scale[k])


def test_reconstruction_of_a_cell_subset_equals_the_full_run(small_voronoi_wl):
    """Restricting the oracle to a list of cells (used for sampled checks on
    meshes too large to reconstruct whole) changes nothing on those cells."""
    wl = small_voronoi_wl
    geom = oracle.geometry(wl.mesh)
    full = oracle.reconstruct(wl.mesh, wl.alpha, geom)
    mixed = np.nonzero(full["status"] != oracle.NOT_MIXED)[0]
    pick = mixed[::7]
    part = oracle.reconstruct(wl.mesh, wl.alpha, geom, cells=pick)
    for k in ("s", "A", "d", "alpha_got", "status", "iters"):
        np.testing.assert_array_equal(part[k][pick], full[k][pick])
    np.testing.assert_array_equal(part["n"][:, pick], full["n"][:, pick])
    rest = np.setdiff1d(np.arange(wl.mesh.n_cells), pick)
    assert np.all(part["status"][rest] == -1)


def test_gradient_of_a_cell_subset_equals_the_full_run(small_voronoi_wl):
    """Restricting the oracle gradient to a list of cells (the band, in the
    CPU timing) changes nothing on those cells; the others are marked."""
    wl = small_voronoi_wl
    geom = oracle.geometry(wl.mesh)
    full, fst = oracle.grad(wl.mesh, geom, wl.T, wl.T_bface, wl.T_sat, wl.alpha)
    band = np.nonzero(oracle.band_mask(wl.mesh, wl.alpha))[0]
    part, pst = oracle.grad(wl.mesh, geom, wl.T, wl.T_bface, wl.T_sat, wl.alpha, cells=band)
    np.testing.assert_array_equal(part[:, band], full[:, band])
    np.testing.assert_array_equal(pst[band], fst[band])
    rest = np.setdiff1d(np.arange(wl.mesh.n_cells), band)
    assert np.all(pst[rest] == -1) and np.all(np.isnan(part[:, rest]))


@pytest.mark.parametrize("n_sides,fan", [(5, False), (24, False), (64, False), (80, True)])
def test_prismatoid_horizontal_cut_matches_the_cross_section_integral(n_sides, fan):
    """Cells bounded by two parallel regular n-gons (faces with up to 64
    vertices, the large-cell sizes) cut by the field phi = z: the liquid part
    (phi >= s) is the part above the plane z = s, whose volume is the
    integral of the cross-section area, a regular n-gon of radius varying
    linearly in z (the sideways shift of the rings does not change it); the
    interface is that cross-section, with the normal +z (with fan caps the
    cut crosses all 80 side faces: one iso-loop of 80 chords)."""
    mesh = meshes.prism_column(n_sides, 3, radius=0.4, height=0.9, shear=0.25, taper=0.2, fan_caps=fan)
    om = oracle.OMesh(mesh)
    geom = oracle.geometry(om)
    phi = mesh.vert_xyz[2].copy()
    an = 0.5 * n_sides * np.sin(2 * np.pi / n_sides)    # area of the unit-radius n-gon
    h = 0.9 / 3
    for P in range(3):
        z0, z1 = P * h, (P + 1) * h
        r0 = 0.4 * (1 + 0.2 * np.sin(P))
        r1 = 0.4 * (1 + 0.2 * np.sin(P + 1))
        rad = lambda z: r0 + (r1 - r0) * (z - z0) / h  # noqa: E731
        # integral of an * r(z)^2 from s to z1, r linear: (r(s)^3 - r1^3) / (3 dr/dz) form
        def above(s):
            k = (r1 - r0) / h
            return an * (r1 ** 3 - rad(s) ** 3) / (3 * k) if abs(k) > 0 else an * r0 ** 2 * (z1 - s)
        assert geom.V[P] == pytest.approx(above(z0), rel=1e-13)
        for t in (0.1, 0.37, 0.5, 0.81):
            s = z0 + t * h
            res = oracle.cut_cell(om, P, geom.xc, phi, s)
            assert res["V"] == pytest.approx(above(s), rel=1e-12, abs=1e-15)
            assert res["A"] == pytest.approx(an * rad(s) ** 2, rel=1e-12)
            np.testing.assert_allclose(res["S"] / np.linalg.norm(res["S"]), [0, 0, 1], atol=1e-12)
            assert res["nloops"] == 1


def test_vertex_field_invariants():
    """The vertex field (the reading of the paper's vertex values: the
    inverse-distance average of the cells sharing the vertex): a constant
    fraction gives that constant; every vertex value is a convex
    combination of its cells' fractions (both up to the rounding of the
    normalised weights); on a uniform hexahedral mesh an
    interior vertex is equidistant from its eight cells, so its value is
    their plain mean, and the plain-mean mode gives the same there.  These
    fix the set of cells and the normalisation; the inverse-distance weight
    itself is the reading of the silent paper, with no reference beyond its
    definition."""
    rng = np.random.default_rng(17)
    vm = meshes.voronoi_box_mesh(5, seed=4)
    om = oracle.OMesh(vm)
    geom = oracle.geometry(om)
    phi = oracle.vertex_field(om, geom.xc, np.full(vm.n_cells, 0.37))
    np.testing.assert_allclose(phi, 0.37, rtol=0, atol=1e-15)
    a = rng.uniform(0, 1, vm.n_cells)
    phi = oracle.vertex_field(om, geom.xc, a)
    # cells of each vertex
    lo = np.full(vm.n_verts, np.inf)
    hi = np.full(vm.n_verts, -np.inf)
    for P in range(vm.n_cells):
        ids = _cell_vertex_ids(vm, P)
        lo[ids] = np.minimum(lo[ids], a[P])
        hi[ids] = np.maximum(hi[ids], a[P])
    assert np.all(phi >= lo - 1e-15) and np.all(phi <= hi + 1e-15)
    n = 4
    hm = meshes.hex_mesh(n)
    omh = oracle.OMesh(hm)
    gh = oracle.geometry(omh)
    a = rng.uniform(0, 1, hm.n_cells)
    pi = oracle.vertex_field(omh, gh.xc, a)
    pm = oracle.vertex_field(omh, gh.xc, a, mode=1)
    m = n + 1
    for k in range(1, n):
        for j in range(1, n):
            for i in range(1, n):
                v = i + m * (j + m * k)
                cells = [(i - di) + n * ((j - dj) + n * (k - dk)) for di in (0, 1) for dj in (0, 1) for dk in (0, 1)]
                mean = np.mean(a[cells])
                assert abs(pi[v] - mean) < 1e-15 and abs(pm[v] - mean) < 1e-15
