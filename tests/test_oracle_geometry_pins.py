"""Pins of the oracle's cell and face centroids, its inverse-distance vertex
values and its mass transfer rate, against values the mathematics fixes.

The cell centroid x_P is the centre of the least-squares stencil (App. B)
and the origin of the distance d; the face area centroid x_f is the virtual
neighbour of a boundary face (App. B).  Both are checked on shapes whose
centroid differs from the mean of their vertices, by constructions the oracle
does not use: closed forms of frusta and prisms, the shoelace centroid of
polygons, and a Delaunay tetrahedralisation of convex cells.  A vertex-mean
centroid fails every one of them.
"""
import numpy as np
import pytest
from scipy.spatial import ConvexHull, Delaunay

import oracle
from synth import meshes
from tests import polytools as pt


def _rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q *= np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _moved(mesh, R, t):
    """The mesh under the rigid motion x -> R x + t."""
    X = R @ mesh.vert_xyz + t[:, None]
    return pt.single_cell_mesh(X.T, [mesh.face_vert[mesh.face_vert_off[f]:mesh.face_vert_off[f + 1]]
                                     for f in range(mesh.n_faces)])


def _frustum(a, b, h, dx, dy):
    """Square frustum: side a at z = 0 centred on the z axis, side b at z = h
    centred at (dx, dy, h).  Side faces are trapezoids (their top and bottom
    edges are parallel), so every face is planar."""
    lo = [(-a / 2, -a / 2, 0.0), (a / 2, -a / 2, 0.0), (a / 2, a / 2, 0.0), (-a / 2, a / 2, 0.0)]
    hi = [(dx - b / 2, dy - b / 2, h), (dx + b / 2, dy - b / 2, h), (dx + b / 2, dy + b / 2, h),
          (dx - b / 2, dy + b / 2, h)]
    faces = [[0, 3, 2, 1], [4, 5, 6, 7], [0, 1, 5, 4], [1, 2, 6, 5], [2, 3, 7, 6], [3, 0, 4, 7]]
    return pt.single_cell_mesh(np.array(lo + hi), faces)


@pytest.mark.parametrize("a,b,dx,dy", [(1.0, 0.4, 0.0, 0.0), (0.6, 1.3, 0.25, -0.4), (1.0, 0.05, -0.3, 0.2)])
def test_frustum_volume_and_centroid_closed_form(a, b, dx, dy):
    """V = h (a^2 + ab + b^2)/3; the cross-section at height z is a square
    centred at (dx, dy) z/h, so the centroid is (dx, dy, h) zc/h with
    zc = h (a^2 + 2ab + 3b^2) / (4 (a^2 + ab + b^2)).  The vertex mean sits
    at h/2, which differs whenever a != b."""
    h = 0.7
    V = h * (a * a + a * b + b * b) / 3.0
    zc = h * (a * a + 2 * a * b + 3 * b * b) / (4.0 * (a * a + a * b + b * b))
    c = np.array([dx * zc / h, dy * zc / h, zc])
    rng = np.random.default_rng(int(100 * (a + b)))
    for _ in range(4):
        R, t = _rotation(rng), rng.normal(size=3)
        mesh = _moved(_frustum(a, b, h, dx, dy), R, t)
        geom = oracle.geometry(mesh)
        assert geom.V[0] == pytest.approx(V, rel=1e-13)
        np.testing.assert_allclose(geom.xc[:, 0], R @ c + t, rtol=0, atol=1e-13)
        vmean = mesh.vert_xyz.mean(1)
        assert np.linalg.norm(vmean - (R @ c + t)) > 1e-3   # the pin separates the two


def _convex_polygon(rng, n):
    """Counter-clockwise convex polygon (2-D) from the hull of random points."""
    P = rng.normal(size=(n, 2)) * [1.0, 0.45] + [0.3, -0.2]
    hull = ConvexHull(P)
    return P[hull.vertices]          # scipy gives 2-D hull vertices counter-clockwise


def _shoelace(P):
    x, y = P[:, 0], P[:, 1]
    x1, y1 = np.roll(x, -1), np.roll(y, -1)
    cr = x * y1 - x1 * y
    A = 0.5 * cr.sum()
    return A, np.array([((x + x1) * cr).sum(), ((y + y1) * cr).sum()]) / (6.0 * A)


def _prism(poly, h, sx, sy):
    """Oblique prism over a counter-clockwise polygon: the bottom cap at z = 0,
    the top cap shifted by (sx, sy, h), side parallelograms."""
    n = len(poly)
    bot = np.c_[poly, np.zeros(n)]
    top = np.c_[poly + [sx, sy], np.full(n, h)]
    faces = [list(range(n - 1, -1, -1)), list(range(n, 2 * n))]
    faces += [[j, (j + 1) % n, n + (j + 1) % n, n + j] for j in range(n)]
    return pt.single_cell_mesh(np.concatenate([bot, top]), faces)


def test_face_and_cell_centroids_of_oblique_prisms():
    """Caps of a prism over an irregular convex polygon: |S_f| is the shoelace
    area and x_f the shoelace area centroid (shifted for the top cap); the cell
    is the polygon swept along (sx, sy, h), so V = A h and x_P = C + (sx, sy,
    h)/2.  A polygon with clustered vertices puts its vertex mean far from its
    area centroid."""
    rng = np.random.default_rng(23)
    for _ in range(12):
        poly = _convex_polygon(rng, int(rng.integers(8, 40)))
        A, C = _shoelace(poly)
        h, sx, sy = rng.uniform(0.2, 1.0), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5)
        R, t = _rotation(rng), rng.normal(size=3)
        mesh = _moved(_prism(poly, h, sx, sy), R, t)
        geom = oracle.geometry(mesh)
        scale = np.sqrt(A)
        # bottom cap (face 0) faces -z, top cap (face 1) +z
        np.testing.assert_allclose(geom.Sf[:, 0], R @ [0, 0, -A], rtol=0, atol=1e-13 * A)
        np.testing.assert_allclose(geom.Sf[:, 1], R @ [0, 0, A], rtol=0, atol=1e-13 * A)
        np.testing.assert_allclose(geom.xf[:, 0], R @ [C[0], C[1], 0.0] + t, rtol=0, atol=1e-13 * scale)
        np.testing.assert_allclose(geom.xf[:, 1], R @ [C[0] + sx, C[1] + sy, h] + t, rtol=0, atol=1e-13 * scale)
        assert geom.V[0] == pytest.approx(A * h, rel=1e-12)
        np.testing.assert_allclose(geom.xc[:, 0], R @ [C[0] + sx / 2, C[1] + sy / 2, h / 2] + t, rtol=0,
                                   atol=1e-12 * scale)
        vm2 = poly.mean(0)
        assert np.linalg.norm(vm2 - C) > 1e-4 * scale   # the polygon tells the two centres apart


def _cell_vertex_ids(mesh, P):
    fs = mesh.cell_face[mesh.cell_face_off[P]:mesh.cell_face_off[P + 1]]
    return np.unique(np.concatenate([mesh.face_vert[mesh.face_vert_off[f]:mesh.face_vert_off[f + 1]] for f in fs]))


def _delaunay_centroid(X):
    """Volume and centroid of conv(X) from a Delaunay tetrahedralisation."""
    tri = Delaunay(X)
    T = X[tri.simplices]                          # [nt, 4, 3]
    v = np.abs(np.einsum("ij,ij->i", T[:, 1] - T[:, 0], np.cross(T[:, 2] - T[:, 0], T[:, 3] - T[:, 0]))) / 6.0
    return v.sum(), (v[:, None] * T.mean(1)).sum(0) / v.sum()


def test_cell_centroids_by_independent_tetrahedralisation():
    """Convex cells (random triangulated hulls and box-clipped Voronoi cells):
    volume and centroid agree with a Delaunay tetrahedralisation of the cell's
    vertices, a decomposition that shares nothing with the oracle's fan about
    its vertex mean."""
    rng = np.random.default_rng(31)
    for _ in range(15):
        pts = rng.normal(size=(int(rng.integers(10, 40)), 3)) * [1.0, 0.5, 0.3]
        pts[: len(pts) // 3] *= 0.3            # cluster a third of the points
        mesh = pt.hull_mesh(pts)
        geom = oracle.geometry(mesh)
        V, c = _delaunay_centroid(mesh.vert_xyz.T)
        assert geom.V[0] == pytest.approx(V, rel=1e-12)
        np.testing.assert_allclose(geom.xc[:, 0], c, rtol=0, atol=1e-12)
    vm = meshes.voronoi_box_mesh(6, seed=12)
    geom = oracle.geometry(vm)
    far = 0.0
    for P in range(0, vm.n_cells, 7):
        X = vm.vert_xyz[:, _cell_vertex_ids(vm, P)].T
        V, c = _delaunay_centroid(X)
        assert geom.V[P] == pytest.approx(V, rel=1e-11)
        np.testing.assert_allclose(geom.xc[:, P], c, rtol=0, atol=1e-12 * vm.h)
        far = max(far, np.linalg.norm(X.mean(0) - c) / vm.h)
    assert far > 1e-2   # vertex means of these cells are visibly off their centroids


def test_voronoi_face_centroids_match_the_shoelace_formula():
    """Every face of a Voronoi mesh, projected to its own plane (Newell normal
    of the loop): the oracle's area vector and area centroid equal the
    shoelace area and centroid of the projected polygon."""
    vm = meshes.voronoi_box_mesh(5, seed=8)
    geom = oracle.geometry(vm)
    off = vm.face_vert_off
    far = 0.0
    for f in range(vm.n_faces):
        X = vm.vert_xyz[:, vm.face_vert[off[f]:off[f + 1]]].T
        nw = np.cross(X, np.roll(X, -1, 0)).sum(0)          # Newell: twice the area vector
        nh = nw / np.linalg.norm(nw)
        u = X[1] - X[0]
        u -= nh * (nh @ u)
        u /= np.linalg.norm(u)
        w = np.cross(nh, u)
        o = X[0]
        P2 = np.stack([(X - o) @ u, (X - o) @ w], 1)
        A, C = _shoelace(P2)
        assert A > 0
        np.testing.assert_allclose(geom.Sf[:, f], A * nh, rtol=0, atol=1e-13 * vm.h ** 2)
        xf = o + C[0] * u + C[1] * w + nh * ((X - o) @ nh).mean()
        np.testing.assert_allclose(geom.xf[:, f], xf, rtol=0, atol=1e-12 * vm.h)
        if len(X) > 3:
            far = max(far, np.linalg.norm(X.mean(0) - xf) / vm.h)
    assert far > 1e-2


def _graded_hex(n, power):
    """Tensor-product hexahedra of the unit cube with nodes (i/n)^power per axis."""
    m = meshes.hex_mesh(n)
    idx = np.rint(m.vert_xyz * n).astype(int)
    m.vert_xyz = (idx / n) ** power
    return m, (np.arange(n + 1) / n) ** power


@pytest.mark.parametrize("power", [1.6, 0.7])
def test_inverse_distance_vertex_value_on_a_graded_mesh(power):
    """On a graded tensor-product mesh an interior vertex (i, j, k) is shared
    by the eight boxes around it, whose centroids are the box midpoints; its
    value is sum_c alpha_c / |x_v - m_c| over sum_c 1/|x_v - m_c|, computed
    here by hand from the nodes.  The plain mean and 1/|r|^2 weights fail."""
    n = 5
    mesh, x = _graded_hex(n, power)
    om = oracle.OMesh(mesh)
    geom = oracle.geometry(om)
    rng = np.random.default_rng(7)
    a = rng.uniform(0, 1, mesh.n_cells)
    phi = oracle.vertex_field(om, geom.xc, a)
    phim = oracle.vertex_field(om, geom.xc, a, mode=1)
    m = n + 1
    worst_plain = worst_sq = 0.0
    for k in range(1, n):
        for j in range(1, n):
            for i in range(1, n):
                v = i + m * (j + m * k)
                xv = np.array([x[i], x[j], x[k]])
                num = den = num2 = den2 = 0.0
                vals = []
                for di in (0, 1):
                    for dj in (0, 1):
                        for dk in (0, 1):
                            ci, cj, ck = i - di, j - dj, k - dk
                            mid = 0.5 * np.array([x[ci] + x[ci + 1], x[cj] + x[cj + 1], x[ck] + x[ck + 1]])
                            al = a[ci + n * (cj + n * ck)]
                            dist = np.linalg.norm(xv - mid)
                            num += al / dist
                            den += 1.0 / dist
                            num2 += al / dist ** 2
                            den2 += 1.0 / dist ** 2
                            vals.append(al)
                assert phi[v] == pytest.approx(num / den, rel=0, abs=1e-14)
                assert phim[v] == pytest.approx(np.mean(vals), rel=0, abs=1e-15)
                worst_plain = max(worst_plain, abs(np.mean(vals) - num / den))
                worst_sq = max(worst_sq, abs(num2 / den2 - num / den))
    assert worst_plain > 1e-3 and worst_sq > 1e-3


@pytest.mark.parametrize("d_over_h", [0.3, 0.5, 0.7])
def test_mass_transfer_on_the_one_dimensional_setup(d_over_h):
    """App. C's one-dimensional configuration run through the whole oracle
    path (reconstruction, modified gradient, Eq. mass_transfer): alpha is
    linear in x across the liquid cell P and its vapour neighbour Q, so the
    vertex field depends on x alone and the volume-matched cut of P is the
    plane x = x_P + h/2 - alpha_P h with A_int = h^2, n = +x (vapour -> liquid)
    and d = alpha_P h - h/2; the x-gradient of P is Eq. g_fm, so
    mdot_P = k_l g_fm h^2 / (h_lv h^3) and Qdot = -mdot h_lv.  Q is vapour
    with T = T_sat on every stencil point: mdot_Q = 0.  Distinct k_l and k_v
    (water and steam, Table material_properties) catch a swapped phase."""
    n = 8
    mesh = meshes.hex_mesh(n)
    geom = oracle.geometry(mesh)
    h = mesh.h
    x = geom.xc[0]
    xP = (n // 2 + 0.5) * h
    d = d_over_h * h
    x_int = xP - d
    alpha = np.clip(0.5 + (0.4 / h) * (x - x_int), 0.0, 1.0)
    T_sat, dT, theta = 373.15, 2.0, 0.3
    T_far = T_sat + dT
    T = np.where(x > x_int, T_sat + dT * np.clip((x - x_int) / (h + d), 0, 1), T_sat)
    T = np.where(np.isclose(x, xP), T_sat + theta, T)
    T = np.where(np.isclose(x, xP + h), T_far, T)
    Tb = np.full(mesh.n_faces, T_sat)
    k_l, k_v, h_lv = 0.679, 0.025, 2.26e6
    rec = oracle.reconstruct(mesh, alpha, geom)
    grad, _ = oracle.grad(mesh, geom, T, Tb, T_sat, alpha, modified=True)
    mdot, Qdot = oracle.mass_transfer(geom, alpha, rec["n"], rec["A"], grad, k_l, k_v, h_lv)
    mid = (n // 2 + 0.5) * h
    col = np.isclose(geom.xc[1], mid) & np.isclose(geom.xc[2], mid)
    P = np.nonzero(col & np.isclose(x, xP))[0][0]
    Q = np.nonzero(col & np.isclose(x, xP - h))[0][0]
    aP = alpha[P]
    assert rec["status"][P] == oracle.OK and rec["status"][Q] == oracle.OK
    assert rec["A"][P] == pytest.approx(h * h, rel=1e-12)
    np.testing.assert_allclose(rec["n"][:, P], [1.0, 0.0, 0.0], atol=1e-12)
    assert rec["d"][P] == pytest.approx(aP * h - 0.5 * h, abs=1e-12 * h)
    g_fm = (theta * d + (T_far - T_sat - theta) * h) / (d * d + h * h)       # Eq. g_fm
    assert grad[0, P] == pytest.approx(g_fm, rel=1e-12)
    assert mdot[P] == pytest.approx(k_l * g_fm * h * h / (h_lv * h ** 3), rel=1e-12)
    assert Qdot[P] == pytest.approx(-k_l * g_fm * h * h / h ** 3, rel=1e-12)
    assert mdot[P] > 0                                                        # superheated liquid evaporates
    assert abs(mdot[Q]) <= 1e-12 * abs(mdot[P])
    # the two-sided form with the phase gradients given explicitly: a vapour
    # gradient G_v adds -k_v (G_v . n) A / (h_lv V)
    gv = np.zeros_like(grad)
    gv[0, P] = -3.0
    gl = np.where(alpha >= 0.5, grad, 0.0)
    m2, _ = oracle.mass_transfer(geom, alpha, rec["n"], rec["A"], grad, k_l, k_v, h_lv, gl=gl, gv=gv)
    assert m2[P] == pytest.approx((k_l * g_fm + 3.0 * k_v) * h * h / (h_lv * h ** 3), rel=1e-12)
