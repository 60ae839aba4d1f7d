"""The seeded mesh and field generators produce valid inputs."""
import numpy as np
import pytest

from synth import meshes, workloads


def _closed_and_oriented(m):
    """Every cell's outward loops use each directed edge once, with its reverse."""
    cfo = m.cell_face_off
    cells = np.repeat(np.arange(m.n_cells), np.diff(cfo))
    faces = m.cell_face.astype(np.int64)
    sz = np.diff(m.face_vert_off)[faces]
    owner_side = m.face_owner[faces] == cells
    a_list, b_list, c_list = [], [], []
    for f_i, (f, n, own, P) in enumerate(zip(faces, sz, owner_side, cells)):
        lp = m.face_vert[m.face_vert_off[f]:m.face_vert_off[f] + n]
        if not own:
            lp = lp[::-1]
        a_list.append(lp)
        b_list.append(np.roll(lp, -1))
        c_list.append(np.full(n, P))
    a = np.concatenate(a_list).astype(np.int64)
    b = np.concatenate(b_list).astype(np.int64)
    c = np.concatenate(c_list).astype(np.int64)
    NV = m.n_verts
    fwd = (c * NV + a) * NV + b
    rev = (c * NV + b) * NV + a
    assert len(np.unique(fwd)) == len(fwd), "a directed edge repeats within a cell"
    assert np.all(np.isin(rev, fwd)), "a cell surface is not closed"


def test_hex_mesh_is_closed():
    m = meshes.hex_mesh(5)
    _closed_and_oriented(m)
    assert m.n_faces == 3 * 5 * 5 * 6


@pytest.mark.parametrize("n,seed", [(6, 1), (12, 7)])
def test_voronoi_mesh_is_closed_and_fills_the_box(n, seed):
    import oracle
    m = meshes.voronoi_box_mesh(n, seed)
    _closed_and_oriented(m)
    g = oracle.geometry(m)
    assert g.V.sum() == pytest.approx(1.0, rel=1e-12)
    assert np.all(g.V > 0)
    nf = np.diff(m.cell_face_off)
    assert 12.0 < nf.mean() < 16.0


def test_bench_sized_voronoi_mesh_is_closed():
    m = meshes.voronoi_box_mesh(46, 2)
    assert m.n_cells == 194672
    _closed_and_oriented(m)


def test_alpha_fractions_match_the_sphere_volume():
    wl = workloads.hex_sphere()
    vap = (1 - wl.alpha).sum() / wl.mesh.n_cells
    assert vap == pytest.approx(4 / 3 * np.pi * 0.3 ** 3, rel=1e-4)
    assert 400 < wl.n_mixed < 440


def test_host_concat_is_the_disjoint_union():
    """Oracle geometry of the host-side union equals the parts' geometry laid
    end to end (so batch tests compare against the right reference)."""
    import oracle
    from synth import meshes
    parts = [meshes.hex_mesh(4), meshes.voronoi_box_mesh(4, seed=3)]
    whole = meshes.concat(parts)
    gw = oracle.geometry(whole)
    gp = [oracle.geometry(p) for p in parts]
    np.testing.assert_array_equal(gw.V, np.concatenate([g.V for g in gp]))
    np.testing.assert_array_equal(gw.xc, np.concatenate([g.xc for g in gp], 1))
    np.testing.assert_array_equal(gw.Sf, np.concatenate([g.Sf for g in gp], 1))
    assert whole.n_cells == sum(p.n_cells for p in parts)
    assert np.all(whole.face_owner[parts[0].n_faces:] >= parts[0].n_cells)


@pytest.mark.parametrize("n_sides,fan", [(4, False), (24, False), (64, False), (40, True)])
def test_prism_columns_are_closed_outward_polyhedra(n_sides, fan):
    """Every cell of a prismatoid column is closed (its outward face area
    vectors sum to zero) and every face is planar, and the caps are shared
    by consecutive cells."""
    m = meshes.prism_column(n_sides, 5, fan_caps=fan)
    X = m.vert_xyz
    S = np.zeros((m.n_faces, 3))
    for f in range(m.n_faces):
        v = m.face_vert[m.face_vert_off[f]:m.face_vert_off[f + 1]]
        p = X[:, v].T
        c = p.mean(0)
        for a in range(len(v)):
            S[f] += 0.5 * np.cross(p[a] - c, p[(a + 1) % len(v)] - c)
        nrm = S[f] / np.linalg.norm(S[f])
        assert np.abs((p - c) @ nrm).max() < 1e-12       # planar
    for P in range(m.n_cells):
        tot = np.zeros(3)
        for f in m.cell_face[m.cell_face_off[P]:m.cell_face_off[P + 1]]:
            tot += S[f] if m.face_owner[f] == P else -S[f]
        assert np.abs(tot).max() < 1e-13
    inner = m.face_neigh >= 0
    assert np.all(m.face_neigh[inner] == m.face_owner[inner] + 1)
    assert inner.sum() == (m.n_cells - 1) * (n_sides if fan else 1)


def _cell_geometry_by_seed(m):
    import oracle
    g = oracle.geometry(m)
    order = np.lexsort(m.seeds.T[::-1])
    return g.V[order], g.xc[:, order], np.diff(m.cell_face_off)[order]


@pytest.mark.parametrize("n,seed", [(5, 9), (9, 4)])
def test_native_voronoi_equals_qhull(n, seed):
    """The native construction (cells clipped by bisectors) and scipy's Qhull
    (mirror seeds) give the same box-clipped cells: counts, faces per cell,
    volumes and centroids per seed."""
    a = meshes.voronoi_box_mesh(n, seed)
    b = meshes.voronoi_box_mesh(n, seed, engine="qhull")
    assert (a.n_cells, a.n_faces, a.n_verts) == (b.n_cells, b.n_faces, b.n_verts)
    Va, xa, fa = _cell_geometry_by_seed(a)
    Vb, xb, fb = _cell_geometry_by_seed(b)
    np.testing.assert_array_equal(fa, fb)
    np.testing.assert_allclose(Va, Vb, rtol=1e-11, atol=0)
    np.testing.assert_allclose(xa, xb, rtol=0, atol=1e-13)
    _closed_and_oriented(a)


def test_native_pipe_equals_qhull():
    """The pipe (kept seeds r <= R, dropped neighbours give boundary faces)."""
    a = meshes.voronoi_pipe_mesh(8, 1.0, 52.0 / 9.5, 4)
    b = meshes.voronoi_pipe_mesh(8, 1.0, 52.0 / 9.5, 4, engine="qhull")
    assert (a.n_cells, a.n_faces, a.n_verts) == (b.n_cells, b.n_faces, b.n_verts)
    assert np.sum(a.face_neigh < 0) == np.sum(b.face_neigh < 0)
    Va, xa, fa = _cell_geometry_by_seed(a)
    Vb, xb, fb = _cell_geometry_by_seed(b)
    np.testing.assert_array_equal(fa, fb)
    np.testing.assert_allclose(Va, Vb, rtol=1e-11, atol=0)
    np.testing.assert_allclose(xa, xb, rtol=0, atol=1e-13)
    _closed_and_oriented(a)


def test_native_face_planes_hold_their_vertices():
    """Every face's half-space n.x <= c (owner side) passes through the face's
    vertices, and the owner's seed lies inside it."""
    m = meshes.voronoi_pipe_mesh(6, 1.0, 52.0 / 9.5, 5)
    fp = m.extra["face_plane"]
    fid = np.repeat(np.arange(m.n_faces), np.diff(m.face_vert_off))
    X = m.vert_xyz[:, m.face_vert].T
    nrm = np.linalg.norm(fp[:, :3], axis=1)
    res = (np.einsum("ij,ij->i", X, fp[fid, :3]) - fp[fid, 3]) / nrm[fid]
    assert np.abs(res).max() < 1e-12
    own = m.seeds[m.face_owner]
    assert np.all(np.einsum("ij,ij->i", own, fp[:, :3]) < fp[:, 3])
