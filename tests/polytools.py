"""Small single-cell meshes and independent geometry used by the oracle pins."""
import numpy as np
from scipy.spatial import ConvexHull

from synth.meshes import Mesh


def single_cell_mesh(points: np.ndarray, faces: list) -> Mesh:
    """One cell bounded by ``faces`` (vertex loops, counter-clockwise from outside)."""
    nf = len(faces)
    off = np.zeros(nf + 1, np.int64)
    off[1:] = np.cumsum([len(f) for f in faces])
    return Mesh(
        n_cells=1, n_faces=nf, n_verts=len(points),
        cell_face_off=np.array([0, nf], np.int64), cell_face=np.arange(nf, dtype=np.int32),
        face_vert_off=off, face_vert=np.concatenate(faces).astype(np.int32),
        face_owner=np.zeros(nf, np.int32), face_neigh=np.full(nf, -1, np.int32),
        face_bc=np.ones(nf, np.int8), vert_xyz=np.ascontiguousarray(np.asarray(points, float).T),
    )


def tet_mesh(P: np.ndarray) -> Mesh:
    P = np.asarray(P, float)
    if np.linalg.det(np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]])) < 0:
        P = P[[0, 2, 1, 3]]
    faces = [[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]]
    return single_cell_mesh(P, faces)


def hull_mesh(points: np.ndarray) -> Mesh:
    """Convex hull of random points as one cell with triangular faces."""
    h = ConvexHull(points)
    used = np.unique(h.simplices)
    remap = -np.ones(len(points), int)
    remap[used] = np.arange(len(used))
    P = points[used]
    faces = []
    for simp, eq in zip(h.simplices, h.equations):
        a, b, c = points[simp]
        if np.dot(np.cross(b - a, c - a), eq[:3]) < 0:
            simp = simp[[0, 2, 1]]
        faces.append(remap[simp])
    return single_cell_mesh(P, faces)


def below_unit_cube(m, a):
    """Volume of {x in [0,1]^3 : m.x <= a} for m > 0 (inclusion-exclusion over
    the cube's corners, the classical plane/cuboid relation)."""
    m = np.asarray(m, float)
    F = lambda y: max(y, 0.0) ** 3  # noqa: E731
    v = F(a) - F(a - m[0]) - F(a - m[1]) - F(a - m[2]) + F(a - m[0] - m[1]) + F(a - m[0] - m[2]) \
        + F(a - m[1] - m[2]) - F(a - m.sum())
    return v / (6.0 * m.prod())


def below_unit_cube_area(m, a):
    """Area of the plane m.x = a inside the unit cube (derivative of the volume
    relation times |m|)."""
    m = np.asarray(m, float)
    F = lambda y: max(y, 0.0) ** 2  # noqa: E731
    v = F(a) - F(a - m[0]) - F(a - m[1]) - F(a - m[2]) + F(a - m[0] - m[1]) + F(a - m[0] - m[2]) \
        + F(a - m[1] - m[2]) - F(a - m.sum())
    return v / (2.0 * m.prod()) * np.linalg.norm(m)


def tet_fraction_below(f, s):
    """Fraction of a tetrahedron where a linear field with vertex values f is <= s:
    sum_i (s - f_i)_+^3 / prod_{j != i} (f_j - f_i)."""
    f = np.asarray(f, float)
    tot = 0.0
    for i in range(4):
        den = np.prod([f[j] - f[i] for j in range(4) if j != i])
        tot += max(s - f[i], 0.0) ** 3 / den
    return tot


def clip_hull_volume_area(points, g, s):
    """Volume of conv(points) cut to g.x >= s and the area of the cut polygon,
    by an independent convex-hull construction."""
    h = ConvexHull(points)
    P = points[np.unique(h.simplices)]
    f = P @ g
    keep = P[f >= s]
    cuts = []
    for i in range(len(P)):
        for j in range(i + 1, len(P)):
            if (f[i] >= s) != (f[j] >= s):
                lam = (s - f[i]) / (f[j] - f[i])
                cuts.append(P[i] + lam * (P[j] - P[i]))
    cuts = np.array(cuts)
    # conv of kept vertices and all pairwise segment crossings (a superset of
    # the edge crossings that still lies in the clipped region)
    pts = np.concatenate([keep, cuts]) if len(keep) else cuts
    vol = ConvexHull(pts).volume if len(pts) >= 4 else 0.0
    n = g / np.linalg.norm(g)
    u = np.cross(n, [1.0, 0.0, 0.0] if abs(n[0]) < 0.9 else [0.0, 1.0, 0.0])
    u /= np.linalg.norm(u)
    w = np.cross(n, u)
    area = ConvexHull(np.stack([cuts @ u, cuts @ w], 1)).volume if len(cuts) >= 3 else 0.0
    return vol, area
