"""Mesh generators: uniform hexahedra and box-clipped jittered-BCC Voronoi cells.

Every mesh is returned in the CSR form the library and the oracle both take:

* ``cell_face_off[N+1]`` (int64), ``cell_face`` (int32): faces of each cell;
* ``face_vert_off[NF+1]`` (int64), ``face_vert`` (int32): the vertex loop of
  each face, ordered counter-clockwise seen from outside the owner cell, so the
  right-hand normal points from the owner into the neighbour;
* ``face_owner``/``face_neigh`` (int32, neighbour -1 on the boundary) and
  ``face_bc`` (int8: 0 interior, 1 boundary value, 2 symmetry);
* ``vert_xyz[3][NV]`` (float64, structure of arrays).

The Voronoi mesh stands in for the dualised GMSH polyhedra of the paper's
polyhedral runs (Sec. 3.3), which are not available: a body-centred cubic
lattice jittered by +-0.3 h_eff per coordinate gives about 14 faces per cell.
Two constructions give the same cells: a native one (``_voronoi.c``: each
cell is the box clipped by the bisectors of its nearest seeds, OpenMP over
cells; millions of cells in seconds), the default, and scipy's Qhull with
mirror seeds (the Voronoi cell of a seed among the seeds and their
reflections in the six box planes is exactly the box-clipped cell, because a
reflected seed is never nearer than its original to a point of the box),
kept to cross-check the native one.
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess
from dataclasses import dataclass, field
from functools import lru_cache

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_VSRC = os.path.join(_HERE, "_voronoi.c")
_VSO = os.path.join(_HERE, "_voronoi.so")


@dataclass
class Mesh:
    n_cells: int
    n_faces: int
    n_verts: int
    cell_face_off: np.ndarray
    cell_face: np.ndarray
    face_vert_off: np.ndarray
    face_vert: np.ndarray
    face_owner: np.ndarray
    face_neigh: np.ndarray
    face_bc: np.ndarray
    vert_xyz: np.ndarray          # [3, NV] float64
    kind: str = "poly"
    h: float = 0.0                # nominal cell size
    seeds: np.ndarray | None = None   # [N, 3] generating points (Voronoi)
    extra: dict = field(default_factory=dict)

    # ---- cheap helpers used only to place input fields ----------------
    # (each is computed once per mesh and kept in `extra` under a "_" key:
    # meshes are not modified after construction)
    def _cached(self, key, fn):
        if key not in self.extra:
            self.extra[key] = fn()
        return self.extra[key]

    def cell_vertex_mean(self) -> np.ndarray:
        return self._cached("_cell_vertex_mean", self._cell_vertex_mean)

    def face_vertex_mean(self) -> np.ndarray:
        return self._cached("_face_vertex_mean", self._face_vertex_mean)

    def cell_bbox(self) -> np.ndarray:
        return self._cached("_cell_bbox", self._cell_bbox)

    def _cell_vertex_mean(self) -> np.ndarray:
        """Mean of the distinct vertices of each cell, [N, 3].

        Used only to evaluate synthetic input profiles (temperature); the
        method's own cell centroid is computed by the library and the oracle.
        """
        N = self.n_cells
        fv_cnt = np.diff(self.face_vert_off)
        cf_cnt = np.diff(self.cell_face_off)
        cell_of_slot = np.repeat(np.arange(N), cf_cnt)
        faces = self.cell_face.astype(np.int64)
        # (cell, vertex) pairs over all faces of each cell, then unique
        rep = fv_cnt[faces]
        cells = np.repeat(cell_of_slot, rep)
        starts = self.face_vert_off[faces]
        idx = np.repeat(starts - np.cumsum(np.r_[0, rep[:-1]]), rep) + np.arange(rep.sum())
        verts = self.face_vert[idx].astype(np.int64)
        key = np.unique(cells * self.n_verts + verts)
        c = key // self.n_verts
        v = key % self.n_verts
        cnt = np.bincount(c, minlength=N).astype(np.float64)
        out = np.empty((N, 3))
        for a in range(3):
            out[:, a] = np.bincount(c, weights=self.vert_xyz[a, v], minlength=N) / cnt
        return out

    def _face_vertex_mean(self) -> np.ndarray:
        """Mean of each face's vertices, [NF, 3] (input-profile placement only)."""
        cnt = np.diff(self.face_vert_off)
        fid = np.repeat(np.arange(self.n_faces), cnt)
        out = np.empty((self.n_faces, 3))
        for a in range(3):
            out[:, a] = np.bincount(fid, weights=self.vert_xyz[a, self.face_vert], minlength=self.n_faces) / cnt
        return out

    def _cell_bbox(self) -> np.ndarray:
        """Axis-aligned bounding box of each cell, [N, 6] = (lo xyz, hi xyz)."""
        N = self.n_cells
        cf_cnt = np.diff(self.cell_face_off)
        faces = self.cell_face.astype(np.int64)
        rep = np.diff(self.face_vert_off)[faces]
        starts = self.face_vert_off[faces]
        idx = np.repeat(starts - np.cumsum(np.r_[0, rep[:-1]]), rep) + np.arange(rep.sum())
        verts = self.face_vert[idx]
        # the incidences run cell by cell: one segment reduction per axis
        per_cell = np.bincount(np.repeat(np.arange(N), cf_cnt), weights=rep, minlength=N).astype(np.int64)
        seg = np.r_[0, np.cumsum(per_cell)[:-1]]
        out = np.empty((N, 6))
        for a in range(3):
            x = self.vert_xyz[a, verts]
            out[:, a] = np.minimum.reduceat(x, seg)
            out[:, 3 + a] = np.maximum.reduceat(x, seg)
        return out

    def face_neighbours(self) -> tuple[np.ndarray, np.ndarray]:
        """CSR (off, nbr) of interior face neighbours per cell."""
        N = self.n_cells
        interior = self.face_neigh >= 0
        o = self.face_owner[interior]
        n = self.face_neigh[interior]
        a = np.concatenate([o, n])
        b = np.concatenate([n, o])
        order = np.argsort(a, kind="stable")
        off = np.zeros(N + 1, np.int64)
        np.cumsum(np.bincount(a, minlength=N), out=off[1:])
        return off, b[order].astype(np.int32)


def _cell_face_csr(n_cells: int, owner: np.ndarray, neigh: np.ndarray):
    nf = len(owner)
    fid = np.arange(nf, dtype=np.int64)
    inner = neigh >= 0
    cells = np.concatenate([owner, neigh[inner]]).astype(np.int64)
    faces = np.concatenate([fid, fid[inner]])
    order = np.lexsort((faces, cells))
    off = np.zeros(n_cells + 1, np.int64)
    np.cumsum(np.bincount(cells, minlength=n_cells), out=off[1:])
    return off, faces[order].astype(np.int32)


def hex_mesh(n: int, length: float = 1.0, origin=(0.0, 0.0, 0.0)) -> Mesh:
    """Uniform n^3 hexahedral mesh of the cube [origin, origin+length]^3."""
    h = length / n
    m = n + 1
    ii, jj, kk = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    vid = lambda i, j, k: i + m * (j + m * k)  # noqa: E731
    cid = lambda i, j, k: i + n * (j + n * k)  # noqa: E731
    xyz = np.empty((3, m ** 3))
    xyz[0, vid(ii, jj, kk).ravel()] = origin[0] + ii.ravel() * h
    xyz[1, vid(ii, jj, kk).ravel()] = origin[1] + jj.ravel() * h
    xyz[2, vid(ii, jj, kk).ravel()] = origin[2] + kk.ravel() * h

    loops, owners, neighs = [], [], []
    a, b = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    a = a.ravel()
    b = b.ravel()
    for axis in range(3):
        for p in range(n + 1):
            # (u, w) are the two in-plane axes in right-handed order
            if axis == 0:   # normal +x, loop in (y, z)
                v0 = vid(p, a, b); v1 = vid(p, a + 1, b); v2 = vid(p, a + 1, b + 1); v3 = vid(p, a, b + 1)
                lo = cid(p - 1, a, b); hi = cid(p, a, b)
            elif axis == 1:  # normal +y, loop in (z, x): a->z, b->x
                v0 = vid(b, p, a); v1 = vid(b, p, a + 1); v2 = vid(b + 1, p, a + 1); v3 = vid(b + 1, p, a)
                lo = cid(b, p - 1, a); hi = cid(b, p, a)
            else:            # normal +z, loop in (x, y)
                v0 = vid(a, b, p); v1 = vid(a + 1, b, p); v2 = vid(a + 1, b + 1, p); v3 = vid(a, b + 1, p)
                lo = cid(a, b, p - 1); hi = cid(a, b, p)
            lp = np.stack([v0, v1, v2, v3], 1)
            if p == 0:        # boundary, owner is the cell above, normal must flip
                loops.append(lp[:, ::-1]); owners.append(hi); neighs.append(np.full(n * n, -1))
            elif p == n:
                loops.append(lp); owners.append(lo); neighs.append(np.full(n * n, -1))
            else:
                loops.append(lp); owners.append(lo); neighs.append(hi)
    fv = np.concatenate(loops).astype(np.int32)
    owner = np.concatenate(owners).astype(np.int32)
    neigh = np.concatenate(neighs).astype(np.int32)
    nf = len(owner)
    cfo, cf = _cell_face_csr(n ** 3, owner, neigh)
    return Mesh(
        n_cells=n ** 3, n_faces=nf, n_verts=m ** 3,
        cell_face_off=cfo, cell_face=cf,
        face_vert_off=np.arange(0, 4 * nf + 1, 4, dtype=np.int64), face_vert=fv.ravel(),
        face_owner=owner, face_neigh=neigh, face_bc=(neigh < 0).astype(np.int8),
        vert_xyz=xyz, kind="hex", h=h,
    )


def prism_column(n_sides: int, n_layers: int, radius: float = 0.5, height: float = 1.0, shear: float = 0.3,
                 taper: float = 0.1, origin=(0.0, 0.0, 0.0), fan_caps: bool = False) -> Mesh:
    """A column of n_layers cells, each the convex hull of two parallel
    regular n_sides-gons (ring k at height k h, radius radius (1 + taper
    sin k), centre shifted in x by shear k h): cells with 2 n_sides vertices,
    n_sides + 2 faces and n_sides-gon faces, for the large-cell kernel
    variants.  Side faces are planar trapezoids; all of them and the two end
    caps are boundary faces.  fan_caps: every cap is split into n_sides
    triangles around the ring centre (an extra vertex per ring), so a cell
    has 3 n_sides faces of at most four vertices and a cut across the column
    crosses every side face."""
    n, L = n_sides, n_layers
    h = height / L
    ang = 2.0 * np.pi * np.arange(n) / n
    nr = n + 1 if fan_caps else n            # vertices per ring (centre last)
    xyz = np.empty((3, (L + 1) * nr))
    for k in range(L + 1):
        r = radius * (1.0 + taper * np.sin(k))
        cx = origin[0] + shear * k * h
        xyz[0, k * nr:k * nr + n] = cx + r * np.cos(ang)
        xyz[1, k * nr:k * nr + n] = origin[1] + r * np.sin(ang)
        xyz[2, k * nr:(k + 1) * nr] = origin[2] + k * h
        if fan_caps:
            xyz[0, k * nr + n] = cx
            xyz[1, k * nr + n] = origin[1]
    ring = lambda k: k * nr + np.arange(n)  # noqa: E731
    loops, owners, neighs = [], [], []

    def cap(k, own, nb, up):
        # ring k, normal +z when up (counter-clockwise seen from +z)
        if fan_caps:
            c = k * nr + n
            for j in range(n):
                tri = np.array([c, k * nr + j, k * nr + (j + 1) % n])
                loops.append(tri if up else tri[::-1]); owners.append(own); neighs.append(nb)
        else:
            loops.append(ring(k) if up else ring(k)[::-1]); owners.append(own); neighs.append(nb)

    # caps: ring k between cell k-1 (owner, below) and cell k
    cap(0, 0, -1, False)
    for k in range(1, L):
        cap(k, k - 1, k, True)
    cap(L, L - 1, -1, True)
    # side trapezoids, outward: (k, j) -> (k, j+1) -> (k+1, j+1) -> (k+1, j)
    for k in range(L):
        for j in range(n):
            j1 = (j + 1) % n
            loops.append(np.array([k * nr + j, k * nr + j1, (k + 1) * nr + j1, (k + 1) * nr + j]))
            owners.append(k); neighs.append(-1)
    fvo = np.zeros(len(loops) + 1, np.int64)
    np.cumsum([len(lp) for lp in loops], out=fvo[1:])
    owner = np.array(owners, np.int32)
    neigh = np.array(neighs, np.int32)
    cfo, cf = _cell_face_csr(L, owner, neigh)
    return Mesh(
        n_cells=L, n_faces=len(loops), n_verts=(L + 1) * nr,
        cell_face_off=cfo, cell_face=cf,
        face_vert_off=fvo, face_vert=np.concatenate(loops).astype(np.int32),
        face_owner=owner, face_neigh=neigh, face_bc=(neigh < 0).astype(np.int8),
        vert_xyz=xyz, kind="prism", h=h,
    )


def bcc_seeds(n, rng: np.random.Generator, jitter: float = 0.3,
              lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Two interleaved lattices (BCC) of n[0]*n[1]*n[2] points each in [lo, hi],
    jittered uniformly by +-jitter*h_eff per coordinate (h_eff = (V/N)^(1/3))."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    n = np.broadcast_to(np.asarray(n, np.int64), (3,))
    span = hi - lo
    h = span / n
    g = [lo[a] + (np.arange(n[a]) + 0.25) * h[a] for a in range(3)]
    a = np.stack(np.meshgrid(*g, indexing="ij"), -1).reshape(-1, 3)
    p = np.concatenate([a, a + 0.5 * h])
    heff = (np.prod(span) / len(p)) ** (1.0 / 3.0)
    return p + rng.uniform(-jitter * heff, jitter * heff, p.shape)


def _voronoi_from_seeds(seeds: np.ndarray, lo, hi, keep=None):
    """Box-clipped Voronoi cells of ``seeds`` (optionally only cells in ``keep``).

    Returns owner, neigh (-1 at the box or at the cut to dropped cells),
    face loops (ragged: off, verts) oriented outward from the owner, and the
    vertex coordinates.
    """
    from scipy.spatial import Voronoi

    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    N = len(seeds)
    h_eff = (np.prod(hi - lo) / N) ** (1.0 / 3.0)
    dm = 3.0 * h_eff
    pts = [seeds]
    src = [np.arange(N)]
    for ax in range(3):
        for side in (lo[ax], hi[ax]):
            sel = np.nonzero(np.abs(seeds[:, ax] - side) < dm)[0]
            q = seeds[sel].copy()
            q[:, ax] = 2.0 * side - q[:, ax]
            pts.append(q)
            src.append(sel)
    P = np.concatenate(pts)
    srcs = np.concatenate(src)
    vor = Voronoi(P)
    rp = vor.ridge_points
    rv = vor.ridge_vertices
    lens = np.fromiter(map(len, rv), np.int64, count=len(rv))
    flat = np.fromiter(itertools.chain.from_iterable(rv), np.int64, count=int(lens.sum()))
    roff = np.zeros(len(rv) + 1, np.int64)
    np.cumsum(lens, out=roff[1:])

    a, b = rp[:, 0], rp[:, 1]
    a_orig = a < N
    b_orig = b < N
    both = a_orig & b_orig
    one = a_orig ^ b_orig
    p_ = np.where(a_orig, a, b)
    m_ = np.where(a_orig, b, a)
    own_mirror = one & (srcs[m_] == p_)
    if keep is None:
        keep = np.ones(N, bool)
    # interior faces between kept cells; faces between kept and dropped cells
    # become boundary faces of the kept one; faces to own mirror are box faces
    k_a = keep[np.minimum(a, N - 1)] & a_orig
    k_b = keep[np.minimum(b, N - 1)] & b_orig
    sel_int = both & k_a & k_b
    sel_cut_a = both & k_a & ~k_b
    sel_cut_b = both & k_b & ~k_a
    keep_p = np.zeros(len(rp), bool)
    keep_p[one] = keep[p_[one]]
    sel_box = own_mirror & keep_p
    owner = np.concatenate([np.minimum(a, b)[sel_int], a[sel_cut_a], b[sel_cut_b], p_[sel_box]])
    neigh = np.concatenate([np.maximum(a, b)[sel_int], np.full(sel_cut_a.sum(), -1),
                            np.full(sel_cut_b.sum(), -1), np.full(sel_box.sum(), -1)])
    # direction the outward normal must follow (owner seed -> other seed)
    other = np.concatenate([np.maximum(a, b)[sel_int], b[sel_cut_a], a[sel_cut_b], m_[sel_box]])
    ridx = np.concatenate([np.nonzero(sel_int)[0], np.nonzero(sel_cut_a)[0],
                           np.nonzero(sel_cut_b)[0], np.nonzero(sel_box)[0]])
    flens = lens[ridx]
    fo = np.zeros(len(ridx) + 1, np.int64)
    np.cumsum(flens, out=fo[1:])
    gidx = np.repeat(roff[ridx] - fo[:-1], flens) + np.arange(fo[-1])
    fverts = flat[gidx]
    if np.any(fverts < 0):
        raise RuntimeError("Voronoi face reaches infinity; mirror band too thin")

    # drop degenerate ridges between a cell and another cell's mirror: they
    # must have zero area (checked) and are not faces of the clipped cell
    deg = one & ~own_mirror & keep_p
    if np.any(deg):
        for r in np.nonzero(deg)[0][:64]:
            X = vor.vertices[flat[roff[r]:roff[r + 1]]]
            if np.ptp(X, axis=0).max() > 1e-9 * h_eff:
                c = X.mean(0)
                S = np.cross(X - c, np.roll(X, -1, 0) - c).sum(0)
                if np.linalg.norm(S) > 1e-12 * h_eff ** 2:
                    raise RuntimeError("non-degenerate ridge to a foreign mirror")

    # renumber the used vertices; snap coordinates on the box planes
    used, inv = np.unique(fverts, return_inverse=True)
    X = vor.vertices[used].copy()
    for ax in range(3):
        for side in (lo[ax], hi[ax]):
            near = np.abs(X[:, ax] - side) < 1e-10 * h_eff
            X[near, ax] = side
    fv = inv.astype(np.int32)

    # orient loops: right-hand normal must point from owner to the other seed
    fid = np.repeat(np.arange(len(ridx)), flens)
    nxt = np.arange(len(fv)) + 1
    nxt[fo[1:] - 1] = fo[:-1]
    # relative to the owner seed: a small face far from the origin would
    # otherwise lose its orientation to cancellation
    ref = np.repeat(seeds[owner], flens, axis=0)
    A = X[fv] - ref
    B = X[fv[nxt]] - ref
    cr = np.cross(A, B)
    S = np.stack([np.bincount(fid, weights=cr[:, k], minlength=len(ridx)) for k in range(3)], 1)
    d = P[other] - seeds[owner]
    flip = np.einsum("ij,ij->i", S, d) < 0
    if np.any(flip):
        pos = np.arange(len(fv)) - np.repeat(fo[:-1], flens)
        rev = np.repeat(fo[:-1] + flens - 1, flens) - pos
        fv = np.where(np.repeat(flip, flens), fv[rev], fv)
    return owner.astype(np.int64), neigh.astype(np.int64), fo, fv, X, P[other]


def _finish(owner, neigh, fo, fv, X, keep_idx, kind, h, seeds, extra=None, other_pt=None) -> Mesh:
    # renumber cells to the kept set (in seed order) and faces by owner
    N_all = int(max(owner.max(), neigh.max())) + 1 if len(owner) else 0
    remap = np.full(max(N_all, (keep_idx.max() + 1) if len(keep_idx) else 0), -1, np.int64)
    remap[keep_idx] = np.arange(len(keep_idx))
    ow = remap[owner]
    ne = np.where(neigh >= 0, remap[np.maximum(neigh, 0)], -1)
    assert np.all(ow >= 0)
    # order faces: by owner, then neighbour (boundary last per owner)
    order = np.lexsort((np.where(ne < 0, np.iinfo(np.int64).max, ne), ow))
    flens = np.diff(fo)[order]
    nfo = np.zeros(len(order) + 1, np.int64)
    np.cumsum(flens, out=nfo[1:])
    gidx = np.repeat(fo[:-1][order] - nfo[:-1], flens) + np.arange(nfo[-1])
    nfv = fv[gidx].astype(np.int32)
    ow = ow[order].astype(np.int32)
    ne = ne[order].astype(np.int32)
    N = len(keep_idx)
    cfo, cf = _cell_face_csr(N, ow, ne)
    extra = dict(extra or {})
    if other_pt is not None:
        # bisector plane of each face, n.x <= c on the owner side
        q = other_pt[order]
        p = seeds[owner[order]]
        extra["face_plane"] = np.concatenate(
            [q - p, (0.5 * (np.einsum("ij,ij->i", q, q) - np.einsum("ij,ij->i", p, p)))[:, None]], 1)
    return Mesh(
        n_cells=N, n_faces=len(ow), n_verts=X.shape[0],
        cell_face_off=cfo, cell_face=cf, face_vert_off=nfo, face_vert=nfv,
        face_owner=ow, face_neigh=ne, face_bc=(ne < 0).astype(np.int8),
        vert_xyz=np.ascontiguousarray(X.T), kind=kind, h=h,
        seeds=seeds[keep_idx] if seeds is not None else None, extra=extra,
    )


def build_voronoi_helper(force: bool = False) -> str:
    """Compile the native Voronoi helper in place (gcc, OpenMP)."""
    if force or not os.path.exists(_VSO) or os.path.getmtime(_VSO) < os.path.getmtime(_VSRC):
        tmp = _VSO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _VSRC, "-lm"])
        os.replace(tmp, _VSO)
    return _VSO


class _VGResult(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int64), ("n_faces", ctypes.c_int64), ("n_verts", ctypes.c_int64),
                ("n_fv", ctypes.c_int64), ("cell_face_off", ctypes.c_void_p), ("cell_face", ctypes.c_void_p),
                ("face_vert_off", ctypes.c_void_p), ("face_vert", ctypes.c_void_p), ("face_owner", ctypes.c_void_p),
                ("face_neigh", ctypes.c_void_p), ("vert_xyz", ctypes.c_void_p), ("face_plane", ctypes.c_void_p),
                ("cell_seed", ctypes.c_void_p)]


@lru_cache(maxsize=1)
def _vlib():
    # SYNTH_VORONOI_SO names another build of _voronoi.c to load (the
    # sanitizer test's instrumented one); else the in-place build
    lib = ctypes.CDLL(os.environ.get("SYNTH_VORONOI_SO") or build_voronoi_helper())
    P = ctypes.c_void_p
    lib.vg_build.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_int, P, P]
    lib.vg_build.restype = ctypes.c_int
    lib.vg_free.argtypes = [P]
    lib.vg_free.restype = None
    return lib


def _take(ptr, n, ctype, dtype):
    if n == 0:
        return np.zeros(0, dtype)
    a = np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ctype)), shape=(n,))
    return np.array(a, dtype=dtype, copy=True)


def _voronoi_native(seeds: np.ndarray, lo, hi, keep=None, threads: int | None = None) -> dict:
    """Box-clipped Voronoi cells of the kept seeds by the native helper."""
    P = np.ascontiguousarray(seeds, np.float64)
    N = len(P)
    lo = np.ascontiguousarray(lo, np.float64)
    hi = np.ascontiguousarray(hi, np.float64)
    kp = np.ascontiguousarray(np.ones(N, np.uint8) if keep is None else np.asarray(keep, np.uint8))
    if threads is None:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    r = _VGResult()
    err = ctypes.c_int64(-1)
    vp = ctypes.c_void_p
    rc = _vlib().vg_build(N, P.ctypes.data_as(vp), lo.ctypes.data_as(vp), hi.ctypes.data_as(vp),
                          kp.ctypes.data_as(vp), int(threads), ctypes.byref(r), ctypes.byref(err))
    if rc != 0:
        raise RuntimeError(f"native Voronoi construction failed ({rc}) at seed {err.value}")
    try:
        NC, NF, NV, NFV = r.n_cells, r.n_faces, r.n_verts, r.n_fv
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        out = dict(
            cell_face_off=_take(r.cell_face_off, NC + 1, i64, np.int64),
            cell_face=_take(r.cell_face, int(_take(r.cell_face_off, NC + 1, i64, np.int64)[-1]), i32, np.int32),
            face_vert_off=_take(r.face_vert_off, NF + 1, i64, np.int64),
            face_vert=_take(r.face_vert, NFV, i32, np.int32),
            face_owner=_take(r.face_owner, NF, i32, np.int32),
            face_neigh=_take(r.face_neigh, NF, i32, np.int32),
            vert_xyz=_take(r.vert_xyz, 3 * NV, f64, np.float64).reshape(3, NV),
            face_plane=_take(r.face_plane, 4 * NF, f64, np.float64).reshape(NF, 4),
            cell_seed=_take(r.cell_seed, NC, i32, np.int64),
            n_cells=NC, n_faces=NF, n_verts=NV,
        )
    finally:
        _vlib().vg_free(ctypes.byref(r))
    return out


def _native_mesh(seeds, lo, hi, keep, kind, h, extra=None) -> Mesh:
    o = _voronoi_native(seeds, lo, hi, keep)
    ex = dict(extra or {})
    ex["face_plane"] = o["face_plane"]
    return Mesh(
        n_cells=o["n_cells"], n_faces=o["n_faces"], n_verts=o["n_verts"],
        cell_face_off=o["cell_face_off"], cell_face=o["cell_face"], face_vert_off=o["face_vert_off"],
        face_vert=o["face_vert"], face_owner=o["face_owner"], face_neigh=o["face_neigh"],
        face_bc=(o["face_neigh"] < 0).astype(np.int8), vert_xyz=np.ascontiguousarray(o["vert_xyz"]),
        kind=kind, h=h, seeds=np.asarray(seeds)[o["cell_seed"]], extra=ex,
    )


def voronoi_box_mesh(n: int, seed: int, jitter: float = 0.3,
                     lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), engine: str = "native") -> Mesh:
    """Voronoi cells of 2 n^3 jittered BCC seeds, clipped to the box [lo, hi]
    (engine "native" or "qhull": the same cells, numbered differently)."""
    rng = np.random.default_rng(seed)
    seeds = bcc_seeds(n, rng, jitter, lo, hi)
    N = len(seeds)
    h = (np.prod(np.asarray(hi) - np.asarray(lo)) / N) ** (1.0 / 3.0)
    if engine == "native":
        return _native_mesh(seeds, lo, hi, None, "voronoi", h)
    owner, neigh, fo, fv, X, oth = _voronoi_from_seeds(seeds, lo, hi)
    return _finish(owner, neigh, fo, fv, X, np.arange(N), "voronoi", h, seeds, other_pt=oth)


def voronoi_pipe_mesh(n_radial: int, R: float, L: float, seed: int, jitter: float = 0.3,
                      engine: str = "native") -> Mesh:
    """Voronoi cells of a pipe r <= R, 0 <= y <= L (axis along y).

    BCC seeds fill the bounding box; cells whose seed lies in the pipe are
    kept.  Faces toward dropped cells become boundary faces (a staircase wall),
    as do the two end caps of the box.
    """
    rng = np.random.default_rng(seed)
    lo = np.array([-R, 0.0, -R])
    hi = np.array([R, L, R])
    ny = max(1, int(round(n_radial * L / (2.0 * R))))
    seeds = bcc_seeds((n_radial, ny, n_radial), rng, jitter, lo, hi)
    r = np.hypot(seeds[:, 0], seeds[:, 2])
    keep = r <= R
    N = len(seeds)
    h = (np.prod(hi - lo) / N) ** (1.0 / 3.0)
    if engine == "native":
        return _native_mesh(seeds, lo, hi, keep, "voronoi-pipe", h, extra={"R": R, "L": L})
    owner, neigh, fo, fv, X, oth = _voronoi_from_seeds(seeds, lo, hi, keep=keep)
    keep_idx = np.nonzero(keep)[0]
    return _finish(owner, neigh, fo, fv, X, keep_idx, "voronoi-pipe", h, seeds,
                   extra={"R": R, "L": L}, other_pt=oth)


def concat(meshes: list) -> Mesh:
    """Disjoint union of meshes: cells, faces and vertices of mesh i follow
    those of meshes 0..i-1, ids and offsets shifted (vertex coordinates per
    component, [3][total])."""
    cfo, cf, fvo, fv, ow, ne, bc, xyz = [], [], [], [], [], [], [], []
    bN = bF = bV = bcf = bfv = 0
    for i, m in enumerate(meshes):
        cfo.append(np.asarray(m.cell_face_off[: (None if i == len(meshes) - 1 else -1)], np.int64) + bcf)
        fvo.append(np.asarray(m.face_vert_off[: (None if i == len(meshes) - 1 else -1)], np.int64) + bfv)
        cf.append(np.asarray(m.cell_face, np.int64) + bF)
        fv.append(np.asarray(m.face_vert, np.int64) + bV)
        ow.append(np.asarray(m.face_owner, np.int64) + bN)
        ne.append(np.where(m.face_neigh >= 0, np.asarray(m.face_neigh, np.int64) + bN, m.face_neigh))
        bc.append(np.asarray(m.face_bc, np.int8))
        xyz.append(np.asarray(m.vert_xyz, np.float64))
        bN += m.n_cells
        bF += m.n_faces
        bV += m.n_verts
        bcf += len(m.cell_face)
        bfv += len(m.face_vert)
    hs = [m.h for m in meshes]
    return Mesh(
        n_cells=bN, n_faces=bF, n_verts=bV,
        cell_face_off=np.concatenate(cfo), cell_face=np.concatenate(cf).astype(np.int32),
        face_vert_off=np.concatenate(fvo), face_vert=np.concatenate(fv).astype(np.int32),
        face_owner=np.concatenate(ow).astype(np.int32), face_neigh=np.concatenate(ne).astype(np.int32),
        face_bc=np.concatenate(bc), vert_xyz=np.ascontiguousarray(np.concatenate(xyz, 1)),
        kind="+".join(m.kind for m in meshes), h=float(min(hs)),
        extra={"parts": [(m.n_cells, m.n_faces, m.n_verts) for m in meshes]},
    )
