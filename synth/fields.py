"""Synthetic input fields: volume fractions, temperatures, boundary values.

Volume fractions come from sub-point counting (a K^3 grid over each cell's
bounding box, restricted to the cell by its bisector planes), only for cells
the region boundary can touch; all other cells are exactly 0 or 1.  The
counting runs in a small C helper (``_subsample.c``) built with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from functools import lru_cache

import numpy as np
from scipy.special import erf

from .meshes import Mesh

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "_subsample.c")
_SO = os.path.join(_HERE, "_subsample.so")


def build_helper(force: bool = False) -> str:
    """Compile the sub-sampling helper in place (gcc, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


@lru_cache(maxsize=1)
def _lib():
    # SYNTH_SUBSAMPLE_SO names another build of _subsample.c to load (the
    # sanitizer test's instrumented one); else the in-place build
    lib = ctypes.CDLL(os.environ.get("SYNTH_SUBSAMPLE_SO") or build_helper())
    P = ctypes.c_void_p
    lib.synth_subsample.argtypes = [ctypes.c_int64, P, P, P, P, P, ctypes.c_int, P, ctypes.c_int, P]
    lib.synth_subsample.restype = None
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _cell_planes(mesh: Mesh, cells: np.ndarray):
    """Half-spaces bounding each listed cell (empty for hexahedra)."""
    if "face_plane" not in mesh.extra:
        return np.zeros(len(cells) + 1, np.int64), np.zeros((0, 4))
    fp = mesh.extra["face_plane"]
    off = mesh.cell_face_off
    cnt = off[cells + 1] - off[cells]
    po = np.zeros(len(cells) + 1, np.int64)
    np.cumsum(cnt, out=po[1:])
    idx = np.repeat(off[cells] - po[:-1], cnt) + np.arange(po[-1])
    faces = mesh.cell_face[idx]
    cell_rep = np.repeat(cells, cnt)
    pl = fp[faces].copy()
    flip = mesh.face_owner[faces] != cell_rep
    pl[flip] *= -1.0
    return po, np.ascontiguousarray(pl)


def subsample(mesh: Mesh, cells: np.ndarray, bbox: np.ndarray, kind: int,
              sph_off: np.ndarray, sph: np.ndarray, prm=None, K: int = 64) -> np.ndarray:
    cells = np.ascontiguousarray(cells, np.int64)
    po, pl = _cell_planes(mesh, cells)
    bb = np.ascontiguousarray(bbox[cells])
    out = np.empty(len(cells))
    prm = np.ascontiguousarray(np.zeros(5) if prm is None else np.asarray(prm, float))
    sph = np.ascontiguousarray(sph, float).reshape(-1, 4)
    if sph.size == 0:
        sph = np.zeros((1, 4))
    _lib().synth_subsample(len(cells), _ptr(bb), _ptr(po), _ptr(pl), _ptr(np.ascontiguousarray(sph_off, np.int64)),
                           _ptr(sph), kind, _ptr(prm), K, _ptr(out))
    if np.any(out < 0):
        raise RuntimeError("sub-sampling found an empty cell")
    return out


def _cell_vertices(mesh: Mesh):
    """(cell, vertex) incidence pairs with repeats, for min/max queries
    (computed once per mesh)."""
    return mesh._cached("_cell_vertices", lambda: _cell_vertices_of(mesh))


def _cell_vertices_of(mesh: Mesh):
    N = mesh.n_cells
    cf_cnt = np.diff(mesh.cell_face_off)
    faces = mesh.cell_face.astype(np.int64)
    rep = np.diff(mesh.face_vert_off)[faces]
    cells = np.repeat(np.repeat(np.arange(N), cf_cnt), rep)
    starts = mesh.face_vert_off[faces]
    idx = np.repeat(starts - np.cumsum(np.r_[0, rep[:-1]]), rep) + np.arange(rep.sum())
    return cells, mesh.face_vert[idx]


def _ranges(off: np.ndarray, rows: np.ndarray) -> np.ndarray:
    cnt = off[rows + 1] - off[rows]
    return np.repeat(off[rows] - np.cumsum(np.r_[0, cnt[:-1]]), cnt) + np.arange(cnt.sum())


def sphere_alpha(mesh: Mesh, spheres: np.ndarray, K: int = 64) -> np.ndarray:
    """Liquid fraction with vapour bubbles ``spheres`` [S, 4] = (centre, r)."""
    spheres = np.asarray(spheres, float).reshape(-1, 4)
    N = mesh.n_cells
    bbox = mesh.cell_bbox()
    alpha = np.ones(N)
    cells_v, verts_v = _cell_vertices(mesh)          # sorted by cell
    cv_off = np.zeros(N + 1, np.int64)
    np.cumsum(np.bincount(cells_v, minlength=N), out=cv_off[1:])
    X = mesh.vert_xyz
    touch_cells, touch_sph = [], []
    inside_any = np.zeros(N, bool)
    # cells whose box meets the sphere's box have their box centre within
    # r + (largest box half-diagonal) of the sphere's centre
    from scipy.spatial import cKDTree

    def box_tree():
        bc = 0.5 * (bbox[:, :3] + bbox[:, 3:])
        return cKDTree(bc), 0.5 * float(np.sqrt(((bbox[:, 3:] - bbox[:, :3]) ** 2).sum(1)).max())

    tree, ext = mesh._cached("_box_tree", box_tree)
    for s, (cx, cy, cz, r) in enumerate(spheres):
        c = np.array([cx, cy, cz])
        near = np.sort(np.asarray(tree.query_ball_point(c, r * np.sqrt(3.0) + ext + 1e-12), np.int64))
        cand = near[np.all(bbox[near, :3] <= c + r, 1) & np.all(bbox[near, 3:] >= c - r, 1)]
        if len(cand) == 0:
            continue
        q = np.clip(c, bbox[cand, :3], bbox[cand, 3:])
        cand = cand[((q - c) ** 2).sum(1) < r * r]
        if len(cand) == 0:
            continue
        # a convex cell whose vertices all lie inside the sphere is vapour
        idx = _ranges(cv_off, cand)
        dd = ((X[:, verts_v[idx]].T - c) ** 2).sum(1) - r * r
        worst = np.maximum.reduceat(dd, np.r_[0, np.cumsum(cv_off[cand + 1] - cv_off[cand])[:-1]])
        inside_any[cand[worst < 0]] = True
        touch_cells.append(cand)
        touch_sph.append(np.full(len(cand), s))
    alpha[inside_any] = 0.0
    if not touch_cells:
        return alpha
    tc = np.concatenate(touch_cells)
    ts = np.concatenate(touch_sph)
    mixed = np.unique(tc[~inside_any[tc]])
    if len(mixed):
        m_of = np.full(N, -1, np.int64)
        m_of[mixed] = np.arange(len(mixed))
        keep = m_of[tc] >= 0
        mc = m_of[tc[keep]]
        so = np.argsort(mc, kind="stable")
        sph_list = spheres[ts[keep][so]]
        off = np.zeros(len(mixed) + 1, np.int64)
        np.cumsum(np.bincount(mc, minlength=len(mixed)), out=off[1:])
        alpha[mixed] = subsample(mesh, mixed, bbox, 0, off, sph_list, None, K)
    return alpha


def film_alpha(mesh: Mesh, R: float, d0: float, amp: float, waves: float, L: float, K: int = 32) -> np.ndarray:
    """Liquid film on the pipe wall: liquid where r > R - d0 (1 + amp sin(2 pi waves y/L))."""
    N = mesh.n_cells
    cells_v, verts_v = _cell_vertices(mesh)
    X = mesh.vert_xyz[:, verts_v]
    r = np.hypot(X[0], X[2])
    delta = d0 * (1.0 + amp * np.sin(2.0 * np.pi * waves * X[1] / L))
    liq = r > R - delta
    nl = np.bincount(cells_v, weights=liq.astype(float), minlength=N)
    nt = np.bincount(cells_v, minlength=N)
    alpha = (nl == nt).astype(float)
    mixed = np.nonzero((nl > 0) & (nl < nt))[0]
    # cells with all vertices on one side can still be cut by the curved
    # film surface; widen the set by one face-neighbour ring
    off, nb = mesh.face_neighbours()
    ring = np.zeros(N, bool)
    ring[mixed] = True
    cnt = off[mixed + 1] - off[mixed]
    idx = np.repeat(off[mixed] - np.cumsum(np.r_[0, cnt[:-1]]), cnt) + np.arange(cnt.sum())
    ring[nb[idx]] = True
    cand = np.nonzero(ring)[0]
    if len(cand):
        bbox = mesh.cell_bbox()
        alpha[cand] = subsample(mesh, cand, bbox, 1, np.zeros(len(cand) + 1, np.int64), np.zeros((1, 4)),
                                [R, d0, amp, waves, L], K)
    return alpha


def plane_alpha(mesh: Mesh, normal, c: float, K: int = 16) -> np.ndarray:
    """Liquid where n.x >= c (a planar interface), by sub-point counting in the
    cells the plane crosses."""
    n = np.asarray(normal, float)
    n = n / np.linalg.norm(n)
    N = mesh.n_cells
    cells_v, verts_v = _cell_vertices(mesh)
    d = n @ mesh.vert_xyz[:, verts_v] - c
    seg = np.r_[0, np.cumsum(np.bincount(cells_v, minlength=N))[:-1]]   # incidences run cell by cell
    lo = np.minimum.reduceat(d, seg)
    hi = np.maximum.reduceat(d, seg)
    alpha = (lo >= 0).astype(float)
    cut = np.nonzero((lo < 0) & (hi > 0))[0]
    if len(cut):
        bbox = mesh.cell_bbox()
        alpha[cut] = subsample(mesh, cut, bbox, 2, np.zeros(len(cut) + 1, np.int64), np.zeros((1, 4)),
                               [n[0], n[1], n[2], c, 0.0], K)
    return alpha


# ---------------------------------------------------------------- temperatures
def radial_linear_T(points: np.ndarray, c, r0: float, slope: float, T_sat: float) -> np.ndarray:
    """T_sat inside |x-c| <= r0, T_sat + slope (|x-c| - r0) outside."""
    rho = np.linalg.norm(points - np.asarray(c), axis=1)
    return np.where(rho > r0, T_sat + slope * (rho - r0), T_sat)


def radial_erf_T(points: np.ndarray, c, r0: float, width: float, dT: float, T_sat: float) -> np.ndarray:
    """T_sat inside, T_sat + dT erf((|x-c| - r0)/width) outside (Scriven-like decay)."""
    rho = np.linalg.norm(points - np.asarray(c), axis=1)
    return np.where(rho > r0, T_sat + dT * erf((rho - r0) / width), T_sat)


def nearest_bubble_T(points: np.ndarray, spheres: np.ndarray, slopes: np.ndarray, T_sat: float,
                     chunk: int = 1 << 16, k: int = 8) -> np.ndarray:
    """T_sat inside any bubble, else T_sat + g_b (|x - c_b| - r_b) for the bubble b
    whose surface is nearest (ties: lowest bubble index).

    The k bubbles with the nearest centres are tried first; a point whose best
    surface distance among them is not provably the global minimum (every other
    bubble is at least |x - c_(k)| - r_max away) is checked against all."""
    spheres = np.asarray(spheres, float).reshape(-1, 4)
    S = len(spheres)
    out = np.empty(len(points))
    if S == 0:
        out[:] = T_sat
        return out
    kk = min(k, S)
    from scipy.spatial import cKDTree
    tree = cKDTree(spheres[:, :3])
    rmax = spheres[:, 3].max()
    for s in range(0, len(points), chunk):
        p = points[s:s + chunk]
        dc, ic = tree.query(p, k=kk)
        if kk == 1:
            dc, ic = dc[:, None], ic[:, None]
        order = np.argsort(ic, axis=1, kind="stable")        # candidates by bubble index
        ic = np.take_along_axis(ic, order, 1)
        d = np.linalg.norm(p[:, None, :] - spheres[ic, :3], axis=2) - spheres[ic, 3]
        j = np.argmin(d, 1)
        b = ic[np.arange(len(p)), j]
        dist = d[np.arange(len(p)), j]
        if kk < S:
            unsure = np.nonzero(dist > dc.max(1) - rmax)[0]
            if len(unsure):
                q = p[unsure]
                dd = np.linalg.norm(q[:, None, :] - spheres[None, :, :3], axis=2) - spheres[None, :, 3]
                bb = np.argmin(dd, 1)
                b[unsure] = bb
                dist[unsure] = dd[np.arange(len(q)), bb]
        out[s:s + chunk] = np.where(dist > 0, T_sat + slopes[b] * dist, T_sat)
    return out


def film_T(points: np.ndarray, R: float, d0: float, amp: float, waves: float, L: float,
           dT_wall: float, T_sat: float) -> np.ndarray:
    """T_sat in the vapour core, rising linearly across the film to T_sat + dT_wall at the wall."""
    r = np.hypot(points[:, 0], points[:, 2])
    delta = d0 * (1.0 + amp * np.sin(2.0 * np.pi * waves * points[:, 1] / L))
    return np.where(r > R - delta, T_sat + dT_wall * (r - (R - delta)) / delta, T_sat)


def rsa_spheres(rng: np.random.Generator, n_max: int, r_lo: float, r_hi: float, clearance: float,
                lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), max_attempts: int = 10000) -> np.ndarray:
    """Random sequential addition of non-overlapping spheres.

    Radii are drawn i.i.d. from U[r_lo, r_hi]; a sphere is kept when it keeps
    ``clearance`` from the walls and from every earlier sphere; each sphere
    gets at most ``max_attempts`` tries and placement stops at the first
    sphere that runs out of tries or at ``n_max``.
    """
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    out = []
    for _ in range(n_max):
        r = rng.uniform(r_lo, r_hi)
        placed = False
        # vectorised tries in blocks
        if np.any(lo + r + clearance > hi - r - clearance):
            break                     # no room for this sphere at all
        for _blk in range(0, max_attempts, 500):
            c = rng.uniform(lo + r + clearance, hi - r - clearance, size=(500, 3))
            if out:
                S = np.asarray(out)
                d = np.linalg.norm(c[:, None, :] - S[None, :, :3], axis=2) - S[None, :, 3] - r
                ok = np.all(d >= clearance, axis=1)
            else:
                ok = np.ones(500, bool)
            if ok.any():
                out.append([*c[np.argmax(ok)], r])
                placed = True
                break
        if not placed:
            break
    return np.asarray(out).reshape(-1, 4)
