"""CPU oracle for the interface hot path (TEST INFRASTRUCTURE ONLY).

A plain, single-threaded FP64 implementation in C (``vof_oracle.c``) plus a
numpy reference of the bracket network (``mlp_ref``).  Only the tests, the
smoke check and the bench's CPU-baseline leg use this package; the product
library never imports, links or calls it, and the two share no code.

Functions here take :class:`synth.Mesh`-like objects (any object with the CSR
attributes) and numpy arrays, and return numpy arrays.  Vector fields are
structure-of-arrays ``[3, N]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from functools import lru_cache

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vof_oracle.c")
_SO = os.path.join(_HERE, "_vof_oracle.so")

OK, NOT_MIXED, LEARNED_FALLBACK, DEGENERATE, MAX_ITER, G_SINGULAR, BAD_INPUT, NO_ROOT = range(8)

CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC"]


def build(force: bool = False) -> str:
    """Compile the oracle in place with gcc (no FMA contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _CMesh(ctypes.Structure):
    _fields_ = [
        ("n_cells", ctypes.c_int64), ("n_faces", ctypes.c_int64), ("n_verts", ctypes.c_int64),
        ("cell_face_off", ctypes.c_void_p), ("cell_face", ctypes.c_void_p),
        ("face_vert_off", ctypes.c_void_p), ("face_vert", ctypes.c_void_p),
        ("face_owner", ctypes.c_void_p), ("face_neigh", ctypes.c_void_p),
        ("face_bc", ctypes.c_void_p), ("vert_xyz", ctypes.c_void_p),
    ]


class _COpts(ctypes.Structure):
    _fields_ = [
        ("eps_mixed", ctypes.c_double), ("tol_rel", ctypes.c_double), ("max_iter", ctypes.c_int),
        ("vertex_mode", ctypes.c_int), ("fixed_iso", ctypes.c_int), ("iso", ctypes.c_double),
    ]


@lru_cache(maxsize=1)
def _lib():
    # ORACLE_SO names another build of vof_oracle.c to load (the sanitizer
    # test's instrumented one); else the in-place build
    so = os.environ.get("ORACLE_SO") or build()
    lib = ctypes.CDLL(so)
    P = ctypes.c_void_p
    lib.orc_face_geometry.argtypes = [P, P, P]
    lib.orc_cell_geometry.argtypes = [P, P, P]
    lib.orc_vertex_field.argtypes = [P, P, P, ctypes.c_int, P]
    lib.orc_cut_cell.argtypes = [P, ctypes.c_int64, P, P, ctypes.c_double, P]
    lib.orc_grad.argtypes = [P, P, P, P, P, ctypes.c_double, P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                             ctypes.c_int, P, P, P]
    lib.orc_reconstruct.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.orc_mass_transfer.argtypes = [ctypes.c_int64, P, P, P, P, P, P, P, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, P, P]
    D, I = ctypes.c_double, ctypes.c_int
    lib.orc_extrapolate.argtypes = [P, P, P, P, P, P, P, P, D, I, I, D, P, P, P, P]
    lib.orc_robin.argtypes = [P, P, P, P, P, P, D, D, P, P, P, P, P]
    lib.orc_csf_smooth.argtypes = [P, P, P, P, P, I, P]
    lib.orc_lsq_interior.argtypes = [P, P, P, P]
    lib.orc_csf_normal.argtypes = [P, P, P, P]
    lib.orc_csf_raw_curvature.argtypes = [P, P, P, P, P, P, P]
    lib.orc_csf_smooth_curvature.argtypes = [P, P, P, P, P, P, P]
    lib.orc_csf.argtypes = [P, P, P, P, P, P, I, D, P, P, P, P, P, P]
    for f in ("orc_face_geometry", "orc_cell_geometry", "orc_vertex_field", "orc_cut_cell",
              "orc_grad", "orc_reconstruct", "orc_mass_transfer", "orc_extrapolate"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OMesh:
    """Holds contiguous copies of a mesh's arrays and the C view onto them."""

    def __init__(self, mesh):
        self.n_cells = int(mesh.n_cells)
        self.n_faces = int(mesh.n_faces)
        self.n_verts = int(mesh.n_verts)
        self._keep = dict(
            cfo=np.ascontiguousarray(mesh.cell_face_off, np.int64),
            cf=np.ascontiguousarray(mesh.cell_face, np.int32),
            fvo=np.ascontiguousarray(mesh.face_vert_off, np.int64),
            fv=np.ascontiguousarray(mesh.face_vert, np.int32),
            ow=np.ascontiguousarray(mesh.face_owner, np.int32),
            ne=np.ascontiguousarray(mesh.face_neigh, np.int32),
            bc=np.ascontiguousarray(mesh.face_bc, np.int8),
            xyz=np.ascontiguousarray(mesh.vert_xyz, np.float64).reshape(3, -1),
        )
        k = self._keep
        self.c = _CMesh(self.n_cells, self.n_faces, self.n_verts, _p(k["cfo"]), _p(k["cf"]), _p(k["fvo"]),
                        _p(k["fv"]), _p(k["ow"]), _p(k["ne"]), _p(k["bc"]), _p(k["xyz"]))

    @property
    def ref(self):
        return ctypes.byref(self.c)


def _om(mesh) -> OMesh:
    return mesh if isinstance(mesh, OMesh) else OMesh(mesh)


@dataclass
class Geometry:
    V: np.ndarray      # [N]
    xc: np.ndarray     # [3, N]
    Sf: np.ndarray     # [3, NF]
    xf: np.ndarray     # [3, NF]


def geometry(mesh) -> Geometry:
    om = _om(mesh)
    Sf = np.empty((3, om.n_faces))
    xf = np.empty((3, om.n_faces))
    V = np.empty(om.n_cells)
    xc = np.empty((3, om.n_cells))
    e = _lib().orc_face_geometry(om.ref, _p(Sf), _p(xf))
    if e:
        raise RuntimeError(f"orc_face_geometry failed ({e})")
    e = _lib().orc_cell_geometry(om.ref, _p(V), _p(xc))
    if e:
        raise RuntimeError(f"orc_cell_geometry failed ({e})")
    return Geometry(V, xc, Sf, xf)


def vertex_field(mesh, xc, alpha, mode: int = 0) -> np.ndarray:
    om = _om(mesh)
    phi = np.empty(om.n_verts)
    e = _lib().orc_vertex_field(om.ref, _p(np.ascontiguousarray(xc)), _p(np.ascontiguousarray(alpha, float)),
                                mode, _p(phi))
    if e:
        raise RuntimeError("orc_vertex_field failed")
    return phi


def cut_cell(mesh, P: int, xc, phi, s: float) -> dict:
    om = _om(mesh)
    res = np.empty(9)
    e = _lib().orc_cut_cell(om.ref, int(P), _p(np.ascontiguousarray(xc)), _p(np.ascontiguousarray(phi, float)),
                            float(s), _p(res))
    if e:
        raise RuntimeError(f"orc_cut_cell failed ({e})")
    return {"V": res[0], "S": res[1:4].copy(), "A": res[4], "c": res[5:8].copy(), "nloops": int(res[8])}


def reconstruct(mesh, alpha, geom: Geometry | None = None, *, eps_mixed=1e-8, tol_rel=1e-13, max_iter=100,
                vertex_mode=0, fixed_iso=False, iso=0.5, phi=None, hint_lo=None, hint_hi=None, cells=None) -> dict:
    """Volume-matched (or fixed-isovalue) reconstruction of every mixed cell;
    `cells` (optional index array) restricts it to those cells, the others
    getting status -1 (not processed)."""
    om = _om(mesh)
    geom = geom or geometry(om)
    N = om.n_cells
    alpha = np.ascontiguousarray(alpha, float)
    out = dict(s=np.empty(N), n=np.empty((3, N)), A=np.empty(N), d=np.empty(N), alpha_got=np.empty(N),
               status=np.empty(N, np.int32), iters=np.empty(N, np.int32))
    op = _COpts(eps_mixed, tol_rel, max_iter, vertex_mode, int(bool(fixed_iso)), iso)
    hl = None if hint_lo is None else np.ascontiguousarray(hint_lo, float)
    hh = None if hint_hi is None else np.ascontiguousarray(hint_hi, float)
    ph = None if phi is None else np.ascontiguousarray(phi, float)
    only = None
    if cells is not None:
        only = np.zeros(N, np.int8)
        only[np.asarray(cells)] = 1
    e = _lib().orc_reconstruct(om.ref, _p(geom.V), _p(geom.xc), _p(alpha), ctypes.byref(op), _p(ph), _p(hl),
                               _p(hh), _p(out["s"]), _p(out["n"]), _p(out["A"]), _p(out["d"]),
                               _p(out["alpha_got"]), _p(out["status"]), _p(out["iters"]), _p(only))
    if e:
        raise RuntimeError(f"orc_reconstruct failed ({e})")
    return out


def grad(mesh, geom: Geometry, T, Tb, T_sat, alpha, modified=True, printed=False, weight=0, extended=False,
         cells=None):
    """Least-squares gradient (App. B): weight 0 uniform, 1 inverse distance,
    2 inverse distance squared; extended: vertex neighbours instead of face
    neighbours.  `cells` (optional index array) restricts it to those cells,
    the others getting status -1 and a NaN gradient."""
    om = _om(mesh)
    N = om.n_cells
    g = np.empty((3, N))
    st = np.empty(N, np.int32)
    only = None
    if cells is not None:
        only = np.zeros(N, np.int8)
        only[np.asarray(cells)] = 1
    e = _lib().orc_grad(om.ref, _p(geom.xc), _p(geom.xf), _p(np.ascontiguousarray(T, float)),
                        _p(np.ascontiguousarray(Tb, float)), float(T_sat), _p(np.ascontiguousarray(alpha, float)),
                        int(modified), int(printed), int(weight), int(extended), _p(g), _p(st), _p(only))
    if e:
        raise RuntimeError("orc_grad failed")
    return g, st


def mass_transfer(geom: Geometry, alpha, n, A, gradT, k_l, k_v, h_lv, gl=None, gv=None):
    N = len(A)
    mdot = np.empty(N)
    Qdot = np.empty(N)
    e = _lib().orc_mass_transfer(N, _p(geom.V), _p(np.ascontiguousarray(alpha, float)),
                                 _p(np.ascontiguousarray(n)), _p(np.ascontiguousarray(A)),
                                 _p(np.ascontiguousarray(gradT)),
                                 _p(None if gl is None else np.ascontiguousarray(gl)),
                                 _p(None if gv is None else np.ascontiguousarray(gv)),
                                 float(k_l), float(k_v), float(h_lv), _p(mdot), _p(Qdot))
    if e:
        raise RuntimeError("orc_mass_transfer failed")
    return mdot, Qdot


def extrapolate(mesh, geom: Geometry, alpha, grad, n_int, A, eps_mixed=1e-8, layers=2, max_iter=120, tol=1e-3):
    """Phase gradients by pseudo-time extrapolation (Eq. extrapolation):
    returns (G_l [3,N], G_v [3,N], sweeps, domain mask [N] bool)."""
    om = _om(mesh)
    N = om.n_cells
    gl = np.empty((3, N))
    gv = np.empty((3, N))
    it = np.zeros(1, np.int32)
    dom = np.zeros(N, np.int8)
    e = _lib().orc_extrapolate(om.ref, _p(geom.V), _p(geom.xc), _p(geom.Sf), _p(np.ascontiguousarray(alpha, float)),
                               _p(np.ascontiguousarray(grad, float)), _p(np.ascontiguousarray(n_int, float)),
                               _p(np.ascontiguousarray(A, float)), float(eps_mixed), int(layers), int(max_iter),
                               float(tol), _p(gl), _p(gv), _p(it), _p(dom))
    if e:
        raise RuntimeError("orc_extrapolate failed")
    return gl, gv, int(it[0]), dom.astype(bool)


def band_mask(mesh, alpha, eps_mixed=1e-8) -> np.ndarray:
    """Cells that are mixed or own a face crossed by the alpha = 1/2 level."""
    a = np.asarray(alpha)
    mixed = (a > eps_mixed) & (a < 1 - eps_mixed)
    inner = mesh.face_neigh >= 0
    o = mesh.face_owner[inner]
    q = mesh.face_neigh[inner]
    cross = (a[o] - 0.5) * (a[q] - 0.5) < 0
    band = mixed.copy()
    band[o[cross]] = True
    band[q[cross]] = True
    return band


def run_path(wl, **kw) -> dict:
    """Reconstruct + interface-modified gradient + mass transfer on a workload."""
    om = OMesh(wl.mesh)
    geom = geometry(om)
    rec = reconstruct(om, wl.alpha, geom, **kw)
    g, gst = grad(om, geom, wl.T, wl.T_bface, wl.T_sat, wl.alpha)
    mdot, Qdot = mass_transfer(geom, wl.alpha, rec["n"], rec["A"], g, wl.k_l, wl.k_v, wl.h_lv)
    return dict(geom=geom, rec=rec, grad=g, grad_status=gst, mdot=mdot, Qdot=Qdot, omesh=om)


def robin(mesh, geom: Geometry, alpha, n_int, A, k_l, k_v):
    """Interface heat-transfer coefficients of the detached faces
    (Eq. interface_htc): returns dict with a_cell [N], a_face [2,NF] (owner,
    neighbour side), d_face [2,NF], area_face [NF], crossing [NF] bool."""
    om = _om(mesh)
    N, NF = om.n_cells, om.n_faces
    a_cell = np.empty(N)
    a_face = np.empty((2, NF))
    d_face = np.empty((2, NF))
    area = np.empty(NF)
    cross = np.zeros(NF, np.int8)
    e = _lib().orc_robin(om.ref, _p(geom.xc), _p(geom.Sf), _p(np.ascontiguousarray(alpha, float)),
                         _p(np.ascontiguousarray(n_int, float)), _p(np.ascontiguousarray(A, float)),
                         float(k_l), float(k_v), _p(a_cell), _p(a_face), _p(d_face), _p(area), _p(cross))
    if e:
        raise RuntimeError("orc_robin failed")
    return dict(a_cell=a_cell, a_face=a_face, d_face=d_face, area_face=area, crossing=cross.astype(bool))


# ------------------------------------------------------------- CSF curvature
def csf(mesh, geom: Geometry, alpha, n_smooth=2, sigma=1.0):
    """The surface-tension curvature chain (Sec. 2.4, surface tension):
    dict with alpha_hat [N], n [3,N], kappa_raw, kappa_star, kappa [N], F [3,N]."""
    om = _om(mesh)
    N = om.n_cells
    out = dict(alpha_hat=np.empty(N), n=np.empty((3, N)), kappa_raw=np.empty(N), kappa_star=np.empty(N),
               kappa=np.empty(N), F=np.empty((3, N)))
    e = _lib().orc_csf(om.ref, _p(geom.V), _p(geom.xc), _p(geom.Sf), _p(geom.xf),
                       _p(np.ascontiguousarray(alpha, float)), int(n_smooth), float(sigma), _p(out["alpha_hat"]),
                       _p(out["n"]), _p(out["kappa_raw"]), _p(out["kappa_star"]), _p(out["kappa"]), _p(out["F"]))
    if e:
        raise RuntimeError("orc_csf failed")
    return out


def csf_smooth(mesh, geom: Geometry, alpha, n_smooth):
    om = _om(mesh)
    out = np.empty(om.n_cells)
    if _lib().orc_csf_smooth(om.ref, _p(geom.xc), _p(geom.Sf), _p(geom.xf), _p(np.ascontiguousarray(alpha, float)),
                             int(n_smooth), _p(out)):
        raise RuntimeError("orc_csf_smooth failed")
    return out


def lsq_interior(mesh, geom: Geometry, val):
    om = _om(mesh)
    g = np.empty((3, om.n_cells))
    _lib().orc_lsq_interior(om.ref, _p(geom.xc), _p(np.ascontiguousarray(val, float)), _p(g))
    return g


def csf_raw_curvature(mesh, geom: Geometry, n):
    om = _om(mesh)
    k = np.empty(om.n_cells)
    _lib().orc_csf_raw_curvature(om.ref, _p(geom.V), _p(geom.xc), _p(geom.Sf), _p(geom.xf),
                                 _p(np.ascontiguousarray(n, float)), _p(k))
    return k


def csf_smooth_curvature(mesh, geom: Geometry, alpha_hat, n, kraw):
    om = _om(mesh)
    ks = np.empty(om.n_cells)
    k = np.empty(om.n_cells)
    _lib().orc_csf_smooth_curvature(om.ref, _p(geom.xc), _p(np.ascontiguousarray(alpha_hat, float)),
                                    _p(np.ascontiguousarray(n, float)), _p(np.ascontiguousarray(kraw, float)),
                                    _p(ks), _p(k))
    return ks, k
