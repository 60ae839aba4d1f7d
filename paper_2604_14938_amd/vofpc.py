"""ctypes binding of ``libvofpc.so`` (argument marshalling only).

Every function here forwards to the C entry point of the same name; all the
work runs in the library's HIP kernels.  Device buffers are torch tensors on
the context's device (their ``data_ptr()`` is passed through); the stream is
torch's current stream unless another is given.  There is no fallback: if the
library is missing or fails to load, importing raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvofpc.so")

# per-cell outcome codes
CELL_OK, CELL_NOT_MIXED, CELL_LEARNED_FALLBACK, CELL_DEGENERATE, CELL_MAX_ITER, CELL_G_SINGULAR, \
    CELL_BAD_INPUT, CELL_NO_ROOT = range(8)
BRACKET_PLAIN, BRACKET_HINT = 0, 1
VERTEX_IDW, VERTEX_MEAN = 0, 1
SCOPE_BAND, SCOPE_ALL = 0, 1
GRAD_MODIFIED, GRAD_STANDARD, GRAD_PRINTED = 0, 1, 2
GRAD_W_INV_DIST, GRAD_W_INV_DIST2, GRAD_VERTEX_STENCIL = 0x10, 0x20, 0x40   # flags or-ed into the variant

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
D = ctypes.c_double


class VofpcError(RuntimeError):
    pass


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_cells", I64), ("n_faces", I64), ("n_verts", I64),
                ("cell_face_off", P), ("cell_face", P), ("face_vert_off", P), ("face_vert", P),
                ("face_owner", P), ("face_neigh", P), ("face_bc", P), ("vert_xyz", P)]


class ReconOpts(ctypes.Structure):
    _fields_ = [("eps_mixed", D), ("tol_rel", D), ("max_iter", I32), ("vertex_mode", I32),
                ("fixed_iso", I32), ("bracket", I32), ("iso", D), ("phi_vertex", P)]


class CInterface(ctypes.Structure):
    _fields_ = [("s", P), ("n", P), ("A", P), ("d", P), ("alpha_got", P), ("status", P), ("iters", P),
                ("cap", I64)]


class ExtrapOpts(ctypes.Structure):
    _fields_ = [("eps_mixed", ctypes.c_double), ("layers", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("tol", ctypes.c_double)]


class StepArgs(ctypes.Structure):
    _fields_ = [("alpha", P), ("T", P), ("T_bface", P), ("T_sat", D), ("k_l", D), ("k_v", D), ("h_lv", D),
                ("opts", ReconOpts), ("hint_lo", P), ("hint_hi", P), ("mixed_idx", P), ("band_idx", P),
                ("counts", P), ("itf", CInterface), ("gradT", P), ("grad_status", P), ("mdot", P), ("Qdot", P),
                ("mlp", P), ("delta_scale", D)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_14938_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "vofpc_last_error": ([], ctypes.c_char_p),
        "vofpc_version": ([], ctypes.c_int),
        "vofpc_ctx_create": ([ctypes.c_int, P, P], ctypes.c_int),
        "vofpc_ctx_set_stream": ([P, P], ctypes.c_int),
        "vofpc_ctx_destroy": ([P], ctypes.c_int),
        "vofpc_mesh_upload": ([P, P, P], ctypes.c_int),
        "vofpc_mesh_free": ([P], ctypes.c_int),
        "vofpc_mesh_info": ([P, P], ctypes.c_int),
        "vofpc_mesh_geometry": ([P, P, P, P, P], ctypes.c_int),
        "vofpc_compact": ([P, P, P, D, P, P, P], ctypes.c_int),
        "vofpc_compact_noalloc": ([P, P, P, D, P, P, P], ctypes.c_int),
        "vofpc_recon_opts_default": ([P], ctypes.c_int),
        "vofpc_reconstruct": ([P, P, P, P, P, P, P, P, P], ctypes.c_int),
        "vofpc_grad_T": ([P, P, P, P, D, P, P, P, I32, I32, P, P], ctypes.c_int),
        "vofpc_mass_transfer": ([P, P, P, P, P, P, P, P, P, D, D, D, P, P, P, P], ctypes.c_int),
        "vofpc_step": ([P, P, P], ctypes.c_int),
        "vofpc_graph_create": ([P, P, P, P], ctypes.c_int),
        "vofpc_graph_launch": ([P], ctypes.c_int),
        "vofpc_graph_destroy": ([P], ctypes.c_int),
        "vofpc_mlp_param_count": ([], ctypes.c_int),
        "vofpc_mlp_create": ([P, I64, P], ctypes.c_int),
        "vofpc_mlp_destroy": ([P], ctypes.c_int),
        "vofpc_mlp_set_params": ([P, P, I64], ctypes.c_int),
        "vofpc_mlp_get_params": ([P, P, I64], ctypes.c_int),
        "vofpc_mlp_forward": ([P, P, P, I64, P], ctypes.c_int),
        "vofpc_mlp_gradient": ([P, P, P, P, I64, P, P], ctypes.c_int),
        "vofpc_mlp_train_step": ([P, P, P, P, I64, ctypes.c_float, P], ctypes.c_int),
        "vofpc_features": ([P, P, P, P, P, P, P, P, I64], ctypes.c_int),
        "vofpc_mlp_bracket": ([P, P, P, P, P, I64, D, P, P], ctypes.c_int),
        "vofpc_reconstruct_learned": ([P, P, P, P, P, P, P, D, P, P, P], ctypes.c_int),
        "vofpc_mesh_concat": ([P, P, ctypes.c_int32, P], ctypes.c_int),
        "vofpc_mesh_classes": ([P, P, P, P], ctypes.c_int),
        "vofpc_mesh_set_tune": ([P, P], ctypes.c_int),
        "vofpc_ctx_time_classes": ([P, ctypes.c_int32], ctypes.c_int),
        "vofpc_ctx_overlap_classes": ([P, ctypes.c_int32], ctypes.c_int),
        "vofpc_ctx_class_ms": ([P, P], ctypes.c_int),
        "vofpc_extrap_opts_default": ([P], ctypes.c_int),
        "vofpc_extrapolate": ([P, P, P, P, P, D, P, P, P, P, P, P, P], ctypes.c_int),
        "vofpc_autotune": ([P, P, P, P, ctypes.c_char_p, P, P], ctypes.c_int),
        "vofpc_robin": ([P, P, P, P, P, P, P, D, D, P, I64, P, P, P, P, P], ctypes.c_int),
        "vofpc_csf_opts_default": ([P], ctypes.c_int),
        "vofpc_curvature": ([P, P, P, P, P, P, P, P, P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def _check(rc: int, what: str) -> None:
    if rc != 0:
        msg = lib.vofpc_last_error().decode(errors="replace")
        raise VofpcError(f"{what} failed ({rc}): {msg}")


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if not t.is_cuda:
            raise ValueError("device buffers must be GPU tensors")
        if not t.is_contiguous():
            raise ValueError("device buffers must be contiguous")
        return t.data_ptr()
    return int(t)


def _dev_f64(t, n=None, dev=None):
    if t.dtype != torch.float64:
        raise TypeError("expected a float64 tensor")
    if n is not None and t.numel() < n:
        raise ValueError(f"tensor too small ({t.numel()} < {n})")
    if dev is not None and t.device != dev:
        raise ValueError("tensor on the wrong device")
    return t


class Context:
    """A library context bound to one device and one HIP stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.device = torch.device("cuda", device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        h = P()
        _check(lib.vofpc_ctx_create(device, self.stream.cuda_stream, ctypes.byref(h)), "vofpc_ctx_create")
        self.h = h

    def set_stream(self, stream: torch.cuda.Stream) -> None:
        self.stream = stream
        _check(lib.vofpc_ctx_set_stream(self.h, stream.cuda_stream), "vofpc_ctx_set_stream")

    def overlap_classes(self, enable: bool = True) -> None:
        """Run the classes of a bucketed reconstruction side by side on two
        streams (the default) or in turn (vofpc_ctx_overlap_classes)."""
        _check(lib.vofpc_ctx_overlap_classes(self.h, int(bool(enable))), "vofpc_ctx_overlap_classes")

    def time_classes(self, enable: bool = True) -> None:
        """Record an event pair around each class kernel of later eager
        reconstructions on this context (vofpc_ctx_time_classes)."""
        _check(lib.vofpc_ctx_time_classes(self.h, int(bool(enable))), "vofpc_ctx_time_classes")

    def class_ms(self) -> tuple:
        """Durations (ms) of the class kernels of the latest reconstruction
        and of their bracket passes (learned form), -1 where none ran
        (vofpc_ctx_class_ms): (kernels[4], passes[4])."""
        a = (ctypes.c_float * 8)()
        _check(lib.vofpc_ctx_class_ms(self.h, a), "vofpc_ctx_class_ms")
        v = [float(x) for x in a]
        return v[:4], v[4:]

    def close(self) -> None:
        if getattr(self, "h", None):
            lib.vofpc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover - best effort
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    """A mesh uploaded to the device; built from any object with the CSR
    attributes of :class:`vofpc_mesh_desc` (host numpy arrays)."""

    def __init__(self, ctx: Context, m, _handle=None):
        self.ctx = ctx
        if _handle is not None:   # built by the library (concat)
            self.h = _handle
            info = self.info()
            self.n_cells, self.n_faces, self.n_verts = info["n_cells"], info["n_faces"], info["n_verts"]
            return
        arrs = dict(
            cfo=np.ascontiguousarray(m.cell_face_off, np.int64), cf=np.ascontiguousarray(m.cell_face, np.int32),
            fvo=np.ascontiguousarray(m.face_vert_off, np.int64), fv=np.ascontiguousarray(m.face_vert, np.int32),
            ow=np.ascontiguousarray(m.face_owner, np.int32), ne=np.ascontiguousarray(m.face_neigh, np.int32),
            bc=np.ascontiguousarray(m.face_bc, np.int8),
            xyz=np.ascontiguousarray(np.asarray(m.vert_xyz, np.float64).reshape(3, -1)),
        )
        desc = MeshDesc(int(m.n_cells), int(m.n_faces), int(m.n_verts),
                        *(a.ctypes.data for a in (arrs["cfo"], arrs["cf"], arrs["fvo"], arrs["fv"], arrs["ow"],
                                                  arrs["ne"], arrs["bc"], arrs["xyz"])))
        h = P()
        _check(lib.vofpc_mesh_upload(ctx.h, ctypes.byref(desc), ctypes.byref(h)), "vofpc_mesh_upload")
        self.h = h
        self.n_cells, self.n_faces, self.n_verts = int(m.n_cells), int(m.n_faces), int(m.n_verts)

    @classmethod
    def concat(cls, ctx: Context, meshes: list) -> "Mesh":
        """Disjoint union of uploaded meshes (see vofpc_mesh_concat)."""
        arr = (P * len(meshes))(*[m.h for m in meshes])
        h = P()
        _check(lib.vofpc_mesh_concat(ctx.h, arr, len(meshes), ctypes.byref(h)), "vofpc_mesh_concat")
        return cls(ctx, None, _handle=h)

    def classes(self) -> dict:
        cells = (ctypes.c_int64 * 4)()
        tune = (ctypes.c_int32 * 4)()
        b = ctypes.c_int32()
        _check(lib.vofpc_mesh_classes(self.h, cells, tune, ctypes.byref(b)), "vofpc_mesh_classes")
        return {"cells": list(cells), "tune": list(tune), "bucketed": bool(b.value)}

    def set_tune(self, tune) -> None:
        """Reconstruction kernel flavour per class (vofpc_mesh_set_tune):
        3 or 4 (one cell per wavefront), 10 + G (G lanes per cell)."""
        t = (ctypes.c_int32 * 4)(*[int(x) for x in tune])
        _check(lib.vofpc_mesh_set_tune(self.h, t), "vofpc_mesh_set_tune")

    def info(self) -> dict:
        a = (ctypes.c_int64 * 8)()
        _check(lib.vofpc_mesh_info(self.h, a), "vofpc_mesh_info")
        keys = ["n_cells", "n_faces", "n_verts", "max_faces", "max_verts", "max_face_verts", "max_edges", "bytes"]
        return dict(zip(keys, list(a)))

    def geometry(self):
        dev = self.ctx.device
        V = torch.empty(self.n_cells, dtype=torch.float64, device=dev)
        xc = torch.empty(3, self.n_cells, dtype=torch.float64, device=dev)
        Sf = torch.empty(3, self.n_faces, dtype=torch.float64, device=dev)
        xf = torch.empty(3, self.n_faces, dtype=torch.float64, device=dev)
        _check(lib.vofpc_mesh_geometry(self.h, _ptr(V), _ptr(xc), _ptr(Sf), _ptr(xf)), "vofpc_mesh_geometry")
        return V, xc, Sf, xf

    def close(self) -> None:
        if getattr(self, "h", None):
            lib.vofpc_mesh_free(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


def recon_opts(**kw) -> ReconOpts:
    o = ReconOpts()
    _check(lib.vofpc_recon_opts_default(ctypes.byref(o)), "vofpc_recon_opts_default")
    phi = kw.pop("phi_vertex", None)
    for k, v in kw.items():
        setattr(o, k, v)
    o.phi_vertex = _ptr(phi)
    o._phi_keep = phi  # keep the tensor alive with the struct
    return o


@dataclass
class Interface:
    s: torch.Tensor
    n: torch.Tensor
    A: torch.Tensor
    d: torch.Tensor
    alpha_got: torch.Tensor
    status: torch.Tensor
    iters: torch.Tensor

    @classmethod
    def empty(cls, cap: int, device) -> "Interface":
        f = dict(dtype=torch.float64, device=device)
        return cls(torch.empty(cap, **f), torch.empty(3, cap, **f), torch.empty(cap, **f), torch.empty(cap, **f),
                   torch.empty(cap, **f), torch.empty(cap, dtype=torch.int32, device=device),
                   torch.empty(cap, dtype=torch.int32, device=device))

    @property
    def cap(self) -> int:
        return self.s.numel()

    def c(self) -> CInterface:
        return CInterface(_ptr(self.s), _ptr(self.n), _ptr(self.A), _ptr(self.d), _ptr(self.alpha_got),
                          _ptr(self.status), _ptr(self.iters), self.cap)


def compact(ctx: Context, mesh: Mesh, alpha, mixed_idx, band_idx, counts, eps_mixed: float = 1e-8) -> None:
    _check(lib.vofpc_compact(ctx.h, mesh.h, _ptr(alpha), eps_mixed, _ptr(mixed_idx), _ptr(band_idx), _ptr(counts)),
           "vofpc_compact")


def compact_noalloc(ctx: Context, mesh: Mesh, alpha, mixed_idx, band_idx, counts, eps_mixed: float = 1e-8) -> None:
    """vofpc_compact on the library's fixed per-GPU scratch (allocates nothing)."""
    _check(lib.vofpc_compact_noalloc(ctx.h, mesh.h, _ptr(alpha), eps_mixed, _ptr(mixed_idx), _ptr(band_idx),
                                     _ptr(counts)), "vofpc_compact_noalloc")


def reconstruct(ctx: Context, mesh: Mesh, alpha, mixed_idx, counts, itf: Interface, opts: ReconOpts | None = None,
                hint_lo=None, hint_hi=None) -> None:
    opts = opts or recon_opts()
    ci = itf.c()
    _check(lib.vofpc_reconstruct(ctx.h, mesh.h, _ptr(alpha), _ptr(mixed_idx), _ptr(counts), ctypes.byref(opts),
                                 _ptr(hint_lo), _ptr(hint_hi), ctypes.byref(ci)), "vofpc_reconstruct")


def reconstruct_learned(ctx: Context, mesh: Mesh, alpha, mixed_idx, counts, itf: Interface, mlp: "Mlp",
                        delta_scale: float, opts: ReconOpts | None = None, hint_lo=None, hint_hi=None) -> None:
    opts = opts or recon_opts()
    ci = itf.c()
    _check(lib.vofpc_reconstruct_learned(ctx.h, mesh.h, _ptr(alpha), _ptr(mixed_idx), _ptr(counts), ctypes.byref(opts),
                                         mlp.h, float(delta_scale), _ptr(hint_lo), _ptr(hint_hi), ctypes.byref(ci)),
           "vofpc_reconstruct_learned")


def autotune(ctx: Context, mesh: Mesh, alpha, opts: ReconOpts | None = None, cache_path: str | None = None):
    """Pick the reconstruction kernel flavour per class by timing (see
    vofpc_autotune); returns (flavours per class, taken from the cache)."""
    choice = (ctypes.c_int32 * 4)()
    hit = ctypes.c_int32()
    _check(lib.vofpc_autotune(ctx.h, mesh.h, _ptr(alpha), ctypes.byref(opts) if opts is not None else None,
                              cache_path.encode() if cache_path else None, choice, ctypes.byref(hit)),
           "vofpc_autotune")
    return list(choice), bool(hit.value)


def extrap_opts(**kw) -> ExtrapOpts:
    o = ExtrapOpts()
    _check(lib.vofpc_extrap_opts_default(ctypes.byref(o)), "vofpc_extrap_opts_default")
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def extrapolate(ctx: Context, mesh: Mesh, alpha, T, T_bface, T_sat: float, mixed_idx, counts, itf: Interface,
                gradT_l, gradT_v, report=None, opts: ExtrapOpts | None = None) -> None:
    """Phase gradients by pseudo-time extrapolation (see vofpc_extrapolate)."""
    ci = itf.c()
    _check(lib.vofpc_extrapolate(ctx.h, mesh.h, _ptr(alpha), _ptr(T), _ptr(T_bface), float(T_sat), _ptr(mixed_idx),
                                 _ptr(counts), ctypes.byref(ci), ctypes.byref(opts) if opts is not None else None,
                                 _ptr(gradT_l), _ptr(gradT_v), _ptr(report)), "vofpc_extrapolate")


class CsfOpts(ctypes.Structure):
    _fields_ = [("n_smooth", ctypes.c_int32), ("sigma", ctypes.c_double)]


def csf_opts(**kw) -> CsfOpts:
    o = CsfOpts()
    _check(lib.vofpc_csf_opts_default(ctypes.byref(o)), "vofpc_csf_opts_default")
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def curvature(ctx: Context, mesh: Mesh, alpha, alpha_hat, n, kappa, kappa_raw=None, force=None,
              opts: CsfOpts | None = None) -> None:
    """Surface-tension curvature chain (see vofpc_curvature)."""
    _check(lib.vofpc_curvature(ctx.h, mesh.h, _ptr(alpha), ctypes.byref(opts) if opts is not None else None,
                               _ptr(alpha_hat), _ptr(n), _ptr(kappa_raw), _ptr(kappa), _ptr(force)),
           "vofpc_curvature")


def robin(ctx: Context, mesh: Mesh, alpha, mixed_idx, band_idx, counts, itf: Interface, k_l: float, k_v: float,
          a_diag=None, face_idx=None, face_a=None, face_d=None, face_area=None, n_face=None) -> None:
    """Interface coupling coefficients of the detached faces (see vofpc_robin).
    face_cap is the length of face_idx (or face_area, or face_a's rows)."""
    cap = 0
    for t, rows in ((face_idx, 1), (face_area, 1), (face_a, 2), (face_d, 2)):
        if t is not None:
            cap = t.numel() // rows
            break
    ci = itf.c()
    _check(lib.vofpc_robin(ctx.h, mesh.h, _ptr(alpha), _ptr(mixed_idx), _ptr(band_idx), _ptr(counts),
                           ctypes.byref(ci), float(k_l), float(k_v), _ptr(a_diag), int(cap), _ptr(face_idx),
                           _ptr(face_a), _ptr(face_d), _ptr(face_area), _ptr(n_face)), "vofpc_robin")


def grad_T(ctx: Context, mesh: Mesh, T, T_bface, T_sat: float, alpha, band_idx, counts, grad, status=None,
           scope: int = SCOPE_BAND, variant: int = GRAD_MODIFIED) -> None:
    _check(lib.vofpc_grad_T(ctx.h, mesh.h, _ptr(T), _ptr(T_bface), float(T_sat), _ptr(alpha), _ptr(band_idx),
                            _ptr(counts), scope, variant, _ptr(grad), _ptr(status)), "vofpc_grad_T")


def mass_transfer(ctx: Context, mesh: Mesh, alpha, mixed_idx, counts, itf: Interface, gradT, k_l, k_v, h_lv,
                  mdot, Qdot, gradT_l=None, gradT_v=None, mdot_cells=None, Qdot_cells=None) -> None:
    ci = itf.c()
    _check(lib.vofpc_mass_transfer(ctx.h, mesh.h, _ptr(alpha), _ptr(mixed_idx), _ptr(counts), ctypes.byref(ci),
                                   _ptr(gradT), _ptr(gradT_l), _ptr(gradT_v), float(k_l), float(k_v), float(h_lv),
                                   _ptr(mdot), _ptr(Qdot), _ptr(mdot_cells), _ptr(Qdot_cells)), "vofpc_mass_transfer")


class Mlp:
    """The bracket network on a context's device."""

    def __init__(self, ctx: Context, max_batch: int = 1 << 16):
        self.ctx = ctx
        self.n_params = int(lib.vofpc_mlp_param_count())
        h = P()
        _check(lib.vofpc_mlp_create(ctx.h, int(max_batch), ctypes.byref(h)), "vofpc_mlp_create")
        self.h = h
        self.max_batch = int(max_batch)

    def set_params(self, v: np.ndarray) -> None:
        v = np.ascontiguousarray(v, np.float32)
        _check(lib.vofpc_mlp_set_params(self.h, v.ctypes.data, v.size), "vofpc_mlp_set_params")

    def get_params(self) -> np.ndarray:
        v = np.empty(self.n_params, np.float32)
        _check(lib.vofpc_mlp_get_params(self.h, v.ctypes.data, v.size), "vofpc_mlp_get_params")
        return v

    def forward(self, X, Y) -> None:
        _check(lib.vofpc_mlp_forward(self.ctx.h, self.h, _ptr(X), X.shape[0], _ptr(Y)), "vofpc_mlp_forward")

    def gradient(self, X, T, grad=None, loss=None) -> None:
        _check(lib.vofpc_mlp_gradient(self.ctx.h, self.h, _ptr(X), _ptr(T), X.shape[0], _ptr(grad), _ptr(loss)),
               "vofpc_mlp_gradient")

    def train_step(self, X, T, lr: float, loss=None) -> None:
        _check(lib.vofpc_mlp_train_step(self.ctx.h, self.h, _ptr(X), _ptr(T), X.shape[0], float(lr), _ptr(loss)),
               "vofpc_mlp_train_step")

    def bracket(self, features, phi_range, counts, cap, delta_scale, hint_lo, hint_hi) -> None:
        _check(lib.vofpc_mlp_bracket(self.ctx.h, self.h, _ptr(features), _ptr(phi_range), _ptr(counts), int(cap),
                                     float(delta_scale), _ptr(hint_lo), _ptr(hint_hi)), "vofpc_mlp_bracket")

    def close(self) -> None:
        if getattr(self, "h", None):
            lib.vofpc_mlp_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


def features(ctx: Context, mesh: Mesh, alpha, mixed_idx, counts, feat, phi_range, opts: ReconOpts | None = None):
    _check(lib.vofpc_features(ctx.h, mesh.h, _ptr(alpha), _ptr(mixed_idx), _ptr(counts),
                              ctypes.byref(opts) if opts is not None else None, _ptr(feat), _ptr(phi_range),
                              feat.shape[0]), "vofpc_features")


class StepBuffers:
    """Every device buffer of one step, sized for a mesh (capacity n_cells).
    With `mlp` set the step runs the learned form (the reconstruction kernel
    runs the network; hint_lo/hint_hi receive its brackets)."""

    def __init__(self, ctx: Context, mesh: Mesh, alpha, T, T_bface, T_sat, k_l, k_v, h_lv,
                 opts: ReconOpts | None = None, hint_lo=None, hint_hi=None, mlp: "Mlp | None" = None,
                 delta_scale: float = 0.0):
        dev = ctx.device
        N = mesh.n_cells
        self.alpha, self.T, self.T_bface = alpha, T, T_bface
        self.T_sat, self.k_l, self.k_v, self.h_lv = float(T_sat), float(k_l), float(k_v), float(h_lv)
        self.opts = opts or recon_opts()
        self.hint_lo, self.hint_hi = hint_lo, hint_hi
        i32 = dict(dtype=torch.int32, device=dev)
        self.mixed_idx = torch.zeros(N, **i32)
        self.band_idx = torch.zeros(N, **i32)
        self.counts = torch.zeros(2, **i32)
        self.itf = Interface.empty(N, dev)
        self.gradT = torch.zeros(3, N, dtype=torch.float64, device=dev)
        self.grad_status = torch.zeros(N, **i32)
        self.mdot = torch.zeros(N, dtype=torch.float64, device=dev)
        self.Qdot = torch.zeros(N, dtype=torch.float64, device=dev)
        self.mlp = mlp
        self.delta_scale = float(delta_scale)
        if mlp is not None:
            if self.hint_lo is None:
                self.hint_lo = torch.zeros(N, dtype=torch.float64, device=dev)
                self.hint_hi = torch.zeros(N, dtype=torch.float64, device=dev)

    def args(self) -> StepArgs:
        a = StepArgs()
        a.alpha, a.T, a.T_bface = _ptr(self.alpha), _ptr(self.T), _ptr(self.T_bface)
        a.T_sat, a.k_l, a.k_v, a.h_lv = self.T_sat, self.k_l, self.k_v, self.h_lv
        a.opts = self.opts
        a.hint_lo, a.hint_hi = _ptr(self.hint_lo), _ptr(self.hint_hi)
        a.mixed_idx, a.band_idx, a.counts = _ptr(self.mixed_idx), _ptr(self.band_idx), _ptr(self.counts)
        a.itf = self.itf.c()
        a.gradT, a.grad_status = _ptr(self.gradT), _ptr(self.grad_status)
        a.mdot, a.Qdot = _ptr(self.mdot), _ptr(self.Qdot)
        a.mlp = self.mlp.h if self.mlp is not None else None
        a.delta_scale = self.delta_scale
        return a


def step(ctx: Context, mesh: Mesh, buf: StepBuffers) -> None:
    a = buf.args()
    _check(lib.vofpc_step(ctx.h, mesh.h, ctypes.byref(a)), "vofpc_step")


class Graph:
    """One captured step (compaction, reconstruction, band gradient, mass
    transfer) replayed with :meth:`launch`."""

    def __init__(self, ctx: Context, mesh: Mesh, buf: StepBuffers):
        self.ctx, self.mesh, self.buf = ctx, mesh, buf
        a = buf.args()
        h = P()
        _check(lib.vofpc_graph_create(ctx.h, mesh.h, ctypes.byref(a), ctypes.byref(h)), "vofpc_graph_create")
        self.h = h

    def launch(self) -> None:
        _check(lib.vofpc_graph_launch(self.h), "vofpc_graph_launch")

    def close(self) -> None:
        if getattr(self, "h", None):
            lib.vofpc_graph_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass
