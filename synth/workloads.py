"""The seeded workloads: mesh + alpha + T + boundary T + material constants.

* ``hex_sphere``     16^3 hexahedra of the unit cube, vapour sphere r=0.3 at
  the centre, alpha from 64^3 sub-points per cell, T rising linearly by 5 K
  over 0.3 outside the sphere, k = 0.025 W/m/K and h_lv = 2.26e6 J/kg (the
  paper's steam conductivity and latent heat, Table 1), T_sat = 373.15 K.
* ``voronoi_bubble`` box-clipped jittered-BCC Voronoi mesh (2 n^3 seeds,
  n = 46 gives 194,672 cells, ~14.5 faces per cell), one bubble r=0.25 at the
  centre, T = T_sat + 1.25 K erf((rho - 0.25)/0.05) outside (the Scriven
  superheat of Sec. 3.3), T_sat inside.
* ``random_bubbles`` a mesh with many non-overlapping bubbles placed by random
  sequential addition (radii U[2h, 12h], clearance 2h), T rising from each
  bubble with its own slope U[1, 20] K per unit length.
* ``pipe_film``      Voronoi cells of a pipe with a wavy liquid film on the wall.
* ``batched``        several meshes with many bubbles each (a hexahedral and a
  Voronoi mesh by default), stepped as one disjoint union.
* ``learned_full``   the batched pair plus a Voronoi pipe of about 4M cells
  with the wavy film: the learned-bracket configuration at full size.
* ``static_sphere``  one vapour sphere at rest with the Scriven-like erf
  temperature profile on a hexahedral (n^3) or Voronoi (2 n^3) mesh: the
  static analogue of the gradient-anisotropy study (Sec. 3.3, gradient
  anisotropy on structured vs polyhedral meshes).
* ``multi_instance`` many independent Voronoi meshes of log-uniform sizes, each
  with one bubble moving on a circle around the vertical axis through the box
  centre (rigid rotation, one revolution over the time steps).

Temperatures are evaluated at the mean of a cell's vertices and boundary
temperatures at the mean of a face's vertices (input placement only).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import fields
from .meshes import Mesh, concat, hex_mesh, voronoi_box_mesh, voronoi_pipe_mesh

T_SAT = 373.15
K_STEAM = 0.025
H_LV = 2.26e6


@dataclass
class Workload:
    name: str
    mesh: Mesh
    alpha: np.ndarray
    T: np.ndarray
    T_bface: np.ndarray           # [NF], used on boundary faces only
    T_sat: float = T_SAT
    k_l: float = K_STEAM
    k_v: float = K_STEAM
    h_lv: float = H_LV
    meta: dict = field(default_factory=dict)

    @property
    def n_mixed(self) -> int:
        a = self.alpha
        return int(np.count_nonzero((a > 1e-8) & (a < 1.0 - 1e-8)))


def hex_sphere(n: int = 16, r: float = 0.3, K: int = 64, dT: float = 5.0) -> Workload:
    mesh = hex_mesh(n)
    c = (0.5, 0.5, 0.5)
    alpha = fields.sphere_alpha(mesh, np.array([[*c, r]]), K=K)
    T = fields.radial_linear_T(mesh.cell_vertex_mean(), c, r, dT / r, T_SAT)
    Tb = fields.radial_linear_T(mesh.face_vertex_mean(), c, r, dT / r, T_SAT)
    return Workload(f"hex{n}^3 sphere r={r}", mesh, alpha, T, Tb, meta={"spheres": np.array([[*c, r]])})


def voronoi_bubble(n: int = 46, seed: int = 2, r: float = 0.25, width: float = 0.05,
                   dT: float = 1.25, K: int = 64) -> Workload:
    mesh = voronoi_box_mesh(n, seed)
    c = (0.5, 0.5, 0.5)
    alpha = fields.sphere_alpha(mesh, np.array([[*c, r]]), K=K)
    T = fields.radial_erf_T(mesh.cell_vertex_mean(), c, r, width, dT, T_SAT)
    Tb = fields.radial_erf_T(mesh.face_vertex_mean(), c, r, width, dT, T_SAT)
    return Workload(f"voronoi {mesh.n_cells} cells bubble r={r}", mesh, alpha, T, Tb,
                    meta={"spheres": np.array([[*c, r]])})


def static_sphere(kind: str = "hex", n: int = 75, seed: int = 11, r: float = 0.25, width: float = 0.05,
                  dT: float = 1.25, K: int = 16) -> Workload:
    """A vapour sphere r at the centre of the unit cube, T = T_sat inside and
    T_sat + dT erf((rho - r)/width) outside, on hex_mesh(n) or
    voronoi_box_mesh(n, seed) (2 n^3 cells)."""
    mesh = hex_mesh(n) if kind == "hex" else voronoi_box_mesh(n, seed)
    c = (0.5, 0.5, 0.5)
    alpha = fields.sphere_alpha(mesh, np.array([[*c, r]]), K=K)
    T = fields.radial_erf_T(mesh.cell_vertex_mean(), c, r, width, dT, T_SAT)
    Tb = fields.radial_erf_T(mesh.face_vertex_mean(), c, r, width, dT, T_SAT)
    return Workload(f"static sphere on {kind} {mesh.n_cells} cells", mesh, alpha, T, Tb,
                    meta={"spheres": np.array([[*c, r]]), "centre": np.array(c), "r": r, "width": width,
                          "dT": dT, "kind": kind})


def random_bubbles(mesh: Mesh, seed: int, n_max: int = 1000, K: int = 16,
                   r_lo_h: float = 2.0, r_hi_h: float = 12.0) -> Workload:
    rng = np.random.default_rng(seed)
    h = mesh.h
    sph = fields.rsa_spheres(rng, n_max, r_lo_h * h, r_hi_h * h, 2.0 * h)
    if len(sph) == 0:
        raise ValueError(f"random_bubbles: no bubble of radius up to {r_hi_h} h fits the box")
    slopes = rng.uniform(1.0, 20.0, len(sph))
    alpha = fields.sphere_alpha(mesh, sph, K=K)
    T = fields.nearest_bubble_T(mesh.cell_vertex_mean(), sph, slopes, T_SAT)
    Tb = fields.nearest_bubble_T(mesh.face_vertex_mean(), sph, slopes, T_SAT)
    return Workload(f"{mesh.kind} {mesh.n_cells} cells, {len(sph)} bubbles", mesh, alpha, T, Tb,
                    meta={"spheres": sph, "slopes": slopes, "n_bubbles": len(sph)})


def pipe_film(n_radial: int = 40, seed: int = 4, R: float = 1.0, K: int = 16) -> Workload:
    L = 52.0 / 9.5 * R
    mesh = voronoi_pipe_mesh(n_radial, R, L, seed)
    d0, amp, waves = 0.1 * R, 0.3, 5.0
    alpha = fields.film_alpha(mesh, R, d0, amp, waves, L, K=K)
    T = fields.film_T(mesh.cell_vertex_mean(), R, d0, amp, waves, L, 1.0, T_SAT)
    Tb = fields.film_T(mesh.face_vertex_mean(), R, d0, amp, waves, L, 1.0, T_SAT)
    return Workload(f"pipe {mesh.n_cells} cells film", mesh, alpha, T, Tb,
                    meta={"R": R, "L": L, "d0": d0, "amp": amp, "waves": waves})


def concat_workloads(wls: list, name: str | None = None) -> Workload:
    """One workload over the disjoint union of the workloads' meshes (their
    material constants must agree)."""
    w0 = wls[0]
    for w in wls[1:]:
        assert (w.T_sat, w.k_l, w.k_v, w.h_lv) == (w0.T_sat, w0.k_l, w0.k_v, w0.h_lv)
    mesh = concat([w.mesh for w in wls])
    return Workload(name or " + ".join(w.name for w in wls), mesh,
                    np.concatenate([w.alpha for w in wls]), np.concatenate([w.T for w in wls]),
                    np.concatenate([w.T_bface for w in wls]), w0.T_sat, w0.k_l, w0.k_v, w0.h_lv,
                    meta={"parts": [w.name for w in wls],
                          "cell_offsets": np.cumsum([0] + [w.mesh.n_cells for w in wls])})


def batched(hex_n: int = 128, vor_n: int = 79, seed: int = 3, n_max: int = 1000, K: int = 16,
            r_hi_h: float = 12.0) -> list:
    """A hexahedral mesh (hex_n^3 cells) and a jittered-BCC Voronoi mesh
    (2 vor_n^3 cells), each with up to n_max bubbles r ~ U[2h, r_hi_h h] placed
    by random sequential addition (the count that fits is used).  Returns the
    two workloads; step them as one with ``concat_workloads``."""
    out = []
    for i, m in enumerate((hex_mesh(hex_n), voronoi_box_mesh(vor_n, seed))):
        out.append(random_bubbles(m, seed=seed + 17 * i, n_max=n_max, K=K, r_hi_h=r_hi_h))
    return out


def learned_full(hex_n: int = 128, vor_n: int = 79, pipe_radial: int = 98, seed: int = 3, log=None) -> list:
    """The batched pair (hex_n^3 hexahedra and 2 vor_n^3 Voronoi cells, random
    bubbles) and a Voronoi pipe with `pipe_radial` seeds across its diameter
    (98 gives 4,043,057 cells) carrying the wavy film; returns the three
    workloads, stepped as one disjoint union."""
    out = batched(hex_n=hex_n, vor_n=vor_n, seed=seed)
    if log:
        log(f"batched pair: {[w.mesh.n_cells for w in out]} cells, {[w.n_mixed for w in out]} mixed")
    out.append(pipe_film(n_radial=pipe_radial, seed=4))
    if log:
        log(f"pipe: {out[-1].mesh.n_cells} cells, {out[-1].n_mixed} mixed")
    return out


_MESH_ARRAYS = ("cell_face_off", "cell_face", "face_vert_off", "face_vert", "face_owner", "face_neigh", "face_bc",
                "vert_xyz")


def save_parts(path: str, wls: list) -> None:
    """Write workloads (meshes, fields, constants; not `meta`) to one .npz
    file, no pickled objects."""
    arr = {"n_parts": np.array(len(wls))}
    for i, w in enumerate(wls):
        m = w.mesh
        for k in _MESH_ARRAYS:
            arr[f"p{i}_{k}"] = getattr(m, k)
        arr[f"p{i}_sizes"] = np.array([m.n_cells, m.n_faces, m.n_verts], np.int64)
        arr[f"p{i}_h"] = np.array(m.h)
        arr[f"p{i}_kind"] = np.array(m.kind)
        arr[f"p{i}_name"] = np.array(w.name)
        arr[f"p{i}_alpha"], arr[f"p{i}_T"], arr[f"p{i}_Tb"] = w.alpha, w.T, w.T_bface
        arr[f"p{i}_const"] = np.array([w.T_sat, w.k_l, w.k_v, w.h_lv])
        if "n_bubbles" in w.meta:
            arr[f"p{i}_n_bubbles"] = np.array(w.meta["n_bubbles"])
    tmp = path + ".tmp.npz"
    np.savez(tmp, **arr)
    import os
    os.replace(tmp, path)


def load_parts(path: str) -> list:
    """Read workloads written by `save_parts`."""
    z = np.load(path, allow_pickle=False)
    out = []
    for i in range(int(z["n_parts"])):
        N, NF, NV = (int(x) for x in z[f"p{i}_sizes"])
        m = Mesh(N, NF, NV, *[z[f"p{i}_{k}"] for k in _MESH_ARRAYS], kind=str(z[f"p{i}_kind"]),
                 h=float(z[f"p{i}_h"]))
        c = z[f"p{i}_const"]
        meta = {"n_bubbles": int(z[f"p{i}_n_bubbles"])} if f"p{i}_n_bubbles" in z else {}
        out.append(Workload(str(z[f"p{i}_name"]), m, z[f"p{i}_alpha"], z[f"p{i}_T"], z[f"p{i}_Tb"],
                            float(c[0]), float(c[1]), float(c[2]), float(c[3]), meta=meta))
    return out


def _log_uniform_sizes(rng, n_inst: int, n_lo: float, n_hi: float) -> list:
    N = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), n_inst))
    return [max(2, int(round((x / 2.0) ** (1.0 / 3.0)))) for x in N]   # BCC seeds per axis


def multi_instance(n_inst: int = 64, n_lo: float = 1e4, n_hi: float = 5e5, seed: int = 5,
                   steps: int = 100, K: int = 16, width: float = 0.05, dT: float = 1.25, log=None):
    """Meshes and per-step fields of the multi-instance batch: instance i is a
    box-clipped Voronoi mesh of about N_i = exp(U[ln n_lo, ln n_hi]) cells with
    one bubble r ~ U[0.10, 0.20] whose centre sits 0.15 from the vertical axis
    through (0.5, 0.5) and turns once around it over `steps` steps; T is the
    erf profile of ``voronoi_bubble`` around the moving centre.

    Returns (meshes, radii, phases, field) where field(i, t) gives the
    Workload of instance i at step t.  `log` (optional) is called with a line
    of progress after each mesh."""
    rng = np.random.default_rng(seed)
    ns = _log_uniform_sizes(rng, n_inst, n_lo, n_hi)
    radii = rng.uniform(0.10, 0.20, n_inst)
    phases = rng.uniform(0.0, 2.0 * np.pi, n_inst)
    seeds = rng.integers(1 << 30, size=n_inst)
    meshes = []
    for i, (n, sd) in enumerate(zip(ns, seeds)):
        meshes.append(voronoi_box_mesh(n, int(sd)))
        if log is not None:
            log(f"instance mesh {i + 1}/{n_inst}: {meshes[-1].n_cells} cells")

    def field(i: int, t: int) -> Workload:
        m = meshes[i]
        th = phases[i] + 2.0 * np.pi * t / steps
        c = (0.5 + 0.15 * np.cos(th), 0.5 + 0.15 * np.sin(th), 0.5)
        r = radii[i]
        alpha = fields.sphere_alpha(m, np.array([[*c, r]]), K=K)
        T = fields.radial_erf_T(m.cell_vertex_mean(), c, r, width, dT, T_SAT)
        Tb = fields.radial_erf_T(m.face_vertex_mean(), c, r, width, dT, T_SAT)
        return Workload(f"instance {i} step {t}", m, alpha, T, Tb, meta={"spheres": np.array([[*c, r]])})

    return meshes, radii, phases, field
