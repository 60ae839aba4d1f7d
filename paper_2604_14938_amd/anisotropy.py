"""Angular analysis of an interface field around a sphere (Sec. 3.3, the
temperature-gradient anisotropy study): the cells next to the interface in
an equatorial slab, their azimuth about the sphere's axis, the magnitude
binned by azimuth, the min/max ratio of the bins and the azimuthal Fourier
amplitudes of the binned profile in percent of its mean.

Host post-processing of the library's outputs (numpy, no device work).
"""
from __future__ import annotations

import numpy as np


def interface_cells(alpha: np.ndarray, face_owner: np.ndarray, face_neigh: np.ndarray) -> np.ndarray:
    """Liquid cells (alpha >= 1/2) with a face whose cells lie on opposite
    sides of alpha = 1/2: the cells whose gradient stencil is modified."""
    q = face_neigh
    inner = q >= 0
    o, q = face_owner[inner], q[inner]
    cross = (alpha[o] - 0.5) * (alpha[q] - 0.5) < 0.0
    cells = np.union1d(o[cross], q[cross])
    return cells[alpha[cells] >= 0.5]


def erf_profile_gradient(points: np.ndarray, centre, r: float, width: float, dT: float) -> np.ndarray:
    """|dT/drho| of T_sat + dT erf((rho - r)/width) at points [3, n] (the
    analytic magnitude the computed gradient is compared with)."""
    rho = np.linalg.norm(points - np.asarray(centre, float)[:, None], axis=0)
    return 2.0 * dT / (np.sqrt(np.pi) * width) * np.exp(-((rho - r) / width) ** 2)


def polar(xc: np.ndarray, value: np.ndarray, cells: np.ndarray, centre, slab: float, n_bins: int = 36,
          m_max: int = 8) -> dict:
    """Bin value[cells] by the azimuth of xc[:, cells] - centre about z, over
    the cells with |z - z_c| < slab.  Returns the bin means, the min/max
    ratio of the bins, and the Fourier amplitude of modes 1..m_max of the
    binned profile in percent of its mean (mode m: 2 |sum_k b_k e^{-i m
    theta_k}| / n_bins)."""
    c = np.asarray(centre, float)
    rel = xc[:, cells] - c[:, None]
    sel = np.abs(rel[2]) < slab
    th = np.arctan2(rel[1, sel], rel[0, sel])
    v = value[cells][sel]
    k = np.minimum(((th + np.pi) / (2 * np.pi) * n_bins).astype(int), n_bins - 1)
    cnt = np.bincount(k, minlength=n_bins)
    if (cnt == 0).any():
        raise ValueError(f"polar: {int((cnt == 0).sum())} empty azimuth bins; use fewer bins or a wider slab")
    b = np.bincount(k, weights=v, minlength=n_bins) / cnt
    theta = -np.pi + (np.arange(n_bins) + 0.5) * 2 * np.pi / n_bins
    mean = b.mean()
    modes = [float(2.0 * abs(np.sum(b * np.exp(-1j * m * theta))) / n_bins / mean * 100.0)
             for m in range(1, m_max + 1)]
    return dict(n_cells=int(sel.sum()), mean=float(mean), min_max=float(b.min() / b.max()), bins=b,
                modes_pct=modes, m4_pct=modes[3] if m_max >= 4 else None)


def polar_coarsened(xc, value, cells, centre, slab, n_bins, min_bins: int = 12, m_max: int = 8) -> dict | None:
    """polar() with the bin count halved until no bin is empty (sparse sets
    such as the mixed cells of one phase); None below min_bins."""
    while n_bins >= min_bins:
        try:
            P = polar(xc, value, cells, centre, slab, n_bins, m_max)
            P["n_bins"] = n_bins
            return P
        except ValueError:
            n_bins //= 2
    return None


# --------------------------------------------------------------- the study
VARIANTS = ("modified", "standard", "inv_dist", "inv_dist2", "vertex")


def _variant_code(V, name: str) -> int:
    return {"modified": V.GRAD_MODIFIED, "standard": V.GRAD_STANDARD,
            "inv_dist": V.GRAD_MODIFIED | V.GRAD_W_INV_DIST,
            "inv_dist2": V.GRAD_MODIFIED | V.GRAD_W_INV_DIST2,
            "vertex": V.GRAD_MODIFIED | V.GRAD_VERTEX_STENCIL}[name]


def study(wl, n_bins: int = 36, steps: int = 20, variants=VARIANTS) -> dict:
    """Run a static-sphere workload through the library on the GPU: the
    whole step (timed by graph replays), the gradient variants over the band
    (each timed), the two-sided mass transfer with extrapolated phase
    gradients, and the angular analysis of |grad T| / |grad T|_exact over the
    liquid interface cells and of mdot over the mixed cells with an interface
    (one-sided: liquid cells; two-sided: all), in the equatorial slab
    |z - z_c| < h."""
    import torch

    from . import runner
    from . import vofpc as V

    meta = wl.meta
    run = runner.PathRun(wl)
    ctx, stream = run.ctx, run.ctx.stream
    run.step()
    res = run.results()
    g = run.capture()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps

    step_us = timed(g.launch, steps)
    _, xc_t, _, _ = run.mesh.geometry()
    xc = xc_t.cpu().numpy()
    N = wl.mesh.n_cells
    h = wl.mesh.h
    centre = meta["centre"]
    cells = interface_cells(wl.alpha, wl.mesh.face_owner, wl.mesh.face_neigh)
    exact = erf_profile_gradient(xc, centre, meta["r"], meta["width"], meta["dT"])
    b = run.buf
    out = dict(workload=wl.name, n_cells=int(N), n_mixed=int(res["n_mixed"]), n_band=int(res["n_band"]),
               interface_cells=int(len(cells)), step_us=step_us,
               mixed_cells_per_s=res["n_mixed"] / (step_us * 1e-6), grad={}, mdot={})
    grad = torch.zeros(3, N, dtype=torch.float64, device=run.dev)
    for name in variants:
        code = _variant_code(V, name)
        call = lambda: V.grad_T(ctx, run.mesh, run.T, run.Tb, wl.T_sat, run.alpha, b.band_idx, b.counts, grad,
                                variant=code)
        us = timed(call, steps)
        mag = np.linalg.norm(grad.cpu().numpy(), axis=0)
        P = polar(xc, mag / exact, cells, centre, h, n_bins)
        out["grad"][name] = dict(us=us, mean_ratio=P["mean"], min_max=P["min_max"], m4_pct=P["m4_pct"],
                                 modes_pct=P["modes_pct"], n_slab=P["n_cells"])
    # mass transfer: one-sided (the step's) and two-sided (extrapolated phase gradients)
    mixed = res["mixed_idx"]
    ok = res["A"] > 0
    dense = np.zeros(N)
    dense[mixed] = res["mdot"]
    liq = mixed[ok & (wl.alpha[mixed] >= 0.5)]
    P1 = polar_coarsened(xc, dense, liq, centre, h, n_bins)
    gl = torch.zeros(3, N, dtype=torch.float64, device=run.dev)
    gv = torch.zeros(3, N, dtype=torch.float64, device=run.dev)
    md = torch.zeros(N, dtype=torch.float64, device=run.dev)
    qd = torch.zeros(N, dtype=torch.float64, device=run.dev)
    rep = torch.zeros(2, dtype=torch.int32, device=run.dev)

    def two_sided():
        V.extrapolate(ctx, run.mesh, run.alpha, run.T, run.Tb, wl.T_sat, b.mixed_idx, b.counts, b.itf, gl, gv, rep)
        V.mass_transfer(ctx, run.mesh, run.alpha, b.mixed_idx, b.counts, b.itf, None, wl.k_l, wl.k_v, wl.h_lv,
                        md, qd, gradT_l=gl, gradT_v=gv)

    us2 = timed(two_sided, max(3, steps // 4))
    dense2 = np.zeros(N)
    dense2[mixed] = md[:len(mixed)].cpu().numpy()
    P2 = polar_coarsened(xc, dense2, mixed[ok], centre, h, n_bins)
    for key, P in (("one_sided", P1), ("two_sided", P2)):
        out["mdot"][key] = None if P is None else dict(
            min_max=P["min_max"], m4_pct=P["m4_pct"], modes_pct=P["modes_pct"], mean=P["mean"],
            n_slab=P["n_cells"], n_bins=P["n_bins"])
    out["mdot"]["two_sided_us"] = us2
    out["mdot"]["sweeps"] = int(rep[0].item())
    run.close()
    return out


def main() -> int:
    import argparse
    import json
    import os
    import sys
    import time
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    from synth import workloads
    ap = argparse.ArgumentParser(description="temperature-gradient anisotropy of a static sphere, hex vs Voronoi")
    ap.add_argument("--hex", type=int, nargs="*", default=[75], help="hex meshes n^3")
    ap.add_argument("--voronoi", type=int, nargs="*", default=[59], help="Voronoi meshes of 2 n^3 cells")
    ap.add_argument("--bins", type=int, default=36)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    results = []
    for kind, ns in (("hex", a.hex), ("voronoi", a.voronoi)):
        for n in ns:
            t0 = time.time()
            wl = workloads.static_sphere(kind, n)
            print(f"[anisotropy] {wl.name}: {wl.n_mixed} mixed, built in {time.time() - t0:.1f} s", flush=True)
            r = study(wl, a.bins)
            g = r["grad"]
            print(f"[anisotropy] {kind} {n}: step {r['step_us']:.1f} us; m=4 of |grad T|: "
                  + ", ".join(f"{k} {v['m4_pct']:.2f}%" for k, v in g.items())
                  + "; mdot m=4 " + ", ".join(
                      f"{k} {r['mdot'][k]['m4_pct']:.2f}%" for k in ("one_sided", "two_sided") if r["mdot"][k]),
                  flush=True)
            results.append(r)
    text = json.dumps(results, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    else:
        print(text)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
