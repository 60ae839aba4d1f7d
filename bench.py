"""Throughput of the interface hot path on one MI355X.

One step = compaction + volume-matched reconstruction of every mixed cell +
interface-modified band gradient + mass transfer, replayed as one captured
HIP graph with inputs resident in HBM.  Default workload: 194,672-cell
box-clipped jittered-BCC Voronoi mesh of the unit cube with one vapour bubble
(r = 0.25) and a Scriven-like erf temperature profile, FP64.

Both forms are timed on the same inputs: plain (search from the cell's full
vertex-value range) and learned (the bracket network inside the
reconstruction kernel gives the first guess).  The headline value is the
learned form when trained weights are present, else the plain one.

Prints one JSON line: the metric and its value (mixed cells per second of
the headline form), the step time, `config` (the workload, both forms'
figures: evaluations per cell, fallback rate, agreement of the two forms,
and the follow-on rows timed on the same interface), `roofline` (the
reconstruction kernel against the FP64 vector peak, its HBM fraction beside
it, and the HBM traffic measured by rocprofv3 for the current kernel sources,
else null) and `cpu_baseline` (the CPU oracle on one host thread).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "mixed cells/s (reconstruct+∇T+ṁ, FP64), learned vs plain at |Δα|≤1e-10"
HBM_PEAK_GBS = 8000.0
# FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (fused multiply-add) x 2.4 GHz
FP64_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# algorithmic FP64 work of one mixed cell's reconstruction: ~46 bisection
# evaluations of the volume over the straddling edges and faces, 600-1300
# flops each on a Voronoi cell (~14 faces) and 300-600 on a hexahedron;
# the midpoints of the two ranges
FLOPS_VORONOI_CELL = 40.0e3
FLOPS_HEX_CELL = 18.5e3


def recon_flops(mesh, mixed: np.ndarray) -> float:
    nf = mesh.cell_face_off[mixed + 1] - mesh.cell_face_off[mixed]
    return float(np.where(nf <= 6, FLOPS_HEX_CELL, FLOPS_VORONOI_CELL).sum())


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def recon_bytes(mesh, mixed: np.ndarray) -> int:
    """Unique HBM footprint one reconstruction launch must touch for the mixed
    cells: the index list, per-cell topology and geometry, the vertices of the
    mixed cells with their vertex->cell weights and the alpha of those cells,
    and the interface record written back."""
    M = len(mixed)
    cfo = mesh.cell_face_off
    nf = cfo[mixed + 1] - cfo[mixed]
    # distinct vertices per mixed cell
    verts = []
    nl = 0
    for P in mixed:
        fs = mesh.cell_face[cfo[P]:cfo[P + 1]]
        vv = np.concatenate([mesh.face_vert[mesh.face_vert_off[f]:mesh.face_vert_off[f + 1]] for f in fs])
        nl += len(vv)
        verts.append(np.unique(vv))
    nv_tot = sum(len(v) for v in verts)
    U = np.unique(np.concatenate(verts)) if verts else np.zeros(0, int)
    # (cell, vertex) incidences of those vertices: ids and weights read, and
    # the alpha of every cell met
    from synth.fields import _cell_vertices
    vmask = np.zeros(mesh.n_verts, bool)
    vmask[U] = True
    cv_c, cv_v = _cell_vertices(mesh)
    key = np.unique(cv_c.astype(np.int64) * mesh.n_verts + cv_v)
    c = key // mesh.n_verts
    v = key % mesh.n_verts
    sel = vmask[v]
    deg = int(sel.sum())
    inc_cells = np.unique(c[sel])
    b = 0
    b += 4 * M                      # mixed_idx
    b += M * (16 + 16 + 16)         # cell_face_off, cv_off, cl_off pairs
    b += M * (8 + 24)               # V, centroid
    b += int(nf.sum()) * 3          # per-face loop offset (2) and size (1)
    b += 4 * nv_tot + nl            # local vertex ids, packed loops
    b += len(U) * (24 + 16)         # vertex coordinates, vertex->cell offsets
    b += deg * (4 + 8)              # vertex->cell ids and weights
    b += 8 * len(inc_cells)         # alpha of the cells sharing those vertices
    b += M * 64                     # interface record written
    return int(b)


def step_bytes(mesh, mixed, band, recon_b) -> int:
    """Unique footprint of the whole step: the alpha scan with the neighbour
    lists it needs for the band test, the lists written, the band gradient's
    gathers, the reconstruction and the mass transfer."""
    N = mesh.n_cells
    ncf = len(mesh.cell_face)
    b = 8 * N + 8 * (N + 1) + 4 * ncf + N      # alpha, cell_face_off, neighbour ids, flags
    b += 4 * (len(mixed) + len(band))
    cfo = mesh.cell_face_off
    nfb = int((cfo[band + 1] - cfo[band]).sum())
    b += nfb * (4 + 24 + 8 + 8) + len(band) * (16 + 24 + 8 + 8 + 24 + 4)
    b += recon_b
    b += len(mixed) * (4 + 8 + 24 + 8 + 8 + 24 + 16)
    return int(b)


RECON_SOURCES = ("recon.hip", "mlp_core.h", "vofpc_internal.h", "wave_ops.h")


def recon_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in RECON_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2604_14938_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(form: str):
    """HBM bytes per reconstruction launch of `form` from the committed
    rocprofv3 counter summary, if the kernel sources have not changed since;
    else None."""
    path = os.path.join(ROOT, "profiles", "recon_kernel_voronoi195k_traffic.json")
    try:
        info = json.load(open(path))
        cur = recon_source_hash()
    except (OSError, ValueError):
        return None
    if info.get("recon_sources_sha256") != cur or form not in info.get("traffic_bytes_per_launch", {}):
        return None
    return float(info["traffic_bytes_per_launch"][form])


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_pass(oracle, om, geom, wl):
    """One pass of the path on the oracle: reconstruction of every mixed
    cell, gradient on the band.  Returns the reconstruction and gradient."""
    band = np.nonzero(oracle.band_mask(wl.mesh, wl.alpha))[0]
    rec = oracle.reconstruct(om, wl.alpha, geom)
    g, _ = oracle.grad(om, geom, wl.T, wl.T_bface, wl.T_sat, wl.alpha, cells=band)
    return rec, g


def cpu_baseline(wl, budget_s: float = 10.0) -> dict:
    """The oracle timed on one host thread over the same step: mixed-cell
    scan and band, reconstruction of every mixed cell (its vertex field is
    built for the whole mesh on every call), band gradient and mass transfer.
    The mesh geometry is computed once beforehand, as the device path
    computes it at upload, outside its timed region."""
    import oracle
    om = oracle.OMesh(wl.mesh)
    geom = oracle.geometry(om)
    times = []
    t_end = time.perf_counter() + budget_s
    n = 0
    while time.perf_counter() < t_end or n < 2:
        t0 = time.perf_counter()
        rec, g = _oracle_pass(oracle, om, geom, wl)
        oracle.mass_transfer(geom, wl.alpha, rec["n"], rec["A"], g, wl.k_l, wl.k_v, wl.h_lv)
        times.append(time.perf_counter() - t0)
        n += 1
    M = wl.n_mixed
    t = statistics.median(times)
    out = {"value": M / t, "unit": "mixed cells/s", "cores": 1, "kind": "oracle",
           "sample": f"whole workload ({M} mixed of {wl.mesh.n_cells} cells; geometry precomputed once, untimed; "
                     f"gradient on the band), {n} single-thread passes in {sum(times):.1f} s, median {t * 1e3:.1f} ms per pass"}
    out["cpu"] = _cpu_model()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--form", choices=("both", "plain", "learned"), default="both",
                    help="which forms to time (profiling runs time one)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the default kernel flavours instead of autotuning them on the workload before timing")
    ap.add_argument("--workload", choices=("voronoi_bubble", "batched", "pipe", "multi"), default="voronoi_bubble",
                    help="batched: a 128^3 hexahedral and a 986,078-cell Voronoi mesh with random bubbles, "
                         "stepped as one (a throughput-regime check); pipe: a Voronoi pipe with a wavy liquid "
                         "film on its wall; multi: 64 independent Voronoi meshes with a bubble each, stepped through "
                         "time steps in one captured launch; the default is the metric's workload")
    ap.add_argument("--pipe-radial", type=int, default=40, help="Voronoi seeds across the pipe diameter")
    ap.add_argument("--multi-sizes", type=float, nargs=2, default=[1e4, 5e5],
                    help="range of the multi-instance mesh sizes (cells, log-uniform)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (to scale HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        return 2
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 2
    if args.copy_calibration:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8, "launches": 3}))
        return 0
    from paper_2604_14938_amd import runner
    from synth import workloads

    log("generating workload")
    t0 = time.time()
    parts = None
    step_fields = None   # multi-instance: host (alpha, T, T_bface) of each timed time step
    if args.workload == "multi":
        n_inst, n_steps, t_list = 64, 100, (0, 25, 50, 75)
        n_lo, n_hi = args.multi_sizes
        meshes_, _, _, field = workloads.multi_instance(n_inst=n_inst, n_lo=n_lo, n_hi=n_hi, seed=5, steps=n_steps,
                                                        K=12, log=log)
        step_fields = []
        for t in t_list:
            w = workloads.concat_workloads([field(i, t) for i in range(n_inst)])
            step_fields.append((w.alpha, w.T, w.T_bface))
            log(f"fields of time step {t}: {w.n_mixed} mixed")
            if t == t_list[0]:
                wl = w
        parts = meshes_
        wl_desc = (f"multi: {n_inst} independent jittered-BCC Voronoi meshes of log-uniform sizes in "
                   f"[{n_lo:.0f}, {n_hi:.0f}] cells ({wl.mesh.n_cells:,} in all), one bubble r ~ U[0.10, 0.20] each "
                   f"turning around the box axis (one revolution in {n_steps} steps), erf T profile; time steps "
                   f"{list(t_list)} cycled through one captured step over the union")
    elif args.workload == "batched":
        from synth import meshes as synth_meshes
        wls = []
        for i, build in enumerate((lambda: synth_meshes.hex_mesh(128), lambda: synth_meshes.voronoi_box_mesh(79, 3))):
            m = build()
            log(f"mesh {i}: {m.n_cells} cells")
            wls.append(workloads.random_bubbles(m, seed=3 + 17 * i, n_max=1000, K=16, r_hi_h=12.0))
            log(f"fields {i}: {wls[-1].meta['n_bubbles']} bubbles, {wls[-1].n_mixed} mixed")
        wl = workloads.concat_workloads(wls)
        parts = [w.mesh for w in wls]
        wl_desc = (f"batched: 128^3 hexahedra ({wls[0].meta['n_bubbles']} bubbles) + jittered-BCC Voronoi mesh "
                   f"of {wls[1].mesh.n_cells:,} cells ({wls[1].meta['n_bubbles']} bubbles), r ~ U[2h, 12h], "
                   f"per-bubble linear T, one disjoint union")
    elif args.workload == "pipe":
        wl = workloads.pipe_film(n_radial=args.pipe_radial, seed=4)
        wl_desc = (f"pipe: Voronoi pipe of {wl.mesh.n_cells:,} cells (jittered BCC, {args.pipe_radial} seeds across "
                   f"the diameter, length 52/9.5 R), liquid film on the wall of mean thickness 0.1 R with 5 axial "
                   f"waves of amplitude 0.3 of the thickness, T rising linearly across the film from T_sat at its "
                   f"surface to T_sat + 1 K at the wall")
    else:
        wl = workloads.voronoi_bubble()
        wl_desc = ("voronoi_bubble: 194,672-cell box-clipped jittered-BCC Voronoi mesh of the unit cube "
                   "(seed 2), vapour bubble r=0.25 at the centre, T_sat + 1.25 K erf((rho-0.25)/0.05) outside")
    log(f"workload ready in {time.time() - t0:.1f} s: {wl.mesh.n_cells} cells, {wl.n_mixed} mixed")
    from paper_2604_14938_amd import vofpc as V
    from paper_2604_14938_amd import train

    def time_form(mlp=None, dscale=0.0):
        """Capture the step of one form, warm up, time exactly `steps` graph
        replays (HIP events on the context stream), then time the
        reconstruction launch alone the same way."""
        run = runner.PathRun(wl, device=0, ctx=V.Context(0, stream=torch.cuda.Stream()), mlp=mlp,
                             delta_scale=dscale, parts=parts)
        stream = run.ctx.stream
        if args.autotune:
            choice, _ = V.autotune(run.ctx, run.mesh, run.alpha)
            log(f"autotuned flavours per class: {choice}")
        run.step()
        res = run.results()
        g = run.capture()
        if step_fields is not None:
            # time steps resident on the device; before each timed replay the
            # step's fields are copied into the captured inputs (not timed)
            dev_fields = [tuple(torch.as_tensor(x, dtype=torch.float64, device=run.dev) for x in f)
                          for f in step_fields]
            torch.cuda.synchronize()

            def load(t):
                with torch.cuda.stream(stream):
                    run.alpha.copy_(dev_fields[t][0])
                    run.T.copy_(dev_fields[t][1])
                    run.Tb.copy_(dev_fields[t][2])

            mixed_t = []
            for t in range(len(dev_fields)):
                load(t)
                g.launch()
                torch.cuda.synchronize()
                mixed_t.append(int(run.buf.counts[0].item()))
            for i in range(args.warmup):
                load(i % len(dev_fields))
                g.launch()
            torch.cuda.synchronize()
            pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                     for _ in range(args.steps)]
            cells = 0
            t_start = time.perf_counter()
            for i, (a, b_) in enumerate(pairs):
                t = i % len(dev_fields)
                load(t)
                a.record(stream)
                g.launch()
                b_.record(stream)
                cells += mixed_t[t]
            torch.cuda.synchronize()
            wall = time.perf_counter() - t_start
            per = [a.elapsed_time(b_) for a, b_ in pairs]
            ms = sum(per) / args.steps
            res["mixed_per_step"] = cells / args.steps
            res["mixed_by_time_step"] = mixed_t
            load(0)          # step 0 again, lists refreshed, for the kernel timing below
            g.launch()
            torch.cuda.synchronize()
        else:
            for _ in range(args.warmup):
                g.launch()
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
            torch.cuda.synchronize()
            t_start = time.perf_counter()
            ev[0].record(stream)
            for i in range(args.steps):
                g.launch()
                ev[i + 1].record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t_start
            per = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
            ms = ev[0].elapsed_time(ev[-1]) / args.steps
            res["mixed_per_step"] = res["n_mixed"]
        b = run.buf
        if mlp is None:
            rec = lambda: V.reconstruct(run.ctx, run.mesh, run.alpha, b.mixed_idx, b.counts, b.itf, b.opts)
        else:
            rec = lambda: V.reconstruct_learned(run.ctx, run.mesh, run.alpha, b.mixed_idx, b.counts, b.itf, mlp,
                                                dscale, b.opts)
        reps = max(10, args.steps)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        rec()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            rec()
        e1.record(stream)
        torch.cuda.synchronize()
        recon_ms = e0.elapsed_time(e1) / reps
        run.close()
        return res, ms, statistics.median(per), wall, recon_ms

    plain = learned = None
    if args.form in ("both", "plain"):
        plain, ms_p, med_p, wall_p, rms_p = time_form()
        log(f"plain step: {ms_p * 1e3:.1f} us mean, {med_p * 1e3:.1f} us median (wall {wall_p:.3f} s); "
            f"reconstruction {rms_p * 1e3:.1f} us")
    if args.form in ("both", "learned") and os.path.exists(train.DEFAULT_WEIGHTS):
        params, dscale, tinfo = train.load()
        ctx_m = V.Context(0, stream=torch.cuda.Stream())
        mlp = V.Mlp(ctx_m)
        mlp.set_params(params)
        learned, ms_l, med_l, wall_l, rms_l = time_form(mlp, dscale)
        log(f"learned step: {ms_l * 1e3:.1f} us mean, {med_l * 1e3:.1f} us median (wall {wall_l:.3f} s); "
            f"reconstruction {rms_l * 1e3:.1f} us")
    # two-sided mass transfer (Eq. extrapolation + Eq. mass_transfer) on the
    # plain step's interface: extrapolation plus the two-sided rate, timed
    # alone with HIP events on the context stream (not part of `value`)
    two = None
    if args.workload == "voronoi_bubble":
        run = runner.PathRun(wl, device=0, ctx=V.Context(0, stream=torch.cuda.Stream()), parts=parts)
        run.step()
        b = run.buf
        N = wl.mesh.n_cells
        gl = torch.full((3, N), float("nan"), dtype=torch.float64, device=run.dev)
        gv = torch.full((3, N), float("nan"), dtype=torch.float64, device=run.dev)
        md = torch.zeros(N, dtype=torch.float64, device=run.dev)
        qd = torch.zeros(N, dtype=torch.float64, device=run.dev)
        repd = torch.zeros(2, dtype=torch.int32, device=run.dev)
        torch.cuda.synchronize()

        def two_sided(max_iter):
            V.extrapolate(run.ctx, run.mesh, run.alpha, run.T, run.Tb, wl.T_sat, b.mixed_idx, b.counts, b.itf,
                          gl, gv, repd, opts=V.extrap_opts(max_iter=max_iter))
            V.mass_transfer(run.ctx, run.mesh, run.alpha, b.mixed_idx, b.counts, b.itf, None, wl.k_l, wl.k_v,
                            wl.h_lv, md, qd, gradT_l=gl, gradT_v=gv)

        def timed(fn, reps=20):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(run.ctx.stream):
                e0.record(run.ctx.stream)
                for _ in range(reps):
                    fn()
                e1.record(run.ctx.stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) * 1e3 / reps

        two_sided(120)
        torch.cuda.synchronize()
        dom = int((~torch.isnan(gl[0])).sum().item())
        two = {"two_sided_mdot": {"sweeps": int(repd[0].item()), "domain_cells": dom}}
        tsm = two["two_sided_mdot"]
        # the paper's cap of 120 sweeps, and a cap of 32 that still covers its
        # typical 10-30 sweeps: every sweep is a kernel, idle once converged
        for cap, name in ((120, "max_sweeps_120"), (32, "max_sweeps_32")):
            two_sided(cap)
            torch.cuda.synchronize()
            ok = int(repd[1].item()) == 0 and int(repd[0].item()) == tsm["sweeps"]
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=run.ctx.stream):
                two_sided(cap)
            graph.replay()
            torch.cuda.synchronize()
            tsm[name] = {"us_eager": timed(lambda: two_sided(cap)), "us_graph_replay": timed(graph.replay),
                         "report_ok": ok}
            log(f"two-sided mass transfer, {name}: eager {tsm[name]['us_eager']:.1f} us, graph replay "
                f"{tsm[name]['us_graph_replay']:.1f} us ({tsm['sweeps']} sweeps over {dom} cells)")
        del graph
        # interface coupling coefficients (Eq. interface_htc) on the same
        # interface, and the surface-tension curvature chain over every cell
        nf_cap = wl.mesh.n_faces
        ad = torch.zeros(N, dtype=torch.float64, device=run.dev)
        fi = torch.zeros(nf_cap, dtype=torch.int32, device=run.dev)
        fa = torch.zeros(2, nf_cap, dtype=torch.float64, device=run.dev)
        fd = torch.zeros(2, nf_cap, dtype=torch.float64, device=run.dev)
        fr = torch.zeros(nf_cap, dtype=torch.float64, device=run.dev)
        nfo = torch.zeros(1, dtype=torch.int32, device=run.dev)

        def robin():
            V.robin(run.ctx, run.mesh, run.alpha, b.mixed_idx, b.band_idx, b.counts, b.itf, wl.k_l, wl.k_v,
                    a_diag=ad, face_idx=fi, face_a=fa, face_d=fd, face_area=fr, n_face=nfo)

        ah = torch.zeros(N, dtype=torch.float64, device=run.dev)
        cn = torch.zeros(3, N, dtype=torch.float64, device=run.dev)
        kp = torch.zeros(N, dtype=torch.float64, device=run.dev)
        fs = torch.zeros(3, N, dtype=torch.float64, device=run.dev)

        def curvature():
            V.curvature(run.ctx, run.mesh, run.alpha, ah, cn, kp, force=fs,
                        opts=V.csf_opts(n_smooth=2, sigma=0.0589))

        for name, fn in (("robin", robin), ("curvature", curvature)):
            fn()
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=run.ctx.stream):
                fn()
            graph.replay()
            torch.cuda.synchronize()
            two[name] = {"us_graph_replay": timed(graph.replay)}
            del graph
        two["robin"]["detached_faces"] = int(nfo.item())
        two["curvature"]["cells"] = int(N)
        two["curvature"]["n_smooth"] = 2
        log(f"interface coupling: {two['robin']['us_graph_replay']:.1f} us ({two['robin']['detached_faces']} "
            f"detached faces); curvature chain: {two['curvature']['us_graph_replay']:.1f} us over {N} cells")
        run.close()
    if plain is None and learned is None:
        print(json.dumps({"error": "no trained weights for the learned form"}))
        return 2
    head = learned if learned is not None else plain
    M = head["n_mixed"]
    ms_per_step = ms_l if learned is not None else ms_p
    recon_ms = rms_l if learned is not None else rms_p
    form = "learned" if learned is not None else "plain"
    ok = head["status"] != 1
    parity_alpha = float(np.abs(head["alpha_got"][head["status"] == 0] -
                                wl.alpha[head["mixed_idx"][head["status"] == 0]]).max(initial=0))
    mixed = head["mixed_idx"]
    rb = recon_bytes(wl.mesh, mixed)
    if learned is not None:
        cfo = wl.mesh.cell_face_off
        rb += int((cfo[mixed + 1] - cfo[mixed]).sum()) * (4 + 4 + 24) + 6 * 6532   # faces read by the features, weights
    sb = step_bytes(wl.mesh, mixed, head["band_idx"], rb)
    achieved = rb / (recon_ms * 1e-3) / 1e9
    rf = recon_flops(wl.mesh, mixed)
    tflops = rf / (recon_ms * 1e-3) / 1e12
    log(f"{form} reconstruction kernel: {recon_ms * 1e3:.1f} us, {rf / 1e6:.1f} MFLOP and {rb / 1e6:.2f} MB "
        f"algorithmic -> {tflops:.3f} TFLOP/s, {achieved:.1f} GB/s")
    cfg = {
        "workload": wl_desc,
        "n_cells": int(wl.mesh.n_cells),
        "n_mixed": int(M),
        "n_band": int(head["n_band"]),
        "form": form,
        "max_abs_dalpha_vs_input": parity_alpha,
        "step_algorithmic_bytes": sb,
        "step_GBps": sb / (ms_per_step * 1e-3) / 1e9,
    }
    if step_fields is not None:
        cfg["mixed_per_timed_step"] = head["mixed_per_step"]
        cfg["mixed_by_time_step"] = head["mixed_by_time_step"]
    if two is not None:
        cfg["follow_on"] = two
    if plain is not None:
        cfg["plain"] = {"cells_per_s": plain["mixed_per_step"] / (ms_p * 1e-3), "ms_per_step": ms_p, "recon_us": rms_p * 1e3,
                        "evals_per_cell_mean": float(plain["iters"].mean()),
                        "evals_per_cell_p99": float(np.percentile(plain["iters"], 99))}
    if learned is not None:
        cfg["learned"] = {
            "cells_per_s": learned["mixed_per_step"] / (ms_l * 1e-3), "ms_per_step": ms_l, "recon_us": rms_l * 1e3,
            "evals_per_cell_mean": float(learned["iters"].mean()),
            "evals_per_cell_p99": float(np.percentile(learned["iters"], 99)),
            "fallback_rate": float(np.mean(learned["status"] == 2)),
            "delta_scale": dscale, "weights_sigma_val": tinfo.get("sigma_val"),
        }
    if learned is not None and plain is not None:
        same = (learned["status"] == plain["status"]) | ((learned["status"] == 2) & (plain["status"] == 0))
        both = same & (plain["status"] != 1)
        cfg["learned"].update({
            "speedup_vs_plain": ms_p / ms_l,
            "statuses_agree_fraction": float(np.mean(same)),
            "max_abs_dalpha_vs_plain": float(np.abs(learned["alpha_got"] - plain["alpha_got"])[both].max(initial=0)),
            "bitwise_equal_fraction": float(np.mean((learned["alpha_got"] == plain["alpha_got"]) &
                                                    (learned["A"] == plain["A"]))),
        })
    out = {
        "metric": METRIC,
        "value": head["mixed_per_step"] / (ms_per_step * 1e-3),
        "unit": "mixed cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": cfg,
        # the reconstruction's algorithmic intensity (FLOP per algorithmic
        # byte) is above the FP64 ridge point (78.6 TFLOP/s / 8 TB/s), so the
        # FP64 vector ALU is its roof; the HBM figures are reported beside it
        "roofline": {
            "bound": "alu",
            "kernel": "recon_kernel",
            "achieved": tflops,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": tflops / FP64_PEAK_TFLOPS,
            "traffic": measured_traffic(form) if args.workload == "voronoi_bubble" else None,
            "kernel_us": recon_ms * 1e3,
            "algorithmic_flops": rf,
            "algorithmic_bytes": rb,
            "intensity_flop_per_byte": rf / rb,
            "hbm": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS},
        },
    }
    if not args.no_cpu:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
