"""Throughput of the interface hot path on one MI355X.

One step = compaction + volume-matched reconstruction of every mixed cell +
interface-modified band gradient + mass transfer, replayed as one captured
HIP graph with inputs resident in HBM.  Default workload (`full`): the
learned-bracket configuration at full size, one disjoint union of a 128^3
hexahedral mesh and a 986,078-cell box-clipped jittered-BCC Voronoi mesh
(random bubbles r ~ U[2h, 12h], per-bubble linear T) and a 4,043,057-cell
Voronoi pipe with a wavy liquid film on its wall, FP64.  The other
workloads (`--workload`) are the single-bubble Voronoi mesh, the batched
pair alone, the pipe alone and the multi-instance time-step batch.

Both forms are timed on the same inputs: plain (search from the cell's full
vertex-value range) and learned (the bracket network inside the
reconstruction kernel gives the first guess, checked with a cut at each
end).  The headline value is the learned form when trained weights are
present, else the plain one.

Prints one JSON line: the metric and its value (mixed cells per second of
the headline form), the step time, `config` (the workload, both forms'
figures: evaluations per cell, per-cell outcome rates, agreement of the two
forms), `roofline` (the dominant reconstruction class kernel against the FP64
vector peak, timed with HIP events on its stream, its HBM fraction beside
it, and the HBM traffic measured by rocprofv3 for the current kernel sources,
else null) and `cpu_baseline` (the CPU oracle, one process per host core
over contiguous chunks of the mixed list).
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
# kernel classes by cell size: largest vertices, faces, loop positions and
# edges of a cell each class's kernels are built for (class 3: larger)
CLASS_CAPS = ((16, 8, 48, 24), (32, 20, 96, 48), (48, 32, 128, 64))
HEX_CAPS = (8, 6, 24, 12)
STATUS_NAMES = ("ok", "not_mixed", "learned_fallback", "degenerate", "max_iter", "g_singular", "bad_input",
                "no_root")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "recon_kernel_traffic.json")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def recon_flops(mesh, mixed: np.ndarray) -> float:
    nf = mesh.cell_face_off[mixed + 1] - mesh.cell_face_off[mixed]
    return float(np.where(nf <= 6, FLOPS_HEX_CELL, FLOPS_VORONOI_CELL).sum())


def _ranges(off: np.ndarray, rows: np.ndarray) -> np.ndarray:
    cnt = off[rows + 1] - off[rows]
    return np.repeat(off[rows] - np.cumsum(np.r_[0, cnt[:-1]]), cnt) + np.arange(cnt.sum())


def cell_incidence(mesh, cells: np.ndarray):
    """Distinct (row, vertex) pairs of the cells (row = position in `cells`)
    and each cell's face count and loop positions."""
    cells = np.asarray(cells, np.int64)
    cfo, fvo = mesh.cell_face_off, mesh.face_vert_off
    nf = cfo[cells + 1] - cfo[cells]
    faces = mesh.cell_face[_ranges(cfo, cells)].astype(np.int64)
    fsz = fvo[faces + 1] - fvo[faces]
    row_f = np.repeat(np.arange(len(cells)), nf)
    nl = np.bincount(row_f, weights=fsz, minlength=len(cells)).astype(np.int64)
    verts = mesh.face_vert[_ranges(fvo, faces)].astype(np.int64)
    key = np.unique(np.repeat(row_f, fsz) * mesh.n_verts + verts)
    return key // mesh.n_verts, key % mesh.n_verts, nf, nl


def _classes_and_hex(mesh, cells: np.ndarray):
    row, _, nf, nl = cell_incidence(mesh, cells)
    nv = np.bincount(row, minlength=len(cells))
    out = np.full(len(cells), len(CLASS_CAPS), np.int64)
    for c in range(len(CLASS_CAPS) - 1, -1, -1):
        v, f, l, e = CLASS_CAPS[c]
        out[(nv <= v) & (nf <= f) & (nl <= l) & (nl // 2 <= e)] = c
    v, f, l, e = HEX_CAPS
    return out, (nv <= v) & (nf <= f) & (nl <= l) & (nl // 2 <= e)


def mesh_hex0(mesh) -> bool:
    """Whether the mesh's class 0 is all but at most 1 % hexahedral-sized
    cells (then the library moves the other class-0 cells to class 1)."""
    cls, hexfit = _classes_and_hex(mesh, np.arange(mesh.n_cells))
    c0 = int(np.count_nonzero(cls == 0))
    rest = c0 - int(np.count_nonzero((cls == 0) & hexfit))
    return rest > 0 and rest * 100 <= c0


def cell_classes(mesh, cells: np.ndarray, hex0: bool | None = None) -> np.ndarray:
    """Kernel class of each cell as the library assigns it: the first class
    whose caps hold its vertices, faces, loop positions and edges (loop
    positions / 2), class-0 cells beyond the hexahedral caps in class 1 when
    the mesh's class 0 is hexahedral (mesh_hex0)."""
    out, hexfit = _classes_and_hex(mesh, cells)
    if hex0 is None:
        hex0 = mesh_hex0(mesh)
    if hex0:
        out[(out == 0) & ~hexfit] = 1
    return out


def recon_bytes(mesh, mixed: np.ndarray, learned: bool = False) -> int:
    """Unique HBM footprint one reconstruction launch over `mixed` must
    touch: the index list, per-cell topology and geometry, the vertices of
    the cells with their vertex->cell weights and the alpha of the cells
    sharing them, and the interface record written back; the learned form
    adds the faces its features read and the network weights."""
    M = len(mixed)
    if M == 0:
        return 0
    row, verts, nf, nl = cell_incidence(mesh, mixed)
    nv_tot = len(row)
    U = np.unique(verts)
    # vertex -> cell incidences of those vertices: (cell, vertex) pairs of
    # the mesh restricted to U
    cfo, fvo = mesh.cell_face_off, mesh.face_vert_off
    fsz = np.diff(fvo)
    cell_of_face_slot = np.repeat(np.arange(mesh.n_cells), np.diff(cfo))
    rep = fsz[mesh.cell_face]
    c_all = np.repeat(cell_of_face_slot, rep)
    v_all = mesh.face_vert[_ranges(fvo, mesh.cell_face.astype(np.int64))]
    vmask = np.zeros(mesh.n_verts, bool)
    vmask[U] = True
    sel = vmask[v_all]
    key = np.unique(c_all[sel].astype(np.int64) * mesh.n_verts + v_all[sel])
    deg = len(key)
    inc_cells = len(np.unique(key // mesh.n_verts))
    b = 4 * M                       # mixed_idx
    b += M * (16 + 16 + 16)         # cell_face_off, cv_off, cl_off pairs
    b += M * (8 + 24)               # V, centroid
    b += int(nf.sum()) * 3          # per-face loop offset (2) and size (1)
    b += 4 * nv_tot + int(nl.sum())  # local vertex ids, packed loops
    b += 2 * int(nl.sum())          # edge table (4 bytes per edge)
    b += len(U) * (24 + 16)         # vertex coordinates, vertex->cell offsets
    b += deg * (4 + 8)              # vertex->cell ids and weights
    b += 8 * inc_cells              # alpha of the cells sharing those vertices
    b += M * 64                     # interface record written
    if learned:
        b += int(nf.sum()) * (4 + 4 + 24) + 6 * 6532   # faces read by the features, weights
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


RECON_SOURCES = ("recon.hip", "recon_thin.hip", "recon_common.h", "mlp_core.h", "vofpc_internal.h", "wave_ops.h")


def recon_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in RECON_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2604_14938_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(workload: str, form: str, kernel_class: int):
    """HBM bytes per launch of the class kernel of `form` on `workload` from
    the committed rocprofv3 counter summary, if the kernel sources have not
    changed since; else None."""
    try:
        info = json.load(open(TRAFFIC_FILE))
        cur = recon_source_hash()
    except (OSError, ValueError):
        return None
    if info.get("recon_sources_sha256") != cur or info.get("workload") != workload:
        return None
    rec = info.get("traffic_bytes_per_launch", {}).get(form, {})
    v = rec.get(str(kernel_class))
    return None if v is None else float(v)


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------- CPU oracle
_CPU = {}


def _cpu_worker(i: int, reps: int, barrier, queue) -> None:
    """One process of the oracle baseline: `reps` passes over chunk i, each
    started together with the other processes."""
    import oracle
    g = _CPU
    chunk, bchunk = g["chunks"][i], g["bchunks"][i]
    wl, om, geom = g["wl"], g["om"], g["geom"]
    times = []
    for _ in range(reps):
        barrier.wait()
        t0 = time.perf_counter()
        rec = oracle.reconstruct(om, wl.alpha, geom, cells=chunk)
        gr, _ = oracle.grad(om, geom, wl.T, wl.T_bface, wl.T_sat, wl.alpha, cells=bchunk)
        sub = np.ascontiguousarray
        oracle.mass_transfer(oracle.Geometry(sub(geom.V[chunk]), None, None, None), wl.alpha[chunk],
                             sub(rec["n"][:, chunk]), sub(rec["A"][chunk]), sub(gr[:, chunk]), wl.k_l, wl.k_v,
                             wl.h_lv)
        times.append(time.perf_counter() - t0)
    queue.put((i, times))


def cpu_baseline(wl, budget_s: float, procs: int) -> dict:
    """The oracle over the same step, one process per host core, the mixed
    list and the band list each split into `procs` contiguous chunks: each
    process reconstructs its mixed cells (the oracle builds the vertex field
    of the whole mesh on every call), takes the gradient on its band cells
    and the mass transfer of its mixed cells.  The mesh geometry is computed
    once beforehand, untimed, as the device path computes it at upload.  A
    pass ends when the slowest process ends; value = mixed cells / median
    pass time.  Runs before anything touches the GPU (the processes are
    forked)."""
    import multiprocessing as mp
    import oracle
    t0 = time.perf_counter()
    om = oracle.OMesh(wl.mesh)
    geom = oracle.geometry(om)
    a = wl.alpha
    mixed = np.nonzero((a > 1e-8) & (a < 1.0 - 1e-8))[0]
    band = np.nonzero(oracle.band_mask(wl.mesh, a))[0]
    log(f"oracle geometry of {wl.mesh.n_cells} cells in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    oracle.vertex_field(om, geom.xc, a)
    t_vf = time.perf_counter() - t0
    P = max(1, min(procs, len(mixed)))
    _CPU.update(wl=wl, om=om, geom=geom, chunks=np.array_split(mixed, P), bchunks=np.array_split(band, P))
    # one calibration pass of the first chunk on this process sets the count
    q = mp.get_context("fork").SimpleQueue()

    class _NoBarrier:
        def wait(self):
            pass

    _cpu_worker(0, 1, _NoBarrier(), q)
    t_cal = q.get()[1][0]
    reps = int(min(10, max(2, budget_s // max(t_cal, 1e-3))))
    ctx = mp.get_context("fork")
    barrier = ctx.Barrier(P)
    queue = ctx.SimpleQueue()
    ps = [ctx.Process(target=_cpu_worker, args=(i, reps, barrier, queue)) for i in range(P)]
    t1 = time.perf_counter()
    for p in ps:
        p.start()
    res = dict(queue.get() for _ in range(P))
    for p in ps:
        p.join()
    wall = time.perf_counter() - t1
    bad = [p.exitcode for p in ps if p.exitcode != 0]
    if bad:
        raise RuntimeError(f"oracle baseline processes failed: {bad}")
    per_pass = [max(res[i][r] for i in range(P)) for r in range(reps)]
    t = statistics.median(per_pass)
    M = len(mixed)
    _CPU.clear()
    return {"value": M / t, "unit": "mixed cells/s", "cores": P, "kind": "oracle",
            "sample": (f"whole workload: {M} mixed and {len(band)} band cells of {wl.mesh.n_cells} in {P} "
                       f"contiguous chunks, one forked process each, {reps} passes started together "
                       f"({wall:.1f} s wall); a pass = reconstruction of the chunk (the oracle builds the vertex "
                       f"field of the whole mesh on each call: {t_vf * 1e3:.0f} ms of it) + band gradient + mass "
                       f"transfer, geometry precomputed once untimed; median of the slowest process's pass "
                       f"{t * 1e3:.1f} ms"),
            "cpu": _cpu_model()}


# ---------------------------------------------------------------- workloads
def build_workload(args):
    """(workload, parts or None, description, per-step fields or None)."""
    from synth import workloads
    cache = None
    if args.cache and args.workload in ("full", "batched", "pipe"):
        os.makedirs(args.cache, exist_ok=True)
        cache = os.path.join(args.cache, f"{args.workload}_r{args.pipe_radial}.npz")
    wls = None
    if cache and os.path.exists(cache):
        wls = workloads.load_parts(cache)
        log(f"workload read from {cache}")
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
        desc = (f"multi: {n_inst} independent jittered-BCC Voronoi meshes of log-uniform sizes in "
                f"[{n_lo:.0f}, {n_hi:.0f}] cells ({wl.mesh.n_cells:,} in all), one bubble r ~ U[0.10, 0.20] each "
                f"turning around the box axis (one revolution in {n_steps} steps), erf T profile; time steps "
                f"{list(t_list)} cycled through one captured step over the union")
        return wl, meshes_, desc, step_fields
    if args.workload == "voronoi_bubble":
        wl = workloads.voronoi_bubble()
        return wl, None, ("voronoi_bubble: 194,672-cell box-clipped jittered-BCC Voronoi mesh of the unit cube "
                          "(seed 2), vapour bubble r=0.25 at the centre, T_sat + 1.25 K erf((rho-0.25)/0.05) "
                          "outside"), None
    if wls is None:
        if args.workload == "full":
            wls = workloads.learned_full(pipe_radial=args.pipe_radial, log=log)
        elif args.workload == "batched":
            wls = workloads.batched()
        else:
            wls = [workloads.pipe_film(n_radial=args.pipe_radial, seed=4)]
        if cache:
            workloads.save_parts(cache, wls)
            log(f"workload written to {cache}")
    pipe_desc = (f"Voronoi pipe of {{:,}} cells (jittered BCC, {args.pipe_radial} seeds across the diameter, "
                 f"length 52/9.5 R), liquid film on the wall of mean thickness 0.1 R with 5 axial waves of "
                 f"amplitude 0.3 of the thickness, T rising linearly across the film from T_sat at its surface "
                 f"to T_sat + 1 K at the wall")
    if args.workload == "pipe":
        wl = wls[0]
        return wl, None, "pipe: " + pipe_desc.format(wl.mesh.n_cells), None
    nb = [w.meta.get("n_bubbles", "?") for w in wls]
    desc = (f"128^3 hexahedra ({nb[0]} bubbles) + jittered-BCC Voronoi mesh of {wls[1].mesh.n_cells:,} cells "
            f"({nb[1]} bubbles), r ~ U[2h, 12h] placed by random sequential addition, per-bubble linear T")
    if args.workload == "full":
        desc = ("full (learned-bracket configuration): " + desc + "; + " + pipe_desc.format(wls[2].mesh.n_cells) +
                "; one disjoint union stepped as one, mixed cells bucketed by kernel class")
    else:
        desc = "batched: " + desc + ", one disjoint union"
    wl = workloads.concat_workloads(wls)
    return wl, [w.mesh for w in wls], desc, None


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle passes (about)")
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="oracle processes (default: the cores this process may run on, at most 16)")
    ap.add_argument("--form", choices=("both", "plain", "learned"), default="both",
                    help="which forms to time (profiling runs time one)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the default kernel flavours instead of autotuning them on the workload before timing")
    ap.add_argument("--tune", default=None,
                    help="kernel flavour per class, e.g. 14,26,4,3 (no autotuning; a profiled run then holds only "
                         "the timed launches)")
    ap.add_argument("--workload", choices=("full", "voronoi_bubble", "batched", "pipe", "multi"), default="full",
                    help="full (default): the learned-bracket configuration (128^3 hexahedra + 986,078 Voronoi "
                         "cells with random bubbles + a 4M-cell Voronoi pipe with a wavy film); voronoi_bubble: "
                         "194,672 Voronoi cells with one bubble and the follow-on rows; batched: the first two "
                         "meshes alone; pipe: the pipe alone; multi: 64 independent Voronoi meshes stepped "
                         "through time steps in one captured launch")
    ap.add_argument("--pipe-radial", type=int, default=98, help="Voronoi seeds across the pipe diameter")
    ap.add_argument("--multi-sizes", type=float, nargs=2, default=[1e4, 5e5],
                    help="range of the multi-instance mesh sizes (cells, log-uniform)")
    ap.add_argument("--cache", default=None,
                    help="directory for the generated workload (.npz, read back when present)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (to scale HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        return 2
    import torch
    if torch.cuda.device_count() < 1:      # counts devices without initialising them
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

    log("generating workload")
    t0 = time.time()
    wl, parts, wl_desc, step_fields = build_workload(args)
    log(f"workload ready in {time.time() - t0:.1f} s: {wl.mesh.n_cells} cells, {wl.n_mixed} mixed")
    cpu = None
    if not args.no_cpu:
        procs = args.cpu_procs or min(16, len(os.sched_getaffinity(0)))
        log(f"timing the CPU oracle on {procs} processes (before the GPU is touched)")
        cpu = cpu_baseline(wl, args.cpu_budget, procs)
        log(f"oracle: {cpu['value']:.0f} mixed cells/s on {cpu['cores']} processes")

    from paper_2604_14938_amd import runner
    from paper_2604_14938_amd import vofpc as V
    from paper_2604_14938_amd import train

    def time_form(mlp=None, dscale=0.0):
        """Capture the step of one form, warm up, time exactly `steps` graph
        replays (HIP events on the context stream), then time the
        reconstruction launch and each of its class kernels the same way."""
        run = runner.PathRun(wl, device=0, ctx=V.Context(0, stream=torch.cuda.Stream()), mlp=mlp,
                             delta_scale=dscale, parts=parts)
        stream = run.ctx.stream
        tune = None
        if args.tune:
            tune = [int(x) for x in args.tune.split(",")]
            run.mesh.set_tune(tune)
        elif args.autotune:
            tune, _ = V.autotune(run.ctx, run.mesh, run.alpha)
            log(f"autotuned flavours per class: {tune}")
        run.step()
        res = run.results()
        res["classes"] = run.mesh.classes()
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
        # each class kernel alone: an event pair around it on the context
        # stream (the library records them), averaged over the launches
        # each class kernel's own time: the classes in turn for these calls
        # (the timed step runs them side by side)
        run.ctx.overlap_classes(False)
        run.ctx.time_classes(True)
        cls_ms = np.zeros(4)
        pass_ms = np.zeros(4)
        for _ in range(reps):
            rec()
            km, pm = run.ctx.class_ms()
            cls_ms += np.array(km)
            pass_ms += np.array(pm)
        run.ctx.time_classes(False)
        run.ctx.overlap_classes(True)
        res["class_ms"] = (cls_ms / reps).tolist()
        res["pass_ms"] = (pass_ms / reps).tolist()
        res["tune"] = tune if tune is not None else res["classes"]["tune"]
        run.close()
        return res, ms, statistics.median(per), wall, recon_ms

    plain = learned = None
    if args.form in ("both", "plain"):
        plain, ms_p, med_p, wall_p, rms_p = time_form()
        log(f"plain step: {ms_p * 1e3:.1f} us mean, {med_p * 1e3:.1f} us median (wall {wall_p:.3f} s); "
            f"reconstruction {rms_p * 1e3:.1f} us, class kernels {plain['class_ms']} ms")
    if args.form in ("both", "learned") and os.path.exists(train.DEFAULT_WEIGHTS):
        params, dscale, tinfo = train.load()
        ctx_m = V.Context(0, stream=torch.cuda.Stream())
        mlp = V.Mlp(ctx_m)
        mlp.set_params(params)
        learned, ms_l, med_l, wall_l, rms_l = time_form(mlp, dscale)
        log(f"learned step: {ms_l * 1e3:.1f} us mean, {med_l * 1e3:.1f} us median (wall {wall_l:.3f} s); "
            f"reconstruction {rms_l * 1e3:.1f} us, class kernels {learned['class_ms']} ms, bracket passes "
            f"{learned['pass_ms']} ms")
    two = follow_on(args, wl, parts, runner, V, torch) if args.workload == "voronoi_bubble" else None
    if plain is None and learned is None:
        print(json.dumps({"error": "no trained weights for the learned form"}))
        return 2
    head = learned if learned is not None else plain
    M = head["n_mixed"]
    ms_per_step = ms_l if learned is not None else ms_p
    recon_ms = rms_l if learned is not None else rms_p
    form = "learned" if learned is not None else "plain"
    ok = head["status"] == V.CELL_OK
    parity_alpha = float(np.abs(head["alpha_got"][ok] - wl.alpha[head["mixed_idx"][ok]]).max(initial=0))
    mixed = head["mixed_idx"]
    # the dominant class kernel: the launched kernel with the longest time
    cls = head["classes"]
    cms = np.array(head["class_ms"])
    kc = int(np.argmax(cms))
    if cls["bucketed"]:
        kcells = mixed[cell_classes(wl.mesh, mixed) == kc]
    else:
        kcells = mixed
    k_ms = float(cms[kc])
    kp_ms = float(head["pass_ms"][kc])
    # the learned class kernel reads its brackets (16 bytes per cell) when a
    # bracket pass made them, else its network's inputs
    rb_k = recon_bytes(wl.mesh, kcells, learned=form == "learned" and kp_ms < 0)
    if form == "learned" and kp_ms >= 0:
        rb_k += 16 * len(kcells)
    rf_k = recon_flops(wl.mesh, kcells)
    tflops = rf_k / (k_ms * 1e-3) / 1e12
    achieved = rb_k / (k_ms * 1e-3) / 1e9
    log(f"{form} dominant reconstruction kernel (class {kc}, flavour {head['tune'][kc]}): {k_ms * 1e3:.1f} us over "
        f"{len(kcells)} cells, {rf_k / 1e6:.1f} MFLOP and {rb_k / 1e6:.2f} MB algorithmic -> {tflops:.3f} TFLOP/s, "
        f"{achieved:.1f} GB/s")
    rb = recon_bytes(wl.mesh, mixed, learned=form == "learned")
    rf = recon_flops(wl.mesh, mixed)
    sb = step_bytes(wl.mesh, mixed, head["band_idx"], rb)

    def outcome(r):
        st = r["status"]
        n = max(len(st), 1)
        return {name: float(np.count_nonzero(st == i)) / n for i, name in enumerate(STATUS_NAMES)
                if i != V.CELL_NOT_MIXED}

    cfg = {
        "workload": wl_desc,
        "n_cells": int(wl.mesh.n_cells),
        "n_mixed": int(M),
        "n_band": int(head["n_band"]),
        "form": form,
        "max_abs_dalpha_vs_input": parity_alpha,
        "kernel_classes": {"cells": cls["cells"], "bucketed": cls["bucketed"], "flavours": head["tune"]},
        "recon_us": recon_ms * 1e3,
        "recon_all_classes": {"algorithmic_flops": rf, "algorithmic_bytes": rb,
                              "TFLOPs": rf / (recon_ms * 1e-3) / 1e12},
        "step_algorithmic_bytes": sb,
        "step_GBps": sb / (ms_per_step * 1e-3) / 1e9,
    }
    if step_fields is not None:
        cfg["mixed_per_timed_step"] = head["mixed_per_step"]
        cfg["mixed_by_time_step"] = head["mixed_by_time_step"]
    if two is not None:
        cfg["follow_on"] = two
    if plain is not None:
        cfg["plain"] = {"cells_per_s": plain["mixed_per_step"] / (ms_p * 1e-3), "ms_per_step": ms_p,
                        "recon_us": rms_p * 1e3, "class_kernel_us": [x * 1e3 for x in plain["class_ms"]],
                        "kernel_flavours": plain["tune"],
                        "evals_per_cell_mean": float(plain["iters"].mean()),
                        "evals_per_cell_p99": float(np.percentile(plain["iters"], 99)),
                        "outcome_rates": outcome(plain)}
    if learned is not None:
        cfg["learned"] = {
            "cells_per_s": learned["mixed_per_step"] / (ms_l * 1e-3), "ms_per_step": ms_l, "recon_us": rms_l * 1e3,
            "class_kernel_us": [x * 1e3 for x in learned["class_ms"]],
            "bracket_pass_us": [x * 1e3 for x in learned["pass_ms"]],
            "kernel_flavours": learned["tune"],
            "evals_per_cell_mean": float(learned["iters"].mean()),
            "evals_per_cell_p99": float(np.percentile(learned["iters"], 99)),
            "outcome_rates": outcome(learned),
            "delta_scale": dscale, "weights_sigma_val": tinfo.get("sigma_val"),
            "weights_labels": tinfo.get("samples"), "weights_labels_by_kind": tinfo.get("labels_by_kind"),
        }
    if learned is not None and plain is not None:
        same = (learned["status"] == plain["status"]) | ((learned["status"] == V.CELL_LEARNED_FALLBACK) &
                                                         (plain["status"] == V.CELL_OK))
        both = same & (plain["status"] != V.CELL_NOT_MIXED)
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
            "kernel": f"reconstruction class {kc} kernel (flavour {head['tune'][kc]})",
            "achieved": tflops,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": tflops / FP64_PEAK_TFLOPS,
            "traffic": measured_traffic(args.workload, form, kc),
            "kernel_us": k_ms * 1e3,
            "bracket_pass_us": kp_ms * 1e3 if kp_ms >= 0 else None,
            "cells": int(len(kcells)),
            "algorithmic_flops": rf_k,
            "algorithmic_bytes": rb_k,
            "intensity_flop_per_byte": rf_k / max(rb_k, 1),
            "hbm": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS},
        },
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))
    return 0


def extrap_sweep_bytes(mesh, dom, us) -> dict:
    """Algorithmic bytes of one busy extrapolation sweep over the domain
    cells `dom` (boolean per cell): per domain cell its list entry (4), its
    packed-stencil range (8), theta (8), its advanced components read (24)
    and written (24), and its record as a neighbour (24); per upwind face
    slot its weight (8) and neighbour (4).  The upwind slots are taken as half
    of the face slots between two domain cells (such a face is upwind for
    exactly one of its cells when their velocities agree)."""
    nd = int(dom.sum())
    nb = np.asarray(mesh.face_neigh)
    inner = nb >= 0
    slots = int(np.count_nonzero(dom[mesh.face_owner[inner]] & dom[nb[inner]]))   # 2 slots per face, half upwind
    b = nd * (4 + 8 + 8 + 24 + 24 + 24) + slots * 12
    gbs = b / (us * 1e-6) / 1e9 if us > 0 else float("nan")
    return {"domain_cells": nd, "upwind_slots_est": slots, "algorithmic_bytes": b, "GBps": gbs,
            "hbm_frac": gbs / HBM_PEAK_GBS}


def follow_on(args, wl, parts, runner, V, torch) -> dict:
    """Two-sided mass transfer (Eq. extrapolation + Eq. mass_transfer), the
    interface coupling coefficients (Eq. interface_htc) and the surface-tension
    curvature chain on the plain step's interface, each timed alone with HIP
    events on the context stream (not part of `value`)."""
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
    # typical 10-30 sweeps
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
    # the sweep kernel alone: graph replays with no sweeps (set-up and
    # finish), with exactly the sweeps convergence needs (all busy) and with
    # the cap of 120 (the rest idle)
    sw = tsm["sweeps"]
    t_cap = {}
    for cap in (0, sw, 120):
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=run.ctx.stream):
            two_sided(cap)
        graph.replay()
        torch.cuda.synchronize()
        t_cap[cap] = timed(graph.replay)
        del graph
    busy = (t_cap[sw] - t_cap[0]) / max(sw, 1)
    idle = (t_cap[120] - t_cap[sw]) / max(120 - sw, 1)
    tsm["sweep_kernel"] = extrap_sweep_bytes(wl.mesh, (~torch.isnan(gl[0])).cpu().numpy(), busy)
    tsm["sweep_kernel"].update(busy_us=busy, idle_us=idle, setup_and_finish_us=t_cap[0])
    sk = tsm["sweep_kernel"]
    log(f"extrapolation sweep: busy {busy:.2f} us, idle {idle:.2f} us, set-up and finish {t_cap[0]:.1f} us; "
        f"{sk['algorithmic_bytes'] / 1e6:.2f} MB algorithmic per sweep -> {sk['GBps']:.0f} GB/s "
        f"({100 * sk['hbm_frac']:.1f} % of HBM)")
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
        V.curvature(run.ctx, run.mesh, run.alpha, ah, cn, kp, force=fs, opts=V.csf_opts(n_smooth=2, sigma=0.0589))

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
    return two


if __name__ == "__main__":
    sys.exit(main())
