"""Batches through one step: meshes uploaded separately and joined on the
device (vofpc_mesh_concat), stepped as one mesh, against the oracle on the
union built on the host."""
import sys

import numpy as np
import pytest

from synth import meshes, workloads
from tests import parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_14938_amd import runner
    return runner


def _check_step(wl, g):
    ref = parity.oracle_path(wl)
    parity.check_lists(wl, g)
    rep = {}
    parity.check_interface(wl, g, ref["rec"], report=rep)
    band = g["band_idx"]
    parity.check_grad(wl, g["gradT"], ref["grad"], band)
    np.testing.assert_array_equal(g["grad_status"][band], ref["grad_status"][band])
    parity.check_mdot(g["mdot"], ref["mdot"][g["mixed_idx"]])
    return rep


def test_device_concat_equals_host_concat(R):
    """Geometry of parts joined on the device equals that of the union
    uploaded whole, bit for bit (each cell's geometry uses only its own faces
    and vertices)."""
    import torch
    from paper_2604_14938_amd import vofpc as V
    parts = [meshes.hex_mesh(6), meshes.voronoi_box_mesh(5, seed=11), meshes.hex_mesh(3)]
    whole = meshes.concat(parts)
    _say(f"concat geometry: {[p.n_cells for p in parts]} cells")
    ctx = V.Context(0, stream=torch.cuda.Stream())
    ups = [V.Mesh(ctx, p) for p in parts]
    joined = V.Mesh.concat(ctx, ups)
    direct = V.Mesh(ctx, whole)
    info_j, info_d = joined.info(), direct.info()
    for k in ("n_cells", "n_faces", "n_verts", "max_faces", "max_verts", "max_face_verts", "max_edges"):
        assert info_j[k] == info_d[k], k
    for a, b in zip(joined.geometry(), direct.geometry()):
        torch.cuda.synchronize()
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    for m in ups + [joined, direct]:
        m.close()


def test_batched_hex_and_voronoi_step(R):
    """A hexahedral and a Voronoi mesh with many bubbles each, one step over
    both (the batched structure at reduced size: the CPU generators are the
    limit at full size)."""
    wls = workloads.batched(hex_n=32, vor_n=14, seed=3, n_max=300, K=12, r_hi_h=4.0)
    wl = workloads.concat_workloads(wls)
    _say(f"batched: {[w.mesh.n_cells for w in wls]} cells, {wl.n_mixed} mixed")
    run = R.PathRun(wl, parts=[w.mesh for w in wls])
    run.step()
    g = run.results()
    rep = _check_step(wl, g)
    kinds = np.searchsorted(wl.meta["cell_offsets"], g["mixed_idx"], side="right") - 1
    assert set(kinds.tolist()) == {0, 1}
    _say(f"batched ok: {rep}")
    run.close()


def test_multi_instance_time_steps_in_one_graph(R):
    """Independent Voronoi meshes of different sizes, each with a bubble
    turning around the box axis: one captured step over all of them, replayed
    after the fields of the next time step are written into its inputs."""
    import torch
    meshes_, radii, phases, field = workloads.multi_instance(n_inst=6, n_lo=2e3, n_hi=2e4, seed=5, steps=3, K=12)
    _say(f"multi-instance: {[m.n_cells for m in meshes_]} cells")
    wl0 = workloads.concat_workloads([field(i, 0) for i in range(len(meshes_))])
    run = R.PathRun(wl0, parts=meshes_)
    graph = run.capture()
    for t in range(3):
        wl = wl0 if t == 0 else workloads.concat_workloads([field(i, t) for i in range(len(meshes_))])
        run.alpha.copy_(torch.as_tensor(wl.alpha))
        run.T.copy_(torch.as_tensor(wl.T))
        run.Tb.copy_(torch.as_tensor(wl.T_bface))
        torch.cuda.synchronize()
        graph.launch()
        g = run.results()
        rep = _check_step(wl, g)
        _say(f"step {t}: {g['n_mixed']} mixed ok {rep}")
    run.close()


def test_buckets_and_autotune(R, tmp_path):
    """A hex + Voronoi union is bucketed by kernel class; every flavour the
    autotuner may pick gives the oracle's results; the choice is cached."""
    import torch
    from paper_2604_14938_amd import vofpc as V
    wls = workloads.batched(hex_n=24, vor_n=12, seed=8, n_max=200, K=12, r_hi_h=3.0)
    wl = workloads.concat_workloads(wls)
    _say(f"buckets + autotune: {[w.mesh.n_cells for w in wls]} cells, {wl.n_mixed} mixed")
    run = R.PathRun(wl, parts=[w.mesh for w in wls])
    cls = run.mesh.classes()
    assert cls["bucketed"] and cls["cells"][0] >= wls[0].mesh.n_cells and cls["cells"][1] > 0
    # the library's class counts are the host's assignment (the small
    # Voronoi cells leave the hexahedral class 0 of this union)
    import bench
    assert bench.mesh_hex0(wl.mesh)
    assert cls["cells"] == np.bincount(bench.cell_classes(wl.mesh, np.arange(wl.mesh.n_cells)), minlength=4).tolist()
    assert cls["cells"][0] == wls[0].mesh.n_cells
    ref = parity.oracle_path(wl)
    # the tuner's own pick (timing decides it: any flavour with a build)
    flavours = {3, 4} | {10 + g for g in (1, 2, 4, 8, 16)}
    choice, hit = V.autotune(run.ctx, run.mesh, run.alpha, cache_path=str(tmp_path / "tune.txt"))
    assert not hit and set(choice) <= flavours, choice
    assert run.mesh.classes()["tune"] == list(choice)
    run.step()
    g = run.results()
    parity.check_lists(wl, g)
    parity.check_interface(wl, g, ref["rec"])
    _say(f"tuned flavours {choice} ok")
    for flavour in (3, 4):
        # force a flavour through the cache file, then check the results
        path = tmp_path / f"tune{flavour}.txt"
        choice, hit = V.autotune(run.ctx, run.mesh, run.alpha, cache_path=str(path))
        assert not hit and set(choice) <= flavours, choice
        line = path.read_text().strip().rsplit(":", 1)[0] + f": {flavour} {flavour} 3 3\n"
        path.write_text(line)
        choice, hit = V.autotune(run.ctx, run.mesh, run.alpha, cache_path=str(path))
        assert hit and choice[:2] == [flavour, flavour]
        assert run.mesh.classes()["tune"][:2] == [flavour, flavour]
        run.step()
        g = run.results()
        parity.check_lists(wl, g)
        parity.check_interface(wl, g, ref["rec"])
        _say(f"flavour {flavour} ok")
    run.close()
    torch.cuda.synchronize()


def test_follow_on_rows_on_a_concatenated_mesh(R):
    """Extrapolated phase gradients, interface coupling and curvature on a
    hexahedral and a Voronoi mesh joined on the device, against the oracle on
    the union."""
    import torch
    import oracle
    from paper_2604_14938_amd import vofpc as V
    wls = [workloads.random_bubbles(meshes.hex_mesh(14), seed=41, n_max=12, K=12, r_hi_h=3.0),
           workloads.random_bubbles(meshes.voronoi_box_mesh(9, seed=42), seed=43, n_max=12, K=12, r_hi_h=2.5)]
    wl = workloads.concat_workloads(wls)
    _say(f"follow-on rows on a union of {[w.mesh.n_cells for w in wls]} cells, {wl.n_mixed} mixed")
    run = R.PathRun(wl, parts=[w.mesh for w in wls])
    run.step()
    g = run.results()
    b = run.buf
    N, NF = wl.mesh.n_cells, wl.mesh.n_faces
    f64 = dict(dtype=torch.float64, device=run.dev)
    gl, gv = torch.full((3, N), np.nan, **f64), torch.full((3, N), np.nan, **f64)
    rep = torch.zeros(2, dtype=torch.int32, device=run.dev)
    ad = torch.zeros(N, **f64)
    fi = torch.zeros(NF, dtype=torch.int32, device=run.dev)
    fa = torch.zeros(2, NF, **f64)
    nfo = torch.zeros(1, dtype=torch.int32, device=run.dev)
    ah, k = torch.zeros(N, **f64), torch.zeros(N, **f64)
    cn, F = torch.zeros(3, N, **f64), torch.zeros(3, N, **f64)
    torch.cuda.synchronize()
    V.extrapolate(run.ctx, run.mesh, run.alpha, run.T, run.Tb, wl.T_sat, b.mixed_idx, b.counts, b.itf, gl, gv, rep)
    V.robin(run.ctx, run.mesh, run.alpha, b.mixed_idx, b.band_idx, b.counts, b.itf, wl.k_l, wl.k_v, a_diag=ad,
            face_idx=fi, face_a=fa, n_face=nfo)
    V.curvature(run.ctx, run.mesh, run.alpha, ah, cn, k, force=F)
    torch.cuda.synchronize()
    geom = oracle.geometry(wl.mesh)
    rec = oracle.reconstruct(wl.mesh, wl.alpha, geom)
    grad, _ = oracle.grad(wl.mesh, geom, wl.T, wl.T_bface, wl.T_sat, wl.alpha)
    ogl, ogv, sweeps, dom = oracle.extrapolate(wl.mesh, geom, wl.alpha, grad, rec["n"], rec["A"])
    assert int(rep[0].item()) == sweeps
    scale = np.abs(grad[:, dom]).max()
    for a, o in ((gl, ogl), (gv, ogv)):
        assert np.abs(a.cpu().numpy()[:, dom] - o[:, dom]).max() <= 1e-9 * scale
    rb = oracle.robin(wl.mesh, geom, wl.alpha, rec["n"], rec["A"], wl.k_l, wl.k_v)
    nf = int(nfo.item())
    assert nf == rb["crossing"].sum()
    order = np.argsort(fi[:nf].cpu().numpy())
    np.testing.assert_array_equal(fi[:nf].cpu().numpy()[order], np.nonzero(rb["crossing"])[0])
    am = np.abs(rb["a_face"]).max()
    np.testing.assert_allclose(fa[:, :nf].cpu().numpy()[:, order], rb["a_face"][:, rb["crossing"]], rtol=0,
                               atol=1e-8 * am)
    cs = oracle.csf(wl.mesh, geom, wl.alpha, n_smooth=2)
    np.testing.assert_allclose(k.cpu().numpy(), cs["kappa"], rtol=0, atol=1e-9 * np.abs(cs["kappa"]).max())
    np.testing.assert_allclose(F.cpu().numpy(), cs["F"], rtol=0, atol=1e-9 * np.abs(cs["F"]).max())
    run.close()


@pytest.mark.parametrize("tune", [None, (3, 3, 3, 3), (4, 4, 4, 3), (14, 26, 4, 3), (12, 18, 26, 3)])
def test_learned_form_in_the_bucketed_launch(R, tune):
    """The learned bracket inside every kernel class of a bucketed launch
    (hexahedral and Voronoi cells together) gives the oracle's results, with
    the default flavours and with each flavour the tuner can pick per class
    (the full workload's pick is 14, 26, 4, 3)."""
    import os
    import torch
    from paper_2604_14938_amd import train, vofpc as V
    if not os.path.exists(train.DEFAULT_WEIGHTS):
        pytest.skip("no trained weights")
    params, dscale, _ = train.load()
    wls = workloads.batched(hex_n=24, vor_n=12, seed=9, n_max=200, K=12, r_hi_h=3.0)
    wl = workloads.concat_workloads(wls)
    _say(f"learned, bucketed: {[w.mesh.n_cells for w in wls]} cells, {wl.n_mixed} mixed")
    ctx = V.Context(0, stream=torch.cuda.Stream())
    mlp = V.Mlp(ctx)
    mlp.set_params(params)
    run = R.PathRun(wl, ctx=ctx, parts=[w.mesh for w in wls], mlp=mlp, delta_scale=dscale)
    assert run.mesh.classes()["bucketed"]
    if tune is not None:
        run.mesh.set_tune(list(tune))
        assert run.mesh.classes()["tune"] == list(tune)
    run.step()
    g = run.results()
    fb = g["status"] == V.CELL_LEARNED_FALLBACK
    g["status"] = np.where(fb, V.CELL_OK, g["status"])
    rep = _check_step(wl, g)
    _say(f"learned bucketed {tune} ok: {rep}; fallback rate {fb.mean():.3f}, mean evaluations {g['iters'].mean():.1f}")
    run.close()
    mlp.close()


@pytest.mark.parametrize("form", ["plain", "learned"])
def test_classes_side_by_side_or_in_turn_give_the_same_bits(R, form):
    """A bucketed step with the classes on two streams (the default) and
    with them in turn on one: every output bit for bit the same."""
    import os
    import torch
    from paper_2604_14938_amd import train, vofpc as V
    wls = workloads.batched(hex_n=24, vor_n=12, seed=11, n_max=200, K=12, r_hi_h=3.0)
    wl = workloads.concat_workloads(wls)
    mlp = dscale = None
    ctx = V.Context(0, stream=torch.cuda.Stream())
    if form == "learned":
        if not os.path.exists(train.DEFAULT_WEIGHTS):
            pytest.skip("no trained weights")
        params, dscale, _ = train.load()
        mlp = V.Mlp(ctx)
        mlp.set_params(params)
    run = R.PathRun(wl, ctx=ctx, parts=[w.mesh for w in wls], mlp=mlp, delta_scale=dscale or 0.0)
    cls = run.mesh.classes()
    assert cls["bucketed"] and cls["cells"][1] > 0 and cls["cells"][0] > 0
    _say(f"classes side by side / in turn ({form}): {wl.n_mixed} mixed, tune {cls['tune']}")
    out = []
    for overlap in (True, False, True):
        run.ctx.overlap_classes(overlap)
        run.step()
        out.append(run.results())
    for g in out[1:]:
        for k in ("mixed_idx", "status", "iters", "s", "n", "A", "d", "alpha_got", "mdot", "gradT"):
            np.testing.assert_array_equal(np.asarray(g[k]).view(np.uint8), np.asarray(out[0][k]).view(np.uint8), k)
    run.close()
    if mlp is not None:
        mlp.close()
