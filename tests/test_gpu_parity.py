"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Every test runs the library on seeded synthetic workloads and compares with
the oracle element by element (lists and status codes exactly; floating point
to the tolerances in tests/parity.py).
"""
import sys

import numpy as np
import pytest

import oracle
from synth import meshes, workloads
from tests import parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def V():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_14938_amd import vofpc
    return vofpc


@pytest.fixture(scope="module")
def runner(V):
    from paper_2604_14938_amd import runner as R
    return R


_WL = {}


def _wl(name):
    if name not in _WL:
        if name == "hex16":
            _WL[name] = workloads.hex_sphere()
        elif name == "vor12":
            _WL[name] = workloads.voronoi_bubble(n=12, seed=7, r=0.3)
        elif name == "vor46":
            _WL[name] = workloads.voronoi_bubble()
        elif name == "hex_small_bubbles":
            _WL[name] = workloads.random_bubbles(meshes.hex_mesh(24), seed=31, n_max=40, K=16, r_hi_h=5.0)
        elif name == "vor_small_bubbles":
            _WL[name] = workloads.random_bubbles(meshes.voronoi_box_mesh(16, seed=32), seed=33, n_max=40, K=16,
                                                 r_hi_h=3.0)
    return _WL[name]


@pytest.mark.parametrize("name", ["hex16", "vor12", "hex_small_bubbles", "vor_small_bubbles", "vor46"])
def test_step_matches_oracle(runner, name):
    wl = _wl(name)
    _say(f"step parity {name}: {wl.mesh.n_cells} cells, {wl.n_mixed} mixed")
    run = runner.PathRun(wl)
    run.step()
    g = run.results()
    ref = parity.oracle_path(wl)
    parity.check_lists(wl, g)
    # geometry
    import torch
    Vd, xc, Sf, xf = (t.cpu().numpy() for t in run.mesh.geometry())
    torch.cuda.synchronize()
    np.testing.assert_allclose(Vd, ref["geom"].V, rtol=1e-12)
    np.testing.assert_allclose(xc, ref["geom"].xc, atol=1e-12 * wl.mesh.h, rtol=0)
    np.testing.assert_allclose(Sf, ref["geom"].Sf, atol=1e-13 * wl.mesh.h ** 2, rtol=1e-12)
    rep = {}
    parity.check_interface(wl, g, ref["rec"], report=rep)
    band = g["band_idx"]
    parity.check_grad(wl, g["gradT"], ref["grad"], band)
    np.testing.assert_array_equal(g["grad_status"][band], ref["grad_status"][band])
    parity.check_mdot(g["mdot"], ref["mdot"][g["mixed_idx"]])
    np.testing.assert_allclose(g["Qdot"], -g["mdot"] * wl.h_lv, rtol=1e-15)
    _say(f"{name} ok: {rep}; mean iters {g['iters'].mean():.1f}")
    run.close()


def test_graph_replay_matches_eager(runner):
    wl = _wl("vor12")
    _say("graph replay vor12")
    import torch
    run = runner.PathRun(wl)
    run.step()
    eager = run.results()
    gr = run.capture()
    for rep in range(3):
        # clobber the outputs with eager work between replays
        run.buf.itf.A.fill_(-1.0)
        run.buf.mdot.fill_(7.0)
        run.buf.counts.zero_()
        torch.cuda.synchronize()
        gr.launch()
        got = run.results()
        for k in ("mixed_idx", "band_idx", "alpha_got", "A", "n", "d", "status", "iters", "mdot"):
            np.testing.assert_array_equal(got[k], eager[k], err_msg=f"replay {rep}: {k}")
        np.testing.assert_array_equal(got["gradT"][:, got["band_idx"]], eager["gradT"][:, eager["band_idx"]])
    run.close()


def test_replays_are_bitwise_deterministic(runner):
    wl = _wl("vor12")
    _say("determinism vor12")
    run = runner.PathRun(wl)
    outs = []
    for _ in range(3):
        run.step()
        outs.append(run.results())
    for k in ("alpha_got", "A", "n", "d", "s", "mdot"):
        np.testing.assert_array_equal(outs[0][k], outs[1][k])
        np.testing.assert_array_equal(outs[0][k], outs[2][k])
    run.close()


def test_separate_calls_match_the_step(V, runner):
    """compact -> reconstruct -> grad_T -> mass_transfer issued one by one,
    with the mean vertex rule and the two-sided gradients."""
    import torch
    wl = _wl("hex16")
    _say("separate calls hex16")
    run = runner.PathRun(wl, opts=V.recon_opts(vertex_mode=V.VERTEX_MEAN))
    b = run.buf
    V.compact(run.ctx, run.mesh, run.alpha, b.mixed_idx, b.band_idx, b.counts)
    V.reconstruct(run.ctx, run.mesh, run.alpha, b.mixed_idx, b.counts, b.itf, b.opts)
    V.grad_T(run.ctx, run.mesh, run.T, run.Tb, wl.T_sat, run.alpha, b.band_idx, b.counts, b.gradT, b.grad_status)
    N = wl.mesh.n_cells
    gl = torch.tensor(np.tile([[1.0], [0.5], [0.0]], (1, N)), device=run.dev)
    gv = torch.tensor(np.tile([[0.0], [0.0], [-2.0]], (1, N)), device=run.dev)
    md_c = torch.full((N,), 3.0, dtype=torch.float64, device=run.dev)
    qd_c = torch.full((N,), 3.0, dtype=torch.float64, device=run.dev)
    V.mass_transfer(run.ctx, run.mesh, run.alpha, b.mixed_idx, b.counts, b.itf, b.gradT, 0.6, 0.03, wl.h_lv,
                    b.mdot, b.Qdot, gradT_l=gl, gradT_v=gv, mdot_cells=md_c, Qdot_cells=qd_c)
    g = run.results()
    om = oracle.OMesh(wl.mesh)
    geom = oracle.geometry(om)
    rec = oracle.reconstruct(om, wl.alpha, geom, vertex_mode=1)
    parity.check_interface(wl, g, rec)
    md, _ = oracle.mass_transfer(geom, wl.alpha, rec["n"], rec["A"], np.zeros((3, N)), 0.6, 0.03, wl.h_lv,
                                 gl=gl.cpu().numpy(), gv=gv.cpu().numpy())
    parity.check_mdot(g["mdot"], md[g["mixed_idx"]])
    dense = md_c.cpu().numpy()
    expect = np.zeros(N)
    expect[g["mixed_idx"]] = g["mdot"]
    np.testing.assert_array_equal(dense, expect)
    np.testing.assert_array_equal(qd_c.cpu().numpy(), -expect * wl.h_lv)
    run.close()


@pytest.mark.parametrize("variant", ["standard", "printed", "all"])
def test_gradient_variants(V, runner, variant):
    import torch
    wl = _wl("vor12")
    _say(f"gradient variant {variant}")
    run = runner.PathRun(wl)
    run.step()
    b = run.buf
    N = wl.mesh.n_cells
    out = torch.zeros(3, N, dtype=torch.float64, device=run.dev)
    st = torch.zeros(N, dtype=torch.int32, device=run.dev)
    if variant == "all":
        V.grad_T(run.ctx, run.mesh, run.T, run.Tb, wl.T_sat, run.alpha, None, None, out, st, scope=V.SCOPE_ALL)
        cells = np.arange(N)
        ref, rst = oracle.grad(wl.mesh, oracle.geometry(wl.mesh), wl.T, wl.T_bface, wl.T_sat, wl.alpha)
    else:
        var = V.GRAD_STANDARD if variant == "standard" else V.GRAD_PRINTED
        V.grad_T(run.ctx, run.mesh, run.T, run.Tb, wl.T_sat, run.alpha, b.band_idx, b.counts, out, st, variant=var)
        cells = run.results()["band_idx"]
        ref, rst = oracle.grad(wl.mesh, oracle.geometry(wl.mesh), wl.T, wl.T_bface, wl.T_sat, wl.alpha,
                               modified=(variant != "standard"), printed=(variant == "printed"))
    torch.cuda.synchronize()
    parity.check_grad(wl, out.cpu().numpy(), ref, cells)
    np.testing.assert_array_equal(st.cpu().numpy()[cells], rst[cells])
    run.close()


@pytest.mark.parametrize("name", ["vor12", "hex_small_bubbles"])
@pytest.mark.parametrize("weight,extended,scope", [(1, False, "band"), (2, False, "all"), (0, True, "band"),
                                                   (1, True, "all"), (2, True, "band")])
def test_gradient_weights_and_vertex_stencil(V, runner, name, weight, extended, scope):
    """Least-squares weights 1/|r|, 1/|r|^2 and the vertex-neighbour stencil
    (App. B) against the oracle, over the band and over every cell."""
    import torch
    wl = _wl(name)
    _say(f"gradient weight={weight} extended={extended} scope={scope} on {name}")
    run = runner.PathRun(wl)
    run.step()
    b = run.buf
    N = wl.mesh.n_cells
    out = torch.zeros(3, N, dtype=torch.float64, device=run.dev)
    st = torch.zeros(N, dtype=torch.int32, device=run.dev)
    var = V.GRAD_MODIFIED | {0: 0, 1: V.GRAD_W_INV_DIST, 2: V.GRAD_W_INV_DIST2}[weight]
    if extended:
        var |= V.GRAD_VERTEX_STENCIL
    torch.cuda.synchronize()
    if scope == "all":
        V.grad_T(run.ctx, run.mesh, run.T, run.Tb, wl.T_sat, run.alpha, None, None, out, st, scope=V.SCOPE_ALL,
                 variant=var)
        cells = np.arange(N)
    else:
        V.grad_T(run.ctx, run.mesh, run.T, run.Tb, wl.T_sat, run.alpha, b.band_idx, b.counts, out, st, variant=var)
        cells = run.results()["band_idx"]
    torch.cuda.synchronize()
    ref, rst = oracle.grad(wl.mesh, oracle.geometry(wl.mesh), wl.T, wl.T_bface, wl.T_sat, wl.alpha,
                           weight=weight, extended=extended)
    parity.check_grad(wl, out.cpu().numpy(), ref, cells)
    np.testing.assert_array_equal(st.cpu().numpy()[cells], rst[cells])
    run.close()


def test_gradient_variant_flags_are_checked(V, runner):
    import torch
    wl = _wl("vor12")
    run = runner.PathRun(wl)
    N = wl.mesh.n_cells
    out = torch.zeros(3, N, dtype=torch.float64, device=run.dev)
    for bad in (V.GRAD_W_INV_DIST | V.GRAD_W_INV_DIST2, 0x80, 3):
        with pytest.raises(V.VofpcError):
            V.grad_T(run.ctx, run.mesh, run.T, run.Tb, wl.T_sat, run.alpha, None, None, out, scope=V.SCOPE_ALL,
                     variant=bad)
    run.close()


def test_fixed_isovalue_and_vertex_override(V, runner):
    import torch
    wl = _wl("vor12")
    _say("fixed iso + vertex override vor12")
    rng = np.random.default_rng(4)
    om = oracle.OMesh(wl.mesh)
    geom = oracle.geometry(om)
    phi = oracle.vertex_field(om, geom.xc, wl.alpha) + rng.uniform(-0.02, 0.02, wl.mesh.n_verts)
    phi_t = torch.tensor(phi, device="cuda")
    for fixed in (False, True):
        run = runner.PathRun(wl, opts=V.recon_opts(fixed_iso=int(fixed), iso=0.5, phi_vertex=phi_t))
        run.step()
        g = run.results()
        rec = oracle.reconstruct(om, wl.alpha, geom, fixed_iso=fixed, iso=0.5, phi=phi)
        parity.check_interface(wl, g, rec)
        if fixed:
            assert np.all(g["s"][g["status"] == 0] == 0.5)
        run.close()


def test_hint_bracket_same_result_fewer_evaluations(V, runner):
    import torch
    wl = _wl("vor12")
    _say("hint bracket vor12")
    om = oracle.OMesh(wl.mesh)
    geom = oracle.geometry(om)
    plain = oracle.reconstruct(om, wl.alpha, geom)
    mixed = np.nonzero(plain["status"] != oracle.NOT_MIXED)[0]
    s = plain["s"]
    rng = np.random.default_rng(9)
    # good hints for most cells, wrong ones for every fifth cell
    off = np.where(np.arange(wl.mesh.n_cells) % 5 == 0, 0.02, 0.0) + rng.uniform(-2e-4, 2e-4, wl.mesh.n_cells)
    lo = s + off - 1e-3
    hi = s + off + 1e-3
    ref = oracle.reconstruct(om, wl.alpha, geom, hint_lo=lo, hint_hi=hi)
    hl = torch.tensor(lo[mixed], device="cuda")
    hh = torch.tensor(hi[mixed], device="cuda")
    run = runner.PathRun(wl, opts=V.recon_opts(bracket=V.BRACKET_HINT), hint_lo=hl, hint_hi=hh)
    run.step()
    g = run.results()
    parity.check_interface(wl, g, ref)
    assert np.mean(g["iters"]) < np.mean(plain["iters"][mixed])
    assert np.sum(g["status"] == V.CELL_LEARNED_FALLBACK) > 0
    run.close()


def test_edge_cases_empty_all_and_single(V, runner):
    """No mixed cell; every cell mixed with a constant field; one mixed cell."""
    import torch
    mesh = meshes.hex_mesh(6)
    N = mesh.n_cells
    for label, alpha in (("empty", np.ones(N)), ("uniform", np.full(N, 0.37)),
                         ("single_interior", np.where(np.arange(N) == 100, 0.3, 1.0)),
                         ("single_corner", np.where(np.arange(N) == 0, 0.3, 1.0))):
        _say(f"edge case {label}")
        wl = workloads.Workload(label, mesh, alpha, np.full(N, 373.15), np.full(mesh.n_faces, 373.15))
        run = runner.PathRun(wl)
        run.step()
        g = run.results()
        parity.check_lists(wl, g)
        rec = oracle.reconstruct(wl.mesh, wl.alpha)
        parity.check_interface(wl, g, rec)
        if label == "uniform":
            assert np.all(g["status"] == V.CELL_DEGENERATE) and np.all(g["A"] == 0)
        if label == "single_interior":
            # every vertex of an interior cell of a uniform grid gets the same
            # inverse-distance value and the alpha gradient vanishes
            assert g["n_mixed"] == 1 and g["status"][0] == V.CELL_DEGENERATE and g["A"][0] == 0
        if label == "single_corner":
            assert g["n_mixed"] == 1 and g["status"][0] == V.CELL_OK and g["A"][0] > 0
        run.close()
    torch.cuda.synchronize()


def test_repeated_launches_share_the_cell_queue(V, runner):
    """Launches of different sizes in a row on one context (the reconstruction
    hands cells to blocks through a per-context counter) give the results of
    a full launch for every cell they cover."""
    import torch
    wl = _wl("vor12")
    _say("repeated launches vor12")
    run = runner.PathRun(wl)
    run.step()
    full = run.results()
    b = run.buf
    M = full["n_mixed"]
    cnt = torch.zeros(2, dtype=torch.int32, device=run.dev)
    for m in (M, 3, 0, 1, M - 1, M):
        cnt[0] = m
        cnt[1] = full["n_band"]
        b.itf.status.fill_(-1)
        torch.cuda.synchronize()
        V.reconstruct(run.ctx, run.mesh, run.alpha, b.mixed_idx, cnt, b.itf)
        torch.cuda.synchronize()
        st = b.itf.status.cpu().numpy()
        np.testing.assert_array_equal(st[:m], full["status"][:m])
        assert np.all(st[m:] == -1)
        np.testing.assert_array_equal(b.itf.alpha_got[:m].cpu().numpy(), full["alpha_got"][:m])
    run.close()


def _prism_workload(sides, layers=12, fan=False, tilt=0.3):
    """Columns of n-gon prismatoids side by side (one column per entry of
    `sides`), a tilted plane through each: cells of every kernel class, up
    to 128 vertices, 66 faces and 64-vertex faces (with fan caps, 240 faces
    and cuts of 80 chords)."""
    parts = [meshes.prism_column(n, layers, origin=(2.0 * i, 0.0, 0.0), fan_caps=fan) for i, n in enumerate(sides)]
    mesh = meshes.concat(parts)
    c = mesh.cell_vertex_mean()
    x0 = 2.0 * np.floor((c[:, 0] + 1.0) / 2.0)
    d = (c[:, 2] - 0.5) - tilt * (c[:, 0] - x0 - 0.3 * c[:, 2])
    h = 1.0 / layers
    alpha = np.clip(0.5 - d / (6.0 * h), 0.0, 1.0)
    fc = mesh.face_vertex_mean()
    T = 373.15 + 2.0 * c[:, 2] + 0.5 * (c[:, 0] - x0)
    Tb = 373.15 + 2.0 * fc[:, 2] + 0.5 * (fc[:, 0] - 2.0 * np.floor((fc[:, 0] + 1.0) / 2.0))
    wl = workloads.Workload(f"prisms{sides}", mesh, alpha, T, Tb)
    return wl, parts


@pytest.mark.parametrize("sides,fan", [((4, 8, 20, 40, 64), False), ((64,), False), ((80,), True)])
def test_large_cells_use_the_wide_kernel_variants(V, runner, sides, fan):
    """Cells beyond the Voronoi sizes (n-gon faces up to 64 vertices, up to
    162 vertices and 240 faces per cell) run in the wide kernel variants,
    bucketed by class with the small ones or alone, and give the oracle's
    results; their cuts have more chords than a cached topology holds, so the
    search runs on full evaluations, and the nearly flat cuts of the fan-capped
    column (80 chords, more than the lanes of a wave) label their loop
    through LDS."""
    wl, parts = _prism_workload(sides, fan=fan, tilt=0.02 if fan else 0.3)
    _say(f"large cells {sides}: {wl.mesh.n_cells} cells, {wl.n_mixed} mixed")
    run = runner.PathRun(wl, parts=parts if len(parts) > 1 else None)
    cls = run.mesh.classes()
    if len(sides) > 1:
        assert cls["bucketed"] and all(k > 0 for k in cls["cells"]), cls
    else:
        assert not cls["bucketed"] and cls["cells"][3] == wl.mesh.n_cells, cls
    run.step()
    g = run.results()
    ref = parity.oracle_path(wl)
    parity.check_lists(wl, g)
    rep = {}
    parity.check_interface(wl, g, ref["rec"], report=rep)
    assert np.all(g["status"] == V.CELL_OK) and np.all(g["A"] > 0)
    band = g["band_idx"]
    parity.check_grad(wl, g["gradT"], ref["grad"], band)
    np.testing.assert_array_equal(g["grad_status"][band], ref["grad_status"][band])
    parity.check_mdot(g["mdot"], ref["mdot"][g["mixed_idx"]])
    _say(f"large cells ok: {rep}; {g['n_mixed']} mixed, mean iters {g['iters'].mean():.1f}")
    run.close()


def test_out_of_range_and_nan_fractions(V, runner):
    """Volume fractions outside [0, 1] or NaN are never mixed (the lists
    skip them, the crossing test sees them as they are), and a mixed list
    that names them explicitly gets the BAD_INPUT status for them with the
    empty interface, while the other entries are reconstructed as usual."""
    import torch
    base = workloads.hex_sphere()
    N = base.mesh.n_cells
    alpha = base.alpha.copy()
    bad = [0, 15, N - 1]
    alpha[bad] = [np.nan, -0.1, 1.2]
    wl = workloads.Workload("bad_fractions", base.mesh, alpha, base.T, base.T_bface)
    _say(f"bad fractions at {bad}")
    run = runner.PathRun(wl)
    run.step()
    g = run.results()
    parity.check_lists(wl, g)
    assert not set(bad) & set(g["mixed_idx"].tolist())
    ref = parity.oracle_path(wl)
    parity.check_interface(wl, g, ref["rec"])
    band = g["band_idx"]
    parity.check_grad(wl, g["gradT"], ref["grad"], band)
    parity.check_mdot(g["mdot"], ref["mdot"][g["mixed_idx"]])
    # an explicit list with the bad cells and one mixed cell
    good = int(g["mixed_idx"][0])
    lst = torch.tensor(bad + [good] + [0] * (N - 4), dtype=torch.int32, device=run.dev)
    cnt = torch.tensor([4, 0], dtype=torch.int32, device=run.dev)
    itf = V.Interface.empty(N, run.dev)
    torch.cuda.synchronize()
    V.reconstruct(run.ctx, run.mesh, run.alpha, lst, cnt, itf)
    torch.cuda.synchronize()
    st = itf.status[:4].cpu().numpy()
    np.testing.assert_array_equal(st, [V.CELL_BAD_INPUT] * 3 + [ref["rec"]["status"][good]])
    assert np.all(np.isnan(itf.s[:3].cpu().numpy())) and np.all(itf.A[:3].cpu().numpy() == 0)
    assert abs(itf.alpha_got[3].item() - ref["rec"]["alpha_got"][good]) <= 1e-10
    np.testing.assert_array_equal(ref["rec"]["status"][bad], [oracle.BAD_INPUT] * 3)
    run.close()


def test_iteration_cap_gives_consistent_cuts(V, runner):
    """With the evaluation cap far below what the tolerance needs, cells end
    with MAX_ITER (or OK when the cap sufficed, NO_ROOT where the volume
    jumps over the target) and report the kept bracket end; whatever the
    search did, every reported interface must be the cut at the reported
    isovalue.  Both sides take the oracle's vertex field (the library's
    caller-supplied field option), so that the breakpoints of the volume
    function, where it may jump, are the same numbers on both: the oracle's
    cut at the GPU's s then gives the same liquid fraction, area, normal and
    distance."""
    import torch
    wl = _wl("vor12")
    geom = oracle.geometry(wl.mesh)
    phi = oracle.vertex_field(wl.mesh, geom.xc, wl.alpha)
    h = wl.mesh.h
    for cap in (3, 9):
        phi_d = torch.as_tensor(phi, dtype=torch.float64, device="cuda")
        run = runner.PathRun(wl, opts=V.recon_opts(max_iter=cap, phi_vertex=phi_d))
        run.step()
        g = run.results()
        st = g["status"]
        _say(f"iteration cap {cap}: {len(st)} mixed, statuses {np.bincount(st, minlength=8)}")
        assert set(np.unique(st).tolist()) <= {V.CELL_OK, V.CELL_MAX_ITER, V.CELL_NO_ROOT}
        assert (st == V.CELL_MAX_ITER).any()
        for k, P in enumerate(g["mixed_idx"]):
            c = oracle.cut_cell(wl.mesh, int(P), geom.xc, phi, float(g["s"][k]))
            assert abs(c["V"] / geom.V[P] - g["alpha_got"][k]) <= 1e-12, (cap, int(P))
            assert abs(c["A"] - g["A"][k]) <= 1e-9 * c["A"] + 1e-9 * h * h
            n = c["S"] / np.linalg.norm(c["S"])
            assert np.linalg.norm(n - g["n"][:, k]) <= 1e-9
            assert abs(-(n @ c["c"]) - g["d"][k]) <= 1e-9 * h
        run.close()
    torch.cuda.synchronize()


def test_singular_least_squares_matrix(V):
    """A column of cells with only the cells above and below as neighbours
    (every side face a symmetry face): the least-squares matrix has rank one,
    so every cell gets G_SINGULAR and a zero gradient, as in the oracle."""
    import torch
    mesh = meshes.prism_column(6, 5)
    mesh.face_bc = np.where(mesh.face_neigh < 0, 2, 0).astype(np.int8)
    N = mesh.n_cells
    T = 373.15 + 2.0 * mesh.cell_vertex_mean()[:, 2]
    alpha = np.ones(N)
    geom = oracle.geometry(mesh)
    og, ost = oracle.grad(mesh, geom, T, np.zeros(mesh.n_faces), 373.15, alpha)
    assert np.all(ost == oracle.G_SINGULAR) and np.all(og == 0)
    ctx = V.Context(0, stream=torch.cuda.Stream())
    m = V.Mesh(ctx, mesh)
    f64 = dict(dtype=torch.float64, device=ctx.device)
    g = torch.full((3, N), np.nan, **f64)
    st = torch.full((N,), -1, dtype=torch.int32, device=ctx.device)
    torch.cuda.synchronize()
    V.grad_T(ctx, m, torch.as_tensor(T, **f64), torch.zeros(mesh.n_faces, **f64), 373.15,
             torch.as_tensor(alpha, **f64), None, None, g, st, scope=V.SCOPE_ALL)
    torch.cuda.synchronize()
    _say("singular least squares on a symmetric column")
    np.testing.assert_array_equal(st.cpu().numpy(), np.full(N, V.CELL_G_SINGULAR))
    assert np.all(g.cpu().numpy() == 0)
    m.close()
