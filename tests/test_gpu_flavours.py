"""GPU parity of every reconstruction kernel flavour (tile shape) the tuner
can pick: one cell per wavefront (3 or 4 waves per SIMD) and G lanes per cell
(G = 1, 2, 4 for class 0, 4, 8, 16 for the Voronoi classes 1 and 2), each
forced through vofpc_mesh_set_tune and compared with the oracle to the parity
bar."""
import sys

import numpy as np
import pytest

import oracle
from synth import meshes, workloads
from tests import parity

pytestmark = pytest.mark.gpu

C0 = [3, 4, 11, 12, 14]      # class 0 (hexahedra and smaller cells)
C1 = [3, 4, 14, 18, 26]      # classes 1 and 2 (Voronoi cells)


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
        elif name == "hex_bubbles":
            _WL[name] = workloads.random_bubbles(meshes.hex_mesh(24), seed=31, n_max=40, K=16, r_hi_h=5.0)
        elif name == "vor_bubbles":
            _WL[name] = workloads.random_bubbles(meshes.voronoi_box_mesh(16, seed=32), seed=33, n_max=40, K=16,
                                                 r_hi_h=3.0)
        elif name == "batch":
            a = workloads.random_bubbles(meshes.hex_mesh(20), seed=41, n_max=30, K=16, r_hi_h=5.0)
            b = workloads.random_bubbles(meshes.voronoi_box_mesh(12, seed=42), seed=43, n_max=20, K=16,
                                         r_hi_h=3.0)
            _WL[name] = (workloads.concat_workloads([a, b]), [a.mesh, b.mesh])
    return _WL[name]


def _tune_for(run, f0, f1):
    """Flavour f0 for class 0, f1 for the Voronoi classes 1 and 2."""
    cls = run.mesh.classes()
    t = [f0 if cls["cells"][0] else 3, f1 if cls["cells"][1] else 3, f1 if cls["cells"][2] else 3, 3]
    run.mesh.set_tune(t)
    assert run.mesh.classes()["tune"][:3] == t[:3]
    return cls


def _check_step(wl, g, ref):
    parity.check_lists(wl, g)
    rep = {}
    parity.check_interface(wl, g, ref["rec"], report=rep)
    band = g["band_idx"]
    parity.check_grad(wl, g["gradT"], ref["grad"], band)
    parity.check_mdot(g["mdot"], ref["mdot"][g["mixed_idx"]])
    return rep


_REF = {}


def _ref(name, wl):
    if name not in _REF:
        _REF[name] = parity.oracle_path(wl)
    return _REF[name]


@pytest.mark.parametrize("f", C0)
@pytest.mark.parametrize("name", ["hex16", "hex_bubbles"])
def test_class0_flavours_match_the_oracle(runner, name, f):
    wl = _wl(name)
    _say(f"flavour {f} on {name}: {wl.n_mixed} mixed")
    run = runner.PathRun(wl)
    cls = _tune_for(run, f, 3)
    assert cls["cells"][0] == wl.mesh.n_cells and not cls["bucketed"]
    run.step()
    g = run.results()
    rep = _check_step(wl, g, _ref(name, wl))
    _say(f"flavour {f} {name} ok: {rep}; mean iters {g['iters'].mean():.1f}")
    run.close()


@pytest.mark.parametrize("f", C1)
@pytest.mark.parametrize("name", ["vor12", "vor_bubbles", "vor46"])
def test_class1_flavours_match_the_oracle(runner, name, f):
    wl = _wl(name)
    _say(f"flavour {f} on {name}: {wl.n_mixed} mixed")
    run = runner.PathRun(wl)
    cls = _tune_for(run, 3, f)
    assert cls["cells"][1] > 0.9 * wl.mesh.n_cells and cls["cells"][3] == 0, cls
    assert run.mesh.classes()["tune"][1] == f
    run.step()
    g = run.results()
    rep = _check_step(wl, g, _ref(name, wl))
    _say(f"flavour {f} {name} ok: {rep}; mean iters {g['iters'].mean():.1f}")
    run.close()


@pytest.mark.parametrize("f0,f1", [(12, 14), (14, 18), (12, 26), (3, 14), (12, 3)])
def test_bucketed_batch_with_group_flavours(runner, f0, f1):
    """Hexahedra and Voronoi cells in one mesh: two classes, each launched
    on its own entries with its own flavour (class 0 holds the hexahedra and
    the smallest Voronoi cells, so its build is the general class-0 one)."""
    wl, parts = _wl("batch")
    _say(f"bucketed batch flavours {f0}/{f1}: {wl.n_mixed} mixed")
    run = runner.PathRun(wl, parts=parts)
    cls = _tune_for(run, f0, f1)
    assert cls["bucketed"], cls
    run.step()
    g = run.results()
    rep = _check_step(wl, g, _ref("batch", wl))
    _say(f"bucketed {f0}/{f1} ok: {rep}")
    run.close()


@pytest.mark.parametrize("f", [14, 18, 26])
def test_hint_bracket_checked_with_two_cuts(V, runner, f):
    """A narrowed bracket per cell (good for most cells, off by 0.02 for every
    fifth): its centre and the end on the root's side are cut first; the
    statuses (LEARNED_FALLBACK where the root is outside the bracket) and
    results equal the oracle's hint path, which cuts both ends."""
    import torch
    wl = _wl("vor12")
    om = oracle.OMesh(wl.mesh)
    geom = oracle.geometry(om)
    plain = oracle.reconstruct(om, wl.alpha, geom)
    mixed = np.nonzero(plain["status"] != oracle.NOT_MIXED)[0]
    rng = np.random.default_rng(9)
    off = np.where(np.arange(wl.mesh.n_cells) % 5 == 0, 0.02, 0.0) + rng.uniform(-2e-4, 2e-4, wl.mesh.n_cells)
    lo = plain["s"] + off - 1e-3
    hi = plain["s"] + off + 1e-3
    ref = oracle.reconstruct(om, wl.alpha, geom, hint_lo=lo, hint_hi=hi)
    _say(f"hint bracket flavour {f}")
    run = runner.PathRun(wl, opts=V.recon_opts(bracket=V.BRACKET_HINT),
                         hint_lo=torch.tensor(lo[mixed], device="cuda"), hint_hi=torch.tensor(hi[mixed], device="cuda"))
    _tune_for(run, 3, f)
    run.step()
    g = run.results()
    parity.check_interface(wl, g, ref)
    assert np.sum(g["status"] == V.CELL_LEARNED_FALLBACK) > 0
    assert np.mean(g["iters"]) < np.mean(plain["iters"][mixed])
    run.close()


@pytest.mark.parametrize("f0,f1", [(12, 14), (11, 26)])
def test_fixed_isovalue_override_and_iteration_cap(V, runner, f0, f1):
    """The fixed-isovalue cut, a caller-supplied vertex field and an
    evaluation cap far below the tolerance's needs (every reported interface
    is the oracle's cut at the reported isovalue on the same vertex field)."""
    import torch
    for name, f in (("hex16", (f0, 3)), ("vor12", (3, f1))):
        wl = _wl(name)
        geom = oracle.geometry(wl.mesh)
        phi = oracle.vertex_field(wl.mesh, geom.xc, wl.alpha)
        phi_d = torch.as_tensor(phi, dtype=torch.float64, device="cuda")
        _say(f"fixed isovalue / override / cap on {name} flavours {f}")
        run = runner.PathRun(wl, opts=V.recon_opts(fixed_iso=1, iso=0.5))
        _tune_for(run, *f)
        run.step()
        g = run.results()
        ref = oracle.reconstruct(wl.mesh, wl.alpha, geom, fixed_iso=True, iso=0.5)
        parity.check_interface(wl, g, ref)
        run.close()
        run = runner.PathRun(wl, opts=V.recon_opts(phi_vertex=phi_d))
        _tune_for(run, *f)
        run.step()
        g = run.results()
        parity.check_interface(wl, g, oracle.reconstruct(wl.mesh, wl.alpha, geom, phi=phi))
        run.close()
        h = wl.mesh.h
        for cap in (3, 9):
            run = runner.PathRun(wl, opts=V.recon_opts(max_iter=cap, phi_vertex=phi_d))
            _tune_for(run, *f)
            run.step()
            g = run.results()
            st = g["status"]
            assert set(np.unique(st).tolist()) <= {V.CELL_OK, V.CELL_MAX_ITER, V.CELL_NO_ROOT}
            assert (st == V.CELL_MAX_ITER).any()
            for k, P in enumerate(g["mixed_idx"]):
                c = oracle.cut_cell(wl.mesh, int(P), geom.xc, phi, float(g["s"][k]))
                assert abs(c["V"] / geom.V[P] - g["alpha_got"][k]) <= 1e-12, (cap, int(P))
                assert abs(c["A"] - g["A"][k]) <= 1e-9 * c["A"] + 1e-9 * h * h
                if c["A"] > 0:
                    n = c["S"] / np.linalg.norm(c["S"])
                    assert np.linalg.norm(n - g["n"][:, k]) <= 1e-9
                    assert abs(-(n @ c["c"]) - g["d"][k]) <= 1e-9 * h
            run.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("f", [11, 12, 14])
def test_edge_cases_with_group_flavours(V, runner, f):
    """No mixed cell, every cell mixed with a constant field (degenerate
    vertex field everywhere), one interior mixed cell (degenerate), one corner
    cell, and NaN / out-of-range fractions named in an explicit list."""
    import torch
    mesh = meshes.hex_mesh(6)
    N = mesh.n_cells
    for label, alpha in (("empty", np.ones(N)), ("uniform", np.full(N, 0.37)),
                         ("single_interior", np.where(np.arange(N) == 100, 0.3, 1.0)),
                         ("single_corner", np.where(np.arange(N) == 0, 0.3, 1.0))):
        _say(f"edge case {label} flavour {f}")
        wl = workloads.Workload(label, mesh, alpha, np.full(N, 373.15), np.full(mesh.n_faces, 373.15))
        run = runner.PathRun(wl)
        _tune_for(run, f, 3)
        run.step()
        g = run.results()
        parity.check_lists(wl, g)
        parity.check_interface(wl, g, oracle.reconstruct(wl.mesh, wl.alpha))
        run.close()
    base = _wl("hex16")
    alpha = base.alpha.copy()
    bad = [0, 15, N - 1]
    alpha[bad] = [np.nan, -0.1, 1.2]
    wl = workloads.Workload("bad", base.mesh, alpha, base.T, base.T_bface)
    run = runner.PathRun(wl)
    _tune_for(run, f, 3)
    run.step()
    g = run.results()
    ref = oracle.reconstruct(wl.mesh, wl.alpha)
    parity.check_interface(wl, g, ref)
    good = int(g["mixed_idx"][0])
    Nb = base.mesh.n_cells
    lst = torch.tensor(bad + [good] + [0] * (Nb - 4), dtype=torch.int32, device=run.dev)
    cnt = torch.tensor([4, 0], dtype=torch.int32, device=run.dev)
    itf = V.Interface.empty(Nb, run.dev)
    torch.cuda.synchronize()
    V.reconstruct(run.ctx, run.mesh, run.alpha, lst, cnt, itf)
    torch.cuda.synchronize()
    st = itf.status[:4].cpu().numpy()
    np.testing.assert_array_equal(st, [V.CELL_BAD_INPUT] * 3 + [ref["status"][good]])
    run.close()


def test_repeated_launches_and_replays_with_group_flavours(V, runner):
    """Launches of different sizes in a row share the batch counter, and a
    captured step replays to the eager results, with a group flavour."""
    import torch
    wl = _wl("vor12")
    _say("repeated launches / replay flavour 14")
    run = runner.PathRun(wl)
    _tune_for(run, 3, 14)
    run.step()
    full = run.results()
    b = run.buf
    M = full["n_mixed"]
    cnt = torch.zeros(2, dtype=torch.int32, device=run.dev)
    for m in (M, 3, 0, 1, 17, M - 1, M):
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
    gr = run.capture()
    for rep in range(3):
        run.buf.itf.A.fill_(-1.0)
        run.buf.counts.zero_()
        torch.cuda.synchronize()
        gr.launch()
        got = run.results()
        for k in ("mixed_idx", "alpha_got", "A", "n", "d", "status", "iters", "mdot"):
            np.testing.assert_array_equal(got[k], full[k], err_msg=f"replay {rep}: {k}")
    run.close()


def test_set_tune_rejects_flavours_without_a_build(V, runner):
    wl = _wl("vor12")
    run = runner.PathRun(wl)
    for bad in ([3, 12, 3, 3], [3, 7, 3, 3], [3, 3, 12, 3] if run.mesh.classes()["cells"][2] else [3, 19, 3, 3]):
        before = run.mesh.classes()["tune"]
        with pytest.raises(V.VofpcError):
            run.mesh.set_tune(bad)
        assert run.mesh.classes()["tune"] == before
    run.close()
