"""Phase gradients by pseudo-time extrapolation (Eq. extrapolation) and the
two-sided mass transfer: the HIP path against the oracle."""
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
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_14938_amd import runner
    return runner


def _run(R, wl, **opts):
    """One step, then the extrapolation on its interface; returns host arrays."""
    import torch
    from paper_2604_14938_amd import vofpc as V
    run = R.PathRun(wl)
    run.step()
    g = run.results()
    N = wl.mesh.n_cells
    gl = torch.full((3, N), float("nan"), dtype=torch.float64, device=run.dev)
    gv = torch.full((3, N), float("nan"), dtype=torch.float64, device=run.dev)
    rep = torch.zeros(2, dtype=torch.int32, device=run.dev)
    b = run.buf
    torch.cuda.synchronize()
    V.extrapolate(run.ctx, run.mesh, run.alpha, run.T, run.Tb, wl.T_sat, b.mixed_idx, b.counts, b.itf, gl, gv, rep,
                  opts=V.extrap_opts(**opts) if opts else None)
    md = torch.zeros(N, dtype=torch.float64, device=run.dev)
    qd = torch.zeros(N, dtype=torch.float64, device=run.dev)
    V.mass_transfer(run.ctx, run.mesh, run.alpha, b.mixed_idx, b.counts, b.itf, None, wl.k_l, wl.k_v, wl.h_lv,
                    md, qd, gradT_l=gl, gradT_v=gv)
    torch.cuda.synchronize()
    out = dict(step=g, gl=gl.cpu().numpy(), gv=gv.cpu().numpy(), sweeps=int(rep[0].item()), err=int(rep[1].item()),
               mdot=md[:g["n_mixed"]].cpu().numpy(), run=run)
    return out


def _oracle(wl, **opts):
    om = oracle.OMesh(wl.mesh)
    geom = oracle.geometry(om)
    rec = oracle.reconstruct(om, wl.alpha, geom)
    grad, _ = oracle.grad(om, geom, wl.T, wl.T_bface, wl.T_sat, wl.alpha)
    gl, gv, sweeps, dom = oracle.extrapolate(om, geom, wl.alpha, grad, rec["n"], rec["A"], **opts)
    mdot, _ = oracle.mass_transfer(geom, wl.alpha, rec["n"], rec["A"], grad, wl.k_l, wl.k_v, wl.h_lv, gl=gl, gv=gv)
    return dict(gl=gl, gv=gv, sweeps=sweeps, dom=dom, mdot=mdot, grad=grad)


@pytest.mark.parametrize("name", ["vor12", "hex_bubbles", "vor_bubbles"])
def test_extrapolation_matches_oracle(R, name):
    if name == "vor12":
        wl = workloads.voronoi_bubble(n=12, seed=7, r=0.3)
    elif name == "hex_bubbles":
        wl = workloads.random_bubbles(meshes.hex_mesh(24), seed=31, n_max=40, K=16, r_hi_h=5.0)
    else:
        wl = workloads.random_bubbles(meshes.voronoi_box_mesh(16, seed=32), seed=33, n_max=40, K=16, r_hi_h=3.0)
    _say(f"extrapolation {name}: {wl.mesh.n_cells} cells, {wl.n_mixed} mixed")
    g = _run(R, wl)
    ref = _oracle(wl)
    assert g["err"] == 0
    assert g["sweeps"] == ref["sweeps"], (g["sweeps"], ref["sweeps"])
    dom = ref["dom"]
    # written exactly on the domain
    np.testing.assert_array_equal(~np.isnan(g["gl"][0]), dom)
    scale = np.abs(ref["grad"][:, dom]).max()
    for k in ("gl", "gv"):
        err = np.abs(g[k][:, dom] - ref[k][:, dom])
        assert err.max() <= 1e-9 * scale, (k, err.max(), scale)
    parity.check_mdot(g["mdot"], ref["mdot"][g["step"]["mixed_idx"]])
    _say(f"{name}: {g['sweeps']} sweeps, domain {dom.sum()} cells ok")
    g["run"].close()


def test_extrapolation_edge_options(R):
    """No sweeps (outputs = the gradient on the domain), no rings (domain =
    mixed cells), and a loose tolerance, each against the oracle."""
    wl = workloads.voronoi_bubble(n=10, seed=4, r=0.3)
    for opts in (dict(max_iter=0), dict(layers=0), dict(tol=10.0), dict(layers=4, tol=1e-6)):
        _say(f"extrapolation options {opts}")
        g = _run(R, wl, **opts)
        ref = _oracle(wl, **opts)
        assert g["err"] == 0 and g["sweeps"] == ref["sweeps"]
        dom = ref["dom"]
        np.testing.assert_array_equal(~np.isnan(g["gl"][0]), dom)
        scale = np.abs(ref["grad"][:, dom]).max()
        for k in ("gl", "gv"):
            assert np.abs(g[k][:, dom] - ref[k][:, dom]).max() <= 1e-9 * scale
        g["run"].close()


def test_extrapolation_replays_in_a_graph(R):
    """After one eager call (which sets up the mesh's scratch), extrapolation
    and the two-sided mass transfer replay from a captured graph with the
    eager results."""
    import torch
    from paper_2604_14938_amd import vofpc as V
    wl = workloads.voronoi_bubble(n=10, seed=6, r=0.28)
    _say("extrapolation graph replay")
    g = _run(R, wl)
    run = g["run"]
    b = run.buf
    N = wl.mesh.n_cells
    gl = torch.zeros(3, N, dtype=torch.float64, device=run.dev)
    gv = torch.zeros(3, N, dtype=torch.float64, device=run.dev)
    md = torch.zeros(N, dtype=torch.float64, device=run.dev)
    qd = torch.zeros(N, dtype=torch.float64, device=run.dev)
    rep = torch.zeros(2, dtype=torch.int32, device=run.dev)
    torch.cuda.synchronize()
    s = run.ctx.stream
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        V.extrapolate(run.ctx, run.mesh, run.alpha, run.T, run.Tb, wl.T_sat, b.mixed_idx, b.counts, b.itf, gl, gv,
                      rep)
        V.mass_transfer(run.ctx, run.mesh, run.alpha, b.mixed_idx, b.counts, b.itf, None, wl.k_l, wl.k_v, wl.h_lv,
                        md, qd, gradT_l=gl, gradT_v=gv)
    for r in range(3):
        gl.zero_()
        md.fill_(7.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        dom = ~np.isnan(g["gl"][0])
        np.testing.assert_array_equal(gl.cpu().numpy()[:, dom], g["gl"][:, dom])
        np.testing.assert_array_equal(md[:g["step"]["n_mixed"]].cpu().numpy(), g["mdot"])
        assert int(rep[0].item()) == g["sweeps"] and int(rep[1].item()) == 0
    run.close()
