"""Parity at full size and on the pipe-film mesh family.

* The 128^3 hexahedral part of the batched configuration (2,097,152 cells,
  random bubbles r ~ U[2h, 12h]) joined on the device with a Voronoi mesh, so
  the reconstruction runs bucketed by kernel class as in the batched bench.
  The oracle reconstructs a seeded sample of the mixed cells one by one;
  every cell is checked against properties that hold at any size.
* A Voronoi pipe with a wavy liquid film on its wall (the learned-bracket
  configuration's mesh family, at a size the oracle finishes in seconds):
  the whole step, both forms, and the follow-on rows against the oracle."""
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


def test_full_size_hex_part_of_the_batch_sampled(R):
    _say("full-size batch part: building 128^3 hexahedra with random bubbles")
    w_hex = workloads.random_bubbles(meshes.hex_mesh(128), seed=3, n_max=1000, K=8, r_hi_h=12.0)
    w_vor = workloads.random_bubbles(meshes.voronoi_box_mesh(24, seed=5), seed=20, n_max=60, K=8, r_hi_h=4.0)
    wl = workloads.concat_workloads([w_hex, w_vor])
    _say(f"full-size batch part: {wl.mesh.n_cells} cells, {wl.n_mixed} mixed; stepping on the GPU")
    run = R.PathRun(wl, parts=[w_hex.mesh, w_vor.mesh])
    cls = run.mesh.classes()
    assert cls["bucketed"], cls
    run.step()
    g = run.results()
    run.close()
    parity.check_lists(wl, g)
    M = g["n_mixed"]
    idx = g["mixed_idx"]
    # properties of every mixed cell
    ok = g["status"] == oracle.OK
    assert ok.mean() > 0.999, np.bincount(g["status"])
    tol = 1e-13 * np.minimum(wl.alpha[idx], 1 - wl.alpha[idx])
    assert np.all(np.abs(g["alpha_got"][ok] - wl.alpha[idx][ok]) <= np.maximum(tol[ok], 1e-15))
    assert np.all(g["A"][ok] > 0)
    np.testing.assert_allclose(np.linalg.norm(g["n"][:, ok], axis=0), 1.0, atol=1e-12)
    # a seeded sample, plus the cells that took the most evaluations
    rng = np.random.default_rng(0)
    pick = np.union1d(rng.choice(M, 400, replace=False), np.argsort(g["iters"])[-50:])
    cells = idx[pick]
    _say(f"full-size batch part: oracle on {len(pick)} sampled cells")
    geom = oracle.geometry(wl.mesh)
    rec = oracle.reconstruct(wl.mesh, wl.alpha, geom, cells=cells)
    sub = {k: (g[k][:, pick] if k == "n" else g[k][pick]) for k in ("s", "n", "A", "d", "alpha_got", "status")}
    sub["mixed_idx"] = cells
    parity.check_interface(wl, sub, rec)
    grad, gst = oracle.grad(wl.mesh, geom, wl.T, wl.T_bface, wl.T_sat, wl.alpha)
    band = g["band_idx"]
    bs = band[rng.choice(len(band), min(5000, len(band)), replace=False)]
    parity.check_grad(wl, g["gradT"], grad, bs)
    np.testing.assert_array_equal(g["grad_status"][bs], gst[bs])
    md, _ = oracle.mass_transfer(geom, wl.alpha, rec["n"], rec["A"], grad, wl.k_l, wl.k_v, wl.h_lv)
    parity.check_mdot(g["mdot"][pick], md[cells])


def test_pipe_film_step_and_follow_on_rows(R):
    import torch
    from paper_2604_14938_amd import train
    from paper_2604_14938_amd import vofpc as V
    wl = workloads.pipe_film(n_radial=14, seed=4)
    _say(f"pipe film: {wl.mesh.n_cells} cells, {wl.n_mixed} mixed")
    ref = parity.oracle_path(wl)
    params, dscale, _ = train.load()
    for form in ("plain", "learned"):
        mlp = None
        if form == "learned":
            mlp = V.Mlp(V.Context(0, stream=torch.cuda.Stream()))
            mlp.set_params(params)
        run = R.PathRun(wl, mlp=mlp, delta_scale=dscale if mlp else 0.0)
        run.step()
        g = run.results()
        parity.check_lists(wl, g)
        st = g["status"].copy()
        st[st == oracle.LEARNED_FALLBACK] = oracle.OK
        g2 = dict(g, status=st)
        parity.check_interface(wl, g2, ref["rec"])
        parity.check_grad(wl, g["gradT"], ref["grad"], g["band_idx"])
        parity.check_mdot(g["mdot"], ref["mdot"][g["mixed_idx"]])
        if form == "plain":
            # extrapolated phase gradients, coupling coefficients and curvature
            b = run.buf
            N, NF = wl.mesh.n_cells, wl.mesh.n_faces
            f64 = dict(dtype=torch.float64, device=run.dev)
            gl, gv = torch.full((3, N), np.nan, **f64), torch.full((3, N), np.nan, **f64)
            rep = torch.zeros(2, dtype=torch.int32, device=run.dev)
            fi = torch.zeros(NF, dtype=torch.int32, device=run.dev)
            fa = torch.zeros(2, NF, **f64)
            nfo = torch.zeros(1, dtype=torch.int32, device=run.dev)
            ah, k = torch.zeros(N, **f64), torch.zeros(N, **f64)
            cn, F = torch.zeros(3, N, **f64), torch.zeros(3, N, **f64)
            torch.cuda.synchronize()
            V.extrapolate(run.ctx, run.mesh, run.alpha, run.T, run.Tb, wl.T_sat, b.mixed_idx, b.counts, b.itf, gl,
                          gv, rep)
            V.robin(run.ctx, run.mesh, run.alpha, b.mixed_idx, b.band_idx, b.counts, b.itf, wl.k_l, wl.k_v,
                    face_idx=fi, face_a=fa, n_face=nfo)
            V.curvature(run.ctx, run.mesh, run.alpha, ah, cn, k, force=F)
            torch.cuda.synchronize()
            geom = ref["geom"]
            rec = ref["rec"]
            ogl, ogv, sweeps, dom = oracle.extrapolate(wl.mesh, geom, wl.alpha, ref["grad"], rec["n"], rec["A"])
            assert int(rep[0].item()) == sweeps
            scale = np.abs(ref["grad"][:, dom]).max()
            for a, o in ((gl, ogl), (gv, ogv)):
                assert np.abs(a.cpu().numpy()[:, dom] - o[:, dom]).max() <= 1e-9 * scale
            rb = oracle.robin(wl.mesh, geom, wl.alpha, rec["n"], rec["A"], wl.k_l, wl.k_v)
            nf = int(nfo.item())
            assert nf == rb["crossing"].sum()
            order = np.argsort(fi[:nf].cpu().numpy())
            np.testing.assert_array_equal(fi[:nf].cpu().numpy()[order], np.nonzero(rb["crossing"])[0])
            np.testing.assert_allclose(fa[:, :nf].cpu().numpy()[:, order], rb["a_face"][:, rb["crossing"]], rtol=0,
                                       atol=1e-8 * np.abs(rb["a_face"]).max())
            cs = oracle.csf(wl.mesh, geom, wl.alpha, n_smooth=2)
            np.testing.assert_allclose(k.cpu().numpy(), cs["kappa"], rtol=0, atol=1e-9 * np.abs(cs["kappa"]).max())
            np.testing.assert_allclose(F.cpu().numpy(), cs["F"], rtol=0, atol=1e-9 * np.abs(cs["F"]).max())
        run.close()
        if mlp is not None:
            mlp.close()
    _say("pipe film ok")
