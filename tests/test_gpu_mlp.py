"""GPU bracket network and features against the reference (oracle/mlp_ref.py,
oracle/features.py), and the learned step against the plain one."""
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import features as OF
from oracle import mlp_ref as R
from synth import workloads
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


def _params(seed):
    rng = np.random.default_rng(seed)
    p = R.init_params(seed)
    for k in p:
        p[k] = (p[k] + 0.05 * rng.normal(size=p[k].shape)).astype(np.float32)
    return p


def _cos(a, b):
    return float(np.dot(a.ravel(), b.ravel()) / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))


def test_forward_matches_reference(V):
    import torch
    _say("mlp forward")
    ctx = V.Context(0, stream=torch.cuda.Stream())
    mlp = V.Mlp(ctx, 4096)
    p = _params(1)
    mlp.set_params(R.flatten(p))
    rng = np.random.default_rng(2)
    X = rng.normal(size=(1003, 32)).astype(np.float32)   # ragged: not a multiple of 16
    Xd = torch.tensor(X, device="cuda")
    Yd = torch.zeros(1003, 4, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()   # inputs were written on torch's stream
    mlp.forward(Xd, Yd)
    torch.cuda.synchronize()
    y = Yd.cpu().numpy()
    ref = R.forward(p, X)["y"]
    err = np.abs(y - ref)
    assert err.max() < 3e-2, err.max()
    assert np.mean(err) < 2e-3
    for c in range(4):
        assert _cos(y[:, c], ref[:, c]) > 0.9999
    mlp.close()


def test_gradient_matches_reference(V):
    import torch
    _say("mlp gradient")
    ctx = V.Context(0, stream=torch.cuda.Stream())
    mlp = V.Mlp(ctx, 8192)
    p = _params(3)
    mlp.set_params(R.flatten(p))
    rng = np.random.default_rng(4)
    X = rng.normal(size=(2000, 32)).astype(np.float32)
    T = rng.normal(size=(2000, 4)).astype(np.float32)
    g = torch.zeros(mlp.n_params, dtype=torch.float32, device="cuda")
    L = torch.zeros(1, dtype=torch.float32, device="cuda")
    Xd, Td = torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda")
    torch.cuda.synchronize()
    mlp.gradient(Xd, Td, g, L)
    torch.cuda.synchronize()
    Lr, gr = R.backward(p, X, T)
    gg = R.unflatten(g.cpu().numpy())
    assert float(L.item()) == pytest.approx(Lr, rel=1e-3)
    for k in R.ORDER:
        a, b = gg[k].astype(np.float64), gr[k]
        assert _cos(a, b) >= 0.9999, k
        assert np.abs(a - b).max() <= 1e-2 * np.abs(b).max(), k
    mlp.close()


def test_adam_first_step_and_loss_decrease(V):
    import torch
    _say("mlp adam")
    ctx = V.Context(0, stream=torch.cuda.Stream())
    mlp = V.Mlp(ctx, 4096)
    p = _params(5)
    mlp.set_params(R.flatten(p))
    rng = np.random.default_rng(6)
    X = rng.normal(size=(4096, 32)).astype(np.float32)
    W = rng.normal(size=(32, 4)).astype(np.float32) * 0.2
    T = np.tanh(X @ W).astype(np.float32)
    Xd, Td = torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda")
    L = torch.zeros(1, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    lr = 1e-3
    mlp.train_step(Xd, Td, lr)
    after = R.unflatten(mlp.get_params())
    _, gr = R.backward(p, X, T)
    state = {}
    ref = {k: v.copy() for k, v in p.items()}
    R.adam_step(ref, gr, state, lr)
    for k in R.ORDER:
        big = np.abs(gr[k]) > 1e-3 * np.abs(gr[k]).max()
        np.testing.assert_allclose(after[k][big], ref[k][big], atol=1e-6, err_msg=k)
    losses = []
    for it in range(300):
        mlp.train_step(Xd, Td, 3e-3, L)
        if it % 50 == 0:
            torch.cuda.synchronize()
            losses.append(float(L.item()))
    assert losses[-1] < 0.2 * losses[0], losses
    mlp.close()


def test_features_match_reference(V):
    import torch
    _say("features vor12")
    wl = workloads.voronoi_bubble(n=12, seed=7, r=0.3)
    from paper_2604_14938_amd import runner
    run = runner.PathRun(wl)
    b = run.buf
    N = wl.mesh.n_cells
    V.compact(run.ctx, run.mesh, run.alpha, b.mixed_idx, b.band_idx, b.counts)
    feat = torch.zeros(N, 32, dtype=torch.float32, device="cuda")
    pr = torch.zeros(N, 2, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    V.features(run.ctx, run.mesh, run.alpha, b.mixed_idx, b.counts, feat, pr)
    torch.cuda.synchronize()
    M = int(b.counts[0].item())
    cells = b.mixed_idx[:M].cpu().numpy()
    geom = oracle.geometry(wl.mesh)
    phi = oracle.vertex_field(wl.mesh, geom.xc, wl.alpha)
    ref, rr = OF.cell_features(wl.mesh, geom, phi, wl.alpha, cells)
    np.testing.assert_allclose(feat[:M].cpu().numpy(), ref, rtol=2e-6, atol=2e-6)
    np.testing.assert_allclose(pr[:M].cpu().numpy(), rr, rtol=1e-12, atol=1e-14)
    run.close()


def _weights():
    from paper_2604_14938_amd import train
    if not os.path.exists(train.DEFAULT_WEIGHTS):
        return None
    return train.load()


@pytest.mark.parametrize("which", ["trained", "corrupted"])
def test_learned_step_gives_the_plain_results(V, which):
    """The network only narrows the bracket: with trained weights and with
    deliberately wrong ones (every bracket fails its check) the results stay
    within the parity tolerance of the oracle, the statuses differ only by
    the fallback flag."""
    import torch
    from paper_2604_14938_amd import runner
    w = _weights()
    if w is None:
        pytest.skip("no trained weights")
    params, dscale, _ = w
    wl = workloads.voronoi_bubble(n=12, seed=7, r=0.3)
    _say(f"learned step ({which}) vor12")
    ctx = V.Context(0, stream=torch.cuda.Stream())
    mlp = V.Mlp(ctx)
    if which == "corrupted":
        bad = params.copy()
        bad[-4] = 50.0          # output bias of u: every bracket far above [0, 1]
        mlp.set_params(bad)
    else:
        mlp.set_params(params)
    run = runner.PathRun(wl, ctx=ctx, mlp=mlp, delta_scale=dscale)
    run.step()
    g = run.results()
    rec = oracle.reconstruct(wl.mesh, wl.alpha)
    st = g["status"].copy()
    fb = st == V.CELL_LEARNED_FALLBACK
    g2 = dict(g)
    g2["status"] = np.where(fb, V.CELL_OK, st)
    parity.check_interface(wl, g2, rec)
    if which == "corrupted":
        assert fb.mean() > 0.9
    else:
        assert fb.mean() < 0.2
    run.close()
    mlp.close()


def test_fused_network_bracket_matches_the_separate_kernels(V):
    """The reconstruction kernel's in-wave features and forward pass give the
    brackets of the features kernel followed by the bracket kernel (up to the
    summation order of the feature sums)."""
    import torch
    from paper_2604_14938_amd import runner
    w = _weights()
    if w is None:
        pytest.skip("no trained weights")
    params, dscale, _ = w
    wl = workloads.voronoi_bubble(n=12, seed=7, r=0.3)
    _say("fused vs separate network bracket vor12")
    ctx = V.Context(0, stream=torch.cuda.Stream())
    mlp = V.Mlp(ctx)
    mlp.set_params(params)
    run = runner.PathRun(wl, ctx=ctx, mlp=mlp, delta_scale=dscale)
    run.step()
    b = run.buf
    N = wl.mesh.n_cells
    feat = torch.zeros(N, 32, dtype=torch.float32, device="cuda")
    pr = torch.zeros(N, 2, dtype=torch.float64, device="cuda")
    hl = torch.zeros(N, dtype=torch.float64, device="cuda")
    hh = torch.zeros(N, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    V.features(ctx, run.mesh, run.alpha, b.mixed_idx, b.counts, feat, pr)
    mlp.bracket(feat, pr, b.counts, N, dscale, hl, hh)
    torch.cuda.synchronize()
    M = int(b.counts[0].item())
    W = pr[:M, 1].cpu().numpy()
    ok = W > 1e-12
    d_lo = np.abs(b.hint_lo[:M].cpu().numpy() - hl[:M].cpu().numpy())[ok] / W[ok]
    d_hi = np.abs(b.hint_hi[:M].cpu().numpy() - hh[:M].cpu().numpy())[ok] / W[ok]
    assert ok.sum() > 0.9 * M
    assert np.median(d_lo) <= 1e-6 and np.median(d_hi) <= 1e-6
    assert np.percentile(d_lo, 99) <= 1e-3 and np.percentile(d_hi, 99) <= 1e-3
    run.close()
    mlp.close()


def test_trained_network_saves_evaluations(V):
    """What the trained network gains: on a Voronoi bubble (different seed
    and size from the training meshes) the learned bracket reaches the same
    results with fewer volume evaluations per cell than the plain search."""
    import torch
    from paper_2604_14938_amd import runner
    w = _weights()
    if w is None:
        pytest.skip("no trained weights")
    params, dscale, _ = w
    wl = workloads.voronoi_bubble(n=24, seed=13, r=0.27)
    _say(f"evaluations, plain vs learned: {wl.mesh.n_cells} cells, {wl.n_mixed} mixed")
    ctx = V.Context(0, stream=torch.cuda.Stream())
    plain = runner.PathRun(wl, ctx=ctx)
    plain.step()
    gp = plain.results()
    mlp = V.Mlp(ctx)
    mlp.set_params(params)
    learned = runner.PathRun(wl, ctx=ctx, mlp=mlp, delta_scale=dscale)
    learned.step()
    gl = learned.results()
    np.testing.assert_array_equal(gl["mixed_idx"], gp["mixed_idx"])
    assert np.abs(gl["alpha_got"] - gp["alpha_got"]).max() <= 1e-10
    ep, el = gp["iters"].mean(), gl["iters"].mean()
    fb = (gl["status"] == V.CELL_LEARNED_FALLBACK).mean()
    _say(f"mean evaluations per cell: plain {ep:.2f}, learned {el:.2f}; fallback rate {fb:.3f}")
    assert el < 0.95 * ep
    plain.close()
    learned.close()
    mlp.close()
