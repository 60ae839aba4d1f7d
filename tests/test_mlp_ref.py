"""Pins of the bracket-network reference and of the feature definitions."""
import numpy as np
import pytest
import torch

import oracle
from oracle import features as F
from oracle import mlp_ref as R
from synth import meshes


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=20000).astype(np.float32) * 10 ** rng.uniform(-8, 8, 20000),
                        # exact ties between two bfloat16 neighbours
                        (np.arange(1, 2000, dtype=np.uint32) << 16 | 0x8000).view(np.float32)])
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(R.bf16(x), ref)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = R.init_params(3)
    for k in p:
        p[k] = (p[k] + 0.1 * rng.normal(size=p[k].shape)).astype(np.float64)
    X = rng.normal(size=(37, 32))
    T = rng.normal(size=(37, 4))
    L0, g = R.backward(p, X, T, exact=True)
    eps = 1e-6
    for name in R.ORDER:
        flat = p[name].ravel()
        idx = rng.choice(flat.size, min(12, flat.size), replace=False)
        for i in idx:
            q = {k: v.copy() for k, v in p.items()}
            q[name].ravel()[i] += eps
            Lp = R.loss(R.forward(q, X, exact=True)["y"], T)
            q[name].ravel()[i] -= 2 * eps
            Lm = R.loss(R.forward(q, X, exact=True)["y"], T)
            fd = (Lp - Lm) / (2 * eps)
            assert g[name].ravel()[i] == pytest.approx(fd, rel=1e-7, abs=1e-10), (name, i)


def test_adam_matches_torch():
    rng = np.random.default_rng(2)
    p = R.init_params(5)
    tp = {k: torch.nn.Parameter(torch.tensor(v)) for k, v in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    state = {}
    for _ in range(5):
        g = {k: rng.normal(size=R.SHAPES[k]).astype(np.float32) for k in R.ORDER}
        R.adam_step(p, g, state, 3e-3)
        opt.zero_grad()
        for k in R.ORDER:
            tp[k].grad = torch.tensor(g[k])
        opt.step()
    for k in R.ORDER:
        np.testing.assert_allclose(p[k], tp[k].detach().numpy(), rtol=2e-6, atol=2e-8)


def test_flatten_roundtrip_and_sizes():
    p = R.init_params(7)
    v = R.flatten(p)
    assert v.size == R.N_PARAMS == 64 * 32 + 64 + 64 * 64 + 64 + 4 * 64 + 4
    q = R.unflatten(v)
    for k in R.ORDER:
        np.testing.assert_array_equal(p[k], q[k])


def test_features_closed_forms_on_a_hex_grid():
    """Shape tensor of a cube is I/3; the first alpha moment of a linear field
    on a uniform hex grid is g h / 3; the quantiles of a linear vertex field
    on a cube are those of its 8 corner values."""
    n = 6
    mesh = meshes.hex_mesh(n)
    geom = oracle.geometry(mesh)
    g = np.array([0.02, -0.05, 0.03])
    alpha = 0.5 + g @ (geom.xc - 0.5) * n
    phi = 0.5 + g @ (mesh.vert_xyz - 0.5) * n
    interior = [P for P in range(mesh.n_cells)
                if np.all((geom.xc[:, P] > 1.0 / n) & (geom.xc[:, P] < 1 - 1.0 / n))]
    f, rng = F.cell_features(mesh, geom, phi, alpha, interior)
    np.testing.assert_allclose(f[:, 19:22], 1.0 / 3.0, atol=1e-14)
    np.testing.assert_allclose(f[:, 22:25], 0.0, atol=1e-14)
    np.testing.assert_allclose(f[:, 10:13], np.tile(g * n * (1.0 / n) / 3.0, (len(interior), 1)), atol=1e-14)
    assert np.all(f[:, 25] == 6 / 32)
    # corner values of a linear field: u-quantiles of {0, a, b, c, a+b, ...}/W
    h = 1.0 / n
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)]) * h
    vals = np.sort(corners @ (g * n))
    vals = (vals - vals[0]) / (vals[-1] - vals[0])
    for qi in range(7):
        t = (qi + 1) / 8 * 7
        i = int(t)
        expect = vals[i] + (t - i) * (vals[i + 1] - vals[i])
        np.testing.assert_allclose(f[:, 1 + qi], expect, atol=1e-12)
    np.testing.assert_allclose(rng[:, 1], np.abs(g * n * h).sum(), rtol=1e-12)
