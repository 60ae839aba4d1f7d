"""The static-sphere anisotropy study run through the library on the GPU:
its metrics equal those computed from the oracle's gradient (the gradients
agree to the parity bar, so the binned statistics agree to about that)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2604_14938_amd import anisotropy as an
from synth import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_ok():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("kind,n", [("hex", 32), ("voronoi", 16)])
def test_study_metrics_match_oracle(torch_ok, kind, n):
    wl = workloads.static_sphere(kind, n)
    print(f"[gpu-case] anisotropy study {wl.name}", flush=True)
    sys.stdout.flush()
    r = an.study(wl, n_bins=24, steps=3)
    geom = oracle.geometry(wl.mesh)
    cells = an.interface_cells(wl.alpha, wl.mesh.face_owner, wl.mesh.face_neigh)
    exact = an.erf_profile_gradient(geom.xc, wl.meta["centre"], wl.meta["r"], wl.meta["width"], wl.meta["dT"])
    kw = {"modified": {}, "standard": dict(modified=False), "inv_dist": dict(weight=1),
          "inv_dist2": dict(weight=2), "vertex": dict(extended=True)}
    for name, args in kw.items():
        g, _ = oracle.grad(wl.mesh, geom, wl.T, wl.T_bface, wl.T_sat, wl.alpha, **args)
        P = an.polar(geom.xc, np.linalg.norm(g, axis=0) / exact, cells, wl.meta["centre"], wl.mesh.h, n_bins=24)
        got = r["grad"][name]
        assert got["n_slab"] == P["n_cells"]
        assert got["mean_ratio"] == pytest.approx(P["mean"], rel=1e-8)
        assert got["min_max"] == pytest.approx(P["min_max"], rel=1e-8)
        np.testing.assert_allclose(got["modes_pct"], P["modes_pct"], rtol=1e-6, atol=1e-6)
    assert r["mdot"]["sweeps"] >= 1 and r["mdot"]["two_sided"] is not None
    assert r["step_us"] > 0 and r["mixed_cells_per_s"] > 0
