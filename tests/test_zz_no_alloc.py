"""The allocation-free compaction (vofpc_compact_noalloc) against the
allocating one (vofpc_compact) through the C-ABI: identical mixed and band
lists and counts (index work: bit-exact), on two calls in a row, the second
on a smaller mesh (the shared scratch keeps the first call's contents), on
a mesh of faces beyond eight per cell (the face pass and its band marks) and
of hexahedra (the cell pass); and a mesh above the scratch's size is
refused before any work."""
import sys

import numpy as np
import pytest

from synth import meshes, workloads

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


def _lists(V, ctx, mesh, alpha, fn):
    import torch
    N = mesh.n_cells
    mixed = torch.full((N,), -7, dtype=torch.int32, device="cuda")
    band = torch.full((N,), -7, dtype=torch.int32, device="cuda")
    counts = torch.full((2,), -7, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    fn(ctx, mesh, alpha, mixed, band, counts)
    torch.cuda.synchronize()
    nm, nb = (int(x) for x in counts.cpu())
    return nm, nb, mixed[:nm].cpu().numpy(), band[:nb].cpu().numpy()


def test_noalloc_compaction_matches_the_allocating_one(V):
    import torch
    ctx = V.Context(0, stream=torch.cuda.Stream())
    cases = [("voronoi 2x24^3", workloads.voronoi_bubble(n=24, seed=3, r=0.3)),
             ("voronoi 2x14^3", workloads.voronoi_bubble(n=14, seed=4, r=0.25)),
             ("hex 40^3", workloads.random_bubbles(meshes.hex_mesh(40), seed=5, n_max=60, K=8, r_hi_h=5.0)),
             ("hex 20^3", workloads.random_bubbles(meshes.hex_mesh(20), seed=6, n_max=20, K=8, r_hi_h=4.0))]
    for name, wl in cases:
        _say(f"noalloc compaction: {name}, {wl.mesh.n_cells} cells")
        mesh = V.Mesh(ctx, wl.mesh)
        alpha = torch.as_tensor(wl.alpha, device="cuda")
        ref = _lists(V, ctx, mesh, alpha, V.compact)
        got = _lists(V, ctx, mesh, alpha, V.compact_noalloc)
        assert got[0] == ref[0] and got[1] == ref[1], (name, got[:2], ref[:2])
        np.testing.assert_array_equal(got[2], ref[2])
        np.testing.assert_array_equal(got[3], ref[3])
        # the lists are those of the definition (ascending; mixed; band)
        a = wl.alpha
        np.testing.assert_array_equal(got[2], np.nonzero((a > 1e-8) & (a < 1 - 1e-8))[0])
        assert ref[0] > 0 and ref[1] >= ref[0]
        # again on the same mesh: the same lists
        got2 = _lists(V, ctx, mesh, alpha, V.compact_noalloc)
        for x, y in zip(got2, got):
            np.testing.assert_array_equal(x, y)
        mesh.close()
    ctx.close()


def test_noalloc_compaction_refuses_meshes_beyond_its_scratch(V):
    import torch
    ctx = V.Context(0, stream=torch.cuda.Stream())
    m = meshes.hex_mesh(204)            # 8,489,664 cells > 8,388,608
    _say(f"noalloc compaction refusal: {m.n_cells} cells")
    mesh = V.Mesh(ctx, m)
    alpha = torch.zeros(m.n_cells, dtype=torch.float64, device="cuda")
    out = torch.zeros(m.n_cells, dtype=torch.int32, device="cuda")
    counts = torch.full((2,), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(V.VofpcError, match="8,388,608"):
        V.compact_noalloc(ctx, mesh, alpha, out, out, counts)
    torch.cuda.synchronize()
    assert counts.cpu().tolist() == [-7, -7]
    mesh.close()
    ctx.close()
