"""Compaction at sizes whose block totals (one per 256 cells) are scanned by
the separate one-block scan kernel (above 4096 blocks) rather than summed by
each scatter block: the mixed and band lists and their lengths against their
definitions (index work: bit-exact).  A 180^3 hexahedral mesh (22,782 blocks:
three scan tiles of 8192, the last one ragged) takes the cell pass; a
2 x 84^3 Voronoi box (1,185,408 cells, 4,631 blocks: one ragged tile) takes
the face pass; a 100^3 mesh (3,907 blocks) stays on the in-scatter prefix."""
import sys

import numpy as np
import pytest

import oracle
from synth import meshes

pytestmark = pytest.mark.gpu
EPS = 1e-8


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


def _field(n, seed):
    """Mostly pure cells, a tenth fractional, and values on and beside the
    mixed-cell thresholds."""
    rng = np.random.default_rng(seed)
    a = np.where(rng.uniform(size=n) < 0.75, 0.0, 1.0)
    frac = rng.uniform(size=n) < 0.1
    a[frac] = rng.uniform(size=int(frac.sum()))
    edge = rng.choice(n, 64, replace=False)
    a[edge] = rng.choice([EPS, 1 - EPS, np.nextafter(EPS, 1), np.nextafter(1 - EPS, 0)], 64)
    return a


@pytest.mark.parametrize("kind", ["hex 180^3", "voronoi 2x84^3", "hex 100^3"])
def test_compaction_with_many_blocks(V, kind):
    import torch
    if kind == "hex 180^3":
        m = meshes.hex_mesh(180)
    elif kind == "hex 100^3":
        m = meshes.hex_mesh(100)
    else:
        m = meshes.voronoi_box_mesh(84, seed=9)
    N = m.n_cells
    _say(f"compaction {kind}: {N} cells, {(N + 255) // 256} blocks")
    a = _field(N, N % 1000)
    ctx = V.Context(0, stream=torch.cuda.Stream())
    mesh = V.Mesh(ctx, m)
    alpha = torch.as_tensor(a, device="cuda")
    mixed = torch.full((N,), -7, dtype=torch.int32, device="cuda")
    band = torch.full((N,), -7, dtype=torch.int32, device="cuda")
    counts = torch.full((2,), -7, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    for rep in range(2):          # a second call on the same scratch: the same lists
        V.compact(ctx, mesh, alpha, mixed, band, counts, eps_mixed=EPS)
        torch.cuda.synchronize()
        nm, nb = (int(x) for x in counts.cpu())
        want_m = np.nonzero((a > EPS) & (a < 1 - EPS))[0]
        want_b = np.nonzero(oracle.band_mask(m, a, EPS))[0]
        assert (nm, nb) == (len(want_m), len(want_b)), (rep, nm, nb, len(want_m), len(want_b))
        np.testing.assert_array_equal(mixed[:nm].cpu().numpy(), want_m)
        np.testing.assert_array_equal(band[:nb].cpu().numpy(), want_b)
    _say(f"compaction {kind} ok: {nm} mixed, {nb} band")
    mesh.close()
    ctx.close()
