"""Interface coupling coefficients of the detached faces (Eq. interface_htc):
the HIP path against the oracle, face by face and cell by cell."""
import sys

import numpy as np
import pytest

import oracle
from synth import meshes, workloads

pytestmark = pytest.mark.gpu

K_L, K_V = 0.68, 0.025


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


def _gpu(R, wl, face_cap=None):
    import torch
    from paper_2604_14938_amd import vofpc as V
    run = R.PathRun(wl)
    run.step()
    g = run.results()
    NF = wl.mesh.n_faces
    cap = NF if face_cap is None else face_cap
    dev = run.dev
    out = dict(a_diag=torch.full((wl.mesh.n_cells,), float("nan"), dtype=torch.float64, device=dev),
               face_idx=torch.full((max(cap, 1),), -7, dtype=torch.int32, device=dev)[:cap],
               face_a=torch.zeros(2, cap, dtype=torch.float64, device=dev),
               face_d=torch.zeros(2, cap, dtype=torch.float64, device=dev),
               face_area=torch.zeros(cap, dtype=torch.float64, device=dev),
               n_face=torch.full((1,), -1, dtype=torch.int32, device=dev))
    b = run.buf
    torch.cuda.synchronize()
    V.robin(run.ctx, run.mesh, run.alpha, b.mixed_idx, b.band_idx, b.counts, b.itf, K_L, K_V, **_fwd(out))
    torch.cuda.synchronize()
    host = {k: v.cpu().numpy() for k, v in out.items()}
    host["n_face"] = int(host["n_face"][0])
    host["band_idx"] = g["band_idx"]
    host["a_diag"] = host["a_diag"][:g["n_band"]]
    return host, run, out


def _fwd(out):
    return dict(a_diag=out["a_diag"], face_idx=out["face_idx"], face_a=out["face_a"],
                face_d=out["face_d"], face_area=out["face_area"], n_face=out["n_face"])


def _oracle(wl):
    geom = oracle.geometry(wl.mesh)
    rec = oracle.reconstruct(wl.mesh, wl.alpha, geom)
    return oracle.robin(wl.mesh, geom, wl.alpha, rec["n"], rec["A"], K_L, K_V)


def _compare(wl, g, ref):
    """Face set exactly; A_int,f, d and a per side within the bound the
    interface parity gives (|dA| <= 1e-9 A + 1e-9 h^2, |dn| <= 1e-9 make
    |d A_int,f| <= 1e-8 h^2; a = k A_int,f / d then moves by k 1e-8 h^2 / d)."""
    h = wl.mesh.h
    nf = g["n_face"]
    faces = np.nonzero(ref["crossing"])[0]
    assert nf == len(faces), (nf, len(faces))
    order = np.argsort(g["face_idx"][:nf])
    fi = g["face_idx"][:nf][order]
    np.testing.assert_array_equal(fi, faces)
    area = g["face_area"][:nf][order]
    assert np.all(np.abs(area - ref["area_face"][faces]) <= 1e-8 * h * h)
    bound_face = []
    for side in (0, 1):
        d_o = ref["d_face"][side, faces]
        d_g = g["face_d"][side, :nf][order]
        assert np.all(np.abs(d_g - d_o) <= 1e-12 * d_o + 1e-14 * h)
        cells = wl.mesh.face_owner[faces] if side == 0 else wl.mesh.face_neigh[faces]
        k = np.where(wl.alpha[cells] >= 0.5, K_L, K_V)
        bound = k * 1e-8 * h * h / d_o + 1e-10 * ref["a_face"][side, faces]
        a_g = g["face_a"][side, :nf][order]
        err = np.abs(a_g - ref["a_face"][side, faces])
        assert np.all(err <= bound), (side, err.max())
        bound_face.append((cells, bound))
    # per band cell: the sum over its detached faces
    cb = np.zeros(wl.mesh.n_cells)
    for cells, bound in bound_face:
        np.add.at(cb, cells, bound)
    band = g["band_idx"]
    err = np.abs(g["a_diag"] - ref["a_cell"][band])
    assert np.all(err <= cb[band] + 1e-300), err.max()
    # band cells without a detached face get 0
    assert np.all(g["a_diag"][ref["a_cell"][band] == 0] == 0)


@pytest.mark.parametrize("name", ["vor12", "hex_bubbles", "vor_bubbles"])
def test_robin_matches_oracle(R, name):
    if name == "vor12":
        wl = workloads.voronoi_bubble(n=12, seed=7, r=0.3)
    elif name == "hex_bubbles":
        wl = workloads.random_bubbles(meshes.hex_mesh(24), seed=31, n_max=40, K=16, r_hi_h=5.0)
    else:
        wl = workloads.random_bubbles(meshes.voronoi_box_mesh(16, seed=32), seed=33, n_max=40, K=16, r_hi_h=3.0)
    _say(f"robin {name}: {wl.mesh.n_cells} cells, {wl.n_mixed} mixed")
    g, run, _ = _gpu(R, wl)
    ref = _oracle(wl)
    _compare(wl, g, ref)
    _say(f"robin {name}: {g['n_face']} detached faces ok")
    run.close()


def test_robin_capacity_and_empty(R):
    """A face capacity below the count: n_face still reports every detached
    face and the records written are valid ones; a field with no interface
    detaches nothing."""
    wl = workloads.voronoi_bubble(n=10, seed=4, r=0.3)
    ref = _oracle(wl)
    total = int(ref["crossing"].sum())
    _say(f"robin capacity {total // 3} of {total}")
    g, run, _ = _gpu(R, wl, face_cap=total // 3)
    assert g["n_face"] == total
    fi = g["face_idx"]
    assert len(np.unique(fi)) == len(fi) and ref["crossing"][fi].all()
    run.close()
    wl.alpha[:] = 1.0
    _say("robin without interface")
    g, run, _ = _gpu(R, wl)
    assert g["n_face"] == 0 and len(g["a_diag"]) == 0
    run.close()


def test_robin_replays_in_a_graph(R):
    import torch
    from paper_2604_14938_amd import vofpc as V
    wl = workloads.voronoi_bubble(n=10, seed=6, r=0.28)
    _say("robin graph replay")
    g, run, out = _gpu(R, wl)
    b = run.buf
    s = run.ctx.stream
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        V.robin(run.ctx, run.mesh, run.alpha, b.mixed_idx, b.band_idx, b.counts, b.itf, K_L, K_V, **_fwd(out))
    nf = g["n_face"]
    order = np.argsort(g["face_idx"][:nf])
    for r in range(3):
        out["a_diag"].fill_(-1.0)
        out["face_a"].zero_()
        out["n_face"].fill_(-5)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert int(out["n_face"].item()) == nf
        fi = out["face_idx"][:nf].cpu().numpy()
        o2 = np.argsort(fi)
        np.testing.assert_array_equal(fi[o2], g["face_idx"][:nf][order])
        np.testing.assert_array_equal(out["face_a"][:, :nf].cpu().numpy()[:, o2], g["face_a"][:, :nf][:, order])
        np.testing.assert_array_equal(out["a_diag"][:len(g["a_diag"])].cpu().numpy(), g["a_diag"])
    run.close()
