"""The bench's command line contract on the host: more than one GPU is
refused with a message (this build measures one GPU), and its helper
figures are consistent."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_algorithmic_flops_by_cell_kind():
    sys.path.insert(0, ROOT)
    import bench
    from synth import meshes
    hexm = meshes.hex_mesh(3)
    vor = meshes.voronoi_box_mesh(4, seed=1)
    assert bench.recon_flops(hexm, np.arange(5)) == 5 * bench.FLOPS_HEX_CELL
    assert bench.recon_flops(vor, np.arange(3)) == 3 * bench.FLOPS_VORONOI_CELL
    assert abs(bench.FP64_PEAK_TFLOPS - 78.6432) < 1e-9


def test_kernel_classes_and_footprint():
    sys.path.insert(0, ROOT)
    import bench
    from synth import meshes, workloads
    hexm = meshes.hex_mesh(4)
    cells = np.arange(hexm.n_cells)
    assert np.all(bench.cell_classes(hexm, cells) == 0)
    row, verts, nf, nl = bench.cell_incidence(hexm, cells[:3])
    assert np.all(np.bincount(row) == 8) and np.all(nf == 6) and np.all(nl == 24)
    vor = meshes.voronoi_box_mesh(6, seed=1)
    c = bench.cell_classes(vor, np.arange(vor.n_cells))
    row, _, nf, nl = bench.cell_incidence(vor, np.arange(vor.n_cells))
    nv = np.bincount(row)
    # every cell in the first class whose caps hold it
    for k in range(len(bench.CLASS_CAPS)):
        v, f, l, e = bench.CLASS_CAPS[k]
        fits = (nv <= v) & (nf <= f) & (nl <= l) & (nl // 2 <= e)
        assert np.all(c[fits] <= k) and np.all(c[~fits] > k)
    # the footprint grows with the cells and counts each shared vertex once
    b1 = bench.recon_bytes(hexm, cells[:1])
    b2 = bench.recon_bytes(hexm, cells[:2])
    assert 0 < b1 < b2 < 2 * b1
    assert bench.recon_bytes(hexm, cells[:2], learned=True) > b2


def test_hexahedral_class_zero_rule_on_the_host():
    """The bench assigns kernel classes as the library does: a union of a
    hexahedral mesh and a small Voronoi box moves the Voronoi cells of
    class 0 to class 1 (at most 1 % of class 0); a Voronoi box alone keeps
    them."""
    import bench
    from synth import meshes
    hexm = meshes.hex_mesh(12)
    vor = meshes.voronoi_box_mesh(6, seed=3)
    both = meshes.concat([hexm, vor])
    cv = bench.cell_classes(vor, np.arange(vor.n_cells))
    assert np.count_nonzero(cv == 0) > 0 and not bench.mesh_hex0(vor)
    assert bench.mesh_hex0(both)
    cb = bench.cell_classes(both, np.arange(both.n_cells))
    assert np.all(cb[:hexm.n_cells] == 0)
    assert np.all(cb[hexm.n_cells:] >= 1)
    assert np.array_equal(cb[hexm.n_cells:][cv >= 1], cv[cv >= 1])


def test_extrapolation_sweep_bytes_count():
    """The sweep's algorithmic bytes: 92 B per domain cell and 12 B per
    upwind slot, one upwind slot per face between two domain cells."""
    import bench
    from synth import meshes
    m = meshes.hex_mesh(4)
    dom = np.zeros(m.n_cells, bool)
    dom[:16] = True          # the first 16 cells
    inner = m.face_neigh >= 0
    faces = int(np.count_nonzero(dom[m.face_owner[inner]] & dom[m.face_neigh[inner]]))
    r = bench.extrap_sweep_bytes(m, dom, 1.0)
    assert r["domain_cells"] == 16 and r["upwind_slots_est"] == faces
    assert r["algorithmic_bytes"] == 16 * 92 + 12 * faces
    assert abs(r["GBps"] - r["algorithmic_bytes"] / 1e-6 / 1e9) < 1e-9
