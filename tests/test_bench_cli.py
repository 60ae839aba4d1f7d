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
