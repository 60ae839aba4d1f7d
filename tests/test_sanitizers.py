"""The CPU C code under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle (oracle/vof_oracle.c) and the synthetic-input helpers
(synth/_subsample.c, synth/_voronoi.c) are rebuilt with
-fsanitize=address,undefined (UB reports abort), and the CPU pin and
generator tests run against those builds in a child process with the
sanitizer runtime preloaded (Python itself is not instrumented, so leak
checking is off).  Any invalid access or undefined operation fails the run.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
TESTS = ["tests/test_oracle_pins.py", "tests/test_oracle_geometry_pins.py", "tests/test_oracle_csf.py",
         "tests/test_synth.py"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_and_generators_are_clean_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    sys.path.insert(0, ROOT)
    import oracle
    builds = {
        "ORACLE_SO": (os.path.join(ROOT, "oracle", "vof_oracle.c"),
                      [f for f in oracle.CFLAGS if not f.startswith("-O")]),
        "SYNTH_SUBSAMPLE_SO": (os.path.join(ROOT, "synth", "_subsample.c"), ["-fopenmp", "-shared", "-fPIC"]),
        "SYNTH_VORONOI_SO": (os.path.join(ROOT, "synth", "_voronoi.c"), ["-fopenmp", "-shared", "-fPIC"]),
    }
    env = dict(os.environ)
    for var, (src, flags) in builds.items():
        out = str(tmp_path / (os.path.basename(src)[:-2] + "_san.so"))
        subprocess.check_call(["gcc", *SAN, *flags, "-o", out, src, "-lm"])
        env[var] = out
    env["LD_PRELOAD"] = f"{asan}:{ubsan}"
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "4"
    # the instrumented builds are the ones loaded, and they catch a read
    # past the end of the mesh arrays (a cell index one past the last)
    probe = ("import sys, numpy as np; sys.path.insert(0, '.'); import oracle; from synth import fields, meshes; "
             "print(oracle._lib()._name, fields._lib()._name, meshes._vlib()._name, flush=True); "
             "m = meshes.hex_mesh(8); g = oracle.geometry(m); phi = np.zeros(m.n_verts); "
             "oracle.cut_cell(m, m.n_cells, g.xc, phi, 0.5)")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.stdout.split() == [env["ORACLE_SO"], env["SYNTH_SUBSAMPLE_SO"], env["SYNTH_VORONOI_SO"]], r.stdout
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr, r.stderr[-2000:]
    r = subprocess.run([sys.executable, "-m", "pytest", *TESTS, "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "runtime error" not in r.stdout + r.stderr, tail
    assert "AddressSanitizer" not in r.stdout + r.stderr, tail
