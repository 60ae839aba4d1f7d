"""The C-ABI library loads and exports every entry point the header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vofpc.h")
LIB = os.path.join(ROOT, "paper_2604_14938_amd", "libvofpc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(vofpc_[A-Za-z_0-9]+)\s*\(", text)
    return sorted(set(n for n in names if not n.endswith("_s")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("vofpc_mesh_upload", "vofpc_compact", "vofpc_reconstruct", "vofpc_grad_T",
                     "vofpc_mass_transfer", "vofpc_step", "vofpc_graph_create"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (vofpc_\w+)", out))
    assert set(declared_functions()) <= exported


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_version_and_error_string_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.vofpc_version.restype = ctypes.c_int
    assert lib.vofpc_version() >= 10000
    lib.vofpc_last_error.restype = ctypes.c_char_p
    assert lib.vofpc_last_error() == b""


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_null_arguments_are_rejected_without_touching_the_device():
    lib = ctypes.CDLL(LIB)
    lib.vofpc_last_error.restype = ctypes.c_char_p
    assert lib.vofpc_recon_opts_default(None) == -1
    assert b"null" in lib.vofpc_last_error()
    assert lib.vofpc_ctx_create(0, None, None) == -1
    assert lib.vofpc_mesh_free(None) == 0
    assert lib.vofpc_graph_destroy(None) == 0
    for name in ("vofpc_ctx_overlap_classes", "vofpc_ctx_time_classes"):
        assert getattr(lib, name)(None, 1) == -1, name
        assert b"null context" in lib.vofpc_last_error(), name


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2604_14938_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "vof_oracle" not in text, f
