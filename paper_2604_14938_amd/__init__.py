"""vofpc: the interface hot path of sharp-interface phase-change VOF on
unstructured meshes (reconstruction, interface-modified gradient, mass
transfer) as a gfx950 HIP library with a thin Python binding.

``import paper_2604_14938_amd`` does not load the native library; use
``paper_2604_14938_amd.vofpc`` (which raises if ``libvofpc.so`` is missing).
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvofpc.so")
HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "vofpc.h")


def native():
    """Return the binding module (loads ``libvofpc.so``; raises if absent)."""
    from . import vofpc
    return vofpc
