"""libdg.so loads on the CPU and exports every function include/dg.h
declares (no device call is made)."""
import ctypes
import os
import re

import paper_1710_03887_amd as dg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(dg_\w+)\s*\(", src, flags=re.M)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "dg_mesh_setup" in names and "dg_run" in names
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1710_03887_amd", "libdg.so"))
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    assert sorted(dg.EXPORTED) == declared_functions()
