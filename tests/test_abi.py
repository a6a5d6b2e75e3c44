"""CPU-side checks of the C ABI: the library loads and exports every function
that include/mg.h declares (no compute calls: no GPU here)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mg.h")
LIB = os.path.join(ROOT, "paper_1508_03954_amd", "libmg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("mg_setup", "mg_apply", "mg_cycle", "mg_solve", "mg_flush", "mg_destroy"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmg.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmg.so not built")
def test_binding_lists_match_header():
    from paper_1508_03954_amd import mg
    assert sorted(mg.EXPORTED) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmg.so not built")
def test_params_layout_and_error_paths_without_gpu():
    """mg_params_default and argument validation run on the host only."""
    from paper_1508_03954_amd import mg
    lib = mg.load_library()
    p = mg.Params()
    lib.mg_params_default(ctypes.byref(p))
    assert p.dim == 3 and p.level_min == 1 and abs(p.omega.re - 0.6) < 1e-15
    p.dim = 4
    ctx = ctypes.c_void_p()
    assert lib.mg_setup(ctypes.byref(p), None, ctypes.byref(ctx)) == mg.MG_EINVAL
    assert b"dim" in lib.mg_last_error()
    assert lib.mg_setup(None, None, ctypes.byref(ctx)) == mg.MG_EINVAL
