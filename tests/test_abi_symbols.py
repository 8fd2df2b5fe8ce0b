"""The C-ABI library loads on the host and exports every entry point that
include/emstep.h declares (no compute call: no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2503_17608_amd", "libemstep.so")


def declared():
    src = open(os.path.join(ROOT, "include", "emstep.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ems_[a-z0-9_]+)\s*\(", src)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (the library binds to torch's HIP runtime)
    lib = ctypes.CDLL(LIB)
    names = declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_declared_symbols_and_version():
    from paper_2503_17608_amd import emstep
    assert set(declared()) == set(emstep.exported_symbols())
    assert emstep._lib.ems_abi_version() == emstep.ABI_VERSION


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_option_validation_on_host():
    # argument validation runs before any device call
    from paper_2503_17608_amd import emstep
    o = emstep.Options()
    o.abi_version = emstep.ABI_VERSION
    o.n_slots = 0
    n = ctypes.c_uint64(0)
    assert emstep._lib.ems_query_workspace(ctypes.byref(o), ctypes.byref(n)) == emstep.ERR_INVALID_ARG
    o.n_slots = 4096
    o.n_initializers = 1 << 16
    o.n_primaries = 1 << 16
    o.max_events = 10
    o.max_slabs = 40
    o.max_materials = 2
    assert emstep._lib.ems_query_workspace(ctypes.byref(o), ctypes.byref(n)) == emstep.OK
    assert n.value > 4096 * 100
    o.block_size = 100
    assert emstep._lib.ems_query_workspace(ctypes.byref(o), ctypes.byref(n)) == emstep.ERR_INVALID_ARG
    o.block_size = 0
    o.abi_version = emstep.ABI_VERSION - 1
    assert emstep._lib.ems_query_workspace(ctypes.byref(o), ctypes.byref(n)) == emstep.ERR_INVALID_ARG
