"""The C ABI library: it loads, exports every entry point the header
declares, computes its recall-model table on the host, and rejects bad
arguments before touching the device."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "quake.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(quake_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2506_03437_amd import load_library
    lib = load_library()
    names = _declared()
    assert "quake_search" in names and "quake_build" in names
    for n in names:
        assert hasattr(lib, n), f"{n} missing from the library"


def test_binding_uses_the_c_names():
    import paper_2506_03437_amd as pkg
    for n in _declared():
        if n != "quake_last_error":
            assert hasattr(pkg, n), f"binding lacks {n}"


@pytest.mark.parametrize("d", [1, 2, 3, 16, 128, 768, 1024])
def test_cap_table_matches_oracle_table(d):
    from oracle import aps
    from paper_2506_03437_amd import quake_cap_table
    got = quake_cap_table(d)
    ref = aps.CapTable(d).values
    assert np.abs(got - ref).max() < 1e-12
    assert got[0] == pytest.approx(0.5, abs=1e-15) and got[-1] == 0.0
    assert (np.diff(got) <= 1e-15).all()


def test_host_side_argument_errors():
    from paper_2506_03437_amd import quake
    lib = quake.load_library()
    p = quake.BuildParams(0, 0, 1, 1, 4, 0, 0, None, None, 0, 0.0)
    h = ctypes.c_void_p()
    assert lib.quake_build(None, None, 10, 8, ctypes.byref(p), None, None, ctypes.byref(h)) == quake.E_INVALID
    assert b"x" in lib.quake_last_error()
    fake = ctypes.c_void_p(1234)  # pointer value only, never dereferenced by the check below
    assert lib.quake_build(fake, None, 10, 0, ctypes.byref(p), None, None, ctypes.byref(h)) == quake.E_INVALID
    p.metric = 7
    assert lib.quake_build(fake, None, 10, 8, ctypes.byref(p), None, None, ctypes.byref(h)) == quake.E_INVALID
    p.metric = 0
    p.nlist = 11
    assert lib.quake_build(fake, None, 10, 8, ctypes.byref(p), None, None, ctypes.byref(h)) == quake.E_INVALID
    sp = quake.SearchParams(10, 4, 0.0, 0, 0, 0, 0, 0, 0, 0, 0)
    assert lib.quake_search(None, None, 1, ctypes.byref(sp), None, None, None, None, None) == quake.E_STATE
    assert lib.quake_insert(None, None, None, 1, None) == quake.E_STATE
    assert lib.quake_delete(None, None, 1, None) == quake.E_STATE
    assert lib.quake_cap_table(0, (ctypes.c_double * 1024)()) == quake.E_INVALID
    srv = ctypes.c_void_p()
    spp = quake.ServerParams(8, 0, 0, sp)
    assert lib.quake_server_create(None, ctypes.byref(spp), ctypes.byref(srv)) == quake.E_STATE
    assert srv.value is None
    assert lib.quake_server_create(None, None, ctypes.byref(srv)) == quake.E_INVALID
    assert lib.quake_server_search(None, None, 1, None) == quake.E_INVALID
    assert lib.quake_server_wait(None, 1, 0.0, None, None, None, None) == quake.E_INVALID
    lib.quake_server_destroy(None)


def test_autotune_argument_errors():
    from paper_2506_03437_amd import quake
    lib = quake.load_library()
    sp = quake.SearchParams(10, 4, 0.0, 0, 0, 0, 0, 0, 0, 0, 0)
    assert lib.quake_autotune(None, None, 1, ctypes.byref(sp), 3, None, None, None) == quake.E_STATE


def test_maintenance_argument_errors():
    from paper_2506_03437_amd import quake
    lib = quake.load_library()
    p = quake.MaintainParams()
    assert lib.quake_maintain(None, ctypes.byref(p), None, None) == quake.E_STATE
    assert lib.quake_access_stats(None, 0, None, None, 0, None) == quake.E_STATE
    assert b"handle" in lib.quake_last_error()
