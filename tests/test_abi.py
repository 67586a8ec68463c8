"""The C-ABI library loads and exports every function include/lst.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lst.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lst_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_three_calls():
    names = declared()
    for n in ("lst_load_geometry", "lst_build_event", "lst_get_track_candidates"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2207_08207_amd as lst
    if not os.path.exists(lst.LIB_PATH):
        pytest.fail("liblst.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(lst.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(lst.EXPORTED) == declared()


def test_errors_without_device_work():
    """Argument errors are reported before any device work (no GPU touched)."""
    import paper_2207_08207_amd as lst
    lib = lst.load_library()
    assert lib.lst_default_capacity(-1, 0, None) == lst.LST_E_INVALID
    assert "bad argument" in lst.lst_last_error()
    c = lst.lst_default_capacity(534129, 8889)
    assert c.md == 534129 and c.ls == 4 * 534129 and c.pt5 == 16 * 8889
    assert lib.lst_load_geometry(None, None) == lst.LST_E_INVALID
    assert lib.lst_release_event(None) == lst.LST_OK
