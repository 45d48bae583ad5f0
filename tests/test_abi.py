"""The C-ABI library loads and exports every entry point include/bt.h declares
(CPU only: no call reaches the device)."""
import os
import re

import paper_2512_23314_amd as bt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^BT_API\s+[\w\s\*]+?\b(bt_\w+)\s*\(", src, flags=re.M)
    return names


def test_every_declared_symbol_is_exported():
    names = declared()
    assert len(names) >= 20
    L = bt.lib()
    for n in names:
        assert hasattr(L, n), n
    # the binding covers the same surface
    assert set(names) == set(bt.SIGNATURES)


def test_status_strings():
    L = bt.lib()
    assert L.bt_strerror(0) == b"ok"
    assert L.bt_strerror(-1) == b"invalid argument"
    assert L.bt_strerror(-99) == b"unknown status"


def test_params_layout():
    import ctypes
    assert ctypes.sizeof(bt.bt_params) == 40


def test_ctx_create_ex_rejects_incomplete_allocator():
    """An allocator without both functions is refused before any device call."""
    import ctypes
    al = bt.bt_allocator(bt.ALLOC_FN(), bt.FREE_FN(), None)
    h = ctypes.c_void_p()
    assert bt.lib().bt_ctx_create_ex(0, None, ctypes.byref(al), ctypes.byref(h)) == bt.BT_E_INVAL
    assert not h.value


def test_trees_free_argument_checks():
    """bt_trees_free: nothing to free is fine; a null array with a count is not."""
    L = bt.lib()
    assert L.bt_trees_free(None, 0) == bt.BT_OK
    assert L.bt_trees_free(None, 3) == bt.BT_E_INVAL
