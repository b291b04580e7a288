"""CPU-only checks of the boundary: the HIP library loads and exports every
entry point declared in include/isci.h (no compute call without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "isci.h")
LIB = os.path.join(ROOT, "paper_1609_07757_amd", "libisci.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(isci_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("isci_create", "isci_sigma", "isci_davidson", "isci_destroy"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libisci.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libisci.so not built")
def test_binding_symbol_list_matches_header():
    from paper_1609_07757_amd import _lib
    assert set(_lib.ABI_SYMBOLS) == set(_declared())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libisci.so not built")
def test_status_strings_without_gpu():
    from paper_1609_07757_amd import _lib
    L = _lib.load()
    assert L.isci_status_string(0) == b"ok"
    assert L.isci_status_string(-4) == b"not converged"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libisci.so not built")
def test_invalid_arguments_rejected_before_any_device_work():
    """Null pointers and bad sizes return ISCI_E_INVALID without touching a GPU."""
    from paper_1609_07757_amd import _lib
    L = _lib.load()
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    assert L.isci_create(None, fake, fake, 4, 1, 1, 2, 0.0, None) == _lib.ISCI_E_INVALID
    assert L.isci_create(ctypes.byref(out), None, fake, 4, 1, 1, 2, 0.0, None) == _lib.ISCI_E_INVALID
    assert L.isci_create(ctypes.byref(out), fake, fake, 0, 1, 1, 2, 0.0, None) == _lib.ISCI_E_INVALID
    assert L.isci_create(ctypes.byref(out), fake, fake, 4, 5, 1, 2, 0.0, None) == _lib.ISCI_E_INVALID
    assert L.isci_create(ctypes.byref(out), fake, fake, 4, 1, 1, -1, 0.0, None) == _lib.ISCI_E_INVALID
    assert L.isci_create(ctypes.byref(out), fake, fake, 4, 1, 1, 2, -1.0, None) == _lib.ISCI_E_INVALID
    assert L.isci_create(ctypes.byref(out), fake, fake, 4, 1, 1, 2, float("nan"), None) == _lib.ISCI_E_INVALID
    assert L.isci_create(ctypes.byref(out), fake, fake, 300, 1, 1, 2, 0.0, None) == _lib.ISCI_E_UNSUPPORTED
    assert L.isci_create(ctypes.byref(out), fake, fake, 20, 5, 1, 2, 0.0, None) == _lib.ISCI_E_UNSUPPORTED
    bad = _lib.IsciCreateOpts(7)
    assert L.isci_create_ex(ctypes.byref(out), fake, fake, 4, 1, 1, 2, 0.0, ctypes.byref(bad),
                            None) == _lib.ISCI_E_INVALID
    assert L.isci_create_ex(None, fake, fake, 4, 1, 1, 2, 0.0, None, None) == _lib.ISCI_E_INVALID
    half = _lib.IsciAllocator()   # NULL function pointers
    ao = _lib.IsciCreateOpts(0, ctypes.pointer(half))
    assert L.isci_create_ex(ctypes.byref(out), fake, fake, 4, 1, 1, 2, 0.0, ctypes.byref(ao),
                            None) == _lib.ISCI_E_INVALID
    assert L.isci_sigma(None, 1, fake, 1, fake, 1, None) == _lib.ISCI_E_INVALID
    assert L.isci_density1(None, 1, fake, 1, fake, None) == _lib.ISCI_E_INVALID
    assert L.isci_probe_fp64(2, 1, 1, fake, None, None) == _lib.ISCI_E_INVALID
    g = ctypes.c_void_p(0x2000)
    assert L.isci_sigma_graph_create(None, 1, fake, 1, fake, 1, ctypes.byref(g)) == _lib.ISCI_E_INVALID
    assert g.value is None   # *out cleared on failure
    assert L.isci_sigma_graph_create(None, 1, fake, 1, fake, 1, None) == _lib.ISCI_E_INVALID
    assert L.isci_graph_launch(None, None) == _lib.ISCI_E_INVALID
    L.isci_graph_destroy(None)
    assert L.isci_last_error()
