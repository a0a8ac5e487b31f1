"""Host-side checks of the C ABI (no GPU): the library loads and exports every
entry point declared in include/hci.h, with the binding's argument lists."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hci.h")
LIB = os.path.join(ROOT, "paper_1708_07544_amd", "libhci.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(hci_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_variational_step_calls():
    names = declared_functions()
    for required in ["hci_select", "hci_sigma", "hci_davidson", "hci_rdm12",
                     "hci_energy_backward", "hci_pt2", "hci_pt2_stochastic", "hci_pt2_semistochastic",
                     "hci_orbital_gradient", "hci_rotate_integrals", "hci_extrapolate"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_every_declared_symbol():
    from paper_1708_07544_amd import _lib
    assert set(declared_functions()) == set(_lib.exported_symbols())


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_null_arguments_are_rejected_without_a_gpu():
    """Argument validation happens before any device work."""
    from paper_1708_07544_amd import _lib
    L = _lib.lib()
    out = ctypes.c_void_p()
    assert L.hci_ctx_create(0, 1, 1, None, None, 0.0, None, None, ctypes.byref(out)) == _lib.HCI_E_ARG
    assert L.hci_ctx_create(65, 1, 1, None, None, 0.0, None, None, ctypes.byref(out)) == _lib.HCI_E_ARG
    assert b"norb" in L.hci_last_error()
    assert L.hci_sigma(None, None, 0, None, None, 0, 0, None) == _lib.HCI_E_ARG
    assert L.hci_ctx_destroy(None) == _lib.HCI_OK
