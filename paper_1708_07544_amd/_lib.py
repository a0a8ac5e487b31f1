"""ctypes binding of libhci.so: argument marshalling only.

Every computation runs in the HIP library; this module converts torch
tensors to device pointers, passes torch's current HIP stream, and routes
the library's scratch allocations through torch's caching allocator.  If
the library has not been built the import fails loudly: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhci.so")

HCI_OK = 0
HCI_E_ARG = -1
HCI_E_NOMEM = -2
HCI_E_CAPACITY = -3
HCI_E_NOCONV = -4
HCI_E_HIP = -5
HCI_E_UNSUPPORTED = -6

FP64 = 0
FP32_MIXED = 1
SIGMA_AUTO = 0
SIGMA_STORED = 1
SIGMA_RECOMPUTE = 2

_STATUS = {
    HCI_E_ARG: "HCI_E_ARG", HCI_E_NOMEM: "HCI_E_NOMEM", HCI_E_CAPACITY: "HCI_E_CAPACITY",
    HCI_E_NOCONV: "HCI_E_NOCONV", HCI_E_HIP: "HCI_E_HIP", HCI_E_UNSUPPORTED: "HCI_E_UNSUPPORTED",
}


class HCIError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class hci_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int
_f64 = ctypes.c_double
_SIGNATURES = {
    "hci_ctx_create": [_i32, _i32, _i32, _vp, _vp, _f64, _vp, _vp, _vp],
    "hci_ctx_update_integrals": [_vp, _vp, _vp, _f64, _vp],
    "hci_ctx_destroy": [_vp],
    "hci_ctx_release_cache": [_vp],
    "hci_ctx_set_stored_budget": [_vp, _i64],
    "hci_ctx_set_stage_window": [_vp, ctypes.c_int],
    "hci_layout_info": [_vp, _vp, _i64, _vp, _vp],
    "hci_ctx_set_timing": [_vp, _i32],
    "hci_ctx_kernel_time": [_vp, ctypes.c_char_p, _vp, _vp, _i32],
    "hci_select": [_vp, _vp, _vp, _i64, _f64, _vp, _i64, _vp, _vp],
    "hci_select_roots": [_vp, _vp, _vp, _i32, _i64, _f64, _vp, _i64, _vp, _vp],
    "hci_embed": [_vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp],
    "hci_sigma": [_vp, _vp, _i64, _vp, _vp, _i32, _i32, _vp],
    "hci_connections": [_vp, _vp, _i64, _vp, _vp],
    "hci_diagonal": [_vp, _vp, _i64, _vp, _vp],
    "hci_davidson": [_vp, _vp, _i64, _vp, _vp, _f64, _i32, _i32, _i32, _vp, _vp],
    "hci_davidson_roots": [_vp, _vp, _i64, _i32, _vp, _vp, _f64, _i32, _i32, _i32, _vp, _vp],
    "hci_spin_square": [_vp, _vp, _i64, _vp, _vp, _vp],
    "hci_rdm12": [_vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp],
    "hci_energy_backward": [_vp, _vp, _i64, _vp, _f64, _f64, _vp, _f64, _f64, _i32, _vp, _vp,
                            _vp, _vp, _vp],
    "hci_pt2": [_vp, _vp, _i64, _vp, _f64, _f64, _vp, _vp, _vp, _vp],
    "hci_pt2_freeze": [_vp, _vp, _i64, _vp, _f64, _vp, _vp],
    "hci_energy": [_vp, _vp, _i64, _vp, _f64, _i32, _i32, _i32, _f64, _i32, _vp, _vp, _vp],
    "hci_ctx_set_pt2_budget": [_vp, _i64],
    "hci_orbital_gradient": [_vp, _vp, _vp, _vp, _vp],
    "hci_orbital_gradient_noalloc": [_vp, _vp, _vp, _vp, _vp],
    "hci_extrapolate": [_vp, _vp, _i64, _vp, _f64, _i32, _f64, _f64, _i32, _vp, _vp, _vp, _vp, _vp],
    "hci_rotate_integrals": [_vp, _vp, _vp, _vp, _vp],
    "hci_pt2_stochastic": [_vp, _vp, _i64, _vp, _f64, _f64, _f64, _vp, _i64, _i64, _vp, _vp, _vp],
    "hci_pt2_semistochastic": [_vp, _vp, _i64, _vp, _f64, _f64, _f64, _vp, _i64, _i64, _vp, _vp, _vp,
                               _vp],
}

_lib = None


def lib():
    """Load libhci.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_1708_07544_amd/build.py "
                              "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.hci_last_error.restype = ctypes.c_char_p
        L.hci_last_error.argtypes = []
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGNATURES) + ["hci_last_error"]


def check(code: int, allow=()):
    if code != HCI_OK and code not in allow:
        raise HCIError(code, lib().hci_last_error().decode())
    return code


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> ctypes.c_void_p:
    if t is None:
        return ctypes.c_void_p(0)
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class TorchAllocator:
    """Routes library scratch through torch's caching allocator."""

    def __init__(self, device: torch.device):
        self.device = device
        self.live = {}
        self._alloc = ALLOC_FN(self._do_alloc)
        self._free = FREE_FN(self._do_free)
        self.struct = hci_allocator(self._alloc, self._free, None)

    def _do_alloc(self, nbytes, stream, user):
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except RuntimeError:
            return None
        p = t.data_ptr()
        self.live[p] = t
        return p

    def _do_free(self, ptr, user):
        self.live.pop(ptr, None)
