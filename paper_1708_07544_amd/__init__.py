"""MI355X (gfx950) Heat-bath CI variational step.

Smith, Mussard, Holmes, Sharma, "Cheap and near exact CASSCF with large
active spaces" (arXiv:1708.07544): HCI selection, the Hamiltonian product
inside Davidson, density matrices and the energy's integral derivatives, as
hand-written HIP kernels behind the C ABI of ``include/hci.h``.  This
package is the thin torch-facing binding of that library.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import numpy as np
import torch

from . import _lib
from ._lib import (FP32_MIXED, FP64, HCIError, SIGMA_AUTO, SIGMA_RECOMPUTE, SIGMA_STORED,
                   check, lib)

__all__ = ["HCIContext", "HCIError", "FP64", "FP32_MIXED", "SIGMA_AUTO", "SIGMA_STORED",
           "SIGMA_RECOMPUTE", "dets_to_device", "dets_to_numpy"]

_PREC = {"fp64": FP64, "fp32_mixed": FP32_MIXED, "mixed": FP32_MIXED, FP64: FP64,
         FP32_MIXED: FP32_MIXED}
_MODE = {"auto": SIGMA_AUTO, "stored": SIGMA_STORED, "recompute": SIGMA_RECOMPUTE,
         SIGMA_AUTO: SIGMA_AUTO, SIGMA_STORED: SIGMA_STORED, SIGMA_RECOMPUTE: SIGMA_RECOMPUTE}


def dets_to_device(dets, device="cuda") -> torch.Tensor:
    """[m,2] uint64 (alpha, beta) words -> contiguous int64 device tensor (same bits)."""
    if isinstance(dets, torch.Tensor):
        return dets.to(device=device, dtype=torch.int64).contiguous()
    a = np.ascontiguousarray(np.asarray(dets, dtype=np.uint64).reshape(-1, 2))
    return torch.from_numpy(a.view(np.int64)).to(device).contiguous()


def dets_to_numpy(dets: torch.Tensor) -> np.ndarray:
    return np.ascontiguousarray(dets.detach().cpu().numpy()).view(np.uint64).reshape(-1, 2)


class HCIContext:
    """Integrals staged on one GPU plus the heat-bath tables (hci_ctx)."""

    def __init__(self, h, g, nalpha: int, nbeta: int, ecore: float = 0.0, device=None):
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        h = torch.as_tensor(h, dtype=torch.float64).to(self.device).contiguous()
        g = torch.as_tensor(g, dtype=torch.float64).to(self.device).contiguous()
        n = h.shape[0]
        if h.shape != (n, n) or g.shape != (n, n, n, n):
            raise ValueError("h must be [n,n] and g [n,n,n,n]")
        self.norb, self.nalpha, self.nbeta, self.ecore = n, int(nalpha), int(nbeta), float(ecore)
        self._alloc = _lib.TorchAllocator(self.device)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().hci_ctx_create(n, self.nalpha, self.nbeta, _lib._ptr(h), _lib._ptr(g),
                                       self.ecore, ctypes.byref(self._alloc.struct),
                                       _lib._stream(), ctypes.byref(handle)))
        self.handle = handle

    def close(self):
        if getattr(self, "handle", None):
            lib().hci_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- options
    def update_integrals(self, h, g, ecore: float = 0.0):
        h = torch.as_tensor(h, dtype=torch.float64).to(self.device).contiguous()
        g = torch.as_tensor(g, dtype=torch.float64).to(self.device).contiguous()
        self.ecore = float(ecore)
        check(lib().hci_ctx_update_integrals(self.handle, _lib._ptr(h), _lib._ptr(g), self.ecore,
                                             _lib._stream()))

    def release_cache(self):
        check(lib().hci_ctx_release_cache(self.handle))

    def set_stored_budget(self, nbytes: int):
        check(lib().hci_ctx_set_stored_budget(self.handle, int(nbytes)))

    def set_stage_window(self, log2_window: int):
        """Stored-matrix layout: 0 = plain CSR, 6..16 = alpha-bucket-staged
        with 2**log2_window entries of c per on-chip window."""
        check(lib().hci_ctx_set_stage_window(self.handle, int(log2_window)))

    def set_timing(self, on: bool):
        check(lib().hci_ctx_set_timing(self.handle, 1 if on else 0))

    def kernel_time(self, name: str, reset: bool = False) -> Tuple[int, float]:
        launches = ctypes.c_int64()
        ms = ctypes.c_double()
        check(lib().hci_ctx_kernel_time(self.handle, name.encode(), ctypes.byref(launches),
                                        ctypes.byref(ms), 1 if reset else 0))
        return int(launches.value), float(ms.value)

    # ---------------------------------------------------------------- calls
    def _dets(self, dets) -> torch.Tensor:
        d = dets_to_device(dets, self.device)
        if d.dim() != 2 or d.shape[1] != 2:
            raise ValueError("dets must be [m,2]")
        return d

    def select(self, dets, c, eps1: float, cap: Optional[int] = None) -> torch.Tensor:
        """V + C(eps1), sorted and unique (int64 [m,2] on the device).  A 2-D c
        holds several states as rows: the union of their selections."""
        d = self._dets(dets)
        c = torch.as_tensor(c, dtype=torch.float64).to(self.device).contiguous()
        n = d.shape[0]
        if c.dim() == 2 and c.shape[1] != n or c.dim() == 1 and c.shape[0] != n or c.dim() > 2:
            raise ValueError("c must be [n] or [nroots, n]")
        cap = int(cap) if cap is not None else max(4 * n, 1 << 16)
        n_out = ctypes.c_int64()
        for _ in range(2):
            out = torch.empty((max(cap, 1), 2), dtype=torch.int64, device=self.device)
            if c.dim() == 2:
                call = lib().hci_select_roots(self.handle, _lib._ptr(d), _lib._ptr(c), c.shape[0], n,
                                              float(eps1), _lib._ptr(out), cap, ctypes.byref(n_out),
                                              _lib._stream())
            else:
                call = lib().hci_select(self.handle, _lib._ptr(d), _lib._ptr(c), n, float(eps1),
                                        _lib._ptr(out), cap, ctypes.byref(n_out), _lib._stream())
            code = check(call, allow=(_lib.HCI_E_CAPACITY,))
            if code == _lib.HCI_OK:
                return out[: n_out.value].contiguous()
            cap = int(n_out.value)
        raise HCIError(_lib.HCI_E_CAPACITY, "selection capacity retry failed")

    def embed(self, dets, c, dets_new) -> torch.Tensor:
        """c carried from V to the superset V' (zeros on the new members)."""
        d = self._dets(dets)
        dn = self._dets(dets_new)
        c = torch.as_tensor(c, dtype=torch.float64).to(self.device).contiguous()
        out = torch.empty(dn.shape[0], dtype=torch.float64, device=self.device)
        check(lib().hci_embed(self.handle, _lib._ptr(d), d.shape[0], _lib._ptr(c), _lib._ptr(dn),
                              dn.shape[0], _lib._ptr(out), _lib._stream()))
        return out

    def sigma(self, dets, c, precision="fp64", mode="auto") -> torch.Tensor:
        d = self._dets(dets)
        c = torch.as_tensor(c, dtype=torch.float64).to(self.device).contiguous()
        out = torch.empty_like(c)
        check(lib().hci_sigma(self.handle, _lib._ptr(d), d.shape[0], _lib._ptr(c), _lib._ptr(out),
                              _PREC[precision], _MODE[mode], _lib._stream()))
        return out

    def connections(self, dets) -> int:
        d = self._dets(dets)
        nnz = ctypes.c_int64()
        check(lib().hci_connections(self.handle, _lib._ptr(d), d.shape[0], ctypes.byref(nnz),
                                    _lib._stream()))
        return int(nnz.value)

    def layout_info(self, dets) -> dict:
        """Statistics of the stored Hamiltonian of `dets` (layout, entries,
        window, beta-group entries, staged c entries, workgroups)."""
        d = self._dets(dets)
        info = (ctypes.c_int64 * 8)()
        check(lib().hci_layout_info(self.handle, _lib._ptr(d), d.shape[0],
                                    ctypes.cast(info, ctypes.c_void_p), _lib._stream()))
        keys = ["layout", "nnz_off", "stored_entries", "log2_window", "group_entries",
                "staged_c_entries", "workgroups", "group_workgroups"]
        return dict(zip(keys, (int(x) for x in info)))

    def diagonal(self, dets) -> torch.Tensor:
        d = self._dets(dets)
        out = torch.empty(d.shape[0], dtype=torch.float64, device=self.device)
        check(lib().hci_diagonal(self.handle, _lib._ptr(d), d.shape[0], _lib._ptr(out),
                                 _lib._stream()))
        return out

    def davidson(self, dets, c0=None, tol: float = 1e-8, max_iter: int = 500,
                 precision="fp64", mode="auto", allow_noconv: bool = False):
        """Lowest eigenpair on V: returns (E, c, products)."""
        d = self._dets(dets)
        n = d.shape[0]
        if c0 is None:
            c = torch.zeros(n, dtype=torch.float64, device=self.device)
        else:
            c = torch.as_tensor(c0, dtype=torch.float64).to(self.device).clone().contiguous()
        e = ctypes.c_double()
        iters = ctypes.c_int()
        allow = (_lib.HCI_E_NOCONV,) if allow_noconv else ()
        check(lib().hci_davidson(self.handle, _lib._ptr(d), n, _lib._ptr(c), ctypes.byref(e),
                                 float(tol), int(max_iter), _PREC[precision], _MODE[mode],
                                 ctypes.byref(iters), _lib._stream()), allow=allow)
        return float(e.value), c, int(iters.value)

    def energy(self, dets, c0=None, tol: float = 1e-10, max_iter: int = 500, precision="fp64",
               mode="auto", eps2: float = 0.0, frozen: bool = False, allow_noconv: bool = False):
        """E_var + E2 of the list (E2 over the frozen pair set when frozen,
        else re-screened at eps2): returns ((E_var, E2, E_var + E2), c, products)."""
        d = self._dets(dets)
        n = d.shape[0]
        if c0 is None:
            c = torch.zeros(n, dtype=torch.float64, device=self.device)
        else:
            c = torch.as_tensor(c0, dtype=torch.float64).to(self.device).clone().contiguous()
        e = (ctypes.c_double * 3)()
        iters = ctypes.c_int()
        allow = (_lib.HCI_E_NOCONV,) if allow_noconv else ()
        check(lib().hci_energy(self.handle, _lib._ptr(d), n, _lib._ptr(c), float(tol), int(max_iter),
                               _PREC[precision], _MODE[mode], float(eps2), int(bool(frozen)),
                               ctypes.cast(e, ctypes.c_void_p), ctypes.byref(iters), _lib._stream()),
              allow=allow)
        return (float(e[0]), float(e[1]), float(e[2])), c, int(iters.value)

    def pt2_freeze(self, dets, c, eps2: float) -> int:
        """Freeze the screened pair set of (dets, c) at eps2 for energy(..., frozen=True); returns |M|."""
        d = self._dets(dets)
        c = torch.as_tensor(c, dtype=torch.float64).to(self.device).contiguous()
        m = ctypes.c_int64()
        check(lib().hci_pt2_freeze(self.handle, _lib._ptr(d), d.shape[0], _lib._ptr(c), float(eps2),
                                   ctypes.byref(m), _lib._stream()))
        return int(m.value)

    def davidson_roots(self, dets, nroots: int, c0=None, tol: float = 1e-8, max_iter: int = 500,
                       precision="fp64", mode="auto", allow_noconv: bool = False):
        """The nroots lowest eigenpairs on V: returns (E [nroots] numpy,
        C [nroots, n] orthonormal rows, products per state)."""
        d = self._dets(dets)
        n = d.shape[0]
        if c0 is None:
            c = torch.zeros((nroots, n), dtype=torch.float64, device=self.device)
        else:
            c = torch.as_tensor(c0, dtype=torch.float64).to(self.device).clone().contiguous()
            if c.shape != (nroots, n):
                raise ValueError("c0 must be [nroots, n]")
        e = (ctypes.c_double * max(nroots, 1))()
        iters = (ctypes.c_int * max(nroots, 1))()
        allow = (_lib.HCI_E_NOCONV,) if allow_noconv else ()
        check(lib().hci_davidson_roots(self.handle, _lib._ptr(d), n, int(nroots), _lib._ptr(c),
                                       ctypes.cast(e, ctypes.c_void_p), float(tol), int(max_iter),
                                       _PREC[precision], _MODE[mode], ctypes.cast(iters, ctypes.c_void_p),
                                       _lib._stream()), allow=allow)
        return np.array(e[:nroots]), c, [int(x) for x in iters[:nroots]]

    def spin_square(self, dets, c) -> float:
        """<S^2> of the state c on V."""
        d = self._dets(dets)
        c = torch.as_tensor(c, dtype=torch.float64).to(self.device).contiguous()
        s2 = ctypes.c_double()
        check(lib().hci_spin_square(self.handle, _lib._ptr(d), d.shape[0], _lib._ptr(c), ctypes.byref(s2),
                                    _lib._stream()))
        return float(s2.value)

    def rdm12(self, dets, bra, ket=None, two_body: bool = True):
        d = self._dets(dets)
        bra = torch.as_tensor(bra, dtype=torch.float64).to(self.device).contiguous()
        ket = bra if ket is None else torch.as_tensor(ket, dtype=torch.float64).to(self.device).contiguous()
        n = self.norb
        r1 = torch.empty((n, n), dtype=torch.float64, device=self.device)
        r2 = torch.empty((n, n, n, n), dtype=torch.float64, device=self.device) if two_body else None
        check(lib().hci_rdm12(self.handle, _lib._ptr(d), d.shape[0], _lib._ptr(bra), _lib._ptr(ket),
                              _lib._ptr(r1), _lib._ptr(r2), _lib._stream()))
        return r1, r2

    def energy_backward(self, dets, c, e: float, grad_e: float = 1.0, r=None, eps2: float = 0.0,
                        z_tol: float = 1e-8, precision="fp64", want_z: bool = False):
        """(dh, dg, z or None, E2)."""
        d = self._dets(dets)
        c = torch.as_tensor(c, dtype=torch.float64).to(self.device).contiguous()
        n = self.norb
        dh = torch.empty((n, n), dtype=torch.float64, device=self.device)
        dg = torch.empty((n, n, n, n), dtype=torch.float64, device=self.device)
        rr = None if r is None else torch.as_tensor(r, dtype=torch.float64).to(self.device).contiguous()
        z = torch.empty_like(c) if want_z else None
        e2 = ctypes.c_double()
        check(lib().hci_energy_backward(self.handle, _lib._ptr(d), d.shape[0], _lib._ptr(c),
                                        float(e), float(grad_e), _lib._ptr(rr), float(eps2),
                                        float(z_tol), _PREC[precision], _lib._ptr(dh), _lib._ptr(dg),
                                        _lib._ptr(z), ctypes.byref(e2), _lib._stream()))
        return dh, dg, z, float(e2.value)

    def pt2(self, dets, c, e0: float, eps2: float, want_r: bool = True):
        """(E2, r = dE2/dc or None, |C(eps2)|)."""
        d = self._dets(dets)
        c = torch.as_tensor(c, dtype=torch.float64).to(self.device).contiguous()
        r = torch.empty_like(c) if want_r else None
        e2 = ctypes.c_double()
        nc = ctypes.c_int64()
        check(lib().hci_pt2(self.handle, _lib._ptr(d), d.shape[0], _lib._ptr(c), float(e0),
                            float(eps2), ctypes.byref(e2), _lib._ptr(r), ctypes.byref(nc),
                            _lib._stream()))
        return float(e2.value), r, int(nc.value)

    def extrapolate(self, dets, c, fraction: float = 0.33, levels: int = 4, eps2: float = 1e-5,
                    tol: float = 1e-8, precision="fp64") -> dict:
        """Extrapolation to the full-CI limit over nested truncations of (dets, c):
        dict(sizes, evar, e2, e_extrap, slope, error)."""
        d = self._dets(dets)
        c = torch.as_tensor(c, dtype=torch.float64).to(self.device).contiguous()
        nv = np.zeros(levels, dtype=np.int64)
        ev = np.zeros(levels)
        e2 = np.zeros(levels)
        fit = np.zeros(3)
        vp = ctypes.c_void_p
        check(lib().hci_extrapolate(self.handle, _lib._ptr(d), d.shape[0], _lib._ptr(c), float(fraction),
                                    int(levels), float(eps2), float(tol), _PREC[precision],
                                    nv.ctypes.data_as(vp), ev.ctypes.data_as(vp), e2.ctypes.data_as(vp),
                                    fit.ctypes.data_as(vp), _lib._stream()))
        return dict(sizes=[int(x) for x in nv], evar=ev, e2=e2, e_extrap=float(fit[0]), slope=float(fit[1]),
                    error=float(fit[2]))

    def orbital_gradient(self, rdm1, rdm2) -> torch.Tensor:
        """dE/dkappa (antisymmetric [n][n]) of E = sum h gamma + 1/2 sum g Gamma
        for active-active rotations of this context's orbitals."""
        r1 = torch.as_tensor(rdm1, dtype=torch.float64).to(self.device).contiguous()
        r2 = torch.as_tensor(rdm2, dtype=torch.float64).to(self.device).contiguous()
        n = self.norb
        if r1.shape != (n, n) or r2.shape != (n, n, n, n):
            raise ValueError("rdm1 must be [n,n] and rdm2 [n,n,n,n]")
        grad = torch.empty((n, n), dtype=torch.float64, device=self.device)
        check(lib().hci_orbital_gradient(self.handle, _lib._ptr(r1), _lib._ptr(r2), _lib._ptr(grad),
                                         _lib._stream()))
        return grad

    def orbital_gradient_noalloc(self, rdm1, rdm2, grad) -> torch.Tensor:
        """The same gradient written into the caller's grad ([n][n] float64 on
        this device) by the entry point that allocates nothing."""
        n = self.norb
        for t, shape in ((rdm1, (n, n)), (rdm2, (n, n, n, n)), (grad, (n, n))):
            if (not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda
                    or tuple(t.shape) != shape or not t.is_contiguous()):
                raise ValueError("rdm1, rdm2, grad must be contiguous float64 tensors of shapes "
                                 "[n,n], [n,n,n,n], [n,n] on the context's device")
        check(lib().hci_orbital_gradient_noalloc(self.handle, _lib._ptr(rdm1), _lib._ptr(rdm2),
                                                 _lib._ptr(grad), _lib._stream()))
        return grad

    def rotate_integrals(self, U) -> Tuple[torch.Tensor, torch.Tensor]:
        """(U^T h U, (U x U x U x U)^T g) of this context's integrals."""
        n = self.norb
        U = torch.as_tensor(U, dtype=torch.float64).to(self.device).contiguous()
        if U.shape != (n, n):
            raise ValueError("U must be [n,n]")
        h2 = torch.empty((n, n), dtype=torch.float64, device=self.device)
        g2 = torch.empty((n, n, n, n), dtype=torch.float64, device=self.device)
        check(lib().hci_rotate_integrals(self.handle, _lib._ptr(U), _lib._ptr(h2), _lib._ptr(g2),
                                         _lib._stream()))
        return h2, g2

    def set_pt2_budget(self, nbytes: int) -> None:
        """Device bytes the screened PT2 pairs may hold at once."""
        check(lib().hci_ctx_set_pt2_budget(self.handle, int(nbytes)))

    def _uniforms(self, u):
        u = torch.as_tensor(u, dtype=torch.float64).to(self.device).contiguous()
        if u.dim() != 2:
            raise ValueError("u must have shape [n_batch, n_samp]")
        return u

    def pt2_stochastic(self, dets, c, e0: float, eps2: float, eps2_d: float, u):
        """Per-batch sampled estimates (E2^S(eps2), E2^S(eps2_d)) of eq. semistoc
        from the uniforms u [n_batch, n_samp] (numpy arrays of n_batch)."""
        d = self._dets(dets)
        c = torch.as_tensor(c, dtype=torch.float64).to(self.device).contiguous()
        u = self._uniforms(u)
        nb, ns = u.shape
        a = np.zeros(nb)
        b = np.zeros(nb)
        check(lib().hci_pt2_stochastic(self.handle, _lib._ptr(d), d.shape[0], _lib._ptr(c), float(e0),
                                       float(eps2), float(eps2_d), _lib._ptr(u), ns, nb,
                                       a.ctypes.data_as(ctypes.c_void_p), b.ctypes.data_as(ctypes.c_void_p),
                                       _lib._stream()))
        return a, b

    def pt2_semistochastic(self, dets, c, e0: float, eps2: float, eps2_d: float, u):
        """eq. semistoc: (E2, standard error over batches, E2^D(eps2_d))."""
        d = self._dets(dets)
        c = torch.as_tensor(c, dtype=torch.float64).to(self.device).contiguous()
        u = self._uniforms(u)
        nb, ns = u.shape
        e2, err, e2d = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        check(lib().hci_pt2_semistochastic(self.handle, _lib._ptr(d), d.shape[0], _lib._ptr(c),
                                           float(e0), float(eps2), float(eps2_d), _lib._ptr(u), ns, nb,
                                           ctypes.byref(e2), ctypes.byref(err), ctypes.byref(e2d),
                                           _lib._stream()))
        return float(e2.value), float(err.value), float(e2d.value)

    # ------------------------------------------------------------ HCI loop
    def hci(self, eps1: float, max_macro: int = 20, tol: float = 1e-8, precision="fp64",
            mode="auto", dets0=None, log=None, nroots: int = 1):
        """HCI variational stage: V0 = aufbau (or dets0), then repeatedly
        V <- V + C(eps1) and re-diagonalise until nothing is added.  With
        nroots > 1 the nroots lowest states are followed and C is the union
        of their selections (dets0 must then hold at least nroots
        determinants); returns (V, C [nroots, n], E [nroots], history)."""
        if nroots > 1:
            return self._hci_roots(eps1, nroots, dets0, max_macro, tol, precision, mode, log)
        if dets0 is None:
            dets0 = np.array([[(1 << self.nalpha) - 1, (1 << self.nbeta) - 1]], dtype=np.uint64)
        V = self._dets(dets0)
        e, c, it = self.davidson(V, None, tol=tol, precision=precision, mode=mode)
        hist = [(int(V.shape[0]), e, it)]
        for _ in range(max_macro):
            Vn = self.select(V, c, eps1)
            if Vn.shape[0] == V.shape[0]:
                break
            c0 = self.embed(V, c, Vn)
            V = Vn
            e, c, it = self.davidson(V, c0, tol=tol, precision=precision, mode=mode)
            hist.append((int(V.shape[0]), e, it))
            if log:
                log(hist[-1])
        return V, c, e, hist

    def _hci_roots(self, eps1, nroots, dets0, max_macro, tol, precision, mode, log):
        if dets0 is None:
            raise ValueError("several states need a start list dets0 of at least nroots determinants")
        V = self._dets(dets0)
        e, C, it = self.davidson_roots(V, nroots, tol=tol, precision=precision, mode=mode)
        hist = [(int(V.shape[0]), e, it)]
        for _ in range(max_macro):
            Vn = self.select(V, C, eps1)
            if Vn.shape[0] == V.shape[0]:
                break
            C0 = torch.stack([self.embed(V, C[r], Vn) for r in range(nroots)])
            V = Vn
            e, C, it = self.davidson_roots(V, nroots, c0=C0, tol=tol, precision=precision, mode=mode)
            hist.append((int(V.shape[0]), e, it))
            if log:
                log(hist[-1])
        return V, C, e, hist
