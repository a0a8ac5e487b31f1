"""The HCI energy as a differentiable function of the active-space integrals.

Forward: E(h, g) on a frozen determinant list V: the lowest eigenvalue of H
on V (the library's Davidson solver), plus, with eps2 > 0, the screened
second-order energy E2(eps2), both summed by the library (hci_energy).
Backward: the library's density matrices, dE/dh = gamma and dE/dg = 1/2
Gamma averaged over the 8-fold integral symmetry (Hellmann-Feynman;
eq. vdedk2 of the paper), or with eps2 > 0 the Lagrangian-relaxed density
matrices (eq. lambda).  V is held fixed so that finite differences of the
energy are defined (re-selecting at perturbed integrals would jump); with
``frozen=True`` the screened pair set of E2 is frozen too (hci_pt2_freeze
at the first evaluation, or by the caller), so E_var + E2 is smooth in the
integrals.

A context passed as ``context`` is reused across calls (its integrals are
replaced by hci_ctx_update_integrals), so repeated evaluations do not create
a context each; otherwise one is created per forward.
"""
from __future__ import annotations

import torch

from . import HCIContext

__all__ = ["HCIEnergy", "hci_energy"]


class HCIEnergy(torch.autograd.Function):
    """E = HCIEnergy.apply(h, g, dets, nalpha, nbeta, options)."""

    @staticmethod
    def forward(fctx, h, g, dets, nalpha, nbeta, options=None):
        opts = dict(options or {})
        tol = opts.get("tol", 1e-10)
        precision = opts.get("precision", "fp64")
        eps2 = float(opts.get("eps2", 0.0))
        frozen = bool(opts.get("frozen", False))
        ctx = opts.get("context")
        if ctx is None:
            ctx = HCIContext(h.detach(), g.detach(), nalpha, nbeta)
        else:
            ctx.update_integrals(h.detach(), g.detach(), ctx.ecore)
        c0 = opts.get("c0")
        if frozen and not opts.get("keep_frozen", False):
            # freeze the pair set at these integrals from this point's eigenvector
            (ev, _, _), c0, _ = ctx.energy(dets, c0, tol=tol, precision=precision)
            ctx.pt2_freeze(dets, c0, eps2)
        (e, e2, e_tot), c, _ = ctx.energy(dets, c0, tol=tol, precision=precision, eps2=eps2, frozen=frozen)
        fctx.hci = ctx
        fctx.dets = dets
        fctx.c = c
        fctx.e = e
        fctx.eps2 = eps2
        fctx.precision = precision
        fctx.z_tol = opts.get("z_tol", 1e-10)
        return torch.tensor(e_tot, dtype=torch.float64, device=h.device)

    @staticmethod
    def backward(fctx, grad_e):
        ge = float(grad_e.detach().cpu())
        dh, dg, _, _ = fctx.hci.energy_backward(fctx.dets, fctx.c, fctx.e, grad_e=ge, eps2=fctx.eps2,
                                                z_tol=fctx.z_tol, precision=fctx.precision)
        return dh, dg, None, None, None, None


def hci_energy(h, g, dets, nalpha, nbeta, **options):
    return HCIEnergy.apply(h, g, dets, nalpha, nbeta, options)
