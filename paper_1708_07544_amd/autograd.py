"""The HCI energy as a differentiable function of the active-space integrals.

Forward: E(h, g) on a frozen determinant list V (the lowest eigenvalue of H
on V, found by the library's Davidson solver).  Backward: the library's
density matrices, dE/dh = gamma and dE/dg = 1/2 Gamma averaged over the
8-fold integral symmetry (Hellmann-Feynman; eq. vdedk2 of the paper).  With
eps2 > 0 the energy is E_var + E2(eps2) with V, C(eps2) and the screening
mask frozen, and the backward is the Lagrangian-relaxed density matrix
(eq. lambda).  V is held fixed so that finite differences of the energy are
well defined (re-selecting at perturbed integrals would jump).
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
        ctx = HCIContext(h.detach(), g.detach(), nalpha, nbeta)
        c0 = opts.get("c0")
        e, c, _ = ctx.davidson(dets, c0, tol=tol, precision=precision)
        e_tot = e
        if eps2 > 0.0:
            e2, _, _ = ctx.pt2(dets, c, e, eps2, want_r=False)
            e_tot = e + e2
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
