"""Orbital step (active-active rotations) on the matrix cores against the oracle.

* Gradient dE/dkappa and rotated integrals at n = 3, 8, 16, 30, 44 and the
  largest supported n = 64 (ragged against the 16-wide tiles except n = 16
  and 64), the density matrices of a selected state (n = 8, 16) or random
  tensors with the index symmetries of a real state (other n);
  contractions of n^3 terms in another order: 1e-12 of the largest entry.
* Through the library end to end: the full-CI energy of (8e,8o) with
  rotated integrals equals the unrotated one, and the orbital gradient of
  the full-CI state vanishes.
"""
import numpy as np
import pytest
import scipy.linalg
import torch

import hci_synth as hs
import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P(gpu_available):
    import paper_1708_07544_amd as P
    return P


def _sym_tensors(n, seed):
    rng = np.random.default_rng(seed)
    r1 = rng.normal(size=(n, n))
    r1 = r1 + r1.T
    r2 = rng.normal(size=(n, n, n, n))
    r2 = r2 + r2.transpose(2, 3, 0, 1)
    r2 = r2 + r2.transpose(1, 0, 3, 2)
    return r1, r2


def _case(n):
    if n == 8:
        w = hs.WORKLOADS["cas8"]
        h, g = hs.workload_integrals(w)
        na = nb = 4
    elif n == 16:
        w = hs.WORKLOADS["cas16"]
        h, g = hs.workload_integrals(w)
        na = nb = 8
    else:
        h, g = hs.make_integrals(n, 3 * n, n)
        na = nb = max(1, n // 2)
    return h, g, na, nb


@pytest.mark.parametrize("n", [3, 8, 16, 30, 44, 64])
def test_gradient_and_rotation_match_oracle(P, n):
    h, g, na, nb = _case(n)
    ctx = P.HCIContext(h, g, na, nb)
    if n in (8, 16):  # density matrices of a selected state
        V0 = hs.aufbau_det(na, nb)
        V = O.merge(V0, O.select(h, g, V0, np.array([1.0]), 5e-2 if n == 16 else 1e-2))
        e, c, _ = ctx.davidson(V, None, tol=1e-9)
        r1t, r2t = ctx.rdm12(V, c)
        r1, r2 = r1t.cpu().numpy(), r2t.cpu().numpy()
    else:
        r1, r2 = _sym_tensors(n, n)
    print(f"[orbital n={n}]", flush=True)
    G = ctx.orbital_gradient(r1, r2).cpu().numpy()
    Gref = O.orbital_gradient(h, g, r1, r2)
    assert np.abs(G - Gref).max() <= 1e-12 * max(1.0, np.abs(Gref).max()), np.abs(G - Gref).max()
    assert np.abs(G + G.T).max() == 0.0
    rng = np.random.default_rng(100 + n)
    k = rng.normal(scale=0.2, size=(n, n))
    U = scipy.linalg.expm(k - k.T)
    h2, g2 = ctx.rotate_integrals(U)
    rh, rg = O.rotate_integrals(h, g, U)
    h2, g2 = h2.cpu().numpy(), g2.cpu().numpy()
    assert np.abs(h2 - rh).max() <= 1e-12 * np.abs(rh).max()
    assert np.abs(g2 - rg).max() <= 1e-12 * np.abs(rg).max(), np.abs(g2 - rg).max()
    ctx.close()


def test_rotated_full_ci_energy_and_vanishing_gradient(P):
    w = hs.WORKLOADS["cas8"]
    h, g = hs.workload_integrals(w)
    V = hs.full_space(8, 4, 4)
    ctx = P.HCIContext(h, g, 4, 4)
    e, c, _ = ctx.davidson(V, None, tol=1e-10)
    r1, r2 = ctx.rdm12(V, c)
    G = ctx.orbital_gradient(r1, r2).cpu().numpy()
    assert np.abs(G).max() < 1e-8, np.abs(G).max()
    rng = np.random.default_rng(8)
    k = rng.normal(scale=0.3, size=(8, 8))
    U = scipy.linalg.expm(k - k.T)
    h2, g2 = ctx.rotate_integrals(U)
    ctx2 = P.HCIContext(h2.cpu().numpy(), g2.cpu().numpy(), 4, 4)
    e2, _, _ = ctx2.davidson(V, None, tol=1e-10)
    assert abs(e2 - e) < 1e-9, (e, e2)
    ctx2.close()
    ctx.close()
