"""Pins of the oracle's orbital step (active-active rotations).

* Gradient: central finite differences of E(kappa) = sum h'(kappa) gamma +
  1/2 sum g'(kappa) Gamma with the density matrices of a truncated (HCI-
  like) state held fixed, U = expm(kappa) (scipy), along every independent
  kappa_xy; for the full-CI state it vanishes (the energy of a complete
  active space does not depend on active-active rotations).
* Rotation: the FCI energy is invariant under any orbital rotation (dense
  LAPACK on the rotated integrals); a permutation matrix permutes h and g
  exactly.
"""
import numpy as np
import pytest
import scipy.linalg

import hci_synth as hs
import oracle as O


@pytest.fixture(scope="module")
def fci6():
    n, na, nb = 6, 3, 2
    h, g = hs.make_integrals(n, 18, 41)
    V = hs.full_space(n, na, nb)
    e, c = O.lowest_eigenpair(h, g, V)
    r1, r2 = O.rdm12(n, V, c, c)
    return n, na, nb, h, g, V, e, r1, r2


def _energy(h, g, r1, r2):
    return float(np.sum(h * r1) + 0.5 * np.sum(g * r2))


def test_gradient_vanishes_for_full_ci(fci6):
    n, na, nb, h, g, V, e, r1, r2 = fci6
    assert abs(_energy(h, g, r1, r2) - e) < 1e-10
    assert np.abs(O.orbital_gradient(h, g, r1, r2)).max() < 1e-10


def test_gradient_matches_finite_differences(fci6):
    n, na, nb, h, g, Vf, ef, r1f, r2f = fci6
    # a truncated space: the aufbau determinant and its 40 largest-|H_0a| connections
    V0 = hs.aufbau_det(na, nb)
    C = O.select(h, g, V0, np.array([1.0]), 0.0)
    hv = np.array([abs(O.hij(h, g, V0[0], x)) for x in C])
    V = O.merge(V0, C[np.argsort(-hv)[:40]])
    e, c = O.lowest_eigenpair(h, g, V)
    r1, r2 = O.rdm12(n, V, c, c)
    assert abs(_energy(h, g, r1, r2) - e) < 1e-10
    G = O.orbital_gradient(h, g, r1, r2)
    assert np.abs(G + G.T).max() < 1e-12
    assert np.abs(G).max() > 1e-3  # a truncated state is not stationary in kappa
    step = 1e-5
    for x in range(n):
        for y in range(x):
            k = np.zeros((n, n))
            k[x, y], k[y, x] = step, -step
            ep = _energy(*O.rotate_integrals(h, g, scipy.linalg.expm(k)), r1, r2)
            em = _energy(*O.rotate_integrals(h, g, scipy.linalg.expm(-k)), r1, r2)
            fd = (ep - em) / (2 * step)
            assert abs(fd - G[x, y]) < 1e-7, (x, y, fd, G[x, y])


def test_fci_energy_invariant_under_rotation(fci6):
    n, na, nb, h, g, V, e, r1, r2 = fci6
    rng = np.random.default_rng(3)
    U = scipy.linalg.expm(0.3 * (lambda a: a - a.T)(rng.normal(size=(n, n))))
    h2, g2 = O.rotate_integrals(h, g, U)
    e2, _ = O.lowest_eigenpair(h2, g2, V)
    assert abs(e2 - e) < 1e-10
    # 8-fold symmetry and symmetry of h survive
    assert np.abs(h2 - h2.T).max() < 1e-13
    for p in [(1, 0, 2, 3), (2, 3, 0, 1), (0, 1, 3, 2)]:
        assert np.abs(g2 - g2.transpose(p)).max() < 1e-13


def test_permutation_permutes_integrals(fci6):
    n, na, nb, h, g, V, e, r1, r2 = fci6
    perm = np.array([3, 0, 5, 1, 4, 2])
    U = np.zeros((n, n))
    U[perm, np.arange(n)] = 1.0  # new orbital p is old orbital perm[p]
    h2, g2 = O.rotate_integrals(h, g, U)
    assert np.array_equal(h2, h[np.ix_(perm, perm)])
    assert np.array_equal(g2, g[np.ix_(perm, perm, perm, perm)])
