"""Pins of the oracle's several-state functions (no GPU).

* The k lowest eigenvalues of a Hamiltonian without two-electron terms are
  the k smallest sums of one-electron eigenvalues over N_alpha and N_beta
  distinct orbitals (closed form).
* The spectrum of a spin projection M_s = (N_alpha - N_beta)/2 > 0 is
  contained in that of every smaller |M_s| with the same electron count
  (every spin multiplet has a component in each sector): pins the two-electron
  terms between unequal alpha and beta counts, the paper's triplet and
  quintet states.
* Both eigensolver routes (dense and Lanczos) against the eigenvalues of the
  operator-built Hamiltonian.
* The union selection against brute force over the whole space with the
  criterion maximised over states, and against the single-state selection.
"""
import itertools

import numpy as np
import pytest

import hci_synth as hs
import oracle as O


@pytest.mark.parametrize("n,na,nb,k,seed", [(6, 3, 2, 10, 1), (7, 2, 2, 12, 2), (5, 4, 1, 5, 3)])
def test_noninteracting_spectrum(n, na, nb, k, seed):
    rng = np.random.default_rng(seed)
    h = rng.normal(size=(n, n))
    h = h + h.T
    g = np.zeros((n, n, n, n))
    eps = np.linalg.eigvalsh(h)
    sums = sorted(sum(eps[list(A)]) + sum(eps[list(B)])
                  for A in itertools.combinations(range(n), na)
                  for B in itertools.combinations(range(n), nb))
    V = hs.full_space(n, na, nb)
    e, C = O.lowest_eigenpairs(h, g, V, k)
    assert np.abs(e - np.array(sums[:k])).max() < 1e-10
    assert np.all(np.diff(e) >= 0)


@pytest.mark.parametrize("n,N,seed", [(6, 6, 4), (6, 5, 5), (7, 4, 6)])
def test_spin_sector_spectra_nested(n, N, seed):
    h, g = hs.make_integrals(n, 3 * n, seed)
    spectra = {}
    for na in range((N + 1) // 2, min(n, N) + 1):
        nb = N - na
        V = hs.full_space(n, na, nb)
        spectra[na] = np.linalg.eigvalsh(O.hamiltonian_csr(h, g, V).toarray())
    keys = sorted(spectra)
    for lo, hi in zip(keys, keys[1:]):
        a, b = spectra[hi], spectra[lo]
        assert len(a) < len(b)
        # every level of the higher projection appears in the lower one
        d = np.abs(a[:, None] - b[None, :]).min(axis=1)
        assert d.max() < 1e-9, (lo, hi, d.max())
    # the sectors are not all the same: the lowest state is a low-spin one
    assert spectra[keys[0]][0] < spectra[keys[-1]][0] - 1e-6


@pytest.mark.parametrize("route", ["dense", "lanczos"])
def test_lowest_eigenpairs_both_routes(route):
    n, na, nb = 7, 3, 3
    h, g = hs.make_integrals(n, 21, 9)
    V = hs.random_dets(n, na, nb, 300, seed=9, bias=0.2)
    H_op = O.hamiltonian_by_operators(h, g, V)
    ref = np.linalg.eigvalsh(H_op)
    k = 6
    e, C = O.lowest_eigenpairs(h, g, V, k, dense_max=3000 if route == "dense" else 0)
    assert np.abs(e - ref[:k]).max() < 1e-9
    # eigenvectors: orthonormal, residuals small, sign convention
    assert np.abs(C @ C.T - np.eye(k)).max() < 1e-9
    assert np.abs(C @ H_op - e[:, None] * C).max() < 1e-7
    for c in C:
        j = int(np.argmax(np.abs(c)))
        assert c[j] > 0


def test_lowest_eigenpairs_rejects_bad_k():
    h, g = hs.make_integrals(4, 12, 1)
    V = hs.full_space(4, 1, 1)
    with pytest.raises(ValueError):
        O.lowest_eigenpairs(h, g, V, 0)
    with pytest.raises(ValueError):
        O.lowest_eigenpairs(h, g, V, len(V) + 1)


@pytest.mark.parametrize("eps", [1e-3, 2e-2, 1e-1])
def test_select_roots_union_matches_bruteforce(eps):
    n, na, nb = 6, 3, 2
    h, g = hs.make_integrals(n, 18, 11)
    space = hs.full_space(n, na, nb)
    V = hs.random_dets(n, na, nb, 12, seed=11, bias=0.3)
    C = np.stack([hs.random_coeffs(len(V), 20 + r) for r in range(3)])
    got = O.select_roots(h, g, V, C, eps)
    ref = O.select_bruteforce(h, g, V, C, eps, space)
    assert np.array_equal(got, ref)
    # one state is the single-state selection; the union holds each state's
    single = [O.select(h, g, V, c, eps) for c in C]
    assert np.array_equal(O.select_roots(h, g, V, C[:1], eps), single[0])
    have = {tuple(x) for x in got.tolist()}
    for s in single:
        assert {tuple(x) for x in s.tolist()} <= have
    assert len(got) <= sum(len(s) for s in single)


def test_hci_roots_reaches_full_ci_states_and_is_variational():
    """eps1 = 0 grows V until the tracked states are the full-CI ones; on the
    way each state's energy never rises (the k lowest eigenvalues of a
    larger space are below those of a subspace, by interlacing)."""
    n, na, nb, k = 6, 3, 2, 3
    h, g = hs.make_integrals(n, 18, 13)
    full = np.linalg.eigvalsh(O.hamiltonian_csr(h, g, hs.full_space(n, na, nb)).toarray())
    V0 = O.merge(hs.aufbau_det(na, nb), O.select(h, g, hs.aufbau_det(na, nb), np.array([1.0]), 0.2))
    assert len(V0) >= k
    V, C, e, hist = O.hci_roots(h, g, na, nb, 0.0, k, V0)
    assert np.abs(e - full[:k]).max() < 1e-10
    E = np.array([x for _, x in hist])
    assert np.all(np.diff(E, axis=0) <= 1e-12)
    assert len(hist) > 2


def _det(alpha_orbs, beta_orbs):
    return [hs.det_bits(alpha_orbs), hs.det_bits(beta_orbs)]


def test_spin_square_hand_cases():
    """Closed shell 0; one alpha and one beta electron in different orbitals
    1 (half singlet, half triplet); their two combinations 0 and 2; a
    high-spin determinant S_z (S_z + 1)."""
    assert abs(O.spin_square(np.array([_det([0, 1], [0, 1])]), [1.0])) < 1e-15
    assert abs(O.spin_square(np.array([_det([0], [1])]), [1.0]) - 1.0) < 1e-15
    V = O.sort_unique(np.array([_det([0], [1]), _det([1], [0])], dtype=np.uint64))
    got = sorted(O.spin_square(V, np.array([1.0, s]) / np.sqrt(2.0)) for s in (1.0, -1.0))
    assert abs(got[0]) < 1e-15 and abs(got[1] - 2.0) < 1e-15
    assert abs(O.spin_square(np.array([_det([0, 1, 3], [])]), [1.0]) - 1.5 * 2.5) < 1e-15


@pytest.mark.parametrize("n,na,nb,seed", [(6, 3, 3, 4), (6, 4, 2, 5), (5, 3, 2, 6)])
def test_spin_square_of_eigenstates_matches_the_spin_sectors(n, na, nb, seed):
    """Every eigenstate of a full space has <S^2> = S(S+1) with S integer or
    half-integer as N; and S is also what the spectra say: the state's energy
    appears in the M_s = S sector and not in M_s = S + 1."""
    h, g = hs.make_integrals(n, 3 * n, seed)
    N = na + nb
    spectra = {}
    for a in range((N + 1) // 2, min(n, N) + 1):
        spectra[a] = np.linalg.eigvalsh(O.hamiltonian_csr(h, g, hs.full_space(n, a, N - a)).toarray())
    V = hs.full_space(n, na, nb)
    w, U = np.linalg.eigh(O.hamiltonian_csr(h, g, V).toarray())
    for k in range(10):
        s2 = O.spin_square(V, U[:, k])
        S = (np.sqrt(1.0 + 4.0 * s2) - 1.0) / 2.0
        assert abs(2 * S - round(2 * S)) < 1e-8 and round(2 * S) % 2 == N % 2, (k, s2)
        S = round(2 * S) / 2
        a_top = int(round((N + 2 * S) / 2))  # the sector with M_s = S
        assert np.abs(spectra[a_top] - w[k]).min() < 1e-9, (k, S)
        if a_top + 1 in spectra:
            assert np.abs(spectra[a_top + 1] - w[k]).min() > 1e-7, (k, S)


def test_sign_convention_ties():
    """The first entry within 1e-6 (relative) of the largest magnitude is
    made positive: a near-tie resolves to the first index, a clear maximum
    decides by itself."""
    c = np.array([0.1, -0.5, 0.5 * (1 - 1e-9), 0.2])
    assert O._fix_sign(c)[1] > 0 and O._fix_sign(-c)[1] > 0
    c = np.array([0.1, -0.5, 0.5 + 1e-3, 0.2])
    assert O._fix_sign(c)[2] > 0 and O._fix_sign(-c)[2] > 0
