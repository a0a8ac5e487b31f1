"""Pins of the CPU oracle against what the physics and the paper fix.

No GPU here.  Each test checks the oracle against something other than
itself: closed forms, textbook reductions (one- and two-electron problems),
an independent second-quantised construction of H, brute force over the
whole determinant space, variational and density-matrix identities, and
finite differences.  A plausible slip in a sign, an index or a dropped term
of the Slater-Condon rules, the selection criterion or the density
matrices fails at least one of them.
"""
import itertools

import numpy as np
import pytest

import hci_synth as hs
import oracle as O


def small_integrals(n, seed, L=None):
    return hs.make_integrals(n, L or 3 * n, seed)


# ------------------------------------------------------------ Hamiltonian
@pytest.mark.parametrize("n,na,nb,seed", [(5, 2, 2, 0), (6, 3, 2, 1), (6, 2, 0, 2), (5, 1, 3, 3),
                                          (4, 4, 1, 4)])
def test_slater_condon_matches_operator_definition(n, na, nb, seed):
    """Method (ii) (rules) == method (i) (apply every operator term) on a full space."""
    h, g = small_integrals(n, seed)
    sp = hs.full_space(n, na, nb)
    H_op = O.hamiltonian_by_operators(h, g, sp)
    H_sc = O.hamiltonian_csr(h, g, sp).toarray()
    assert np.abs(H_op - H_sc).max() < 1e-12
    assert np.abs(H_op - H_op.T).max() < 1e-12


def test_slater_condon_spot_pairs_larger_space():
    """Random connected pairs in (5a,4b) of 10 orbitals: rules vs operators."""
    n = 10
    h, g = small_integrals(n, 7)
    rng = np.random.default_rng(0)
    dets = hs.random_dets(n, 5, 4, 40, seed=3, bias=0.05)
    for d in dets[:25]:
        amp = O.apply_h(h, g, d)
        exc = O.excitations(n, d)
        pick = rng.choice(len(exc), 30, replace=False)
        for k in pick:
            key = (int(exc[k, 0]), int(exc[k, 1]))
            assert abs(O.hij(h, g, d, exc[k]) - amp.get(key, 0.0)) < 1e-12
        assert abs(O.diag(h, g, d) - amp[(int(d[0]), int(d[1]))]) < 1e-12


def test_noninteracting_closed_form():
    """g = 0: E0 = sum of the lowest nalpha + lowest nbeta eigenvalues of h."""
    n, na, nb = 6, 3, 2
    h, _ = small_integrals(n, 11)
    g = np.zeros((n, n, n, n))
    e0, _ = O.lowest_eigenpair(h, g, hs.full_space(n, na, nb))
    w = np.linalg.eigvalsh(h)
    assert abs(e0 - (w[:na].sum() + w[:nb].sum())) < 1e-11


def test_two_electrons_opposite_spin_first_quantised():
    """1 alpha + 1 beta: H[(p,q),(r,s)] = h_pr d_qs + d_pr h_qs + (pr|qs)."""
    n = 6
    h, g = small_integrals(n, 12)
    H = np.zeros((n * n, n * n))
    for p, q, r, s in itertools.product(range(n), repeat=4):
        H[p * n + q, r * n + s] = h[p, r] * (q == s) + (p == r) * h[q, s] + g[p, r, q, s]
    ref = np.linalg.eigvalsh(H)
    e = np.linalg.eigvalsh(O.hamiltonian_csr(h, g, hs.full_space(n, 1, 1)).toarray())
    assert np.abs(np.sort(e) - np.sort(ref)).max() < 1e-11


def test_two_electrons_same_spin_first_quantised():
    """2 alpha: antisymmetrised pairs p<q with <pq||rs> = (pr|qs) - (ps|qr)."""
    n = 6
    h, g = small_integrals(n, 13)
    pairs = [(p, q) for p in range(n) for q in range(p + 1, n)]
    m = len(pairs)
    H = np.zeros((m, m))
    for a, (p, q) in enumerate(pairs):
        for b, (r, s) in enumerate(pairs):
            H[a, b] = (h[p, r] * (q == s) + h[q, s] * (p == r) - h[p, s] * (q == r)
                       - h[q, r] * (p == s) + g[p, r, q, s] - g[p, s, q, r])
    ref = np.linalg.eigvalsh(H)
    e = np.linalg.eigvalsh(O.hamiltonian_csr(h, g, hs.full_space(n, 2, 0)).toarray())
    assert np.abs(np.sort(e) - np.sort(ref)).max() < 1e-11


def test_hubbard_dimer_closed_form():
    t, U = 0.7, 2.3
    h = np.array([[0.0, -t], [-t, 0.0]])
    g = np.zeros((2, 2, 2, 2))
    g[0, 0, 0, 0] = g[1, 1, 1, 1] = U
    e0, _ = O.lowest_eigenpair(h, g, hs.full_space(2, 1, 1))
    assert abs(e0 - (U - np.sqrt(U * U + 16 * t * t)) / 2) < 1e-13


def test_excitation_enumeration_counts():
    """Singles + doubles of one determinant: the combinatorial count, all distinct."""
    n, na, nb = 9, 4, 3
    d = hs.random_dets(n, na, nb, 1, seed=1, include_aufbau=True)[0]
    exc = O.excitations(n, d)
    va, vb = n - na, n - nb
    expect = (na * va + nb * vb + (na * (na - 1) // 2) * (va * (va - 1) // 2)
              + (nb * (nb - 1) // 2) * (vb * (vb - 1) // 2) + na * va * nb * vb)
    assert len(exc) == expect
    assert len(O.sort_unique(exc)) == expect
    for x in exc:
        deg = (bin(int(x[0]) ^ int(d[0])).count("1") + bin(int(x[1]) ^ int(d[1])).count("1")) // 2
        assert deg in (1, 2)


# ------------------------------------------------------------ selection
@pytest.mark.parametrize("eps", [0.0, 1e-3, 3e-2, 0.2])
def test_selection_definition_matches_bruteforce(eps):
    """Enumerating excitations of V == max_i |H_ai c_i| > eps over the whole space."""
    n, na, nb = 6, 3, 3
    h, g = small_integrals(n, 21)
    space = hs.full_space(n, na, nb)
    V = hs.random_dets(n, na, nb, 25, seed=5, bias=0.3)
    c = hs.random_coeffs(len(V), seed=6)
    a = O.select(h, g, V, c, eps)
    b = O.select_bruteforce(h, g, V, c, eps, space)
    assert a.shape == b.shape and np.array_equal(a, b)


def test_selection_threshold_is_strict():
    """A determinant whose |H_ai c_i| equals eps exactly is not selected."""
    n = 4
    h, g = small_integrals(n, 22)
    V = hs.aufbau_det(2, 2)
    c = np.array([1.0])
    exc = O.excitations(n, V[0])
    vals = np.array([abs(O.hij(h, g, V[0], x)) for x in exc])
    k = int(np.argmax(vals))
    sel = O.select(h, g, V, c, float(vals[k]))
    keys = {(int(x[0]), int(x[1])) for x in sel}
    assert (int(exc[k, 0]), int(exc[k, 1])) not in keys
    sel2 = O.select(h, g, V, c, float(np.nextafter(vals[k], 0)))
    assert (int(exc[k, 0]), int(exc[k, 1])) in {(int(x[0]), int(x[1])) for x in sel2}


def test_hci_eps0_reaches_fci_cas8():
    """eps1 = 0 grows V over every determinant of non-negligible FCI weight
    (those of zero weight by spin symmetry are reached, or not, through
    rounding-level c_i) and E to the dense FCI energy."""
    w = hs.WORKLOADS["cas8"]
    h, g = hs.workload_integrals(w)
    V, c, e, hist = O.hci(h, g, w.nalpha, w.nbeta, 0.0)
    sp = hs.full_space(8, 4, 4)
    H = O.hamiltonian_csr(h, g, sp).toarray()
    w_, U = np.linalg.eigh(H)
    assert abs(e - w_[0]) < 1e-10
    need = sp[np.abs(U[:, 0]) > 1e-8]
    assert np.all(O.find(V, need) >= 0)
    es = [x[1] for x in hist]
    assert all(es[k + 1] <= es[k] + 1e-12 for k in range(len(es) - 1))


def test_variational_energy_monotone_in_nested_eps1():
    """A decreasing eps1 schedule, each run started from the previous V,
    gives non-increasing energies, all above FCI (variational bound)."""
    n, na, nb = 8, 4, 4
    h, g = hs.make_integrals(n, 24, 0)
    e_fci = np.linalg.eigvalsh(O.hamiltonian_csr(h, g, hs.full_space(n, na, nb)).toarray())[0]
    V = None
    prev = np.inf
    for eps in [3e-1, 1e-1, 3e-2, 1e-2, 3e-3]:
        V, c, e, _ = O.hci(h, g, na, nb, eps, V0=V)
        assert e <= prev + 1e-12
        assert e >= e_fci - 1e-10
        prev = e


# ------------------------------------------------------------ density matrices
@pytest.fixture(scope="module")
def cas6_state():
    n, na, nb = 6, 3, 3
    h, g = small_integrals(n, 31)
    sp = hs.full_space(n, na, nb)
    e, c = O.lowest_eigenpair(h, g, sp)
    r1, r2 = O.rdm12(n, sp, c, c)
    return n, na + nb, h, g, sp, e, c, r1, r2


def test_rdm_traces_and_partial_trace(cas6_state):
    n, N, h, g, sp, e, c, r1, r2 = cas6_state
    assert abs(np.trace(r1) - N) < 1e-12
    assert abs(np.einsum("pprr->", r2) - N * (N - 1)) < 1e-11
    assert np.abs(np.einsum("pqrr->pq", r2) - (N - 1) * r1).max() < 1e-11


def test_rdm_symmetries_and_bounds(cas6_state):
    n, N, h, g, sp, e, c, r1, r2 = cas6_state
    assert np.abs(r2 - r2.transpose(2, 3, 0, 1)).max() < 1e-12
    assert np.abs(r2 - r2.transpose(1, 0, 3, 2)).max() < 1e-12
    w = np.linalg.eigvalsh(r1)
    assert w.min() > -1e-12 and w.max() < 2 + 1e-12


def test_energy_from_rdms(cas6_state):
    n, N, h, g, sp, e, c, r1, r2 = cas6_state
    assert abs(O.energy_from_rdms(h, g, r1, r2) - e) < 1e-10


def test_transition_rdm_contracts_to_matrix_element(cas6_state):
    """<bra|H|ket> = sum h gamma(bra,ket) + 1/2 sum g Gamma(bra,ket)."""
    n, N, h, g, sp, e, c, r1, r2 = cas6_state
    rng = np.random.default_rng(3)
    bra, ket = rng.normal(size=len(sp)), rng.normal(size=len(sp))
    t1, t2 = O.rdm12(n, sp, bra, ket)
    H = O.hamiltonian_by_operators(h, g, sp)
    assert abs(bra @ H @ ket - O.energy_from_rdms(h, g, t1, t2)) < 1e-10
    # the rdm of (ket, bra) is the index-reversed one of (bra, ket)
    s1, s2 = O.rdm12(n, sp, ket, bra)
    assert np.abs(s1 - t1.T).max() < 1e-12
    assert np.abs(s2 - t2.transpose(1, 0, 3, 2)).max() < 1e-12


def test_rdm_element_matches_full(cas6_state):
    n, N, h, g, sp, e, c, r1, r2 = cas6_state
    for (p, q, r, s) in [(0, 1, 2, 3), (1, 1, 2, 2), (3, 0, 0, 3), (5, 4, 2, 1)]:
        assert abs(O.rdm2_element(n, sp, c, c, p, q, r, s) - r2[p, q, r, s]) < 1e-12
    for (p, q) in [(0, 0), (1, 4), (5, 2)]:
        assert abs(O.rdm1_element(n, sp, c, c, p, q) - r1[p, q]) < 1e-12


def test_hellmann_feynman_finite_differences(cas6_state):
    """dE/dh_pq (h_pq and h_qp moved together) = 2 gamma_pq; dE/d(orbit of g)
    = orbit size * 1/2 Gamma^sym: central differences, step 1e-5."""
    n, N, h, g, sp, e, c, r1, r2 = cas6_state
    step = 1e-5
    gsym = O.symmetrize8(r2)

    def energy(hh, gg):
        return O.lowest_eigenpair(hh, gg, sp)[0]

    for (p, q) in [(0, 1), (2, 2), (4, 1)]:
        dh = np.zeros_like(h)
        dh[p, q] += step
        if p != q:
            dh[q, p] += step
        fd = (energy(h + dh, g) - energy(h - dh, g)) / (2 * step)
        ana = (2 if p != q else 1) * r1[p, q]
        assert abs(fd - ana) < 1e-6
    for idx in [(0, 1, 2, 3), (1, 1, 0, 0), (2, 3, 2, 3), (5, 5, 5, 5)]:
        orbit = {tuple(np.array(idx)[list(pm)]) for pm in
                 [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2), (2, 3, 0, 1),
                  (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]}
        dg = np.zeros_like(g)
        for o in orbit:
            dg[o] = step
        fd = (energy(h, g + dg) - energy(h, g - dg)) / (2 * step)
        ana = len(orbit) * 0.5 * gsym[idx]
        assert abs(fd - ana) < 1e-6


def test_sigma_matches_operator_matrix():
    n, na, nb = 6, 2, 3
    h, g = small_integrals(n, 41)
    sp = hs.full_space(n, na, nb)
    V = sp[::3].copy()
    c = hs.random_coeffs(len(V), 9)
    H = O.hamiltonian_by_operators(h, g, V)
    assert np.abs(O.sigma(h, g, V, c) - H @ c).max() < 1e-12
    rows = np.array([0, 5, len(V) - 1])
    assert np.abs(O.sigma(h, g, V, c, rows) - (H @ c)[rows]).max() < 1e-12


def test_golden_cas8_values():
    """Stored oracle output (tests/golden/cas8.json, written by
    tests/golden/make_golden.py which calls only the oracle)."""
    import json
    import os
    here = os.path.join(os.path.dirname(__file__), "golden", "cas8.json")
    ref = json.load(open(here))
    w = hs.WORKLOADS["cas8"]
    h, g = hs.workload_integrals(w)
    sp = hs.full_space(8, 4, 4)
    e, c = O.lowest_eigenpair(h, g, sp)
    assert abs(e - ref["e_fci"]) < 1e-10
    assert int(O.row_counts(8, sp).sum()) == ref["nnz"]
