"""Pins of the oracle's eps2-screened PT2, z-vector and relaxed gradient.

E2 is checked against a dense Epstein-Nesbet evaluation with the
operator-built Hamiltonian; r = dE2/dc against finite differences in c; the
relaxed density matrices against central finite differences of the total
energy E0 + E2 with V, C(eps2) and the screening mask frozen (eq. lambda).
"""
import numpy as np
import pytest

import hci_synth as hs
import oracle as O


@pytest.fixture(scope="module")
def state():
    n, na, nb = 6, 3, 3
    h, g = hs.make_integrals(n, 18, 31)
    V = hs.random_dets(n, na, nb, 60, seed=2, bias=0.3)
    e0, c = O.lowest_eigenpair(h, g, V)
    eps2 = 1e-3
    pt = O.pt2(h, g, V, c, e0, eps2)
    return dict(n=n, h=h, g=g, V=V, e0=e0, c=c, eps2=eps2, pt=pt)


def test_e2_matches_dense_epstein_nesbet(state):
    s = state
    pt = s["pt"]
    full = O.merge(s["V"], pt["C"])
    Hf = O.hamiltonian_by_operators(s["h"], s["g"], full)
    iv, ic = O.find(full, s["V"]), O.find(full, pt["C"])
    HCV = Hf[np.ix_(ic, iv)]
    M = (np.abs(HCV) * np.abs(s["c"])[None, :]) > s["eps2"]
    N = (HCV * M) @ s["c"]
    E2 = np.sum(N ** 2 / (s["e0"] - np.diag(Hf)[ic]))
    assert abs(E2 - pt["E2"]) < 1e-12
    # eps2 = 0 keeps every connected determinant: the unscreened eq. pt
    pt0 = O.pt2(s["h"], s["g"], s["V"], s["c"], s["e0"], 0.0)
    full0 = O.merge(s["V"], pt0["C"])
    H0 = O.hamiltonian_by_operators(s["h"], s["g"], full0)
    iv0, ic0 = O.find(full0, s["V"]), O.find(full0, pt0["C"])
    N0 = H0[np.ix_(ic0, iv0)] @ s["c"]
    assert abs(np.sum(N0 ** 2 / (s["e0"] - np.diag(H0)[ic0])) - pt0["E2"]) < 1e-12


def test_hylleraas_stationary_at_d(state):
    """H[d] = sum d^2 (H_aa - E0) + 2 sum d N equals E2 at d and is stationary."""
    pt = state["pt"]
    d, N, Haa, e0 = pt["d"], pt["N"], pt["Haa"], state["e0"]

    def hyl(x):
        return float(np.sum(x * x * (Haa - e0)) + 2 * np.sum(x * N))

    assert abs(hyl(d) - pt["E2"]) < 1e-12
    grad = 2 * d * (Haa - e0) + 2 * N
    assert np.abs(grad).max() < 1e-12


def test_r_is_gradient_of_e2_in_c(state):
    s = state
    a, idx, hv, pos = s["pt"]["pairs"]
    C = s["pt"]["C"]
    Haa = s["pt"]["Haa"]

    def e2_of(c):
        N = np.zeros(len(C))
        np.add.at(N, pos, hv * c[idx])
        return float(np.sum(N ** 2 / (s["e0"] - Haa)))

    step = 1e-6
    for k in [0, 5, 17, len(s["V"]) - 1]:
        cp, cm = s["c"].copy(), s["c"].copy()
        cp[k] += step
        cm[k] -= step
        fd = (e2_of(cp) - e2_of(cm)) / (2 * step)
        assert abs(fd - s["pt"]["r"][k]) < 1e-7


def _frozen_total(h, g, V, pairs, C):
    """E0 + E2 with V, C and the screened pair list frozen."""
    a, idx, _, pos = pairs
    e0, c = O.lowest_eigenpair(h, g, V)
    hv = np.array([O.hij(h, g, V[i], a[k]) for k, i in enumerate(idx)])
    N = np.zeros(len(C))
    np.add.at(N, pos, hv * c[idx])
    Haa = np.array([O.diag(h, g, x) for x in C])
    return e0 + float(np.sum(N ** 2 / (e0 - Haa)))


def test_relaxed_gradient_finite_differences(state):
    s = state
    n, h, g, V, c, e0, pt = s["n"], s["h"], s["g"], s["V"], s["c"], s["e0"], s["pt"]
    H = O.hamiltonian_csr(h, g, V).toarray()
    z = O.zvector_dense(H, c, e0, pt["r"])
    assert abs(z @ c) < 1e-12
    Q = np.eye(len(c)) - np.outer(c, c)
    res = Q @ (H - e0 * np.eye(len(c))) @ Q @ z + Q @ pt["r"]
    assert np.linalg.norm(res) < 1e-10
    r1, r2 = O.relaxed_rdms(n, V, c, e0, z, pt)
    g8 = O.symmetrize8(r2)
    step = 1e-5
    for (p, q) in [(0, 1), (2, 2), (5, 3)]:
        dh = np.zeros_like(h)
        dh[p, q] += step
        if p != q:
            dh[q, p] += step
        fd = (_frozen_total(h + dh, g, V, pt["pairs"], pt["C"]) -
              _frozen_total(h - dh, g, V, pt["pairs"], pt["C"])) / (2 * step)
        ana = (2 if p != q else 1) * r1[p, q]
        assert abs(fd - ana) < 1e-6, (p, q, fd, ana)
    perms = [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2), (2, 3, 0, 1),
             (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]
    for idx in [(0, 1, 2, 3), (1, 1, 0, 0), (4, 2, 4, 2)]:
        orbit = {tuple(np.array(idx)[list(pm)]) for pm in perms}
        dg = np.zeros_like(g)
        for o in orbit:
            dg[o] = step
        fd = (_frozen_total(h, g + dg, V, pt["pairs"], pt["C"]) -
              _frozen_total(h, g - dg, V, pt["pairs"], pt["C"])) / (2 * step)
        ana = len(orbit) * 0.5 * g8[idx]
        assert abs(fd - ana) < 1e-6, (idx, fd, ana)


def test_unscreened_relaxation_is_nontrivial(state):
    """The z term matters: dropping it breaks the finite-difference match."""
    s = state
    n, h, g, V, c, e0, pt = s["n"], s["h"], s["g"], s["V"], s["c"], s["e0"], s["pt"]
    r1, _ = O.relaxed_rdms(n, V, c, e0, np.zeros_like(c), pt)
    dh = np.zeros_like(h)
    dh[0, 1] = dh[1, 0] = 1e-5
    fd = (_frozen_total(h + dh, g, V, pt["pairs"], pt["C"]) -
          _frozen_total(h - dh, g, V, pt["pairs"], pt["C"])) / 2e-5
    assert abs(fd - 2 * r1[0, 1]) > 1e-6
