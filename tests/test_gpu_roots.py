"""Several states of one space, and unequal spin projections, against the oracle.

* hci_davidson_roots: energies of the lowest states (1e-9 Ha, residual
  tolerance 1e-10) and eigenvectors (1e-6 per entry, the residual over the
  gap to the neighbouring states) of (8e,8o) and (5a,3b) full spaces and a
  (16e,16o) HCI space, in both precisions, from zero and from warm starts;
  the whole spectrum of a four-determinant space; one state equals
  hci_davidson; argument errors.
* A spin check through the library: the lowest M_s = 1 energies are
  M_s = 0 states (other components of the same multiplets).
* hci_select_roots: identical bit for bit to the oracle's union of
  single-state selections.
"""
import numpy as np
import pytest

import hci_synth as hs
import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P(gpu_available):
    import paper_1708_07544_amd as P
    return P


def _space(name):
    if name == "cas8":
        h, g = hs.workload_integrals(hs.WORKLOADS["cas8"])
        return h, g, 4, 4, hs.full_space(8, 4, 4)
    if name == "ms1":
        h, g = hs.workload_integrals(hs.WORKLOADS["cas8"])
        return h, g, 5, 3, hs.full_space(8, 5, 3)
    h, g = hs.workload_integrals(hs.WORKLOADS["cas16"])
    V0 = hs.aufbau_det(8, 8)
    return h, g, 8, 8, O.merge(V0, O.select(h, g, V0, np.array([1.0]), 5e-2))


def _check_states(e, C, eref, Cref, tol_e=1e-9, tol_c=1e-6):
    """Energies; vectors up to sign (against another solver, whose rounding
    may place an entry just inside or outside the tie band); the sign
    convention on the library's own vectors: the first entry within 1e-6
    (relative) of the largest |c_i| is positive."""
    k = len(eref)
    assert np.abs(e - eref).max() < tol_e, (e, eref)
    assert np.abs(C @ C.T - np.eye(k)).max() < 1e-10
    for r in range(k):
        d = min(np.abs(C[r] - Cref[r]).max(), np.abs(C[r] + Cref[r]).max())
        assert d < tol_c, (r, d)
        a = np.abs(C[r])
        assert C[r][int(np.flatnonzero(a >= a.max() * (1 - 1e-6))[0])] > 0


@pytest.mark.parametrize("name,k,precision", [("cas8", 4, "fp64"), ("cas8", 4, "fp32_mixed"),
                                              ("ms1", 3, "fp64"), ("ms1", 3, "fp32_mixed"),
                                              ("cas16", 3, "fp32_mixed")])
def test_roots_match_oracle(P, name, k, precision):
    h, g, na, nb, V = _space(name)
    eref, Cref = O.lowest_eigenpairs(h, g, V, k + 1)
    assert np.diff(eref).min() > 1e-4  # states separated: vectors compare one by one
    eref, Cref = eref[:k], Cref[:k]
    print(f"[roots {name} |V|={len(V)} k={k} {precision}]", flush=True)
    ctx = P.HCIContext(h, g, na, nb)
    e, C, its = ctx.davidson_roots(V, k, tol=1e-10, precision=precision)
    print(f"  E={e} products={its}", flush=True)
    _check_states(e, C.cpu().numpy(), eref, Cref)
    # warm start from perturbed reference vectors: same states, fewer products
    rng = np.random.default_rng(5)
    C0 = Cref + 1e-4 * rng.normal(size=Cref.shape)
    e2, C2, its2 = ctx.davidson_roots(V, k, c0=C0, tol=1e-10, precision=precision)
    _check_states(e2, C2.cpu().numpy(), eref, Cref)
    assert sum(its2) <= sum(its)
    ctx.close()


def test_ms1_states_are_ms0_states(P):
    """Spin symmetry through the library: each of the three lowest M_s = 1
    energies equals one of the M_s = 0 states (the other component of the
    same multiplet; which one is read from the oracle's full spectrum)."""
    h, g = hs.workload_integrals(hs.WORKLOADS["cas8"])
    V1 = hs.full_space(8, 5, 3)
    V0 = hs.full_space(8, 4, 4)
    full0 = np.linalg.eigvalsh(O.hamiltonian_csr(h, g, V0).toarray())
    e1ref, _ = O.lowest_eigenpairs(h, g, V1, 3)
    idx = [int(np.argmin(np.abs(full0 - x))) for x in e1ref]
    assert max(abs(full0[i] - x) for i, x in zip(idx, e1ref)) < 1e-9 and max(idx) < 8
    c1 = P.HCIContext(h, g, 5, 3)
    e1, _, _ = c1.davidson_roots(V1, 3, tol=1e-10)
    c1.close()
    c0 = P.HCIContext(h, g, 4, 4)
    e0, _, _ = c0.davidson_roots(V0, max(idx) + 1, tol=1e-10)
    c0.close()
    print(f"[Ms=1 in Ms=0] {e1} at {idx} of {e0}", flush=True)
    for i, x in zip(idx, e1):
        assert abs(e0[i] - x) < 1e-9


def test_roots_whole_spectrum_and_single_state(P):
    h, g = hs.make_integrals(4, 12, 3)
    V = hs.full_space(4, 1, 1)[:4]  # four determinants
    eref = np.linalg.eigvalsh(O.hamiltonian_by_operators(h, g, V))
    ctx = P.HCIContext(h, g, 1, 1)
    e, C, _ = ctx.davidson_roots(V, 4, tol=1e-12)
    assert np.abs(e - eref).max() < 1e-12
    Cn = C.cpu().numpy()
    assert np.abs(Cn @ Cn.T - np.eye(4)).max() < 1e-12
    # one state is the state of hci_davidson
    hb, gb = hs.workload_integrals(hs.WORKLOADS["cas8"])
    Vb = hs.full_space(8, 4, 4)
    cb = P.HCIContext(hb, gb, 4, 4)
    e1, c1, it1 = cb.davidson(Vb, None, tol=1e-10)
    er, Cr, itr = cb.davidson_roots(Vb, 1, tol=1e-10)
    assert abs(er[0] - e1) < 1e-10
    # the largest entries of this S = 4 state come in pairs of equal
    # magnitude; the sign convention takes the first entry of the tie band,
    # so both solves return the same signed vector
    d = float((Cr[0] - c1).abs().max())
    assert d < 1e-7, d
    # a start row inside the span of the earlier states falls back to a seed
    C0 = np.zeros((2, len(Vb)))
    C0[0] = c1.cpu().numpy()
    C0[1] = c1.cpu().numpy()
    eref2, Cref2 = O.lowest_eigenpairs(hb, gb, Vb, 2)
    e2, C2, _ = cb.davidson_roots(Vb, 2, c0=C0, tol=1e-10)
    _check_states(e2, C2.cpu().numpy(), eref2, Cref2)
    cb.close()
    ctx.close()


def test_roots_rejects_bad_arguments(P):
    h, g = hs.make_integrals(4, 12, 3)
    V = hs.full_space(4, 1, 1)[:4]
    ctx = P.HCIContext(h, g, 1, 1)
    for k in (0, 5):
        with pytest.raises(P.HCIError) as ei:
            ctx.davidson_roots(V, k)
        assert ei.value.code == -1, k
    h8, g8 = hs.workload_integrals(hs.WORKLOADS["cas8"])
    c8 = P.HCIContext(h8, g8, 4, 4)
    with pytest.raises(P.HCIError) as ei:
        c8.davidson_roots(hs.full_space(8, 4, 4), 32)
    assert ei.value.code == -1
    with pytest.raises(P.HCIError) as ei:
        c8.select(hs.full_space(8, 4, 4)[:40], np.ones((32, 40)), 1e-3)
    assert ei.value.code == -1
    c8.close()
    ctx.close()


@pytest.mark.parametrize("n,na,nb,m,nroots,seed", [(10, 3, 5, 500, 3, 2), (12, 6, 6, 1200, 4, 3),
                                                   (14, 7, 6, 64, 2, 5)])
@pytest.mark.parametrize("eps", [1e-4, 1e-2])
def test_select_roots_bit_exact(P, n, na, nb, m, nroots, seed, eps):
    h, g = hs.make_integrals(n, 3 * n, seed)
    V = hs.random_dets(n, na, nb, m, seed=seed, bias=0.2)
    C = np.stack([hs.random_coeffs(len(V), seed + 100 + r) for r in range(nroots)])
    C[-1] = C[0]  # a repeated state changes nothing
    ref = O.merge(V, O.select_roots(h, g, V, C, eps))
    ctx = P.HCIContext(h, g, na, nb)
    out = P.dets_to_numpy(ctx.select(V, C, eps))
    print(f"[select_roots n={n} m={len(V)} k={nroots} eps={eps}] ref={len(ref)} gpu={len(out)}", flush=True)
    assert np.array_equal(out, ref)
    one = P.dets_to_numpy(ctx.select(V, C[:1], eps))
    assert np.array_equal(one, P.dets_to_numpy(ctx.select(V, C[0], eps)))
    ctx.close()


@pytest.mark.parametrize("na,nb", [(4, 4), (5, 3)])
def test_hci_several_states_matches_oracle(P, na, nb):
    """The several-state variational stage (union selection, deflated
    Davidson, warm starts carried by hci_embed) against the oracle's loop:
    the same determinant lists at every step and the same energies.  With
    N_alpha = N_beta the selected spaces are closed under the exchange of
    alpha and beta strings and the warm starts have a definite parity under
    it that the next space's states do not share (at 1927 determinants the
    starts are odd, even, even and the lowest states even, odd, odd): the
    case that needs the symmetry-breaking start of the several-state
    solver."""
    h, g = hs.workload_integrals(hs.WORKLOADS["cas8"])
    a = hs.aufbau_det(na, nb)
    V0 = O.merge(a, O.select(h, g, a, np.array([1.0]), 0.2))
    Vr, Cr, er, hr = O.hci_roots(h, g, na, nb, 3e-2, 3, V0)
    ctx = P.HCIContext(h, g, na, nb)
    V, C, e, hist = ctx.hci(3e-2, nroots=3, dets0=V0, tol=1e-10)
    ctx.close()
    print(f"[hci roots {na},{nb}] sizes {[x[0] for x in hist]} vs {[x[0] for x in hr]}: {e} vs {er}", flush=True)
    assert [x[0] for x in hist] == [x[0] for x in hr]
    assert np.array_equal(P.dets_to_numpy(V), Vr)
    assert np.abs(e - er).max() < 1e-9


@pytest.mark.parametrize("case", ["cas8", "ms1", "random12", "random20", "hand"])
def test_spin_square_matches_oracle(P, case):
    """<S^2> through the library against the oracle on the same vectors:
    eigenstates of full spaces (where it is S(S+1) exactly), random lists
    with random vectors (N_alpha != N_beta included, 50,000 determinants of
    20 orbitals), hand cases; a zero vector is an argument error."""
    if case in ("cas8", "ms1"):
        h, g, na, nb, V = _space(case)
        e, C = O.lowest_eigenpairs(h, g, V, 4)
        vecs = list(C)
    elif case == "hand":
        h, g = hs.make_integrals(4, 12, 1)
        na, nb = 1, 1
        V = O.sort_unique(np.array([[hs.det_bits([0]), hs.det_bits([1])],
                                    [hs.det_bits([1]), hs.det_bits([0])],
                                    [hs.det_bits([2]), hs.det_bits([2])]], dtype=np.uint64))
        vecs = [np.array([1.0, 1.0, 0.0]), np.array([1.0, -1.0, 0.0]), np.array([0.0, 0.0, 2.0]),
                np.array([0.3, -0.2, 0.9])]
    else:
        n, na, nb, m = (12, 6, 5, 3000) if case == "random12" else (20, 10, 10, 50_000)
        h, g = hs.make_integrals(n, 3 * n, n)
        V = hs.random_dets(n, na, nb, m, seed=n, bias=0.1)
        vecs = [hs.random_coeffs(len(V), 90 + k) for k in range(2)]
    ctx = P.HCIContext(h, g, na, nb)
    for k, c in enumerate(vecs):
        got = ctx.spin_square(V, c)
        ref = O.spin_square(V, c)
        print(f"[S^2 {case} {k}] {got:.12f} oracle {ref:.12f}", flush=True)
        assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (got, ref)
        if case in ("cas8", "ms1"):
            S = (np.sqrt(1.0 + 4.0 * got) - 1.0) / 2.0
            assert abs(S - round(S)) < 1e-8
    with pytest.raises(P.HCIError) as ei:
        ctx.spin_square(V, np.zeros(len(V)))
    assert ei.value.code == -1
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_roots_at_the_largest_count(P, precision):
    """HCI_MAX_ROOTS = 31 states of a 60-determinant space: the last solves
    deflate 30 locked vectors and work in complements of a few dimensions."""
    n, na, nb = 6, 2, 2
    h, g = hs.make_integrals(n, 18, 21)
    V = hs.random_dets(n, na, nb, 60, seed=21, bias=0.0)
    ref = np.linalg.eigvalsh(O.hamiltonian_by_operators(h, g, V))
    ctx = P.HCIContext(h, g, na, nb)
    e, C, its = ctx.davidson_roots(V, 31, tol=1e-10, precision=precision)
    ctx.close()
    Cn = C.cpu().numpy()
    print(f"[31 roots {precision}] |V|={len(V)} max dE {np.abs(e - ref[:31]).max():.2e}", flush=True)
    assert np.abs(e - ref[:31]).max() < 1e-9
    assert np.abs(Cn @ Cn.T - np.eye(31)).max() < 1e-9


def test_spin_square_without_beta_electrons(P):
    """N_beta = 0: S_+ has no images and <S^2> = S_z (S_z + 1) exactly."""
    n, na, nb = 7, 3, 0
    h, g = hs.make_integrals(n, 21, 4)
    V = hs.full_space(n, na, nb)
    c = hs.random_coeffs(len(V), 5)
    ctx = P.HCIContext(h, g, na, nb)
    assert ctx.spin_square(V, c) == 1.5 * 2.5 == O.spin_square(V, c)
    ctx.close()
