"""GPU parity of the HIP library against the CPU oracle on small spaces.

Every expected value comes from the oracle (or the seeded generator) on the
same inputs; tolerances: integer/index results bit-exact, float64 products
1e-12 relative to the largest entry, energies 1e-8 Ha, mixed-precision
products 1e-6 relative (float32 element rounding, 2^-24 per term).
"""
import ctypes

import numpy as np
import pytest
import torch

import hci_synth as hs
import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib_mod(gpu_available):
    import paper_1708_07544_amd as P
    return P


@pytest.fixture(scope="module")
def cas8(lib_mod):
    w = hs.WORKLOADS["cas8"]
    h, g = hs.workload_integrals(w)
    sp = hs.full_space(w.norb, w.nalpha, w.nbeta)
    e_ref, c_ref = O.lowest_eigenpair(h, g, sp)
    ctx = lib_mod.HCIContext(h, g, w.nalpha, w.nbeta)
    print(f"[cas8] n_det={len(sp)} e_ref={e_ref:.12f}", flush=True)
    return dict(w=w, h=h, g=g, sp=sp, e=e_ref, c=c_ref, ctx=ctx)


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_diagonal_cas8(cas8):
    ctx, h, g, sp = cas8["ctx"], cas8["h"], cas8["g"], cas8["sp"]
    d = ctx.diagonal(sp).cpu().numpy()
    ref = np.array([O.diag(h, g, x) for x in sp])
    assert np.abs(d - ref).max() < 1e-12


def test_connection_count_cas8(cas8):
    ctx, sp = cas8["ctx"], cas8["sp"]
    assert ctx.connections(sp) == int(O.row_counts(8, sp).sum())


@pytest.mark.parametrize("mode", ["stored", "recompute"])
def test_sigma_fp64_cas8(cas8, mode):
    ctx, h, g, sp = cas8["ctx"], cas8["h"], cas8["g"], cas8["sp"]
    c = hs.random_coeffs(len(sp), 3)
    ref = O.sigma(h, g, sp, c)
    out = ctx.sigma(sp, c, precision="fp64", mode=mode).cpu().numpy()
    assert rel_err(out, ref) < 1e-12


@pytest.mark.parametrize("mode", ["stored", "recompute"])
def test_sigma_mixed_cas8(cas8, mode):
    ctx, h, g, sp = cas8["ctx"], cas8["h"], cas8["g"], cas8["sp"]
    c = hs.random_coeffs(len(sp), 4)
    ref = O.sigma(h, g, sp, c)
    out = ctx.sigma(sp, c, precision="fp32_mixed", mode=mode).cpu().numpy()
    assert rel_err(out, ref) < 1e-6


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_davidson_cas8(cas8, precision):
    ctx, sp = cas8["ctx"], cas8["sp"]
    e, c, it = ctx.davidson(sp, None, tol=1e-10, precision=precision)
    print(f"[davidson {precision}] products={it} dE={e - cas8['e']:.3e}", flush=True)
    assert abs(e - cas8["e"]) < 1e-8
    c = c.cpu().numpy()
    assert abs(np.linalg.norm(c) - 1) < 1e-12
    assert np.abs(np.abs(c) - np.abs(cas8["c"])).max() < 1e-6
    assert abs(abs(c @ cas8["c"]) - 1.0) < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_davidson_scalars_by_stream_wait(cas8, monkeypatch, precision):
    """Each iteration's convergence scalars reach the host through pinned
    memory that the host polls; after the poll time (HCI_DAVIDSON_POLL_MS,
    0 here) it waits on the stream instead.  Both ways give the oracle's
    eigenpair and the same bytes."""
    ctx, sp = cas8["ctx"], cas8["sp"]
    e1, c1, it1 = ctx.davidson(sp, None, tol=1e-10, precision=precision)
    monkeypatch.setenv("HCI_DAVIDSON_POLL_MS", "0")
    e2, c2, it2 = ctx.davidson(sp, None, tol=1e-10, precision=precision)
    monkeypatch.delenv("HCI_DAVIDSON_POLL_MS", raising=False)
    print(f"[davidson wait {precision}] products {it1} / {it2}", flush=True)
    assert abs(e2 - cas8["e"]) < 1e-8
    assert e1 == e2 and it1 == it2
    assert torch.equal(c1, c2)


@pytest.mark.parametrize("n,na,nb,m,seed", [(8, 4, 4, 300, 1), (10, 3, 5, 700, 2), (12, 6, 6, 1500, 3),
                                           (7, 2, 0, 9, 4), (14, 7, 6, 64, 5)])
@pytest.mark.parametrize("eps", [0.0, 1e-4, 1e-2])
def test_select_bit_exact(lib_mod, n, na, nb, m, seed, eps):
    """Same (V, c) into both: V + C(eps) identical bit for bit."""
    h, g = hs.make_integrals(n, 3 * n, seed)
    V = hs.random_dets(n, na, nb, m, seed=seed, bias=0.2)
    c = hs.random_coeffs(len(V), seed + 100)
    ref = O.merge(V, O.select(h, g, V, c, eps))
    ctx = lib_mod.HCIContext(h, g, na, nb)
    out = lib_mod.dets_to_numpy(ctx.select(V, c, eps))
    print(f"[select n={n} m={len(V)} eps={eps}] ref={len(ref)} gpu={len(out)}", flush=True)
    assert out.shape == ref.shape
    assert np.array_equal(out, ref)


def test_hci_eps0_reaches_fci(cas8):
    """eps1 = 0 keeps every determinant reachable through a nonzero c_i.
    Determinants whose FCI amplitude vanishes by spin symmetry may stay out
    (their coupling to V is through c_i that are zero up to rounding), so the
    check is: the energy is the FCI energy and V holds every determinant of
    non-negligible FCI weight."""
    ctx = cas8["ctx"]
    V, c, e, hist = ctx.hci(0.0, tol=1e-10)
    assert abs(e - cas8["e"]) < 1e-8
    Vn = hs_sorted(V)
    have = {(int(a), int(b)) for a, b in Vn}
    full = {(int(a), int(b)) for a, b in cas8["sp"]}
    assert have <= full
    need = {(int(a), int(b)) for (a, b), x in zip(cas8["sp"], cas8["c"]) if abs(x) > 1e-8}
    assert need <= have


def hs_sorted(V):
    import paper_1708_07544_amd as P
    return P.dets_to_numpy(V)


def test_rdm_ground_state_cas8(cas8):
    ctx, sp, c = cas8["ctx"], cas8["sp"], cas8["c"]
    r1, r2 = ctx.rdm12(sp, c)
    o1, o2 = O.rdm12(8, sp, c, c)
    assert np.abs(r1.cpu().numpy() - o1).max() < 1e-12
    assert np.abs(r2.cpu().numpy() - o2).max() < 1e-12


def test_transition_rdm_small(lib_mod):
    n, na, nb = 6, 3, 2
    h, g = hs.make_integrals(n, 18, 7)
    sp = hs.full_space(n, na, nb)
    rng = np.random.default_rng(1)
    bra, ket = rng.normal(size=len(sp)), rng.normal(size=len(sp))
    ctx = lib_mod.HCIContext(h, g, na, nb)
    r1, r2 = ctx.rdm12(sp, bra, ket)
    o1, o2 = O.rdm12(n, sp, bra, ket)
    assert np.abs(r1.cpu().numpy() - o1).max() < 1e-11
    assert np.abs(r2.cpu().numpy() - o2).max() < 1e-11


def test_energy_backward_unrelaxed_cas8(cas8):
    ctx, sp, c, h, g = cas8["ctx"], cas8["sp"], cas8["c"], cas8["h"], cas8["g"]
    dh, dg, z, e2 = ctx.energy_backward(sp, c, cas8["e"], grad_e=2.0)
    o1, o2 = O.rdm12(8, sp, c, c)
    assert np.abs(dh.cpu().numpy() - 2.0 * o1).max() < 1e-11
    assert np.abs(dg.cpu().numpy() - 2.0 * 0.5 * O.symmetrize8(o2)).max() < 1e-11


def test_invalid_lists_are_rejected(cas8, lib_mod):
    ctx, sp = cas8["ctx"], cas8["sp"]
    bad = sp[::-1].copy()
    with pytest.raises(lib_mod.HCIError) as ei:
        ctx.sigma(bad, np.ones(len(bad)))
    assert ei.value.code == lib_mod._lib.HCI_E_ARG
    wrong = sp[:3].copy()
    wrong[1, 0] = np.uint64(0b111)  # 3 alpha electrons
    with pytest.raises(lib_mod.HCIError):
        ctx.sigma(wrong, np.ones(3))


def test_select_capacity_reports_required(cas8, lib_mod):
    ctx = cas8["ctx"]
    V = lib_mod.dets_to_device(hs.aufbau_det(4, 4))
    c = torch.ones(1, dtype=torch.float64, device="cuda")
    out = torch.empty((2, 2), dtype=torch.int64, device="cuda")
    n_out = ctypes.c_int64()
    L = lib_mod._lib
    code = L.lib().hci_select(ctx.handle, L._ptr(V), L._ptr(c), 1, 0.0, L._ptr(out), 2,
                              ctypes.byref(n_out), L._stream())
    assert code == L.HCI_E_CAPACITY
    assert n_out.value == 361


def test_select_capacity_retry_keeps_result(lib_mod):
    """A call refused for capacity keeps its result for the retry: the retry
    with room returns the oracle's V + C(eps) bit for bit, and a retry whose c
    changed in between (same buffer) selects from the new c."""
    n, na, nb, eps = 12, 5, 5, 2e-3
    h, g = hs.make_integrals(n, 3 * n, 21)
    V = hs.random_dets(n, na, nb, 300, seed=21, bias=0.2)
    c1 = hs.random_coeffs(len(V), 121)
    c2 = hs.random_coeffs(len(V), 122)
    ctx = lib_mod.HCIContext(h, g, na, nb)
    L = lib_mod._lib
    d = lib_mod.dets_to_device(V)
    cd = torch.as_tensor(c1, dtype=torch.float64, device="cuda").contiguous()
    n_out = ctypes.c_int64()

    def call(cap):
        out = torch.zeros((max(cap, 1), 2), dtype=torch.int64, device="cuda")
        code = L.lib().hci_select(ctx.handle, L._ptr(d), L._ptr(cd), len(V), eps, L._ptr(out), cap,
                                  ctypes.byref(n_out), L._stream())
        return code, out

    for c, change_to in [(c1, None), (c1, c2)]:
        cd.copy_(torch.as_tensor(c, dtype=torch.float64))
        code, _ = call(2)
        assert code == L.HCI_E_CAPACITY
        m = n_out.value
        if change_to is not None:
            cd.copy_(torch.as_tensor(change_to, dtype=torch.float64))
            c = change_to
        ref = O.merge(V, O.select(h, g, V, c, eps))
        code, out = call(max(m, len(ref)))
        assert code == L.HCI_OK
        got = lib_mod.dets_to_numpy(out[: n_out.value])
        print(f"[select retry] refused at 2, required {m}, retry gives {len(got)}, oracle {len(ref)}", flush=True)
        assert np.array_equal(got, ref)
    ctx.close()


def test_stored_matrix_rebuilds_agree(lib_mod):
    """The stored Hamiltonian built in several fresh contexts gives the
    oracle's product every time (guards against build-order dependence)."""
    w = hs.WORKLOADS["cas8"]
    h, g = hs.workload_integrals(w)
    sp = hs.full_space(8, 4, 4)
    c = hs.random_coeffs(len(sp), 11)
    ref = O.sigma(h, g, sp, c)
    for trial in range(4):
        ctx = lib_mod.HCIContext(h, g, 4, 4)
        for prec, tol in [("fp64", 1e-12), ("fp32_mixed", 1e-6)]:
            out = ctx.sigma(sp, c, precision=prec, mode="stored").cpu().numpy()
            assert rel_err(out, ref) < tol, (trial, prec)
        ctx.close()


@pytest.mark.parametrize("m", [1, 2, 63, 65, 257])
def test_ragged_sizes(lib_mod, m):
    n, na, nb = 9, 4, 3
    h, g = hs.make_integrals(n, 27, 9)
    V = hs.random_dets(n, na, nb, m, seed=m, bias=0.1)
    c = hs.random_coeffs(len(V), m)
    ctx = lib_mod.HCIContext(h, g, na, nb)
    for mode in ["stored", "recompute"]:
        out = ctx.sigma(V, c, mode=mode).cpu().numpy()
        assert rel_err(out, O.sigma(h, g, V, c)) < 1e-12
    assert ctx.connections(V) == int(O.row_counts(n, V).sum())
    r1, r2 = ctx.rdm12(V, c)
    o1, o2 = O.rdm12(n, V, c, c)
    assert np.abs(r1.cpu().numpy() - o1).max() < 1e-12
    assert np.abs(r2.cpu().numpy() - o2).max() < 1e-12


@pytest.mark.parametrize("cap", [1, 3])
def test_row_kernels_stride_over_a_clamped_grid(lib_mod, monkeypatch, cap):
    """One launch covers at most 2^32 work-items, so the row kernels of the
    selection walk, the connection count and the recomputed product stride
    over the rows of a clamped grid.  HCI_ROW_GRID_CAP forces the grid down
    to `cap` workgroups: every row is then reached through the stride."""
    monkeypatch.setenv("HCI_ROW_GRID_CAP", str(cap))
    n, na, nb = 12, 6, 5
    h, g = hs.make_integrals(n, 36, 12)
    V = hs.random_dets(n, na, nb, 3000, seed=12, bias=0.15)
    c = hs.random_coeffs(len(V), 77)
    ctx = lib_mod.HCIContext(h, g, na, nb)
    ref = O.sigma(h, g, V, c)
    for precision, tol in (("fp64", 1e-12), ("fp32_mixed", 1e-6)):
        out = ctx.sigma(V, c, precision=precision, mode="recompute").cpu().numpy()
        assert rel_err(out, ref) < tol, precision
    ctx.set_stage_window(0)  # plain layout: its count pass is a row kernel
    ctx.release_cache()
    assert ctx.connections(V) == int(O.row_counts(n, V).sum())
    sel = lib_mod.dets_to_numpy(ctx.select(V, c, 1e-3))
    assert np.array_equal(sel, O.merge(V, O.select(h, g, V, c, 1e-3)))
    ctx.close()


def _layout_space(name):
    if name == "cas8":
        w = hs.WORKLOADS["cas8"]
        h, g = hs.workload_integrals(w)
        return 8, 4, 4, h, g, hs.full_space(8, 4, 4)
    if name == "n12":
        h, g = hs.make_integrals(12, 36, 12)
        return 12, 6, 5, h, g, hs.random_dets(12, 6, 5, 3000, seed=12, bias=0.15)
    if name == "n52":
        h, g = hs.make_integrals(52, 60, 52)
        return 52, 3, 3, h, g, hs.random_dets(52, 3, 3, 2000, seed=52, bias=0.3)
    # (10e,10o) full space: stage lists of 6552 entries, more than 63
    # windows of 64, so the staged layout declines and plain CSR is used
    h, g = hs.make_integrals(10, 30, 10)
    return 10, 5, 5, h, g, hs.full_space(10, 5, 5)


@pytest.mark.parametrize("space,wlog", [("cas8", 0), ("cas8", 6), ("cas8", 8), ("cas8", 13),
                                        ("n12", 0), ("n12", 6), ("n12", 13), ("fci10", 6),
                                        ("n52", 6), ("n52", 13)])
def test_stored_layouts(lib_mod, space, wlog):
    """Plain CSR (window 0) and the alpha-bucket-staged layout at several
    window sizes (2^6 splits the stage lists into many windows) give the
    oracle's products in both precisions and the oracle's pair count.  n52
    (52 orbitals) takes the element pass's search for the stage range of a
    position (beta strings wider than 48 bits leave no room for its index)."""
    n, na, nb, h, g, V = _layout_space(space)
    c = hs.random_coeffs(len(V), 31)
    ref = O.sigma(h, g, V, c)
    ctx = lib_mod.HCIContext(h, g, na, nb)
    ctx.set_stage_window(wlog)
    print(f"[layout {space} |V|={len(V)} wlog={wlog}]", flush=True)
    assert ctx.connections(V) == int(O.row_counts(n, V).sum())
    for prec, tol in [("fp64", 1e-12), ("fp32_mixed", 1e-6), ("fp64", 1e-12)]:
        out = ctx.sigma(V, c, precision=prec, mode="stored").cpu().numpy()
        assert rel_err(out, ref) < tol, prec
    ctx.close()


@pytest.mark.parametrize("space,wlog", [("cas8", 6), ("n12", 6), ("n12", 13), ("cas16s", 14),
                                        ("n20", 12)])
def test_stored_layout_beta_maps_match_search(lib_mod, monkeypatch, space, wlog):
    """The alpha single x beta single connections are found through per-
    workgroup bitmaps of the neighbours' beta strings, or (HCI_AB_SEARCH=1,
    and for spaces with more than 65535 beta strings) by searching each
    neighbour bucket.  Both discover the same entries in the same order, so
    the stored layouts and the products agree bit for bit, and both match the
    oracle; the density matrices (same choice of path) agree to rounding.
    The recomputed product scans neighbour buckets or looks the rows' beta
    singles up in the same bitmaps (chosen per chunk by cost; HCI_AB_SEARCH=1
    forces the scan, HCI_RC_LOOKUP=1 the lookup): every path against the
    oracle."""
    if space == "cas16s":
        w = hs.WORKLOADS["cas16"]
        h, g = hs.workload_integrals(w)
        n, na, nb = 16, 8, 8
        V = hs.random_dets(16, 8, 8, 6000, seed=16, bias=0.2)
    elif space == "n20":
        # every pair of (aufbau, aufbau singles) strings of (20e,20o): the
        # aufbau beta string has 100 beta singles (more than one wavefront)
        h, g = hs.make_integrals(20, 60, 20)
        n, na, nb = 20, 10, 10
        base = (1 << 10) - 1
        strs = sorted({base} | {(base & ~(1 << i)) | (1 << a) for i in range(10) for a in range(10, 20)})
        V = np.array([(x, y) for x in strs for y in strs], dtype=np.uint64)
    else:
        n, na, nb, h, g, V = _layout_space(space)
    c = hs.random_coeffs(len(V), 32)
    ref = O.sigma(h, g, V, c)
    outs = {}
    for path in ["maps", "search", "lookup"]:
        if path == "search":
            monkeypatch.setenv("HCI_AB_SEARCH", "1")
        else:
            monkeypatch.delenv("HCI_AB_SEARCH", raising=False)
        if path == "lookup":  # the recomputed product looks every neighbour bucket up
            monkeypatch.setenv("HCI_RC_LOOKUP", "1")
        else:
            monkeypatch.delenv("HCI_RC_LOOKUP", raising=False)
        print(f"[beta maps {space} |V|={len(V)} wlog={wlog} {path}]", flush=True)
        ctx = lib_mod.HCIContext(h, g, na, nb)
        ctx.set_stage_window(wlog)
        assert ctx.layout_info(V)["layout"] == 2
        assert ctx.connections(V) == int(O.row_counts(n, V).sum())
        for prec in ["fp64", "fp32_mixed"]:
            outs[path, prec] = ctx.sigma(V, c, precision=prec, mode="stored").cpu().numpy()
            outs[path, "rc", prec] = ctx.sigma(V, c, precision=prec, mode="recompute").cpu().numpy()
        r1, r2 = ctx.rdm12(V, c)
        outs[path, "rdm"] = (r1.cpu().numpy(), r2.cpu().numpy())
        ctx.close()
    for prec, tol in [("fp64", 1e-12), ("fp32_mixed", 1e-6)]:
        assert np.array_equal(outs["maps", prec], outs["search", prec]), prec
        assert np.array_equal(outs["maps", prec], outs["lookup", prec]), prec
        assert rel_err(outs["maps", prec], ref) < tol, prec
        # recomputed product: neighbour buckets scanned (search) or looked up
        # (lookup), connections met in another order, so rounding only
        for path in ["maps", "search", "lookup"]:
            assert rel_err(outs[path, "rc", prec], ref) < tol, (path, prec)
    # density matrices: same pairs, met in another order (bitmap lookup or bucket scan)
    for k in range(2):
        a, b = outs["maps", "rdm"][k], outs["search", "rdm"][k]
        assert np.abs(a - b).max() <= 1e-12 * max(1.0, np.abs(b).max()), k
    if len(V) <= 5000:  # the oracle's density matrices take seconds here
        o1, o2 = O.rdm12(n, V, c, c)
        assert np.abs(outs["maps", "rdm"][0] - o1).max() < 1e-12
        assert np.abs(outs["maps", "rdm"][1] - o2).max() < 1e-12

def test_stage_window_rejects_bad_values(cas8, lib_mod):
    ctx = cas8["ctx"]
    for bad in [-1, 1, 5, 17]:
        assert lib_mod._lib.lib().hci_ctx_set_stage_window(ctx.handle, bad) == -1


@pytest.mark.parametrize("n,na,nb,m", [(20, 10, 9, 500), (24, 12, 12, 300), (44, 22, 22, 20)])
def test_rdm_larger_orbital_counts(lib_mod, n, na, nb, m):
    """Density matrices where the on-chip accumulators shrink or do not fit
    (n = 20: the same-spin spectator sums go straight into the private copies;
    n = 24 and 44: so do the alpha single x beta single tiles), against the
    oracle; a second call gives the same bytes."""
    h, g = hs.make_integrals(n, 3 * n, n)
    V = hs.random_dets(n, na, nb, m, seed=n, bias=0.1)
    bra = hs.random_coeffs(len(V), n)
    ket = hs.random_coeffs(len(V), n + 1)
    print(f"[rdm n={n} |V|={len(V)}]", flush=True)
    ctx = lib_mod.HCIContext(h, g, na, nb)
    r1, r2 = ctx.rdm12(V, bra, ket)
    o1, o2 = O.rdm12(n, V, bra, ket)
    assert np.abs(r1.cpu().numpy() - o1).max() < 1e-11
    assert np.abs(r2.cpu().numpy() - o2).max() < 1e-11
    s1, s2 = ctx.rdm12(V, bra, ket)
    assert s1.cpu().numpy().tobytes() == r1.cpu().numpy().tobytes()
    assert s2.cpu().numpy().tobytes() == r2.cpu().numpy().tobytes()
