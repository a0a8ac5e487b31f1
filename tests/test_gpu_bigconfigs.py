"""The (30e,30o) and porphyrin-shaped (44e,44o) workloads at full size.

The oracle selects V1 = aufbau + C(eps1) by the definition of the criterion
and gives the first-order amplitudes on it (c_0 = 1 on the aufbau
determinant, c_i = H_i0 / (H_00 - H_ii) elsewhere, normalised), which decay
like an HCI vector; they drive the library's selection of V2, a space of
millions of determinants, the size of these workloads' HCI spaces.  The
oracle cannot select V2 whole, so the output is checked by what it can
compute one by one:

* structure: sorted, unique, the right electron counts, V1 contained;
* no misses: for sampled rows i of V1, every determinant the oracle selects
  from D_i alone (its excitations by definition) is in V2;
* no false members: for sampled D_a in V2 outside V1, the oracle finds the
  members of V1 among D_a's excitations and one of them passes
  fl(|H_ai| |c_i|) > eps1;
* sigma = H c on V2 with recomputed connections (what the automatic mode
  picks at these sizes, whose stored Hamiltonians exceed the 64 GiB budget;
  asking for it directly skips the count pass that the automatic choice
  runs first), in both precisions, on sampled rows and the last rows
  against the oracle's row sums.

(30e,30o) selects V2 at its eps1 = 3e-5 (31.9 million determinants).  The
porphyrin-shaped (44e,44o) space has ten near-degenerate frontier orbitals,
so several first-order amplitudes are near 1/sqrt(2) (a converged state
spreads that weight): at eps1 = 1e-4 they would select over 10^9
determinants, beyond the 2^32 slots of the selection set (the library then
reports HCI_E_NOMEM).  At eps1 = 3e-4 they select 109.6 million: one
wavefront per row is then 7.0e9 work-items, more than the 32-bit grid size
of one dispatch (a launch that large once ran only part of its rows and
returned wrong products).  The row kernels of the selection walk, the
connection count and the recomputed product now stride over the rows of a
clamped grid; test_gpu_core.py checks the striding on small lists with the
grid forced down to a few workgroups, since a product over 109.6 million
rows takes minutes.  Here the selection is checked at 109.6 million and the
product at eps1 = 5e-4 (66.4 million, float32-mixed; float64 at 31.9
million rows above).
"""
import time

import numpy as np
import pytest

import hci_synth as hs
import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P(gpu_available):
    import paper_1708_07544_amd as P
    return P


def _selected(P, name, eps2_step):
    w = hs.WORKLOADS[name]
    h, g = hs.workload_integrals(w)
    V0 = hs.aufbau_det(w.nalpha, w.nbeta)
    V1 = O.merge(V0, O.select(h, g, V0, np.array([1.0]), w.eps1))
    i0 = int(O.find(V1, V0)[0])
    h00 = O.diag(h, g, V1[i0])
    c1 = np.array([1.0 if i == i0 else O.hij(h, g, V1[i0], V1[i]) / (h00 - O.diag(h, g, V1[i]))
                   for i in range(len(V1))])
    c1 /= np.linalg.norm(c1)
    print(f"[{name}] |V1|={len(V1)}, first-order amplitudes ready", flush=True)
    ctx = P.HCIContext(h, g, w.nalpha, w.nbeta)
    t = time.perf_counter()
    V2 = P.dets_to_numpy(ctx.select(V1, c1, eps2_step))
    print(f"[{name}] |V1|={len(V1)} |V2|={len(V2)} at eps1={eps2_step}: selection "
          f"{time.perf_counter() - t:.2f} s", flush=True)
    return w, h, g, V1, c1, V2, ctx, eps2_step


@pytest.fixture(scope="module")
def cas30(P):
    r = _selected(P, "cas30", hs.WORKLOADS["cas30"].eps1)
    yield r
    r[6].close()


@pytest.fixture(scope="module")
def cas44(P):
    r = _selected(P, "cas44", 3e-4)
    yield r
    r[6].close()


@pytest.fixture(scope="module")
def cas44_sigma(P):
    r = _selected(P, "cas44", 5e-4)
    yield r
    r[6].close()


def _check_selection(w, h, g, V1, c1, V2, eps, n_rows, n_members, seed):
    n = w.norb
    assert 2 * len(V1) < len(V2) < 400_000_000
    a, b = V2[:, 0], V2[:, 1]
    assert np.all((a[1:] > a[:-1]) | ((a[1:] == a[:-1]) & (b[1:] > b[:-1])))  # sorted and unique
    pa = np.array([bin(int(x)).count("1") for x in a[:: max(1, len(V2) // 20000)]])
    pb = np.array([bin(int(x)).count("1") for x in b[:: max(1, len(V2) // 20000)]])
    assert np.all(pa == w.nalpha) and np.all(pb == w.nbeta)
    assert np.all(O.find(V2, V1) >= 0)
    print(f"  structure checked on {len(V2)} determinants", flush=True)
    rng = np.random.default_rng(seed)
    # no misses from sampled rows (the lead determinant and the largest |c_i| included)
    rows = np.unique(np.concatenate([[int(np.argmax(np.abs(c1)))],
                                     rng.choice(len(V1), n_rows, replace=False)]))
    for i in rows:
        C = O.select(h, g, V1[i:i + 1], c1[i:i + 1], eps)
        if len(C):
            assert np.all(O.find(V2, C) >= 0), i
    print(f"  no misses from {len(rows)} sampled rows", flush=True)
    # no false members among sampled new determinants
    pick = rng.choice(len(V2), 8 * n_members, replace=False)
    new = pick[O.find(V1, V2[pick]) < 0][:n_members]
    assert len(new) == n_members
    for k in new:
        Da = V2[k]
        idx = O.find(V1, O.excitations(n, Da))
        idx = idx[idx >= 0]
        assert len(idx) > 0
        # largest |c_i| first: the first row that passes settles it
        passed = False
        for i in idx[np.argsort(-np.abs(c1[idx]), kind="stable")]:
            if abs(O.hij(h, g, V1[i], Da)) * abs(c1[i]) > eps:
                passed = True
                break
        assert passed, k
    print(f"  {n_members} sampled new determinants pass the criterion", flush=True)


def _check_sigma(P, ctx, h, g, V2, seed, n_rows, precisions=("fp64", "fp32_mixed")):
    c2 = hs.random_coeffs(len(V2), seed)
    rng = np.random.default_rng(seed)
    # sampled rows, the last rows of the list among them (the end of the grid)
    rows = np.unique(np.concatenate([rng.choice(len(V2), n_rows, replace=False),
                                     np.arange(len(V2) - 4, len(V2))]))
    ref = O.sigma(h, g, V2, c2, rows=rows)
    print(f"  oracle sigma on {len(rows)} rows", flush=True)
    scale = np.abs(ref).max()
    tols = {"fp64": 1e-12, "fp32_mixed": 1e-6}
    for precision in precisions:
        tol = tols[precision]
        t = time.perf_counter()
        out = ctx.sigma(V2, c2, precision=precision, mode="recompute").cpu().numpy()
        print(f"  sigma {precision} on {len(V2)} determinants: {time.perf_counter() - t:.2f} s, "
              f"max err {np.abs(out[rows] - ref).max() / scale:.2e}", flush=True)
        assert np.abs(out[rows] - ref).max() <= tol * scale, precision


def test_cas30_full_size_selection(cas30):
    w, h, g, V1, c1, V2, ctx, eps = cas30
    _check_selection(w, h, g, V1, c1, V2, eps, n_rows=24, n_members=64, seed=30)


def test_cas30_full_size_sigma_sampled_rows(P, cas30):
    w, h, g, V1, c1, V2, ctx, eps = cas30
    _check_sigma(P, ctx, h, g, V2, 31, 200)


def test_cas44_full_size_selection(cas44):
    w, h, g, V1, c1, V2, ctx, eps = cas44
    _check_selection(w, h, g, V1, c1, V2, eps, n_rows=16, n_members=32, seed=44)


def test_cas44_full_size_sigma_sampled_rows(P, cas44_sigma):
    w, h, g, V1, c1, V2, ctx, eps = cas44_sigma
    _check_sigma(P, ctx, h, g, V2, 45, 100, precisions=("fp32_mixed",))

