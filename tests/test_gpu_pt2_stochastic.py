"""Semistochastic second-order energy (eq. semistoc) and the deterministic
screened E2 in several passes (its memory bottleneck), against the oracle.

The uniforms of every batch are drawn here and handed to both sides, so the
draws (integer cumulative weights) are identical and each batch is compared
value by value.  Tolerances: the per-pair arithmetic is the oracle's, the
sums run in another order, and S1^2 - S2 cancels when one draw dominates a
determinant a; 1e-10 relative to the batch value.
"""
import numpy as np
import pytest

import hci_synth as hs
import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib_mod(gpu_available):
    import paper_1708_07544_amd as P
    return P


def _space(name):
    if name == "cas8":
        w = hs.WORKLOADS["cas8"]
        h, g = hs.workload_integrals(w)
        n, na, nb = 8, 4, 4
        V0 = hs.aufbau_det(na, nb)
        V = O.merge(V0, O.select(h, g, V0, np.array([1.0]), 0.05))
        V = O.merge(V, O.select(h, g, V, np.ones(len(V)) / np.sqrt(len(V)), 0.05))
    elif name == "n10_53":  # N_alpha != N_beta
        n, na, nb = 10, 5, 3
        h, g = hs.make_integrals(n, 30, 10)
        V = hs.random_dets(n, na, nb, 400, seed=10, bias=0.25)
    else:  # (16e,16o): aufbau plus one selection (4,473 determinants)
        w = hs.WORKLOADS["cas16"]
        h, g = hs.workload_integrals(w)
        n, na, nb = 16, 8, 8
        V0 = hs.aufbau_det(na, nb)
        V = O.merge(V0, O.select(h, g, V0, np.array([1.0]), 5e-2))
    e0, c = O.lowest_eigenpair(h, g, V)
    return n, na, nb, h, g, V, e0, c


# (eps2, eps2_d) per space: the (16e,16o) thresholds keep the oracle's pair
# lists at ~1.6 M pairs
EPS = {"cas8": (1e-5, 1e-3), "n10_53": (1e-5, 1e-3), "cas16": (3e-3, 1e-2)}


@pytest.fixture(scope="module", params=["cas8", "n10_53", "cas16"])
def case(request, lib_mod):
    n, na, nb, h, g, V, e0, c = _space(request.param)
    print(f"[pt2s {request.param}] |V|={len(V)}", flush=True)
    ctx = lib_mod.HCIContext(h, g, na, nb)
    yield dict(name=request.param, n=n, h=h, g=g, V=V, e0=e0, c=c, ctx=ctx, eps=EPS[request.param])
    ctx.close()


def _close(a, b, tol=1e-10):
    return abs(a - b) <= tol * max(abs(b), 1e-300)


def test_stochastic_batches_match_oracle(case):
    h, g, V, e0, c, ctx = case["h"], case["g"], case["V"], case["e0"], case["c"], case["ctx"]
    eps2, eps2_d = case["eps"]
    rng = np.random.default_rng(7)
    u = rng.random((3, 64))
    a, b = ctx.pt2_stochastic(V, c, e0, eps2, eps2_d, u)
    for k in range(u.shape[0]):
        ra, rb = O.pt2_stochastic(h, g, V, c, e0, eps2, eps2_d, u[k])
        print(f"[pt2s {case['name']} batch {k}] gpu {a[k]:.15f} {b[k]:.15f} oracle {ra:.15f} {rb:.15f}",
              flush=True)
        assert _close(a[k], ra) and _close(b[k], rb), (k, a[k], ra, b[k], rb)


def test_semistochastic_matches_oracle(case):
    h, g, V, e0, c, ctx = case["h"], case["g"], case["V"], case["e0"], case["c"], case["ctx"]
    eps2, eps2_d = case["eps"]
    rng = np.random.default_rng(8)
    u = rng.random((3, 32))
    e2, err, e2d = ctx.pt2_semistochastic(V, c, e0, eps2, eps2_d, u)
    re2, rerr, re2d, _ = O.pt2_semistochastic(h, g, V, c, e0, eps2, eps2_d, list(u))
    assert _close(e2d, re2d, 1e-12)
    assert _close(e2, re2) and _close(err, rerr, 1e-8), (e2, re2, err, rerr)
    # one batch: no standard error
    _, err1, _ = ctx.pt2_semistochastic(V, c, e0, eps2, eps2_d, u[:1])
    assert np.isnan(err1)
    # thresholds that meet: the bracket of eq. semistoc vanishes exactly
    e2m, errm, e2dm = ctx.pt2_semistochastic(V, c, e0, eps2_d, eps2_d, u)
    assert e2m == e2dm and errm == 0.0


def test_deterministic_e2_in_passes(case, lib_mod):
    h, g, V, e0, c, ctx = case["h"], case["g"], case["V"], case["e0"], case["c"], case["ctx"]
    eps2 = case["eps"][0]
    ref = O.pt2(h, g, V, c, e0, eps2)
    e2_1, r_1, nc_1 = ctx.pt2(V, c, e0, eps2)
    npairs = len(ref["pairs"][1])
    # a budget of about a fifth of the pairs forces several passes
    ctx.set_pt2_budget(max(128, 128 * npairs // 5))
    try:
        e2_p, r_p, nc_p = ctx.pt2(V, c, e0, eps2)
    finally:
        ctx.set_pt2_budget(64 << 30)
    print(f"[pt2 passes {case['name']}] pairs {npairs} |C| {len(ref['C'])} E2 {e2_1:.15f} {e2_p:.15f}",
          flush=True)
    assert nc_1 == nc_p == len(ref["C"])
    for e2, r in [(e2_1, r_1), (e2_p, r_p)]:
        assert _close(e2, ref["E2"], 1e-12)
        rr = r.cpu().numpy()
        assert np.abs(rr - ref["r"]).max() <= 1e-12 * max(1.0, np.abs(ref["r"]).max())


def test_stochastic_rejects_bad_arguments(case, lib_mod):
    V, e0, c, ctx = case["V"], case["e0"], case["c"], case["ctx"]
    u = np.full((1, 4), 0.5)
    bad = []
    for args in [(1e-3, 1e-4, u),                    # eps2_d < eps2
                 (1e-4, 1e-3, u[:, :1]),             # one draw
                 (1e-4, 1e-3, np.array([[0.5, 1.0, 0.2, 0.1]])),   # u = 1
                 (1e-4, 1e-3, np.array([[0.5, -0.1, 0.2, 0.1]]))]:  # u < 0
        with pytest.raises(lib_mod.HCIError) as ei:
            ctx.pt2_stochastic(V, c, e0, *args)
        bad.append(ei.value.code)
    assert bad == [-1, -1, -1, -1]
    with pytest.raises(lib_mod.HCIError):
        ctx.pt2_stochastic(V, np.zeros(len(V)), e0, 1e-4, 1e-3, u)


def test_stochastic_edge_draws(lib_mod):
    """Two draws on the same row (w = 2, the off-diagonal part vanishes) and a
    one-determinant space, against the oracle."""
    w = hs.WORKLOADS["cas8"]
    h, g = hs.workload_integrals(w)
    V0 = hs.aufbau_det(4, 4)
    V = O.merge(V0, O.select(h, g, V0, np.array([1.0]), 0.05))
    e0, c = O.lowest_eigenpair(h, g, V)
    ctx = lib_mod.HCIContext(h, g, 4, 4)
    # both uniforms in the first row's cumulative range
    _, q, Q = O.pt2_sample(c, np.array([0.0]))
    first = int(np.nonzero(q)[0][0])
    hi = q[first] / Q
    u = np.array([[0.0, 0.5 * hi]])
    wref, _, _ = O.pt2_sample(c, u[0])
    assert wref[first] == 2 and wref.sum() == 2
    a, b = ctx.pt2_stochastic(V, c, e0, 1e-5, 1e-3, u)
    ra, rb = O.pt2_stochastic(h, g, V, c, e0, 1e-5, 1e-3, u[0])
    assert abs(a[0] - ra) <= 1e-10 * abs(ra) and abs(b[0] - rb) <= 1e-10 * max(abs(rb), 1e-300)
    # a single determinant: every draw picks it
    V1 = V0
    c1 = np.array([1.0])
    e1 = O.diag(h, g, V1[0])
    u1 = np.array([[0.3, 0.9, 0.1]])
    a1, b1 = ctx.pt2_stochastic(V1, c1, e1, 1e-5, 1e-3, u1)
    ra1, rb1 = O.pt2_stochastic(h, g, V1, c1, e1, 1e-5, 1e-3, u1[0])
    assert abs(a1[0] - ra1) <= 1e-10 * abs(ra1) and abs(b1[0] - rb1) <= 1e-10 * abs(rb1)
    # with every draw on the one row the estimate is the deterministic E2
    assert abs(ra1 - O.pt2(h, g, V1, c1, e1, 1e-5)["E2"]) <= 1e-12 * abs(ra1)
    ctx.close()
