"""Pins of the oracle's semistochastic second-order energy (eq. semistoc).

* Draws: integer weights and the row each uniform picks, at the edges of the
  cumulative ranges, worked out by hand.
* Estimator: its expectation over every ordered outcome of a few draws
  (probabilities multiplied out exactly) equals the deterministic screened
  E2 of eq. pt_hci at both thresholds.  A dropped or mis-weighted term (the
  squares, the (N_d - 1) factor, the normalisation) changes the expectation.
* Combination: with eps2_d = eps2 the bracket of eq. semistoc vanishes and
  the result is the deterministic E2.
"""
import itertools

import numpy as np
import pytest

import hci_synth as hs
import oracle as O


def test_sample_weights_and_cumulative_edges():
    c = np.array([0.5, -0.25, 0.0, 0.125, 1e-12])
    two31 = 2 ** 31
    q_ref = [two31, two31 // 2, 0, two31 // 4, 1]  # |c| / max|c| * 2^31, at least 1
    Q = sum(q_ref)
    starts = np.cumsum([0] + q_ref[:-1])
    # target t = floor(u Q): first and last unit of each nonempty range
    targets = [0, two31 - 1, two31, starts[3] - 1, starts[3], starts[4] - 1, Q - 1]
    want = [0, 0, 1, 1, 3, 3, 4]
    u = (np.array(targets, dtype=np.float64) + 0.5) / Q
    w, q, QQ = O.pt2_sample(c, u)
    assert list(q) == q_ref and QQ == Q
    assert list(w) == list(np.bincount(want, minlength=len(c)))
    # u just below 1 is clamped into the last range
    w1, _, _ = O.pt2_sample(c, np.array([1.0 - 2.0 ** -53]))
    assert w1[4] == 1


@pytest.fixture(scope="module")
def tiny():
    w = hs.WORKLOADS["cas8"]
    h, g = hs.workload_integrals(w)
    V0 = hs.aufbau_det(4, 4)
    # the aufbau determinant and the two most important connections
    C = O.select(h, g, V0, np.array([1.0]), 0.0)
    hv = np.array([abs(O.hij(h, g, V0[0], x)) for x in C])
    V = O.merge(V0, C[np.argsort(-hv)[:2]])
    e0, c = O.lowest_eigenpair(h, g, V)
    return h, g, V, e0, c


@pytest.mark.parametrize("nd", [2, 3])
def test_estimator_expectation_is_the_screened_e2(tiny, nd):
    h, g, V, e0, c = tiny
    eps_list = [1e-4, 3e-3]
    # integer-weight probabilities, as the draws use them
    w0, q, Q = O.pt2_sample(c, np.array([0.5]))
    p = q / float(Q)
    expect = np.zeros(len(eps_list))
    for draw in itertools.product(range(len(V)), repeat=nd):
        prob = float(np.prod([p[i] for i in draw]))
        w = np.bincount(draw, minlength=len(V))
        expect += prob * np.array(O.pt2_stochastic_counts(h, g, V, c, e0, eps_list, w, p, nd))
    for k, eps in enumerate(eps_list):
        ref = O.pt2(h, g, V, c, e0, eps)["E2"]
        assert ref != 0.0
        assert abs(expect[k] - ref) <= 1e-12 * abs(ref), (nd, eps, expect[k], ref)


def test_semistochastic_reduces_to_deterministic_when_thresholds_meet(tiny):
    h, g, V, e0, c = tiny
    rng = np.random.default_rng(5)
    u = [rng.random(4) for _ in range(3)]
    e2, err, e2d, per = O.pt2_semistochastic(h, g, V, c, e0, 1e-3, 1e-3, u)
    assert e2 == e2d == O.pt2(h, g, V, c, e0, 1e-3)["E2"]
    assert err == 0.0
    assert all(x == y for x, y in per)
