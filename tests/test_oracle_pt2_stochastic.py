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


# ---------------------------------------------------------------- eq. semistoc
# The combination E2^D(eps2_d) + [E2^S(eps2) - E2^S(eps2_d)] is unbiased for
# the deterministic E2(eps2): averaged over every ordered outcome of the
# draws of one batch it must give E2(eps2) exactly (up to rounding), with
# eps2 < eps2_d so that the bracket does not vanish.  A flipped bracket, the
# deterministic part taken at eps2 instead of eps2_d, or the two sampled
# terms swapped all move the expectation away from E2(eps2).


def _draw_u(c, rows):
    """Uniforms whose draws pick exactly the given rows (the centre of each
    row's cumulative weight range)."""
    _, q, Q = O.pt2_sample(c, np.array([0.5]))
    before = np.concatenate([[0], np.cumsum(q)[:-1]])
    return np.array([(before[i] + q[i] // 2 + 0.5) / Q for i in rows], dtype=np.float64)


def _semistoc_expectation(tiny, nd, eps2, eps2_d, combine):
    h, g, V, e0, c = tiny
    _, q, Q = O.pt2_sample(c, np.array([0.5]))
    p = q / float(Q)
    e2d = O.pt2(h, g, V, c, e0, eps2_d)["E2"]
    expect = 0.0
    for draw in itertools.product(range(len(V)), repeat=nd):
        prob = float(np.prod([p[i] for i in draw]))
        u = _draw_u(c, draw)
        w, _, _ = O.pt2_sample(c, u)
        assert list(w) == list(np.bincount(draw, minlength=len(V)))
        per = [O.pt2_stochastic(h, g, V, c, e0, eps2, eps2_d, u)]
        expect += prob * combine(e2d, per, eps2)
    return expect


def _oracle_combine(tiny):
    def f(e2d, per, eps2):
        return O.semistochastic_combine(e2d, per)[0]
    return f


EPS_PAIR = (1e-4, 3e-3)


@pytest.mark.parametrize("nd", [2, 3])
def test_semistochastic_expectation_is_deterministic_e2(tiny, nd):
    h, g, V, e0, c = tiny
    eps2, eps2_d = EPS_PAIR
    ref = O.pt2(h, g, V, c, e0, eps2)["E2"]
    refd = O.pt2(h, g, V, c, e0, eps2_d)["E2"]
    assert abs(ref - refd) > 1e-6 * abs(ref)  # the bracket carries weight
    got = _semistoc_expectation(tiny, nd, eps2, eps2_d, _oracle_combine(tiny))
    assert abs(got - ref) <= 1e-12 * abs(ref), (nd, got, ref)
    # the full routine on one outcome equals the combination of its pieces
    u = _draw_u(c, [0, 1])
    e2, err, e2d, per = O.pt2_semistochastic(h, g, V, c, e0, eps2, eps2_d, [u])
    assert e2d == refd and np.isnan(err)
    assert e2 == O.semistochastic_combine(e2d, per)[0]


def test_semistochastic_planted_mistakes_fail(tiny):
    """Each plausible mistake in the combination breaks the expectation pin."""
    h, g, V, e0, c = tiny
    eps2, eps2_d = EPS_PAIR
    ref = O.pt2(h, g, V, c, e0, eps2)["E2"]
    e2_at_eps2 = ref

    def flipped(e2d, per, _):
        x, y = per[0]
        return e2d - (x - y)

    def det_at_eps2(e2d, per, _):
        x, y = per[0]
        return e2_at_eps2 + (x - y)

    def swapped(e2d, per, _):
        x, y = per[0]
        return e2d + (y - x)

    def bracket_only_eps2(e2d, per, _):
        x, _y = per[0]
        return e2d + x

    for bad in (flipped, det_at_eps2, swapped, bracket_only_eps2):
        got = _semistoc_expectation(tiny, 2, eps2, eps2_d, bad)
        assert abs(got - ref) > 1e-6 * abs(ref), bad.__name__


def test_semistochastic_standard_error_closed_forms():
    """Standard error of the mean of the brackets, from hand algebra: two
    batches with brackets x, y give |x - y| / 2; three batches x, x, y give
    |x - y| / 3 (sample variance with n_b - 1, divided by sqrt(n_b))."""
    e2d = -0.75
    x, y = -0.0123, -0.0071
    per2 = [(x + 0.5, 0.5), (y - 0.25, -0.25)]
    e2, err = O.semistochastic_combine(e2d, per2)
    assert abs(e2 - (e2d + (x + y) / 2)) < 1e-15
    assert abs(err - abs(x - y) / 2) < 1e-15
    per3 = [(x + 1.0, 1.0), (x - 2.0, -2.0), (y, 0.0)]
    e2, err = O.semistochastic_combine(e2d, per3)
    assert abs(e2 - (e2d + (2 * x + y) / 3)) < 1e-14
    assert abs(err - abs(x - y) / 3) < 1e-15
    # planted mistakes in the error: population variance, division by n_b
    diff = np.array([x, y])
    assert abs(np.std(diff) / np.sqrt(2) - abs(x - y) / 2) > 1e-4
    assert abs(np.std(diff, ddof=1) / 2 - abs(x - y) / 2) > 1e-4
    # one batch: no error estimate
    assert np.isnan(O.semistochastic_combine(e2d, [(x, 0.0)])[1])
