"""Pins of the oracle's extrapolation to the full-CI limit.

* Ranking by |c| with ties broken by index, level sizes, nesting.
* The fit: points on a known line give its intercept and slope exactly (to
  rounding); two points give the line through them.
* Nested spaces: the lowest eigenvalue never decreases from one level to
  the next (Rayleigh-Ritz), E2 < 0 below the ground state; on the full
  determinant space E2 = 0 and E_var is the full-CI energy (dense LAPACK).
"""
import numpy as np

import hci_synth as hs
import oracle as O


def test_ranking_and_sizes():
    c = np.array([0.1, -0.5, 0.5, 0.0, -0.1, 0.3])
    assert list(O.extrapolation_ranking(c)) == [1, 2, 5, 0, 4, 3]
    assert O.extrapolation_sizes(100, 0.33, 5) == [100, 67, 45, 31, 21]
    assert O.extrapolation_sizes(2, 0.9, 3) == [2, 1, 1]


def test_fit_closed_forms():
    x = np.array([-0.3, -0.2, -0.11, -0.05])
    y = -7.25 + 0.8 * x
    a, b = O.extrapolation_fit(x, y)
    assert abs(a + 7.25) < 1e-14 and abs(b - 0.8) < 1e-13
    a2, b2 = O.extrapolation_fit([-0.2, -0.1], [-7.4, -7.3])
    assert abs(b2 - 1.0) < 1e-13 and abs(a2 + 7.2) < 1e-13


def test_levels_are_nested_and_variational():
    w = hs.WORKLOADS["cas8"]
    h, g = hs.workload_integrals(w)
    V, _, _, _ = O.hci(h, g, 4, 4, 3e-2)
    e, c = O.lowest_eigenpair(h, g, V)
    res = O.extrapolation(h, g, V, c, 0.33, 4, 1e-5)
    assert res["sizes"] == O.extrapolation_sizes(len(V), 0.33, 4)
    assert abs(res["evar"][0] - e) < 1e-10
    # nested spaces: the lowest eigenvalue cannot go down as determinants go
    assert all(b >= a - 1e-12 for a, b in zip(res["evar"], res["evar"][1:])), res["evar"]
    assert all(x < 0 for x in res["e2"])
    # the full space: nothing outside it, E2 = 0 and E_var = E_FCI
    F = hs.full_space(8, 4, 4)
    efci, cf = O.lowest_eigenpair(h, g, F)
    full = O.extrapolation(h, g, F, cf, 0.33, 2, 1e-5)
    assert full["e2"][0] == 0.0 and abs(full["evar"][0] - efci) < 1e-10
