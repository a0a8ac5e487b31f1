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


def test_assembly_fits_total_energy_against_e2():
    """Hand-made levels: E2 = (-0.3, -0.2, -0.1) and totals E_var + E2 =
    (1, 3, 2).  By hand: mean E2 = -0.2, mean total 2, S_xx = 0.02,
    S_xy = 0.1, so the line is 3 + 5 E2; the error bar is a quarter of
    |3 - 1| = 0.5 (level 0 is the most accurate total energy).  A fit of
    E_var instead of the total gives slope 4; an error taken from E_var_0
    gives 0.425; an error from the last level gives 0.25."""
    e2 = np.array([-0.3, -0.2, -0.1])
    etot = np.array([1.0, 3.0, 2.0])
    evar = etot - e2
    a, b, err = O.extrapolation_assemble(evar, e2)
    assert abs(a - 3.0) < 1e-12 and abs(b - 5.0) < 1e-12
    assert abs(err - 0.5) < 1e-12
    # the planted alternatives give other numbers
    a_v, b_v = O.extrapolation_fit(e2, evar)
    assert abs(b_v - 4.0) < 1e-12
    assert abs(0.25 * abs(a - evar[0]) - 0.425) < 1e-12
    assert abs(0.25 * abs(a - etot[-1]) - 0.25) < 1e-12


def test_assembly_two_levels_is_the_line_through_them():
    """Two levels: the line through (E2_0, T_0), (E2_1, T_1) evaluated at
    E2 = 0 is (T_1 E2_0 - T_0 E2_1) / (E2_0 - E2_1)."""
    e2 = np.array([-0.02, -0.05])
    evar = np.array([-100.10, -100.04])
    t = evar + e2
    a, b, err = O.extrapolation_assemble(evar, e2)
    a_ref = (t[1] * e2[0] - t[0] * e2[1]) / (e2[0] - e2[1])
    assert abs(a - a_ref) < 1e-12
    assert abs(b - (t[0] - t[1]) / (e2[0] - e2[1])) < 1e-12
    assert abs(err - 0.25 * abs(a_ref - t[0])) < 1e-13
