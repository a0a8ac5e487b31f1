"""Extrapolation to the full-CI limit against the oracle.

Both sides rank the determinants by the same input vector (the oracle's
eigenvector of the largest space), so the nested levels are identical and
the determinant counts compare exactly; each level's E_var comes from the
library's Davidson (tolerance 1e-9, f64 refinement in mixed precision) and
the oracle's dense or Lanczos eigensolver (1e-8 Ha), E2 from the screened
walk on each side's own eigenvector (1e-8 relative + 1e-10 Ha), and the fit
follows from them (1e-7 Ha).
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
        w = hs.WORKLOADS["cas8"]
        h, g = hs.workload_integrals(w)
        V, _, _, _ = O.hci(h, g, 4, 4, 3e-2)
        return h, g, 4, 4, V, 1e-5, 4
    w = hs.WORKLOADS["cas16"]
    h, g = hs.workload_integrals(w)
    V0 = hs.aufbau_det(8, 8)
    V = O.merge(V0, O.select(h, g, V0, np.array([1.0]), 5e-2))
    return h, g, 8, 8, V, 3e-3, 3


@pytest.mark.parametrize("name,precision", [("cas8", "fp64"), ("cas8", "fp32_mixed"), ("cas16", "fp64")])
def test_extrapolation_matches_oracle(P, name, precision):
    h, g, na, nb, V, eps2, levels = _space(name)
    e, c = O.lowest_eigenpair(h, g, V)
    print(f"[extrap {name} |V|={len(V)} {precision}]", flush=True)
    ref = O.extrapolation(h, g, V, c, 0.33, levels, eps2)
    ctx = P.HCIContext(h, g, na, nb)
    res = ctx.extrapolate(V, c, fraction=0.33, levels=levels, eps2=eps2, tol=1e-9, precision=precision)
    ctx.close()
    print(f"  gpu {res['evar']} {res['e2']} -> {res['e_extrap']:.9f}; oracle {ref['evar']} {ref['e2']} -> "
          f"{ref['e_extrap']:.9f}", flush=True)
    assert res["sizes"] == ref["sizes"]
    assert np.abs(res["evar"] - ref["evar"]).max() < 1e-8
    assert np.all(np.abs(res["e2"] - ref["e2"]) <= 1e-8 * np.abs(ref["e2"]) + 1e-10)
    assert abs(res["e_extrap"] - ref["e_extrap"]) < 1e-7
    assert abs(res["slope"] - ref["slope"]) < 1e-6 * max(1.0, abs(ref["slope"]))
    assert abs(res["error"] - ref["error"]) < 1e-7


def test_extrapolation_rejects_bad_arguments(P):
    h, g, na, nb, V, eps2, levels = _space("cas8")
    c = np.ones(len(V)) / np.sqrt(len(V))
    ctx = P.HCIContext(h, g, na, nb)
    for kw in [dict(levels=1), dict(fraction=0.0), dict(fraction=1.0), dict(eps2=-1.0), dict(tol=0.0)]:
        with pytest.raises(P.HCIError) as ei:
            ctx.extrapolate(V, c, **kw)
        assert ei.value.code == -1, kw
    ctx.close()


def test_extrapolation_down_to_one_determinant(P):
    """Levels that shrink to a single determinant (sizes 4, 2, 1, 1): each
    level against the oracle; the repeated last point leaves the fit defined."""
    w = hs.WORKLOADS["cas8"]
    h, g = hs.workload_integrals(w)
    V0 = hs.aufbau_det(4, 4)
    C = O.select(h, g, V0, np.array([1.0]), 0.0)
    hv = np.array([abs(O.hij(h, g, V0[0], x)) for x in C])
    V = O.merge(V0, C[np.argsort(-hv)[:3]])
    e, c = O.lowest_eigenpair(h, g, V)
    ref = O.extrapolation(h, g, V, c, 0.5, 4, 1e-4)
    assert ref["sizes"] == [4, 2, 1, 1]
    ctx = P.HCIContext(h, g, 4, 4)
    res = ctx.extrapolate(V, c, fraction=0.5, levels=4, eps2=1e-4, tol=1e-10)
    ctx.close()
    assert res["sizes"] == ref["sizes"]
    assert np.abs(res["evar"] - ref["evar"]).max() < 1e-9
    assert np.all(np.abs(res["e2"] - ref["e2"]) <= 1e-9 * np.abs(ref["e2"]) + 1e-12)
    assert abs(res["e_extrap"] - ref["e_extrap"]) < 1e-8
