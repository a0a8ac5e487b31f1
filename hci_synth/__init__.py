"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws numbers and lays them out; it holds none of the method's
arithmetic (no matrix elements, no selection, no eigensolver).  Both the CPU
oracle and the GPU path receive exactly the arrays produced here.

Integral recipe (the active spaces the paper studies are replaced by
synthetic ones of the same shape, since the molecules' integrals are not
available):

    rng  = numpy.random.default_rng(seed)
    eps  = linspace(-2, 1, n)                (porphyrin-shaped variant below)
    h    = diag(eps) + S,   S symmetric, off-diagonal N(0, 0.05)
    B^L  symmetric n x n, entries N(0, 0.15),  L = 3n
    g    = sum_L B^L_pq B^L_rs                chemist (pq|rs), 8-fold symmetric,
                                              positive semidefinite as (pq)x(rs),
                                              made exactly symmetric under (pq)<->(rs)

Draw order is fixed: the off-diagonal block of h first, then B.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Optional, Tuple

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "make_integrals", "aufbau_det", "det_bits",
    "random_dets", "random_coeffs", "orbitals_of",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    """A synthetic active space: n orbitals, nalpha + nbeta electrons."""
    name: str
    norb: int
    nalpha: int
    nbeta: int
    naux: int
    seed: int
    eps1: float
    porphyrin: bool = False
    eps2: float = 0.0


# (8e,8o) full space; (16e,16o) at eps1 = 1e-4; (30e,30o) at eps1 = 3e-5;
# (44e,44o) porphyrin-shaped at eps1 = 1e-4 and at 5e-5 with eps2 for the
# relaxed density matrix.
WORKLOADS: Dict[str, Workload] = {
    "cas8": Workload("cas8", 8, 4, 4, 24, 0, 0.0),
    "cas16": Workload("cas16", 16, 8, 8, 48, 1, 1e-4),
    "cas30": Workload("cas30", 30, 15, 15, 90, 2, 3e-5),
    "cas44": Workload("cas44", 44, 22, 22, 132, 3, 1e-4, porphyrin=True),
    "cas44r": Workload("cas44r", 44, 22, 22, 132, 3, 5e-5, porphyrin=True, eps2=1e-5),
}


def make_integrals(norb: int, naux: int, seed: int, porphyrin: bool = False
                   ) -> Tuple[np.ndarray, np.ndarray]:
    """Return (h [n,n], g [n,n,n,n]) float64, C-contiguous, chemist order."""
    n = int(norb)
    rng = np.random.default_rng(seed)
    eps = np.linspace(-2.0, 1.0, n)
    if porphyrin:
        # ten orbitals (five below, five above) within 0.1 Ha of the Fermi level
        nocc = n // 2
        ef = 0.5 * (eps[nocc - 1] + eps[nocc])
        eps[nocc - 5:nocc + 5] = np.linspace(ef - 0.09, ef + 0.09, 10)
    h = np.diag(eps)
    u = rng.normal(0.0, 0.05, (n, n))
    h = h + np.triu(u, 1) + np.triu(u, 1).T
    b = rng.normal(0.0, 0.15, (naux, n, n))
    b = np.triu(b) + np.transpose(np.triu(b, 1), (0, 2, 1))
    bm = b.reshape(naux, n * n)
    g = (bm.T @ bm).reshape(n, n, n, n)
    # a GEMM may round (pq,rs) and (rs,pq) differently; averaging makes the
    # pair symmetry exact (and changes nothing where it already holds)
    g = 0.5 * (g + g.transpose(2, 3, 0, 1))
    return np.ascontiguousarray(h), np.ascontiguousarray(g)


def workload_integrals(w: Workload) -> Tuple[np.ndarray, np.ndarray]:
    return make_integrals(w.norb, w.naux, w.seed, w.porphyrin)


def det_bits(orbs) -> int:
    """Occupation word with bit p set for each orbital p in `orbs`."""
    x = 0
    for p in orbs:
        x |= 1 << int(p)
    return x


def orbitals_of(word: int):
    """Ascending orbital indices set in an occupation word."""
    word = int(word)
    out = []
    p = 0
    while word:
        if word & 1:
            out.append(p)
        word >>= 1
        p += 1
    return out


def aufbau_det(nalpha: int, nbeta: int) -> np.ndarray:
    """Lowest-index occupation: alpha 0..nalpha-1, beta 0..nbeta-1, shape [1,2] uint64."""
    return np.array([[(1 << nalpha) - 1, (1 << nbeta) - 1]], dtype=np.uint64)


def _random_string(rng, norb, nel, bias):
    # orbitals weighted towards low indices so the set looks like a CI expansion
    w = np.exp(-bias * np.arange(norb))
    w = w / w.sum()
    occ = rng.choice(norb, size=nel, replace=False, p=w)
    return det_bits(occ)


def random_dets(norb: int, nalpha: int, nbeta: int, count: int, seed: int,
                bias: float = 0.15, include_aufbau: bool = True) -> np.ndarray:
    """Sorted, unique determinant set of (up to) `count` members, shape [m,2] uint64.

    Rows are (alpha word, beta word); order is lexicographic by alpha then beta.
    """
    rng = np.random.default_rng(seed)
    seen = set()
    if include_aufbau:
        seen.add(((1 << nalpha) - 1, (1 << nbeta) - 1))
    tries = 0
    while len(seen) < count and tries < 50 * count + 1000:
        tries += 1
        a = _random_string(rng, norb, nalpha, bias)
        b = _random_string(rng, norb, nbeta, bias)
        seen.add((a, b))
    arr = np.array(sorted(seen), dtype=np.uint64).reshape(-1, 2)
    return arr


def random_coeffs(m: int, seed: int, decay: float = 3.0,
                  lead: Optional[int] = 0) -> np.ndarray:
    """Normalised float64 vector with a dominant entry and log-uniform tail."""
    rng = np.random.default_rng(seed)
    mag = np.exp(-decay * rng.uniform(0.0, 3.0, m))
    sgn = np.where(rng.uniform(size=m) < 0.5, -1.0, 1.0)
    c = mag * sgn
    if lead is not None and m > 0:
        c[lead] = 3.0 * max(1.0, np.abs(c).max())
    c /= np.linalg.norm(c) if m else 1.0
    return c


def all_strings(norb: int, nel: int):
    """All occupation words of `nel` electrons in `norb` orbitals, ascending."""
    from itertools import combinations
    out = [det_bits(c) for c in combinations(range(norb), nel)]
    out.sort()
    return out


def full_space(norb: int, nalpha: int, nbeta: int) -> np.ndarray:
    """Every determinant with the given electron counts, sorted by (alpha, beta)."""
    sa = all_strings(norb, nalpha)
    sb = all_strings(norb, nbeta)
    arr = np.array([(a, b) for a in sa for b in sb], dtype=np.uint64).reshape(-1, 2)
    return arr
