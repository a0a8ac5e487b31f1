"""CPU oracle for the Heat-bath CI variational step -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct implementations of what the GPU library
computes, used only by ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg.  The product path never imports this package.
It shares no code with the GPU library; the only common dependency is the
seeded input generator ``hci_synth``, which holds none of the method's
arithmetic.

Where each function comes from (paper sections/equations):

* ``hamiltonian_by_operators`` / ``hij`` -- the second-quantised active-space
  Hamiltonian applied to determinants, by the operator definition and by the
  textbook Slater-Condon rules (the paper notes double-excitation elements
  depend on the orbitals only: Sec. "Variational Stage").
* ``select`` -- the HCI criterion, Sec. "Variational Stage", eq. (criteria) and
  the HCI importance function: D_a is kept when |H_ai c_i| > eps1 for some
  D_i in V.  Written as its definition (every excitation of every D_i is
  evaluated), not as the heat-bath walk.
* ``select_bruteforce`` -- the same criterion evaluated over the whole
  determinant space with the operator-built H (tiny spaces).
* ``spin_square`` -- <S^2> = S_z (S_z + 1) + |S_+ c|^2 of a state, by the
  definition of the spin raising operator on the determinants.
* ``select_roots`` / ``lowest_eigenpairs`` -- several states of one
  calculation (the paper's excited states are the lowest states of other
  spin projections, N_alpha != N_beta, which every function here accepts):
  the k lowest eigenpairs by a library eigensolver, and the union of the
  single-state selections (a reading: the paper selects for one state).
* ``hci`` -- the variational macro-iteration V <- V + C(eps1) followed by
  re-diagonalisation (Sec. "Variational Stage", Fig. 1a), with a library
  eigensolver standing in for Davidson (eq. variational).
* ``rdm12`` -- density matrices by operator application (Sec.
  "Computational Details": contracted with integral derivatives in
  eq. vdedk2 / eq. lambda).
* ``pt2_*`` -- eps2-screened Epstein-Nesbet PT2 and its pieces
  (eq. h0, eq. pt, eq. pt_hci, Hylleraas functional eq. hylleraas).
* ``zvector_dense`` -- the Lagrange-multiplier equation for lambda_c
  (eq. lagd, eq. lagc and the simplified form after them).
* ``orbital_gradient`` / ``rotate_integrals`` -- the orbital step of
  aHCISCF (Sec. "HCI self-consistent field", eq. lambda and eq. vdedk2: the
  energy gradient in the orbital rotation parameters kappa is the integral
  derivatives contracted with the density matrices).  Only active-active
  rotations exist here: h' = U^T h U, (pq|rs)' = sum U_ap U_bq U_cr U_ds
  (ab|cd) with U = exp(kappa), kappa antisymmetric.  The paper refers the
  integral derivatives to other work; written out for
  E = sum h_pq gamma_pq + 1/2 sum (pq|rs) Gamma_pqrs they give
  dE/dkappa_xy = 2 (F_xy - F_yx), F = h gamma + G,
  G_xy = sum_qrs (xq|rs) Gamma_yqrs (density matrices with the index
  symmetries of a real state).
* ``extrapolation_*`` -- the extrapolation to the full-CI limit of Sec.
  "Results and discussion" (butadiene): after the largest HCI calculation,
  single-step calculations each drop a fraction (0.33) of the least
  important determinants; a straight line through (E2, E_var + E2) is
  evaluated at E2 = 0.  Readings: importance is |c_i| of the largest
  calculation (one ranking, ties by determinant index, so the spaces are
  nested), each level keeps ceil(m (1 - fraction)) of the previous m, E2 is
  the deterministic screened E2 of each level's own eigenpair, the line is the
  least-squares fit over all levels, and the error estimate is 25% of the
  distance from the extrapolated energy to the largest calculation's total
  energy (as the paper's Fe-porphyrin table states).
* ``pt2_sample`` / ``pt2_stochastic*`` / ``pt2_semistochastic`` -- the
  semistochastic second-order energy, eq. semistoc: a deterministic E2 at a
  loose eps2_d plus the difference of two sampled estimates (tight eps2 and
  eps2_d) taken from the same draws.  The paper defers the sampling
  estimator to its reference; the reading used here is the unbiased estimate
  of sum_a (sum_i x_ai)^2 / (E0 - H_aa) from N_d draws with replacement
  (probability p_i, multiplicity w_i, x_ai = H_ai c_i): for each a
  [S1^2 - S2 + (N_d - 1) S3] / (N_d (N_d - 1)) with S1 = sum w x / p,
  S2 = sum (w x / p)^2, S3 = sum w x^2 / p (distinct draws give the
  off-diagonal products, single draws the squares).  p_i = q_i / Q with
  integer weights q_i = max(1, round(2^31 |c_i| / max|c|)) (c_i != 0), so
  the cumulative weights are exact integers; draw k picks the row whose
  cumulative range holds floor(u_k Q) for a caller-supplied uniform u_k.

Readings where the paper is silent (sign convention, integral notation,
RDM index order, threshold rounding) are listed in the C source header.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hci_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

u64p = ctypes.POINTER(ctypes.c_uint64)
f64p = ctypes.POINTER(ctypes.c_double)
i64p = ctypes.POINTER(ctypes.c_long)


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_diag.restype = ctypes.c_double
        L.orc_diag.argtypes = [ctypes.c_int, f64p, f64p, ctypes.c_uint64, ctypes.c_uint64]
        L.orc_hij.restype = ctypes.c_double
        L.orc_hij.argtypes = [ctypes.c_int, f64p, f64p] + [ctypes.c_uint64] * 4
        L.orc_excitations.restype = ctypes.c_long
        L.orc_excitations.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, u64p, ctypes.c_long]
        L.orc_find.restype = ctypes.c_long
        L.orc_find.argtypes = [u64p, ctypes.c_long, ctypes.c_uint64, ctypes.c_uint64]
        L.orc_select.restype = ctypes.c_long
        L.orc_select.argtypes = [ctypes.c_int, f64p, f64p, u64p, ctypes.c_long, f64p,
                                 ctypes.c_double, u64p, ctypes.c_long]
        L.orc_sigma_rows.restype = None
        L.orc_sigma_rows.argtypes = [ctypes.c_int, f64p, f64p, u64p, ctypes.c_long, f64p,
                                     i64p, ctypes.c_long, f64p, i64p]
        L.orc_row_counts.restype = None
        L.orc_row_counts.argtypes = [ctypes.c_int, u64p, ctypes.c_long, i64p]
        L.orc_csr_fill.restype = None
        L.orc_csr_fill.argtypes = [ctypes.c_int, f64p, f64p, u64p, ctypes.c_long, i64p, i64p, f64p]
        L.orc_rdm12.restype = None
        L.orc_rdm12.argtypes = [ctypes.c_int, u64p, ctypes.c_long, f64p, f64p, f64p, f64p]
        L.orc_rdm2_element.restype = ctypes.c_double
        L.orc_rdm2_element.argtypes = [ctypes.c_int, u64p, ctypes.c_long, f64p, f64p] + [ctypes.c_int] * 4
        L.orc_rdm1_element.restype = ctypes.c_double
        L.orc_rdm1_element.argtypes = [ctypes.c_int, u64p, ctypes.c_long, f64p, f64p] + [ctypes.c_int] * 2
        L.orc_apply_h.restype = ctypes.c_long
        L.orc_apply_h.argtypes = [ctypes.c_int, f64p, f64p, ctypes.c_uint64, ctypes.c_uint64,
                                  u64p, f64p, ctypes.c_long]
        _lib = L
    return _lib


def _f64(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    return x, x.ctypes.data_as(f64p)


def _u64(x):
    x = np.ascontiguousarray(x, dtype=np.uint64)
    return x, x.ctypes.data_as(u64p)


def _i64(x):
    x = np.ascontiguousarray(x, dtype=np.int64)
    return x, x.ctypes.data_as(i64p)


# ---------------------------------------------------------------- elements
def diag(h, g, det) -> float:
    n = h.shape[0]
    h, hp = _f64(h)
    g, gp = _f64(g)
    return lib().orc_diag(n, hp, gp, int(det[0]), int(det[1]))


def hij(h, g, det_i, det_j) -> float:
    """<D_j|H|D_i> by the Slater-Condon rules."""
    n = h.shape[0]
    h, hp = _f64(h)
    g, gp = _f64(g)
    return lib().orc_hij(n, hp, gp, int(det_i[0]), int(det_i[1]), int(det_j[0]), int(det_j[1]))


def excitations(n, det) -> np.ndarray:
    L = lib()
    m = L.orc_excitations(n, int(det[0]), int(det[1]), None, 0)
    out = np.zeros((m, 2), dtype=np.uint64)
    L.orc_excitations(n, int(det[0]), int(det[1]), out.ctypes.data_as(u64p), m)
    return out


def apply_h(h, g, det):
    """H|D> as {det: amplitude}, by applying each operator term (no rules)."""
    n = h.shape[0]
    h, hp = _f64(h)
    g, gp = _f64(g)
    L = lib()
    cap = (2 * n) ** 2 + (2 * n) ** 4
    dets = np.zeros((cap, 2), dtype=np.uint64)
    amp = np.zeros(cap)
    k = L.orc_apply_h(n, hp, gp, int(det[0]), int(det[1]), dets.ctypes.data_as(u64p),
                      amp.ctypes.data_as(f64p), cap)
    out = {}
    for t in range(k):
        key = (int(dets[t, 0]), int(dets[t, 1]))
        out[key] = out.get(key, 0.0) + float(amp[t])
    return out


def hamiltonian_by_operators(h, g, dets) -> np.ndarray:
    """Dense H on a determinant list built by operator application."""
    dets = np.asarray(dets, dtype=np.uint64)
    index = {(int(a), int(b)): k for k, (a, b) in enumerate(dets)}
    m = len(dets)
    H = np.zeros((m, m))
    for j in range(m):
        for key, amp in apply_h(h, g, dets[j]).items():
            i = index.get(key)
            if i is not None:
                H[i, j] += amp
    return H


def row_counts(n, V) -> np.ndarray:
    V, vp = _u64(V)
    cnt = np.zeros(len(V), dtype=np.int64)
    lib().orc_row_counts(n, vp, len(V), cnt.ctypes.data_as(i64p))
    return cnt


def hamiltonian_csr(h, g, V):
    """Sparse H on the sorted space V by the Slater-Condon rules (scipy CSR)."""
    import scipy.sparse as sp
    n = h.shape[0]
    h, hp = _f64(h)
    g, gp = _f64(g)
    V, vp = _u64(V)
    cnt = row_counts(n, V)
    rowptr = np.zeros(len(V) + 1, dtype=np.int64)
    np.cumsum(cnt, out=rowptr[1:])
    cols = np.zeros(rowptr[-1], dtype=np.int64)
    vals = np.zeros(rowptr[-1])
    lib().orc_csr_fill(n, hp, gp, vp, len(V), rowptr.ctypes.data_as(i64p),
                       cols.ctypes.data_as(i64p), vals.ctypes.data_as(f64p))
    return sp.csr_matrix((vals, cols, rowptr), shape=(len(V), len(V)))


def sigma(h, g, V, c, rows=None, with_pairs=False):
    """sigma_i = sum_j H_ij c_j (j over V), for all rows or the listed ones.
    with_pairs: also return the number of connected j of each row."""
    n = h.shape[0]
    h, hp = _f64(h)
    g, gp = _f64(g)
    V, vp = _u64(V)
    c, cp = _f64(c)
    m = len(V) if rows is None else len(rows)
    out = np.zeros(m)
    pairs = np.zeros(m, dtype=np.int64)
    if rows is None:
        lib().orc_sigma_rows(n, hp, gp, vp, len(V), cp, None, 0, out.ctypes.data_as(f64p),
                             pairs.ctypes.data_as(i64p))
    else:
        rows, rp = _i64(rows)
        lib().orc_sigma_rows(n, hp, gp, vp, len(V), cp, rp, len(rows), out.ctypes.data_as(f64p),
                             pairs.ctypes.data_as(i64p))
    return (out, pairs) if with_pairs else out


# ---------------------------------------------------------------- spaces
def sort_unique(dets) -> np.ndarray:
    dets = np.asarray(dets, dtype=np.uint64).reshape(-1, 2)
    if len(dets) == 0:
        return dets
    order = np.lexsort((dets[:, 1], dets[:, 0]))
    d = dets[order]
    keep = np.ones(len(d), dtype=bool)
    keep[1:] = (d[1:, 0] != d[:-1, 0]) | (d[1:, 1] != d[:-1, 1])
    return np.ascontiguousarray(d[keep])


def merge(V, C) -> np.ndarray:
    return sort_unique(np.concatenate([np.asarray(V, np.uint64).reshape(-1, 2),
                                       np.asarray(C, np.uint64).reshape(-1, 2)]))


def select(h, g, V, c, eps) -> np.ndarray:
    """C(eps): every determinant outside V with fl(|H_ai| |c_i|) > eps for some
    D_i in V (HCI criterion, eq. criteria), sorted and unique."""
    n = h.shape[0]
    h, hp = _f64(h)
    g, gp = _f64(g)
    V, vp = _u64(V)
    c, cp = _f64(c)
    L = lib()
    total = L.orc_select(n, hp, gp, vp, len(V), cp, float(eps), None, 0)
    out = np.zeros((max(total, 1), 2), dtype=np.uint64)
    L.orc_select(n, hp, gp, vp, len(V), cp, float(eps), out.ctypes.data_as(u64p), total)
    return sort_unique(out[:total])


def select_roots(h, g, V, C, eps) -> np.ndarray:
    """Selection for several states at once: the union over the rows c of C
    of C(eps) (a determinant enters when it passes the criterion of eq.
    criteria for at least one state).  The paper computes each state it
    reports separately; the union is the reading taken for several roots of
    one calculation."""
    C = np.atleast_2d(np.asarray(C, dtype=np.float64))
    parts = [select(h, g, V, c, eps) for c in C]
    return sort_unique(np.concatenate([p.reshape(-1, 2) for p in parts]))


def select_bruteforce(h, g, V, c, eps, space) -> np.ndarray:
    """The same criterion over a whole determinant space with the
    operator-built H: keep a outside V when max_i |H_ai c_i| > eps; c may
    hold several states as rows (then the maximum runs over them too)."""
    space = np.asarray(space, dtype=np.uint64)
    Hs = hamiltonian_by_operators(h, g, space)
    index = {(int(a), int(b)): k for k, (a, b) in enumerate(space)}
    vi = np.array([index[(int(a), int(b))] for a, b in V], dtype=np.int64)
    inV = np.zeros(len(space), dtype=bool)
    inV[vi] = True
    C = np.atleast_2d(np.abs(np.asarray(c, dtype=np.float64)))
    f = np.max(np.abs(Hs[:, vi])[None, :, :] * C[:, None, :], axis=(0, 2))
    keep = (f > eps) & ~inV
    return sort_unique(space[keep])


# ---------------------------------------------------------------- solvers
def lowest_eigenpair(h, g, V, tol=1e-12, v0=None, dense_max=3000):
    """Lowest eigenpair of H on V: dense LAPACK below dense_max, else Lanczos
    (scipy eigsh) on the CSR matrix.  Sign fixed so the largest |c_i| is > 0."""
    m = len(V)
    if m <= dense_max:
        H = hamiltonian_csr(h, g, V).toarray()
        w, U = np.linalg.eigh(H)
        e, c = float(w[0]), U[:, 0].copy()
    else:
        import scipy.sparse.linalg as sla
        H = hamiltonian_csr(h, g, V)
        w, U = sla.eigsh(H, k=1, which="SA", tol=tol, v0=v0)
        e, c = float(w[0]), U[:, 0].copy()
    k = int(np.argmax(np.abs(c)))
    if c[k] < 0:
        c = -c
    return e, c


def spin_square(V, c) -> float:
    """<S^2> of the state c on V, for characterising the states (the paper
    reports states of given spin: the pentacene triplet, the Fe-porphyrin
    triplet and quintet).  S^2 = S_z (S_z + 1) + S_- S_+, so
    <S^2> = S_z (S_z + 1) + |S_+ c|^2 / |c|^2 with S_+ = sum_p a+_pa a_pb.
    a+_pa a_pb acts on D = (alpha, beta) with p in beta and not in alpha and
    gives D' = (alpha + p, beta - p) with the sign (-1)^(N_alpha + #beta
    below p + #alpha below p) (alpha creators left of beta creators,
    ascending orbitals).  Written out per orbital over the whole list."""
    V = np.asarray(V, dtype=np.uint64).reshape(-1, 2)
    c = np.asarray(c, dtype=np.float64)
    a, b = V[:, 0], V[:, 1]
    na = int(np.bitwise_count(a[0])) if len(V) else 0
    nb = int(np.bitwise_count(b[0])) if len(V) else 0
    keys, vals = [], []
    for p in range(64):
        bit = np.uint64(1) << np.uint64(p)
        below = bit - np.uint64(1)
        sel = ((b & bit) != 0) & ((a & bit) == 0)
        if not sel.any():
            continue
        nbelow = np.bitwise_count(b[sel] & below).astype(np.int64) + np.bitwise_count(a[sel] & below).astype(np.int64)
        sign = np.where((na + nbelow) % 2 == 0, 1.0, -1.0)
        keys.append(np.stack([a[sel] | bit, b[sel] & ~bit], axis=1))
        vals.append(sign * c[sel])
    sz = 0.5 * (na - nb)
    norm2 = float(c @ c)
    if not keys:
        return sz * (sz + 1.0)
    K = np.concatenate(keys)
    X = np.concatenate(vals)
    kv = np.ascontiguousarray(K).view([("a", np.uint64), ("b", np.uint64)]).ravel()
    _, inv = np.unique(kv, return_inverse=True)
    amp = np.zeros(inv.max() + 1)
    np.add.at(amp, inv, X)
    return sz * (sz + 1.0) + float(amp @ amp) / norm2


SIGN_TIE = 1e-6


def _fix_sign(c):
    """Sign convention of the eigenvectors (a reading: the paper fixes none):
    the first entry whose magnitude is within SIGN_TIE (relative) of the
    largest is positive, so entries equal by symmetry tie whatever rounding
    a solver leaves in them."""
    a = np.abs(c)
    k = int(np.flatnonzero(a >= a.max() * (1.0 - SIGN_TIE))[0])
    return -c if c[k] < 0 else c


def lowest_eigenpairs(h, g, V, k, tol=1e-12, dense_max=3000):
    """The k lowest eigenpairs of H on V in ascending order (several states
    of one determinant space): dense LAPACK below dense_max, else Lanczos
    (scipy eigsh).  Each vector's largest |c_i| (first index on ties) is made
    positive.  Returns (e [k], C [k, m])."""
    m = len(V)
    if not 1 <= k <= m:
        raise ValueError("need 1 <= k <= len(V)")
    if m <= dense_max:
        w, U = np.linalg.eigh(hamiltonian_csr(h, g, V).toarray())
        e, C = w[:k].copy(), U[:, :k].T.copy()
    else:
        import scipy.sparse.linalg as sla
        w, U = sla.eigsh(hamiltonian_csr(h, g, V), k=k, which="SA", tol=tol)
        o = np.argsort(w)
        e, C = w[o].copy(), U[:, o].T.copy()
    C = np.array([_fix_sign(c) for c in C])
    return e, C


def hci(h, g, nalpha, nbeta, eps1, max_iter=20, V0=None, tol=1e-12, dense_max=3000):
    """HCI variational stage: start from the aufbau determinant (or V0), select
    C(eps1), merge, re-diagonalise, until nothing new is added or max_iter."""
    n = h.shape[0]
    if V0 is None:
        V = np.array([[(1 << nalpha) - 1, (1 << nbeta) - 1]], dtype=np.uint64)
    else:
        V = sort_unique(V0)
    e, c = lowest_eigenpair(h, g, V, tol=tol, dense_max=dense_max)
    history = [(len(V), e)]
    for _ in range(max_iter):
        C = select(h, g, V, c, eps1)
        if len(C) == 0:
            break
        Vn = merge(V, C)
        # warm start: previous coefficients placed at their new rows
        pos = np.searchsorted(_keys(Vn), _keys(V))
        v0 = np.zeros(len(Vn))
        v0[pos] = c
        V = Vn
        e, c = lowest_eigenpair(h, g, V, tol=tol, v0=v0, dense_max=dense_max)
        history.append((len(V), e))
    return V, c, e, history


def hci_roots(h, g, nalpha, nbeta, eps1, nroots, V0, max_iter=20, tol=1e-12, dense_max=3000):
    """The variational stage for several states of one space: from V0 (at
    least nroots determinants), V <- V + union of the states' C(eps1), then the
    nroots lowest eigenpairs, until nothing is added or max_iter."""
    V = sort_unique(V0)
    e, C = lowest_eigenpairs(h, g, V, nroots, tol=tol, dense_max=dense_max)
    history = [(len(V), e.copy())]
    for _ in range(max_iter):
        A = select_roots(h, g, V, C, eps1)
        if len(A) == 0:
            break
        V = merge(V, A)
        e, C = lowest_eigenpairs(h, g, V, nroots, tol=tol, dense_max=dense_max)
        history.append((len(V), e.copy()))
    return V, C, e, history


def _keys(V):
    """Structured view for ordered searches over (alpha, beta)."""
    V = np.ascontiguousarray(V, dtype=np.uint64)
    return V.view(np.dtype([("a", np.uint64), ("b", np.uint64)])).ravel()


def find(V, dets) -> np.ndarray:
    """Row index in sorted V of each determinant (-1 if absent)."""
    kv, kd = _keys(V), _keys(np.asarray(dets, np.uint64).reshape(-1, 2))
    pos = np.searchsorted(kv, kd)
    ok = pos < len(kv)
    res = np.full(len(kd), -1, dtype=np.int64)
    res[ok] = np.where(kv[pos[ok]] == kd[ok], pos[ok], -1)
    return res


# ---------------------------------------------------------------- RDMs
def rdm12(n, V, bra, ket) -> Tuple[np.ndarray, np.ndarray]:
    """gamma_pq = sum_s <bra|a+_ps a_qs|ket>,
    Gamma_pqrs = sum_st <bra|a+_ps a+_rt a_st a_qs|ket>, by operator application."""
    V, vp = _u64(V)
    bra, bp = _f64(bra)
    ket, kp = _f64(ket)
    r1 = np.zeros((n, n))
    r2 = np.zeros((n, n, n, n))
    lib().orc_rdm12(n, vp, len(V), bp, kp, r1.ctypes.data_as(f64p), r2.ctypes.data_as(f64p))
    return r1, r2


def rdm2_element(n, V, bra, ket, p, q, r, s) -> float:
    V, vp = _u64(V)
    bra, bp = _f64(bra)
    ket, kp = _f64(ket)
    return lib().orc_rdm2_element(n, vp, len(V), bp, kp, p, q, r, s)


def rdm1_element(n, V, bra, ket, p, q) -> float:
    V, vp = _u64(V)
    bra, bp = _f64(bra)
    ket, kp = _f64(ket)
    return lib().orc_rdm1_element(n, vp, len(V), bp, kp, p, q)


def energy_from_rdms(h, g, r1, r2, ecore=0.0) -> float:
    """E = E_core + sum h_pq gamma_pq + 1/2 sum (pq|rs) Gamma_pqrs."""
    return float(ecore + np.sum(h * r1) + 0.5 * np.sum(g * r2))


def _lib_pt2():
    L = lib()
    if not getattr(L, "_pt2_ready", False):
        L.orc_pt2_pairs.restype = ctypes.c_long
        L.orc_pt2_pairs.argtypes = [ctypes.c_int, f64p, f64p, u64p, ctypes.c_long, f64p,
                                    ctypes.c_double, u64p, i64p, f64p, ctypes.c_long]
        L.orc_pair_rdm_add.restype = None
        L.orc_pair_rdm_add.argtypes = [ctypes.c_int] + [ctypes.c_uint64] * 4 + [ctypes.c_double,
                                                                                f64p, f64p]
        L._pt2_ready = True
    return L


def pt2_pairs(h, g, V, c, eps2):
    """Screened pairs of eq. pt_hci: every (i, a), D_a outside V one excitation
    from D_i, with fl(|H_ai| |c_i|) > eps2.  Returns (a_dets, i, H_ai) in i order."""
    n = h.shape[0]
    h, hp = _f64(h)
    g, gp = _f64(g)
    V, vp = _u64(V)
    c, cp = _f64(c)
    L = _lib_pt2()
    total = L.orc_pt2_pairs(n, hp, gp, vp, len(V), cp, float(eps2), None, None, None, 0)
    a = np.zeros((max(total, 1), 2), dtype=np.uint64)
    idx = np.zeros(max(total, 1), dtype=np.int64)
    hv = np.zeros(max(total, 1))
    L.orc_pt2_pairs(n, hp, gp, vp, len(V), cp, float(eps2), a.ctypes.data_as(u64p),
                    idx.ctypes.data_as(i64p), hv.ctypes.data_as(f64p), total)
    return a[:total], idx[:total], hv[:total]


def pt2(h, g, V, c, e0, eps2):
    """eps2-screened Epstein-Nesbet PT2 on a frozen (V, c, E0): eq. pt_hci with
    the Hylleraas minimiser d_a = N_a / (E0 - H_aa) (eq. hylleraas).

    Returns a dict: C (sorted connected determinants), N, Haa, d, E2,
    r = dE2/dc at fixed E0 (= 2 sum_a M_ai H_ai d_a), and the pair list."""
    a, idx, hv = pt2_pairs(h, g, V, c, eps2)
    C = sort_unique(a)
    pos = find(C, a)
    c = np.asarray(c, dtype=np.float64)
    N = np.zeros(len(C))
    np.add.at(N, pos, hv * c[idx])
    Haa = np.array([diag(h, g, x) for x in C]) if len(C) else np.zeros(0)
    d = N / (e0 - Haa)
    E2 = float(np.sum(N * d))
    r = np.zeros(len(V))
    np.add.at(r, idx, 2.0 * hv * d[pos])
    return dict(C=C, N=N, Haa=Haa, d=d, E2=E2, r=r, pairs=(a, idx, hv, pos))


def pt2_rdms(n, V, c, pt):
    """Gamma^{dc} over the screened pairs (sum d_a c_i <D_a|..|D_i>) and
    Gamma^{dd} = sum_a d_a^2 <D_a|..|D_a> (H0 is diagonal outside V), by
    operator application (Sec. "Computational Details")."""
    L = _lib_pt2()
    a, idx, hv, pos = pt["pairs"]
    d, C = pt["d"], pt["C"]
    dc1, dc2 = np.zeros((n, n)), np.zeros((n, n, n, n))
    for k in range(len(idx)):
        L.orc_pair_rdm_add(n, int(a[k, 0]), int(a[k, 1]), int(V[idx[k], 0]), int(V[idx[k], 1]),
                           float(d[pos[k]] * c[idx[k]]), dc1.ctypes.data_as(f64p),
                           dc2.ctypes.data_as(f64p))
    dd1, dd2 = np.zeros((n, n)), np.zeros((n, n, n, n))
    for k in range(len(C)):
        L.orc_pair_rdm_add(n, int(C[k, 0]), int(C[k, 1]), int(C[k, 0]), int(C[k, 1]),
                           float(d[k] ** 2), dd1.ctypes.data_as(f64p), dd2.ctypes.data_as(f64p))
    return (dc1, dc2), (dd1, dd2)


def zvector_dense(H, c, e0, r):
    """Lagrange multiplier equation (eq. lagc after lambda_d = 0) on c-perp:
    z = -(Q (H - E0) Q)^+ Q r, Q = 1 - c c^T (dense pseudo-inverse)."""
    m = len(c)
    Q = np.eye(m) - np.outer(c, c)
    A = Q @ (H - e0 * np.eye(m)) @ Q
    return -np.linalg.pinv(A, rcond=1e-12) @ (Q @ r)


def relaxed_rdms(n, V, c, e0, z, pt):
    """gamma/Gamma of the relaxed gradient (eq. lambda with lambda_c =
    z/2 - (d.d) c/2): (1 - d.d) G^cc + G^zc + 2 G^dc + G^dd, transition parts
    symmetrised over bra/ket."""
    g1, g2 = rdm12(n, V, c, c)
    z1, z2 = rdm12(n, V, z, c)
    (dc1, dc2), (dd1, dd2) = pt2_rdms(n, V, c, pt)
    dd = float(np.dot(pt["d"], pt["d"]))
    sym1 = lambda x: 0.5 * (x + x.T)  # noqa: E731
    sym2 = lambda x: 0.5 * (x + x.transpose(1, 0, 3, 2))  # noqa: E731
    r1 = (1 - dd) * g1 + sym1(z1) + 2 * sym1(dc1) + dd1
    r2 = (1 - dd) * g2 + sym2(z2) + 2 * sym2(dc2) + dd2
    return r1, r2


def symmetrize8(t) -> np.ndarray:
    """Average of a 4-index tensor over the 8 real-orbital integral symmetries."""
    perms = [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2),
             (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]
    return sum(np.transpose(t, p) for p in perms) / 8.0


def pt2_sample(c, u):
    """Multiplicities of the draws of eq. semistoc's sampled estimate: integer
    weights q_i = max(1, round(2^31 |c_i| / max|c|)) for c_i != 0 (0 for
    c_i = 0), Q = sum q, draw k picks the row i with
    Q_<i <= min(Q - 1, floor(u_k Q)) < Q_<i + q_i.  Returns (w, q, Q)."""
    c = np.asarray(c, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    cabs = np.abs(c)
    cmax = float(cabs.max())
    q = np.zeros(len(c), dtype=np.int64)
    nz = cabs > 0
    q[nz] = np.maximum(1, np.floor(np.ldexp(cabs[nz] / cmax, 31) + 0.5)).astype(np.int64)
    Q = int(q.sum())
    before = np.concatenate([[0], np.cumsum(q)[:-1]])
    t = np.minimum(Q - 1, np.floor(u * float(Q)).astype(np.int64))
    rows = np.searchsorted(before, t, side="right") - 1
    w = np.bincount(rows, minlength=len(c)).astype(np.int64)
    return w, q, Q


def pt2_stochastic_counts(h, g, V, c, e0, eps_list, w, p, nd):
    """Sampled estimate of eq. pt_hci for given multiplicities w_i of nd draws
    with probabilities p_i, one value per threshold in eps_list (every
    threshold on the same draws): sum_a [S1^2 - S2 + (nd - 1) S3] /
    (nd (nd - 1) (E0 - H_aa)) over the screened pairs of the drawn rows."""
    c = np.asarray(c, dtype=np.float64)
    w = np.asarray(w)
    cs = np.where(w > 0, c, 0.0)  # only drawn rows produce pairs
    a, idx, hv = pt2_pairs(h, g, V, cs, min(eps_list))
    out = []
    for eps in eps_list:
        keep = np.abs(hv) * np.abs(c[idx]) > eps
        ak, ik, hk = a[keep], idx[keep], hv[keep]
        if len(ik) == 0:
            out.append(0.0)
            continue
        C = sort_unique(ak)
        pos = find(C, ak)
        x = hk * c[ik]
        wp = w[ik] / p[ik]
        S1, S2, S3 = np.zeros(len(C)), np.zeros(len(C)), np.zeros(len(C))
        np.add.at(S1, pos, wp * x)
        np.add.at(S2, pos, (wp * x) ** 2)
        np.add.at(S3, pos, wp * x * x)
        Haa = np.array([diag(h, g, y) for y in C])
        T = (S1 ** 2 - S2 + (nd - 1) * S3) / (nd * (nd - 1))
        out.append(float(np.sum(T / (e0 - Haa))))
    return out


def pt2_stochastic(h, g, V, c, e0, eps2, eps2_d, u):
    """One batch (len(u) draws): the sampled estimates E2^S(eps2) and
    E2^S(eps2_d) of eq. semistoc from the same draws."""
    w, q, Q = pt2_sample(c, u)
    p = q / float(Q)
    return tuple(pt2_stochastic_counts(h, g, V, c, e0, [eps2, eps2_d], w, p, len(u)))


def semistochastic_combine(e2d, per):
    """eq. semistoc from its pieces: E2^D(eps2_d) plus the mean over batches
    of the bracket [E2^S(eps2) - E2^S(eps2_d)] (both terms of a batch from
    the same draws), and the standard error of that mean, i.e. the sample
    standard deviation of the brackets (n_b - 1 in the denominator) over
    sqrt(n_b); nan for one batch.  per: [(E2^S(eps2), E2^S(eps2_d)), ...]."""
    diff = np.array([x - y for x, y in per], dtype=np.float64)
    nb = len(diff)
    mean = float(np.sum(diff) / nb)
    if nb > 1:
        var = float(np.sum((diff - mean) ** 2) / (nb - 1))
        err = float(np.sqrt(var) / np.sqrt(nb))
    else:
        err = float("nan")
    return e2d + mean, err


def pt2_semistochastic(h, g, V, c, e0, eps2, eps2_d, u_batches):
    """eq. semistoc: E2^D(eps2_d) + mean over batches of
    [E2^S(eps2) - E2^S(eps2_d)]; returns (E2, standard error of the mean
    (nan for one batch), E2^D(eps2_d), per-batch pairs)."""
    e2d = pt2(h, g, V, c, e0, eps2_d)["E2"]
    per = [pt2_stochastic(h, g, V, c, e0, eps2, eps2_d, u) for u in u_batches]
    e2, err = semistochastic_combine(e2d, per)
    return e2, err, e2d, per


def orbital_gradient(h, g, rdm1, rdm2):
    """dE/dkappa for active-active rotations (antisymmetric [n][n], entry
    (x, y) the derivative along kappa_xy = -kappa_yx): 2 (F - F^T) with
    F_xy = sum_r h_xr gamma_ry + sum_qrs (xq|rs) Gamma_yqrs."""
    F = np.asarray(h) @ np.asarray(rdm1) + np.einsum("xqrs,yqrs->xy", g, rdm2)
    return 2.0 * (F - F.T)


def rotate_integrals(h, g, U):
    """h' = U^T h U and (pq|rs)' = sum_abcd U_ap U_bq U_cr U_ds (ab|cd)."""
    U = np.asarray(U, dtype=np.float64)
    h2 = U.T @ np.asarray(h) @ U
    g2 = np.einsum("abcd,ap,bq,cr,ds->pqrs", g, U, U, U, U, optimize=True)
    return h2, g2


def extrapolation_ranking(c):
    """Determinant indices by decreasing |c_i| (ties: increasing index)."""
    c = np.asarray(c, dtype=np.float64)
    return np.lexsort((np.arange(len(c)), -np.abs(c)))


def extrapolation_sizes(n, fraction, levels):
    """m_0 = n, m_k = max(1, ceil(m_{k-1} (1 - fraction)))."""
    import math
    m = [int(n)]
    for _ in range(1, levels):
        m.append(max(1, math.ceil(m[-1] * (1.0 - fraction))))
    return m


def extrapolation_fit(e2, etot):
    """Least-squares line etot = a + b e2: (a, b), written out."""
    x = np.asarray(e2, dtype=np.float64)
    y = np.asarray(etot, dtype=np.float64)
    xm, ym = x.mean(), y.mean()
    b = float(np.sum((x - xm) * (y - ym)) / np.sum((x - xm) ** 2))
    return float(ym - b * xm), b


def extrapolation(h, g, V, c, fraction, levels, eps2):
    """Levels of the extrapolation: nested spaces ranked by the given c, each
    level's lowest eigenpair and its screened E2; the line through
    (E2, E_var + E2) at E2 = 0.  Returns dict(sizes, evar, e2, e_extrap,
    slope, error)."""
    V = np.asarray(V)
    order = extrapolation_ranking(c)
    sizes = extrapolation_sizes(len(V), fraction, levels)
    evar, e2 = [], []
    for m in sizes:
        Vk = V[np.sort(order[:m])]
        e, ck = lowest_eigenpair(h, g, Vk)
        evar.append(e)
        e2.append(pt2(h, g, Vk, ck, e, eps2)["E2"])
    a, b, err = extrapolation_assemble(evar, e2)
    return dict(sizes=sizes, evar=np.array(evar), e2=np.array(e2), e_extrap=a, slope=b,
                error=err)


def extrapolation_assemble(evar, e2):
    """The extrapolation from the levels' energies (Sec. "Results and
    discussion": the total energy E_var + E2 of each level against its E2,
    a straight line taken to E2 = 0; the Fe-porphyrin table's error bar is a
    quarter of the distance from the extrapolated energy to the most accurate
    total energy, that of level 0).  Returns (a, b, error) of the
    least-squares line E_var + E2 = a + b E2."""
    evar = np.asarray(evar, dtype=np.float64)
    e2 = np.asarray(e2, dtype=np.float64)
    etot = evar + e2
    a, b = extrapolation_fit(e2, etot)
    return a, b, 0.25 * abs(a - float(etot[0]))
