"""Benchmark of the Heat-bath CI variational step on one MI355X.

Workload: the (16e,16o) synthetic active space (seed 1, L = 48) at
eps1 = 1e-4.  Set-up (untimed) runs the first two HCI macro-iterations from
the aufbau determinant, giving V1 (5,793 determinants) and its ground state
c1.  One timed step is the next full variational macro-iteration, from
(V1, c1) resident in HBM:

  select   V2 = V1 + C(eps1)                      (1,138,281 determinants)
  build    buckets, adjacency, stored Hamiltonian (connectivity + elements)
  Davidson lowest eigenpair on V2 (float32-mixed products, float64
           refinement), residual tol 1e-5
  backward one- and two-particle density matrices -> dE/dh, dE/dg

Every cache of the library is released at the start of a step, so nothing
built by a previous step is reused.  The reported value is whole-step
throughput: Hamiltonian-product det-pairs processed per second of step time
(pairs = ordered (i, j) in V2 x V2 at excitation degree <= 2, diagonal
included).  Beside it: Davidson iterations per second, the same step in the
all-float64 path, the energy difference between the two, the product
kernel's HBM roofline fraction and the CPU oracle's throughput on a sample
of rows.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sigma det-pairs/s + Davidson iter/s, FP32-mixed vs FP64 at ≤1e-6 Ha error"
HBM_PEAK_GBS = 8000.0
MFMA_F64_PEAK_TFLOPS = 78.6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--cold-davidson", type=int, default=1,
                    help="time a mixed-precision Davidson from a cold start on the final space (0 skips it)")
    ap.add_argument("--cas8", type=int, default=1,
                    help="time the (8e,8o) full-CI workload on the GPU and in the oracle (0 skips it)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU oracle legs and the copy-peak probe")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy a 4 GiB buffer once (calibrates HBM byte counters)")
    ap.add_argument("--pt2-batches", type=int, default=16,
                    help="batches of the semistochastic PT2 leg (0: skip the leg)")
    ap.add_argument("--pt2-samples", type=int, default=2000, help="draws per PT2 batch")
    ap.add_argument("--pt2-eps2", type=float, default=1e-6, help="sampled PT2 threshold")
    ap.add_argument("--pt2-eps2d", type=float, default=1e-4, help="deterministic PT2 threshold")
    ap.add_argument("--extrap-levels", type=int, default=3,
                    help="levels of the full-CI extrapolation leg on the final space (0: skip it)")
    ap.add_argument("--orbital-reps", type=int, default=20,
                    help="timed repetitions of the orbital-step leg (0: skip it)")
    ap.add_argument("--recompute-reps", type=int, default=2,
                    help="products timed in recompute mode on the final space (0 skips it)")
    ap.add_argument("--roots", type=int, default=3,
                    help="states of the several-state leg (0 skips it)")
    ap.add_argument("--pt2-cpu-rows", type=int, default=2000,
                    help="rows of the final space the oracle's PT2 pair walk times")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the multi-GPU "
              "sharding of this path is a design, not a measured configuration.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import hci_synth as hs
    import paper_1708_07544_amd as P

    w = hs.WORKLOADS["cas16"]
    h, g = hs.workload_integrals(w)
    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy probe: 4 GiB read + 4 GiB written by one copy kernel")
        del src, dst
    ctx = P.HCIContext(h, g, w.nalpha, w.nbeta)
    # ---------------------------------------------------------------- set-up
    V0 = P.dets_to_device(hs.aufbau_det(w.nalpha, w.nbeta))
    e0, c0, _ = ctx.davidson(V0, None, tol=args.tol)
    V1 = ctx.select(V0, c0, w.eps1)
    e1, c1, _ = ctx.davidson(V1, ctx.embed(V0, c0, V1), tol=args.tol)
    log(f"[bench] set-up: |V1| = {V1.shape[0]}, E1 = {e1:.10f}")

    def step(precision):
        ctx.release_cache()
        V2 = ctx.select(V1, c1, w.eps1)
        cs = ctx.embed(V1, c1, V2)
        e, c, products = ctx.davidson(V2, cs, tol=args.tol, precision=precision, max_iter=2000)
        dh, dg, _, _ = ctx.energy_backward(V2, c, e)
        return V2, e, c, products, (dh, dg)

    for k in range(args.warmup):
        V2, e, c, products, _ = step("fp32_mixed")
        log(f"[bench] warmup {k}: |V2| = {V2.shape[0]}, E = {e:.10f}, products = {products}")
    # ---------------------------------------------------------------- timed
    ctx.set_timing(True)
    ctx.kernel_time("x", reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_products = 0
    for k in range(args.steps):
        V2, e_mixed, c_mixed, products, grads = step("fp32_mixed")
        total_products += products
        log(f"[bench] step {k}: E = {e_mixed:.10f}, products = {products}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    kernels = {}
    for name in ["sigma_stored_f32", "sigma_stored_f32_g", "sigma_stored_f64", "sigma_stored_f64_g",
                 "sigma_recompute_f64", "select_walk", "csr_cols", "csr_vals_f32", "csr_vals_f64",
                 "conn_count", "rdm_offdiag", "dv_eig", "dv_dots", "dv_combine"]:
        n_, ms = ctx.kernel_time(name)
        if n_:
            kernels[name] = {"launches": n_, "avg_ms": ms / n_, "total_ms_per_step": ms / args.steps}
    ctx.set_timing(False)
    nv = int(V2.shape[0])
    pairs = ctx.connections(V2)                      # diagonal included
    nnz_off = pairs - nv
    layout = ctx.layout_info(V2)
    value = total_products * pairs / (t1 - t0)
    # ---------------------------------------------------------------- fp64 path
    fp64 = None
    if args.fp64_steps > 0:
        ctx.set_timing(True)
        ctx.kernel_time("x", reset=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        p64 = 0
        for k in range(args.fp64_steps):
            _, e64, c64, products64, grads64 = step("fp64")
            p64 += products64
            log(f"[bench] fp64 step {k}: E = {e64:.10f}, products = {products64}")
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        n64, ms64 = ctx.kernel_time("sigma_stored_f64")
        ng64, msg64 = ctx.kernel_time("sigma_stored_f64_g")
        if n64:
            ms64 = ms64 + (msg64 / ng64 * n64 if ng64 else 0.0)   # per product: both kernels
        ctx.set_timing(False)
        fp64 = {
            "ms_per_step": (t3 - t2) * 1e3 / args.fp64_steps,
            "value": p64 * pairs / (t3 - t2),
            "products_per_step": p64 / args.fp64_steps,
            "sigma_kernel_avg_ms": ms64 / max(n64, 1),
            "sigma_kernel_pairs_per_s": pairs / (ms64 / max(n64, 1) / 1e3) if n64 else None,
            "energy": e64,
            # density-matrix difference of the two paths (dE/dh = gamma, dE/dg = Gamma/2 sym.)
            "gamma_max_abs_diff": float((grads[0] - grads64[0]).abs().max()),
            "Gamma_max_abs_diff": float(2.0 * (grads[1] - grads64[1]).abs().max()),
        }
    # ---------------------------------------------------------------- PT2
    pt2 = None
    if args.pt2_batches > 0:
        pt2 = pt2_leg(ctx, h, g, V2, c_mixed, e_mixed, args)
    extrap = None
    if args.extrap_levels >= 2:
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        r = ctx.extrapolate(V2, c_mixed, fraction=0.33, levels=args.extrap_levels, eps2=args.pt2_eps2d,
                            tol=args.tol, precision="fp32_mixed")
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        extrap = {"levels": args.extrap_levels, "fraction": 0.33, "eps2": args.pt2_eps2d,
                  "sizes": r["sizes"], "evar": [float(x) for x in r["evar"]], "e2": [float(x) for x in r["e2"]],
                  "e_extrap": r["e_extrap"], "slope": r["slope"], "error": r["error"],
                  "seconds": round(t5 - t4, 3)}
        log(f"[bench] extrapolation: {r['sizes']} -> {r['e_extrap']:.8f} +- {r['error']:.2e} "
            f"({t5 - t4:.2f} s)")
    orbital = None
    if args.orbital_reps > 0:
        orbital = orbital_leg(args)
    recompute = None
    if args.recompute_reps > 0:
        recompute = recompute_leg(ctx, V2, c_mixed, pairs, args)
    roots = None
    if args.roots > 1:
        roots = roots_leg(ctx, V1, c1, V2, c_mixed, w.eps1, args)
    # ---------------------------------------------------------------- roofline
    sk = kernels.get("sigma_stored_f32")
    gk = kernels.get("sigma_stored_f32_g")
    roofline = None
    product_ms = None
    if sk:
        product_ms = sk["avg_ms"] + (gk["avg_ms"] if gk else 0.0)
        if layout["layout"] == 2:
            # alpha-bucket-staged layout, dominant kernel (all but the
            # beta-group segments): float32 value + u16 column per stored
            # entry, 4 B per entry of c copied to LDS, 48 B per row (row
            # pointer, segment base and starts, c_i, H_ii, sigma_i)
            s_entries = layout["stored_entries"] - layout["group_entries"]
            alg_bytes = 6 * s_entries + 4 * layout["staged_c_entries"] + 48 * nv
        else:
            # plain CSR: float32 value + u32 column per stored entry, 32 B per row
            alg_bytes = 8 * layout["stored_entries"] + 32 * nv
        # algorithmic bytes of the scope table: float32 value + u32 column =
        # 8 B per connection, ~24 B per row (row pointer, c_i, sigma_i), over
        # the connections of this kernel (all but the beta-group segments)
        conns = nnz_off - layout["group_entries"]
        survey_bytes = 8 * conns + 24 * nv
        achieved = survey_bytes / (sk["avg_ms"] * 1e-3) / 1e9
        achieved_fmt = alg_bytes / (sk["avg_ms"] * 1e-3) / 1e9
        traffic = measured_traffic(nv)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic,
                    "traffic_source": ("replayed from profiles/sigma_stored_f32_cas16_traffic.json "
                                       "(FETCH_SIZE and WRITE_SIZE runs of the same kernel source on "
                                       "this space; not counted in this run)") if traffic else None,
                    "kernel": "sigma_stored_f32", "bytes_per_launch": survey_bytes,
                    "bytes_rule": "8 B per connection + 24 B per row (connections = off-diagonal "
                                  "pairs minus beta-group entries)",
                    "format": {"bytes_per_launch": alg_bytes, "achieved": round(achieved_fmt, 1),
                               "frac": round(achieved_fmt / HBM_PEAK_GBS, 4),
                               "rule": "6 B per stored entry (f32 value + u16 column, padding "
                                       "included) + 4 B per staged c entry + 48 B per row"},
                    "avg_launch_ms": round(sk["avg_ms"], 4)}
    # ---------------------------------------------------------------- CPU oracle
    cpu = None
    oracle_check = None
    if not args.no_cpu:
        cpu, oracle_check = cpu_baseline(h, g, P.dets_to_numpy(V2), c_mixed.cpu().numpy(), e_mixed, nv, pairs)
    copy_peak = None
    cpu_rows = None
    if not args.no_cpu:
        copy_peak = copy_peak_leg()
        if roofline:
            # the bytes the format moves (not the scope table's larger count)
            # against what a plain copy reaches on this GPU
            roofline["copy_peak_gbs"] = round(copy_peak, 1)
            roofline["format"]["frac_of_copy"] = round(roofline["format"]["achieved"] / copy_peak, 4)
        cpu_rows = cpu_rows_leg(h, g, P.dets_to_numpy(V2), c_mixed.cpu().numpy(), cpu)
    cold = None
    if args.cold_davidson:
        cold = cold_leg(ctx, V2, pairs, args)
        if cpu_rows is not None:
            # the full oracle HCI on this space: as many of the oracle's products
            # as the library's cold solve needs, at the timed rate, plus selection
            cpu_rows["oracle_hci_cas16"] = {
                "run": False, "estimate_s": round(cold["products"] * pairs / cpu["value"], 1),
                "reason": "not run: a solve takes about %d oracle products of %.1f s each on %d threads"
                          % (cold["products"], pairs / cpu["value"], cpu["cores"])}
    small = None
    if args.cas8:
        small = cas8_leg(args)
    torch.cuda.synchronize()
    t6 = time.perf_counter()
    s2 = ctx.spin_square(V2, c_mixed)
    s2_ms = (time.perf_counter() - t6) * 1e3
    log(f"[bench] <S^2> of the final state: {s2:.6f} ({s2_ms:.1f} ms)")
    dav_time_ms = None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "det-pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32_mixed",
        "data": "synthetic",
        "config": {"workload": "cas16: (16e,16o) synthetic integrals seed 1 L=48, eps1=1e-4, "
                               "HCI macro-iteration 5793 -> %d determinants, Davidson tol %g"
                               % (nv, args.tol),
                   "n_det": nv, "det_pairs": pairs, "norb": w.norb, "nelec": w.nalpha + w.nbeta},
        "davidson_iter_per_s": total_products / (t1 - t0),
        "products_per_step": total_products / args.steps,
        "sigma_product_ms": product_ms,
        "sigma_kernel_pairs_per_s": pairs / (product_ms * 1e-3) if product_ms else None,
        "sigma_speedup_vs_fp64": (fp64["sigma_kernel_avg_ms"] / product_ms)
        if (fp64 and product_ms) else None,
        "layout": layout,
        "energy": e_mixed,
        "spin_square": {"value": s2, "ms": round(s2_ms, 2)},
        "fp64": fp64,
        "energy_error_vs_fp64": abs(e_mixed - fp64["energy"]) if fp64 else None,
        "energy_vs_oracle": oracle_check,
        "davidson_cold": cold,
        "cas8": small,
        "host_cpu": cpu_model(),
        "speedup_vs_fp64": (fp64["ms_per_step"] / ms_step) if fp64 else None,
        "kernels": kernels,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_oracle_rows": cpu_rows,
        "pt2": pt2,
        "orbital": orbital,
        "extrapolation": extrap,
        "roots": roots,
        "recompute": recompute,
    }
    del dav_time_ms
    print(json.dumps(out))


def recompute_leg(ctx, V2, c, pairs, args):
    """The product with connections and elements regenerated in every call
    (the mode of spaces whose Hamiltonian exceeds the memory budget), timed
    on the final space after one untimed call."""
    import torch
    out = {"reps": args.recompute_reps, "det_pairs": pairs}
    for precision in ("fp32_mixed", "fp64"):
        ctx.sigma(V2, c, precision=precision, mode="recompute")
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.recompute_reps):
            ctx.sigma(V2, c, precision=precision, mode="recompute")
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / args.recompute_reps
        out[precision] = {"ms": round(ms, 2), "det_pairs_per_s": pairs / (ms * 1e-3)}
    log(f"[bench] recomputed product on {V2.shape[0]} determinants: "
        f"{out['fp32_mixed']['ms']:.1f} ms mixed, {out['fp64']['ms']:.1f} ms f64")
    return out


def roots_leg(ctx, V1, c1, V2, c2, eps1, args):
    """Several states: the lowest args.roots states on V1 (float64), the
    union selection of V1 over them against the single-state selection, and
    the lowest states on the step's space V2 (mixed precision, state 0 warm
    started from the step's vector)."""
    import torch
    k = args.roots
    e1, C1, _ = ctx.davidson_roots(V1, k, tol=args.tol)

    def timed(f):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = f()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t) * 1e3

    single, ms_single = timed(lambda: ctx.select(V1, c1, eps1))
    union, ms_union = timed(lambda: ctx.select(V1, C1, eps1))
    del single, union
    C0 = torch.zeros((k, V2.shape[0]), dtype=torch.float64, device=V2.device)
    C0[0] = c2
    (e2, C2, its), ms = timed(lambda: ctx.davidson_roots(V2, k, c0=C0, tol=args.tol,
                                                         precision="fp32_mixed", max_iter=2000))
    # davidson_ms includes building the stored Hamiltonian of V2, as the step does
    out = {"states": k, "energies": [float(x) for x in e2], "products": its,
           "spin_square": [round(ctx.spin_square(V2, C2[r]), 8) for r in range(k)],
           "davidson_ms": round(ms, 2), "n_det": int(V2.shape[0]),
           "select_single_ms": round(ms_single, 2), "select_union_ms": round(ms_union, 2),
           "n_select_single": int(ctx.select(V1, c1, eps1).shape[0]),
           "n_select_union": int(ctx.select(V1, C1, eps1).shape[0])}
    log(f"[bench] {k} states on {out['n_det']} determinants: {out['energies']} "
        f"({ms:.1f} ms, products {its}); union selection {out['n_select_union']} in {ms_union:.1f} ms "
        f"vs single {out['n_select_single']} in {ms_single:.1f} ms")
    return out


PT2_KERNELS = ["pt2_count", "pt2_fill_pairs", "radix_hist", "radix_scatter", "pt2_reduce", "pt2_r",
               "pt2_insert_v", "pt2_segflags", "pt2_segstarts", "pt2_sum", "pt2s_weights", "pt2s_draw",
               "pt2s_reduce"]


def pt2_leg(ctx, h, g, V2, c, e, args):
    """Second-order energy on the final space (eq. semistoc): the screened E2
    at eps2_d in one call, then the semistochastic total (which repeats the
    deterministic part and adds the batches of draws at eps2); beside it the
    oracle's screened-pair walk timed on a bounded random sample of rows."""
    import numpy as np
    import torch

    import paper_1708_07544_amd as P

    nb, nd = args.pt2_batches, args.pt2_samples
    rng = np.random.default_rng(17)
    u = rng.random((nb, nd))
    ctx.pt2_stochastic(V2, c, e, args.pt2_eps2, args.pt2_eps2d, u[:1])  # warm-up
    ctx.set_timing(True)
    ctx.kernel_time("x", reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e2d, _, nconn = ctx.pt2(V2, c, e, args.pt2_eps2d, want_r=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    e2, err, _ = ctx.pt2_semistochastic(V2, c, e, args.pt2_eps2, args.pt2_eps2d, u)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    kern = {}
    for name in PT2_KERNELS:
        n_, ms = ctx.kernel_time(name)
        if n_:
            kern[name] = {"launches": n_, "total_ms": round(ms, 3)}
    ctx.kernel_time("x", reset=True)
    ctx.set_timing(False)
    nv = int(V2.shape[0])
    det_ms = (t1 - t0) * 1e3
    stoch_ms = (t2 - t1) * 1e3 - det_ms
    log(f"[bench] pt2: E2^D({args.pt2_eps2d:g}) = {e2d:.10f} ({det_ms:.1f} ms), "
        f"E2({args.pt2_eps2:g}) = {e2:.10f} +- {err:.2e}")
    out = {"eps2": args.pt2_eps2, "eps2_d": args.pt2_eps2d, "samples_per_batch": nd, "batches": nb,
           "e2": e2, "e2_stderr": err, "e2_deterministic": e2d, "connected_dets_deterministic": nconn,
           "ms_deterministic": round(det_ms, 2), "ms_per_batch": round(stoch_ms / nb, 3),
           "rows_per_s_deterministic": nv / (det_ms * 1e-3), "kernels": kern}
    if not args.no_cpu and args.pt2_cpu_rows > 0:
        import oracle as O
        Vh = P.dets_to_numpy(V2)
        ch = c.cpu().numpy()
        rows = np.sort(np.random.default_rng(18).choice(nv, args.pt2_cpu_rows, replace=False))
        cs = np.zeros_like(ch)
        cs[rows] = ch[rows]
        t3 = time.perf_counter()
        O.pt2_pairs(h, g, Vh, cs, args.pt2_eps2d)
        dt = time.perf_counter() - t3
        out["cpu_oracle"] = {"rows_per_s": len(rows) / dt, "cores": 1, "kind": "oracle",
                             "sample": f"{len(rows)} random rows of the {nv}-determinant space, "
                                       f"oracle screened-pair walk at eps2 = {args.pt2_eps2d:g} "
                                       f"(every excitation evaluated, count and fill walks), "
                                       f"{dt:.1f} s"}
    return out


def orbital_leg(args):
    """Orbital step at (44e,44o) size: gradient dE/dkappa (an n x n^3 by n^3 x n
    float64 product) and the rotated integrals (four n^3 x n by n x n
    products), timed by the library's events; beside them the oracle's numpy
    contractions of the same definitions."""
    import numpy as np
    import scipy.linalg
    import torch

    import hci_synth as hs
    import paper_1708_07544_amd as P

    w = hs.WORKLOADS["cas44"]
    h, g = hs.workload_integrals(w)
    n = w.norb
    ctx = P.HCIContext(h, g, w.nalpha, w.nbeta)
    rng = np.random.default_rng(44)
    r1 = rng.normal(size=(n, n))
    r1 = r1 + r1.T
    r2 = rng.normal(size=(n, n, n, n))
    r2 = r2 + r2.transpose(2, 3, 0, 1)
    r2 = r2 + r2.transpose(1, 0, 3, 2)
    k = rng.normal(scale=0.1, size=(n, n))
    U = scipy.linalg.expm(k - k.T)
    r1d = torch.as_tensor(r1, device="cuda")
    r2d = torch.as_tensor(r2, device="cuda")
    Ud = torch.as_tensor(U, device="cuda")
    ctx.orbital_gradient(r1d, r2d)
    ctx.rotate_integrals(Ud)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ctx.kernel_time("x", reset=True)
    for _ in range(args.orbital_reps):
        ctx.orbital_gradient(r1d, r2d)
        ctx.rotate_integrals(Ud)
    torch.cuda.synchronize()
    ng, msg = ctx.kernel_time("orb_gradient")
    nr, msr = ctx.kernel_time("orb_rotate")
    ctx.kernel_time("x", reset=True)
    ctx.set_timing(False)
    ctx.close()
    grad_ms = msg / args.orbital_reps
    rot_ms = msr / args.orbital_reps
    grad_flops = 2.0 * n ** 5 + 4.0 * n ** 3
    rot_flops = 4 * 2.0 * n ** 5 + 2 * 2.0 * n ** 3
    rot_bytes = 4 * 16.0 * n ** 4 + 2 * 16.0 * n ** 2 + 8.0 * n ** 2
    t0 = time.perf_counter()
    O_grad_s = None
    import oracle as O
    O.orbital_gradient(h, g, r1, r2)
    t1 = time.perf_counter()
    O.rotate_integrals(h, g, U)
    t2 = time.perf_counter()
    O_grad_s = t1 - t0
    rot_tflops = rot_flops / (rot_ms * 1e-3) / 1e12
    rot_gbs = rot_bytes / (rot_ms * 1e-3) / 1e9
    log(f"[bench] orbital n={n}: gradient {grad_ms:.4f} ms, rotation {rot_ms:.4f} ms")
    return {"n": n, "gradient_ms": round(grad_ms, 4), "rotate_ms": round(rot_ms, 4),
            "gradient_tflops": round(grad_flops / (grad_ms * 1e-3) / 1e12, 3),
            "rotate_tflops": round(rot_tflops, 3),
            "roofline": {"kernel": "quarter transforms of the rotation (4 per call)", "bound": "hbm",
                         "achieved": round(rot_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(rot_gbs / HBM_PEAK_GBS, 4),
                         "mfma_f64_frac": round(rot_tflops / MFMA_F64_PEAK_TFLOPS, 4),
                         "bytes_per_call": rot_bytes, "flops_per_call": rot_flops},
            "cpu_oracle": {"gradient_ms": round(O_grad_s * 1e3, 2), "rotate_ms": round((t2 - t1) * 1e3, 2),
                           "kind": "oracle", "sample": "numpy einsum of the same definitions, one call each"}}


def measured_traffic(nv):
    """HBM bytes per launch of the float32 stored product from the committed
    FETCH_SIZE/WRITE_SIZE counter runs (scaled by a plain 4 GiB copy), or None
    when the kernel sources changed since the counters were taken or the
    space differs from the one they were taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "sigma_stored_f32_cas16_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except OSError:
        return None
    digest = hashlib.sha256()
    for name in rec.get("source_files", []):
        with open(os.path.join(ROOT, name), "rb") as f:
            digest.update(f.read())
    if digest.hexdigest() != rec.get("source_sha256") or rec.get("n_det") != nv:
        return None
    return round(rec["traffic_bytes_per_launch"])


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(h, g, V, c, e, nv, pairs):
    """The oracle's Hamiltonian product (every excitation of each row looked
    up in V by binary search, Slater-Condon elements) over every row of the
    final space, timed on this host's cores (OpenMP threads); the same
    product gives the Rayleigh quotient and residual of the library's
    float32-mixed eigenvector in float64, i.e. its energy error against the
    float64 oracle."""
    import numpy as np

    import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    sig = O.sigma(h, g, V, c)
    dt = time.perf_counter() - t0
    rq = float(c @ sig / (c @ c))
    res = float(np.linalg.norm(sig - rq * c))
    log(f"[bench] cpu oracle: every row ({nv}) in {dt:.1f} s on {threads} threads; "
        f"E_oracle(c) = {rq:.12f}, |E - E_oracle| = {abs(e - rq):.2e}, residual {res:.2e}")
    base = {"value": pairs / dt, "unit": "det-pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole {nv}-determinant final space ({pairs} det-pairs, one product), "
                      f"oracle sigma_i by full excitation enumeration + binary search, {dt:.1f} s",
            "rows_per_s": nv / dt, "cpu_model": cpu_model()}
    check = {"energy_library": e, "energy_oracle_rayleigh": rq, "abs_error": abs(e - rq),
             "oracle_residual_norm": res}
    return base, check


def copy_peak_leg():
    """A plain device copy of 4 GiB (one read and one write stream) timed with
    events: the bandwidth a streaming kernel reaches on this GPU."""
    import torch
    src = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(10):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del src, dst
    gbs = 2 * (4 << 30) / (best * 1e-3) / 1e9
    log(f"[bench] copy peak: 4 GiB copied in {best:.3f} ms, {gbs:.0f} GB/s")
    return gbs


def cpu_rows_leg(h, g, V2, c2, base):
    """The oracle's product on sampled rows: the (16e,16o) final space with one
    thread (against the all-core rate of cpu_baseline), and the first spaces
    of the (30e,30o) and porphyrin-shaped (44e,44o) workloads (aufbau + C(eps1)
    by the oracle's selection) with all threads, as rows per second."""
    import ctypes

    import numpy as np

    import hci_synth as hs
    import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    gomp = None
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        pass
    rng = np.random.default_rng(7)
    out = {"cores": threads}
    if gomp is not None:
        rows = rng.choice(len(V2), 2000, replace=False)
        gomp.omp_set_num_threads(1)
        t = time.perf_counter()
        O.sigma(h, g, V2, c2, rows=rows)
        dt = time.perf_counter() - t
        gomp.omp_set_num_threads(threads)
        out["cas16_single_thread_rows_per_s"] = 2000 / dt
        out["cas16_all_threads_rows_per_s"] = base["rows_per_s"] if base else None
        log(f"[bench] cpu oracle (16e,16o): 2000 rows on one thread in {dt:.2f} s")
    for name, nrows in (("cas30", 1000), ("cas44", 200)):
        w = hs.WORKLOADS[name]
        hh, gg = hs.workload_integrals(w)
        V0 = hs.aufbau_det(w.nalpha, w.nbeta)
        V = O.merge(V0, O.select(hh, gg, V0, np.array([1.0]), w.eps1))
        c = hs.random_coeffs(len(V), 11)
        rows = rng.choice(len(V), nrows, replace=False)
        t = time.perf_counter()
        _, npairs = O.sigma(hh, gg, V, c, rows=rows, with_pairs=True)
        dt = time.perf_counter() - t
        out[name] = {"n_det": len(V), "rows": nrows, "rows_per_s": nrows / dt,
                     "det_pairs_per_s": float(np.sum(npairs)) / dt, "threads": threads}
        log(f"[bench] cpu oracle {name}: {nrows} of {len(V)} rows in {dt:.2f} s on {threads} threads")
    return out


def cold_leg(ctx, V2, pairs, args):
    """Davidson iterations per second from a cold start (zero start vector:
    the lowest-diagonal determinant) on the final space, float32-mixed with
    float64 refinement, the stored Hamiltonian already built."""
    import torch
    ctx.davidson(V2, None, tol=1e-2, precision="fp32_mixed", max_iter=2, allow_noconv=True)  # layout built, untimed
    torch.cuda.synchronize()
    t = time.perf_counter()
    e, c, products = ctx.davidson(V2, None, tol=args.tol, precision="fp32_mixed", max_iter=4000)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    log(f"[bench] cold Davidson: {products} products in {dt:.2f} s, E = {e:.10f}")
    return {"products": products, "seconds": round(dt, 3), "iter_per_s": products / dt,
            "det_pairs_per_s": products * pairs / dt, "energy": e, "tol": args.tol}


def cas8_leg(args):
    """(8e,8o) at eps1 = 0 (the full 4,900-determinant space): the library's
    HCI loop from the aufbau determinant in float64 (Davidson tol 1e-10)
    against the oracle's whole HCI (selection by definition and dense LAPACK
    eigensolves), both timed."""
    import numpy as np
    import torch

    import hci_synth as hs
    import oracle as O
    import paper_1708_07544_amd as P
    w = hs.WORKLOADS["cas8"]
    h, g = hs.workload_integrals(w)
    ctx = P.HCIContext(h, g, 4, 4)
    torch.cuda.synchronize()
    t = time.perf_counter()
    V = P.dets_to_device(hs.aufbau_det(4, 4))
    e, c, _ = ctx.davidson(V, None, tol=1e-10)
    for it in range(20):
        Vn = ctx.select(V, c, 0.0)
        if Vn.shape[0] == V.shape[0]:
            break
        e, c, _ = ctx.davidson(Vn, ctx.embed(V, c, Vn), tol=1e-10)
        V = Vn
    torch.cuda.synchronize()
    gpu_s = time.perf_counter() - t
    t = time.perf_counter()
    Vo, _, eo, _ = O.hci(h, g, 4, 4, 0.0, dense_max=5000)
    cpu_s = time.perf_counter() - t
    ctx.close()
    log(f"[bench] cas8: library {V.shape[0]} dets E = {e:.12f} in {gpu_s:.2f} s; "
        f"oracle {len(Vo)} dets E = {eo:.12f} in {cpu_s:.2f} s")
    return {"n_det": int(V.shape[0]), "energy": e, "energy_oracle": float(eo), "abs_error": abs(e - float(eo)),
            "gpu_seconds": round(gpu_s, 3), "oracle_hci_seconds": round(cpu_s, 3),
            "oracle": "selection by definition + dense LAPACK eigensolves, whole HCI loop",
            "cpu_model": cpu_model()}


if __name__ == "__main__":
    main()
