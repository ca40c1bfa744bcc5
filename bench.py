"""Benchmark: time to the k requested singular triplets at eq. (res) residual
<= 1e-10 ||A|| on one MI355X, plus the roofline of the dominant sparse kernel
(the one-pass A^T A product, its two kernels together, where the matrix has a
plan, else the SpMM), the roofline of the whole solve, and the CPU oracle run
to completion on the same matrix.

A step is one complete svds_solve call (CSR checks, transpose, binning, both
stages when needed, clean-up) on a synthetic matrix already resident in HBM.
The default workload is the "plain FP64 at scale" case: a 1,000,000 x 500,000
banded matrix (64-wide band, 16 nonzeros per row, N(0,1) values) times a
log-uniform column scaling in [1e-4, 1], k = 10 smallest triplets, block 4.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("time to k triplets at ‖r‖≤1e-10‖A‖ (plain vs mixed/learned); "
          "sparse-operator HBM GB/s")
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# HBM bytes per SpMM launch of the default workload from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes scaled by a copy kernel (profiles/spmm_banded_1e6x5e5_b4_fp64_hbm_traffic.md),
# valid while the kernel source is the one those counters were taken on
SPMM_TRAFFIC = {"workload": "banded_1e6x5e5_k10_smallest", "bytes_per_launch": 245.1e6,
                "source": "paper_1607_01404_amd/csrc/k_spmm.hip", "sha256_prefix": "8d27654782fae0d0"}


# the same for one product with C by the one-pass A^T A product: its partial-sum
# kernel (235.3 MB) and its window combine (50.9 MB)
# (profiles/gram_banded_1e6x5e5_b4_fp64_hbm_traffic.md)
GRAM_TRAFFIC = {"workload": "banded_1e6x5e5_k10_smallest", "bytes_per_launch": 286.2e6,
                "source": "paper_1607_01404_amd/csrc/k_gram.hip", "sha256_prefix": "76b9b564500f50c6"}


def counted_traffic(t, workload):
    import hashlib
    if workload != t["workload"] or t["bytes_per_launch"] is None:
        return None
    with open(os.path.join(ROOT, t["source"]), "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()[:16]
    return t["bytes_per_launch"] if h == t["sha256_prefix"] else None

WORKLOADS = {
    "banded_1e6x5e5_k10_smallest": dict(
        gen=lambda: __import__("synth").banded_workload(),
        desc="1,000,000 x 500,000 banded (64-wide band, 16 nnz/row, N(0,1)) x diag(10^U(-4,0)); "
             "k=10 smallest, block 4, basis 35, restart 14, tol 1e-10, Jacobi preconditioner",
        k=10, target="smallest", opts=dict(block_size=4, max_basis_size=35, min_restart_size=14,
                                           precond=1, seed=2002)),
    "powerlaw_2e6x1e6_k20_largest": dict(
        gen=lambda: __import__("synth").powerlaw_workload(),
        desc="2,000,000 x 1,000,000, power-law rows (mean 20, max 2000, exponent 2.1), N(0,1); "
             "k=20 largest, block 8, basis 35, restart 14, tol 1e-10",
        k=20, target="largest", opts=dict(block_size=8, max_basis_size=35, min_restart_size=14,
                                          seed=2003)),
    "random_2000x1000_k5_largest": dict(
        gen=lambda: __import__("synth").uniform_workload(),
        desc="2000 x 1000, 10 nnz/row uniform, N(0,1); k=5 largest, block 1, basis 15, tol 1e-10",
        k=5, target="largest", opts=dict(block_size=1, max_basis_size=15, min_restart_size=6,
                                         seed=2001)),
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(A, w, gpu_sigma, gpu_matvecs, cap):
    """The oracle, as it stands, on the same matrix with the same settings, run
    to completion (stopped after `cap` seconds if it has not converged by then:
    then its seconds per matrix-vector product are scaled to the GPU solve's
    count).  Returns the baseline record and the largest relative difference
    between the GPU's and the oracle's singular values."""
    import numpy as np
    import oracle
    cores = len(os.sched_getaffinity(0))
    opts = dict(w["opts"])
    kw = dict(max_basis=opts.get("max_basis_size"), min_restart=opts.get("min_restart_size"),
              block=opts.get("block_size"), seed=opts.get("seed", 0),
              precond="jacobi" if opts.get("precond") == 1 else "none")
    t0 = time.perf_counter()

    def progress(stage, it, g, lam, rn_, conv):  # a line every 50 iterations
        if it % 50 == 0:
            log(f"oracle stage {stage} iteration {it} converged {int(conv.sum())} "
                f"({time.perf_counter() - t0:.0f} s)")

    sig, U, V, rn, st = oracle.svds(A, w["k"], w["target"], 1e-10, time_limit=cap,
                                    trace=progress, **kw)
    el = time.perf_counter() - t0
    mv = sum(st["matvecs"])
    s_per_mv = el / max(mv, 1)
    done = bool(st["converged"])
    value = el if done else s_per_mv * gpu_matvecs
    sample = (f"the whole solve on the full matrix, same settings: "
              f"{'converged' if done else 'stopped at the cap'} after {el:.1f} s and {mv} "
              f"matrix-vector products ({s_per_mv * 1e3:.2f} ms each)"
              + ("" if done else f"; scaled to the GPU solve's {gpu_matvecs} products"))
    rel = float(np.max(np.abs(np.asarray(gpu_sigma) - sig) / sig)) if done else None
    return ({"value": value, "unit": "s", "cores": cores, "kind": "oracle", "sample": sample,
             "time_to_solution": done, "oracle_iters": st["iters"],
             "oracle_max_rnorm_over_normA": float(rn.max()) / st["norm_A_used"]}, rel)


def no_precond_budget_run(P, torch, ip, ix, dv, m, n, w, budget):
    """The same workload without a preconditioner (K = I) under a budget of
    `budget` matrix-vector products: the residual it reaches."""
    opts = dict(w["opts"], precond=0, max_matvecs=budget)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sig, U, V, rn, st = P.solve(ip, ix, dv, m, n, w["k"], w["target"], 1e-10, **opts)
    torch.cuda.synchronize()
    return {"seconds": time.perf_counter() - t0, "max_matvecs": budget,
            "converged": bool(st["converged"]), "nconv": st["nconv"],
            "matvecs": st["matvecs"], "iters": st["iters"], "stage_exit": st["stage_exit"],
            "max_rnorm_over_normA": float(rn.max()) / st["norm_A_used"],
            "min_rnorm_over_normA": float(rn.min()) / st["norm_A_used"]}


def mixed_comparison(P, torch):
    """FP64 and mixed-precision solves of the power-law workload (k = 20
    largest): wall time of each and the difference of their results."""
    import numpy as np
    w = WORKLOADS["powerlaw_2e6x1e6_k20_largest"]
    log("generating power-law workload")
    A = w["gen"]()
    ip, ix, dv = P._lib.to_device(A)
    m, n = A.shape
    out = {"workload": w["desc"], "nnz": int(A.nnz)}
    sigs = {}
    for name, prec, s2 in (("fp64", P.FP64, P.STAGE2_JD), ("mixed", P.MIXED, P.STAGE2_JD),
                           ("fp64_gdk", P.FP64, P.STAGE2_GDK), ("mixed_gdk", P.MIXED, P.STAGE2_GDK)):
        opts = dict(w["opts"], precision=prec, profile=1, stage2_solver=s2)
        P.solve(ip, ix, dv, m, n, w["k"], w["target"], 1e-10, **opts)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sig, U, V, rn, st = P.solve(ip, ix, dv, m, n, w["k"], w["target"], 1e-10, **opts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        sigs[name] = sig.cpu().numpy()
        out[name] = {"seconds": el, "converged": bool(st["converged"]),
                     "max_rnorm_over_normA": float(rn.max()) / st["norm_A_used"],
                     "matvecs": st["matvecs"], "iters": st["iters"], "stage_exit": st["stage_exit"],
                     "stage_seconds": st["seconds"], "inner_iters": st["inner_iters"],
                     "spmm_GBps": st["spmm_bytes"] / max(st["spmm_seconds"], 1e-12) / 1e9}
        log(f"{name}: {el:.3f} s {st['iters']} {st['matvecs']}")
    out["max_rel_sigma_diff"] = float(np.max(np.abs(sigs["mixed"] - sigs["fp64"]) / sigs["fp64"]))
    out["max_rel_sigma_diff_gdk"] = float(np.max(np.abs(sigs["mixed_gdk"] - sigs["fp64_gdk"])
                                                 / sigs["fp64_gdk"]))
    out["speedup_mixed_over_fp64"] = out["fp64"]["seconds"] / out["mixed"]["seconds"]
    out["speedup_mixed_over_fp64_gdk"] = out["fp64_gdk"]["seconds"] / out["mixed_gdk"]["seconds"]
    return out


def _gen_batched(i):
    import synth
    return synth.batched_problem(i)


def batched_extra(P, torch, nprob, nworkers=16, step_threads=16):
    """Batched workload: nprob independent problems (rows U{5000..200000}, cols rows/2,
    8-12 nnz/row), k = 4 smallest each, block 8.  svds_solve_batched with the problems in
    step (one launch per step of the first-stage iteration for all problems) against
    `nworkers` host workers with a stream each; the first 16 also one after another."""
    import multiprocessing as mp
    import numpy as np
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    t = time.perf_counter()
    if nprob > 32:
        with mp.get_context("spawn").Pool(workers) as pool:
            mats = pool.map(_gen_batched, range(nprob), chunksize=4)
    else:  # small batches (and profiled runs) without worker processes
        mats = [_gen_batched(i) for i in range(nprob)]
    gen = time.perf_counter() - t
    log(f"batched: generated {nprob} problems in {gen:.1f} s")
    dev = [P._lib.to_device(A) + A.shape for A in mats]
    opts = dict(block_size=8, max_basis_size=35, min_restart_size=14, seed=2004)
    k = 4
    sub = dev[:16]
    P.solve_batched(sub, k, "smallest", 1e-10, nworkers=-step_threads, **opts)  # warm-up, autotune
    torch.cuda.synchronize()
    t = time.perf_counter()
    for d in sub:
        P.solve(*d, k, "smallest", 1e-10, **opts)
    torch.cuda.synchronize()
    serial16 = time.perf_counter() - t

    def timed(subset, nw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = P.solve_batched(subset, k, "smallest", 1e-10, nworkers=nw, **opts)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    step16, _ = timed(sub, -step_threads)
    el, (rc, res) = timed(dev, -step_threads)
    log(f"batched: in step {el:.2f} s")
    if nworkers > 0:  # the same problems on host workers, a stream each
        workers16, _ = timed(sub, nworkers)
        elw, (rcw, resw) = timed(dev, nworkers)
        log(f"batched: {nworkers} workers {elw:.2f} s")
        same = all(bool((a[0] == b[0]).all()) and a[4]["matvecs"] == b[4]["matvecs"]
                   for a, b in zip(res, resw))
    else:
        workers16 = elw = rcw = same = None
    conv = sum(1 for r in res if r[4]["converged"])
    rmax = max(float(r[3].max()) / r[4]["norm_A_used"] for r in res)
    nnz = int(sum(A.nnz for A in mats))
    ab = sum(r[4]["alg_bytes"] for r in res)
    return {"workload": f"{nprob} problems, rows U{{5000..200000}}, cols rows/2, 8-12 nnz/row, "
                        "N(0,1); k=4 smallest, block 8, basis 35, restart 14, tol 1e-10",
            "nnz_total": nnz, "seconds": el, "problems_per_second": nprob / el,
            "mode": "in step: one launch per step of the first-stage iteration for all problems; "
                    f"set-up and clean-up on {step_threads} host threads",
            "converged": conv, "status": rc, "max_rnorm_over_normA": rmax,
            "matvecs_total": int(sum(sum(r[4]["matvecs"]) for r in res)),
            "iters_max": int(max(r[4]["iters"][0] for r in res)),
            "iters_mean": float(np.mean([r[4]["iters"][0] for r in res])),
            "stage2_problems": int(sum(1 for r in res if r[4]["stage_exit"] == 2)),
            "roofline": {"bound": "hbm", "achieved": ab / el / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": ab / el / 1e9 / HBM_PEAK_GBS,
                         "alg_bytes": ab,
                         "note": "counted iteration kernels of all problems over the batch's "
                                 "wall time (set-up, norm estimates, clean-up in the time only)"},
            "workers_seconds": elw, "workers": nworkers,
            "workers_problems_per_second": nprob / elw if elw else None, "workers_status": rcw,
            "same_results_as_workers": same,
            "first16_serial_seconds": serial16, "first16_in_step_seconds": step16,
            "first16_workers_seconds": workers16, "generation_seconds": gen}


def learned_extra(P, torch, full_seconds, replica=True, full_runs=None, full_matvecs=0,
                  full_grid=1024):
    """Learned-preconditioner workload: a preconditioner trained on the GPU from residuals of
    Jacobi solves on eight 32x32 coefficient fields (seeds 5001-5008),
    evaluated against Jacobi and no preconditioning on a held-out field
    (seed 5000) at 128x128 and at the full 1024x1024 size (time-capped at
    full_seconds).  full_runs: the preconditioners run at full size (all when
    None); full_matvecs > 0 raises the product budget of the full-size solves;
    full_grid < 1024 runs that leg on a smaller grid instead (scaling runs)."""
    import numpy as np
    import synth
    degree = 15
    t = time.perf_counter()
    sets = []
    for sd in range(5001, 5009):
        M = P.Matrix.from_scipy(synth.convdiff_workload(ng=32, seed=sd))
        R, st = P.collect_residuals(M, 10, "smallest", 1e-10, every=4, max_pairs=64, block_size=1,
                                    seed=1, precond=P.PC_JACOBI)
        sets.append((M, R))
    collect = time.perf_counter() - t
    bias = np.full(8, -8.0)
    bias[7] = 0.0
    params = P.lpc_init(seed=0, out_bias=bias)
    torch.cuda.synchronize()
    t = time.perf_counter()
    hist = P.lpc_train(sets, degree, 200, 1e-2, params)
    torch.cuda.synchronize()
    train = time.perf_counter() - t
    out = {"training": {"sets": "eight 32x32 fields (seeds 5001-5008), Jacobi solves, k=10 smallest,"
                                " a residual every 4th stage-1 iteration, 64 per field",
                        "collect_seconds": collect, "train_seconds": train, "steps": 200,
                        "degree": degree, "loss_first": float(hist[0]), "loss_last": float(hist[-1])}}
    runs = [("none", dict(precond=P.PC_NONE)),
            ("jacobi", dict(precond=P.PC_JACOBI)),
            ("jacobi_gdk", dict(precond=P.PC_JACOBI, stage2_solver=P.STAGE2_GDK)),
            ("block_jacobi_128", dict(precond=P.PC_BLOCKJACOBI, pc_block=128)),
            ("learned", dict(precond=P.PC_LEARNED, pc_model=params, pc_degree=degree))]
    sizes = ((("replica_128x128", 128, 60.0),) if replica else ()) + (
        (f"full_{full_grid}x{full_grid}", full_grid, full_seconds),)
    for label, ng, cap in sizes:
        full = label.startswith("full_")
        B = synth.convdiff_workload(ng=ng, seed=5000)
        MB = P.Matrix.from_scipy(B)
        res = {"shape": list(B.shape), "nnz": int(B.nnz), "max_seconds": cap}
        for name, kw in runs:
            if full and full_runs is not None and name not in full_runs:
                continue
            if full and full_matvecs > 0:
                kw = dict(kw, max_matvecs=full_matvecs)
            if cap > 60.0:  # long solves print a progress line every 2000 iterations
                kw = dict(kw, print_level=2)
            log(f"learned extra: {label} {name}")
            torch.cuda.synchronize()
            t = time.perf_counter()
            sig, U, V, rn, st = MB.solve(10, "smallest", 1e-10, block_size=1, seed=1,
                                         max_seconds=cap, **kw)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            res[name] = {"seconds": el, "converged": bool(st["converged"]), "nconv": st["nconv"],
                         "iters": st["iters"], "matvecs": st["matvecs"],
                         "inner_iters": st["inner_iters"],
                         "max_rnorm_over_normA": float(rn.max()) / st["norm_A_used"],
                         "sigma_min": float(sig[0])}
        out[label] = res
        MB.close()
    for M, _ in sets:
        M.close()
    return out, params


def methods_extra(P, torch, cap):
    """Single-stage methods against the two-stage method (Section 3.4):
    smallest triplets of an ill-conditioned banded matrix (normal equations
    alone vs hybrid) and largest triplets of a power-law matrix (normal,
    augmented, hybrid)."""
    import synth
    out = {}
    cases = [
        ("smallest_banded_2e5x1e5_kappa1e6",
         lambda: synth.banded_scaled(200000, 100000, seed=2005, log_lo=-6.0), 5, "smallest",
         dict(block_size=4, max_basis_size=35, min_restart_size=14, precond=P.PC_JACOBI, seed=2005),
         (("hybrid", P.METHOD_HYBRID), ("normal", P.METHOD_NORMAL))),
        ("largest_powerlaw_2e5x1e5",
         lambda: synth.powerlaw_rows(200000, 100000, seed=2006), 10, "largest",
         dict(block_size=4, max_basis_size=35, min_restart_size=14, seed=2006),
         (("hybrid", P.METHOD_HYBRID), ("normal", P.METHOD_NORMAL),
          ("augmented", P.METHOD_AUGMENTED))),
    ]
    for label, gen, k, target, opts, methods in cases:
        A = gen()
        M = P.Matrix.from_scipy(A)
        res = {"shape": list(A.shape), "nnz": int(A.nnz), "k": k, "target": target,
               "max_seconds": cap}
        for name, meth in methods:
            log(f"methods extra: {label} {name}")
            M.solve(k, target, 1e-10, method=meth, max_seconds=cap, **opts)  # warm-up
            torch.cuda.synchronize()
            t = time.perf_counter()
            sig, U, V, rn, st = M.solve(k, target, 1e-10, method=meth, max_seconds=cap, **opts)
            torch.cuda.synchronize()
            res[name] = {"seconds": time.perf_counter() - t, "converged": bool(st["converged"]),
                         "max_rnorm_over_normA": float(rn.max()) / st["norm_A_used"],
                         "matvecs": st["matvecs"], "iters": st["iters"],
                         "stage_exit": st["stage_exit"]}
        out[label] = res
        M.close()
    return out


def condest_extra(P, torch, main_matrix, learned_params):
    """Condition-number estimate of Section 4.4 (block 1, stage 1 stopped at
    ||r|| < 0.1 sigma): the banded 1e6 x 5e5 matrix with Jacobi, and the
    128 x 128 convection-diffusion field with Jacobi and with the learned
    preconditioner."""
    import synth
    out = {}
    runs = [("banded_1e6x5e5_jacobi", main_matrix, dict(precond=P.PC_JACOBI, seed=7))]
    B = synth.convdiff_workload(ng=128, seed=5000)
    MB = P.Matrix.from_scipy(B)
    runs.append(("convdiff_128x128_jacobi", MB, dict(precond=P.PC_JACOBI, seed=7)))
    runs.append(("convdiff_128x128_block_jacobi_128", MB,
                 dict(precond=P.PC_BLOCKJACOBI, pc_block=128, seed=7)))
    if learned_params is not None:
        runs.append(("convdiff_128x128_learned", MB,
                     dict(precond=P.PC_LEARNED, pc_model=learned_params, pc_degree=15, seed=7)))
    for label, M, kw in runs:
        log(f"condest extra: {label}")
        P.condest(M, 0.1, **kw)  # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        kappa, smax, smin, (s1, s0) = P.condest(M, 0.1, **kw)
        torch.cuda.synchronize()
        out[label] = {"seconds": time.perf_counter() - t, "kappa": kappa, "sigma_max": smax,
                      "sigma_min": smin,
                      "matvecs": int(sum(s1["matvecs"]) + sum(s0["matvecs"]))}
    MB.close()
    return out


def two_product_run(P, torch, ip, ix, dv, m, n, k, w, args):
    """One solve of the same workload with the one-pass product switched off
    (every product with C as A, then A^T by two SpMMs), for comparison."""
    opts = dict(w["opts"], profile=1, fused_gram=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sig, U, V, rn, st = P.solve(ip, ix, dv, m, n, k, w["target"], 1e-10, **opts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ach = st["spmm_bytes"] / max(st["spmm_seconds"], 1e-12) / 1e9
    return {"seconds": el, "converged": bool(st["converged"]), "iters": st["iters"],
            "matvecs": st["matvecs"],
            "spmm": {"achieved_GBps": ach, "frac": ach / HBM_PEAK_GBS,
                     "avg_call_us": st["spmm_seconds"] / max(st["spmm_calls"], 1) * 1e6,
                     "bytes_per_call": st["spmm_bytes"] / max(st["spmm_calls"], 1),
                     "traffic": counted_traffic(SPMM_TRAFFIC, args.workload)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="banded_1e6x5e5_k10_smallest", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=600.0,
                    help="cap of the oracle's solve (it normally converges well before)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the mixed-precision, batched and learned-preconditioner extras "
                         "and the two-product comparison")
    ap.add_argument("--batched", type=int, default=256, help="problems in the batched extra (0: skip)")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--step-threads", type=int, default=16,
                    help="host threads of the in-step batched solve's set-up and clean-up")
    ap.add_argument("--workers", type=int, default=16, help="host workers of the batched extra's comparison (0: in step only)")
    ap.add_argument("--full-runs", default=None,
                    help="comma-separated preconditioners of the full-size learned-workload "
                         "runs (none, jacobi, jacobi_gdk, block_jacobi_128, learned; default all)")
    ap.add_argument("--full-grid", type=int, default=1024,
                    help="grid of the full-size learned-workload leg (smaller for scaling runs)")
    ap.add_argument("--full-matvecs", type=int, default=0,
                    help="product budget of the full-size learned-workload solves (0: default)")
    ap.add_argument("--full-seconds", type=float, default=20.0,
                    help="time budget of each full-size convection-diffusion solve")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="precision of the timed solves (mixed: FP32/BF16 stage 1, FP64 stage 2)")
    ap.add_argument("--only", default=None,
                    choices=["mixed", "batched", "learned", "learned_full", "methods", "condest"],
                    help="run only this extra (for profiling) and print its record")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (scales the HBM byte "
                         "counters of a profiler run) and exit")
    args = ap.parse_args()
    if args.copy_calibration > 0:
        import torch
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "copies": 5}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1607_01404_amd as P

    if args.only:
        torch.cuda.set_device(0)
        if args.only == "mixed":
            out = mixed_comparison(P, torch)
        elif args.only == "batched":
            out = batched_extra(P, torch, max(args.batched, 16), args.workers, args.step_threads)
        elif args.only in ("learned", "learned_full"):
            out, _ = learned_extra(P, torch, args.full_seconds, replica=args.only == "learned",
                                   full_runs=args.full_runs.split(",") if args.full_runs else None,
                                   full_matvecs=args.full_matvecs, full_grid=args.full_grid)
        elif args.only == "methods":
            out = methods_extra(P, torch, 30.0)
        else:
            import synth
            Ab = synth.banded_workload()
            Mb = P.Matrix.from_scipy(Ab)
            out = condest_extra(P, torch, Mb, None)
            Mb.close()
        print(json.dumps({"only": args.only, "record": out}), flush=True)
        return

    w = WORKLOADS[args.workload]
    log("generating", args.workload)
    t = time.perf_counter()
    A = w["gen"]()
    log(f"matrix {A.shape} nnz {A.nnz} in {time.perf_counter() - t:.1f} s")
    torch.cuda.set_device(0)
    ip, ix, dv = P._lib.to_device(A)
    m, n = A.shape
    k = w["k"]
    opts = dict(w["opts"], profile=1, precision=P.MIXED if args.precision == "mixed" else P.FP64)
    torch.cuda.synchronize()

    def step():
        return P.solve(ip, ix, dv, m, n, k, w["target"], 1e-10, **opts)

    for i in range(args.warmup):
        out = step()
        log(f"warmup {i}: {out[4]['seconds']} matvecs {out[4]['matvecs']} iters {out[4]['iters']}")
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = step()
        stats.append(out[4])
        log(f"step {i} done")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sec = el / args.steps
    st = stats[-1]
    sig, U, V, rn, _ = out
    normA = st["norm_A_used"]
    ok = bool(st["converged"]) and float(rn.max()) <= 1e-10 * normA
    # the dominant sparse kernel: the one-pass A^T A product when the solve
    # took it, else the SpMM
    gram = sum(s["gram_calls"] for s in stats) > 0
    key = "gram" if gram else "spmm"
    calls = sum(s[key + "_calls"] for s in stats)
    ssec = sum(s[key + "_seconds"] for s in stats)
    sbytes = sum(s[key + "_bytes"] for s in stats)
    achieved = sbytes / ssec / 1e9 if ssec > 0 else 0.0
    kernel = ("one-pass A^T A product: k_gram_partial then k_gram_combine, timed together "
              "(every stage-1 product with C); bytes: the method's, A read once, X read "
              "and Z written once" if gram else
              "binned CSR SpMM (A and A^T products of every iteration)")
    traffic = counted_traffic(GRAM_TRAFFIC if gram else SPMM_TRAFFIC, args.workload)
    res = {
        "metric": METRIC,
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+bf16 stage 1, f64 stage 2",
        "data": "synthetic",
        "config": {"workload": w["desc"], "m": m, "n": n, "nnz": int(A.nnz), "k": k,
                   "target": w["target"], "tol": 1e-10, "precision": args.precision},
        "converged": ok,
        "sigma": [float(x) for x in sig.cpu().numpy()],
        "max_rnorm_over_normA": float(rn.max()) / normA,
        "matvecs": st["matvecs"],
        "iters": st["iters"],
        "stage_exit": st["stage_exit"],
        "setup_seconds": st["setup_seconds"],
        "stage_seconds": st["seconds"],
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_unit": ("bytes per product with C, both kernels (rocprofv3 FETCH_SIZE/"
                             "WRITE_SIZE, copy-scaled)" if gram else
                             "bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-scaled)"),
            "avg_call_us": ssec / max(calls, 1) * 1e6,
            "bytes_per_call": sbytes / max(calls, 1),
            # the solver times one call in four with events: these two
            # describe that sample, not every call
            "timed_calls_per_solve": calls / max(len(stats), 1),
            "timed_share_of_solve": ssec / el,
        },
    }
    # the two other HBM-bound kernels that lead the solve's time, by the same
    # event timing (one call in four): the basis projections and the residual
    others = {}
    for key, name in (("proj", "k_tsgemm_tn (first Gram-Schmidt projection and new H columns)"),
                      ("resid", "k_residual (fused residual and norms)")):
        c = sum(s[key + "_calls"] for s in stats)
        sec_k = sum(s[key + "_seconds"] for s in stats)
        by = sum(s[key + "_bytes"] for s in stats)
        if c > 0 and sec_k > 0:
            ach = by / sec_k / 1e9
            others[name] = {"achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": ach / HBM_PEAK_GBS, "avg_call_us": sec_k / c * 1e6,
                            "bytes_per_call": by / c, "timed_calls": c}
    res["roofline_others"] = others
    # the whole solve: every counted kernel's algorithmic bytes over the solve's
    # wall time (set-up, norm estimate and clean-up are in the time, not in the
    # bytes, so this is a lower bound)
    ab = sum(s_["alg_bytes"] for s_ in stats) / len(stats)
    res["whole_solve_roofline"] = {
        "bound": "hbm", "achieved": ab / sec / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": ab / sec / 1e9 / HBM_PEAK_GBS, "alg_bytes_per_solve": ab,
        "counted": "sparse products, projections, updates, Cholesky QR passes, residuals, "
                   "restarts and corrections of every iteration; not set-up or clean-up"}
    if gram and not args.no_extras:
        res["two_product_comparison"] = two_product_run(P, torch, ip, ix, dv, m, n, k, w, args)
    if not args.no_extras:
        res["mixed_precision"] = mixed_comparison(P, torch)
        if args.batched > 0:
            res["batched"] = batched_extra(P, torch, args.batched, args.workers, args.step_threads)
        params = None
        if not args.no_learned:
            res["learned_preconditioner"], params = learned_extra(P, torch, args.full_seconds)
        res["methods"] = methods_extra(P, torch, 30.0)
        Mmain = P.Matrix(ip, ix, dv, m, n)
        res["condition_estimate"] = condest_extra(P, torch, Mmain, params)
        Mmain.close()
    if not args.no_extras:
        log("no preconditioner under a budget ...")
        res["no_preconditioner_budget"] = no_precond_budget_run(P, torch, ip, ix, dv, m, n, w,
                                                                200000)
    if not args.no_cpu:
        gpu_mv = int(sum(st["matvecs"]))
        log("cpu baseline (oracle) ...")
        res["cpu_baseline"], res["max_rel_sigma_err_vs_oracle"] = cpu_baseline(
            A, w, res["sigma"], gpu_mv, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
