"""Writes the stored reference results of the large parity cases.

Calls only the oracle (and the seeded generators of ``synth`` for its input);
nothing here touches the HIP path.  Run from the repository root:

    python tests/golden/make_golden.py [case ...]

Each case writes tests/golden/<case>.json with the oracle's singular values
(k + 2 of them: the two beyond the k compared give the gap of the k-th value
for the accuracy bound the parity tests use), their eq. (res) residuals, the
norm estimate, the oracle's counts, wall time and core count.

Cases (the shapes and options of the workloads they stand in for):
  banded_1e6x5e5  1,000,000 x 500,000 banded x diag(10^U(-4,0)), k = 10
                  smallest, block 4, basis 35, restart 14, Jacobi, seed 2002,
                  tol 1e-10: the timed workload as timed.  A second run with
                  k = 12 at tol 1e-8 gives the values beyond the tenth.
  banded_2e4x1e4, banded_1e5x5e4
                  replicas with the same band, scaling and options, reference
                  tolerance 1e-13 (stage 2 reaches it), k = 12.
  convdiff_256, convdiff_512
                  the convection-diffusion operator (Pe = 10, 4 grid lines
                  dropped) on 256^2 and 512^2 grids, k = 12 smallest, block 1,
                  tolerance 1e-13, corrections preconditioned by C^-1 (sparse
                  LU), which leaves the triplets unchanged.
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

BANDED = dict(block=4, max_basis=35, min_restart=14, seed=2002, precond="jacobi")


def _run(A, k, tol, **kw):
    t = time.perf_counter()
    sig, U, V, rn, st = oracle.svds(A, k, "smallest", tol, **kw)
    el = time.perf_counter() - t
    assert st["converged"], st
    return sig, rn, st, el


def _record(name, desc, sig, rn, st, el, tol, k, extra=None):
    out = {"case": name, "workload": desc, "k": k, "tol": tol,
           "sigma": [float(x) for x in sig], "rnorm": [float(x) for x in rn],
           "norm_A": float(st["norm_A_used"]), "iters": st["iters"], "matvecs": st["matvecs"],
           "stage_exit": st["stage_exit"], "oracle_seconds": el,
           "cores": len(os.sched_getaffinity(0))}
    if extra:
        out.update(extra)
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, f"{el:.1f} s", out["sigma"][:3], flush=True)


def banded_full():
    A = synth.banded_workload()
    sig, rn, st, el = _run(A, 10, 1e-10, **BANDED)
    s12, r12, st12, el12 = _run(A, 12, 1e-8, **BANDED)
    _record("banded_1e6x5e5", "1e6 x 5e5 banded (seed 1002) x diag(10^U(-4,0)), Jacobi, b 4",
            sig, rn, st, el, 1e-10, 10,
            {"sigma_beyond": [float(x) for x in s12[10:]], "sigma_beyond_tol": 1e-8})


def banded_replica(m, name):
    A = synth.banded_scaled(m, m // 2, seed=1002)
    sig, rn, st, el = _run(A, 12, 1e-13, **BANDED)
    _record(name, f"{m} x {m // 2} banded (seed 1002) x diag(10^U(-4,0)), Jacobi, b 4",
            sig, rn, st, el, 1e-13, 12)


def convdiff(ng, name):
    A = synth.convdiff_workload(ng=ng, seed=5000)
    K = oracle.exact_inverse(A)
    sig, rn, st, el = _run(A, 12, 1e-13, block=1, seed=1, precond=K)
    _record(name, f"{ng}^2 convection-diffusion (seed 5000, Pe 10, {4 * ng} rows dropped), "
            "b 1, K = C^-1", sig, rn, st, el, 1e-13, 12)


CASES = {
    "banded_2e4x1e4": lambda: banded_replica(20000, "banded_2e4x1e4"),
    "banded_1e5x5e4": lambda: banded_replica(100000, "banded_1e5x5e4"),
    "convdiff_256": lambda: convdiff(256, "convdiff_256"),
    "convdiff_512": lambda: convdiff(512, "convdiff_512"),
    "banded_1e6x5e5": banded_full,
}

if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for n in names:
        CASES[n]()
