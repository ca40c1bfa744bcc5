"""Parity of the HIP path with stored oracle results on the large workloads.

The reference values in tests/golden/*.json were written by
tests/golden/make_golden.py, which runs only the CPU oracle: the timed banded
workload itself (1,000,000 x 500,000, k = 10 smallest, block 4, Jacobi) at the
timed tolerance, its 20,000 x 10,000 and 100,000 x 50,000 replicas and the
256^2 convection-diffusion operator at a reference tolerance of 1e-13.  The
GPU solve runs in the configuration of the workload it stands for; its
singular values are compared element by element (1e-10 relative wherever the
accuracy bound of tests/parity.py allows it, that bound elsewhere), its
eq. (res) residuals are recomputed on the CPU, and U and V must be
orthonormal to 1e-12.

Every test prints the case it runs before touching the GPU."""
import json
import os

import numpy as np
import pytest

import synth
from parity import assert_sigma_parity

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_01404_amd as P
    P.load_library()
    return P


def _golden(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)


def _check(A, g, out, k, what):
    sig, U, V, rn, st = out
    assert st["converged"], (what, st)
    sig = sig.cpu().numpy()
    rn = rn.cpu().numpy()
    normA = g["norm_A"]
    ref = np.array(g["sigma"][:k])
    spectrum = np.array(g["sigma"] + g.get("sigma_beyond", []))
    rel = assert_sigma_parity(sig, ref, spectrum, rn, np.array(g["rnorm"][:k]), normA, what)
    U = U.cpu().numpy()
    V = V.cpu().numpy()
    r = np.sqrt(np.linalg.norm(A @ V - U * sig, axis=0) ** 2 +
                np.linalg.norm(A.T @ U - V * sig, axis=0) ** 2)
    assert np.all(r <= 1e-10 * normA * 1.0001), r / normA
    assert np.allclose(r, rn, rtol=1e-3, atol=1e-13 * normA)
    assert np.abs(U.T @ U - np.eye(k)).max() <= 1e-12
    assert np.abs(V.T @ V - np.eye(k)).max() <= 1e-12
    return rel


BANDED = dict(block_size=4, max_basis_size=35, min_restart_size=14, precond=1, seed=2002,
              profile=1)


@pytest.mark.parametrize("name,m", [("banded_2e4x1e4", 20000), ("banded_1e5x5e4", 100000),
                                    ("banded_1e6x5e5", 1000000)])
def test_banded_workload_against_oracle(P, name, m):
    """The timed path (FP64, Jacobi, block 4, one-pass A^T A product) on the
    banded workload and its replicas."""
    g = _golden(name)
    _say("golden", name, "k=10 smallest b=4 jacobi")
    A = synth.banded_scaled(m, m // 2, seed=1002)
    M = P.Matrix.from_scipy(A)
    out = M.solve(10, "smallest", 1e-10, norm_A=g["norm_A"], **BANDED)
    assert out[4]["gram_calls"] > 0, out[4]
    _check(A, g, out, 10, name)
    M.close()


@pytest.mark.parametrize("pc", ["blockjacobi", "jacobi"])
def test_convdiff_256_against_oracle(P, pc):
    """The convection-diffusion operator on a 256^2 grid (65,536 columns, 1024
    rows dropped), k = 10 smallest, block 1, with block-Jacobi (128 columns)
    or point-Jacobi corrections; the oracle's reference used K = C^-1."""
    g = _golden("convdiff_256")
    _say("golden convdiff_256 k=10 smallest b=1", pc)
    A = synth.convdiff_workload(ng=256, seed=5000)
    M = P.Matrix.from_scipy(A)
    kw = dict(precond=3, pc_block=128) if pc == "blockjacobi" else dict(precond=1)
    out = M.solve(10, "smallest", 1e-10, block_size=1, seed=1, norm_A=g["norm_A"],
                  max_seconds=100.0, **kw)
    _check(A, g, out, 10, f"convdiff_256 {pc}")
    M.close()


def test_convdiff_256_learned_against_oracle(P):
    """The learned preconditioner as the timed workload uses it: trained on the
    GPU from Jacobi-solve residuals of eight 32^2 fields (seeds 5001-5008,
    200 Adam steps, degree 15), then the held-out field (seed 5000) on the
    256^2 grid, k = 10 smallest, block 1, against the stored oracle result."""
    g = _golden("convdiff_256")
    sets = []
    for sd in range(5001, 5009):
        _say("learned training residuals seed", sd)
        M = P.Matrix.from_scipy(synth.convdiff_workload(ng=32, seed=sd))
        R, st = P.collect_residuals(M, 10, "smallest", 1e-10, every=4, max_pairs=64, block_size=1,
                                    seed=1, precond=1)
        sets.append((M, R))
    bias = np.full(8, -8.0)
    bias[7] = 0.0
    params = P.lpc_init(seed=0, out_bias=bias)
    _say("learned training 200 steps")
    hist = P.lpc_train(sets, 15, 200, 1e-2, params)
    assert hist[-1] < 0.5 * hist[0]
    A = synth.convdiff_workload(ng=256, seed=5000)
    _say("golden convdiff_256 k=10 smallest b=1 learned")
    M = P.Matrix.from_scipy(A)
    out = M.solve(10, "smallest", 1e-10, block_size=1, seed=1, norm_A=g["norm_A"],
                  precond=2, pc_model=params, pc_degree=15, max_seconds=100.0)
    _check(A, g, out, 10, "convdiff_256 learned")
    M.close()
    for Ms, _ in sets:
        Ms.close()
