"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Every test prints the case it runs before touching the GPU."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import oracle.phsvds as OP
import synth
from parity import assert_sigma_parity

pytestmark = pytest.mark.gpu


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


def _binned_matrix(seed=3):
    """Rows of every length class: empty, 1..4, ... up to one 5000-long row."""
    rng = np.random.default_rng(seed)
    n = 6000
    lengths = [0, 0, 1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 31, 33, 63, 65, 127, 129, 500, 1000, 4096,
               4097, 5000]
    lengths = lengths + list(rng.integers(0, 40, size=3000))
    m = len(lengths)
    return synth.random_uniform_rows(m, n, np.array(lengths), seed=seed)


@pytest.mark.parametrize("b", [1, 2, 3, 4, 8])
def test_spmm_matches_scipy(P, b):
    import torch
    A = _binned_matrix()
    _say("spmm", A.shape, A.nnz, "b", b)
    M = P.Matrix.from_scipy(A)
    rng = np.random.default_rng(b)
    for trans in (False, True):
        X = rng.standard_normal((A.shape[0] if trans else A.shape[1], b))
        Y = M.spmm(torch.from_numpy(X).cuda(), trans=trans).cpu().numpy()
        ref = (A.T @ X) if trans else (A @ X)
        scale = (abs(A).T @ abs(X)) if trans else (abs(A) @ abs(X))
        assert np.all(np.abs(Y - ref) <= 1e-14 * scale + 1e-300), trans
    M.close()


def test_spmm_deterministic(P):
    import torch
    A = synth.powerlaw_workload(m=20000, n=10000)
    _say("spmm determinism", A.shape)
    M = P.Matrix.from_scipy(A)
    X = torch.from_numpy(np.random.default_rng(0).standard_normal((A.shape[1], 4))).cuda()
    Y1 = M.spmm(X)
    Y2 = M.spmm(X)
    assert torch.equal(Y1, Y2)
    M.close()


@pytest.mark.parametrize("g", [1, 2, 7, 15, 35, 48])
def test_small_eig_matches_lapack(P, g):
    import torch
    _say("small_eig", g)
    rng = np.random.default_rng(g)
    Q, _ = np.linalg.qr(rng.standard_normal((g, g)))
    lam = np.sort(np.concatenate([rng.uniform(-1, 1, g - g // 3), 0.3 + 1e-9 * np.arange(g // 3)]))
    H = (Q * lam) @ Q.T
    for desc in (False, True):
        th, Y = P.small_eig(torch.from_numpy(H).cuda(), descending=desc)
        th = th.cpu().numpy()
        Y = Y.cpu().numpy()
        ref = np.linalg.eigvalsh(H)
        ref = ref[::-1] if desc else ref
        assert np.max(np.abs(th - ref)) <= 1e-14 * max(1.0, np.abs(lam).max()) * g
        assert np.abs(Y.T @ Y - np.eye(g)).max() <= 1e-13
        assert np.abs(H @ Y - Y * th).max() <= 1e-13


@pytest.mark.parametrize("g", [1, 3, 16, 35, 48])
def test_small_svd_matches_lapack(P, g):
    import torch
    _say("small_svd", g)
    rng = np.random.default_rng(100 + g)
    R = np.triu(rng.standard_normal((g, g)))
    R[:, 0] *= 1e-9  # a tiny singular value, as in the refined factor near convergence
    s, Y = P.small_svd(torch.from_numpy(R).cuda())
    s = s.cpu().numpy()
    Y = Y.cpu().numpy()
    ref = np.sort(np.linalg.svd(R, compute_uv=False))
    assert np.all(np.abs(s - ref) <= 1e-13 * ref.max() + 1e-15 * ref)
    assert np.abs(Y.T @ Y - np.eye(g)).max() <= 1e-13
    # smallest right singular vector: ||R y|| = s_min
    assert abs(np.linalg.norm(R @ Y[:, 0]) - s[0]) <= 1e-13 * ref.max()


def _compare(A, sig, U, V, rn, st, ref_sig, tol, normA, ref_rn=None, what=""):
    """Singular values against a reference (the oracle's, with its residuals
    ref_rn, or dense LAPACK's, ref_rn None) to 1e-10 relative where the
    accuracy bound of tests/parity.py allows it and to that bound elsewhere;
    eq. (res) and orthonormality to 1e-12 of the returned triplets."""
    sig = sig.cpu().numpy()
    U = U.cpu().numpy()
    V = V.cpu().numpy()
    rn = rn.cpu().numpy()
    k = sig.size
    # gaps from the whole spectrum when dense LAPACK can give it
    spectrum = (np.linalg.svd(A.toarray(), compute_uv=False) if min(A.shape) <= 3000
                else np.asarray(ref_sig))
    ref_rn = np.zeros(k) if ref_rn is None else np.asarray(ref_rn)
    assert_sigma_parity(sig, ref_sig, spectrum, rn, ref_rn, normA, what)
    # eq. (res) recomputed on the CPU from the returned triplets
    r = np.sqrt(np.linalg.norm(A @ V - U * sig, axis=0) ** 2 + np.linalg.norm(A.T @ U - V * sig, axis=0) ** 2)
    assert np.all(r <= tol * normA * 1.0001), r / normA
    assert np.allclose(r, rn, rtol=1e-3, atol=1e-3 * tol * normA)
    assert np.abs(U.T @ U - np.eye(k)).max() <= 1e-12
    assert np.abs(V.T @ V - np.eye(k)).max() <= 1e-12
    return sig, U, V


@pytest.mark.parametrize("target", ["largest", "smallest"])
@pytest.mark.parametrize("force2", [0, 1])
def test_uniform_workload_against_oracle(P, target, force2):
    A = synth.uniform_workload()
    normA = float(np.linalg.norm(A.toarray(), 2))
    _say("solve uniform_workload", target, "force_stage2", force2)
    sig, U, V, rn, st = P.svds(A, 5, target, 1e-10, max_basis_size=15, min_restart_size=6,
                               block_size=1, norm_A=normA, seed=11, force_stage2=force2)
    ref, Ur, Vr, rr, sr = oracle.svds(A, 5, target, 1e-10, max_basis=15, min_restart=6, block=1,
                                      norm_A=normA, seed=11, force_stage2=bool(force2))
    assert st["converged"], st
    assert st["stage_exit"] == (2 if force2 else 1)
    s, Ug, Vg = _compare(A, sig, U, V, rn, st, ref, 1e-10, normA, rr, "uniform vs oracle")
    # same singular vectors as the oracle (sign convention applied on both)
    assert np.all(np.abs(np.sum(Vg * Vr, axis=0) - 1) < 1e-8)


@pytest.mark.parametrize("target", ["largest", "smallest"])
def test_stage2_from_loose_stage1(P, target):
    A = synth.uniform_workload()
    normA = float(np.linalg.norm(A.toarray(), 2))
    _say("solve uniform_workload stage2 from stage1_tol 1e-4", target)
    sig, U, V, rn, st = P.svds(A, 5, target, 1e-10, max_basis_size=15, min_restart_size=6,
                               norm_A=normA, seed=5, stage1_tol=1e-4)
    ref, _, _, rr, _ = oracle.svds(A, 5, target, 1e-10, max_basis=15, min_restart=6, norm_A=normA,
                                   seed=5, stage1_tol=1e-4)
    assert st["converged"] and st["stage_exit"] == 2 and st["iters"][1] > 0, st
    _compare(A, sig, U, V, rn, st, ref, 1e-10, normA, rr, "loose stage 1 vs oracle")


def test_ill_conditioned_smallest_with_jacobi(P):
    A = synth.banded_scaled(300, 150, seed=1, log_lo=-6)
    normA = float(np.linalg.norm(A.toarray(), 2))
    _say("solve banded_scaled 300x150 kappa~2e6 smallest jacobi")
    sig, U, V, rn, st = P.svds(A, 3, "smallest", 1e-10, block_size=1, norm_A=normA, seed=7,
                               precond=P.PC_JACOBI)
    s = np.sort(np.linalg.svd(A.toarray(), compute_uv=False))[:3]
    assert st["converged"], st
    _compare(A, sig, U, V, rn, st, s, 1e-10, normA, what="kappa 2e6 vs LAPACK")


def test_block_and_wide(P):
    A = synth.random_uniform_rows(300, 600, 12, seed=21)
    normA = float(np.linalg.norm(A.toarray(), 2))
    _say("solve wide 300x600 largest b=2")
    sig, U, V, rn, st = P.svds(A, 4, "largest", 1e-10, block_size=2, norm_A=normA, seed=3)
    assert U.shape == (300, 4) and V.shape == (600, 4)
    s = np.linalg.svd(A.toarray(), compute_uv=False)[:4]
    _compare(A, sig, U, V, rn, st, s, 1e-10, normA)


def test_norm_estimate(P):
    A = synth.uniform_workload()
    normA = float(np.linalg.norm(A.toarray(), 2))
    _say("solve uniform_workload with internal norm estimate")
    sig, U, V, rn, st = P.svds(A, 2, "largest", 1e-10, seed=3)
    assert abs(st["norm_A_used"] - normA) / normA < 1e-6
    assert st["converged"]


def test_malformed_csr_rejected(P):
    import torch
    _say("malformed csr")
    A = synth.uniform_workload(m=50, n=20, nnz_per_row=3)
    ip, ix, dv = P._lib.to_device(A)
    ix_bad = ix.clone()
    ix_bad[5] = 25  # out of range column
    with pytest.raises(P.SvdsError) as e:
        P.solve(ip, ix_bad, dv, 50, 20, 2)
    assert e.value.code == -2
    ip_bad = ip.clone()
    ip_bad[-1] += 1
    with pytest.raises(P.SvdsError) as e:
        P.solve(ip_bad, ix, dv, 50, 20, 2)
    assert e.value.code == -2
    with pytest.raises(P.SvdsError) as e:
        P.solve(ip, ix, dv, 50, 20, 0)
    assert e.value.code == -1


def test_deterministic_solve(P):
    A = synth.uniform_workload()
    _say("solve determinism")
    a = P.svds(A, 3, "smallest", 1e-10, seed=9, norm_A=8.0)
    b = P.svds(A, 3, "smallest", 1e-10, seed=9, norm_A=8.0)
    import torch
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])


def test_rank_deficient_breakdown_repair(P):
    """A rank-3 matrix: the Krylov fill and the corrections run out of new
    directions, so orthogonalisation breakdowns are repaired with counter-based
    random vectors; the three nonzero singular values still match."""
    rng = np.random.default_rng(4)
    Ud, _ = np.linalg.qr(rng.standard_normal((300, 3)))
    Vd, _ = np.linalg.qr(rng.standard_normal((200, 3)))
    A = sp.csr_matrix((Ud * np.array([3.0, 2.0, 1.0])) @ Vd.T)
    A = synth.to_csr(A)
    _say("rank-3 300x200 largest k=3 b=2")
    sig, U, V, rn, st = P.svds(A, 3, "largest", 1e-10, block_size=2, norm_A=3.0, seed=1)
    assert st["breakdowns"] > 0, st
    assert np.max(np.abs(sig.cpu().numpy() - [3.0, 2.0, 1.0])) < 1e-12
    assert float(rn.max()) <= 3e-10


@pytest.mark.parametrize("target", ["largest", "smallest"])
def test_mixed_precision_uniform_workload(P, target):
    """Mixed stage 1 (FP32 basis and SpMM, BF16 MFMA projections), FP64
    stage 2: same triplets as the FP64 oracle."""
    A = synth.uniform_workload()
    normA = float(np.linalg.norm(A.toarray(), 2))
    _say("mixed uniform_workload", target)
    sig, U, V, rn, st = P.svds(A, 5, target, 1e-10, max_basis_size=15, min_restart_size=6,
                               norm_A=normA, seed=11, precision=P.MIXED)
    ref, _, _, rr, _ = oracle.svds(A, 5, target, 1e-10, max_basis=15, min_restart=6, norm_A=normA,
                                   seed=11)
    assert st["converged"], st
    _compare(A, sig, U, V, rn, st, ref, 1e-10, normA, rr, "mixed vs oracle")


def test_mixed_precision_powerlaw_largest(P):
    """Power-law rows (mean 20, max 2000, exponent 2.1) at 20000 x 10000, k = 20
    largest, block 8: mixed and FP64 GPU results against the FP64 oracle."""
    A = synth.powerlaw_workload(m=20000, n=10000)
    normA = float(np.linalg.norm(A.toarray(), 2)) if A.shape[1] <= 4000 else None
    ref, _, _, rr, sref = oracle.svds(A, 20, "largest", 1e-10, block=8, max_basis=35,
                                      min_restart=14, seed=3)
    normA = sref["norm_A_used"]
    for prec in (P.FP64, P.MIXED):
        _say("powerlaw 20000x10000 k=20 largest b=8 precision", prec)
        sig, U, V, rn, st = P.svds(A, 20, "largest", 1e-10, block_size=8, max_basis_size=35,
                                   min_restart_size=14, seed=3, norm_A=normA, precision=prec)
        assert st["converged"], st
        _compare(A, sig, U, V, rn, st, ref, 1e-10, normA, rr, f"powerlaw precision {prec}")


def _batch(count, mmin=2000, mmax=6000):
    return [synth.batched_problem(i, mmin=mmin, mmax=mmax) for i in range(count)]


def test_batched_matches_single_solves(P):
    """svds_solve_batched on problems of uneven sizes: every problem's result is
    bit-identical to its own svds_solve (the kernels are deterministic and the
    workers share nothing but the launch-shape cache, switched off here), and
    the singular values match the oracle."""
    import torch
    As = _batch(6)
    dev = [P._lib.to_device(A) + A.shape for A in As]
    opts = dict(block_size=8, max_basis_size=35, min_restart_size=14, seed=17, autotune=0)
    _say("batched", [A.shape for A in As], "k=4 smallest b=8 workers 3")
    rc, res = P.solve_batched(dev, 4, "smallest", 1e-10, nworkers=3, **opts)
    assert rc == 0, [r[4] for r in res]
    for i, (A, d) in enumerate(zip(As, dev)):
        _say("single", i, A.shape)
        sig, U, V, rn, st = P.solve(*d, 4, "smallest", 1e-10, **opts)
        assert torch.equal(sig, res[i][0]) and torch.equal(U, res[i][1]) and torch.equal(V, res[i][2])
        assert res[i][4]["converged"] and res[i][4]["matvecs"] == st["matvecs"]
    for i in range(2):
        A = As[i]
        ref = np.sort(np.linalg.svd(A.toarray(), compute_uv=False))[:4]
        normA = res[i][4]["norm_A_used"]
        _compare(A, *res[i][:4], res[i][4], ref, 1e-10, normA, what=f"batched {i} vs LAPACK")


@pytest.mark.parametrize("precond", [0, 1])
def test_batched_in_step_matches_single_solves(P, precond):
    """svds_solve_batched with the problems in step (one launch per step of
    the first-stage iteration for all problems): every problem's result,
    counts included, is bit-identical to its own svds_solve; the singular
    values match dense LAPACK."""
    import torch
    As = _batch(7, mmin=1500, mmax=7000)
    dev = [P._lib.to_device(A) + A.shape for A in As]
    opts = dict(block_size=8, max_basis_size=35, min_restart_size=14, seed=19, autotune=0,
                precond=precond)
    _say("batched in step", [A.shape for A in As], "k=4 smallest b=8 precond", precond)
    rc, res = P.solve_batched(dev, 4, "smallest", 1e-10, nworkers=0, **opts)
    assert rc == 0, [r[4] for r in res]
    for i, (A, d) in enumerate(zip(As, dev)):
        _say("single", i, A.shape)
        sig, U, V, rn, st = P.solve(*d, 4, "smallest", 1e-10, **opts)
        assert torch.equal(sig, res[i][0]) and torch.equal(U, res[i][1]) and torch.equal(V, res[i][2])
        assert torch.equal(rn, res[i][3])
        for key in ("matvecs", "iters", "restarts", "resets", "stage_exit"):
            assert res[i][4][key] == st[key], (i, key, res[i][4][key], st[key])
    for i in range(2):
        A = As[i]
        ref = np.sort(np.linalg.svd(A.toarray(), compute_uv=False))[:4]
        _compare(A, *res[i][:4], res[i][4], ref, 1e-10, res[i][4]["norm_A_used"],
                 what=f"in-step {i} vs LAPACK")


def test_batched_in_step_many_problems_few_threads(P):
    """Twenty problems in step (more than the eight XCD runs of a launch, so
    runs hold several problems and large problems span runs) with three
    set-up threads and autotuned launch shapes: every result is
    bit-identical to its own svds_solve run afterwards."""
    import torch
    As = _batch(20, mmin=600, mmax=9000)
    dev = [P._lib.to_device(A) + A.shape for A in As]
    opts = dict(block_size=8, max_basis_size=35, min_restart_size=14, seed=23, precond=1)
    _say("batched in step, 20 problems, 3 set-up threads, autotuned")
    rc, res = P.solve_batched(dev, 4, "smallest", 1e-10, nworkers=-3, **opts)
    assert rc == 0, [r[4] for r in res]
    for i, (A, d) in enumerate(zip(As, dev)):
        _say("single", i, A.shape)
        sig, U, V, rn, st = P.solve(*d, 4, "smallest", 1e-10, **opts)
        assert res[i][4]["converged"]
        assert torch.equal(sig, res[i][0]) and torch.equal(U, res[i][1]) and torch.equal(V, res[i][2])
        assert res[i][4]["matvecs"] == st["matvecs"], i


def test_batched_empty_and_arguments(P):
    _say("batched empty")
    rc, res = P.solve_batched([], 4)
    assert rc == 0 and res == []
    lib = P.load_library()
    assert lib.svds_solve_batched(-1, None, 4, 0, 1e-10, None, None, None, None, None, None,
                                  None, None, 0, None) == -1


def test_autotuned_launch_shapes_agree(P):
    """The autotuner only changes launch shapes (lanes per row and binning),
    hence the summation order of the sparse products: results with and without
    it agree to the solve tolerance and both converge."""
    A = synth.powerlaw_workload(m=20000, n=10000)
    out = {}
    for tune in (0, 1):
        _say("powerlaw 20000x10000 k=10 largest b=8 autotune", tune)
        out[tune] = P.svds(A, 10, "largest", 1e-10, block_size=8, max_basis_size=35,
                           min_restart_size=14, seed=3, autotune=tune)
        assert out[tune][4]["converged"]
    normA = out[0][4]["norm_A_used"]
    ref = out[0][0].cpu().numpy()
    _compare(A, *out[1][:4], out[1][4], ref, 1e-10, normA, out[0][3].cpu().numpy(), "autotune")


def test_normal_method_stops_at_the_stage1_floor(P):
    """Stage 1 alone on a kappa ~ 1e6 smallest problem ends above 1e-10 ||A||
    on both sides; its values agree with the oracle's to the stage-1 level."""
    A = synth.banded_scaled(300, 150, seed=1, log_lo=-6)
    normA = float(np.linalg.norm(A.toarray(), 2))
    _say("normal method banded_scaled 300x150 smallest")
    sig, U, V, rn, st = P.svds(A, 2, "smallest", 1e-10, block_size=1, norm_A=normA, seed=7,
                               precond=P.PC_JACOBI, method=P.METHOD_NORMAL)
    ref, _, _, rr, sr = oracle.svds(A, 2, "smallest", 1e-10, block=1, seed=7, norm_A=normA,
                                    precond="jacobi", method="normal")
    assert st["stage_exit"] == 1 and not st["converged"] and not sr["converged"]
    assert float(rn.max()) > 1e-10 * normA
    spectrum = np.linalg.svd(A.toarray(), compute_uv=False)
    assert_sigma_parity(sig.cpu().numpy(), ref, spectrum, rn.cpu().numpy(), rr, normA,
                        "normal-equations method vs oracle")


def test_augmented_method_largest(P):
    A = synth.uniform_workload()
    normA = float(np.linalg.norm(A.toarray(), 2))
    _say("augmented method uniform_workload largest")
    sig, U, V, rn, st = P.svds(A, 5, "largest", 1e-10, max_basis_size=15, min_restart_size=6,
                               norm_A=normA, seed=11, method=P.METHOD_AUGMENTED)
    ref, _, _, rr, sr = oracle.svds(A, 5, "largest", 1e-10, max_basis=15, min_restart=6,
                                    norm_A=normA, seed=11, method="augmented")
    assert st["converged"] and st["stage_exit"] == 2 and st["matvecs"][0] == 0
    _compare(A, sig, U, V, rn, st, ref, 1e-10, normA, rr, "augmented vs oracle")


def test_condition_estimate(P):
    sigma = np.geomspace(1e-4, 1.0, 60)
    A, _, _, _ = synth.prescribed_dense(90, 60, sigma, seed=5)
    _say("condest prescribed 90x60 kappa 1e4")
    M = P.Matrix.from_scipy(A)
    kappa, smax, smin, (s1, s0) = P.condest(M, 0.1, seed=1)
    k_ref, smax_ref, smin_ref, _ = oracle.condest(A, 0.1, seed=1)
    assert abs(smax - 1.0) < 0.1 and abs(smin - 1e-4) / 1e-4 < 0.1
    assert abs(kappa - 1e4) / 1e4 < 0.2
    assert abs(smax - smax_ref) / smax_ref < 0.05 and abs(smin - smin_ref) / smin_ref < 0.05
    assert s1["stage_exit"] == 1 and s0["stage_exit"] == 1
    M.close()


def test_method_argument_errors(P):
    A = synth.uniform_workload(m=60, n=30, nnz_per_row=4)
    _say("method argument errors")
    for kw in (dict(method=P.METHOD_AUGMENTED), dict(relative_tol=1), dict(method=7)):
        with pytest.raises(P.SvdsError) as e:
            P.svds(A, 2, "smallest", 1e-10, **kw)
        assert e.value.code == -1


@pytest.mark.parametrize("shape", ["wide", "tall"])
def test_blockjacobi_apply_matches_oracle(P, shape):
    import torch
    A = synth.convdiff_workload(ng=12, seed=5015)
    if shape == "tall":
        A = A.T.tocsr()
    M = P.Matrix.from_scipy(A)
    N = min(A.shape)
    Aw = A.T.tocsr() if A.shape[0] < A.shape[1] else A
    rng = np.random.default_rng(4)
    for nb, b in ((1, 1), (7, 3), (64, 2), (128, 8)):
        _say("block-Jacobi apply", shape, "nb", nb, "b", b)
        R = rng.standard_normal((N, b))
        T = P.blockjacobi_apply(M, nb, torch.from_numpy(R).cuda()).cpu().numpy()
        ref = oracle.block_jacobi(Aw, nb)(R)
        assert np.allclose(T, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max()), (nb, b)
    M.close()


def test_blockjacobi_solve(P):
    """Block Jacobi (blocks of 64 columns) on a 16 x 16 convection-diffusion
    field: dense-LAPACK singular values, fewer iterations than point Jacobi,
    and through the stage-2 composition."""
    A = synth.convdiff_workload(ng=16, seed=5001)
    ref = np.sort(np.linalg.svd(A.toarray(), compute_uv=False))[:4]
    out = {}
    for name, kw in (("jacobi", dict(precond=P.PC_JACOBI)),
                     ("block", dict(precond=P.PC_BLOCKJACOBI, pc_block=64)),
                     ("block_stage2", dict(precond=P.PC_BLOCKJACOBI, pc_block=64, force_stage2=1))):
        _say("block-Jacobi solve", name)
        sig, U, V, rn, st = P.svds(A, 4, "smallest", 1e-10, block_size=1, seed=1, **kw)
        assert st["converged"], (name, st)
        _compare(A, sig, U, V, rn, st, ref, 1e-10, st["norm_A_used"], what=f"block-Jacobi {name}")
        out[name] = st
    assert out["block"]["iters"][0] < out["jacobi"]["iters"][0]
    assert out["block_stage2"]["stage_exit"] == 2


@pytest.mark.parametrize("target", ["largest", "smallest"])
def test_jacobi_davidson_stage2(P, target):
    """The JD second stage (symmetric-QMR inner solver) reaches the dense-LAPACK
    values from a loose stage 1 in fewer outer iterations than GD+k, as the
    oracle's JD stage does."""
    A = synth.uniform_workload()
    normA = float(np.linalg.norm(A.toarray(), 2))
    s_all = np.linalg.svd(A.toarray(), compute_uv=False)
    ref = s_all[:5] if target == "largest" else np.sort(s_all)[:5]
    out = {}
    for name, solver in (("gdk", P.STAGE2_GDK), ("jd", P.STAGE2_JD)):
        _say("uniform_workload stage 2", name, target)
        sig, U, V, rn, st = P.svds(A, 5, target, 1e-10, max_basis_size=15, min_restart_size=6,
                                   norm_A=normA, seed=5, stage1_tol=1e-4, stage2_solver=solver)
        assert st["converged"] and st["stage_exit"] == 2, (name, st)
        _compare(A, sig, U, V, rn, st, ref, 1e-10, normA, what=f"stage 2 {name}")
        out[name] = st
    o_s, _, _, o_rn, o_st = oracle.svds(A, 5, target, 1e-10, max_basis=15, min_restart=6,
                                        norm_A=normA, seed=5, stage1_tol=1e-4, stage2_solver="jd")
    assert out["jd"]["inner_iters"] > 0 and out["gdk"]["inner_iters"] == 0
    assert out["jd"]["iters"][1] < out["gdk"]["iters"][1]
    assert_sigma_parity(o_s, ref, s_all, o_rn, np.zeros(5), normA, "oracle JD vs LAPACK")


@pytest.mark.parametrize("pc", ["jacobi", "blockjacobi"])
def test_preconditioned_jd_near_the_null_space_of_B(P, pc):
    """Five smallest values of a kappa ~ 1e6 banded 1200 x 600 matrix, next to
    the 600 zero eigenvalues of B: the default second stage (JD with the
    preconditioned symmetric-QMR correction) converges in a few outer
    iterations, as the oracle's does, to the dense-LAPACK values."""
    A = synth.banded_scaled(1200, 600, seed=2005, log_lo=-6)
    normA = float(np.linalg.norm(A.toarray(), 2))
    ref = np.sort(np.linalg.svd(A.toarray(), compute_uv=False))[:5]
    kw = dict(precond=P.PC_JACOBI) if pc == "jacobi" else dict(precond=P.PC_BLOCKJACOBI,
                                                                pc_block=64)
    _say("preconditioned JD banded_scaled 1200x600 smallest", pc)
    sig, U, V, rn, st = P.svds(A, 5, "smallest", 1e-10, block_size=4, max_basis_size=35,
                               min_restart_size=14, norm_A=normA, seed=2005, **kw)
    assert st["converged"] and st["stage_exit"] == 2, st
    assert st["inner_iters"] > 0 and st["iters"][1] <= 20, st
    _compare(A, sig, U, V, rn, st, ref, 1e-10, normA, what=f"JD {pc} vs LAPACK")
    o_s, _, _, o_rn, o_st = oracle.svds(A, 5, "smallest", 1e-10, block=4, max_basis=35,
                                        min_restart=14, norm_A=normA, seed=2005, precond=pc,
                                        pc_block=64)
    assert o_st["converged"] and o_st["iters"][1] <= 20
    spectrum = np.linalg.svd(A.toarray(), compute_uv=False)
    assert_sigma_parity(sig.cpu().numpy(), o_s, spectrum, rn.cpu().numpy(), o_rn, normA,
                        f"JD {pc} vs oracle")


def test_jacobi_davidson_ill_conditioned_and_wide(P):
    A = synth.banded_scaled(300, 150, seed=1, log_lo=-6)
    normA = float(np.linalg.norm(A.toarray(), 2))
    _say("JD stage 2 banded_scaled 300x150 smallest")
    sig, U, V, rn, st = P.svds(A, 3, "smallest", 1e-10, block_size=1, norm_A=normA, seed=7,
                               precond=P.PC_JACOBI, stage2_solver=P.STAGE2_JD)
    s = np.sort(np.linalg.svd(A.toarray(), compute_uv=False))[:3]
    assert st["converged"] and st["stage_exit"] == 2
    _compare(A, sig, U, V, rn, st, s, 1e-10, normA, what="JD kappa 2e6 vs LAPACK")
    W = synth.random_uniform_rows(300, 600, 12, seed=21)
    nW = float(np.linalg.norm(W.toarray(), 2))
    _say("JD stage 2 wide 300x600 b=2 forced")
    sig, U, V, rn, st = P.svds(W, 4, "smallest", 1e-10, block_size=2, norm_A=nW, seed=3,
                               stage1_tol=1e-3, stage2_solver=P.STAGE2_JD)
    s = np.sort(np.linalg.svd(W.toarray(), compute_uv=False))[:4]
    assert st["converged"] and st["stage_exit"] == 2
    _compare(A=W, sig=sig, U=U, V=V, rn=rn, st=st, ref_sig=s, tol=1e-10, normA=nW)


@pytest.mark.parametrize("target", ["largest", "smallest"])
def test_repeated_singular_values(P, target):
    """Singular values of multiplicity 3 and 2 (a scrambled sparse diagonal
    matrix): the projected matrices carry equal Ritz values, which the
    extraction deflates as equal poles; the values match the prescribed
    ones and the vectors stay orthonormal with eq. (res) residuals."""
    rng = np.random.default_rng(41)
    m, n = 900, 600
    s = np.concatenate([[5.0, 5.0, 5.0, 4.0, 4.0], np.linspace(3.5, 0.5, n - 10), [0.2, 0.2, 0.2, 0.1, 0.1]])
    rows = rng.permutation(m)[:n]
    cols = rng.permutation(n)
    A = sp.csr_matrix((s, (rows, cols)), shape=(m, n))
    normA = 5.0
    ref = np.sort(s)[::-1][:5] if target == "largest" else np.sort(s)[:5]
    _say("repeated singular values 900x600", target)
    sig, U, V, rn, st = P.svds(A, 5, target, 1e-10, block_size=4, max_basis_size=30,
                               min_restart_size=12, norm_A=normA, seed=41)
    assert st["converged"], st
    _compare(A, sig, U, V, rn, st, ref, 1e-10, normA, what=f"repeated values {target}")
