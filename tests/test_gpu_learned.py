"""Learned preconditioner on the GPU: kernels against the FP64 CPU reference
(oracle/learned.py), training on the GPU, and what the trained network gains
over point Jacobi and no preconditioning.

Every test prints the case it runs before touching the GPU."""
import numpy as np
import pytest

import oracle
import oracle.learned as L
import synth
from parity import assert_sigma_parity

pytestmark = pytest.mark.gpu

CO = 16 + 32 + 64 + 32 + 32  # offset of o in the forward cache (units of N)


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


def _dev(x, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).cuda()


def _cos(a, b):
    a = np.ravel(a)
    b = np.ravel(b)
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


def _theta(seed):
    rng = np.random.default_rng(seed)
    th = rng.uniform(-1, 1, L.NPARAMS) * 0.5
    return th.astype(np.float32).astype(np.float64)  # representable in FP32


@pytest.mark.parametrize("shape", ["wide", "tall"])
def test_features_match_reference(P, shape):
    A = synth.convdiff_workload(ng=12, seed=5007)
    if shape == "tall":
        A = A.T.tocsr()
    _say("lpc features", shape, A.shape)
    M = P.Matrix.from_scipy(A)
    f = P.lpc_features(M).cpu().numpy()
    ref = L.features(L.Operator(A))
    assert f.shape == ref.shape
    assert np.allclose(f, ref, rtol=1e-5, atol=1e-5 * np.abs(ref).max())
    M.close()


@pytest.mark.parametrize("degree", [1, 8, 15])
def test_forward_matches_reference(P, degree):
    import torch
    A = synth.convdiff_workload(ng=12, seed=5008)
    _say("lpc forward degree", degree)
    M = P.Matrix.from_scipy(A)
    op = L.Operator(A)
    fr = L.features(op)
    th = _theta(1)
    coef_ref, cache_ref = L.forward(op, th, fr, degree)
    coef, cache = P.lpc_forward(M, _dev(th, torch.float32), _dev(fr, torch.float32), degree)
    coef = coef.cpu().numpy()
    N = op.N
    o = cache.cpu().numpy()[CO * N:(CO + 8) * N].reshape(N, 8)
    # BF16 operands, FP32 accumulation
    assert np.all(np.abs(o - cache_ref["o_raw"]) <= 3e-2 * (1 + np.abs(cache_ref["o_raw"])))
    scale = np.abs(coef_ref).max(axis=1, keepdims=True)
    assert np.all(np.abs(coef[:, :degree + 1] - coef_ref) <= 6e-2 * scale)
    assert np.all(coef[:, degree + 1:] == 0.0)
    M.close()


def test_backward_matches_reference(P):
    import torch
    A = synth.convdiff_workload(ng=12, seed=5009)
    _say("lpc backward")
    M = P.Matrix.from_scipy(A)
    op = L.Operator(A)
    fr = L.features(op)
    th = _theta(2)
    deg = 8
    coef_ref, cache_ref = L.forward(op, th, fr, deg)
    rng = np.random.default_rng(3)
    R = rng.standard_normal((op.N, 6))
    Q, E = L.make_pairs(op, R)
    loss_ref, dc_ref = L.loss_and_dc(op, coef_ref, Q, E, deg)
    g_ref = L.backward(op, th, cache_ref, dc_ref)
    thd = _dev(th, torch.float32)
    coef, cache = P.lpc_forward(M, thd, _dev(fr, torch.float32), deg)
    dc = np.zeros((op.N, 16), dtype=np.float32)
    dc[:, :deg + 1] = dc_ref
    g = P.lpc_backward(M, thd, cache, deg, _dev(dc, torch.float32)).cpu().numpy()
    assert _cos(g, g_ref) >= 0.999
    gr = L.unpack(g_ref)
    gg = L.unpack(g)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert _cos(gg[name], gr[name]) >= 0.99, name
    M.close()


def test_loss_and_dcoef_match_reference(P):
    import torch
    A = synth.convdiff_workload(ng=12, seed=5010)
    _say("lpc loss")
    M = P.Matrix.from_scipy(A)
    op = L.Operator(A)
    deg = 8
    th = _theta(4)
    coef_ref, _ = L.forward(op, th, L.features(op), deg)
    coef32 = np.zeros((op.N, 16), dtype=np.float32)
    coef32[:, :deg + 1] = coef_ref
    rng = np.random.default_rng(5)
    R = rng.standard_normal((op.N, 11))
    R[:, 4] = 0.0  # a zero residual is an invalid pair on both sides
    Q, E = L.make_pairs(op, R)
    loss_ref, dc_ref = L.loss_and_dc(op, coef32[:, :deg + 1].astype(np.float64), Q, E, deg)
    loss, dc = P.lpc_loss(M, _dev(R, torch.float64), _dev(coef32, torch.float32), deg)
    dc = dc.cpu().numpy()
    assert abs(loss - loss_ref) <= 1e-4 * max(loss_ref, 1e-3)
    assert _cos(dc[:, :deg + 1], dc_ref) >= 0.9999
    assert np.all(dc[:, deg + 1:] == 0.0)
    M.close()


@pytest.mark.parametrize("shape", ["wide", "tall"])
def test_apply_matches_reference(P, shape):
    """K(R) in FP64 with the same (FP32-representable) coefficients."""
    import torch
    A = synth.convdiff_workload(ng=12, seed=5011)
    if shape == "tall":
        A = A.T.tocsr()
    _say("lpc apply", shape)
    M = P.Matrix.from_scipy(A)
    op = L.Operator(A)
    rng = np.random.default_rng(6)
    for deg, nb in ((0, 1), (3, 2), (8, 5), (15, 8)):
        c = rng.uniform(0.1, 2.0, (op.N, 16)).astype(np.float32)
        c[:, deg + 1:] = 0.0
        R = rng.standard_normal((op.N, nb))
        T = P.lpc_apply(M, _dev(c, torch.float32), deg, _dev(R, torch.float64)).cpu().numpy()
        ref = L.apply(op, c[:, :deg + 1].astype(np.float64), R, deg)
        assert np.allclose(T, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max()), (deg, nb)
    M.close()


def test_adam_matches_reference(P):
    import torch
    _say("lpc adam")
    rng = np.random.default_rng(7)
    n = 1000
    th = rng.standard_normal(n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    thd, md, vd = _dev(th, torch.float32), _dev(m, torch.float32), _dev(v, torch.float32)
    th64, m64, v64 = th.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in range(1, 4):
        g = rng.standard_normal(n).astype(np.float32)
        P.lpc_adam(thd, _dev(g, torch.float32), md, vd, step, 1e-2)
        L.adam_step(th64, g.astype(np.float64), m64, v64, step, 1e-2)
    assert np.allclose(thd.cpu().numpy(), th64, rtol=1e-5, atol=1e-6)


def test_collect_residuals_match_oracle(P):
    """The residuals the GPU solve captures are the oracle's at the same
    iterations (same method readings, same counter-based start), up to the
    sign of the Ritz vector, which the small eigensolvers fix differently."""
    A = synth.convdiff_workload(ng=12, seed=5012)
    _say("collect residuals 12x12 k=3 smallest every 2")
    M = P.Matrix.from_scipy(A)
    R, st = P.collect_residuals(M, 3, "smallest", 1e-10, every=2, max_pairs=4, block_size=1,
                                seed=3, precond=P.PC_JACOBI)
    cap = {"every": 2, "max": 4}
    oracle.svds(A, 3, "smallest", 1e-10, block=1, seed=3, precond="jacobi", capture=cap)
    Rr = np.array(cap["R"]).T
    R = R.cpu().numpy()
    assert R.shape == Rr.shape == (min(A.shape), 4)
    for j in range(2):
        sgn = 1.0 if R[:, j] @ Rr[:, j] >= 0 else -1.0
        assert np.allclose(sgn * R[:, j], Rr[:, j], rtol=1e-7,
                           atol=1e-9 * np.abs(Rr[:, j]).max()), j
    M.close()


def _grid_dense_sigma(A, k):
    return np.sort(np.linalg.svd(A.toarray(), compute_uv=False))[:k]


def test_trained_network_beats_jacobi_and_none(P):
    """Training on the GPU from residuals of Jacobi-preconditioned solves on
    three coefficient fields (seeds 5001-5003, 16 x 16 grids), evaluated on a
    fourth (seed 5000): the learned preconditioner reaches the same singular
    values as dense LAPACK in fewer iterations and less time than point
    Jacobi and no preconditioning."""
    import time

    import torch
    sets = []
    for sd in (5001, 5002, 5003):
        A = synth.convdiff_workload(ng=16, seed=sd)
        _say("training residuals seed", sd)
        M = P.Matrix.from_scipy(A)
        R, st = P.collect_residuals(M, 4, "smallest", 1e-10, every=3, max_pairs=60, block_size=1,
                                    seed=1, precond=P.PC_JACOBI)
        assert st["converged"] and R.shape[1] == 60
        sets.append((M, R))
    bias = np.full(8, -8.0)
    bias[7] = 0.0
    params = P.lpc_init(seed=0, out_bias=bias)
    _say("training 80 steps")
    hist = P.lpc_train(sets, 8, 80, 1e-2, params)
    assert np.all(np.isfinite(hist)) and hist[-1] < 0.7 * hist[0], hist[[0, -1]]
    B = synth.convdiff_workload(ng=16, seed=5000)
    ref = _grid_dense_sigma(B, 4)
    spec = np.linalg.svd(B.toarray(), compute_uv=False)
    MB = P.Matrix.from_scipy(B)
    res = {}
    for name, kw in (("none", dict(precond=P.PC_NONE)), ("jacobi", dict(precond=P.PC_JACOBI)),
                     ("learned", dict(precond=P.PC_LEARNED, pc_model=params, pc_degree=8))):
        _say("eval solve", name)
        MB.solve(4, "smallest", 1e-10, block_size=1, seed=1, **kw)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sig, U, V, rn, st = MB.solve(4, "smallest", 1e-10, block_size=1, seed=1, **kw)
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0, sum(st["iters"]), st)
        assert st["converged"], (name, st)
        assert_sigma_parity(sig.cpu().numpy(), ref, spec, rn.cpu().numpy(), np.zeros(4),
                            st["norm_A_used"], f"learned-gain {name} vs LAPACK")
        assert float(rn.max()) <= 1e-10 * st["norm_A_used"]
    print("[result]", {k: (round(v[0], 4), v[1]) for k, v in res.items()}, flush=True)
    assert res["learned"][1] < 0.5 * res["jacobi"][1]
    assert res["learned"][1] < 0.5 * res["none"][1]
    assert res["learned"][0] < res["jacobi"][0] and res["learned"][0] < res["none"][0]
    for M, _ in sets:
        M.close()
    MB.close()


@pytest.mark.parametrize("solver", ["jd", "gdk"])
def test_learned_stage2_composition(P, solver):
    """Stage 2 on B with the learned K in the composition [K A^T r_u; A K r_v],
    inside the JD correction's symmetric QMR or on the GD+k residuals."""
    A = synth.convdiff_workload(ng=12, seed=5013)
    _say("learned stage 2 12x12 k=3 smallest", solver)
    params = P.lpc_init(seed=5)
    sig, U, V, rn, st = P.svds(A, 3, "smallest", 1e-10, block_size=1, seed=2, force_stage2=1,
                               precond=P.PC_LEARNED, pc_model=params, pc_degree=6,
                               stage2_solver=P.STAGE2_JD if solver == "jd" else P.STAGE2_GDK)
    assert st["converged"] and st["stage_exit"] == 2 and st["iters"][1] >= 0
    ref = _grid_dense_sigma(A, 3)
    assert_sigma_parity(sig.cpu().numpy(), ref, np.linalg.svd(A.toarray(), compute_uv=False),
                        rn.cpu().numpy(), np.zeros(3), st["norm_A_used"],
                        f"learned stage 2 {solver} vs LAPACK")
    assert float(rn.max()) <= 1e-10 * st["norm_A_used"]


def test_learned_requires_model(P):
    A = synth.convdiff_workload(ng=8, seed=5014)
    _say("learned without model")
    with pytest.raises(P.SvdsError) as e:
        P.svds(A, 2, "smallest", 1e-10, precond=P.PC_LEARNED)
    assert e.value.code == -1
