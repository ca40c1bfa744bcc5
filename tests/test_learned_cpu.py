"""CPU pins of the FP64 reference of the learned preconditioner."""
import math

import numpy as np
import numpy.polynomial.chebyshev as Ch
import pytest
import scipy.sparse as sp

import oracle
import oracle.learned as L
import synth


def _small():
    return synth.convdiff_workload(ng=8, seed=5003)  # 32 dropped rows: 32 x 64 -> work matrix A^T


def _random_theta(seed=0, scale=0.5):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, L.NPARAMS) * scale


def test_parameter_count_and_layout():
    assert L.NPARAMS == 16 * 32 + 32 + 64 * 32 + 32 + 32 * 8 + 8 == 2888
    th = np.arange(L.NPARAMS, dtype=np.float64)
    assert np.array_equal(L.pack(L.unpack(th)), th)


def test_reciprocal_chebyshev_closed_form():
    """The closed-form coefficients of 1/(x + delta) agree with a numerical
    Chebyshev interpolant of high degree (numpy)."""
    for delta in (1e-2, 0.3, 1.0):
        ref = Ch.chebinterpolate(lambda y: 1.0 / ((y + 1) / 2 + delta), 300)
        assert np.allclose(L.reciprocal_chebyshev(delta, 12), ref[:13], rtol=1e-10, atol=1e-10)


def test_jackson_factors():
    """g_0 = 1, decreasing, and the damped series of a positive function is
    positive: the Jackson-damped series of |y| stays >= 0 on [-1, 1]."""
    for d in (0, 1, 8, 15):
        g = L.jackson(d)
        assert g.shape == (d + 1,) and abs(g[0] - 1) < 1e-14
        assert np.all(np.diff(g) <= 1e-15) and np.all(g >= -1e-15)
    y = np.linspace(-1, 1, 4001)
    c = Ch.chebinterpolate(np.abs, 200)[:16] * L.jackson(15)
    assert Ch.chebval(y, c).min() >= -1e-12


def test_every_row_polynomial_is_positive():
    """Whatever the network outputs, each row's polynomial is a positive
    mixture of Jackson-damped reciprocals, hence positive on [0, 1]."""
    A = _small()
    op = L.Operator(A)
    f = L.features(op)
    x = np.linspace(0, 1, 2001)
    for seed in range(3):
        theta = _random_theta(seed, scale=2.0)
        for deg in (1, 8, 15):
            c, _ = L.forward(op, theta, f, deg)
            P = Ch.chebval(2 * x - 1, c.T)  # rows x points
            assert P.min() > 0.0


def test_degree_zero_unit_coefficient_is_point_jacobi():
    A = _small()
    op = L.Operator(A)
    R = np.random.default_rng(1).standard_normal((op.N, 3))
    Aw = L.work_matrix(A).toarray()
    d = np.sum(Aw * Aw, axis=0)
    c = np.ones((op.N, 1))
    assert np.allclose(L.apply(op, c, R, 0), R / d[:, None], rtol=1e-14, atol=0)


def test_chebyshev_polynomial_matches_spectral_evaluation():
    """Row-constant coefficients: K = D^-1/2 p(M) D^-1/2 with p = sum c_l T_l(2x-1);
    evaluated independently through the eigendecomposition of the dense M and
    numpy's Chebyshev series."""
    A = _small()
    op = L.Operator(A)
    Aw = L.work_matrix(A).toarray()
    D = np.sum(Aw * Aw, axis=0)
    Mh = (Aw / np.sqrt(D)).T @ (Aw / np.sqrt(D)) / op.rho
    w, Q = np.linalg.eigh(Mh)
    assert w.min() > -1e-12 and w.max() <= 1 + 1e-12  # Gershgorin bound
    rng = np.random.default_rng(2)
    deg = 8
    coef = rng.standard_normal(deg + 1)
    pw = Ch.chebval(2 * w - 1, coef)
    Kd = np.diag(D ** -0.5) @ Q @ np.diag(pw) @ Q.T @ np.diag(D ** -0.5)
    R = rng.standard_normal((op.N, 2))
    c = np.tile(coef, (op.N, 1))
    assert np.allclose(L.apply(op, c, R, deg), Kd @ R, rtol=1e-11, atol=1e-11 * np.abs(Kd @ R).max())


def test_aggregation_is_a_row_stochastic_average_and_agg_t_its_adjoint():
    op = L.Operator(_small())
    rng = np.random.default_rng(3)
    h = rng.standard_normal((op.N, 5))
    g = rng.standard_normal((op.N, 5))
    assert np.allclose(op.agg(np.ones((op.N, 1))), 1.0, atol=1e-14)
    assert math.isclose(np.sum(op.agg(h) * g), np.sum(h * op.agg_t(g)), rel_tol=1e-12)
    # dense weights: |A|^T |A| with rows scaled to sum one
    Wd = abs(L.work_matrix(_small()).toarray())
    Wd = Wd.T @ Wd
    Wd = Wd / Wd.sum(axis=1, keepdims=True)
    assert np.allclose(op.agg(h), Wd @ h, atol=1e-13)


def test_features_on_a_diagonal_matrix():
    """A diagonal matrix: C is diagonal, M = I / rho with rho = 1, so
    f2 = f3 = f5 = 1, f4 = 1 and f1 = log d - mean log d."""
    dvals = np.array([1.0, 2.0, 3.0, 4.0, 0.5])
    A = synth.to_csr(sp.diags(dvals).tocsr())
    op = L.Operator(A)
    f = L.features(op)
    assert op.rho == pytest.approx(1.0)
    assert np.allclose(f[:, [0, 2, 3, 4, 5]], 1.0)
    ld = np.log(dvals ** 2)
    assert np.allclose(f[:, 1], ld - ld.mean())
    assert np.all(f[:, 6:] == 0)


def test_gelu_and_derivative():
    x = np.linspace(-6, 6, 101)
    from scipy.stats import norm
    assert np.allclose(L.gelu(x), x * norm.cdf(x), atol=1e-15)
    h = 1e-6
    assert np.allclose(L.gelu_grad(x), (L.gelu(x + h) - L.gelu(x - h)) / (2 * h), atol=1e-9)


def _pairs(op, n=6, seed=4):
    rng = np.random.default_rng(seed)
    R = rng.standard_normal((op.N, n))
    E = rng.standard_normal((op.N, n))
    E[:, 2] = 0.0  # an invalid pair is skipped
    return R, E


def _loss(op, theta, f, R, E, deg):
    c, _ = L.forward(op, theta, f, deg)
    return L.loss_and_dc(op, c, R, E, deg)[0]


@pytest.mark.parametrize("deg", [0, 4, 8])
def test_backward_matches_central_differences(deg):
    A = _small()
    op = L.Operator(A)
    f = L.features(op)
    theta = _random_theta(5)
    R, E = _pairs(op)
    c, cache = L.forward(op, theta, f, deg)
    loss, dc = L.loss_and_dc(op, c, R, E, deg)
    assert 0.0 <= loss <= 1.0
    grad = L.backward(op, theta, cache, dc)
    rng = np.random.default_rng(6)
    idx = rng.choice(L.NPARAMS, 80, replace=False)
    h = 1e-5
    fd = np.empty(idx.size)
    for q, i in enumerate(idx):
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd[q] = (_loss(op, tp, f, R, E, deg) - _loss(op, tm, f, R, E, deg)) / (2 * h)
    err = np.abs(fd - grad[idx])
    assert np.all(err <= 1e-6 * np.abs(grad).max() + 1e-6 * np.abs(fd)), (err.max(), np.abs(grad).max())


def test_loss_is_scale_and_sign_invariant():
    op = L.Operator(_small())
    f = L.features(op)
    R, E = _pairs(op)
    c, _ = L.forward(op, _random_theta(7), f, 5)
    l0, _ = L.loss_and_dc(op, c, R, E, 5)
    l1, _ = L.loss_and_dc(op, -3.0 * c, R, E, 5)
    assert math.isclose(l0, l1, rel_tol=1e-12)
    # a perfect output (t parallel to e) has zero loss
    c0 = np.zeros((op.N, 1)); c0[:, 0] = 1.0
    T = L.apply(op, c0, R, 0)
    l2, _ = L.loss_and_dc(op, c0, R, -2.0 * T, 0)
    assert l2 < 1e-14


def test_adam_first_step_moves_by_lr_times_sign():
    theta = np.zeros(5)
    g = np.array([1e-3, -2.0, 5.0, -1e-6, 0.0])
    m = np.zeros(5); v = np.zeros(5)
    L.adam_step(theta, g, m, v, 1, 0.01)
    # m_hat = g and v_hat = g^2 after one step: the update is -lr g / (|g| + eps)
    assert np.allclose(theta, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert theta[4] == 0.0


def test_pairs_from_residuals():
    op = L.Operator(_small())
    rng = np.random.default_rng(8)
    R = rng.standard_normal((op.N, 4)) * np.array([1.0, 1e-8, 3.0, 0.0])
    Q, E = L.make_pairs(op, R)
    assert np.allclose(np.linalg.norm(E[:, :3], axis=0), 1.0) and np.all(E[:, 3] == 0)
    Aw = L.work_matrix(_small()).toarray()
    assert np.allclose(Q, Aw.T @ Aw @ E, atol=1e-12)
    # the exact inverse of C has zero loss on every pair
    Kinv = np.linalg.pinv(Aw.T @ Aw)
    T = Kinv @ Q
    te = np.sum(T * E, 0)[:3]
    assert np.allclose(te ** 2, np.sum(T * T, 0)[:3] * np.sum(E * E, 0)[:3], rtol=1e-8)


def test_oracle_capture_and_training_beat_jacobi():
    """Residuals captured from an oracle solve of a small convection-diffusion
    problem; Adam steps lower the mean pair loss, and the trained
    preconditioner reaches the same singular values in fewer iterations than
    point Jacobi on a problem with another coefficient field."""
    A = synth.convdiff_workload(ng=16, seed=5001)
    cap = {"every": 3, "max": 60}
    sig, U, V, rn, st = oracle.svds(A, 4, "smallest", 1e-10, block=1, seed=1, precond="jacobi",
                                    capture=cap)
    assert st["converged"] and len(cap["R"]) == 60 and all(0 <= i < 5 for i in cap["idx"])
    op = L.Operator(A)
    f = L.features(op)
    Q, E = L.make_pairs(op, np.array(cap["R"]).T)
    deg = 8
    bias = np.full(L.NOUT, -8.0)
    bias[-1] = 0.0  # start from the flattest component (delta = 1)
    theta = L.init_params(np.random.default_rng(0), bias=bias)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    losses = []
    for step in range(1, 41):
        c, cache = L.forward(op, theta, f, deg)
        loss, dc = L.loss_and_dc(op, c, Q, E, deg)
        losses.append(loss)
        L.adam_step(theta, L.backward(op, theta, cache, dc), m, v, step, 1e-2)
    assert losses[-1] < 0.7 * losses[0], losses
    B = synth.convdiff_workload(ng=16, seed=5000)
    opb = L.Operator(B)
    cb, _ = L.forward(opb, theta, L.features(opb), deg)
    K = lambda Rb: L.apply(opb, cb, Rb, deg)
    s1, _, _, _, stj = oracle.svds(B, 4, "smallest", 1e-10, block=1, seed=1, precond="jacobi")
    s2, _, _, _, stl = oracle.svds(B, 4, "smallest", 1e-10, block=1, seed=1, precond=K)
    assert stj["converged"] and stl["converged"]
    assert np.max(np.abs(s2 - s1) / s1) < 1e-9
    assert stl["iters"][0] < 0.5 * stj["iters"][0], (stl["iters"], stj["iters"])
