"""The one-pass product with C = A_w^T A_w (svds_matrix_normal) against SciPy's
two sparse products, and solves through it against the dense SVD and against
solves that take the two products.

Every test prints the case it runs before touching the GPU."""
import numpy as np
import pytest
import scipy.sparse as sp

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


def _banded_with_gaps(m=20011, n=10007, seed=7):
    """Banded rows with a run of empty rows (whole empty blocks) and a ragged
    last block."""
    A = synth.banded_scaled(m, n, seed=seed)
    keep = np.ones(m)
    keep[5000:5400] = 0.0
    keep[7001] = 0.0
    A = sp.diags(keep) @ A
    A = sp.csr_matrix(A)
    A.eliminate_zeros()
    A.sort_indices()
    return A


def _check(A, X, Z):
    W = A.T @ (A @ X)
    scale = abs(A).T @ (abs(A) @ abs(X))
    assert np.all(np.abs(Z - W) <= 1e-13 * scale + 1e-300)


@pytest.mark.parametrize("b", [1, 2, 3, 4, 8])
def test_normal_product_matches_scipy(P, b):
    import torch
    A = _banded_with_gaps()
    _say("normal product banded", A.shape, A.nnz, "b", b)
    M = P.Matrix.from_scipy(A)
    X = np.random.default_rng(b).standard_normal((A.shape[1], b))
    Z, used = M.normal(torch.from_numpy(X).cuda())
    assert used == 1
    _check(A, X, Z.cpu().numpy())
    Z2, used2 = M.normal(torch.from_numpy(X).cuda(), fused=False)
    assert used2 == 0
    _check(A, X, Z2.cpu().numpy())
    M.close()


def test_normal_product_deterministic(P):
    import torch
    A = _banded_with_gaps(seed=8)
    _say("normal product determinism", A.shape)
    M = P.Matrix.from_scipy(A)
    X = torch.from_numpy(np.random.default_rng(0).standard_normal((A.shape[1], 4))).cuda()
    Z1, u1 = M.normal(X)
    Z2, u2 = M.normal(X)
    assert u1 == u2 == 1 and torch.equal(Z1, Z2)
    M.close()


def test_normal_product_wide_and_tiny(P):
    """m < n: the work matrix is A^T, the product A A^T.  Then matrices with a
    single block, a single row and a single column."""
    import torch
    cases = [("wide banded", sp.csr_matrix(synth.banded_scaled(6000, 3000, seed=9).T)),
             ("one block", synth.banded_scaled(40, 20, seed=10, band=8, per_row=4)),
             ("one row", sp.csr_matrix(np.arange(1.0, 6.0)[None, :])),
             ("one column", sp.csr_matrix(np.arange(1.0, 6.0)[:, None]))]
    for name, A in cases:
        A.sort_indices()
        _say("normal product", name, A.shape)
        M = P.Matrix.from_scipy(A)
        Aw = A if A.shape[0] >= A.shape[1] else sp.csr_matrix(A.T)
        X = np.random.default_rng(1).standard_normal((Aw.shape[1], 3))
        Z, used = M.normal(torch.from_numpy(X).cuda())
        _check(Aw, X, Z.cpu().numpy())
        M.close()


@pytest.mark.parametrize("h,want", [(192, 1), (193, 0)])
def test_window_of_512_columns(P, h, want):
    """Square 5120 x 5120, row i with 16 nonzeros in [i - h, i + h] (both ends
    always among them).  At h = 192 every 128-row block spans exactly 512
    columns, the widest window whose column fits the packed index's 9 bits:
    the one-pass product runs.  At h = 193 the blocks span 514 columns, the
    64-row blocks' windows add up to more than 4 x the column count, and
    there is no plan.  Both agree with SciPy.  Block width 2: at 4 the
    windows' partial sums of so sparse a band would cost more bytes than the
    two products, and the product would not be taken either way."""
    import torch
    n = 128 * 40
    rng = np.random.default_rng(12)
    rows, cols = [], []
    for i in range(n):
        c = {min(max(i - h, 0), n - 1), min(max(i + h, 0), n - 1), i}
        while len(c) < 16:
            c.add(int(np.clip(i + rng.integers(-h, h + 1), 0, n - 1)))
        rows += [i] * len(c)
        cols += sorted(c)
    A = sp.csr_matrix((rng.standard_normal(len(rows)), (rows, cols)), shape=(n, n))
    A.sort_indices()
    _say("normal product, windows of", 128 + 2 * h, "columns", A.shape)
    M = P.Matrix.from_scipy(A)
    X = np.random.default_rng(4).standard_normal((n, 2))
    Z, used = M.normal(torch.from_numpy(X).cuda())
    assert used == want
    _check(A, X, Z.cpu().numpy())
    M.close()


def test_normal_product_falls_back_for_scattered_rows(P):
    import torch
    A = synth.powerlaw_workload(m=20000, n=10000)
    _say("normal product power-law rows (no plan)", A.shape)
    M = P.Matrix.from_scipy(A)
    X = np.random.default_rng(2).standard_normal((A.shape[1], 4))
    Z, used = M.normal(torch.from_numpy(X).cuda())
    assert used == 0
    _check(A, X, Z.cpu().numpy())
    M.close()


def test_window_limits(P):
    """A row block whose window is wider than the plan allows at every block
    height (a dense row across 5000 columns): no plan, products still right."""
    import torch
    A = synth.banded_scaled(8000, 6000, seed=11)
    wide = sp.csr_matrix((np.linspace(1.0, 2.0, 5000), (np.full(5000, 100), np.arange(5000))),
                         shape=A.shape)
    A = sp.csr_matrix(A + wide)
    A.sort_indices()
    _say("normal product, a 5000-wide row", A.shape)
    M = P.Matrix.from_scipy(A)
    X = np.random.default_rng(3).standard_normal((A.shape[1], 2))
    Z, used = M.normal(torch.from_numpy(X).cuda())
    assert used == 0
    _check(A, X, Z.cpu().numpy())
    M.close()


@pytest.mark.parametrize("target", ["smallest", "largest"])
def test_solve_through_the_one_pass_product(P, target):
    A = synth.banded_scaled(3000, 1500, seed=13, log_lo=-3)
    normA = float(np.linalg.norm(A.toarray(), 2))
    s_all = np.linalg.svd(A.toarray(), compute_uv=False)
    ref = np.sort(s_all)[:4] if target == "smallest" else s_all[:4]
    _say("solve banded 3000x1500 through the one-pass product", target)
    out = {}
    for fused in (1, 0):
        pc = P.PC_JACOBI if target == "smallest" else P.PC_NONE
        sig, U, V, rn, st = P.svds(A, 4, target, 1e-10, block_size=2, norm_A=normA, seed=5,
                                   precond=pc, fused_gram=fused, profile=1)
        assert st["converged"], st
        assert (st["gram_calls"] > 0) == bool(fused), st
        sig = sig.cpu().numpy()
        rn = rn.cpu().numpy()
        assert_sigma_parity(sig, ref, s_all, rn, np.zeros(4), normA, f"one-pass {fused} vs LAPACK")
        Uc, Vc = U.cpu().numpy(), V.cpu().numpy()
        r = np.sqrt(np.sum((A @ Vc - Uc * sig) ** 2, axis=0) +
                    np.sum((A.T @ Uc - Vc * sig) ** 2, axis=0))
        assert np.all(r <= 1.01e-10 * normA), r
        out[fused] = (sig, rn)
    assert_sigma_parity(out[1][0], out[0][0], s_all, out[1][1], out[0][1], normA,
                        "one-pass vs two products")


def test_normal_product_arguments(P):
    import torch
    A = synth.banded_scaled(400, 200, seed=14)
    _say("normal product argument errors", A.shape)
    M = P.Matrix.from_scipy(A)
    lib = P.load_library()
    X = torch.zeros((200, 9), dtype=torch.float64, device="cuda")
    Z = torch.empty_like(X)
    for b in (0, 9):
        rc = lib.svds_matrix_normal(M.handle, b, X.data_ptr(), Z.data_ptr(), 1, None, None)
        assert rc == -1, (b, rc)
    assert lib.svds_matrix_normal(M.handle, 4, None, Z.data_ptr(), 1, None, None) == -1
    M.close()
