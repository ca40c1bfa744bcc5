"""The allocation-free product with C = A_w^T A_w (svds_matrix_normal_noalloc)
against the allocating one (svds_matrix_normal), through the C ABI: the same
bits on two calls in a row, the second with a smaller input, for the one-pass
product and for the two-SpMM fallback; sizes beyond the static scratch are
rejected."""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1607_01404_amd as P
    L = P.load_library()
    L.svds_matrix_normal_noalloc.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                                             C.POINTER(C.c_int), C.c_void_p]
    L.svds_matrix_normal_noalloc.restype = C.c_int
    return L


def _pair(lib, M, X, fused):
    """(Z from svds_matrix_normal, Z from the no-alloc entry point, used flags)."""
    import torch
    import paper_1607_01404_amd as P
    Zref, used = M.normal(X, fused=fused)
    Z = torch.full_like(X, float("nan"))
    u = C.c_int(-1)
    rc = lib.svds_matrix_normal_noalloc(M.handle, X.shape[1], X.data_ptr(), Z.data_ptr(),
                                        int(fused), C.byref(u), None)
    assert rc == 0, P.error_string(rc)
    torch.cuda.synchronize()
    return Zref, Z, used, u.value


@pytest.mark.parametrize("fused", [1, 0])
def test_noalloc_normal_matches_allocating_entry_point(lib, fused):
    import torch
    import paper_1607_01404_amd as P
    big = synth.banded_scaled(60000, 30000, seed=31, log_lo=-2.0)
    small = synth.banded_scaled(5003, 2500, seed=32, log_lo=-2.0)
    for A, b in ((big, 8), (small, 3)):
        _say("noalloc normal", A.shape, "b", b, "fused", fused)
        M = P.Matrix.from_scipy(A)
        X = torch.from_numpy(np.random.default_rng(b).standard_normal((A.shape[1], b))).cuda()
        Zref, Z, used_ref, used = _pair(lib, M, X, fused)
        assert used == used_ref == (1 if fused else 0)
        assert torch.equal(Z, Zref)
        # and against SciPy: A^T (A X)
        ref = A.T @ (A @ X.cpu().numpy())
        assert np.allclose(Z.cpu().numpy(), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
        M.close()


def test_noalloc_normal_rejects_oversized_scratch(lib):
    import torch
    import paper_1607_01404_amd as P
    # two-SpMM fallback of a 1.2e6-row matrix at b = 8: 76.8 MB of intermediate > 64 MiB
    A = synth.random_uniform_rows(1_200_000, 1000, 2, seed=5)
    _say("noalloc normal oversized", A.shape)
    M = P.Matrix.from_scipy(A)
    X = torch.zeros((A.shape[1], 8), dtype=torch.float64, device="cuda")
    Z = torch.empty_like(X)
    rc = lib.svds_matrix_normal_noalloc(M.handle, 8, X.data_ptr(), Z.data_ptr(), 0, None, None)
    assert rc == -1
    # within the limit at b = 4 (38.4 MB)
    X4 = torch.from_numpy(np.random.default_rng(1).standard_normal((A.shape[1], 4))).cuda()
    Zref, Z4, _, _ = _pair(lib, M, X4, 0)
    assert torch.equal(Z4, Zref)
    M.close()
