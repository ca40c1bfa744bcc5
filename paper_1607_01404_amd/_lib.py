"""ctypes view of include/svds.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))

LARGEST, SMALLEST = 0, 1
FP64, MIXED = 0, 1
PC_NONE, PC_JACOBI, PC_LEARNED, PC_BLOCKJACOBI = 0, 1, 2, 3
METHOD_HYBRID, METHOD_NORMAL, METHOD_AUGMENTED = 0, 1, 2
STAGE2_GDK, STAGE2_JD = 0, 1
LPC_NPARAMS = 2888
LPC_CACHE_PER_ROW = 192

_STATUS = {0: "ok", 1: "not converged", -1: "invalid argument", -2: "malformed CSR",
           -3: "device out of memory", -4: "HIP runtime error", -5: "numerical breakdown"}


class SvdsError(RuntimeError):
    def __init__(self, code, what=""):
        super().__init__(f"svds status {code} ({_STATUS.get(code, 'unknown')}) {what}".strip())
        self.code = code


class Csr(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64),
                ("rowptr", C.c_void_p), ("colind", C.c_void_p), ("values", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("max_basis_size", C.c_int), ("min_restart_size", C.c_int),
                ("block_size", C.c_int), ("max_prev_retain", C.c_int),
                ("max_matvecs", C.c_int64), ("norm_A", C.c_double), ("stage1_tol", C.c_double),
                ("seed", C.c_uint64), ("precision", C.c_int), ("precond", C.c_int),
                ("force_stage2", C.c_int), ("two_sided_cleanup", C.c_int),
                ("print_level", C.c_int), ("profile", C.c_int), ("autotune", C.c_int),
                ("method", C.c_int), ("stage2_solver", C.c_int), ("jd_max_inner", C.c_int),
                ("jd_inner_tol", C.c_double), ("relative_tol", C.c_int),
                ("max_seconds", C.c_double), ("pc_block", C.c_int), ("pc_degree", C.c_int),
                ("pc_model", C.c_void_p), ("fused_gram", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("nconv", C.c_int), ("stage_exit", C.c_int), ("stage1_status", C.c_int),
                ("pad_", C.c_int), ("matvecs", C.c_int64 * 2), ("iters", C.c_int64 * 2),
                ("restarts", C.c_int64 * 2), ("resets", C.c_int64), ("breakdowns", C.c_int64),
                ("seconds", C.c_double * 2), ("setup_seconds", C.c_double),
                ("norm_A_used", C.c_double), ("spmm_calls", C.c_int64),
                ("spmm_seconds", C.c_double), ("spmm_bytes", C.c_double),
                ("inner_iters", C.c_int64), ("gram_calls", C.c_int64),
                ("gram_seconds", C.c_double), ("gram_bytes", C.c_double),
                ("proj_calls", C.c_int64), ("proj_seconds", C.c_double),
                ("proj_bytes", C.c_double), ("resid_calls", C.c_int64),
                ("resid_seconds", C.c_double), ("resid_bytes", C.c_double),
                ("alg_bytes", C.c_double)]

    def to_dict(self):
        return {"nconv": self.nconv, "stage_exit": self.stage_exit,
                "stage1_status": ["converged", "floor", "budget"][self.stage1_status],
                "matvecs": list(self.matvecs), "iters": list(self.iters),
                "restarts": list(self.restarts), "resets": self.resets,
                "breakdowns": self.breakdowns, "seconds": list(self.seconds),
                "setup_seconds": self.setup_seconds, "norm_A_used": self.norm_A_used,
                "spmm_calls": self.spmm_calls, "spmm_seconds": self.spmm_seconds,
                "spmm_bytes": self.spmm_bytes, "inner_iters": self.inner_iters,
                "gram_calls": self.gram_calls, "gram_seconds": self.gram_seconds,
                "gram_bytes": self.gram_bytes, "proj_calls": self.proj_calls,
                "proj_seconds": self.proj_seconds, "proj_bytes": self.proj_bytes,
                "resid_calls": self.resid_calls, "resid_seconds": self.resid_seconds,
                "resid_bytes": self.resid_bytes, "alg_bytes": self.alg_bytes}


_lib = None


def library_path():
    return os.environ.get("SVDS_LIBRARY", os.path.join(HERE, "libsvds_hip.so"))


def load_library():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run paper_1607_01404_amd.build)")
    lib = C.CDLL(path)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int, C.c_double
    lib.svds_opts_init.argtypes = [C.POINTER(Opts)]
    lib.svds_error_string.argtypes = [i32]
    lib.svds_error_string.restype = C.c_char_p
    lib.svds_matrix_create.argtypes = [C.POINTER(Csr), C.POINTER(vp), vp]
    lib.svds_matrix_destroy.argtypes = [vp]
    lib.svds_matrix_spmm.argtypes = [vp, i32, i32, vp, vp, vp]
    lib.svds_matrix_normal.argtypes = [vp, i32, vp, vp, i32, C.POINTER(i32), vp]
    lib.svds_solve.argtypes = [C.POINTER(Csr), i32, i32, dbl, C.POINTER(Opts), vp, vp, i64, vp,
                               i64, vp, C.POINTER(Stats), vp]
    lib.svds_solve_prepared.argtypes = [vp, i32, i32, dbl, C.POINTER(Opts), vp, vp, i64, vp,
                                        i64, vp, vp, C.c_size_t, C.POINTER(Stats), vp]
    lib.svds_workspace_size.argtypes = [vp, i32, i32, C.POINTER(Opts), C.POINTER(C.c_size_t)]
    lib.svds_stream_release.argtypes = [vp]
    lib.svds_solve_batched.argtypes = [i32, vp, i32, i32, dbl, C.POINTER(Opts), vp, vp, vp, vp,
                                       vp, vp, vp, i32, vp]
    f32 = C.c_float
    lib.svds_lpc_init.argtypes = [vp, C.c_uint64, vp, vp]
    lib.svds_lpc_features.argtypes = [vp, vp, vp]
    lib.svds_lpc_forward.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    lib.svds_lpc_backward.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    lib.svds_lpc_loss.argtypes = [vp, i32, vp, i64, vp, i32, vp, C.POINTER(dbl), vp]
    lib.svds_lpc_apply.argtypes = [vp, vp, i32, i32, vp, i64, vp, i64, vp]
    lib.svds_lpc_adam.argtypes = [i32, vp, vp, vp, vp, i32, f32, f32, f32, f32, vp]
    lib.svds_lpc_train.argtypes = [i32, vp, i32, i32, f32, vp, vp, vp]
    lib.svds_collect_residuals.argtypes = [vp, i32, i32, dbl, C.POINTER(Opts), i32, i32, vp, i64,
                                           C.POINTER(i32), C.POINTER(Stats), vp]
    lib.svds_condest.argtypes = [vp, dbl, C.POINTER(Opts), C.POINTER(dbl), C.POINTER(dbl),
                                 C.POINTER(dbl), vp, vp]
    lib.svds_blockjacobi_apply.argtypes = [vp, i32, i32, vp, i64, vp, i64, vp]
    lib.svds_small_eig.argtypes = [i32, vp, i64, i32, vp, vp, i64, vp]
    lib.svds_small_svd.argtypes = [i32, vp, i64, vp, vp, i64, vp]
    _lib = lib
    return lib


def _check(rc, what=""):
    if rc < 0:
        raise SvdsError(rc, what)
    return rc


def error_string(code):
    return load_library().svds_error_string(code).decode()


def opts_init(**kw):
    o = Opts()
    _check(load_library().svds_opts_init(C.byref(o)))
    for key, val in kw.items():
        if not hasattr(o, key):
            raise TypeError(f"unknown option {key}")
        if key == "pc_model" and hasattr(val, "data_ptr"):
            assert val.is_cuda and val.numel() == LPC_NPARAMS and str(val.dtype) == "torch.float32"
            val = val.data_ptr()
        setattr(o, key, val)
    return o


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _csr(indptr, indices, data, m, n):
    import torch
    assert indptr.is_cuda and indices.is_cuda and data.is_cuda
    assert indptr.dtype == torch.int64 and indices.dtype == torch.int32 and data.dtype == torch.float64
    assert indptr.is_contiguous() and indices.is_contiguous() and data.is_contiguous()
    return Csr(m, n, int(indices.numel()), indptr.data_ptr(), indices.data_ptr(), data.data_ptr())


def to_device(A, device="cuda"):
    """Upload a scipy CSR matrix (int64 indptr, int32 indices, float64 data)."""
    import numpy as np
    import torch
    indptr = torch.from_numpy(np.ascontiguousarray(A.indptr, dtype=np.int64)).to(device)
    indices = torch.from_numpy(np.ascontiguousarray(A.indices, dtype=np.int32)).to(device)
    data = torch.from_numpy(np.ascontiguousarray(A.data, dtype=np.float64)).to(device)
    return indptr, indices, data


class Matrix:
    """A prepared matrix (svds_matrix_create) over device CSR tensors."""

    def __init__(self, indptr, indices, data, m, n, stream=None):
        self._keep = (indptr, indices, data)
        self.m, self.n = int(m), int(n)
        self.csr = _csr(indptr, indices, data, self.m, self.n)
        lib = load_library()
        h = C.c_void_p()
        _check(lib.svds_matrix_create(C.byref(self.csr), C.byref(h), _stream(stream)), "create")
        self.handle = h

    @classmethod
    def from_scipy(cls, A, device="cuda", stream=None):
        ip, ix, dv = to_device(A, device)
        return cls(ip, ix, dv, A.shape[0], A.shape[1], stream)

    def close(self):
        if getattr(self, "handle", None):
            load_library().svds_matrix_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def spmm(self, X, trans=False, stream=None):
        """Y = A X (trans=False, X: n x b) or A^T X (X: m x b); row-major blocks."""
        import torch
        b = X.shape[1]
        rows = self.n if trans else self.m
        assert X.shape[0] == (self.m if trans else self.n) and X.is_contiguous()
        Y = torch.empty((rows, b), dtype=torch.float64, device=X.device)
        _check(load_library().svds_matrix_spmm(self.handle, int(trans), b, _ptr(X), _ptr(Y),
                                               _stream(stream)), "spmm")
        return Y

    def normal(self, X, fused=True, stream=None):
        """Z = A_w^T A_w X (svds_matrix_normal); A_w = A if m >= n else A^T.
        Returns (Z, used) with used = 1 when the one-pass product ran."""
        import torch
        p = min(self.m, self.n)
        assert X.shape[0] == p and X.is_contiguous() and X.dtype == torch.float64
        Z = torch.empty_like(X)
        used = C.c_int(-1)
        _check(load_library().svds_matrix_normal(self.handle, X.shape[1], _ptr(X), _ptr(Z),
                                                 int(bool(fused)), C.byref(used),
                                                 _stream(stream)), "normal")
        return Z, used.value

    def workspace_size(self, k, target="largest", **opts):
        """Bytes of caller workspace a solve with these arguments needs
        (svds_workspace_size)."""
        tgt = _target(target)
        o = opts_init(**opts)
        nb = C.c_size_t(0)
        _check(load_library().svds_workspace_size(self.handle, k, tgt, C.byref(o), C.byref(nb)),
               "workspace_size")
        return nb.value

    def solve(self, k, target="largest", tol=1e-10, stream=None, workspace=None, **opts):
        """svds_solve_prepared; workspace: None or a device tensor whose bytes
        the solver's arrays are carved from."""
        wp = _ptr(workspace) if workspace is not None else None
        wb = workspace.numel() * workspace.element_size() if workspace is not None else 0

        def call(k_, tgt, tol_, o, sig, U, ldu, V, ldv, rn, st, strm):
            return load_library().svds_solve_prepared(self.handle, k_, tgt, tol_, o, sig, U, ldu,
                                                      V, ldv, rn, wp, wb, st, strm)
        return _solve(call, self.m, self.n, k, target, tol, stream, opts)


def _target(target):
    return {"largest": LARGEST, "smallest": SMALLEST}[target] if isinstance(target, str) else target


def stream_release(stream=None):
    """Free the device blocks the library keeps for `stream` (svds_stream_release)."""
    _check(load_library().svds_stream_release(_stream(stream)), "stream_release")


def _solve(call, m, n, k, target, tol, stream, opts):
    import torch
    tgt = {"largest": LARGEST, "smallest": SMALLEST}[target] if isinstance(target, str) else target
    o = opts_init(**opts)
    dev = torch.device("cuda", torch.cuda.current_device())
    sigma = torch.empty(k, dtype=torch.float64, device=dev)
    rnorm = torch.empty(k, dtype=torch.float64, device=dev)
    # column-major outputs: allocate (k, m) row-major = (m, k) column-major
    Ut = torch.empty((k, m), dtype=torch.float64, device=dev)
    Vt = torch.empty((k, n), dtype=torch.float64, device=dev)
    st = Stats()
    rc = call(k, tgt, float(tol), C.byref(o), _ptr(sigma), _ptr(Ut), m, _ptr(Vt), n, _ptr(rnorm),
              C.byref(st), _stream(stream))
    _check(rc, "solve")
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    stats = st.to_dict()
    stats["status"] = rc
    stats["converged"] = rc == 0
    return sigma, Ut.t(), Vt.t(), rnorm, stats


def solve(indptr, indices, data, m, n, k, target="largest", tol=1e-10, stream=None, **opts):
    """svds_solve on device CSR tensors.  Returns (sigma, U, V, rnorm, stats)
    with U (m x k) and V (n x k) as column-major views."""
    csr = _csr(indptr, indices, data, int(m), int(n))
    return _solve(lambda *a: load_library().svds_solve(C.byref(csr), *a), int(m), int(n), k,
                  target, tol, stream, opts)


def svds(A, k, target="largest", tol=1e-10, device="cuda", **opts):
    """Convenience: upload a scipy CSR matrix and solve."""
    ip, ix, dv = to_device(A, device)
    return solve(ip, ix, dv, A.shape[0], A.shape[1], k, target, tol, **opts)


def solve_batched(problems, k, target="largest", tol=1e-10, nworkers=0, stream=None, **opts):
    """svds_solve_batched over a list of device CSR tuples (indptr, indices,
    data, m, n).  Returns (status, list of (sigma, U, V, rnorm, stats))."""
    import torch
    n = len(problems)
    tgt = {"largest": LARGEST, "smallest": SMALLEST}[target] if isinstance(target, str) else target
    o = opts_init(**opts)
    dev = torch.device("cuda", torch.cuda.current_device())
    csrs = (Csr * n)()
    outs = []
    for i, (ip, ix, dv, m, nn) in enumerate(problems):
        csrs[i] = _csr(ip, ix, dv, int(m), int(nn))
        outs.append((torch.empty(k, dtype=torch.float64, device=dev),
                     torch.empty((k, int(m)), dtype=torch.float64, device=dev),
                     torch.empty((k, int(nn)), dtype=torch.float64, device=dev),
                     torch.empty(k, dtype=torch.float64, device=dev)))
    P = C.c_void_p * n
    sig = P(*[o_[0].data_ptr() for o_ in outs])
    Up = P(*[o_[1].data_ptr() for o_ in outs])
    Vp = P(*[o_[2].data_ptr() for o_ in outs])
    rp = P(*[o_[3].data_ptr() for o_ in outs])
    ldu = (C.c_int64 * n)(*[int(p[3]) for p in problems])
    ldv = (C.c_int64 * n)(*[int(p[4]) for p in problems])
    st = (Stats * n)()
    rc = load_library().svds_solve_batched(n, C.cast(csrs, C.c_void_p), k, tgt, float(tol),
                                           C.byref(o), C.cast(sig, C.c_void_p),
                                           C.cast(Up, C.c_void_p), C.cast(ldu, C.c_void_p),
                                           C.cast(Vp, C.c_void_p), C.cast(ldv, C.c_void_p),
                                           C.cast(rp, C.c_void_p), C.cast(st, C.c_void_p),
                                           int(nworkers), _stream(stream))
    _check(rc, "solve_batched")
    torch.cuda.synchronize()
    res = []
    for i, o_ in enumerate(outs):
        d = st[i].to_dict()
        d["converged"] = d["nconv"] >= k
        res.append((o_[0], o_[1].t(), o_[2].t(), o_[3], d))
    return rc, res


def small_eig(H, descending=False, stream=None):
    """Device Jacobi eigensolver of a symmetric g x g matrix: eigenvalues in
    ascending (or descending) order and eigenvectors as columns."""
    import torch
    g = H.shape[0]
    Hcm = H.t().contiguous()  # column-major storage of H
    theta = torch.empty(g, dtype=torch.float64, device=H.device)
    Yt = torch.empty((g, g), dtype=torch.float64, device=H.device)
    _check(load_library().svds_small_eig(g, _ptr(Hcm), g, int(descending), _ptr(theta), _ptr(Yt),
                                         g, _stream(stream)), "small_eig")
    torch.cuda.synchronize()
    del Hcm
    return theta, Yt.t()


def small_svd(R, stream=None):
    """Device one-sided Jacobi SVD of a g x g matrix: ascending singular values
    and right singular vectors as columns."""
    import torch
    g = R.shape[0]
    Rcm = R.t().contiguous()
    s = torch.empty(g, dtype=torch.float64, device=R.device)
    Yt = torch.empty((g, g), dtype=torch.float64, device=R.device)
    _check(load_library().svds_small_svd(g, _ptr(Rcm), g, _ptr(s), _ptr(Yt), g, _stream(stream)),
           "small_svd")
    torch.cuda.synchronize()
    del Rcm
    return s, Yt.t()


# ---------------------------------------------------------------------------
# learned preconditioner
# ---------------------------------------------------------------------------
class LpcSet(C.Structure):
    _fields_ = [("A", C.c_void_p), ("npairs", C.c_int), ("R", C.c_void_p), ("ldr", C.c_int64)]


def _dev():
    import torch
    return torch.device("cuda", torch.cuda.current_device())


def lpc_init(seed=0, out_bias=None, stream=None):
    """Initial parameters (device FP32 tensor of LPC_NPARAMS)."""
    import torch
    p = torch.empty(LPC_NPARAMS, dtype=torch.float32, device=_dev())
    ob = None
    if out_bias is not None:
        ob = (C.c_float * 8)(*[float(x) for x in out_bias])
    _check(load_library().svds_lpc_init(_ptr(p), int(seed), ob, _stream(stream)), "lpc_init")
    return p


def _n_c(M):
    return min(M.m, M.n)


def lpc_features(M, stream=None):
    import torch
    f = torch.empty((_n_c(M), 8), dtype=torch.float32, device=_dev())
    _check(load_library().svds_lpc_features(M.handle, _ptr(f), _stream(stream)), "lpc_features")
    return f


def lpc_forward(M, params, feat, degree, stream=None):
    """Returns (coef N x 16, cache)."""
    import torch
    N = _n_c(M)
    coef = torch.empty((N, 16), dtype=torch.float32, device=_dev())
    cache = torch.empty(N * LPC_CACHE_PER_ROW, dtype=torch.float32, device=_dev())
    _check(load_library().svds_lpc_forward(M.handle, _ptr(params), _ptr(feat), int(degree),
                                           _ptr(coef), _ptr(cache), _stream(stream)), "lpc_forward")
    return coef, cache


def lpc_backward(M, params, cache, degree, dcoef, stream=None):
    import torch
    g = torch.empty(LPC_NPARAMS, dtype=torch.float32, device=_dev())
    _check(load_library().svds_lpc_backward(M.handle, _ptr(params), _ptr(cache), int(degree),
                                            _ptr(dcoef), _ptr(g), _stream(stream)), "lpc_backward")
    return g


def _colmajor(R):
    """(N, P) tensor -> contiguous (P, N) storage = column-major N x P."""
    return R.t().contiguous()


def lpc_loss(M, R, coef, degree, stream=None):
    """Mean pair loss of the pairs built from residuals R (N x P) and
    dloss/dcoef (N x 16)."""
    import torch
    Rc = _colmajor(R)
    N, P = R.shape
    dc = torch.empty((N, 16), dtype=torch.float32, device=_dev())
    loss = C.c_double()
    _check(load_library().svds_lpc_loss(M.handle, P, _ptr(Rc), N, _ptr(coef), int(degree),
                                        _ptr(dc), C.byref(loss), _stream(stream)), "lpc_loss")
    return loss.value, dc


def lpc_apply(M, coef, degree, R, stream=None):
    """T = K(R) for R (N x nb), nb <= 8."""
    Rc = _colmajor(R)
    N, nb = R.shape
    T = Rc.clone()
    _check(load_library().svds_lpc_apply(M.handle, _ptr(coef), int(degree), nb, _ptr(Rc), N,
                                         _ptr(T), N, _stream(stream)), "lpc_apply")
    return T.t()


def lpc_adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(load_library().svds_lpc_adam(params.numel(), _ptr(params), _ptr(grad), _ptr(m), _ptr(v),
                                        int(step), lr, beta1, beta2, eps, _stream(stream)),
           "lpc_adam")


def lpc_train(sets, degree, steps, lr, params, stream=None):
    """sets: list of (Matrix, R (N x P device FP64)).  Trains params in place;
    returns the loss of every step (numpy)."""
    import numpy as np
    keep = []
    arr = (LpcSet * len(sets))()
    for i, (M, R) in enumerate(sets):
        Rc = _colmajor(R) if R.shape[1] > 0 else None
        keep.append(Rc)
        arr[i] = LpcSet(M.handle.value if hasattr(M.handle, "value") else M.handle, int(R.shape[1]),
                        Rc.data_ptr() if Rc is not None else None, int(R.shape[0]))
    hist = np.zeros(max(int(steps), 1), dtype=np.float64)
    _check(load_library().svds_lpc_train(len(sets), C.cast(arr, C.c_void_p), int(degree), int(steps),
                                         lr, _ptr(params), hist.ctypes.data_as(C.c_void_p),
                                         _stream(stream)), "lpc_train")
    return hist[: int(steps)]


def collect_residuals(M, k, target="smallest", tol=1e-10, every=1, max_pairs=64, stream=None,
                      **opts):
    """Solve with M, keeping stage-1 residuals; returns (R (N x count), stats)."""
    import torch
    N = _n_c(M)
    tgt = {"largest": LARGEST, "smallest": SMALLEST}[target] if isinstance(target, str) else target
    o = opts_init(**opts)
    Rc = torch.zeros((max(int(max_pairs), 1), N), dtype=torch.float64, device=_dev())
    cnt = C.c_int()
    st = Stats()
    rc = load_library().svds_collect_residuals(M.handle, int(k), tgt, float(tol), C.byref(o),
                                               int(every), int(max_pairs), _ptr(Rc), N,
                                               C.byref(cnt), C.byref(st), _stream(stream))
    _check(rc, "collect_residuals")
    d = st.to_dict()
    d["status"] = rc
    d["converged"] = rc == 0
    return Rc[: cnt.value].t(), d


def condest(M, rtol=0.1, stream=None, **opts):
    """svds_condest on a prepared Matrix: (kappa, sigma_max, sigma_min,
    (stats_largest, stats_smallest))."""
    o = opts_init(**opts)
    smax, smin, kap = C.c_double(), C.c_double(), C.c_double()
    st = (Stats * 2)()
    rc = load_library().svds_condest(M.handle, float(rtol), C.byref(o), C.byref(smax),
                                     C.byref(smin), C.byref(kap), C.cast(st, C.c_void_p),
                                     _stream(stream))
    _check(rc, "condest")
    out = []
    for i in range(2):
        d = st[i].to_dict()
        d["status"] = rc
        out.append(d)
    return kap.value, smax.value, smin.value, tuple(out)


def blockjacobi_apply(M, nb, R, stream=None):
    """T = K R with the block-Jacobi preconditioner (blocks of nb columns)."""
    Rc = _colmajor(R)
    N, b = R.shape
    T = Rc.clone()
    _check(load_library().svds_blockjacobi_apply(M.handle, int(nb), b, _ptr(Rc), N, _ptr(T), N,
                                                 _stream(stream)), "blockjacobi_apply")
    return T.t()
