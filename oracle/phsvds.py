"""Plain FP64 reference implementation of the PHSVDS method (Algorithm 1 of
Wu, Romero and Stathopoulos, "PRIMME_SVDS", Section 3.1, with the solver
changes of Section 3.2).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library.

Stage 1 runs a block GD+k eigensolver on the normal equations C = A^T A (the
smaller Gram matrix, Section 2.1) with soft locking, the per-pair convergence
test of Algorithm 1 (stage 1), the restart error reset of Section 3.2 and a
final Rayleigh-Ritz on the returned vectors.  Stage 2, when needed, runs the
same eigensolver with hard locking on the augmented matrix B = [0 A^T; A 0]
(eq. B_Augmented), seeded with [v; u]/sqrt(2) (eq. B_Initguess); for the
smallest singular values it uses the simplified refined projection with the
stage-1 lower bounds as shifts (Section 3.2).  Acceptance is always the SVD
residual eq. (res).

Every small dense step is a LAPACK call through numpy (eigh, svd, qr,
cholesky); sparse products are scipy CSR products.  The random vectors the
method draws come from a counter-based SplitMix64 stream (Steele, Lea and
Flood, 2014), so that the GPU path can draw the very same numbers from its
own implementation of that published generator.

Readings of points the paper leaves open (all listed with reasons in the
design notes of the repository):
  * GD+k keeps p previous-iteration Ritz coefficient vectors of the block at
    restart (p defaults to the block size); they are orthonormalised in the
    small space against the retained Ritz vectors.
  * Stage 1 starts from b counter-based random vectors and fills a block
    Krylov basis up to the restart size.
  * The block takes the first b unconverged pairs in target order among the
    first k+b; with soft locking the restart keeps at least (#converged + b)
    Ritz vectors.
  * Stage 2 locks a converged prefix of the block at once and forces a
    restart for both targets; one active shift (the first unlocked bound).
  * The stage-1 floor is eps*||C|| as printed.  The attainable accuracy can
    be some hundred times higher, so a wanted pair whose residual did not halve
    over three restart cycles while below 1e4*eps*||C|| counts as practically
    converged (it leaves the block); when every wanted pair is converged or
    practically converged, one reset confirms it and stage 1 hands over to
    stage 2.
  * ||A|| comes from a 30-step Krylov (Lanczos with full
    reorthogonalisation) estimate on C unless given, and grows to the largest
    Ritz value seen.
  * After either stage a two-sided Rayleigh-Ritz (SVD of U^T A V) restores
    orthonormality of U and V; the reported residual is eq. (res) after it.
"""
from __future__ import annotations

import math
import time

import numpy as np
import scipy.sparse as sp

EPS = float(np.finfo(np.float64).eps)  # machine precision 2.2e-16 (Section 4)

# ---------------------------------------------------------------------------
# Counter-based random numbers (SplitMix64 finaliser applied to seed + k*gamma)
# ---------------------------------------------------------------------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

STREAM_INIT = 0       # stage-1 initial block
STREAM_NORM = 1       # start vector of the norm estimate
STREAM_BREAK = 2      # first stream of breakdown replacement vectors


def counter_uniform(seed, stream, nrows, ncols, col0=0):
    """Uniform numbers in [-0.5, 0.5) for entry (i, c) of a random block:
    counter = stream*2^40 + (col0+c)*2^32 + i, z = seed + (counter+1)*gamma
    (mod 2^64), then the SplitMix64 mixing function, then the top 53 bits."""
    with np.errstate(over="ignore"):
        i = np.arange(nrows, dtype=np.uint64)[:, None]
        c = (np.arange(ncols, dtype=np.uint64) + np.uint64(col0))[None, :]
        ctr = (np.uint64(stream) << np.uint64(40)) + (c << np.uint64(32)) + i
        z = np.uint64(seed) + (ctr + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) - 0.5


# ---------------------------------------------------------------------------
# Operators C and B with matrix-vector counting (Section 2.1, Table 3)
# ---------------------------------------------------------------------------
class Operators:
    """Products with A and A^T of a tall (m >= n) CSR matrix.  ``mv`` counts
    one for each column multiplied by A or by A^T, as the paper's tables do."""

    def __init__(self, A):
        self.A = sp.csr_matrix(A)
        self.At = self.A.T.tocsr()
        self.m, self.n = self.A.shape
        self.mv = 0

    def A_mul(self, X):
        self.mv += X.shape[1]
        return np.asarray(self.A @ X)

    def At_mul(self, X):
        self.mv += X.shape[1]
        return np.asarray(self.At @ X)

    def C(self, X):
        """C X = A^T (A X) on dimension n (Algorithm 1, stage 1)."""
        return self.At_mul(self.A_mul(X))

    def B(self, X):
        """B [x_v; x_u] = [A^T x_u; A x_v] on dimension n + m (eq. B_Augmented)."""
        n = self.n
        return np.vstack([self.At_mul(X[n:]), self.A_mul(X[:n])])


def jacobi_diag(A):
    """diag(A^T A): squared column norms (point-Jacobi preconditioner for C)."""
    A = sp.csr_matrix(A)
    d = np.asarray(A.multiply(A).sum(axis=0)).ravel()
    return d


def block_jacobi(A, nb):
    """Block-Jacobi preconditioner for C = A^T A (the generic preconditioner of
    Section 4's preconditioned comparison): the inverses of the diagonal
    blocks C_j of contiguous column ranges [j nb, (j+1) nb), applied block by
    block.  Each block is first scaled to unit diagonal (zero diagonals ->
    1), factored by Cholesky with a pivot below 1e-12 replaced by 1 and its
    column decoupled, and inverted through the factor.  Returns K(R)."""
    A = sp.csc_matrix(A, dtype=np.float64)
    N = A.shape[1]
    invs = []
    for c0 in range(0, N, nb):
        c1 = min(N, c0 + nb)
        Cj = (A[:, c0:c1].T @ A[:, c0:c1]).toarray()
        d = np.diag(Cj).copy()
        d[d <= 0] = 1.0
        sc = 1.0 / np.sqrt(d)
        Ch = Cj * sc[:, None] * sc[None, :]
        nbj = c1 - c0
        for i in range(nbj):
            if Cj[i, i] <= 0:
                Ch[i, :] = 0.0
                Ch[:, i] = 0.0
                Ch[i, i] = 1.0
        L = np.zeros((nbj, nbj))
        for k in range(nbj):
            p = Ch[k, k] - L[k, :k] @ L[k, :k]
            if p <= 1e-12:
                L[k, k] = 1.0
                continue
            L[k, k] = math.sqrt(p)
            for i in range(k + 1, nbj):
                L[i, k] = (Ch[i, k] - L[i, :k] @ L[k, :k]) / L[k, k]
        Li = np.linalg.inv(L)
        invs.append((c0, c1, sc[:, None] * (Li.T @ Li) * sc[None, :]))

    def K(R):
        R = np.asarray(R, dtype=np.float64)
        T = np.empty_like(R)
        for c0, c1, Kj in invs:
            T[c0:c1] = Kj @ R[c0:c1]
        return T

    return K


def exact_inverse(A):
    """K(R) = C^-1 R for the smaller Gram matrix C of A (A^T A when m >= n,
    else A A^T) by a sparse LU factorisation of C (SuperLU through SciPy): a
    preconditioner of the correction step (the hook of Section 3.4) for
    reference runs on operators where point or block Jacobi needs too many
    iterations.  With K = C^-1 the correction K r = x - theta C^-1 x is an
    inverse-iteration step, so GD+k reaches the smallest pairs in few
    iterations; the triplets it converges to are those of A whatever K is."""
    import scipy.sparse.linalg as spl
    A = sp.csr_matrix(A, dtype=np.float64)
    m, n = A.shape
    Aw = A.T.tocsr() if m < n else A
    lu = spl.splu((Aw.T @ Aw).tocsc())
    return lambda R: lu.solve(np.asarray(R, dtype=np.float64))


# ---------------------------------------------------------------------------
# Block orthogonalisation: CGS twice + Cholesky QR twice (Sections 3.2, 3.3)
# ---------------------------------------------------------------------------
BREAK_RATIO = 1e-7   # Cholesky pivot / column norm below this = dependent
COLLAPSE = 1e-12     # column norm after projection / before below this = in span


class _Breakdown(Exception):
    def __init__(self, cols):
        self.cols = cols


def _cholqr_once(T):
    G = T.T @ T
    G = 0.5 * (G + G.T)
    d = np.sqrt(np.maximum(np.diag(G), 0.0))
    b = T.shape[1]
    R = np.zeros((b, b))
    bad = []
    # Cholesky one column at a time so that a dependent column is named
    for j in range(b):
        s = G[j, j] - R[:j, j] @ R[:j, j]
        if not (s > (BREAK_RATIO * d[j]) ** 2) or d[j] == 0.0:
            bad.append(j)
            continue
        R[j, j] = math.sqrt(s)
        for i in range(j + 1, b):
            R[j, i] = (G[j, i] - R[:j, j] @ R[:j, i]) / R[j, j]
    if bad:
        raise _Breakdown(bad)
    return np.linalg.solve(R.T, T.T).T, R


def ortho_block(T, bases, rand_next=None):
    """Orthonormalise the columns of T against the orthonormal ``bases`` and
    among themselves.  Classical Gram-Schmidt is applied twice against the
    bases, then Cholesky QR twice on the block.  A column that collapses (it
    lies in the span already) or is dependent within the block is replaced
    by fresh counter-based random numbers (``rand_next(ncols)`` returns an
    N x ncols block) and the block is redone.  Returns (Q, Rtot, C) with
    T_in ~= [bases] C + Q Rtot when no replacement happened."""
    T = np.array(T, dtype=np.float64, copy=True)
    N, b = T.shape
    for attempt in range(4):
        norm0 = np.linalg.norm(T, axis=0)
        Ctot = []
        Bcat = np.hstack(bases) if bases and sum(Q.shape[1] for Q in bases) else None
        if Bcat is not None:
            C1 = Bcat.T @ T
            T = T - Bcat @ C1
            C2 = Bcat.T @ T
            T = T - Bcat @ C2
            Ctot = C1 + C2
        norm1 = np.linalg.norm(T, axis=0)
        collapsed = [j for j in range(b) if not (norm1[j] > COLLAPSE * norm0[j]) or norm0[j] == 0.0]
        try:
            if collapsed:
                raise _Breakdown(collapsed)
            T1, R1 = _cholqr_once(T)
            T2, R2 = _cholqr_once(T1)
            return T2, R2 @ R1, Ctot
        except _Breakdown as e:
            if rand_next is None:
                raise RuntimeError("orthogonalisation breakdown")
            fresh = rand_next(len(e.cols))
            for i, j in enumerate(e.cols):
                T[:, j] = fresh[:, i]
    raise RuntimeError("repeated orthogonalisation breakdown")


# ---------------------------------------------------------------------------
# Norm estimate of A (reading of the unspecified ||A||)
# ---------------------------------------------------------------------------
def estimate_norm(ops, seed, steps=30):
    """sqrt of the largest Ritz value of C from a ``steps``-dimensional
    Krylov space (Lanczos with full reorthogonalisation) started from a
    counter-based random vector."""
    n = ops.n
    s = max(1, min(steps, n))
    x = counter_uniform(seed, STREAM_NORM, n, 1)
    V = x / np.linalg.norm(x)
    W = ops.C(V)
    for _ in range(s - 1):
        w = W[:, -1:]
        c1 = V.T @ w
        w = w - V @ c1
        c2 = V.T @ w
        w = w - V @ c2
        nw = np.linalg.norm(w)
        if not nw > 1e-12 * np.linalg.norm(W[:, -1]):
            break  # invariant subspace found
        v = w / nw
        V = np.hstack([V, v])
        W = np.hstack([W, ops.C(v)])
    H = V.T @ W
    H = 0.5 * (H + H.T)
    lam = np.linalg.eigvalsh(H)
    return math.sqrt(max(lam[-1], 0.0))


# ---------------------------------------------------------------------------
# The GD+k search space
# ---------------------------------------------------------------------------
PREV_DROP = 1e-10   # +k vector dropped when its new direction is smaller
STALL_RESTARTS = 3  # restart cycles without halving the residual = stalled
FLOOR_GATE = 1e4    # stalled below FLOOR_GATE*eps*||Op|| = at the attainable floor


class SearchSpace:
    """V (orthonormal), W = Op V, H = V^T W and the locked vectors."""

    def __init__(self, op, N, ortho_fn):
        self.op = op
        self.N = N
        self.V = np.zeros((N, 0))
        self.W = np.zeros((N, 0))
        self.H = np.zeros((0, 0))
        self.X = np.zeros((N, 0))       # locked vectors (stage 2)
        self.lock_vals = []
        self.ortho_fn = ortho_fn

    @property
    def g(self):
        return self.V.shape[1]

    def append(self, T):
        """Append an orthonormal block T; computes Op T and the new column
        block of H = V^T Op V."""
        Wt = self.op(T)
        Hn = np.vstack([self.V.T @ Wt, T.T @ Wt])
        g = self.g
        b = T.shape[1]
        H = np.zeros((g + b, g + b))
        H[:g, :g] = self.H
        H[:, g:] = Hn
        H[g:, :g] = Hn[:g].T
        H[g:, g:] = 0.5 * (Hn[g:] + Hn[g:].T)
        self.H = H
        self.V = np.hstack([self.V, T])
        self.W = np.hstack([self.W, Wt])
        return Wt

    def restart(self, Yr):
        """V <- V Yr, W <- W Yr, H <- Yr^T H Yr (Yr orthonormal columns)."""
        self.V = self.V @ Yr
        self.W = self.W @ Yr
        H = Yr.T @ self.H @ Yr
        self.H = 0.5 * (H + H.T)

    def reset(self):
        """Re-orthonormalise V (against the locked vectors, then itself) and
        recompute W = Op V and H directly (Section 3.2, restart error)."""
        V = self.V
        if self.X.shape[1]:
            V = V - self.X @ (self.X.T @ V)
            V = V - self.X @ (self.X.T @ V)
        V, _ = np.linalg.qr(V)
        self.V = V
        self.W = self.op(V)
        H = V.T @ self.W
        self.H = 0.5 * (H + H.T)


def _small_orth_append(Ykeep, cand):
    """Orthonormalise candidate columns against Ykeep (and each other) in the
    small space by modified Gram-Schmidt applied twice; drop columns whose
    new direction has norm below PREV_DROP."""
    cols = [Ykeep[:, j] for j in range(Ykeep.shape[1])]
    out = []
    for j in range(cand.shape[1]):
        y = cand[:, j].copy()
        for _ in range(2):
            for q in cols:
                y -= (q @ y) * q
        ny = np.linalg.norm(y)
        if ny > PREV_DROP:
            y /= ny
            cols.append(y)
            out.append(y)
    if out:
        return np.column_stack([Ykeep] + [o[:, None] for o in out])
    return Ykeep


def _pad(Y, g):
    if Y is None or Y.shape[1] == 0:
        return None
    P = np.zeros((g, Y.shape[1]))
    P[: Y.shape[0]] = Y
    return P


class _TimedBudget(int):
    """A matrix-vector budget that also runs out after ``seconds`` of wall
    time (used to take bounded timing samples of the reference)."""

    def __new__(cls, mv, seconds):
        obj = int.__new__(cls, mv)
        obj.deadline = time.perf_counter() + seconds
        return obj

    def __le__(self, other):
        return time.perf_counter() > self.deadline or int(self) <= other


# ---------------------------------------------------------------------------
# Parameters
# ---------------------------------------------------------------------------
def default_params(k, target, max_basis=None, min_restart=None, block=None, prev_retain=None):
    """Defaults of Section 3.4: basis 15 / restart 6 when seeking fewer than 10
    largest, otherwise 35 / 14; block size 1; +k retention = block size."""
    if max_basis is None or min_restart is None:
        small = target == "largest" and k < 10
        g0, r0 = (15, 6) if small else (35, 14)
        max_basis = g0 if max_basis is None else max_basis
        min_restart = r0 if min_restart is None else min_restart
    b = 1 if block is None else block
    p = b if prev_retain is None else prev_retain
    return max_basis, min_restart, b, p


# ---------------------------------------------------------------------------
# Stage 1: GD+k on C with soft locking (Algorithm 1, first stage)
# ---------------------------------------------------------------------------
def _stage1(ops, k, target, tol, normA, g, r, b, p, seed, precond, budget, stats, rand_state,
            trace=None, capture=None, relative=False):
    n = ops.n
    g = min(g, n)
    r = min(r, max(1, g - b - p))
    normC = normA * normA
    if callable(precond):
        K = precond
    elif precond is not None:
        d = precond.copy()
        d[d <= 0] = 1.0
        K = lambda R: R / d[:, None]
    else:
        K = lambda R: R

    def rand_next(c):
        s = STREAM_BREAK + rand_state["count"]
        rand_state["count"] += 1
        return counter_uniform(seed, s, n, c)

    S = SearchSpace(ops.C, n, None)
    # initial basis: b random vectors and a block Krylov fill up to
    # max(r, k + b) columns (at most g - b)
    fill = min(max(r, k + b), g - b)
    T, _, _ = ortho_block(counter_uniform(seed, STREAM_INIT, n, b), [], rand_next)
    while True:
        Wt = S.append(T)
        if S.g >= fill or S.g + b > g:
            break
        T, _, _ = ortho_block(Wt, [S.V], rand_next)

    descending = target == "largest"
    y_prev = None
    restarts = 0
    since_reset = 0
    resets = 0
    floor_resets = 0
    ncmax = k + b
    best = np.full(ncmax, np.inf)   # best residual per target position
    stall = np.zeros(ncmax, dtype=int)
    iters = 0
    status = "budget"
    while True:
        lam, Y = np.linalg.eigh(S.H)
        if descending:
            lam, Y = lam[::-1], Y[:, ::-1]
        normC = max(normC, float(np.max(np.abs(lam))))
        nc = min(S.g, ncmax)
        X = S.V @ Y[:, :nc]
        R = S.W @ Y[:, :nc] - X * lam[:nc]
        rn = np.linalg.norm(R, axis=0)
        # Algorithm 1 stage-1 test: ||r^C|| <= max(sqrt(|lam| ||C||) delta, eps ||C||)
        if relative:
            # residual below tol times the eigenvalue (the low-accuracy stopping
            # rule of Section 4.4): ||r^C|| <= tol |lambda|, i.e. the SVD
            # residual below tol sigma
            thr = np.maximum(tol * np.abs(lam[:nc]), EPS * normC)
        else:
            thr = np.maximum(np.sqrt(np.abs(lam[:nc]) * normC) * tol, EPS * normC)
        conv = rn <= thr
        # practically converged: stuck near the attainable floor
        pc = (~conv) & (stall[:nc] >= STALL_RESTARTS) & (rn <= FLOOR_GATE * EPS * normC)
        done = conv | pc
        if trace is not None:
            trace(1, iters, S.g, lam[:nc], rn, conv)
        kk = min(k, nc)
        if kk == k and np.all(done[:k]):
            if np.any(pc[:k]) and floor_resets < 1:
                # confirm the floor once with accurate W = C V (Section 3.2 reset)
                S.reset()
                resets += 1
                floor_resets += 1
                since_reset = 0
                y_prev = None
                best[:] = np.inf
                stall[:] = 0
                continue
            status = "floor" if np.any(pc[:k]) else "converged"
            break
        if ops.mv >= budget:
            status = "budget"
            break
        block = [j for j in range(nc) if not done[j]][:b]
        # restart-error reset (Section 3.2)
        if block and since_reset > 0 and min(rn[block]) < math.sqrt(since_reset) * normC * EPS:
            S.reset()
            resets += 1
            since_reset = 0
            y_prev = None
            continue
        Yb = Y[:, block]
        if S.g + (len(block) if block else b) > g:
            # per-position stagnation bookkeeping, once per restart cycle
            improved = rn < 0.5 * best[:nc]
            best[:nc] = np.where(improved, rn, best[:nc])
            stall[:nc] = np.where(improved, 0, stall[:nc] + 1)
            nconv = int(np.sum(done))
            r_eff = min(max(r, nconv + b), g - b)
            Yr = Y[:, :r_eff]
            prev = _pad(y_prev, S.g)
            if prev is not None and p > 0:
                room = max(0, g - b - r_eff)
                Yr = _small_orth_append(Yr, prev[:, : min(p, room)]) if room else Yr
            S.restart(Yr)
            Yb = Yr.T @ Yb
            restarts += 1
            since_reset += 1
        if (capture is not None and block and iters % capture["every"] == 0
                and len(capture["idx"]) < capture["max"]):
            # training pair for a learned preconditioner: residual and Ritz
            # vector of the block's first target
            capture["R"].append(R[:, block[0]].copy())
            capture["X"].append(X[:, block[0]].copy())
            capture["idx"].append(block[0])
        T = K(R[:, block]) if block else rand_next(b)
        T, _, _ = ortho_block(T, [S.V], rand_next)
        y_prev = Yb
        S.append(T)
        iters += 1

    stats["iters"][0] = iters
    stats["restarts"][0] = restarts
    stats["resets"] += resets
    stats["stage1_status"] = status
    lam, Y = np.linalg.eigh(S.H)
    if descending:
        lam, Y = lam[::-1], Y[:, ::-1]
    kk = min(k, S.g)
    Xk = S.V @ Y[:, :kk]
    return Xk, normC, status


def _final_rr(ops, Xk, target):
    """Rayleigh-Ritz on the returned basis through A X (Algorithm 1, steps
    4-5): G = (A X)^T (A X) = X^T C X, sigma = |lambda|^(1/2), v = X z,
    u = A v / sigma.  Returns sigma, U, V and the SVD residual pieces."""
    Y = ops.A_mul(Xk)
    G = Y.T @ Y
    G = 0.5 * (G + G.T)
    lam, Z = np.linalg.eigh(G)
    if target == "largest":
        lam, Z = lam[::-1], Z[:, ::-1]
    V = Xk @ Z
    Y = Y @ Z
    sig = np.sqrt(np.abs(lam))
    U = np.where(sig > 0, Y / np.where(sig > 0, sig, 1.0), 0.0)
    AtU = ops.At_mul(U)
    r_left = np.linalg.norm(Y - U * sig, axis=0)      # A v - sigma u
    r_right = np.linalg.norm(AtU - V * sig, axis=0)   # A^T u - sigma v
    rn = np.sqrt(r_left ** 2 + r_right ** 2)
    rn[sig == 0] = np.inf
    return sig, U, V, rn


# ---------------------------------------------------------------------------
# Stage 2: GD+k on B with hard locking (Algorithm 1, second stage)
# ---------------------------------------------------------------------------
def _halves_residual(x, w, theta, n):
    """eq. (res) for the normalised halves of an eigenvector approximation x of
    B with W-part w = B x and sigma = |theta| (Algorithm 1, second stage)."""
    xv, xu = x[:n], x[n:]
    a, c = np.linalg.norm(xv), np.linalg.norm(xu)
    if a == 0.0 or c == 0.0:
        return np.inf
    s = abs(theta)
    v, u = xv / a, xu / c
    Av = w[n:] / a     # (B x)_u = A x_v
    Atu = w[:n] / c    # (B x)_v = A^T x_u
    return math.sqrt(np.linalg.norm(Av - s * u) ** 2 + np.linalg.norm(Atu - s * v) ** 2)


def minres(Mop, rhs, tol, maxit):
    """MINRES (Paige and Saunders, 1975) for a symmetric, possibly indefinite
    operator, from x0 = 0: Lanczos vectors q_k, the QR factorisation of the
    tridiagonal projection by Givens rotations, and the update
    x_k = x_{k-1} + tau_k d_k.  Stops after maxit steps or when the residual
    norm |phi| falls to tol * ||rhs||."""
    rhs = np.asarray(rhs, dtype=np.float64)
    x = np.zeros_like(rhs)
    beta1 = float(np.linalg.norm(rhs))
    if beta1 == 0.0:
        return x, 0
    q_prev = np.zeros_like(rhs)
    q = rhs / beta1
    d1 = np.zeros_like(rhs)
    d2 = np.zeros_like(rhs)
    c1, s1, c2, s2 = 1.0, 0.0, 1.0, 0.0   # rotations k-1 and k-2
    beta = 0.0                           # coupling of q_k to q_{k-1}
    phi = beta1
    its = 0
    for _ in range(maxit):
        z = Mop(q)
        alpha = float(q @ z)
        z = z - alpha * q - beta * q_prev
        beta_next = float(np.linalg.norm(z))
        eps = s2 * beta                  # entry two rows above the diagonal
        dlt = c2 * beta
        delta = c1 * dlt + s1 * alpha    # entry one row above the diagonal
        gbar = -s1 * dlt + c1 * alpha
        gamma = math.hypot(gbar, beta_next)
        its += 1
        if gamma == 0.0:
            break
        c, sn = gbar / gamma, beta_next / gamma
        tk = c * phi
        phi = -sn * phi
        dn = (q - delta * d1 - eps * d2) / gamma
        x = x + tk * dn
        d2, d1 = d1, dn
        c2, s2, c1, s1 = c1, s1, c, sn
        q_prev = q
        q = z / beta_next if beta_next > 0.0 else np.zeros_like(z)
        beta = beta_next
        if abs(phi) <= tol * beta1 or beta_next == 0.0:
            break
    return x, its


def sqmr(Mop, rhs, tol, maxit, Pop=None):
    """Symmetric QMR (Freund and Nachtigal, 1994) for a symmetric, possibly
    indefinite operator with a symmetric, possibly indefinite preconditioner
    ``Pop`` (None: the identity), from x0 = 0.  The conjugate-gradient-like
    recurrence gives the Lanczos residuals r_k; the quasi-residual norm tau_k
    comes from a running Givens-type smoothing with c_k = 1/sqrt(1 + theta_k^2),
    theta_k = ||r_k|| / tau_{k-1}, and the iterate is advanced by
    d_k = c_k^2 theta_{k-1}^2 d_{k-1} + c_k^2 alpha_k q_k.  Without a
    preconditioner the Lanczos residuals are orthogonal and the iterates are
    those of MINRES.  Stops after maxit steps, when tau_k falls to tol * ||rhs||
    or on a breakdown (q^T M q = 0 or r^T P r = 0)."""
    rhs = np.asarray(rhs, dtype=np.float64)
    x = np.zeros_like(rhs)
    tau0 = float(np.linalg.norm(rhs))
    if tau0 == 0.0:
        return x, 0
    P = Pop if Pop is not None else (lambda y: y)
    r = rhs.copy()
    t = P(r)
    q = t.copy()
    rho = float(r @ t)
    tau = tau0
    theta = 0.0
    d = np.zeros_like(rhs)
    its = 0
    for _ in range(maxit):
        if rho == 0.0:
            break
        w = Mop(q)
        sigma = float(q @ w)
        if sigma == 0.0:
            break
        alpha = rho / sigma
        r = r - alpha * w
        theta_prev = theta
        theta = float(np.linalg.norm(r)) / tau
        c2 = 1.0 / (1.0 + theta * theta)
        tau = tau * theta * math.sqrt(c2)
        d = (c2 * theta_prev * theta_prev) * d + (c2 * alpha) * q
        x = x + d
        its += 1
        if tau <= tol * tau0:
            break
        t = P(r)
        rho_next = float(r @ t)
        q = t + (rho_next / rho) * q
        rho = rho_next
    return x, its


def _stage2(ops, k, target, tol, normA, g, r, b, p, seed, precond, budget, stats, rand_state,
            sig1, U1, V1, rn1, trace=None, solver="gdk", jd_maxit=20, jd_tol=0.1):
    n, m = ops.n, ops.m
    N = n + m
    g = min(g, N)
    r = min(r, max(1, g - b - p))
    normB = normA
    refined = target == "smallest"

    if precond is not None:
        if callable(precond):
            Kc = precond
        else:
            d = precond.copy()
            d[d <= 0] = 1.0
            Kc = lambda R: R / d[:, None]

        def K(R):  # pseudo-inverse composition [K A^T y_u; A K y_v] of B
            return np.vstack([Kc(ops.At_mul(R[n:])), ops.A_mul(Kc(R[:n]))])
    else:
        K = lambda R: R

    def rand_next(c):
        s = STREAM_BREAK + rand_state["count"]
        rand_state["count"] += 1
        return counter_uniform(seed, s, N, c)

    # stage-1 lower bounds: max(sigma - sqrt(2) ||r^C||/sigma, ||A|| eps), ||r^C|| = sigma ||r||
    taus = np.maximum(sig1 - math.sqrt(2.0) * np.where(np.isfinite(rn1), rn1, sig1), normA * EPS)

    S = SearchSpace(ops.B, N, None)
    X0 = np.vstack([V1, U1]) / math.sqrt(2.0)
    T, _, _ = ortho_block(X0, [], rand_next)
    S.append(T)

    y_prev = None
    restarts = 0
    since_reset = 0
    resets = 0
    iters = 0
    status = "budget"
    nlock = 0
    while nlock < k:
        tau = taus[min(nlock, len(taus) - 1)]
        if refined:
            Rq = np.linalg.qr(S.W - tau * S.V, mode="r")
            _, sv, Vh = np.linalg.svd(Rq)
            Y = Vh[::-1].T                     # right singular vectors, ascending
            lam = np.einsum("ij,ij->j", Y, S.H @ Y)
        else:
            lam, Y = np.linalg.eigh(S.H)
            lam, Y = lam[::-1], Y[:, ::-1]
        normB = max(normB, float(np.max(np.abs(lam))))
        nc = min(S.g, b)
        X = S.V @ Y[:, :nc]
        Wy = S.W @ Y[:, :nc]
        R = Wy - X * lam[:nc]
        rn = np.linalg.norm(R, axis=0)
        conv = np.zeros(nc, dtype=bool)
        for j in range(nc):
            if rn[j] <= math.sqrt(2.0) * normB * tol:  # eq. B_secondCriterion
                conv[j] = _halves_residual(X[:, j], Wy[:, j], lam[j], n) < normA * tol
        if trace is not None:
            trace(2, iters, S.g, lam[:nc], rn, conv)
        L = 0
        while L < nc and conv[L]:
            L += 1
        if L > 0:
            S.X = np.hstack([S.X, X[:, :L]])
            S.lock_vals.extend(lam[:L].tolist())
            nlock += L
            if nlock >= k:
                status = "converged"
                break
            # forced restart that drops the locked vectors
            r_eff = min(r, S.g - L)
            Yr = Y[:, L:L + r_eff]
            prev = _pad(y_prev, S.g)
            if prev is not None and p > 0:
                room = max(0, g - b - r_eff)
                if room:
                    Yr = _small_orth_append(np.hstack([Y[:, :L], Yr]), prev[:, : min(p, room)])[:, L:]
            S.restart(Yr)
            restarts += 1
            since_reset += 1
            y_prev = None
            continue
        if ops.mv >= budget:
            status = "budget"
            break
        block = list(range(nc))
        if since_reset > 0 and min(rn[block]) < math.sqrt(since_reset) * normB * EPS:
            S.reset()
            resets += 1
            since_reset = 0
            y_prev = None
            continue
        Yb = Y[:, block]
        if S.g + len(block) > g:
            r_eff = min(r, S.g)
            Yr = Y[:, :r_eff]
            prev = _pad(y_prev, S.g)
            if prev is not None and p > 0:
                room = max(0, g - b - r_eff)
                if room:
                    Yr = _small_orth_append(Yr, prev[:, : min(p, room)])
            S.restart(Yr)
            Yb = Yr.T @ Yb
            restarts += 1
            since_reset += 1
        if solver == "jd":
            # Jacobi-Davidson correction (the paper's second stage, JDQMR):
            # (I - QQ^T)(B - s I)(I - QQ^T) t = r with Q the locked vectors and
            # the block's Ritz vectors, s the active shift (refined) or the
            # Ritz value, solved approximately by symmetric QMR with the
            # preconditioner (I - QQ^T) K (I - QQ^T); the sign of t does not
            # matter for the expansion
            Q = np.hstack([S.X, X[:, block]])
            T = np.empty((N, len(block)))
            proj = lambda y: y - Q @ (Q.T @ y)
            Pop = None if precond is None else (lambda y: proj(K(proj(y)[:, None])[:, 0]))
            for jj, j in enumerate(block):
                shift = tau if refined else lam[j]

                def Mop(y, shift=shift):
                    y = proj(y)
                    return proj(ops.B(y[:, None])[:, 0] - shift * y)

                rj = proj(R[:, j])
                T[:, jj], its = sqmr(Mop, rj, jd_tol, jd_maxit, Pop)
                stats.setdefault("inner_iters", 0)
                stats["inner_iters"] += its
        else:
            T = K(R[:, block])
        T, _, _ = ortho_block(T, [S.X, S.V], rand_next)
        y_prev = Yb
        S.append(T)
        iters += 1

    stats["iters"][1] = iters
    stats["restarts"][1] = restarts
    stats["resets"] += resets
    Xl = S.X
    vals = list(S.lock_vals)
    if Xl.shape[1] < k:  # budget: complete with the current best approximations
        if refined:
            tau = taus[min(nlock, len(taus) - 1)]
            Rq = np.linalg.qr(S.W - tau * S.V, mode="r")
            _, _, Vh = np.linalg.svd(Rq)
            Y = Vh[::-1].T
            lam = np.einsum("ij,ij->j", Y, S.H @ Y)
        else:
            lam, Y = np.linalg.eigh(S.H)
            lam, Y = lam[::-1], Y[:, ::-1]
        extra = min(k - Xl.shape[1], S.g)
        Xl = np.hstack([Xl, S.V @ Y[:, :extra]])
        vals.extend(lam[:extra].tolist())
    Vv = Xl[:n]
    Uu = Xl[n:]
    Vv = Vv / np.maximum(np.linalg.norm(Vv, axis=0), 1e-300)
    Uu = Uu / np.maximum(np.linalg.norm(Uu, axis=0), 1e-300)
    return np.abs(np.array(vals)), Uu, Vv, nlock, status


# ---------------------------------------------------------------------------
# Two-sided Rayleigh-Ritz clean-up and eq. (res)
# ---------------------------------------------------------------------------
def svd_residuals(A, sigma, U, V):
    """eq. (res): sqrt(||A v - sigma u||^2 + ||A^T u - sigma v||^2) per triplet."""
    A = sp.csr_matrix(A)
    r1 = np.linalg.norm(A @ V - U * sigma, axis=0)
    r2 = np.linalg.norm(A.T @ U - V * sigma, axis=0)
    return np.sqrt(r1 ** 2 + r2 ** 2)


def _cleanup(ops, sigma, U, V, target):
    Uq, _ = np.linalg.qr(U)
    Vq, _ = np.linalg.qr(V)
    AV = ops.A_mul(Vq)
    H2 = Uq.T @ AV
    P, s, Qt = np.linalg.svd(H2)
    U2 = Uq @ P
    V2 = Vq @ Qt.T
    order = np.argsort(-s) if target == "largest" else np.argsort(s)
    return s[order], U2[:, order], V2[:, order]


def _sign_normalise(U, V):
    U = U.copy()
    V = V.copy()
    for j in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, j])))
        if V[i, j] < 0:
            V[:, j] *= -1
            U[:, j] *= -1
    return U, V


# ---------------------------------------------------------------------------
# Driver: Algorithm 1
# ---------------------------------------------------------------------------
def svds(A, k, target="largest", tol=1e-10, *, max_basis=None, min_restart=None, block=None,
         prev_retain=None, max_matvecs=None, norm_A=None, seed=0, precond="none",
         force_stage2=False, cleanup=True, stage1_tol=None, trace=None, time_limit=None,
         capture=None, method="hybrid", relative=False, pc_block=64, stage2_solver="jd",
         jd_maxit=20, jd_tol=0.1):
    """k largest or smallest singular triplets of the sparse matrix A with
    eq. (res) residual below tol*||A||.  Returns (sigma, U, V, rnorm, stats);
    U is m x k, V is n x k, both in target order with the largest-magnitude
    entry of each v positive.  ``stage1_tol`` sets the user tolerance of the
    stage-1 test separately (each stage's eigensolver parameters can be set
    apart, Section 3.4); stage 2 and acceptance always use ``tol``.

    ``precond`` is "none", "jacobi", "blockjacobi" (blocks of ``pc_block``
    columns) or a callable applying a linear operator to
    an N x c block of vectors in the space of the smaller Gram matrix (N =
    min(m, n)).  ``capture`` = {"every": e, "max": P} collects, at every e-th
    stage-1 iteration (at most P times), the residual, the Ritz vector and
    the target index of the block's first target into its "R", "X" and "idx"
    lists (training pairs for a learned preconditioner).

    ``method``: "hybrid" (the two-stage method), "normal" (stage 1 on the
    normal equations alone, accepted as it ends) or "augmented" (stage 2 on
    B alone from counter-based random vectors, largest values only: for the
    smallest, B's spectrum is symmetric about the target region and its
    shifts need the stage-1 bounds) -- the single-stage methods of
    Section 3.4.  ``relative``: the stopping rule
    ||r|| <= tol * sigma of the low-accuracy condition estimate (Section 4.4);
    only with method "normal".  ``stage2_solver``: "jd" (the default:
    Jacobi-Davidson with at most ``jd_maxit`` symmetric-QMR steps to a
    quasi-residual reduction of ``jd_tol``, preconditioned by the stage-2
    composition; the paper's second stage is JDQMR, Section 3.4) or "gdk"
    (GD+k with the same preconditioner on the residuals)."""
    t0 = time.perf_counter()
    if target not in ("largest", "smallest"):
        raise ValueError("target must be 'largest' or 'smallest'")
    A = sp.csr_matrix(A, dtype=np.float64)
    m0, n0 = A.shape
    transposed = m0 < n0            # work with the smaller Gram matrix (Section 2.1)
    Aw = A.T.tocsr() if transposed else A
    ops = Operators(Aw)
    m, n = ops.m, ops.n
    if not (1 <= k <= n):
        raise ValueError("k out of range")
    if method not in ("hybrid", "normal", "augmented"):
        raise ValueError("method must be 'hybrid', 'normal' or 'augmented'")
    if relative and method != "normal":
        raise ValueError("the relative stopping rule needs method 'normal'")
    if stage2_solver not in ("gdk", "jd"):
        raise ValueError("stage2_solver must be 'jd' or 'gdk'")
    if method == "augmented" and target == "smallest":
        # on B alone the smallest values are interior, with -sigma as close to a
        # shift near zero as +sigma (and m - n zero eigenvalues when m != n):
        # the shifts need the stage-1 bounds, which is the hybrid method
        raise ValueError("the augmented method alone seeks the largest values only")
    g, r, b, p = default_params(k, target, max_basis, min_restart, block, prev_retain)
    if not (b >= 1 and g >= r + p + b and r >= 1 and min(g, n) >= k + b):
        raise ValueError("need max_basis >= min_restart + prev_retain + block, and k + block "
                         "within the basis and the smaller dimension")
    budget = max_matvecs if max_matvecs else 2_000_000
    if time_limit is not None:
        budget = _TimedBudget(budget, time_limit)
    stats = {"iters": [0, 0], "restarts": [0, 0], "resets": 0, "matvecs": [0, 0],
             "stage_exit": 1, "stage1_status": None, "norm_A_used": None, "nconv": 0,
             "seconds": [0.0, 0.0]}
    rand_state = {"count": 0}
    if callable(precond):
        pc = precond  # a linear operator on vectors of length min(m, n) (the space of C)
    elif precond == "blockjacobi":
        pc = block_jacobi(Aw, pc_block)
    else:
        pc = jacobi_diag(Aw) if precond == "jacobi" else None
    if norm_A is None or norm_A <= 0:
        normA = estimate_norm(ops, seed)
        ops.mv = 0
    else:
        normA = float(norm_A)

    # ---- stage 1 on C
    tol1 = tol if stage1_tol is None else float(stage1_tol)
    if capture is not None:
        capture.setdefault("R", [])
        capture.setdefault("X", [])
        capture.setdefault("idx", [])
    t1 = time.perf_counter()
    if method == "augmented":
        # random start on B: [v; u] from one counter-based block of length n + m
        X0 = counter_uniform(seed, STREAM_INIT, n + m, k)
        V, U = X0[:n], X0[n:]
        sig = np.zeros(k)
        rn = np.full(k, np.inf)
        status = "augmented"
    else:
        Xk, normC, status = _stage1(ops, k, target, tol1, normA, g, r, b, p, seed, pc, budget,
                                    stats, rand_state, trace, capture, relative)
        normA = max(normA, math.sqrt(normC))
        sig, U, V, rn = _final_rr(ops, Xk, target)
        stats["matvecs"][0] = ops.mv
        t1 = time.perf_counter()
        stats["seconds"][0] = t1 - t0
    lim = tol * sig if relative else normA * tol
    ok = np.all(rn < lim)
    nconv = k if ok else int(np.sum(rn < lim))
    if method == "augmented" or (method == "hybrid" and status != "budget"
                                 and (force_stage2 or not ok)):
        # ---- stage 2 on B
        mv0 = ops.mv
        sig, U, V, nconv, status2 = _stage2(ops, k, target, tol, normA, g, r, b, p, seed, pc,
                                            budget, stats, rand_state, sig, U, V, rn, trace,
                                            stage2_solver, jd_maxit, jd_tol)
        stats["matvecs"][1] = ops.mv - mv0
        stats["stage_exit"] = 2
        stats["seconds"][1] = time.perf_counter() - t1
    if cleanup:
        sig, U, V = _cleanup(ops, sig, U, V, target)
    rnorm = svd_residuals(Aw, sig, U, V)
    if transposed:
        U, V = V, U
    U, V = _sign_normalise(U, V)
    stats["norm_A_used"] = normA
    lim = tol * sig if relative else normA * tol
    stats["nconv"] = int(np.sum(rnorm < lim)) if method != "hybrid" else int(nconv)
    stats["converged"] = bool(np.all(rnorm < lim) and stats["nconv"] >= k)
    return sig, U, V, rnorm, stats


def condest(A, tol=0.1, *, seed=0, precond="none", max_basis=None, min_restart=None,
            max_matvecs=None, norm_A=None):
    """Condition-number estimate of Section 4.4: one largest and one smallest
    singular triplet, block size 1, stage 1 stopped when the residual is
    below tol times the singular value (tol = 0.1 gives about 10 %).
    Returns (kappa, sigma_max, sigma_min, (stats_largest, stats_smallest))."""
    kw = dict(block=1, seed=seed, precond=precond, max_basis=max_basis, min_restart=min_restart,
              max_matvecs=max_matvecs, norm_A=norm_A, method="normal", relative=True)
    s1, _, _, _, st1 = svds(A, 1, "largest", tol, **kw)
    s0, _, _, _, st0 = svds(A, 1, "smallest", tol, **kw)
    return float(s1[0] / s0[0]), float(s1[0]), float(s0[0]), (st1, st0)
