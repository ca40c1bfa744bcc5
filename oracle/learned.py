"""FP64 CPU reference of the learned preconditioner for the correction step.

TEST INFRASTRUCTURE ONLY: imported by tests, never by the library.

The paper's solver accepts a user preconditioner for A^T A, A A^T or the
augmented matrix (the applyPreconditioner hook of the interface, Section 3.4)
and gains most from it on hard problems (Section 4, the preconditioned
comparison).  The learned preconditioner plugs into that hook.  It is a
polynomial in the Jacobi-scaled operator whose coefficients vary from row to
row and come out of a small network that reads local features of the sparse
operator:

    K(r) = D^-1/2 sum_{l=0..d} c_l (.) T_l(2M - I) D^-1/2 r,
    M = D^-1/2 A^T A D^-1/2 / rho,

with D = diag(A^T A) (zeros replaced by ones), rho = max_i (D^-1/2 |A|^T |A|
D^-1/2 1)_i (a Gershgorin bound, so the spectrum of M lies in [0, 1]), T_l the
Chebyshev polynomials of the first kind and (.) the row-wise product.  A is
the work matrix (the tall one of A and A^T); vectors live in the space of
C = A^T A.

Each row's polynomial is a positive mixture of fixed positive polynomials:

    c_{l,i} = sum_m exp(o_{m,i}) Psi[l, m],
    Psi[l, m] = g_l a_l(delta_m),

where a_l(delta) are the Chebyshev coefficients of 1/(x + delta) on [0, 1]
(closed form: with y = 2x - 1, a = 1 + 2 delta, q = a - sqrt(a^2 - 1),
1/(x + delta) = 2/sqrt(a^2 - 1) (1 + 2 sum_{l>=1} (-q)^l T_l(y))), g_l the
Jackson damping factors of degree d (they keep the truncated series of a
positive function positive, Jackson 1912; the kernel polynomial method uses
them the same way) and delta_m = 10^(-5 + 5m/7), m = 0..7.  Every row's
polynomial is therefore positive on the spectrum of M for any network output;
an indefinite polynomial stalls the eigensolver.

The network maps local features of the operator to the 8 log-weights o:

    features f (N x 8):
      f0 = 1
      f1 = log d_i - mean_j log d_j
      f2 = (M 1)_i
      f3 = (D^-1/2 |A|^T |A| D^-1/2 1)_i / rho
      f4 = nnz of column i / mean column nnz
      f5 = (M f2)_i                         (= (M^2 1)_i)
      f6 = f7 = 0                           (reserved)
    aggregation over the sparsity of C, weights |A|^T |A|, row-normalised:
      agg(h) = S^-1 |A|^T |A| h,  S = diag(|A|^T |A| 1) (zeros -> 1)
    layer 1: x1 = [f, agg(f)]   (16)  z1 = x1 W1 + b1 (32)   h1 = gelu(z1)
    layer 2: x2 = [h1, agg(h1)] (64)  z2 = x2 W2 + b2 (32)   h2 = gelu(z2)
    output:  o = clip(h2 W3 + b3, -30, 30)   (8)

gelu(x) = x Phi(x) with Phi the standard normal distribution function.

Training pairs come from the solver itself: at selected stage-1 iterations
the residual r of the block's first target is kept.  With r^ = r / |r| the
pair is (q, e) = (C r^, r^): the exact inverse of C maps q to e, so K(q) should
point along e.  The loss of a pair is 1 - (t^T e)^2 / (|t|^2 |e|^2) with
t = K(q): it ignores the scale and sign of t, which the eigensolver ignores
too (the block is orthonormalised before use).  It measures how far K C is
from a multiple of the identity on the vectors the solver produces, the
quantity that governs the convergence of preconditioned eigensolvers of this
kind (Knyazev and Neymeyr's analysis of preconditioned inverse iteration).
Parameters are updated with Adam.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
from scipy.special import erf

NF = 8          # features per row
HID = 32        # hidden width
NOUT = 8        # log-weights of the shifted-reciprocal components
MAX_DEGREE = 15
DELTAS = 10.0 ** (-5.0 + 5.0 * np.arange(NOUT) / (NOUT - 1))
OCLIP = 30.0
SHAPES = [("W1", (2 * NF, HID)), ("b1", (HID,)), ("W2", (2 * HID, HID)), ("b2", (HID,)),
          ("W3", (HID, NOUT)), ("b3", (NOUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    """Flat FP32/FP64 parameter vector -> dict of arrays (row-major)."""
    out, o = {}, 0
    for name, shp in SHAPES:
        sz = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + sz], dtype=np.float64).reshape(shp)
        o += sz
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def work_matrix(A):
    """The tall one of A and A^T (the solver works with C = Aw^T Aw)."""
    A = sp.csr_matrix(A, dtype=np.float64)
    return A.T.tocsr() if A.shape[0] < A.shape[1] else A


class Operator:
    """Quantities of the work matrix used by features, aggregation and K."""

    def __init__(self, A):
        self.Aw = work_matrix(A)
        self.absA = abs(self.Aw)
        d = np.asarray(self.Aw.multiply(self.Aw).sum(axis=0)).ravel()
        d[d <= 0] = 1.0
        self.d = d
        self.dh = 1.0 / np.sqrt(d)
        g = self.dh * (self.absA.T @ (self.absA @ self.dh))
        self.rho = float(g.max()) if g.size and g.max() > 0 else 1.0
        S = np.asarray(self.absA.T @ (self.absA @ np.ones(self.Aw.shape[1])))
        S[S <= 0] = 1.0
        self.S = S
        self.N = self.Aw.shape[1]

    def M(self, z):
        """M z = D^-1/2 Aw^T Aw D^-1/2 z / rho (z may be N x c)."""
        dh = self.dh if z.ndim == 1 else self.dh[:, None]
        return dh * (self.Aw.T @ (self.Aw @ (dh * z))) / self.rho

    def agg(self, h):
        return (self.absA.T @ (self.absA @ h)) / self.S[:, None]

    def agg_t(self, g):
        """Transpose of agg: |A|^T |A| S^-1 g."""
        return self.absA.T @ (self.absA @ (g / self.S[:, None]))


def features(op):
    N = op.N
    f = np.zeros((N, NF))
    f[:, 0] = 1.0
    ld = np.log(op.d)
    f[:, 1] = ld - ld.mean()
    f[:, 2] = op.M(np.ones(N))
    f[:, 3] = op.dh * (op.absA.T @ (op.absA @ op.dh)) / op.rho
    cnt = np.diff(op.Aw.tocsc().indptr).astype(np.float64)
    f[:, 4] = cnt / max(cnt.mean(), 1e-300)
    f[:, 5] = op.M(f[:, 2])
    return f


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def jackson(degree):
    """Jackson damping factors g_0..g_d (g_0 = 1)."""
    n = degree + 1
    l = np.arange(n)
    th = np.pi / (n + 1)
    return ((n - l + 1) * np.cos(l * th) + np.sin(l * th) / np.tan(th)) / (n + 1)


def reciprocal_chebyshev(delta, degree):
    """Chebyshev coefficients a_0..a_d of 1/(x + delta) on x in [0, 1]
    (variable y = 2x - 1)."""
    a = 1.0 + 2.0 * delta
    s = math.sqrt(a * a - 1.0)
    q = a - s
    l = np.arange(degree + 1)
    return np.where(l == 0, 2.0 / s, 4.0 / s * (-q) ** l)


def psi(degree):
    """(d+1) x 8 matrix mapping component weights to coefficients."""
    g = jackson(degree)
    return np.stack([g * reciprocal_chebyshev(dm, degree) for dm in DELTAS], axis=1)


def forward(op, theta, f, degree):
    """Coefficients c (N x (d+1)) and the cache the backward pass needs."""
    p = unpack(theta)
    x1 = np.hstack([f, op.agg(f)])
    z1 = x1 @ p["W1"] + p["b1"]
    h1 = gelu(z1)
    x2 = np.hstack([h1, op.agg(h1)])
    z2 = x2 @ p["W2"] + p["b2"]
    h2 = gelu(z2)
    o_raw = h2 @ p["W3"] + p["b3"]
    o = np.clip(o_raw, -OCLIP, OCLIP)
    w = np.exp(o)
    c = w @ psi(degree).T
    return c, dict(x1=x1, z1=z1, x2=x2, z2=z2, h2=h2, o_raw=o_raw, w=w, degree=degree)


def backward(op, theta, cache, dc):
    """Gradient of a scalar loss with respect to the flat parameters, given
    dloss/dc (N x (d+1))."""
    p = unpack(theta)
    g = {}
    do = (dc @ psi(cache["degree"])) * cache["w"]
    do = np.where(np.abs(cache["o_raw"]) < OCLIP, do, 0.0)
    g["W3"] = cache["h2"].T @ do
    g["b3"] = do.sum(axis=0)
    dh2 = do @ p["W3"].T
    dz2 = dh2 * gelu_grad(cache["z2"])
    g["W2"] = cache["x2"].T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dx2 = dz2 @ p["W2"].T
    dh1 = dx2[:, :HID] + op.agg_t(dx2[:, HID:])
    dz1 = dh1 * gelu_grad(cache["z1"])
    g["W1"] = cache["x1"].T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


def chebyshev_basis(op, R, degree):
    """Z[l] = T_l(2M - I) D^-1/2 R for l = 0..degree (R is N x c)."""
    R = np.asarray(R, dtype=np.float64)
    if R.ndim == 1:
        R = R[:, None]
    Z = [op.dh[:, None] * R]
    if degree >= 1:
        Z.append(2.0 * op.M(Z[0]) - Z[0])
    for _ in range(2, degree + 1):
        Z.append(2.0 * (2.0 * op.M(Z[-1]) - Z[-1]) - Z[-2])
    return Z


def apply(op, c, R, degree):
    """T = K(R) with the coefficient matrix c (N x (d+1) or wider)."""
    Z = chebyshev_basis(op, R, degree)
    acc = sum(c[:, [l]] * Z[l] for l in range(degree + 1))
    return op.dh[:, None] * acc


def loss_and_dc(op, c, R, E, degree):
    """Mean pair loss over the pairs with nonzero label and output, and its
    gradient with respect to c."""
    Z = chebyshev_basis(op, R, degree)
    T = op.dh[:, None] * sum(c[:, [l]] * Z[l] for l in range(degree + 1))
    te = np.sum(T * E, axis=0)
    tt = np.sum(T * T, axis=0)
    ee = np.sum(E * E, axis=0)
    valid = (ee > 0) & (tt > 0)
    nv = max(int(valid.sum()), 1)
    L = np.where(valid, 1.0 - te * te / np.where(valid, tt * ee, 1.0), 0.0)
    # dL/dT per pair: 2/(tt ee) [ te^2/tt T - te E ]
    a = np.where(valid, 2.0 * te * te / np.where(valid, tt * tt * ee, 1.0), 0.0)
    b = np.where(valid, 2.0 * te / np.where(valid, tt * ee, 1.0), 0.0)
    G = (T * a - E * b) / nv
    dc = np.zeros_like(c)
    for l in range(degree + 1):
        dc[:, l] = op.dh * np.sum(G * Z[l], axis=1)
    return float(L.sum() / nv), dc


def make_pairs(op, R):
    """Training pairs (Q, E) from captured residuals R (N x P): E = R with
    unit columns (zero columns stay zero), Q = C E."""
    R = np.asarray(R, dtype=np.float64)
    nr = np.linalg.norm(R, axis=0)
    E = R / np.where(nr > 0, nr, 1.0)
    Q = op.Aw.T @ (op.Aw @ E)
    return Q, E


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) of the flat parameters, in place;
    ``step`` counts from 1."""
    m[:] = beta1 * m + (1.0 - beta1) * grad
    v[:] = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    theta[:] = theta - lr * mh / (np.sqrt(vh) + eps)
    return theta


def init_params(rng, scale=1.0, bias=0.0):
    """Random hidden layers (uniform, variance-preserving), zero output
    weights and output bias ``bias``: every row starts with the same
    positive mixture (equal weights for bias 0)."""
    p = {name: np.zeros(shp) for name, shp in SHAPES}
    p["W1"] = rng.uniform(-1, 1, (2 * NF, HID)) * scale * math.sqrt(3.0 / (2 * NF))
    p["W2"] = rng.uniform(-1, 1, (2 * HID, HID)) * scale * math.sqrt(3.0 / (2 * HID))
    p["b3"][:] = bias
    return pack(p)
