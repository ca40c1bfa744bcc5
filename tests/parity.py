"""Accuracy bound for comparing singular values of two solvers.

Two approximations of the same singular value, each with an eq. (res)
residual r = sqrt(||A v - s u||^2 + ||A^T u - s v||^2) for unit u and v, can
differ by what either may lie from the exact value.  For the two-sided
Rayleigh quotient s = u^T A v the error is at most ||r|| (the augmented
matrix B = [0 A^T; A 0] has the eigenvalue s within ||r_B|| <= ||r|| of the
unit vector [v; u]/sqrt(2)) and, quadratically, at most ||r||^2 / gap, where
gap is the distance from s to the rest of B's spectrum: the other singular
values, their negatives, and zero when A is not square (Section 2, eq. (res)
and the spectrum of B).  Rounding adds a few eps ||A|| to each side.  A
relative error of 1e-10 is asserted wherever this bound allows it; where it
does not (clustered or tiny singular values at a residual near 1e-10 ||A||)
the bound itself is asserted and the case is printed.
"""
from __future__ import annotations

import numpy as np

EPS = 2.220446049250313e-16


def sigma_bound(sigma, spectrum, rnorm, norm_A):
    """Per-value bound on |s_i - sigma_i| for values sigma (k) with residuals
    rnorm (k); spectrum: known singular values around them (at least sigma
    itself) for the gaps.  The negatives of the values and zero lie at least
    s_i away from s_i."""
    sigma = np.asarray(sigma, dtype=np.float64)
    spec = np.asarray(spectrum, dtype=np.float64)
    rn = np.asarray(rnorm, dtype=np.float64)
    out = np.empty_like(sigma)
    for i, s in enumerate(sigma):
        d = np.abs(spec - s)
        d = d[d > 0.0]
        # distance to the other values, and at least s to -sigma_j and to zero
        gap = min(d.min() if d.size else np.inf, s)
        quad = rn[i] ** 2 / gap if gap > 0 else np.inf
        out[i] = min(rn[i], quad) + 8.0 * EPS * norm_A
    return out


def assert_sigma_parity(got, ref, spectrum, rn_got, rn_ref, norm_A, what=""):
    """|got - ref| <= max(1e-10 ref, bound(got) + bound(ref)) elementwise;
    prints the values for which the bound is the wider of the two."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    bnd = sigma_bound(ref, spectrum, rn_got, norm_A) + sigma_bound(ref, spectrum, rn_ref, norm_A)
    tol = np.maximum(1e-10 * ref, bnd)
    err = np.abs(got - ref)
    wide = np.nonzero(bnd > 1e-10 * ref)[0]
    rel = err / ref
    print(f"[parity] {what} max relative sigma error {rel.max():.2e}", flush=True)
    if wide.size:
        print(f"[parity] {what} bound above 1e-10 relative for positions {wide.tolist()}: "
              f"bound/sigma {(bnd[wide] / ref[wide]).tolist()}, measured {rel[wide].tolist()}",
              flush=True)
    assert np.all(err <= tol), (what, got, ref, err / ref, tol / ref)
    return rel.max()
