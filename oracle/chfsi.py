"""Chebyshev-filtered subspace iteration (the eigensolver the paper uses,
Sec. II.B, citing Zhou, Saad, Tiago and Chelikowsky, J. Comput. Phys. 2006).

TEST INFRASTRUCTURE ONLY (see the oracle package header).

The paper cites the method without restating it; the steps below follow the
published scaled three-term recurrence:
  * upper bound b of the spectrum: k-step Lanczos, b = theta_max + |beta_k|;
  * filter bounds: a_L = lowest Ritz value, a = highest kept Ritz value
    (before any Rayleigh-Ritz: a_L = lowest Lanczos value,
    a = a_L + (b - a_L)/10);
  * filter of degree m: e = (b-a)/2, c = (b+a)/2, s = e/(a_L - c), tau = 2/s,
        Y_1 = (s/e)(H X - c X),
        s' = 1/(tau - s),  Y_i = (2 s'/e)(H Y_{i-1} - c Y_{i-1}) - s s' Y_{i-2},
    with Y_0 = X;
  * Rayleigh-Ritz with the quadrature weight dV: S = Y^H Y dV,
    Hs = Y^H (H Y) dV (symmetrised), S = L L^H, Q diag(lam) Q^H =
    L^{-1} Hs L^{-H} (ascending), C = L^{-H} Q, X = Y C.

Pins: on plane waves of the kinetic operator the filter equals the scaled
Chebyshev polynomial evaluated by numpy.polynomial; converged Ritz values
equal dense LAPACK eigenvalues of the assembled matrix (tests).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def lanczos(apply_h, v0, steps):
    """k-step Lanczos from v0.  Returns (theta_min, upper_bound) with
    upper_bound = theta_max + |beta_k| (Zhou and Li's safeguarded bound)."""
    v = v0 / np.linalg.norm(v0)
    alpha, beta = [], []
    v_prev = np.zeros_like(v)
    b_prev = 0.0
    f = None
    for j in range(steps):
        w = apply_h(v)
        a = np.vdot(v, w).real
        w = w - a * v - b_prev * v_prev
        alpha.append(a)
        b = np.linalg.norm(w)
        beta.append(b)
        f = w
        if b == 0.0:
            break
        v_prev, v = v, w / b
        b_prev = b
    T = np.diag(alpha)
    for j in range(len(alpha) - 1):
        T[j, j + 1] = T[j + 1, j] = beta[j]
    th = np.linalg.eigvalsh(T)
    return float(th[0]), float(th[-1] + np.linalg.norm(f))


def cheb_filter(apply_h, X, m, a, b, aL):
    """Scaled degree-m Chebyshev filter of the block X (shape (ns, nd))."""
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    s = e / (aL - c)
    tau = 2.0 / s
    Y = (s / e) * (apply_h(X) - c * X)
    Yprev = X
    for _ in range(2, m + 1):
        s2 = 1.0 / (tau - s)
        Ynew = (2.0 * s2 / e) * (apply_h(Y) - c * Y) - (s * s2) * Yprev
        Yprev, Y = Y, Ynew
        s = s2
    return Y


def rayleigh_ritz(apply_h, Y, dv):
    """Returns (eigenvalues ascending, X = Y C) with X^H X dV = I."""
    HY = apply_h(Y)
    S = dv * (Y.conj() @ Y.T)            # S_ij = <y_i|y_j> dV
    Hs = dv * (Y.conj() @ HY.T)
    Hs = 0.5 * (Hs + Hs.conj().T)
    S = 0.5 * (S + S.conj().T)
    Lc = np.linalg.cholesky(S)
    Linv_H = sla.solve_triangular(Lc, Hs, lower=True)
    A = sla.solve_triangular(Lc, Linv_H.conj().T, lower=True).conj().T
    A = 0.5 * (A + A.conj().T)
    lam, Q = np.linalg.eigh(A)
    C = sla.solve_triangular(Lc.conj().T, Q, lower=False)
    X = (Y.T @ C).T
    return lam, X


def chfsi_pass(apply_h, X, m, bounds, dv):
    """One filter + Rayleigh-Ritz pass.  bounds = (a, b, aL)."""
    a, b, aL = bounds
    Y = cheb_filter(apply_h, X, m, a, b, aL)
    lam, Xn = rayleigh_ritz(apply_h, Y, dv)
    return lam, Xn


def eigensolve(apply_h, X0, m, v0, lanczos_steps, dv, passes, tol=None):
    """Repeated ChFSI passes at a fixed operator; used as a fixed-D reference
    (converges the lowest ns eigenpairs).  Returns (lam, X, passes_done)."""
    th_min, b = lanczos(apply_h, v0, lanczos_steps)
    aL = th_min
    a = aL + (b - aL) / 10.0
    X = X0
    lam_old = None
    for it in range(passes):
        lam, X = chfsi_pass(apply_h, X, m, (a, b, aL), dv)
        aL, a = lam[0], lam[-1]
        if tol is not None and lam_old is not None and np.max(np.abs(lam - lam_old)) < tol:
            return lam, X, it + 1
        lam_old = lam
    return lam, X, passes
