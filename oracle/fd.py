"""Finite differences on the uniform periodic grid (Sec. II.B).

TEST INFRASTRUCTURE ONLY (see the oracle package header).

The paper discretises derivatives with centred finite differences of order
2*n0 on a uniform grid with spacings h_a = L_a / n_a, maps indices that fall
outside the grid back periodically with the Bloch factor, and integrates with
the trapezoidal rule (Sec. II.B, gradient-stencil, weight and quadrature
equations).  It prints the gradient weights but not the Laplacian weights; the
Laplacian here uses the standard centred second-derivative weights of the same
order, which share the gradient's binomial factor.

Pins (tests/test_oracle_fd.py): moment conditions solved independently as a
linear system, Fornberg's recursive algorithm, the closed-form plane-wave
symbol, the dense kinetic spectrum.
"""
from __future__ import annotations

from math import factorial

import numpy as np


def _binom_factor(n0, p):
    return factorial(n0) ** 2 / (factorial(n0 - p) * factorial(n0 + p))


def gradient_weights(n0, h):
    """Centred first-derivative weights w~_p, p = 1..n0 (Sec. II.B, the
    gradient weight equation): (-1)^(p+1) / (h p) * (n0!)^2 / ((n0-p)!(n0+p)!)."""
    return np.array([(-1) ** (p + 1) / (h * p) * _binom_factor(n0, p)
                     for p in range(1, n0 + 1)])


def laplacian_weights(n0, h):
    """Centred second-derivative weights of order 2*n0 for one axis.

    Returns (w0, w) with w[p-1] the weight of f(i+p) and of f(i-p):
        w_p = 2 (-1)^(p+1) / (h^2 p^2) * (n0!)^2 / ((n0-p)!(n0+p)!)
        w0  = -(2 / h^2) * sum_p 1/p^2
    """
    w = np.array([2.0 * (-1) ** (p + 1) / (h * h * p * p) * _binom_factor(n0, p)
                  for p in range(1, n0 + 1)])
    w0 = -2.0 / (h * h) * sum(1.0 / (p * p) for p in range(1, n0 + 1))
    return w0, w


def _shift(f, p, axis, phase):
    """g[i] = f[i + p] along `axis` (grid axis of a (..., n3, n2, n1) array),
    with the Bloch factor applied to values that wrapped around the cell:
    e^{+i k L} past the upper end (p > 0), e^{-i k L} past the lower end."""
    g = np.roll(f, -p, axis=axis)
    if phase != 1.0:
        n = f.shape[axis]
        idx = [slice(None)] * f.ndim
        if p > 0:
            idx[axis] = slice(n - p, n)
            g[tuple(idx)] = g[tuple(idx)] * phase
        elif p < 0:
            idx[axis] = slice(0, -p)
            g[tuple(idx)] = g[tuple(idx)] / phase
    return g


def apply_laplacian(f, L, n, n0, k=(0.0, 0.0, 0.0)):
    """Delta_h f for f of shape (..., n3, n2, n1) (x fastest).

    Each axis a contributes w0_a f_i + sum_p w_{p,a} (f_{i+p e_a} + f_{i-p e_a});
    indices outside [0, n_a) wrap with the Bloch factor e^{+-i k_a L_a}.
    """
    L = np.asarray(L, float)
    n = np.asarray(n)
    k = np.asarray(k, float)
    cplx = np.any(k != 0.0)
    out = np.zeros_like(f, dtype=complex if (cplx or np.iscomplexobj(f)) else float)
    for a in range(3):
        axis = f.ndim - 1 - a          # x is the last axis
        h = L[a] / n[a]
        w0, w = laplacian_weights(n0, h)
        phase = np.exp(1j * k[a] * L[a]) if cplx else 1.0
        out = out + w0 * f
        for p in range(1, n0 + 1):
            out = out + w[p - 1] * (_shift(f, p, axis, phase) + _shift(f, -p, axis, phase))
    return out


def laplacian_symbol(theta, h, n0):
    """Eigenvalue of the 1-D stencil on e^{i theta j}: w0 + 2 sum_p w_p cos(p theta)."""
    w0, w = laplacian_weights(n0, h)
    p = np.arange(1, n0 + 1)
    return w0 + 2.0 * np.sum(w[:, None] * np.cos(np.outer(p, np.atleast_1d(theta))), axis=0)


def integrate(f, L, n):
    """Trapezoidal rule on the periodic grid: h1 h2 h3 * sum f (orthorhombic)."""
    dv = float(np.prod(np.asarray(L, float) / np.asarray(n)))
    return dv * np.sum(f)


def grid_coords(L, n):
    """Cartesian coordinates of all grid nodes, shape (nd, 3), linear index
    i + n1*(j + n2*k), node (i h1, j h2, k h3)."""
    L = np.asarray(L, float)
    n = np.asarray(n)
    h = L / n
    kk, jj, ii = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    return np.stack([ii.ravel() * h[0], jj.ravel() * h[1], kk.ravel() * h[2]], axis=1)
