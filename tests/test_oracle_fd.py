"""Pins of the oracle's finite differences and quadrature (Sec. II.B)
against facts that do not come from the oracle itself."""
import numpy as np
import pytest

import workloads
from oracle import fd
from oracle.atoms import local_potential


def fornberg(x0, nodes, order):
    """Fornberg (1988) recursive weights for derivatives 0..order at x0 -
    an algorithm independent of the closed forms under test."""
    n = len(nodes)
    c = np.zeros((order + 1, n))
    c1 = 1.0
    c4 = nodes[0] - x0
    c[0, 0] = 1.0
    for i in range(1, n):
        mn = min(i, order)
        c2 = 1.0
        c5 = c4
        c4 = nodes[i] - x0
        for j in range(i):
            c3 = nodes[i] - nodes[j]
            c2 *= c3
            if j == i - 1:
                for k in range(mn, 0, -1):
                    c[k, i] = c1 * (k * c[k - 1, i - 1] - c5 * c[k, i - 1]) / c2
                c[0, i] = -c1 * c5 * c[0, i - 1] / c2
            for k in range(mn, 0, -1):
                c[k, j] = (c4 * c[k, j] - k * c[k - 1, j]) / c3
            c[0, j] = c4 * c[0, j] / c3
        c1 = c2
    return c


@pytest.mark.parametrize("n0", [1, 2, 4, 6])
@pytest.mark.parametrize("h", [1.0, 0.24167])
def test_laplacian_weights_match_fornberg(n0, h):
    nodes = np.arange(-n0, n0 + 1) * h
    c = fornberg(0.0, nodes, 2)
    w0, w = fd.laplacian_weights(n0, h)
    assert abs(c[2, n0] - w0) <= 1e-11 * abs(w0)
    for p in range(1, n0 + 1):
        assert abs(c[2, n0 + p] - w[p - 1]) <= 1e-11 * abs(w0)
        assert abs(c[2, n0 - p] - w[p - 1]) <= 1e-11 * abs(w0)


@pytest.mark.parametrize("n0", [1, 3, 6])
def test_paper_gradient_weights_match_fornberg(n0):
    """The printed gradient weights (Sec. II.B) equal the centred first-
    derivative weights of order 2*n0."""
    h = 0.7
    c = fornberg(0.0, np.arange(-n0, n0 + 1) * h, 1)
    wt = fd.gradient_weights(n0, h)
    for p in range(1, n0 + 1):
        assert abs(c[1, n0 + p] - wt[p - 1]) < 1e-12 / h
        assert abs(c[1, n0 - p] + wt[p - 1]) < 1e-12 / h


def test_laplacian_moment_system():
    """Weights solve the moment conditions of a 2nd derivative exact for
    polynomials of degree <= 2*n0 + 1 (solved here as a linear system)."""
    n0, h = 6, 1.0
    A = np.zeros((n0 + 1, n0 + 1))
    rhs = np.zeros(n0 + 1)
    A[0, 0] = 1.0
    A[0, 1:] = 2.0
    for j in range(1, n0 + 1):
        A[j, 1:] = 2.0 * np.arange(1, n0 + 1, dtype=float) ** (2 * j)
    rhs[1] = 2.0
    sol = np.linalg.solve(A, rhs)
    w0, w = fd.laplacian_weights(n0, h)
    np.testing.assert_allclose(sol[0], w0, rtol=1e-10)
    np.testing.assert_allclose(sol[1:], w, rtol=1e-8, atol=1e-12)


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.31, -0.17, 0.4)])
def test_laplacian_plane_wave_symbol(k):
    """Plane waves e^{i(g+k).x} are eigenvectors of the periodic/Bloch stencil
    with eigenvalue sum_a [w0 + 2 sum_p w_p cos(p theta_a)]."""
    L = np.array([3.1, 2.7, 2.3])
    n = np.array([10, 8, 7])
    n0 = 6
    x = fd.grid_coords(L, n)
    rng = np.random.default_rng(3)
    for _ in range(4):
        m = rng.integers(-4, 5, size=3)
        g = 2 * np.pi * m / L + np.asarray(k)
        wave = np.exp(1j * x @ g).reshape(n[2], n[1], n[0])
        lap = fd.apply_laplacian(wave, L, n, n0, k)
        lam = sum(fd.laplacian_symbol(2 * np.pi * m[a] / n[a] + k[a] * L[a] / n[a], L[a] / n[a], n0)[0]
                  for a in range(3))
        np.testing.assert_allclose(lap, lam * wave, rtol=0, atol=1e-10 * abs(lam) + 1e-12)


def test_symbol_consistency_order():
    """Symbol approaches -theta^2/h^2 with a 14th-power leading error."""
    h = 0.25
    for th in (0.05, 0.1, 0.2):
        s = fd.laplacian_symbol(th, h, 6)[0]
        err = abs(s + th * th / (h * h))
        assert err < 1e-3 * th ** 14 / h ** 2 + 1e-9


def test_trapezoid_integrates_periodic_gaussians():
    """Trapezoid quadrature of the periodic Gaussian sum equals its exact
    integral -D * natom * (2 pi s^2)^{3/2} (spectral accuracy)."""
    cfg = workloads.make_config("c1")
    V = local_potential(cfg)
    exact = -2.0 * len(cfg["atom_species"]) * (2 * np.pi) ** 1.5
    got = fd.integrate(V, cfg["L"], cfg["n"])
    assert abs(got - exact) < 1e-9 * abs(exact)
