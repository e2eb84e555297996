"""Pins of the oracle's Chebyshev-filtered subspace iteration."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev

import workloads
from oracle import chfsi, fd
from oracle.hamiltonian import Hamiltonian


def test_filter_is_scaled_chebyshev_on_plane_waves():
    cfg = workloads.make_config("tiny")
    n, L = cfg["n"], cfg["L"]
    nd = int(np.prod(n))
    h = Hamiltonian(cfg, kb=False, hubbard=False, V=np.zeros(nd))
    x = fd.grid_coords(L, n)
    ms = [(0, 0, 0), (1, 0, 0), (2, -1, 1), (3, 3, -2), (5, 4, 3)]
    X = np.stack([np.exp(1j * x @ (2 * np.pi * np.array(m) / L)) for m in ms])
    eps = np.real(np.sum(X.conj() * h.apply(X), axis=1) / np.sum(np.abs(X) ** 2, axis=1))
    a, b, aL, m = 2.0, 190.0, 0.0, 9
    Y = chfsi.cheb_filter(h.apply, X, m, a, b, aL)
    e, c = (b - a) / 2, (b + a) / 2
    Tm = np.zeros(m + 1)
    Tm[m] = 1.0
    p = chebyshev.chebval((eps - c) / e, Tm) / chebyshev.chebval((aL - c) / e, Tm)
    np.testing.assert_allclose(Y, p[:, None] * X, rtol=1e-9, atol=1e-12)


def test_lanczos_bounds_enclose_spectrum():
    cfg = workloads.make_config("tiny")
    h = Hamiltonian(cfg, D=[0.2 * np.eye(5)] * 2)
    ev = np.linalg.eigvalsh(h.dense())
    th_min, b = chfsi.lanczos(h.apply, workloads.random_vector(h.nd, 7), 10)
    assert b >= ev[-1]
    assert th_min >= ev[0] - 1e-12


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.18, -0.18, 0.28)])
def test_chfsi_matches_dense_eigh(k):
    """Converged ChFSI Ritz values equal LAPACK eigenvalues of the assembled
    operator (fixed D) to 1e-8 Ha."""
    cfg = workloads.make_config("tiny")
    cplx = bool(np.any(np.asarray(k) != 0))
    h = Hamiltonian(cfg, k, D=[0.2 * np.eye(5), 0.3 * np.eye(5)])
    ev = np.linalg.eigvalsh(h.dense())
    ns = 24
    X0 = workloads.random_block(h.nd, ns, 1, cplx)
    lam, X, it = chfsi.eigensolve(h.apply, X0, 16, workloads.random_vector(h.nd, 2, cplx),
                                  10, h.dv, 200, tol=1e-12)
    nconv = 16
    np.testing.assert_allclose(lam[:nconv], ev[:nconv], atol=1e-8)
    G = h.dv * (X.conj() @ X.T)
    np.testing.assert_allclose(G, np.eye(ns), atol=1e-10)


def test_rayleigh_ritz_exact_on_eigenbasis():
    cfg = workloads.make_config("tiny")
    h = Hamiltonian(cfg)
    ev, V = np.linalg.eigh(h.dense())
    rng = np.random.default_rng(0)
    B = V[:, :8] @ rng.normal(size=(8, 8))          # mixed basis of an invariant subspace
    lam, X = chfsi.rayleigh_ritz(h.apply, B.T.copy(), h.dv)
    np.testing.assert_allclose(lam, ev[:8], atol=1e-10)
