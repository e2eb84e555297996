"""Pins of the oracle's Hubbard forces and stress (Sec. II.A force and
stress sections; the gradient weights of Sec. II.B).

The force and stress formulas move the derivative from the atomic orbital to
the Kohn-Sham orbital and take it with the printed finite-difference weights.
They are pinned here against the definitions they come from: central
differences of E_U at fixed orbitals when a Hubbard atom moves (force =
-dE_U/dR) and when the cell deforms homogeneously (stress = dE_U/dF /
|Omega|), evaluated by brute force with the orbitals placed directly at the
moved/deformed positions.  Smooth Kohn-Sham orbitals (low Bloch waves) and
almost untruncated Hubbard orbitals (threshold 1e-9) make the
finite-difference gradient and the trapezoid rule accurate, so the two sides
agree to the discretisation level of the grid (the brute-force energy
carries the grid's egg-box error, which falls as about h^5: 8e-4, 2e-4,
6e-5, 2e-5 relative at h = 0.36, 0.27, 0.22, 0.18 bohr on this cell, while
the formula's value moves by less than 1e-4 relative); a wrong sign, a
dropped factor of 2, a missing -delta D term or a transposed occupation
matrix breaks that by orders of magnitude.  Bar: 5e-4 of the largest
component at h = 0.27 bohr.
"""
import numpy as np
import pytest

import workloads
from oracle import fd, forces
from oracle.atoms import hubbard_functions

THR = 1e-9


def test_gradient_weights_moment_conditions():
    """The printed weights w~_p are those of the order-2n0 centred first
    derivative: sum_p 2 p w~_p = 1/h and sum_p 2 p^(2q+1) w~_p = 0 for
    q = 1..n0-1 (the same conditions solved as a linear system)."""
    for n0 in (1, 2, 4, 6):
        h = 0.37
        w = fd.gradient_weights(n0, h)
        p = np.arange(1, n0 + 1)
        assert abs(np.sum(2 * p * w) - 1.0 / h) < 1e-12 / h
        for q in range(1, n0):
            assert abs(np.sum(2 * p ** (2 * q + 1) * w)) < 1e-9 * np.sum(np.abs(2 * p ** (2 * q + 1) * w))
        A = np.array([[2.0 * pp ** (2 * q + 1) for pp in p] for q in range(n0)])
        rhs = np.zeros(n0)
        rhs[0] = 1.0 / h
        np.testing.assert_allclose(np.linalg.solve(A, rhs), w, rtol=1e-10)


def test_gradient_plane_wave_and_bloch_symbol():
    """On a Bloch wave e^{i(g + k) x} the gradient is exactly
    i (2 sum_p w~_p sin(p theta)) times the wave, theta = (g + k) h; the
    wrap-around carries the Bloch factor."""
    L = np.array([8.7, 8.1, 5.6])
    n = np.array([18, 15, 12])
    k = np.array([0.21, -0.13, 0.37])
    x = fd.grid_coords(L, n)
    for a in range(3):
        g = 2 * np.pi * 2 / L[a]
        kv = np.zeros(3)
        kv[a] = g + k[a]
        f = np.exp(1j * (x @ kv))[None, :]
        got = forces.gradient(f, L, n, 6, k, a)
        h = L[a] / n[a]
        w = fd.gradient_weights(6, h)
        sym = 2 * np.sum(w * np.sin(np.arange(1, 7) * (g + k[a]) * h))
        np.testing.assert_allclose(got, 1j * sym * f, atol=1e-11 * abs(sym))


def test_gradient_summation_by_parts():
    """sum_x conj(d_h f) g = - sum_x conj(f) d_h g for Bloch functions (the
    step that moves the derivative between orbitals)."""
    rng = np.random.default_rng(3)
    L = np.array([8.7, 8.7, 5.6])
    n = np.array([14, 12, 10])
    k = np.array([0.3, -0.2, 0.1])
    nd = int(np.prod(n))
    f = rng.normal(size=(1, nd)) + 1j * rng.normal(size=(1, nd))
    g = rng.normal(size=(1, nd)) + 1j * rng.normal(size=(1, nd))
    for a in range(3):
        lhs = np.vdot(forces.gradient(f, L, n, 6, k, a), g)
        rhs = -np.vdot(f, forces.gradient(g, L, n, 6, k, a))
        assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def _smooth_setup(kset, nspin, seed):
    """Tiny cell on a 32x32x20 grid, 4 states per (spin, k) made of the
    lowest Bloch waves, random occupations."""
    cfg = workloads.make_config("tiny")
    cfg["n"] = np.array([32, 32, 20], np.int32)
    cfg["nspin"] = nspin
    cfg["kpts"] = np.array(kset, float)
    cfg["kw"] = np.full(len(kset), 1.0 / len(kset))
    L = np.asarray(cfg["L"])
    x = fd.grid_coords(L, cfg["n"])
    rng = np.random.default_rng(seed)
    ms = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    X_sk, f_sk = [], []
    for s in range(nspin):
        Xs, fs = [], []
        for k in cfg["kpts"]:
            gamma = not np.any(k != 0)
            cols = []
            for j in range(4):
                psi = np.zeros(x.shape[0], complex)
                for m in ms:
                    G = 2 * np.pi * np.array(m) / L + k
                    psi += (rng.normal() + 1j * rng.normal()) * np.exp(1j * (x @ G))
                cols.append(np.real(psi) if gamma else psi)
            Xs.append(np.array(cols))
            fs.append(rng.uniform(0.05, 0.95, 4))
        X_sk.append(Xs)
        f_sk.append(fs)
    return cfg, X_sk, f_sk


CASES = {
    "gamma-unpolarised": ([[0.0, 0.0, 0.0]], 1, 11),
    "k-point-polarised": ([[0.17, -0.11, 0.23]], 2, 12),
}


@pytest.mark.parametrize("case", list(CASES))
def test_forces_are_minus_energy_derivative(case):
    cfg, X_sk, f_sk = _smooth_setup(*CASES[case])
    F, _ = forces.forces_and_stress(cfg, X_sk, f_sk, threshold=THR)
    C = [h["C"] for h in hubbard_functions(cfg, cfg["kpts"][0], THR)]
    eps = 1e-3
    hub = [ia for ia, s in enumerate(cfg["atom_species"]) if s == 0]
    scale = np.max(np.abs(F[hub]))
    assert scale > 1e-3
    for ia in hub:
        for a in range(3):
            ep = forces.hubbard_energy_deformed(cfg, X_sk, f_sk, C, THR, shift=(ia, a, eps), only=[ia])
            em = forces.hubbard_energy_deformed(cfg, X_sk, f_sk, C, THR, shift=(ia, a, -eps), only=[ia])
            fd_force = -(ep - em) / (2 * eps)
            assert abs(F[ia, a] - fd_force) < 5e-4 * scale, (ia, a, F[ia, a], fd_force)
    # atoms without a Hubbard manifold carry no Hubbard force
    assert np.all(F[[ia for ia in range(len(cfg["atom_species"])) if ia not in hub]] == 0)


@pytest.mark.parametrize("case", list(CASES))
def test_stress_is_energy_derivative_over_volume(case):
    cfg, X_sk, f_sk = _smooth_setup(*CASES[case])
    _, S = forces.forces_and_stress(cfg, X_sk, f_sk, threshold=THR)
    C = [h["C"] for h in hubbard_functions(cfg, cfg["kpts"][0], THR)]
    omega = float(np.prod(cfg["L"]))
    eps = 1e-4
    scale = np.max(np.abs(S))
    for a in range(3):
        for b in range(3):
            Fp = np.eye(3)
            Fp[a, b] += eps
            Fm = np.eye(3)
            Fm[a, b] -= eps
            ep = forces.hubbard_energy_deformed(cfg, X_sk, f_sk, C, THR, F=Fp)
            em = forces.hubbard_energy_deformed(cfg, X_sk, f_sk, C, THR, F=Fm)
            fd_s = (ep - em) / (2 * eps) / omega
            assert abs(S[a, b] - fd_s) < 5e-4 * scale, (a, b, S[a, b], fd_s)
