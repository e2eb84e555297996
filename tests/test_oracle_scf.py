"""Pins of the oracle's occupations, occupation matrices, E_U, mixing and
SCF (Sec. II.A energy section, Sec. II.B SCF description)."""
import numpy as np
import pytest

import workloads
from oracle import scf
from oracle.hamiltonian import Hamiltonian, hubbard_atoms


def test_fermi_two_level_closed_form():
    # two non-degenerate levels, one electron, g_s = 1: mu is the midpoint
    eigs = np.array([[[0.1, 0.5]]])
    mu = scf.fermi_level(eigs, [1.0], 1.0, 0.1, 1.0)
    assert abs(mu - 0.3) < 1e-12
    # degenerate level half filled: mu equals the level
    eigs = np.array([[[0.2, 0.2, 0.2, 0.2]]])
    mu = scf.fermi_level(eigs, [1.0], 2.0, 0.003, 1.0)
    assert abs(mu - 0.2) < 1e-12


def test_fermi_count_and_entropy():
    rng = np.random.default_rng(0)
    eigs = np.sort(rng.uniform(-1, 1, size=(2, 3, 20)), axis=-1)
    kw = np.array([0.25, 0.25, 0.5])
    mu = scf.fermi_level(eigs, kw, 13.0, 0.05, 1.0)
    assert abs(scf.electron_count(eigs, kw, mu, 0.05, 1.0) - 13.0) < 1e-12
    # entropy of f = 1/2 is ln 2 per state
    f = np.full((1, 1, 4), 0.5)
    assert abs(scf.entropy(f, [1.0], 2.0) - 8 * np.log(2)) < 1e-14


def test_pulay_solves_linear_fixed_point():
    """On x = A x + b the Pulay/Anderson iteration with history >= dim reaches
    the exact fixed point (it is then equivalent to GMRES)."""
    rng = np.random.default_rng(1)
    dim = 6
    Q, _ = np.linalg.qr(rng.normal(size=(dim, dim)))
    A = Q @ np.diag(rng.uniform(-0.8, 0.8, dim)) @ Q.T
    b = rng.normal(size=dim)
    xstar = np.linalg.solve(np.eye(dim) - A, b)
    mix = scf.Pulay(history=7, beta=0.3)
    x = np.zeros(dim)
    for _ in range(dim + 2):
        x = mix.step(x, A @ x + b - x)
    assert np.linalg.norm(x - xstar) < 1e-9 * np.linalg.norm(xstar)


def test_d_vec_roundtrip():
    rng = np.random.default_rng(2)
    A = rng.normal(size=(5, 5))
    D = [[A + A.T, np.eye(5)], [np.zeros((5, 5)), 2 * np.eye(5)]]
    back = scf.vec_to_d(scf.d_to_vec(D), D)
    for s in range(2):
        for i in range(2):
            np.testing.assert_allclose(back[s][i], D[s][i])


@pytest.fixture(scope="module")
def tiny_run():
    cfg = workloads.make_config("tiny")
    return cfg, scf.scf(cfg)


def test_scf_converges_and_invariants(tiny_run):
    cfg, r = tiny_run
    assert r["converged"]
    assert abs(np.sum(r["rho"]) * r["dv"] - cfg["nelec"]) < 1e-9
    assert np.all(r["rho"] > -1e-14)
    gs = 2.0
    assert abs(scf.electron_count(r["eigs"], cfg["kw"], r["mu"], cfg["kT"], gs) - cfg["nelec"]) < 1e-10
    E = 0.0
    h = Hamiltonian(cfg, D=r["D"][0])
    P = h.project(r["X"][0][0])
    for d, p in zip(r["D"][0], P):
        assert np.max(np.abs(d - d.T)) < 1e-14
        lam = np.linalg.eigvalsh(d)
        assert lam.min() > -1e-12 and lam.max() < 1 + 1e-12
        # trace = projected charge
        assert abs(np.trace(d) - np.sum(r["occ"][0, 0] * np.sum(p ** 2, axis=0))) < 1e-12
        E += 0.147 * np.sum(lam * (1 - lam))            # 2 spins x U/2
    assert abs(E - r["E_U"]) < 1e-12
    assert r["E_U"] >= 0


def test_diagonal_e_u_closed_form():
    d = np.diag([0.1, 0.5, 0.9, 0.0, 1.0])
    e = scf.hubbard_energy([[d]], [0.2], 2)
    assert abs(e - 0.1 * (0.09 + 0.25 + 0.09)) < 1e-15


def _dense_F(cfg, D_in):
    """Free energy functional of D_in with exact (dense) eigenpairs."""
    h = Hamiltonian(cfg, D=D_in)
    lam, V = np.linalg.eigh(h.dense())
    ns = cfg["ns"]
    lam, V = lam[:ns], V[:, :ns] / np.sqrt(h.dv)
    eigs = lam[None, None, :]
    mu = scf.fermi_level(eigs, [1.0], cfg["nelec"], cfg["kT"], 2.0)
    f = scf.occupations(eigs, mu, cfg["kT"])
    P = h.project(V.T)
    D_out = [scf.occupation_matrix([p], [f[0, 0]], [1.0]) for p in P]
    E_U = scf.hubbard_energy([D_out], [0.147] * len(P), 1)
    dc = 2.0 * sum(np.trace(M @ d) for M, d in zip(h.M, D_out))
    F = 2.0 * np.sum(f * eigs) - dc + E_U - cfg["kT"] * scf.entropy(f, [1.0], 2.0)
    return F, D_out


def test_free_energy_stationary_at_fixed_point(tiny_run):
    """At the self-consistent D the free energy, as a function of D_in, is
    stationary: its first-order change vanishes (a wrong sign or factor in
    the double-counting term breaks this)."""
    cfg, r = tiny_run
    D = r["D"][0]
    F0, D_out = _dense_F(cfg, D)
    # the dense and ChFSI fixed points agree
    for a, b in zip(D_out, D):
        assert np.max(np.abs(a - b)) < 1e-6
    rng = np.random.default_rng(3)
    dirs = []
    for _ in D:
        A = rng.normal(size=(5, 5))
        dirs.append(0.5 * (A + A.T))
    eps = 1e-3
    Fp, _ = _dense_F(cfg, [d + eps * x for d, x in zip(D, dirs)])
    Fm, _ = _dense_F(cfg, [d - eps * x for d, x in zip(D, dirs)])
    slope = (Fp - Fm) / (2 * eps)
    # scale of a non-stationary slope: derivative of the band energy alone
    band_slope = abs(sum(np.trace(-0.147 * x @ d) for x, d in zip(dirs, D))) * 2
    assert abs(slope) < 1e-4 * band_slope


def test_d_vec_roundtrip_complex_hermitian():
    """Complex (Bloch) occupation matrices: the upper-triangle vector keeps
    the real and imaginary parts, and mapping back rebuilds the Hermitian
    matrix.  A wrong conjugation of the lower triangle, or an imaginary part
    left on the diagonal, breaks the round trip or the Hermiticity."""
    rng = np.random.default_rng(5)
    D = []
    for s in range(2):
        row = []
        for m in (5, 3):
            A = rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m))
            row.append(0.5 * (A + A.conj().T))
        D.append(row)
    v = scf.d_to_vec(D)
    nreal = 2 * (15 + 6)
    assert v.shape == (2 * nreal,)            # real parts, then imaginary parts
    back = scf.vec_to_d(v, D)
    for s in range(2):
        for i in range(2):
            np.testing.assert_allclose(back[s][i], D[s][i], atol=1e-15)
            assert np.max(np.abs(back[s][i] - back[s][i].conj().T)) == 0.0
            assert np.all(np.imag(np.diag(back[s][i])) == 0.0)
    # the map is linear: mixing two matrices through the vector equals mixing
    # the matrices
    E = [[1j * (x - x.conj().T) / 2 + (x + x.conj().T) / 2 for x in row] for row in D]
    w = scf.vec_to_d(0.3 * scf.d_to_vec(D) + 0.7 * scf.d_to_vec(E), D)
    for s in range(2):
        for i in range(2):
            np.testing.assert_allclose(w[s][i], 0.3 * D[s][i] + 0.7 * E[s][i], atol=1e-14)


def test_pulay_history_truncation():
    """With history h only the last h + 1 (x, f) pairs enter a step: a mixer
    fed a long sequence gives the same step as a fresh mixer fed just the last
    h + 1 pairs (dropping the oldest pair, not the newest, and dropping at
    all, are both checked); on a contractive linear map whose dimension
    exceeds the history the truncated iteration still reaches the fixed
    point."""
    rng = np.random.default_rng(7)
    dim, h = 9, 3
    xs = [rng.normal(size=dim) for _ in range(12)]
    fs = [rng.normal(size=dim) for _ in range(12)]
    long_mix = scf.Pulay(history=h, beta=0.3)
    for x, f in zip(xs, fs):
        out_long = long_mix.step(x, f)
    short_mix = scf.Pulay(history=h, beta=0.3)
    for x, f in zip(xs[-(h + 1):], fs[-(h + 1):]):
        out_short = short_mix.step(x, f)
    np.testing.assert_allclose(out_long, out_short, rtol=1e-13, atol=1e-13)
    full_mix = scf.Pulay(history=50, beta=0.3)
    for x, f in zip(xs, fs):
        out_full = full_mix.step(x, f)
    assert np.max(np.abs(out_full - out_long)) > 1e-6
    Q, _ = np.linalg.qr(rng.normal(size=(dim, dim)))
    A = Q @ np.diag(rng.uniform(-0.7, 0.7, dim)) @ Q.T
    b = rng.normal(size=dim)
    xstar = np.linalg.solve(np.eye(dim) - A, b)
    mix = scf.Pulay(history=h, beta=0.3)
    x = np.zeros(dim)
    for _ in range(60):
        x = mix.step(x, A @ x + b - x)
    assert np.linalg.norm(x - xstar) < 1e-9 * np.linalg.norm(xstar)


def test_spin_polarised_density_integrates_to_electron_count():
    """nspin = 2: each spin density carries g_s = 1, and the two integrate
    (trapezoid rule) to N_e with the Fermi level found with g_s = 1; with
    the unpolarised factor 2 they would give 2 N_e."""
    rng = np.random.default_rng(9)
    nd, ns, dv, nelec = 300, 12, 0.01, 9.0
    kw = np.array([0.25, 0.75])
    X_sk, eigs = [], np.zeros((2, 2, ns))
    for s in range(2):
        row = []
        for k in range(2):
            Q, _ = np.linalg.qr(rng.normal(size=(nd, ns)) + 1j * rng.normal(size=(nd, ns)))
            row.append(Q.T / np.sqrt(dv))           # dV sum |x|^2 = 1, orthogonal
            eigs[s, k] = np.sort(rng.uniform(-1, 1, ns))
        X_sk.append(row)
    mu = scf.fermi_level(eigs, kw, nelec, 0.05, 1.0)
    f = scf.occupations(eigs, mu, 0.05)
    rho = scf.density(X_sk, [[f[s, k] for k in range(2)] for s in range(2)], kw, 2)
    assert rho.shape == (2, nd)
    assert abs(dv * rho.sum() - nelec) < 1e-10
    for s in range(2):
        assert abs(dv * rho[s].sum() - float(np.sum(kw[:, None] * f[s]))) < 1e-10
