"""Pins of the oracle's density-dependent Hamiltonian and density + D
mixing (Sec. II.B).

The Hartree solve and the Kerker operator are checked by applying the
finite-difference Laplacian directly (an independent code path); the
exchange potential as the functional derivative of the exchange energy;
the SCF by its fixed point and by the stationarity of the free energy with
respect to the input density (a wrong sign or factor in any double-counting
term makes F change at first order).
"""
import numpy as np
import pytest

import workloads
from oracle import fd, hxc
from oracle.hamiltonian import Hamiltonian, hubbard_atoms
from oracle import scf as oscf


def _grid():
    L = np.array([8.7, 8.1, 5.6])
    n = np.array([14, 12, 10])
    return L, n, int(np.prod(n)), float(np.prod(L / n))


def test_hartree_solves_the_fd_poisson_equation():
    L, n, nd, dv = _grid()
    rho = np.random.default_rng(1).uniform(0.0, 0.3, nd)
    vh = hxc.hartree_potential(rho, L, n, 6)
    lap = fd.apply_laplacian(vh.reshape(n[2], n[1], n[0]), L, n, 6).ravel()
    np.testing.assert_allclose(-lap, 4 * np.pi * (rho - rho.mean()), atol=1e-11 * np.abs(rho).max() * 4 * np.pi)
    assert abs(vh.mean()) < 1e-13
    # a plane wave: V_H = 4 pi A / lambda cos(g x), lambda the stencil's symbol
    x = fd.grid_coords(L, n)
    g = 2 * np.pi * 2 / L[0]
    rho = 0.1 + 0.05 * np.cos(g * x[:, 0])
    lam = -fd.laplacian_symbol(g * L[0] / n[0], L[0] / n[0], 6)[0]
    np.testing.assert_allclose(hxc.hartree_potential(rho, L, n, 6), 4 * np.pi * 0.05 / lam * np.cos(g * x[:, 0]),
                               atol=1e-12)
    assert abs(hxc.hartree_energy(rho, hxc.hartree_potential(rho, L, n, 6), dv)
               - 0.5 * dv * np.sum(0.05 ** 2 * 4 * np.pi / lam * np.cos(g * x[:, 0]) ** 2)) < 1e-12


def test_exchange_potential_is_the_functional_derivative():
    L, n, nd, dv = _grid()
    rho = np.random.default_rng(2).uniform(0.01, 0.4, nd)
    v = hxc.exchange_potential(rho)
    for i in (0, 17, 500, nd - 1):
        e = 1e-5          # truncation ~e^2, rounding of the summed energy ~1e-9 relative
        rp, rm = rho.copy(), rho.copy()
        rp[i] += e
        rm[i] -= e
        d = (hxc.exchange_energy(rp, dv) - hxc.exchange_energy(rm, dv)) / (2 * e) / dv
        assert abs(d - v[i]) < 1e-7 * abs(v[i])
    # uniform density: E_x = -(3/4)(3/pi)^(1/3) rho^(4/3) Omega
    u = np.full(nd, 0.2)
    assert abs(hxc.exchange_energy(u, dv) + 0.75 * (3 / np.pi) ** (1 / 3) * 0.2 ** (4 / 3) * nd * dv) < 1e-12


def test_kerker_operator():
    L, n, nd, dv = _grid()
    r = np.random.default_rng(3).normal(size=nd)
    k0 = 0.8
    pr = hxc.kerker(r, L, n, 6, k0)
    # (-Delta_h + k0^2) P r = -Delta_h r, with the Laplacian applied directly
    lap = lambda f: fd.apply_laplacian(f.reshape(n[2], n[1], n[0]), L, n, 6).ravel()
    np.testing.assert_allclose(-lap(pr) + k0 * k0 * pr, -lap(r), atol=1e-10 * np.abs(lap(r)).max())
    assert abs(pr.mean()) < 1e-13


@pytest.fixture(scope="module")
def hxc_run():
    cfg = workloads.make_config("tiny")
    cfg["hxc"] = True
    return cfg, hxc.scf_hxc(cfg)


def _dense_F(cfg, rho_in, D_in):
    """Free energy of the model at input (rho, D) with exact eigenpairs."""
    L, n, n0 = cfg["L"], cfg["n"], cfg["n0"]
    from oracle.atoms import local_potential
    dv = float(np.prod(np.asarray(L) / np.asarray(n)))
    V = local_potential(cfg) + hxc.hartree_potential(rho_in, L, n, n0) + hxc.exchange_potential(rho_in)
    h = Hamiltonian(cfg, D=D_in, V=V)
    lam, Vec = np.linalg.eigh(h.dense())
    ns = cfg["ns"]
    lam, Vec = lam[:ns], Vec[:, :ns] / np.sqrt(dv)
    eigs = lam[None, None, :]
    mu = oscf.fermi_level(eigs, [1.0], cfg["nelec"], cfg["kT"], 2.0)
    f = oscf.occupations(eigs, mu, cfg["kT"])
    P = h.project(Vec.T)
    D_out = [oscf.occupation_matrix([p], [f[0, 0]], [1.0]) for p in P]
    rho_out = oscf.density([[Vec.T]], [[f[0, 0]]], [1.0], 1)[0]
    U = [cfg["species"][cfg["atom_species"][ia]]["hub_U"] for ia in hubbard_atoms(cfg)]
    E_U = oscf.hubbard_energy([D_out], U, 1)
    dc = 2.0 * sum(np.trace(M @ d) for M, d in zip(h.M, D_out))
    vh_out = hxc.hartree_potential(rho_out, L, n, n0)
    e_hxc = (-dv * np.dot(rho_out, V - local_potential(cfg)) + hxc.hartree_energy(rho_out, vh_out, dv)
             + hxc.exchange_energy(rho_out, dv))
    return 2.0 * np.sum(f * eigs) - dc + E_U - cfg["kT"] * oscf.entropy(f, [1.0], 2.0) + e_hxc, rho_out


def test_hxc_scf_fixed_point_and_stationarity(hxc_run):
    cfg, r = hxc_run
    assert r["converged"]
    dv = r["dv"]
    assert abs(dv * r["rho"].sum() - cfg["nelec"]) < 1e-9
    # the input density reproduces itself
    assert np.sqrt(dv * np.sum((r["rho"] - r["rho_in"]) ** 2)) / cfg["nelec"] < 1e-6
    # F is stationary in the input density at the fixed point
    F0, rho_out = _dense_F(cfg, r["rho_in"], r["D"][0])
    assert abs(F0 - r["F"]) / len(cfg["atom_species"]) < 1e-6
    x = fd.grid_coords(cfg["L"], cfg["n"])
    g = 2 * np.pi / np.asarray(cfg["L"])
    drho = 0.01 * np.cos(g[0] * x[:, 0] + 0.3) * np.cos(g[2] * x[:, 2])   # zero mean: N_e kept
    eps = 1e-2
    Fp, _ = _dense_F(cfg, r["rho_in"] + eps * drho, r["D"][0])
    Fm, _ = _dense_F(cfg, r["rho_in"] - eps * drho, r["D"][0])
    slope = (Fp - Fm) / (2 * eps)
    # scale of a non-stationary slope: the first-order change of the Hartree and
    # exchange energies alone (a doubled E_H gives ~1x this, V_x off by 10% ~0.1x)
    vh = hxc.hartree_potential(r["rho_in"], cfg["L"], cfg["n"], cfg["n0"])
    scale = abs(dv * np.dot(drho, vh)) + abs(dv * np.dot(drho, hxc.exchange_potential(r["rho_in"])))
    assert abs(slope) < 1e-3 * scale
