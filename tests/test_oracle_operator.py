"""Pins of the oracle's operator H[D] (Sec. II.A potential section)."""
import numpy as np
import pytest

import workloads
from oracle import fd
from oracle.hamiltonian import Hamiltonian, hubbard_atoms
from oracle.scf import hubbard_energy, occupation_matrix

KPT = (0.18, -0.18, 0.28)


def _rand_D(nhub, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nhub):
        A = rng.normal(size=(5, 5)) * 0.1
        out.append(0.3 * np.eye(5) + 0.5 * (A + A.T))
    return out


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), KPT])
def test_dense_hermitian(k):
    cfg = workloads.make_config("tiny")
    H = Hamiltonian(cfg, k, _rand_D(2, 0)).dense()
    assert np.max(np.abs(H - H.conj().T)) < 1e-12 * np.max(np.abs(H))


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), KPT])
def test_kinetic_spectrum_closed_form(k):
    cfg = workloads.make_config("tiny")
    h = Hamiltonian(cfg, k, kb=False, hubbard=False, V=np.zeros(int(np.prod(cfg["n"]))))
    ev = np.linalg.eigvalsh(h.dense())
    n, L = cfg["n"], cfg["L"]
    th = [2 * np.pi * np.arange(n[a]) / n[a] + k[a] * L[a] / n[a] for a in range(3)]
    s = [fd.laplacian_symbol(th[a], L[a] / n[a], cfg["n0"]) for a in range(3)]
    want = np.sort((-0.5 * (s[0][None, None, :] + s[1][None, :, None] + s[2][:, None, None])).ravel())
    np.testing.assert_allclose(ev, want, atol=1e-10 * want.max())


def test_hubbard_special_cases():
    cfg = workloads.make_config("tiny")
    nd = int(np.prod(cfg["n"]))
    X = workloads.random_block(nd, 5, 9)
    h0 = Hamiltonian(cfg, hubbard=False)
    ref = h0.apply(X)
    # D = I/2 makes the Hubbard potential vanish
    h = Hamiltonian(cfg, D=[0.5 * np.eye(5)] * 2, atoms=h0.atoms, V=h0.V)
    np.testing.assert_allclose(h.apply(X), ref, atol=1e-13)
    # U = 0 likewise
    cfg2 = workloads.make_config("tiny")
    cfg2["species"][0]["hub_U"] = 0.0
    h2 = Hamiltonian(cfg2, D=_rand_D(2, 1))
    np.testing.assert_allclose(h2.apply(X), Hamiltonian(cfg2, hubbard=False).apply(X), atol=1e-13)
    # D = 0: V_U = (U/2) Phi Phi^H dV, a sum of projectors on Loewdin orbitals:
    # rank 5 per atom, every nonzero eigenvalue U/2 when atoms do not overlap
    # (here: trace = U/2 * 5 * nTi exactly).
    hz = Hamiltonian(cfg, D=[np.zeros((5, 5))] * 2, atoms=h0.atoms, V=h0.V)
    Vu = hz.dense() - h0.dense()
    assert abs(np.trace(Vu) - 0.5 * 0.147 * 10) < 1e-12


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), KPT])
def test_energy_gradient_is_operator(k):
    """For fixed occupations f, E(X) = g_s sum_j f_j <x_j|H0|x_j> dV + E_U(D(X))
    has directional derivative 2 Re g_s sum_j f_j <d_j|H[D(X)] x_j> dV.  Pins the
    Hubbard potential against the Hubbard energy (including the D_{mm'} vs
    D_{m'm} reading and every factor of 2)."""
    cfg = workloads.make_config("tiny")
    nd = int(np.prod(cfg["n"]))
    cplx = bool(np.any(np.asarray(k) != 0))
    X = workloads.random_block(nd, 6, 4, cplx) * 0.3
    Dl = workloads.random_block(nd, 6, 5, cplx)
    f = np.array([1.0, 0.9, 0.7, 0.5, 0.2, 0.05])
    h0 = Hamiltonian(cfg, k, hubbard=False)
    dv = h0.dv
    hub = hubbard_atoms(cfg)
    U = [0.147] * len(hub)
    hh = Hamiltonian(cfg, k, atoms=h0.atoms, V=h0.V)

    def energy(Z):
        e_band = 2.0 * dv * np.sum(f * np.real(np.sum(Z.conj() * h0.apply(Z), axis=1)))
        P = hh.project(Z)
        D = [occupation_matrix([p], [f], [1.0]) for p in P]
        return e_band + hubbard_energy([D], U, 1), D

    e0, D0 = energy(X)
    hh.set_occupation(D0)
    HX = hh.apply(X)
    want = 2.0 * 2.0 * dv * np.sum(f * np.real(np.sum(Dl.conj() * HX, axis=1)))
    eps = 1e-4
    ep, _ = energy(X + eps * Dl)
    em, _ = energy(X - eps * Dl)
    got = (ep - em) / (2 * eps)
    assert abs(got - want) < 1e-7 * abs(want)


def test_nonlocal_psd_rank():
    cfg = workloads.make_config("tiny")
    nd = int(np.prod(cfg["n"]))
    hk = Hamiltonian(cfg, hubbard=False, V=np.zeros(nd))
    hl = Hamiltonian(cfg, hubbard=False, kb=False, V=np.zeros(nd), atoms=hk.atoms)
    ev = np.linalg.eigvalsh(hk.dense() - hl.dense())
    assert ev.min() > -1e-12
    assert int(np.sum(ev > 1e-8)) == 4 * len(cfg["atom_species"])
