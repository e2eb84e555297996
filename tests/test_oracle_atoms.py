"""Pins of the oracle's atom-centred functions and local potential."""
import numpy as np
import pytest
from scipy import integrate, special

import workloads
from oracle import atoms, fd


def _real_from_complex(l, m, theta, phi):
    """Real spherical harmonic from scipy's complex ones (Condon-Shortley
    phase included in scipy): sqrt2 (-1)^m Re Y_l^m for m > 0,
    sqrt2 (-1)^m Im Y_l^|m| for m < 0."""
    if m == 0:
        return special.sph_harm_y(l, 0, theta, phi).real
    y = special.sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return np.sqrt(2) * (-1) ** m * y.real
    return np.sqrt(2) * (-1) ** m * y.imag


@pytest.mark.parametrize("l", [0, 1, 2])
def test_real_ylm_against_scipy(l):
    rng = np.random.default_rng(0)
    d = rng.normal(size=(200, 3)) * rng.uniform(0.1, 5, size=(200, 1))
    r = np.linalg.norm(d, axis=1)
    theta = np.arccos(d[:, 2] / r)
    phi = np.arctan2(d[:, 1], d[:, 0])
    got = atoms.real_ylm(l, d)
    for i, m in enumerate(range(-l, l + 1)):
        np.testing.assert_allclose(got[i], _real_from_complex(l, m, theta, phi), atol=1e-13)


def test_real_ylm_orthonormal_on_sphere():
    xg, wg = np.polynomial.legendre.leggauss(24)
    nphi = 48
    phi = 2 * np.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=-1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).ravel()
    Y = np.concatenate([atoms.real_ylm(l, d) for l in range(3)], axis=0)
    G = (Y * w) @ Y.T
    np.testing.assert_allclose(G, np.eye(9), atol=1e-13)


def test_radial_normalisation():
    for p, a in [(2, 1.5), (1, 0.7)]:
        v, _ = integrate.quad(lambda r: (atoms.hubbard_radial(r, p, a) * r) ** 2, 0, np.inf)
        assert abs(v - 1) < 1e-10
    for l in (0, 1):
        v, _ = integrate.quad(lambda r: (atoms.kb_radial(r, l, 1.0) * r) ** 2, 0, np.inf)
        assert abs(v - 1) < 1e-10


def test_truncation_radius_is_outermost_crossing():
    sp = workloads.species_table()[0]
    kb, hub = atoms.species_radii(sp)
    f = lambda r: atoms.hubbard_radial(r, 2, 1.5)  # noqa: E731
    assert abs(f(hub) - 5e-3) < 1e-14
    rr = np.linspace(hub + 1e-9, 60, 20000)
    assert np.all(f(rr) < 5e-3)
    for l, rc in zip(sp["kb_l"], kb):
        g = lambda r: atoms.kb_radial(r, l, 1.0)  # noqa: E731
        assert abs(g(rc) - 5e-3) < 1e-14
        assert np.all(g(np.linspace(rc + 1e-9, 30, 5000)) < 5e-3)


def test_local_potential_poisson_summation():
    cfg = workloads.make_config("tiny")
    V = atoms.local_potential(cfg)
    x = fd.grid_coords(cfg["L"], cfg["n"])
    sel = np.random.default_rng(1).choice(len(V), 60, replace=False)
    Vf = atoms.local_potential_fourier(cfg, x[sel])
    np.testing.assert_allclose(V[sel], Vf, atol=1e-11)


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.18, -0.18, 0.28)])
def test_bloch_periodicity(k):
    cfg = workloads.make_config("tiny")
    L = cfg["L"]
    R = cfg["pos"][0]
    pts = np.random.default_rng(2).uniform(0, 1, size=(50, 3)) * L
    f = lambda p: atoms.bloch_function_at(p, R, L, k, lambda r: atoms.hubbard_radial(r, 2, 1.5), 2, 6.37)  # noqa
    base = f(pts)
    for a in range(3):
        sh = np.zeros(3)
        sh[a] = L[a]
        np.testing.assert_allclose(f(pts + sh), np.exp(1j * k[a] * L[a]) * base, atol=1e-13)


def test_support_indices_brute_force():
    cfg = workloads.make_config("tiny")
    L, n = cfg["L"], cfg["n"]
    x = fd.grid_coords(L, n)
    R = cfg["pos"][2]
    rc = 3.69
    idx = atoms.support_indices(R, L, n, rc)
    d = x - R
    d = d - np.round(d / L) * L          # minimum image (rc < L/2 fails here, so check all images)
    best = np.full(len(x), np.inf)
    for t in np.array(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1])).reshape(3, -1).T:
        best = np.minimum(best, np.linalg.norm(x - R - t * L, axis=1))
    want = np.nonzero(best <= rc)[0]
    np.testing.assert_array_equal(idx, want)


def test_lowdin_orthonormal_and_isolated_norm():
    # large cell, one Hubbard atom: before Loewdin the grid Gram is ~I up to
    # truncation and discretisation; after it, exactly I.
    cfg = workloads.make_config("tiny")
    cfg["L"] = np.array([16.0, 16.0, 16.0])
    cfg["n"] = np.array([64, 64, 64])
    cfg["atom_species"] = np.array([0], np.int32)
    cfg["pos"] = np.array([[7.9, 8.1, 8.0]])
    cfg["lowdin"] = False
    a = atoms.atom_functions(cfg)[0]
    dv = float(np.prod(cfg["L"] / cfg["n"]))
    G = dv * a["hub_vals"] @ a["hub_vals"].T
    np.testing.assert_allclose(G, np.eye(5), atol=2e-3)
    v = atoms.lowdin(a["hub_vals"], dv)
    np.testing.assert_allclose(dv * v @ v.T, np.eye(5), atol=1e-12)
