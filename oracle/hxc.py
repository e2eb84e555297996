"""Density-dependent Hamiltonian and the SCF that mixes the density and the
occupation matrices together (Sec. II.B: ground state by Chebyshev-filtered
subspace iteration accelerated by real-space preconditioned Pulay mixing;
the density's mixing coefficients are applied to the occupation matrices
as well).

TEST INFRASTRUCTURE ONLY (see the oracle package header).

    H[rho, D] = -1/2 Delta_h + V_loc + V_H[rho] + V_x[rho] + KB + V_U[D]

  * Hartree: -Delta_h V_H = 4 pi (rho - <rho>) with the same order-2n0
    finite-difference Laplacian as the kinetic term (the mean is removed: a
    uniform neutralising background); on the periodic grid the discrete
    operator is diagonal in plane waves, so the discrete equation is solved
    exactly by FFT with the stencil's symbol.  E_H = 1/2 int rho V_H.
  * Exchange: local density approximation, e_x(rho) = -(3/4)(3/pi)^(1/3)
    rho^(4/3), V_x = -(3 rho / pi)^(1/3) (spin-unpolarised runs).
  * Free energy (output densities, stationary at self-consistency):
        F = E_band - int rho_out (V_H + V_x)[rho_in] + E_H[rho_out] + E_x[rho_out]
            - sum Tr(M(D_in) D_out) + E_U(D_out) - kT S.
  * Mixing: Pulay on the density with coefficients fitted to the density
    residuals (dV-weighted), the residual step preconditioned by the Kerker
    operator P = (-Delta_h)(-Delta_h + k0^2)^-1 (applied exactly by FFT, same
    symbol); the same coefficients mix D (unpreconditioned).
  * Start: uniform density N_e / Omega.

Pins (tests/test_oracle_hxc.py): Hartree potential of plane waves and
-Delta_h V_H = 4 pi (rho - <rho>) with the finite-difference Laplacian
applied directly; V_x as the functional derivative of E_x (central
differences); the Kerker symbol; the self-consistent fixed point (density
and D reproduce themselves) and the stationarity of F under perturbations
of the input density.
"""
from __future__ import annotations

import numpy as np

from . import fd
from .atoms import atom_functions, local_potential
from .chfsi import chfsi_pass, lanczos
from .hamiltonian import Hamiltonian, hubbard_atoms
from .scf import (density, electron_count, entropy, fermi_level, hubbard_energy, initial_occupation,
                  occupation_matrix, occupations, start_blocks, d_to_vec, vec_to_d)


def laplacian_symbol_grid(L, n, n0):
    """lambda(G) >= 0 of -Delta_h on every plane wave of the grid, array of
    shape (n3, n2, n1) in numpy FFT order."""
    L = np.asarray(L, float)
    n = np.asarray(n)
    out = np.zeros((n[2], n[1], n[0]))
    for a in range(3):
        theta = 2 * np.pi * np.fft.fftfreq(n[a])          # m_a / n_a * 2 pi
        s = -fd.laplacian_symbol(theta, L[a] / n[a], n0)  # -(w0 + 2 sum_p w_p cos(p theta)) >= 0
        shape = [1, 1, 1]
        shape[2 - a] = n[a]
        out = out + s.reshape(shape)
    out[0, 0, 0] = 0.0          # the stencil's weights sum to zero; drop their rounding
    return out


def hartree_potential(rho, L, n, n0):
    """V_H with -Delta_h V_H = 4 pi (rho - mean rho), zero mean; rho (nd,)."""
    n = np.asarray(n)
    lam = laplacian_symbol_grid(L, n, n0)
    rh = np.fft.fftn(np.asarray(rho, float).reshape(n[2], n[1], n[0]))
    vh = np.zeros_like(rh)
    nz = lam > 0
    vh[nz] = 4 * np.pi * rh[nz] / lam[nz]
    return np.real(np.fft.ifftn(vh)).ravel()


def hartree_energy(rho, vh, dv):
    return 0.5 * dv * float(np.dot(rho, vh))


def exchange_energy(rho, dv):
    """Unpolarised LDA exchange: E_x = -(3/4)(3/pi)^(1/3) int rho^(4/3)."""
    r = np.maximum(np.asarray(rho, float), 0.0)
    return -0.75 * (3.0 / np.pi) ** (1.0 / 3.0) * dv * float(np.sum(r ** (4.0 / 3.0)))


def exchange_potential(rho):
    r = np.maximum(np.asarray(rho, float), 0.0)
    return -((3.0 / np.pi) * r) ** (1.0 / 3.0)


def kerker(r, L, n, n0, k0):
    """P r with P = (-Delta_h)(-Delta_h + k0^2)^-1 (G = 0 component removed)."""
    n = np.asarray(n)
    lam = laplacian_symbol_grid(L, n, n0)
    rh = np.fft.fftn(np.asarray(r, float).reshape(n[2], n[1], n[0]))
    return np.real(np.fft.ifftn(rh * lam / (lam + k0 * k0))).ravel()


def scf_hxc(cfg, max_iter=None, verbose=False):
    """Self-consistent loop with the density-dependent potential (nspin = 1).
    Returns eigenvalues, occupations, mu, D, density, energies, iterations of
    the last iteration; rho_next / V_next are the input density and potential
    that its mixing step produced (absent once converged)."""
    assert cfg["nspin"] == 1, "the density-dependent model is spin-unpolarised"
    kpts = np.asarray(cfg["kpts"])
    kw = np.asarray(cfg["kw"])
    gs = 2.0
    hub = hubbard_atoms(cfg)
    U = [cfg["species"][cfg["atom_species"][ia]]["hub_U"] for ia in hub]
    L, n, n0 = cfg["L"], cfg["n"], cfg["n0"]
    dv = float(np.prod(np.asarray(L) / np.asarray(n)))
    nd = int(np.prod(n))
    omega = float(np.prod(L))
    natom = len(cfg["atom_species"])
    Vloc = local_potential(cfg)
    atoms_k = [atom_functions(cfg, k) for k in kpts]
    D_in = initial_occupation(cfg)
    rho_in = np.full(nd, cfg["nelec"] / omega)
    X, v0 = start_blocks(cfg)
    k0 = cfg.get("kerker_k0", 0.8)
    beta = cfg["pulay_beta"]
    hist = cfg["pulay_history"]
    tol_rho = cfg.get("scf_tol_rho", 1e-6)

    def veff(rho):
        return Vloc + hartree_potential(rho, L, n, n0) + exchange_potential(rho)

    V = veff(rho_in)
    H = [Hamiltonian(cfg, kpts[ik], D_in[0], atoms_k[ik], V) for ik in range(len(kpts))]
    bounds = []
    for ik in range(len(kpts)):
        th_min, b = lanczos(H[ik].apply, v0[0][ik], cfg["lanczos_steps"])
        bounds.append((th_min + (b - th_min) / 10.0, b, th_min))
    xs, fs, ds, gds = [], [], [], []
    F_old = None
    converged = False
    out = {}
    for it in range(max_iter or cfg["max_iter"]):
        passes = cfg["first_passes"] if it == 0 else 1
        eigs = np.zeros((1, len(kpts), cfg["ns"]))
        for ik in range(len(kpts)):
            h = H[ik]
            for _ in range(passes):
                a, b, aL = bounds[ik]
                lam, X[0][ik] = chfsi_pass(h.apply, X[0][ik], cfg["degree"], (a, b, aL), dv)
                bounds[ik] = (lam[-1], b, lam[0])
            eigs[0, ik] = lam
        mu = fermi_level(eigs, kw, cfg["nelec"], cfg["kT"], gs)
        f = occupations(eigs, mu, cfg["kT"])
        P_k = [H[ik].project(X[0][ik]) for ik in range(len(kpts))]
        D_out = [[occupation_matrix([P_k[ik][i] for ik in range(len(kpts))], [f[0, ik] for ik in range(len(kpts))],
                                    kw) for i in range(len(hub))]]
        rho_out = density(X, [[f[0, ik] for ik in range(len(kpts))]], kw, 1)[0]
        E_U = hubbard_energy(D_out, U, 1)
        e_band = gs * float(np.sum(kw[None, :, None] * f * eigs))
        dc = 2.0 * sum(float(np.real(np.trace(H[0].M[i] @ D_out[0][i]))) for i in range(len(hub)))
        ts = cfg["kT"] * entropy(f, kw, gs)
        vh_in = V - Vloc - exchange_potential(rho_in)          # V_H[rho_in]
        vh_out = hartree_potential(rho_out, L, n, n0)
        e_hxc = (-dv * float(np.dot(rho_out, V - Vloc)) + hartree_energy(rho_out, vh_out, dv)
                 + exchange_energy(rho_out, dv))
        F = e_band - dc + E_U - ts + e_hxc
        res_rho = np.sqrt(dv * float(np.sum((rho_out - rho_in) ** 2))) / cfg["nelec"]
        res_d = float(np.sqrt(sum(np.sum(np.abs(o - i) ** 2) for o, i in zip(D_out[0], D_in[0]))))
        dF = abs(F - F_old) / natom if F_old is not None else np.inf
        if verbose:
            print(f"[oracle hxc] it={it} F={F:.12f} res_rho={res_rho:.3e} res_D={res_d:.3e} dF={dF:.3e}")
        F_old = F
        out = dict(eigs=eigs, occ=f, mu=mu, D=D_out, rho=rho_out, rho_in=rho_in, V=V, F=F, E_U=E_U,
                   e_band=e_band, e_hxc=e_hxc, E_H=hartree_energy(rho_out, vh_out, dv),
                   E_x=exchange_energy(rho_out, dv), iterations=it + 1, X=X, dv=dv, vh_in=vh_in)
        if res_rho < tol_rho and res_d < cfg["scf_tol_d"] and dF < cfg["scf_tol_f"]:
            converged = True
            break
        # Pulay: coefficients from the density residuals, applied to D too
        x_r, f_r = rho_in, rho_out - rho_in
        x_d, f_d = d_to_vec(D_in), d_to_vec(D_out) - d_to_vec(D_in)
        xs.append(x_r); fs.append(f_r); ds.append(x_d); gds.append(f_d)
        if len(xs) > hist + 1:
            xs.pop(0); fs.pop(0); ds.pop(0); gds.pop(0)
        if len(xs) == 1:
            gam = np.zeros(0)
        else:
            dF_r = np.stack([fs[i] - fs[i - 1] for i in range(1, len(fs))], axis=1)
            gam, *_ = np.linalg.lstsq(np.sqrt(dv) * dF_r, np.sqrt(dv) * f_r, rcond=None)
        dX_r = [xs[i] - xs[i - 1] for i in range(1, len(xs))]
        dF_rl = [fs[i] - fs[i - 1] for i in range(1, len(fs))]
        dX_d = [ds[i] - ds[i - 1] for i in range(1, len(ds))]
        dF_d = [gds[i] - gds[i - 1] for i in range(1, len(gds))]
        xr_bar = x_r - sum(g * v for g, v in zip(gam, dX_r))
        fr_bar = f_r - sum(g * v for g, v in zip(gam, dF_rl))
        xd_bar = x_d - sum(g * v for g, v in zip(gam, dX_d))
        fd_bar = f_d - sum(g * v for g, v in zip(gam, dF_d))
        rho_in = xr_bar + beta * kerker(fr_bar, L, n, n0, k0)
        rho_in = rho_in + (cfg["nelec"] / omega - np.mean(rho_in))   # the step keeps N_e exactly
        D_in = vec_to_d(xd_bar + beta * fd_bar, D_in)
        V = veff(rho_in)
        out["rho_next"], out["V_next"] = rho_in, V      # the input of the next iteration
        for ik in range(len(kpts)):
            H[ik] = Hamiltonian(cfg, kpts[ik], D_in[0], atoms_k[ik], V)
    out["converged"] = converged
    return out
