"""Hubbard atomic forces and Hubbard stress tensor (Sec. II.A, the force and
stress sections) of the model DFT+U problem, as the paper writes them for the
finite-difference method: the derivatives are moved from the atomic orbitals
to the Kohn-Sham orbitals and taken with the centred finite-difference
gradient whose weights the paper prints (Sec. II.B, gradient weights).

TEST INFRASTRUCTURE ONLY (see the oracle package header).

With P_mj = <phi_m|psi_j> dV, G^a_mj = <phi_m|d_a psi_j> dV and the moment
projections Q^ab_mj = sum_T <phi_m(.-R-T) (x-R-T)_b e^{ik.T}|d_a psi_j> dV:

  force on Hubbard atom J (Eq. Force1 -> Eq. DerR -> final expression):
    f^J_a = g sum_k w_k sum_j f_j Re sum_mm' U (2 D_m'm - delta_mm') P_mj conj(G^a_m'j)
  stress (Eq. StressDef -> final expression), 1/|Omega| from the definition:
    sigma_ab = (g/|Omega|) sum_I sum_mm' U/2 (delta_mm' - 2 D_m'm)
               [ -2 sum_k w_k sum_j f_j Re(Q^ab_mj conj(P_m'j)) - delta_ab D_mm' ]
  (the printed expressions carry D_mm' in the first factor; for the real D
  of the Gamma point and of k-sets closed under k -> -k the two agree, and
  D_m'm is the exact derivative of E_U for complex D too)

g = 2 for a spin-unpolarised run (both spin channels carry the stored D,
as in E_U), 1 per channel otherwise; D is the occupation matrix of the given
orbitals and occupations (Eq. orbital_occup_ext).  The orbital shape moves
rigidly with its atom (Loewdin coefficients, when used, are constants of the
orbital), which is exact in the continuum where the overlap matrix does not
depend on the atom's position or on a homogeneous strain.

Pins (tests/test_oracle_forces.py): the printed gradient weights against the
moment conditions of a centred first derivative and the plane-wave / Bloch
symbol; summation by parts of the periodic gradient; the force against a
central difference of E_U under a displacement of each Hubbard atom, and
the stress against central differences of E_U under every component of a
homogeneous deformation, both at fixed Kohn-Sham orbitals, with smooth
(almost untruncated) orbitals where the finite-difference gradient is
accurate.
"""
from __future__ import annotations

import numpy as np

from . import fd
from .atoms import hubbard_functions, hubbard_radial, real_ylm, _images
from .scf import hubbard_energy, occupation_matrix


def gradient(X, L, n, n0, k, axis):
    """Centred finite-difference derivative along grid axis `axis` (0 = x)
    of the block X (ns, nd): sum_p w~_p (f(i+p) - f(i-p)), indices outside
    the cell mapped back with the Bloch factor (Sec. II.B)."""
    L = np.asarray(L, float)
    n = np.asarray(n)
    k = np.asarray(k, float)
    ns = X.shape[0]
    f = X.reshape(ns, n[2], n[1], n[0])
    assert n0 < n[axis], "the stencil must not wrap more than once"
    ax = f.ndim - 1 - axis
    w = fd.gradient_weights(n0, L[axis] / n[axis])
    cplx = bool(np.any(k != 0)) or np.iscomplexobj(X)
    phase = np.exp(1j * k[axis] * L[axis]) if np.any(k != 0) else 1.0
    out = np.zeros_like(f, dtype=complex if cplx else float)
    for p in range(1, n0 + 1):
        out = out + w[p - 1] * (fd._shift(f, p, ax, phase) - fd._shift(f, -p, ax, phase))
    return out.reshape(ns, -1)


def projections(cfg, X, k, funcs):
    """Per Hubbard atom: P (m, ns), G[a] (m, ns) and Q[a][b] (m, ns)."""
    dv = float(np.prod(np.asarray(cfg["L"]) / np.asarray(cfg["n"])))
    grads = [gradient(X, cfg["L"], cfg["n"], cfg["n0"], k, a) for a in range(3)]
    out = []
    for h in funcs:
        idx = h["idx"]
        P = dv * (h["vals"].conj() @ X[:, idx].T)
        G = [dv * (h["vals"].conj() @ g[:, idx].T) for g in grads]
        Q = [[dv * (h["moms"][b].conj() @ g[:, idx].T) for b in range(3)] for g in grads]
        out.append((P, G, Q))
    return out


def forces_and_stress(cfg, X_sk, f_sk, threshold=None):
    """Hubbard forces (natom, 3) and stress (3, 3) of the orbitals X_sk
    [spin][k] (ns, nd) with occupations f_sk [spin][k] (ns,), k-points and
    weights from cfg."""
    kpts = np.asarray(cfg["kpts"], float)
    kw = np.asarray(cfg["kw"], float)
    nspin = cfg["nspin"]
    g = 2.0 if nspin == 1 else 1.0
    omega = float(np.prod(np.asarray(cfg["L"], float)))
    funcs_k = [hubbard_functions(cfg, k, threshold) for k in kpts]
    nh = len(funcs_k[0])
    proj = [[projections(cfg, X_sk[s][ik], kpts[ik], funcs_k[ik]) for ik in range(len(kpts))]
            for s in range(nspin)]
    forces = np.zeros((len(cfg["atom_species"]), 3))
    stress = np.zeros((3, 3))
    for s in range(nspin):
        for h in range(nh):
            U = funcs_k[0][h]["U"]
            D = occupation_matrix([proj[s][ik][h][0] for ik in range(len(kpts))], f_sk[s], kw)
            m = D.shape[0]
            # dE_U/dD_mm' = U/2 (delta_mm' - 2 D_m'm): the printed expressions
            # carry D_mm', which equals D_m'm whenever D is real (Gamma, k-sets
            # closed under k -> -k); the transposed form is the exact derivative
            # for complex D as well (the same reading as for the potential)
            Dt = D.T
            W = U * (2.0 * Dt - np.eye(m))           # -2 dE_U/dD
            V = 0.5 * U * (np.eye(m) - 2.0 * Dt)     # dE_U/dD (Eq. DerED)
            atom = funcs_k[0][h]["atom"]
            for ik in range(len(kpts)):
                P, G, Q = proj[s][ik][h]
                fP = P * f_sk[s][ik][None, :]
                for a in range(3):
                    # sum_j f_j sum_mm' W_mm' P_mj conj(G^a_m'j)
                    forces[atom, a] += g * kw[ik] * float(np.real(np.sum(W * (fP @ G[a].conj().T))))
                    for b in range(3):
                        fQ = Q[a][b] * f_sk[s][ik][None, :]
                        stress[a, b] += g / omega * kw[ik] * (-2.0) * float(
                            np.real(np.sum(V * (fQ @ P.conj().T))))
            for a in range(3):
                stress[a, a] -= g / omega * float(np.real(np.sum(V * D)))
    return forces, stress


# ---------------------------------------------------------------- pins
def hubbard_energy_deformed(cfg, X_sk, f_sk, C_list, threshold, shift=None, F=None, only=None):
    """E_U of fixed orbitals X_sk / occupations f_sk with the Hubbard orbitals
    evaluated directly at moved atoms or in a deformed cell (the definition
    the force and stress formulas differentiate):
      shift = (J, a, eps): atom J moved by eps along axis a;
      F (3x3): homogeneous deformation x -> F x of grid, atoms and lattice,
      orbitals carried as psi(F x) = psi(x) / sqrt(det F) (norm kept), so
      P_m = sqrt(det F) dV sum_x conj(phi_m(F (x - R - T))) e^{-ik.T} psi(x).
    C_list: fixed Loewdin coefficients per Hubbard atom (rigid orbital shape).
    only: atom indices whose Hubbard term is summed (default all).
    Brute force over the images of each atom, no support lists."""
    from .atoms import truncation_radius
    L = np.asarray(cfg["L"], float)
    n = np.asarray(cfg["n"])
    kpts = np.asarray(cfg["kpts"], float)
    kw = np.asarray(cfg["kw"], float)
    dv = float(np.prod(L / n))
    Fm = np.eye(3) if F is None else np.asarray(F, float)
    scale = np.sqrt(np.linalg.det(Fm))
    x = fd.grid_coords(L, n)
    hub = [ia for ia, s in enumerate(cfg["atom_species"]) if cfg["species"][s]["hub_l"] >= 0]
    e = 0.0
    for h, ia in enumerate(hub):
        if only is not None and ia not in only:
            continue
        sp = cfg["species"][cfg["atom_species"][ia]]
        rad = (lambda r, sp=sp: hubbard_radial(r, sp["hub_power"], sp["hub_alpha"]))
        rc = truncation_radius(rad, threshold)
        R = np.asarray(cfg["pos"][ia], float).copy()
        if shift is not None and shift[0] == ia:
            R[shift[1]] += shift[2]
        reach = 1.05 * rc
        nim = _images(reach, L)
        phis = []
        for k in kpts:
            phi = np.zeros((2 * sp["hub_l"] + 1, x.shape[0]), complex)
            for t3 in range(-nim[2], nim[2] + 1):
                for t2 in range(-nim[1], nim[1] + 1):
                    for t1 in range(-nim[0], nim[0] + 1):
                        T = np.array([t1, t2, t3]) * L
                        c = R + T
                        gap = np.maximum(np.maximum(-c, c - L), 0.0)
                        if np.sqrt(np.sum(gap * gap)) > reach:
                            continue
                        d = (x - c) @ Fm.T
                        r = np.sqrt(np.sum(d * d, axis=1))
                        msk = r <= rc
                        if not np.any(msk):
                            continue
                        phi[:, msk] += rad(r[msk]) * real_ylm(sp["hub_l"], d[msk]) * np.exp(1j * np.dot(k, T))
            phis.append(C_list[h].T @ phi)
        D = [[occupation_matrix([scale * dv * (phis[ik].conj() @ X_sk[s][ik].T) for ik in range(len(kpts))],
                                f_sk[s], kw)] for s in range(cfg["nspin"])]
        e += hubbard_energy(D, [sp["hub_U"]], cfg["nspin"])
    return e
