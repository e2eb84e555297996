"""The discrete Kohn-Sham operator of the model DFT+U problem.

TEST INFRASTRUCTURE ONLY (see the oracle package header).

    H[D] x = -1/2 Delta_h x + V_loc x
             + sum_I chi_I Gamma_I (chi_I^H x dV)             (nonlocal, KB)
             + sum_{I in U} Phi_I M_I (Phi_I^H x dV)          (Hubbard)
    M_I = U_I (1/2 I - D_I)

The Hubbard term is the potential of the Dudarev energy (Sec. II.A potential
section): the derivative of E_U with respect to the occupation matrix is
U/2 (delta - 2 D) (Eq. DerED) and the occupation matrix is the orbital
projection of the density matrix, D = Phi^H rho Phi, so V_U = Phi M Phi^H.
The printed potential carries D_{mm'} where this derivation gives D_{m'm};
the two agree whenever D is real (Gamma point, or k-sets closed under
k -> -k).  Projections are computed atom by atom on each atom's compact
support, as the paper does for nonlocal projectors (Sec. II.B).

Pins: Hermiticity of the assembled matrix, the plane-wave kinetic spectrum,
special cases of V_U (D = I/2, U = 0), and the finite-difference gradient of
the total energy (tests/test_oracle_operator.py).
"""
from __future__ import annotations

import numpy as np

from . import fd
from .atoms import atom_functions, local_potential


def hubbard_atoms(cfg):
    """Indices of atoms that carry a Hubbard manifold, in atom order."""
    return [ia for ia, s in enumerate(cfg["atom_species"]) if cfg["species"][s]["hub_l"] >= 0]


class Hamiltonian:
    """H[D] for one spin channel and one k-point."""

    def __init__(self, cfg, k=(0.0, 0.0, 0.0), D=None, atoms=None, V=None,
                 kb=True, hubbard=True):
        self.cfg = cfg
        self.L = np.asarray(cfg["L"], float)
        self.n = np.asarray(cfg["n"])
        self.nd = int(np.prod(self.n))
        self.dv = float(np.prod(self.L / self.n))
        self.k = np.asarray(k, float)
        self.cplx = bool(np.any(self.k != 0))
        self.atoms = atoms if atoms is not None else atom_functions(cfg, self.k)
        self.V = V if V is not None else local_potential(cfg)
        self.use_kb = kb
        self.use_hub = hubbard
        self.hub = hubbard_atoms(cfg)
        self.set_occupation(D)

    def set_occupation(self, D):
        """D: list (one per Hubbard atom) of (2l+1)x(2l+1) occupation matrices."""
        if D is None:
            D = [np.zeros((5, 5)) for _ in self.hub]
        self.D = [np.asarray(d) for d in D]
        self.M = []
        for ia, d in zip(self.hub, self.D):
            U = self.atoms[ia]["hub_U"]
            self.M.append(U * (0.5 * np.eye(d.shape[0]) - d))

    def project(self, X, which="hub"):
        """P_I = Phi_I^H X dV for every Hubbard atom (list of (m, ns))."""
        X = np.atleast_2d(X)
        out = []
        for ia in self.hub:
            a = self.atoms[ia]
            out.append(self.dv * (a["hub_vals"].conj() @ X[:, a["hub_idx"]].T))
        return out

    def apply_local(self, X):
        X = np.atleast_2d(X)
        ns = X.shape[0]
        f = X.reshape(ns, self.n[2], self.n[1], self.n[0])
        Y = -0.5 * fd.apply_laplacian(f, self.L, self.n, self.cfg["n0"], self.k).reshape(ns, self.nd)
        return Y + self.V[None, :] * X

    def apply(self, X):
        """Y = H[D] X for X of shape (ns, nd) (or (nd,))."""
        single = X.ndim == 1
        X = np.atleast_2d(X)
        Y = self.apply_local(X)
        if self.cplx or np.iscomplexobj(X):
            Y = Y.astype(complex)
        if self.use_kb:
            for a in self.atoms:
                idx, v = a["kb_idx"], a["kb_vals"]
                P = self.dv * (v.conj() @ X[:, idx].T)
                Y[:, idx] += (v.T @ (a["kb_gamma"][:, None] * P)).T
        if self.use_hub:
            for ia, M in zip(self.hub, self.M):
                a = self.atoms[ia]
                idx, v = a["hub_idx"], a["hub_vals"]
                P = self.dv * (v.conj() @ X[:, idx].T)
                Y[:, idx] += (v.T @ (M @ P)).T
        return Y[0] if single else Y

    def dense(self):
        """Assembled nd x nd matrix (tiny grids only)."""
        dt = complex if self.cplx else float
        eye = np.eye(self.nd, dtype=dt)
        Hm = self.apply(eye)       # row j = H e_j, i.e. H^T
        return np.ascontiguousarray(Hm.T)
