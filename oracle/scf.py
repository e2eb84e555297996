"""Occupations, Hubbard occupation matrices, E_U, density, free energy,
Pulay mixing and the SCF loop of the model DFT+U problem.

TEST INFRASTRUCTURE ONLY (see the oracle package header).

  * Occupations: Fermi-Dirac f = 1/(1 + e^{(lam - mu)/kT}), one Fermi level
    for all spins and k-points, found by bisection on
    g_s sum_sigma sum_k w_k sum_j f = N_e (g_s = 2 spin-unpolarised, 1 spin-
    polarised).  The paper writes occupations f_j(k) and a Brillouin-zone
    average (Eq. orbital_occup_ext) without naming the smearing.
  * Occupation matrix (Eq. orbital_occup_ext): (D_I)_{mm'} =
    sum_k w_k sum_j f_j <psi_j|phi_m'> <phi_m|psi_j>, i.e. D = P F P^H with
    P = Phi^H X dV (Hermitian, size 2l+1).
  * Hubbard energy (Eq. E_U): E_U = sum_sigma sum_I U/2 Tr(D - D^2); in a
    spin-unpolarised run both spin channels hold the same D.
  * Free energy: F = g_s sum w f lam - sum_sigma sum_I Tr(M_I(D_in) D_out)
    + E_U(D_out) - kT S, S = -g_s sum w [f ln f + (1-f) ln(1-f)].
  * Mixing (Sec. II.B): Pulay (Anderson) mixing of the occupation matrices,
    history h, parameter beta; D is updated every SCF iteration.
  * Initial D: diagonal, the isolated-atom average occupation (Sec. II.B).

Pins: sum f = N_e, closed-form Fermi levels, D invariants (symmetry,
spectrum in [0, 1] with Loewdin orbitals, trace = projected charge), E_U >= 0
and its diagonal closed form, Pulay on linear fixed-point problems, SCF
fixed-point and stationarity checks (tests/test_oracle_scf.py).
The SCF fixed point itself is parity unpinned beyond these invariants: the
paper's printed energies are for pseudopotentials not available here.
"""
from __future__ import annotations

import time

import numpy as np
from scipy.special import expit

import workloads
from .atoms import atom_functions, local_potential
from .chfsi import chfsi_pass, lanczos
from .hamiltonian import Hamiltonian, hubbard_atoms


def occupations(eigs, mu, kT):
    return expit(-(np.asarray(eigs) - mu) / kT)


def electron_count(eigs, kw, mu, kT, gs):
    """g_s sum_sigma sum_k w_k sum_j f(lam_j); eigs shape (nspin, nk, ns)."""
    f = occupations(eigs, mu, kT)
    return gs * float(np.sum(np.asarray(kw)[None, :, None] * f))


def fermi_level(eigs, kw, nelec, kT, gs, max_iter=200):
    """Bisection on the electron count, bracket [lam_min - 1, lam_max + 1],
    run until the bracket stops shrinking."""
    eigs = np.asarray(eigs)
    lo, hi = float(eigs.min()) - 1.0, float(eigs.max()) + 1.0
    for _ in range(max_iter):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if electron_count(eigs, kw, mid, kT, gs) < nelec:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def entropy(f, kw, gs):
    """S = -g_s sum w [f ln f + (1-f) ln(1-f)], with 0 ln 0 = 0."""
    f = np.asarray(f)
    t = np.zeros_like(f)
    m = (f > 0) & (f < 1)
    t[m] = f[m] * np.log(f[m]) + (1 - f[m]) * np.log(1 - f[m])
    return -gs * float(np.sum(np.asarray(kw)[None, :, None] * t))


def occupation_matrix(P_list_k, f_k, kw):
    """D = sum_k w_k P F P^H for one atom; P_list_k[k] has shape (m, ns)."""
    D = 0
    for P, f, w in zip(P_list_k, f_k, kw):
        D = D + w * ((P * f[None, :]) @ P.conj().T)
    D = 0.5 * (D + np.conj(np.transpose(D)))
    return D


def hubbard_energy(D, U, nspin):
    """E_U = sum_sigma sum_I U_I/2 Tr(D - D^2); D[sigma][I] matrices.
    nspin = 1 counts the single stored channel twice."""
    e = 0.0
    for Ds in D:
        for d, u in zip(Ds, U):
            e += 0.5 * u * float(np.real(np.trace(d - d @ d)))
    return e * (2.0 if nspin == 1 else 1.0)


def density(X_sk, f_sk, kw, nspin):
    """rho[sigma](x) = (2/nspin) sum_k w_k sum_j f_j |x_j(x)|^2 (total density
    for nspin = 1, spin densities for nspin = 2)."""
    gs = 2.0 if nspin == 1 else 1.0
    out = []
    for s in range(nspin):
        r = 0.0
        for X, f, w in zip(X_sk[s], f_sk[s], kw):
            r = r + w * np.sum(f[:, None] * np.abs(X) ** 2, axis=0)
        out.append(gs * r)
    return np.array(out)


# ---------------------------------------------------------------- mixing
def d_to_vec(D):
    """Upper triangles (row-major, including the diagonal) of every D[sigma][I]
    concatenated; the real part, then the imaginary part if D is complex."""
    v = []
    for Ds in D:
        for d in Ds:
            iu = np.triu_indices(d.shape[0])
            v.append(np.real(d[iu]))
    vec = np.concatenate(v)
    if any(np.iscomplexobj(d) for Ds in D for d in Ds):
        vi = [np.imag(d[np.triu_indices(d.shape[0])]) for Ds in D for d in Ds]
        vec = np.concatenate([vec, np.concatenate(vi)])
    return vec


def vec_to_d(vec, like):
    out = []
    pos = 0
    cplx = any(np.iscomplexobj(d) for Ds in like for d in Ds)
    nreal = sum(d.shape[0] * (d.shape[0] + 1) // 2 for Ds in like for d in Ds)
    for Ds in like:
        row = []
        for d in Ds:
            m = d.shape[0]
            iu = np.triu_indices(m)
            cnt = m * (m + 1) // 2
            up = np.zeros((m, m), dtype=complex if cplx else float)
            up[iu] = vec[pos:pos + cnt]
            if cplx:
                up[iu] += 1j * vec[nreal + pos:nreal + pos + cnt]
            full = up + np.conj(up.T) - np.diag(np.diag(up).real if cplx else np.diag(up))
            if cplx:
                full[np.diag_indices(m)] = np.real(np.diag(up))
            row.append(full)
            pos += cnt
        out.append(row)
    return out


class Pulay:
    """Pulay/Anderson mixing: with residual f = x_out - x_in and the last h
    differences dX, dF, gamma = argmin |f_n - dF gamma|, and
    x_next = (x_n - dX gamma) + beta (f_n - dF gamma)."""

    def __init__(self, history=7, beta=0.3):
        self.h = history
        self.beta = beta
        self.xs, self.fs = [], []

    def step(self, x_in, f):
        self.xs.append(np.array(x_in, float))
        self.fs.append(np.array(f, float))
        if len(self.xs) > self.h + 1:
            self.xs.pop(0)
            self.fs.pop(0)
        if len(self.xs) == 1:
            return x_in + self.beta * f
        dX = np.stack([self.xs[i] - self.xs[i - 1] for i in range(1, len(self.xs))], axis=1)
        dF = np.stack([self.fs[i] - self.fs[i - 1] for i in range(1, len(self.fs))], axis=1)
        g, *_ = np.linalg.lstsq(dF, f, rcond=None)
        xbar = x_in - dX @ g
        fbar = f - dF @ g
        return xbar + self.beta * fbar


# ---------------------------------------------------------------- SCF
def initial_occupation(cfg):
    """Diagonal isolated-atom guess (Sec. II.B); complex Hermitian storage
    when any k-point is not Gamma (D is then complex in general)."""
    hub = hubbard_atoms(cfg)
    cplx = bool(np.any(np.asarray(cfg["kpts"]) != 0))
    D = []
    for s in range(cfg["nspin"]):
        diag = workloads.initial_occupation_diag(cfg, s)
        D.append([g * np.eye(2 * cfg["species"][cfg["atom_species"][ia]]["hub_l"] + 1,
                             dtype=complex if cplx else float)
                  for g, ia in zip(diag, hub)])
    return D


def start_blocks(cfg):
    nd = int(np.prod(cfg["n"]))
    X, v0 = [], []
    for s in range(cfg["nspin"]):
        Xs, vs = [], []
        for ik, k in enumerate(cfg["kpts"]):
            cplx = bool(np.any(np.asarray(k) != 0))
            Xs.append(workloads.random_block(nd, cfg["ns"], workloads.start_seed(cfg, s, ik), cplx))
            vs.append(workloads.random_vector(nd, workloads.lanczos_seed(cfg, s, ik), cplx))
        X.append(Xs)
        v0.append(vs)
    return X, v0


def scf(cfg, D0=None, max_iter=None, verbose=False, fixed_iterations=None):
    """Self-consistent loop.  Returns a dict with eigenvalues (nspin, nk, ns),
    occupations, mu, D (list [sigma][I]), E_U, F, density, iterations,
    converged flag and the per-iteration history."""
    nspin = cfg["nspin"]
    kpts = np.asarray(cfg["kpts"])
    kw = np.asarray(cfg["kw"])
    gs = 2.0 if nspin == 1 else 1.0
    hub = hubbard_atoms(cfg)
    U = [cfg["species"][cfg["atom_species"][ia]]["hub_U"] for ia in hub]
    dv = float(np.prod(np.asarray(cfg["L"]) / np.asarray(cfg["n"])))
    V = local_potential(cfg)
    atoms_k = [atom_functions(cfg, k) for k in kpts]
    D_in = D0 if D0 is not None else initial_occupation(cfg)
    X, v0 = start_blocks(cfg)
    H = [[Hamiltonian(cfg, kpts[ik], D_in[s], atoms_k[ik], V) for ik in range(len(kpts))]
         for s in range(nspin)]
    bounds = [[None] * len(kpts) for _ in range(nspin)]
    for s in range(nspin):
        for ik in range(len(kpts)):
            th_min, b = lanczos(H[s][ik].apply, v0[s][ik], cfg["lanczos_steps"])
            bounds[s][ik] = (th_min + (b - th_min) / 10.0, b, th_min)
    mixer = Pulay(cfg["pulay_history"], cfg["pulay_beta"])
    max_iter = max_iter or cfg["max_iter"]
    hist = []
    F_old = None
    converged = False
    natom = len(cfg["atom_species"])
    for it in range(max_iter):
        passes = cfg["first_passes"] if it == 0 else 1
        eigs = np.zeros((nspin, len(kpts), cfg["ns"]))
        t0 = time.perf_counter()
        for s in range(nspin):
            for ik in range(len(kpts)):
                h = H[s][ik]
                h.set_occupation(D_in[s])
                for _ in range(passes):
                    a, b, aL = bounds[s][ik]
                    lam, X[s][ik] = chfsi_pass(h.apply, X[s][ik], cfg["degree"], (a, b, aL), dv)
                    bounds[s][ik] = (lam[-1], b, lam[0])
                eigs[s, ik] = lam
        mu = fermi_level(eigs, kw, cfg["nelec"], cfg["kT"], gs)
        f = occupations(eigs, mu, cfg["kT"])
        D_out = []
        for s in range(nspin):
            P_k = [H[s][ik].project(X[s][ik]) for ik in range(len(kpts))]
            D_out.append([occupation_matrix([P_k[ik][i] for ik in range(len(kpts))],
                                            [f[s, ik] for ik in range(len(kpts))], kw)
                          for i in range(len(hub))])
        E_U = hubbard_energy(D_out, U, nspin)
        e_band = gs * float(np.sum(kw[None, :, None] * f * eigs))
        dc = 0.0
        for s in range(nspin):
            for i in range(len(hub)):
                dc += float(np.real(np.trace(H[s][0].M[i] @ D_out[s][i])))
        dc *= (2.0 if nspin == 1 else 1.0)
        ts = cfg["kT"] * entropy(f, kw, gs)
        F = e_band - dc + E_U - ts
        x_in, x_out = d_to_vec(D_in), d_to_vec(D_out)
        res = float(np.sqrt(sum(np.sum(np.abs(o - i) ** 2) for Ds_o, Ds_i in zip(D_out, D_in)
                                for o, i in zip(Ds_o, Ds_i))))
        dF = abs(F - F_old) / natom if F_old is not None else np.inf
        hist.append(dict(it=it, F=F, E_U=E_U, mu=mu, res=res, dF=dF,
                         sec=time.perf_counter() - t0))
        if verbose:
            print(f"[oracle scf] it={it} F={F:.12f} E_U={E_U:.3e} res={res:.3e} dF={dF:.3e}")
        F_old = F
        if fixed_iterations is None and res < cfg["scf_tol_d"] and dF < cfg["scf_tol_f"]:
            converged = True
            D_final = D_out
            break
        D_final = D_out
        if fixed_iterations is not None and it + 1 >= fixed_iterations:
            break
        x_next = mixer.step(x_in, x_out - x_in)
        D_in = vec_to_d(x_next, D_in)
    f_sk = [[f[s, ik] for ik in range(len(kpts))] for s in range(nspin)]
    rho = density(X, f_sk, kw, nspin)
    return dict(eigs=eigs, occ=f, mu=mu, D=D_final, D_in=D_in, E_U=E_U, F=F,
                e_band=e_band, ts=ts, rho=rho, iterations=it + 1,
                converged=converged, history=hist, X=X, dv=dv)
