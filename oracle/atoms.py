"""Atom-centred functions and the local potential (Sec. II.A energy section:
the Bloch-mapped atomic orbitals; Sec. II.B: orbitals built from real
spherical harmonics and radial functions, truncated by a value threshold and
not stored beyond it, and handled like nonlocal projectors).

TEST INFRASTRUCTURE ONLY (see the oracle package header).

Synthetic stand-ins replace the paper's pseudopotential data:
  * Hubbard radial function (l = 2): R(r) = N r^p e^{-alpha r}, normalised to
    int R^2 r^2 dr = 1;
  * Kleinman-Bylander radial functions (l <= 1): chi_l(r) = N_l r^l e^{-r^2/(2w^2)},
    normalised the same way;
  * local potential: V(x) = -D sum_I sum_T exp(-|x - R_I - T|^2 / (2 s^2)).
Truncation radius: outermost r at which the normalised radial function equals
the threshold (the paper fixes 5e-3 bohr^-3/2 as sufficient, Sec. III.A).
Bloch mapping: phi(x) = sum_T R(|x-R-T|) Y_lm(x-R-T) e^{+i k.T}, so that
phi(x + L) = e^{i k.L} phi(x), consistent with the Bloch boundary condition
used for the orbitals.
Optional Loewdin step (the paper is silent on orbital orthonormality on the
grid): Phi_I <- Phi_I O_I^{-1/2} with O_I = Phi_I^H Phi_I dV.

Pins (tests/test_oracle_atoms.py): real Y_lm against scipy's complex
spherical harmonics, radial normalisation by quadrature, threshold crossing,
Poisson-summation closed form of the periodic Gaussian sum, Bloch
periodicity, Loewdin orthonormality.
"""
from __future__ import annotations

from math import gamma, pi, sqrt, factorial

import numpy as np
from scipy.optimize import brentq

from . import fd


# ---------------------------------------------------------------- Y_lm
def real_ylm(l, d):
    """Real spherical harmonics for l <= 2, order m = -l..l; d has shape
    (N, 3) (displacements).  Returns shape (2l+1, N).  Value 0 at r = 0 for
    l > 0.

    l = 1: sqrt(3/4pi) * (y, z, x)/r
    l = 2: sqrt(15/4pi) xy, sqrt(15/4pi) yz, sqrt(5/16pi)(3z^2 - r^2),
           sqrt(15/4pi) xz, sqrt(15/16pi)(x^2 - y^2), all over r^2.
    """
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    r2 = x * x + y * y + z * z
    if l == 0:
        return np.full((1, d.shape[0]), 1.0 / sqrt(4 * pi))
    safe = np.where(r2 > 0, r2, 1.0)
    if l == 1:
        r = np.sqrt(safe)
        c = sqrt(3.0 / (4 * pi))
        out = np.stack([c * y / r, c * z / r, c * x / r])
    elif l == 2:
        c1 = sqrt(15.0 / (4 * pi))
        c0 = sqrt(5.0 / (16 * pi))
        c2 = sqrt(15.0 / (16 * pi))
        out = np.stack([c1 * x * y, c1 * y * z, c0 * (3 * z * z - r2), c1 * x * z,
                        c2 * (x * x - y * y)]) / safe
    else:
        raise ValueError("l <= 2 only")
    out[:, r2 == 0] = 0.0
    return out


# ---------------------------------------------------------------- radials
def hubbard_norm(power, alpha):
    """N such that int_0^inf (N r^p e^{-alpha r})^2 r^2 dr = 1."""
    return sqrt((2 * alpha) ** (2 * power + 3) / factorial(2 * power + 2))


def kb_norm(l, width):
    """N_l such that int_0^inf (N r^l e^{-r^2/(2w^2)})^2 r^2 dr = 1."""
    return sqrt(2.0 / (gamma(l + 1.5) * width ** (2 * l + 3)))


def hubbard_radial(r, power, alpha):
    return hubbard_norm(power, alpha) * r ** power * np.exp(-alpha * r)


def kb_radial(r, l, width):
    return kb_norm(l, width) * r ** l * np.exp(-r * r / (2 * width * width))


def truncation_radius(fun, threshold, r_max=60.0, step=1e-3):
    """Outermost r at which fun(r) equals `threshold`: scan inward from r_max
    to the first sample at or above it, then refine with Brent's method."""
    r = r_max
    while r > 0 and fun(r) < threshold:
        r -= step
    if r <= 0:
        raise ValueError("function never reaches the threshold")
    return brentq(lambda s: fun(s) - threshold, r, r + step, xtol=1e-15, rtol=1e-15)


def species_radii(sp):
    """Truncation radii of one species: (kb radii per channel, hubbard radius)."""
    kb = [truncation_radius(lambda r, l=l: kb_radial(r, l, sp["kb_width"]), sp["threshold"])
          for l in sp["kb_l"]]
    hub = None
    if sp["hub_l"] >= 0:
        hub = truncation_radius(lambda r: hubbard_radial(r, sp["hub_power"], sp["hub_alpha"]),
                                sp["threshold"])
    return kb, hub


# ---------------------------------------------------------------- Bloch sums
def _images(rc, L):
    return [int(np.ceil(rc / L[a])) + 1 for a in range(3)]


def _box_indices(c, rc, L, n):
    """Grid nodes (no wrap) inside the axis-aligned box [c - rc, c + rc]:
    returns linear indices and displacements x - c, or None if empty."""
    h = L / n
    rng = []
    for a in range(3):
        lo = max(int(np.ceil((c[a] - rc) / h[a])), 0)
        hi = min(int(np.floor((c[a] + rc) / h[a])), n[a] - 1)
        if lo > hi:
            return None
        rng.append(np.arange(lo, hi + 1))
    kk, jj, ii = np.meshgrid(rng[2], rng[1], rng[0], indexing="ij")
    d = np.stack([ii.ravel() * h[0] - c[0], jj.ravel() * h[1] - c[1], kk.ravel() * h[2] - c[2]], axis=1)
    lin = ii.ravel() + n[0] * (jj.ravel() + n[1] * kk.ravel())
    return lin, d


def bloch_function_at(points, center, L, k, radial, l, rc, moment=None):
    """Bloch-mapped atom-centred functions at arbitrary points.

    Returns (2l+1, N) values of sum_T radial(|x-c-T|) Y_lm(x-c-T) e^{i k.T},
    with the radial factor zero beyond rc.  With moment = b (0, 1, 2) every
    image term is multiplied by its own displacement component (x-c-T)_b
    (the moment functions of the stress expression).
    """
    L = np.asarray(L, float)
    k = np.asarray(k, float)
    cplx = np.any(k != 0)
    out = np.zeros((2 * l + 1, points.shape[0]), dtype=complex if cplx else float)
    nim = _images(rc, L)
    lo, hi = points.min(axis=0), points.max(axis=0)
    for t3 in range(-nim[2], nim[2] + 1):
        for t2 in range(-nim[1], nim[1] + 1):
            for t1 in range(-nim[0], nim[0] + 1):
                T = np.array([t1, t2, t3]) * L
                c = center + T
                # skip images whose sphere misses the points' bounding box
                gap = np.maximum(np.maximum(lo - c, c - hi), 0.0)
                if np.sqrt(np.sum(gap * gap)) > rc:
                    continue
                d = points - c
                r = np.sqrt(np.sum(d * d, axis=1))
                m = r <= rc
                if not np.any(m):
                    continue
                val = radial(r[m]) * real_ylm(l, d[m])
                if moment is not None:
                    val = val * d[m][:, moment][None, :]
                if cplx:
                    val = val * np.exp(1j * np.dot(k, T))
                out[:, m] += val
    return out


def support_indices(center, L, n, rc):
    """Sorted linear indices of grid nodes within rc of any periodic image of
    `center` (the atom's compact support)."""
    L = np.asarray(L, float)
    n = np.asarray(n)
    parts = []
    nim = _images(rc, L)
    for t3 in range(-nim[2], nim[2] + 1):
        for t2 in range(-nim[1], nim[1] + 1):
            for t1 in range(-nim[0], nim[0] + 1):
                box = _box_indices(center + np.array([t1, t2, t3]) * L, rc, L, n)
                if box is None:
                    continue
                lin, d = box
                parts.append(lin[np.sqrt(np.sum(d * d, axis=1)) <= rc])
    if not parts:
        return np.zeros(0, np.int64)
    return np.unique(np.concatenate(parts)).astype(np.int64)


def atom_functions(cfg, k=(0.0, 0.0, 0.0)):
    """Per-atom projector data on the grid for one k-point.

    Returns a list (one entry per atom) of dicts:
      kb_idx   : support indices (sphere of the largest KB radius)
      kb_vals  : (n_kb, nsupp) channel values (each channel truncated at its
                 own radius), channel order l = 0, then l = 1 (m = -1, 0, 1)
      kb_gamma : (n_kb,) channel energies
      hub_idx, hub_vals (5, nsupp), hub_U  (Hubbard atoms only; Loewdin
                 normalised when cfg['lowdin'])
    """
    L = np.asarray(cfg["L"], float)
    n = np.asarray(cfg["n"])
    coords = fd.grid_coords(L, n)
    dv = float(np.prod(L / n))
    out = []
    radii = [species_radii(sp) for sp in cfg["species"]]
    for ia, s in enumerate(cfg["atom_species"]):
        sp = cfg["species"][s]
        R = np.asarray(cfg["pos"][ia], float)
        kb_r, hub_r = radii[s]
        ent = {}
        rmax = max(kb_r)
        idx = support_indices(R, L, n, rmax)
        pts = coords[idx]
        vals, gam = [], []
        for l, g, rc in zip(sp["kb_l"], sp["kb_gamma"], kb_r):
            v = bloch_function_at(pts, R, L, k, lambda r, l=l: kb_radial(r, l, sp["kb_width"]), l, rc)
            vals.append(v)
            gam += [g] * (2 * l + 1)
        ent["kb_idx"] = idx
        ent["kb_vals"] = np.concatenate(vals, axis=0)
        ent["kb_gamma"] = np.array(gam)
        if sp["hub_l"] >= 0:
            hidx = support_indices(R, L, n, hub_r)
            hv = bloch_function_at(coords[hidx], R, L, k,
                                   lambda r: hubbard_radial(r, sp["hub_power"], sp["hub_alpha"]),
                                   sp["hub_l"], hub_r)
            if cfg.get("lowdin", True):
                hv = lowdin(hv, dv)
            ent["hub_idx"] = hidx
            ent["hub_vals"] = hv
            ent["hub_U"] = sp["hub_U"]
        out.append(ent)
    return out


def hubbard_functions(cfg, k=(0.0, 0.0, 0.0), threshold=None):
    """Hubbard orbitals of every Hubbard atom with their moment functions.

    Returns a list (one entry per Hubbard atom, atom order) of dicts:
      atom  : atom index;  U : effective U;  idx : support indices
      vals  : (2l+1, nsupp) orbitals (Loewdin-combined when cfg['lowdin'])
      moms  : (3, 2l+1, nsupp) moment functions sum_T phi(x-R-T) (x-R-T)_b
              e^{ik.T}, combined with the same Loewdin coefficients
      C     : the (2l+1)x(2l+1) Loewdin coefficients (identity without it)
    `threshold` overrides the species' truncation value (the force and
    stress pins use a tiny one so that the orbitals are smooth).
    """
    L = np.asarray(cfg["L"], float)
    n = np.asarray(cfg["n"])
    coords = fd.grid_coords(L, n)
    dv = float(np.prod(L / n))
    out = []
    for ia, s in enumerate(cfg["atom_species"]):
        sp = cfg["species"][s]
        if sp["hub_l"] < 0:
            continue
        thr = sp["threshold"] if threshold is None else threshold
        rad = (lambda r, sp=sp: hubbard_radial(r, sp["hub_power"], sp["hub_alpha"]))
        rc = truncation_radius(rad, thr)
        R = np.asarray(cfg["pos"][ia], float)
        idx = support_indices(R, L, n, rc)
        pts = coords[idx]
        raw = bloch_function_at(pts, R, L, k, rad, sp["hub_l"], rc)
        mom = [bloch_function_at(pts, R, L, k, rad, sp["hub_l"], rc, moment=b) for b in range(3)]
        m = raw.shape[0]
        C = np.eye(m)
        if cfg.get("lowdin", True):
            C = lowdin_coefficients(raw, dv)
        out.append(dict(atom=ia, U=sp["hub_U"], idx=idx, vals=C.T @ raw,
                        moms=np.stack([C.T @ x for x in mom]), C=C))
    return out


def lowdin_coefficients(vals, dv):
    """O^{-1/2} with O = Phi^H Phi dV (Phi = vals^T); the orthonormal
    orbitals are Phi O^{-1/2}."""
    phi = vals.T
    O = dv * (phi.conj().T @ phi)
    O = 0.5 * (O + O.conj().T)
    lam, U = np.linalg.eigh(O)
    return (U * (1.0 / np.sqrt(lam))) @ U.conj().T


def lowdin(vals, dv):
    """Symmetric orthonormalisation of the rows of vals (m, nsupp):
    Phi <- Phi O^{-1/2}, O = Phi^H Phi dV (Phi = vals^T)."""
    phi = vals.T
    O = dv * (phi.conj().T @ phi)
    O = 0.5 * (O + O.conj().T)
    lam, U = np.linalg.eigh(O)
    inv_sqrt = (U * (1.0 / np.sqrt(lam))) @ U.conj().T
    return (phi @ inv_sqrt).T


def local_potential(cfg, tail=1e-17):
    """V(x) on the grid: -D sum_I sum_T exp(-|x-R_I-T|^2/(2 s^2)), summing
    every image term that exceeds `tail` (|x - R_I - T| <= s sqrt(2 ln(D/tail)))."""
    L = np.asarray(cfg["L"], float)
    n = np.asarray(cfg["n"])
    V = np.zeros(int(np.prod(n)))
    for ia, s in enumerate(cfg["atom_species"]):
        sp = cfg["species"][s]
        D, sg = sp["vloc_depth"], sp["vloc_width"]
        rcut = sg * np.sqrt(2.0 * np.log(D / tail))
        nim = _images(rcut, L)
        R = np.asarray(cfg["pos"][ia], float)
        for t3 in range(-nim[2], nim[2] + 1):
            for t2 in range(-nim[1], nim[1] + 1):
                for t1 in range(-nim[0], nim[0] + 1):
                    box = _box_indices(R + np.array([t1, t2, t3]) * L, rcut, L, n)
                    if box is None:
                        continue
                    lin, d = box
                    r2 = np.sum(d * d, axis=1)
                    m = r2 <= rcut * rcut
                    np.subtract.at(V, lin[m], D * np.exp(-r2[m] / (2 * sg * sg)))
    return V


def local_potential_fourier(cfg, points, gmax_sigma=9.0):
    """Closed form of the same periodic Gaussian sum by Poisson summation:
    sum_T g(x-R-T) = (1/Omega) sum_G (2 pi s^2)^{3/2} e^{-s^2 G^2/2} e^{i G.(x-R)}.
    Used only as an independent pin of local_potential."""
    L = np.asarray(cfg["L"], float)
    omega = float(np.prod(L))
    V = np.zeros(points.shape[0])
    for ia, s in enumerate(cfg["atom_species"]):
        sp = cfg["species"][s]
        D, sg = sp["vloc_depth"], sp["vloc_width"]
        mmax = [int(np.ceil(gmax_sigma / sg * L[a] / (2 * pi))) for a in range(3)]
        R = np.asarray(cfg["pos"][ia], float)
        g1 = 2 * pi * np.arange(-mmax[0], mmax[0] + 1) / L[0]
        g2 = 2 * pi * np.arange(-mmax[1], mmax[1] + 1) / L[1]
        g3 = 2 * pi * np.arange(-mmax[2], mmax[2] + 1) / L[2]
        G = np.stack(np.meshgrid(g1, g2, g3, indexing="ij"), axis=-1).reshape(-1, 3)
        amp = (2 * pi * sg * sg) ** 1.5 * np.exp(-0.5 * sg * sg * np.sum(G * G, axis=1)) / omega
        ph = np.cos((points - R) @ G.T)
        V -= D * (ph @ amp)
    return V
