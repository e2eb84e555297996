"""Learned initial guess for the Hubbard occupation matrices: site
descriptors, the per-site frame, density-shell coefficients, and the MLP
(forward, manual backward, MSE loss, Adam).

TEST INFRASTRUCTURE ONLY (see the oracle package header).

The paper starts the SCF from the isolated-atom average occupation
(Sec. II.B, initial guess of the occupation matrices); this module is the
plain FP64 statement of the learned replacement built on top of it:

  * Descriptor of a Hubbard site I: for every species S (in table order) and
    k = 0..31, with centres mu_k = 1 + 5.5 k / 31 bohr, width w = 0.25 bohr
    and cutoff rc = 6.5 bohr,
        G[32 S + k] = sum_{J of species S, images T; 0 < r < rc}
                      exp(-(r - mu_k)^2 / (2 w^2)) * (cos(pi r / rc) + 1) / 2,
    r = |R_J + T - R_I|.  Invariant under rigid motions and relabelling.
  * Site frame: in the rutile-like cells the two Ti sublattices differ by a
    90-degree rotation about z.  A site whose apical O neighbours (r < 4.5,
    |dz| < 1 bohr) lie along (1, -1, 0) is of the second kind (flag 1); its
    occupation matrix is expressed in the rotated frame, D_loc = M D M^T,
    with M the signed permutation that the rotation (x, y, z) -> (y, -x, z)
    induces on the real d orbitals (xy, yz, z^2, xz, x^2 - y^2).
  * Targets per site: the 15 upper-triangle entries of D_loc (row-major) and
    15 density-shell averages c_k = sum_x rho(x) g_k(x) / sum_x g_k(x) with
    g_k(x) = sum_T exp(-(|x - R_I - T| - r_k)^2 / (2 w^2)), r_k = 0.5 + 3.5 k/14.
  * MLP 64 -> 128 -> 128 -> 30, SiLU hidden activations (x / (1 + e^-x)),
    linear output; parameters flat [W1 (N x K, row-major), b1, W2, b2, ...].
    Inputs and targets are standardised with stored means and deviations.
  * Loss L = sum (y - t)^2 / (B * n_out); Adam with bias correction.
  * Using a prediction: D = M^T D_loc M for flag-1 sites, symmetrised, with
    eigenvalues clipped to [0, 1].

Pins (tests/test_oracle_mlp.py): central finite differences of the loss
(backward), torch.nn layers and torch.optim.Adam on the CPU (forward and
optimiser), single-neighbour closed forms and rigid-motion invariance of
the descriptor, the symmetry relation of the two sublattices' converged D
from the oracle SCF (frame), and the constant-density limit of the shells.
"""
from __future__ import annotations

import numpy as np

import workloads

NG = 32
MU = 1.0 + 5.5 * np.arange(NG) / (NG - 1)
WIDTH = 0.25
RCUT = 6.5
NSHELL = 15
SHELL_R = 0.5 + 3.5 * np.arange(NSHELL) / (NSHELL - 1)
APICAL_R = 4.5
APICAL_DZ = 1.0
DIMS = (64, 128, 128, 30)

# signed permutation of the real d orbitals (xy, yz, z^2, xz, x^2-y^2) under
# (x, y, z) -> (y, -x, z): xy -> -xy, yz -> -xz, z^2 -> z^2, xz -> yz,
# x^2-y^2 -> -(x^2-y^2)
FRAME_M = np.array([[-1, 0, 0, 0, 0],
                    [0, 0, 0, -1, 0],
                    [0, 0, 1, 0, 0],
                    [0, 1, 0, 0, 0],
                    [0, 0, 0, 0, -1]], float)

TRIU = np.triu_indices(5)


def _images(L, reach):
    n = [int(np.ceil(reach / L[a])) for a in range(3)]
    return np.array([(i, j, k) for i in range(-n[0], n[0] + 1) for j in range(-n[1], n[1] + 1)
                     for k in range(-n[2], n[2] + 1)], float) * np.asarray(L, float)


def hubbard_sites(cfg):
    spec = cfg["species"]
    return [i for i, s in enumerate(cfg["atom_species"]) if spec[s]["hub_l"] >= 0]


def descriptor(cfg):
    """(nhub, 32 * nspecies) descriptors and (nhub,) frame flags."""
    L = np.asarray(cfg["L"], float)
    pos = np.asarray(cfg["pos"], float)
    spec = np.asarray(cfg["atom_species"])
    nsp = len(cfg["species"])
    T = _images(L, RCUT)
    sites = hubbard_sites(cfg)
    G = np.zeros((len(sites), NG * nsp))
    flags = np.zeros(len(sites), np.int32)
    for a, i in enumerate(sites):
        apical = 0.0
        for j in range(len(pos)):
            d = pos[j] + T - pos[i]
            r = np.sqrt((d * d).sum(1))
            keep = (r > 0) & (r < RCUT)
            for dd, rr in zip(d[keep], r[keep]):
                fc = 0.5 * (np.cos(np.pi * rr / RCUT) + 1.0)
                G[a, NG * spec[j]:NG * (spec[j] + 1)] += np.exp(-(rr - MU) ** 2 / (2 * WIDTH ** 2)) * fc
                if cfg["species"][spec[j]]["hub_l"] < 0 and rr < APICAL_R and abs(dd[2]) < APICAL_DZ:
                    apical += dd[0] * dd[1]
        flags[a] = 1 if apical < 0 else 0
    return G, flags


def to_local(D, flag):
    return FRAME_M @ D @ FRAME_M.T if flag else D.copy()


def from_local(Dl, flag):
    return FRAME_M.T @ Dl @ FRAME_M if flag else Dl.copy()


def pack(D):
    return D[TRIU]


def unpack(v):
    D = np.zeros((5, 5))
    D[TRIU] = v
    return D + D.T - np.diag(np.diag(D))


def guess_from_output(v15, flag):
    """Occupation matrix from the 15 predicted local-frame entries:
    rotate back, symmetrise, clip the spectrum to [0, 1]."""
    D = from_local(unpack(v15), flag)
    D = 0.5 * (D + D.T)
    w, U = np.linalg.eigh(D)
    return (U * np.clip(w, 0.0, 1.0)) @ U.T


def shell_coefficients(cfg, rho):
    """(nhub, 15) shell averages of the density rho (nd,) around each site."""
    L = np.asarray(cfg["L"], float)
    n = np.asarray(cfg["n"])
    h = L / n
    i, j, k = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    # linear index x fastest: flatten in Fortran order
    x = np.stack([i.ravel(order="F") * h[0], j.ravel(order="F") * h[1], k.ravel(order="F") * h[2]], 1)
    T = _images(L, SHELL_R[-1] + 8 * WIDTH)
    pos = np.asarray(cfg["pos"], float)
    out = np.zeros((len(hubbard_sites(cfg)), NSHELL))
    for a, s in enumerate(hubbard_sites(cfg)):
        num = np.zeros(NSHELL)
        den = np.zeros(NSHELL)
        for t in T:
            r = np.sqrt(((x - pos[s] - t) ** 2).sum(1))
            g = np.exp(-(r[None, :] - SHELL_R[:, None]) ** 2 / (2 * WIDTH ** 2))
            num += g @ rho
            den += g.sum(1)
        out[a] = num / den
    return out


# ---------------------------------------------------------------- MLP
def param_count(dims=DIMS):
    return sum(dims[i + 1] * dims[i] + dims[i + 1] for i in range(len(dims) - 1))


def init_params(seed, dims=DIMS):
    """Seeded initial parameters (the shared input generator)."""
    return workloads.mlp_init_params(seed, dims)


def unflatten(theta, dims=DIMS):
    layers, o = [], 0
    for i in range(len(dims) - 1):
        k, n = dims[i], dims[i + 1]
        W = theta[o:o + n * k].reshape(n, k)
        o += n * k
        b = theta[o:o + n]
        o += n
        layers.append((W, b))
    return layers


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, X, dims=DIMS):
    """Returns the output and the per-layer (input, pre-activation) cache."""
    cache = []
    h = X
    layers = unflatten(theta, dims)
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        cache.append((h, z))
        h = silu(z) if li < len(layers) - 1 else z
    return h, cache


def loss(Y, Tg):
    return float(((Y - Tg) ** 2).sum() / Y.size)


def backward(theta, cache, Y, Tg, dims=DIMS):
    """Gradient of loss(Y, Tg) with respect to theta (flat, same layout)."""
    layers = unflatten(theta, dims)
    g = 2.0 * (Y - Tg) / Y.size
    grads = [None] * (2 * len(layers))
    for li in range(len(layers) - 1, -1, -1):
        h, z = cache[li]
        dz = g if li == len(layers) - 1 else g * silu_grad(z)
        W, _ = layers[li]
        grads[2 * li] = (dz.T @ h).ravel()
        grads[2 * li + 1] = dz.sum(0)
        g = dz @ W
    return np.concatenate(grads)


def adam_step(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step count t >= 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
