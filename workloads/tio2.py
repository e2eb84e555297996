"""Synthetic rutile-TiO2-like cells (seeded), standing in for the paper's
rutile supercells (Sec. III.B, Table 2) whose pseudopotentials and
structures are not available.

Every quantity here is an input of the problem: cell, grid, atom positions,
the per-species parameter table, states/electrons/smearing, k-points, and the
seeded random numbers the solver draws (start block, Lanczos start vector).
Nothing here evaluates a potential, an orbital or a stencil.

Layout conventions shared by every consumer:
  * grid node (i, j, k) sits at (i*h1, j*h2, k*h3), 0-based, h_a = L_a / n_a;
  * the linear grid index is i + n1*(j + n2*k) (x fastest);
  * a block of states is a numpy array of shape (ns, nd) in C order, i.e. the
    same memory as an nd x ns column-major matrix with leading dimension nd.
"""
from __future__ import annotations

import copy
import numpy as np

# rutile internal parameter and the 8.7 x 8.7 x 5.6 bohr block (one TiO2
# rutile-like cell: 2 Ti + 4 O).
RUTILE_U = 0.305
BLOCK = (8.7, 8.7, 5.6)
ELECTRONS_PER_TIO2 = 8.0

CONFIG_NAMES = ("tiny", "small", "c1", "c2", "c3", "c5")


def species_table():
    """Parameters of the two synthetic species (index 0 = 'Ti', 1 = 'O').

    vloc_*   : local potential, a Gaussian of the given depth (Ha) and width
               sigma (bohr), exp(-r^2 / (2 sigma^2)).
    kb_l     : angular momenta of the Kleinman-Bylander channels (l <= 1);
    kb_gamma : their energies (Ha); kb_width: Gaussian radial width (bohr).
    hub_l    : angular momentum of the Hubbard manifold (-1 = none);
    hub_U    : effective U (Ha); radial r^hub_power * exp(-hub_alpha r).
    threshold: value (bohr^-3/2) below which radial functions are truncated.
    occ_guess: isolated-atom average occupation per Hubbard spin-orbital.
    """
    ti = dict(name="Ti", vloc_depth=2.0, vloc_width=1.0,
              kb_l=[0, 1], kb_gamma=[1.0, 0.5], kb_width=1.0,
              hub_l=2, hub_U=0.147, hub_power=2, hub_alpha=1.5,
              threshold=5e-3, occ_guess=0.2)
    o = dict(name="O", vloc_depth=2.0, vloc_width=1.0,
             kb_l=[0, 1], kb_gamma=[0.6, 0.3], kb_width=1.0,
             hub_l=-1, hub_U=0.0, hub_power=2, hub_alpha=1.5,
             threshold=5e-3, occ_guess=0.0)
    return [ti, o]


def _motif_full():
    """Fractional positions of the 6-atom rutile-like cell."""
    u = RUTILE_U
    spec = [0, 0, 1, 1, 1, 1]
    frac = [(0.0, 0.0, 0.0), (0.5, 0.5, 0.5),
            (u, u, 0.0), (1 - u, 1 - u, 0.0),
            (0.5 + u, 0.5 - u, 0.5), (0.5 - u, 0.5 + u, 0.5)]
    return spec, np.array(frac)


def _unit(parity):
    """One TiO2 formula unit of the rutile motif (A for even, B for odd)."""
    u = RUTILE_U
    if parity == 0:
        frac = [(0.0, 0.0, 0.0), (u, u, 0.0), (1 - u, 1 - u, 0.0)]
    else:
        frac = [(0.5, 0.5, 0.5), (0.5 + u, 0.5 - u, 0.5), (0.5 - u, 0.5 + u, 0.5)]
    return [0, 1, 1], np.array(frac)


def supercell_full(rep):
    """rep = (r1, r2, r3) copies of the full 6-atom cell."""
    spec0, frac0 = _motif_full()
    spec, pos = [], []
    blk = np.array(BLOCK)
    for c in range(rep[2]):
        for b in range(rep[1]):
            for a in range(rep[0]):
                off = np.array([a, b, c], float)
                for s, f in zip(spec0, frac0):
                    spec.append(s)
                    pos.append((f + off) * blk)
    L = blk * np.array(rep, float)
    return np.array(spec, np.int32), np.array(pos), L


def supercell_units(rep):
    """rep blocks with ONE formula unit each, alternating A/B by the parity of
    the block index sum (16 Ti + 32 O for 2x2x4; 36 Ti + 72 O for 3x3x4)."""
    spec, pos = [], []
    blk = np.array(BLOCK)
    for c in range(rep[2]):
        for b in range(rep[1]):
            for a in range(rep[0]):
                s0, f0 = _unit((a + b + c) % 2)
                off = np.array([a, b, c], float)
                for s, f in zip(s0, f0):
                    spec.append(s)
                    pos.append((f + off) * blk)
    L = blk * np.array(rep, float)
    return np.array(spec, np.int32), np.array(pos), L


def mp_shifted_222(L):
    """Shifted 2x2x2 Monkhorst-Pack set: k_a = +-pi/(2 L_a), weights 1/8
    (Cartesian, bohr^-1).  Closed under k -> -k."""
    ks = []
    for s3 in (-1, 1):
        for s2 in (-1, 1):
            for s1 in (-1, 1):
                ks.append((s1 * np.pi / (2 * L[0]), s2 * np.pi / (2 * L[1]),
                           s3 * np.pi / (2 * L[2])))
    return np.array(ks), np.full(8, 1.0 / 8.0)


def _base(name, spec, pos, L, n, ns, degree, jitter, seed):
    rng = np.random.default_rng(seed)
    pos = pos + rng.normal(0.0, jitter, size=pos.shape)
    nti = int(np.sum(spec == 0))
    return dict(
        name=name, L=np.asarray(L, float), n=np.asarray(n, np.int32), n0=6,
        species=species_table(), atom_species=np.asarray(spec, np.int32),
        pos=pos, ns=int(ns), nelec=ELECTRONS_PER_TIO2 * nti, kT=0.003,
        degree=int(degree), nspin=1, kpts=np.zeros((1, 3)), kw=np.ones(1),
        lowdin=True, first_passes=4, lanczos_steps=10,
        x0_seed=12345, lanczos_seed=777, geom_seed=seed,
        pulay_history=7, pulay_beta=0.3, scf_tol_d=1e-7, scf_tol_f=1e-7,
        max_iter=100, precision="fp64",
    )


def make_config(name, seed=0, jitter=None):
    """Return the named workload as a dict of plain numbers/arrays.

    tiny  : 6-atom cell on a 12x12x8 grid (dense-diagonalisation size)
    small : 6-atom cell on an 18x18x12 grid
    c1    : 6-atom cell, 36x36x24, 32 states, degree 20
    c2    : 48 atoms (2x2x4 blocks of one TiO2), 72x72x96, 256 states, degree 16
    c3    : 108 atoms (3x3x4 blocks), 108x108x96, 640 states, mixed precision
    c5    : 24 atoms (2x2x1 full cells), 72x72x24, 128 states, jitter 0.1
    """
    if name in ("tiny", "small", "c1"):
        spec, pos, L = supercell_full((1, 1, 1))
        n = {"tiny": (12, 12, 8), "small": (18, 18, 12), "c1": (36, 36, 24)}[name]
        ns = {"tiny": 16, "small": 24, "c1": 32}[name]
        cfg = _base(name, spec, pos, L, n, ns, 20, 0.05 if jitter is None else jitter, seed)
        if name != "c1":
            cfg["degree"] = 12
        return cfg
    if name == "c2":
        spec, pos, L = supercell_units((2, 2, 4))
        return _base(name, spec, pos, L, (72, 72, 96), 256, 16,
                     0.05 if jitter is None else jitter, seed)
    if name == "c3":
        spec, pos, L = supercell_units((3, 3, 4))
        cfg = _base(name, spec, pos, L, (108, 108, 96), 640, 16,
                    0.05 if jitter is None else jitter, seed)
        cfg["precision"] = "mixed"
        return cfg
    if name == "c5":
        spec, pos, L = supercell_full((2, 2, 1))
        return _base(name, spec, pos, L, (72, 72, 24), 128, 16,
                     0.1 if jitter is None else jitter, seed)
    raise ValueError(f"unknown config {name!r}")


def with_kpoints(cfg):
    """Spin-polarised copy of cfg with the shifted 2x2x2 k-point set."""
    out = copy.deepcopy(cfg)
    out["nspin"] = 2
    out["kpts"], out["kw"] = mp_shifted_222(out["L"])
    out["name"] = cfg["name"] + "-sk8"
    return out


def batch_cells(seed0=1):
    """The 16 independent cells of the batched workload: four each of
    6 atoms (36x36x24, 32 states), 12 atoms (1x1x2 cells, 36x36x48, 64),
    24 atoms (2x2x1 cells, 72x72x24, 128) and 48 atoms (the c2 cell)."""
    cells = []
    for i in range(16):
        kind = i // 4
        seed = seed0 + i
        if kind == 0:
            c = make_config("c1", seed=seed)
        elif kind == 1:
            spec, pos, L = supercell_full((1, 1, 2))
            c = _base("c12", spec, pos, L, (36, 36, 48), 64, 16, 0.05, seed)
        elif kind == 2:
            spec, pos, L = supercell_full((2, 2, 1))
            c = _base("c24", spec, pos, L, (72, 72, 24), 128, 16, 0.05, seed)
        else:
            c = make_config("c2", seed=seed)
        c["degree"] = 16
        cells.append(c)
    return cells


def random_block(nd, ns, seed, complex_=False):
    """Seeded start block, uniform in [-1/2, 1/2); shape (ns, nd)."""
    rng = np.random.default_rng(seed)
    x = rng.random((ns, nd)) - 0.5
    if complex_:
        x = x + 1j * (rng.random((ns, nd)) - 0.5)
    return np.ascontiguousarray(x)


def random_vector(nd, seed, complex_=False):
    """Seeded Lanczos start vector, uniform in [-1/2, 1/2)."""
    return random_block(nd, 1, seed, complex_)[0]


def start_seed(cfg, spin, ik):
    """Seed of the start block of spin channel `spin`, k-point `ik`."""
    return int(cfg["x0_seed"]) + 1000 * int(spin) + int(ik)


def lanczos_seed(cfg, spin, ik):
    """Seed of the Lanczos start vector of spin channel `spin`, k-point `ik`."""
    return int(cfg["lanczos_seed"]) + 1000 * int(spin) + int(ik)


def initial_occupation_diag(cfg, spin):
    """Diagonal value of the initial Hubbard occupation matrix of each
    Hubbard atom: the isolated-atom average occupation per spin-orbital;
    spin-polarised runs add +-0.1 to break the spin symmetry."""
    out = []
    for s in cfg["atom_species"]:
        sp = cfg["species"][s]
        if sp["hub_l"] < 0:
            continue
        g = sp["occ_guess"]
        if cfg["nspin"] == 2:
            g = g + (0.1 if spin == 0 else -0.1)
        out.append(g)
    return out


def mlp_init_params(seed, dims):
    """Seeded initial parameters of an MLP with layer widths dims, flat
    [W1 (dims[1] x dims[0], row-major), b1, W2, b2, ...], each entry uniform
    in (-1/sqrt(fan_in), 1/sqrt(fan_in))."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(len(dims) - 1):
        k, n = dims[i], dims[i + 1]
        bound = 1.0 / np.sqrt(k)
        out.append(rng.uniform(-bound, bound, size=n * k))
        out.append(rng.uniform(-bound, bound, size=n))
    return np.concatenate(out)

