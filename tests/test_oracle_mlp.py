"""Pins of the learned-guess oracle (oracle/mlp.py) against facts that do
not come from it: finite differences, torch's own layers and optimiser,
closed forms of the descriptor, rigid-motion invariance, the symmetry of the
two Ti sublattices in the oracle's converged SCF, and constant densities."""
import copy

import numpy as np
import pytest

import workloads
from oracle import mlp


def _rand(dims, seed, batch=9):
    rng = np.random.default_rng(seed)
    theta = mlp.init_params(seed, dims)
    X = rng.normal(size=(batch, dims[0]))
    T = rng.normal(size=(batch, dims[-1]))
    return theta, X, T


def test_backward_matches_central_differences():
    dims = (6, 8, 7, 5)
    theta, X, T = _rand(dims, 1)
    Y, cache = mlp.forward(theta, X, dims)
    g = mlp.backward(theta, cache, Y, T, dims)
    h = 1e-6
    fd = np.zeros_like(theta)
    for i in range(theta.size):
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        fd[i] = (mlp.loss(mlp.forward(tp, X, dims)[0], T) - mlp.loss(mlp.forward(tm, X, dims)[0], T)) / (2 * h)
    assert np.max(np.abs(g - fd)) <= 1e-6 * max(1.0, np.max(np.abs(fd)))


def test_forward_and_gradient_match_torch():
    import torch
    dims = mlp.DIMS
    theta, X, T = _rand(dims, 2, batch=17)
    Y, cache = mlp.forward(theta, X, dims)
    g = mlp.backward(theta, cache, Y, T, dims)
    layers = []
    for W, b in mlp.unflatten(theta, dims):
        lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W))
            lin.bias.copy_(torch.from_numpy(b))
        layers.append(lin)
    h = torch.from_numpy(X)
    for i, lin in enumerate(layers):
        h = lin(h)
        if i < len(layers) - 1:
            h = torch.nn.functional.silu(h)
    np.testing.assert_allclose(h.detach().numpy(), Y, rtol=1e-12, atol=1e-12)
    L = torch.nn.functional.mse_loss(h, torch.from_numpy(T))
    L.backward()
    gt = torch.cat([torch.cat([lin.weight.grad.reshape(-1), lin.bias.grad]) for lin in layers]).numpy()
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-13)


def test_adam_matches_torch():
    import torch
    rng = np.random.default_rng(3)
    theta = rng.normal(size=40)
    grads = [rng.normal(size=40) for _ in range(4)]
    p = torch.nn.Parameter(torch.from_numpy(theta.copy()))
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    th = theta.copy()
    for t, g in enumerate(grads, start=1):
        p.grad = torch.from_numpy(g.copy())
        opt.step()
        th, m, v = mlp.adam_step(th, g, m, v, t, 3e-3)
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-13, atol=1e-15)


def _two_atom_cell(r, direction, L=40.0):
    cfg = workloads.make_config("tiny")
    d = np.asarray(direction, float)
    d /= np.linalg.norm(d)
    cfg["L"] = np.array([L, L, L])
    cfg["atom_species"] = np.array([0, 1], np.int32)
    cfg["pos"] = np.array([[10.0, 11.0, 12.0], [10.0, 11.0, 12.0] + r * d])
    return cfg


@pytest.mark.parametrize("r", [1.3, 3.7, 6.2])
def test_descriptor_single_neighbour_closed_form(r):
    cfg = _two_atom_cell(r, (0.3, -0.5, 0.8))
    G, _ = mlp.descriptor(cfg)
    mu = 1.0 + 5.5 * np.arange(32) / 31
    want = np.exp(-(r - mu) ** 2 / (2 * 0.25 ** 2)) * 0.5 * (np.cos(np.pi * r / 6.5) + 1)
    np.testing.assert_allclose(G[0, 32:], want, rtol=1e-10, atol=1e-300)
    assert np.all(G[0, :32] == 0)          # no Ti neighbour inside the cutoff
    far = _two_atom_cell(6.6, (1, 0, 0))
    assert np.all(mlp.descriptor(far)[0] == 0)


def test_descriptor_rigid_motion_and_relabelling():
    cfg = workloads.make_config("c5", seed=1005)
    G, fl = mlp.descriptor(cfg)
    moved = copy.deepcopy(cfg)
    rng = np.random.default_rng(0)
    moved["pos"] = np.mod(cfg["pos"] + rng.normal(size=3) * 3.0, cfg["L"])
    perm = rng.permutation(len(cfg["pos"]))
    moved["pos"] = moved["pos"][perm]
    moved["atom_species"] = cfg["atom_species"][perm]
    G2, fl2 = mlp.descriptor(moved)
    sites = mlp.hubbard_sites(cfg)
    sites2 = mlp.hubbard_sites(moved)
    order = [sites2.index(int(np.where(perm == s)[0][0])) for s in sites]
    np.testing.assert_allclose(G2[order], G, rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(fl2[order], fl)
    # 90-degree rotation about z (L1 = L2) swaps the two frames
    rot = copy.deepcopy(cfg)
    p = cfg["pos"]
    rot["pos"] = np.mod(np.stack([p[:, 1], -p[:, 0], p[:, 2]], 1), cfg["L"])
    G3, fl3 = mlp.descriptor(rot)
    np.testing.assert_allclose(G3, G, rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(fl3, 1 - fl)


def test_frame_maps_one_sublattice_onto_the_other():
    """Unjittered rutile cell: the two Ti sites are related by the 90-degree
    rotation, so their converged occupation matrices agree in the site frame
    (and differ in the lattice frame)."""
    from oracle import scf as oscf
    cfg = workloads.make_config("tiny", jitter=0.0)
    _, fl = mlp.descriptor(cfg)
    assert sorted(fl.tolist()) == [0, 1]
    D = oscf.scf(cfg)["D"][0]
    a, b = (0, 1) if fl[0] == 0 else (1, 0)
    assert np.max(np.abs(D[a] - D[b])) > 1e-3
    np.testing.assert_allclose(mlp.to_local(D[b], 1), D[a], atol=1e-7)
    np.testing.assert_allclose(mlp.from_local(mlp.to_local(D[b], 1), 1), D[b], atol=1e-15)


def test_shells_of_a_constant_density():
    cfg = workloads.make_config("tiny")
    nd = int(np.prod(cfg["n"]))
    c = mlp.shell_coefficients(cfg, np.full(nd, 0.37))
    np.testing.assert_allclose(c, 0.37, rtol=1e-13)


def test_guess_spectrum_and_round_trip():
    rng = np.random.default_rng(4)
    A = rng.normal(size=(5, 5))
    U, _ = np.linalg.qr(A)
    D = (U * np.array([0.0, 0.1, 0.5, 0.9, 1.0])) @ U.T
    for flag in (0, 1):
        np.testing.assert_allclose(mlp.guess_from_output(mlp.pack(mlp.to_local(D, flag)), flag), D, atol=1e-13)
    Dbad = (U * np.array([-0.3, 0.1, 0.5, 0.9, 1.4])) @ U.T
    w = np.linalg.eigvalsh(mlp.guess_from_output(mlp.pack(Dbad), 0))
    np.testing.assert_allclose(w, [0.0, 0.1, 0.5, 0.9, 1.0], atol=1e-13)
