"""Moving atoms in a bound context and the AIMD occupation-matrix
extrapolation (Sec. II.B) through the C ABI, against the oracle.

  * after hcu_move_atoms the operator equals the oracle's operator at the
    new positions (FP64 bar 1e-12 relative), also when the supports change
    size, and equals the operator of a context created at those positions;
  * along a short trajectory (quadratic in time) the extrapolation
    coefficients equal the oracle's for the same positions (1e-10), each
    SCF reaches the oracle's SCF fixed point at that geometry (free energy
    1e-8 Ha/atom), and the extrapolated starts take fewer SCF iterations
    than restarting from the isolated-atom guess.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rand_D(nhub, seed):
    rng = np.random.default_rng(seed)
    D = np.zeros((1, nhub, 5, 5))
    for h in range(nhub):
        A = rng.normal(size=(5, 5)) * 0.05
        D[0, h] = 0.2 * np.eye(5) + A + A.T
    return D


@pytest.mark.parametrize("name", ["tiny", "c1"])
def test_move_atoms_operator_matches_oracle(name):
    torch = _torch()
    from oracle.hamiltonian import Hamiltonian
    from paper_2507_23612_amd import hcu
    cfg = workloads.make_config(name)
    ctx = hcu.HcuContext(cfg, workspace_margin=0.2)
    D = _rand_D(ctx.nhub, 5)
    ctx.set_hubbard_occupation(D)
    before = ctx.get_sizes()["table_nnz"]
    moved = dict(cfg)
    moved["pos"] = cfg["pos"] + np.random.default_rng(7).normal(0.0, 0.25, size=cfg["pos"].shape)
    ctx.move_atoms(moved["pos"], extrapolate=False)
    after = ctx.get_sizes()["table_nnz"]
    print(f"[gpu] move atoms {name}: table entries {before} -> {after}", flush=True)
    X = workloads.random_block(ctx.nd, ctx.ns, 17)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.empty_like(Xd)
    ctx.apply_h(Xd, Yd)
    torch.cuda.synchronize()
    want = Hamiltonian(moved, D=list(D[0])).apply(X)
    err = np.max(np.abs(Yd.cpu().numpy() - want)) / np.max(np.abs(want))
    fresh = hcu.HcuContext(moved)
    fresh.set_hubbard_occupation(D)
    Zd = torch.empty_like(Xd)
    fresh.apply_h(Xd, Zd)
    torch.cuda.synchronize()
    print(f"[gpu] moved operator rel err {err:.2e}; same as a fresh context: {bool(torch.equal(Yd, Zd))}",
          flush=True)
    assert err < 1e-12
    assert torch.equal(Yd, Zd)


def test_aimd_trajectory_extrapolated_starts():
    torch = _torch()
    from oracle import aimd
    from oracle import scf as oscf
    from paper_2507_23612_amd import hcu
    cfg = workloads.make_config("tiny")
    rng = np.random.default_rng(11)
    R0 = cfg["pos"].copy()
    v = rng.normal(0.0, 0.04, size=R0.shape)
    acc = rng.normal(0.0, 0.01, size=R0.shape)
    traj = [R0 + v * t + 0.5 * acc * t * t for t in range(6)]
    natom = len(cfg["atom_species"])

    def start(ctx):
        ctx.set_hubbard_occupation(hcu.initial_occupation(ctx, cfg))
        X0, v0 = hcu.start_inputs(ctx, cfg)
        ctx.set_start(0, 0, X0, v0)

    ext = hcu.HcuContext(cfg, workspace_margin=0.2)      # extrapolated starts
    start(ext)
    plain = hcu.HcuContext(cfg, workspace_margin=0.2)    # isolated-atom start at every step
    it_ext, it_plain = [], []
    for t, R in enumerate(traj):
        if t > 0:
            a, b, order = ext.move_atoms(R, extrapolate=True)
            ao, bo = aimd.extrapolation_coefficients(R, [traj[t - 1 - i] for i in range(min(t, 3))])
            print(f"[gpu] aimd step {t}: coefficients gpu ({a:.6f}, {b:.6f}) order {order}, "
                  f"oracle ({ao:.6f}, {bo:.6f})", flush=True)
            assert abs(a - ao) < 1e-10 and abs(b - bo) < 1e-10
            assert order == min(t, 3) - 1
            plain.move_atoms(R, extrapolate=False)
        start(plain)
        r1 = ext.scf()
        r2 = plain.scf()
        assert r1["converged"] and r2["converged"]
        it_ext.append(r1["iterations"])
        it_plain.append(r2["iterations"])
        step_cfg = dict(cfg)
        step_cfg["pos"] = R
        ref = oscf.scf(step_cfg)
        dF = abs(ext.get_energies()["F"] - ref["F"]) / natom
        print(f"[gpu] aimd step {t}: iterations extrapolated {r1['iterations']} isolated-atom "
              f"{r2['iterations']}; |F - F_oracle|/atom {dF:.2e}", flush=True)
        assert dF < 1e-8
    print(f"[gpu] aimd iterations after the first step: extrapolated {sum(it_ext[1:])}, "
          f"isolated-atom {sum(it_plain[1:])}", flush=True)
    assert sum(it_ext[1:]) < sum(it_plain[1:])
