"""Hubbard forces and stress through the C ABI against the oracle
(Sec. II.A force and stress sections).

Seeded inputs: the same start block is installed as the orbitals on both
sides (hcu_set_start / the oracle's arrays) with the same seeded
occupations, so FP64 results agree to rounding: bar 1e-10 relative to the
largest component.  FP32 blocks (mixed precision): gradients and
projections in FP32 with FP32 accumulation over supports of ~3e4 points,
combined in FP64; bar 1e-4 relative.  SCF level: the GPU's converged c1
orbitals against the oracle's converged orbitals (both SCFs stop at
|dD| < 1e-7), bar 1e-5 relative.
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


def _inputs(cfg, seed):
    nd = int(np.prod(cfg["n"]))
    X_sk, f_sk = [], []
    rng = np.random.default_rng(seed)
    for s in range(cfg["nspin"]):
        Xs, fs = [], []
        for ik, k in enumerate(cfg["kpts"]):
            cplx = bool(np.any(np.asarray(k) != 0))
            Xs.append(workloads.random_block(nd, cfg["ns"], seed + 100 * s + ik, complex_=cplx))
            fs.append(rng.uniform(0.0, 1.0, cfg["ns"]))
        X_sk.append(Xs)
        f_sk.append(fs)
    return X_sk, f_sk


def _gpu(cfg, precision, X_sk, f_sk):
    torch = _torch()
    from paper_2507_23612_amd import hcu
    ctx = hcu.HcuContext(cfg, precision)
    ctx.set_hubbard_occupation(hcu.initial_occupation(ctx, cfg))
    for s in range(ctx.nspin):
        for ik in range(ctx.nk):
            X = torch.from_numpy(X_sk[s][ik]).to(ctx.device).to(ctx.dtype)
            v0 = X[0].clone()
            ctx.set_start(s, ik, X, v0)
    occ = np.array(f_sk)
    F = ctx.hubbard_forces(occ)
    S = ctx.hubbard_stress(occ)
    ctx.close()
    # the oracle gets the same seeded orbitals, rounded on the host to the
    # block precision
    lo = {"fp64": (np.float64, np.complex128), "mixed": (np.float32, np.complex64)}[precision]
    Xr = [[x.astype(lo[1] if np.iscomplexobj(x) else lo[0]).astype(np.complex128 if np.iscomplexobj(x)
                                                                      else np.float64)
           for x in row] for row in X_sk]
    return F, S, Xr


CASES = {
    "tiny-gamma": ("tiny", None, "fp64"),
    "c1-gamma": ("c1", None, "fp64"),
    "tiny-spin-8k": ("tiny", "mp", "fp64"),
    "tiny-one-k": ("tiny", "one", "fp64"),
    "c1-mixed": ("c1", None, "mixed"),
    "tiny-spin-8k-mixed": ("tiny", "mp", "mixed"),
}


@pytest.mark.parametrize("case", list(CASES))
def test_forces_and_stress_match_oracle(case):
    from oracle import forces as oforces
    name, kind, precision = CASES[case]
    cfg = workloads.make_config(name)
    if kind == "mp":
        cfg = workloads.with_kpoints(cfg)
    elif kind == "one":
        cfg["kpts"] = np.array([[0.18, -0.18, 0.28]])      # complex occupation matrices
    print(f"[gpu] forces/stress {case}", flush=True)
    X_sk, f_sk = _inputs(cfg, 81)
    F, S, Xr = _gpu(cfg, precision, X_sk, f_sk)
    Fo, So = oforces.forces_and_stress(cfg, Xr, f_sk)
    ef = np.max(np.abs(F - Fo)) / np.max(np.abs(Fo))
    es = np.max(np.abs(S - So)) / np.max(np.abs(So))
    print(f"[gpu] forces/stress {case}: rel err forces {ef:.2e} stress {es:.2e}; "
          f"max |f| {np.max(np.abs(Fo)):.3e} max |sigma| {np.max(np.abs(So)):.3e}", flush=True)
    bar = 1e-10 if precision == "fp64" else 1e-4
    assert ef < bar and es < bar
    hub = [ia for ia, s in enumerate(cfg["atom_species"]) if cfg["species"][s]["hub_l"] >= 0]
    assert np.all(F[[ia for ia in range(len(cfg["atom_species"])) if ia not in hub]] == 0)


def test_forces_and_stress_after_scf_c1():
    """Forces and stress at the self-consistent ground state of the 6-atom
    cell: GPU SCF against the oracle's SCF."""
    _torch()
    from oracle import forces as oforces
    from oracle import scf as oscf
    from paper_2507_23612_amd import hcu
    cfg = workloads.make_config("c1")
    print("[gpu] forces/stress after SCF c1", flush=True)
    ctx = hcu.HcuContext(cfg)
    ctx.set_hubbard_occupation(hcu.initial_occupation(ctx, cfg))
    X0, v0 = hcu.start_inputs(ctx, cfg)
    ctx.set_start(0, 0, X0, v0)
    assert ctx.scf()["converged"]
    F = ctx.hubbard_forces()
    S = ctx.hubbard_stress()
    ref = oscf.scf(cfg)
    Fo, So = oforces.forces_and_stress(cfg, ref["X"], [[ref["occ"][0, 0]]])
    ef = np.max(np.abs(F - Fo)) / np.max(np.abs(Fo))
    es = np.max(np.abs(S - So)) / np.max(np.abs(So))
    print(f"[gpu] SCF c1: max |f| {np.max(np.abs(Fo)):.3e} Ha/bohr, rel err {ef:.2e}; "
          f"max |sigma| {np.max(np.abs(So)):.3e} Ha/bohr^3, rel err {es:.2e}", flush=True)
    assert ef < 1e-5 and es < 1e-5


@pytest.mark.parametrize("name,precision", [("c2", "fp64"), ("c3", "mixed")])
def test_forces_and_stress_full_size_sampled_states(name, precision):
    """Full-size blocks (c2: 256 states FP64; c3: 640 states FP32) in the
    benchmark's configuration; occupations are zero except on four states
    in different 64-state tiles, so the oracle needs only those columns
    (a state with f = 0 contributes nothing to D, the forces or the stress)."""
    torch = _torch()
    from oracle import forces as oforces
    from paper_2507_23612_amd import hcu
    cfg = workloads.make_config(name)
    nd, ns = int(np.prod(cfg["n"])), int(cfg["ns"])
    print(f"[gpu] forces/stress full size {name} {precision}", flush=True)
    if precision == "fp64":
        X = workloads.random_block(nd, ns, 91)
    else:
        X = np.random.default_rng(91).random((ns, nd), dtype=np.float32) - np.float32(0.5)
    cols = [5, 70, 141, 250] if ns == 256 else [3, 200, 411, 637]
    f = np.zeros(ns)
    f[cols] = [0.9, 0.6, 0.35, 0.1]
    ctx = hcu.HcuContext(cfg, precision)
    ctx.set_hubbard_occupation(hcu.initial_occupation(ctx, cfg))
    Xd = torch.from_numpy(X).to(ctx.device).to(ctx.dtype)
    ctx.set_start(0, 0, Xd, Xd[0].clone())
    torch.cuda.synchronize()
    import time
    t0 = time.perf_counter()
    F = ctx.hubbard_forces(f[None, None, :])
    S = ctx.hubbard_stress(f[None, None, :])
    dt = time.perf_counter() - t0
    ctx.close()
    del Xd
    Xo = X[cols].astype(np.float64)
    Fo, So = oforces.forces_and_stress(cfg, [[Xo]], [[f[cols]]])
    ef = np.max(np.abs(F - Fo)) / np.max(np.abs(Fo))
    es = np.max(np.abs(S - So)) / np.max(np.abs(So))
    print(f"[gpu] full size {name}: forces + stress {dt * 1e3:.1f} ms; rel err forces {ef:.2e} stress {es:.2e}",
          flush=True)
    bar = 1e-10 if precision == "fp64" else 1e-4
    assert ef < bar and es < bar
