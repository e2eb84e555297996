"""Parity of the HIP path (through the C ABI) against the CPU oracle.

FP64 bars: operator and filter to 1e-12 relative (summation order is the
only difference), Ritz values to 1e-8 Ha, SCF free energy to 1e-8 Ha/atom.
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


def _ctx(cfg, precision=None):
    from paper_2507_23612_amd import hcu
    return hcu.HcuContext(cfg, precision)


def _rand_D(nspin, nhub, seed):
    rng = np.random.default_rng(seed)
    D = np.zeros((nspin, nhub, 5, 5))
    for s in range(nspin):
        for h in range(nhub):
            A = rng.normal(size=(5, 5)) * 0.05
            D[s, h] = 0.2 * np.eye(5) + A + A.T
    return D


def _oracle_H(cfg, D, k=(0.0, 0.0, 0.0)):
    from oracle.hamiltonian import Hamiltonian
    return Hamiltonian(cfg, k, D=list(D))


def _ragged():
    cfg = workloads.make_config("tiny")
    cfg["n"] = np.array([20, 18, 14], np.int32)
    cfg["ns"] = 7
    cfg["nelec"] = 8.0
    return cfg


@pytest.mark.parametrize("name", ["c1", "ragged", "tiny"])
def test_apply_h_matches_oracle(name):
    torch = _torch()
    cfg = _ragged() if name == "ragged" else workloads.make_config(name)
    print(f"[gpu] apply_h {name} n={list(cfg['n'])} ns={cfg['ns']}", flush=True)
    ctx = _ctx(cfg)
    D = _rand_D(1, ctx.nhub, 3)
    ctx.set_hubbard_occupation(D)
    X = workloads.random_block(ctx.nd, ctx.ns, 11)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.empty_like(Xd)
    ctx.apply_h(Xd, Yd)
    torch.cuda.synchronize()
    got = Yd.cpu().numpy()
    want = _oracle_H(cfg, D[0]).apply(X)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    print(f"[gpu] apply_h {name} rel err {err:.2e}", flush=True)
    assert err < 1e-12


@pytest.mark.parametrize("shape", [(20, 2, 4, 14), (20, 4, 2, 5), (8, 8, 2, 3), (16, 4, 4, 7), (20, 2, 2, 1),
                                   (20, 4, 2, 5, 1), (16, 6, 2, 7, 1), (20, 8, 1, 14, 1), (20, 4, 2, 1, 1)])
def test_apply_h_tile_shapes_ragged(shape):
    """Every stencil tiling mode (x halo from the tile row or from memory,
    ragged x/y tiles, 2 or 4 rows per thread, z chunks, the halo ring: halo
    rows read with the queue head, also in z chunks shorter than the ring
    and of one plane) against the oracle."""
    torch = _torch()
    cfg = _ragged()
    ctx = _ctx(cfg)
    ctx.set_tuning(*shape)
    D = _rand_D(1, ctx.nhub, 8)
    ctx.set_hubbard_occupation(D)
    X = workloads.random_block(ctx.nd, ctx.ns, 15)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.empty_like(Xd)
    ctx.apply_h(Xd, Yd)
    torch.cuda.synchronize()
    want = _oracle_H(cfg, D[0]).apply(X)
    err = np.max(np.abs(Yd.cpu().numpy() - want)) / np.max(np.abs(want))
    assert err < 1e-12


@pytest.mark.parametrize("precision,shape", [("fp64", (36, 16, 1, 24)), ("fp64", (36, 28, 1, 7)),
                                             ("mixed", (36, 16, 2, 12)), ("mixed", (36, 20, 1, 24))])
def test_apply_h_large_workgroups_c1(precision, shape):
    """Workgroups above 512 threads (the 1024-thread stencil variant), ragged
    in y, against the oracle."""
    torch = _torch()
    cfg = workloads.make_config("c1")
    ctx = _ctx(cfg, precision)
    ctx.set_tuning(*shape)
    D = _rand_D(1, ctx.nhub, 9)
    ctx.set_hubbard_occupation(D)
    X = workloads.random_block(ctx.nd, ctx.ns, 21)
    Xd = torch.from_numpy(X).cuda().to(ctx.dtype)
    Yd = torch.empty_like(Xd)
    ctx.apply_h(Xd, Yd)
    torch.cuda.synchronize()
    got = Yd.double().cpu().numpy()
    want = _oracle_H(cfg, D[0]).apply(X)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    print(f"[gpu] apply_h c1 {precision} shape {shape}: rel err {err:.2e}", flush=True)
    assert err < (1e-12 if precision == "fp64" else 2e-6)


def test_apply_h_after_autotune_c1():
    torch = _torch()
    cfg = workloads.make_config("c1")
    ctx = _ctx(cfg)
    from paper_2507_23612_amd import hcu
    X0, v0 = hcu.start_inputs(ctx, cfg)
    ctx.set_start(0, 0, X0, v0)
    best = ctx.autotune()
    print(f"[gpu] autotune c1 -> {best}", flush=True)
    D = _rand_D(1, ctx.nhub, 9)
    ctx.set_hubbard_occupation(D)
    X = workloads.random_block(ctx.nd, ctx.ns, 16)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.empty_like(Xd)
    ctx.apply_h(Xd, Yd)
    torch.cuda.synchronize()
    want = _oracle_H(cfg, D[0]).apply(X)
    assert np.max(np.abs(Yd.cpu().numpy() - want)) / np.max(np.abs(want)) < 1e-12


def test_apply_h_ld_and_partial_columns():
    torch = _torch()
    cfg = workloads.make_config("tiny")
    ctx = _ctx(cfg)
    D = _rand_D(1, ctx.nhub, 4)
    ctx.set_hubbard_occupation(D)
    ld = ctx.nd + 37
    X = np.zeros((5, ld))
    X[:, :ctx.nd] = workloads.random_block(ctx.nd, 5, 12)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.full_like(Xd, 7.0)
    ctx.apply_h(Xd, Yd, ncol=5, ld=ld)
    torch.cuda.synchronize()
    got = Yd.cpu().numpy()
    want = _oracle_H(cfg, D[0]).apply(X[:, :ctx.nd])
    assert np.max(np.abs(got[:, :ctx.nd] - want)) < 1e-12 * np.max(np.abs(want))
    assert np.all(got[:, ctx.nd:] == 7.0)     # padding untouched


def test_cheb_filter_ld_and_partial_columns():
    """Filter on 5 of the context's columns with a padded leading dimension
    (the fused scatter + projection steps run on a partial block)."""
    torch = _torch()
    from oracle import chfsi
    cfg = workloads.make_config("tiny")
    ctx = _ctx(cfg)
    D = _rand_D(1, ctx.nhub, 5)
    ctx.set_hubbard_occupation(D)
    ld = ctx.nd + 37
    X = np.zeros((5, ld))
    X[:, :ctx.nd] = workloads.random_block(ctx.nd, 5, 13)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.full_like(Xd, 7.0)
    a, b, aL, m = 1.0, 120.0, -0.5, 5
    ctx.cheb_filter(Xd, Yd, m, a, b, aL, ncol=5, ld=ld)
    torch.cuda.synchronize()
    got = Yd.cpu().numpy()
    want = chfsi.cheb_filter(_oracle_H(cfg, D[0]).apply, X[:, :ctx.nd], m, a, b, aL)
    err = np.max(np.abs(got[:, :ctx.nd] - want)) / np.max(np.abs(want))
    print(f"[gpu] filter partial columns rel err {err:.2e}", flush=True)
    assert err < 1e-11
    assert np.all(got[:, ctx.nd:] == 7.0)     # padding untouched


def test_apply_h_c2_sampled_columns():
    """Full-size c2 operator (72x72x96, 256 states) in the benchmark's launch
    configuration; the oracle recomputes 3 sampled columns."""
    torch = _torch()
    cfg = workloads.make_config("c2")
    print("[gpu] apply_h c2 full size", flush=True)
    ctx = _ctx(cfg)
    D = _rand_D(1, ctx.nhub, 5)
    ctx.set_hubbard_occupation(D)
    X = workloads.random_block(ctx.nd, ctx.ns, 13)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.empty_like(Xd)
    ctx.apply_h(Xd, Yd)
    torch.cuda.synchronize()
    cols = [0, 131, 255]
    got = Yd[cols].cpu().numpy()
    want = _oracle_H(cfg, D[0]).apply(X[cols])
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    print(f"[gpu] apply_h c2 rel err {err:.2e}", flush=True)
    assert err < 1e-12


def test_cheb_filter_matches_oracle():
    torch = _torch()
    from oracle import chfsi
    cfg = workloads.make_config("c1")
    ctx = _ctx(cfg)
    D = _rand_D(1, ctx.nhub, 6)
    ctx.set_hubbard_occupation(D)
    X = workloads.random_block(ctx.nd, ctx.ns, 14)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.empty_like(Xd)
    a, b, aL, m = 1.5, 190.0, -0.2, 20
    ctx.cheb_filter(Xd, Yd, m, a, b, aL)
    torch.cuda.synchronize()
    got = Yd.cpu().numpy()
    want = chfsi.cheb_filter(_oracle_H(cfg, D[0]).apply, X, m, a, b, aL)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    print(f"[gpu] filter c1 rel err {err:.2e}", flush=True)
    assert err < 1e-11


@pytest.mark.parametrize("kind", ["fp64", "mixed", "c128", "c64"])
def test_cheb_filter_odd_grid(kind):
    """Chebyshev filter on a 15x13x11 grid (2145 points: the last scatter
    brick and the last projection brick are ragged, rows unaligned), real
    and Bloch blocks; where the block type allows it (real, complex FP32)
    each step after the first takes its projections from the previous
    step's fused scatter pass.  Against the oracle's filter."""
    torch = _torch()
    from oracle import chfsi
    cfg = workloads.make_config("tiny", seed=3)
    cfg["n"] = np.array([15, 13, 11], np.int32)
    cfg["ns"] = 9
    cplx = kind in ("c128", "c64")
    if cplx:
        cfg["kpts"] = np.array([KPT])
    precision = "fp64" if kind in ("fp64", "c128") else "mixed"
    ctx = _ctx(cfg, precision)
    D = _rand_D(1, ctx.nhub, 21)
    ctx.set_hubbard_occupation(D)
    X = workloads.random_block(ctx.nd, ctx.ns, 22, complex_=cplx)
    Xd = torch.from_numpy(X).to(ctx.dtype).cuda()
    Yd = torch.empty_like(Xd)
    a, b, aL, m = 1.0, 120.0, -0.5, 6
    ctx.cheb_filter(Xd, Yd, m, a, b, aL)
    torch.cuda.synchronize()
    Xr = Xd.cpu().numpy().astype(np.complex128 if cplx else np.float64)
    H = _oracle_H(cfg, D[0], KPT if cplx else (0.0, 0.0, 0.0))
    want = chfsi.cheb_filter(H.apply, Xr, m, a, b, aL)
    err = np.max(np.abs(Yd.cpu().numpy() - want)) / np.max(np.abs(want))
    print(f"[gpu] filter odd grid {kind} rel err {err:.2e}", flush=True)
    assert err < (1e-11 if precision == "fp64" else 3e-5)


def test_chfsi_fixed_d_eigenvalues_tiny():
    """At fixed D, repeated passes converge to LAPACK eigenvalues of the
    oracle's assembled operator (1e-8 Ha)."""
    torch = _torch()
    from paper_2507_23612_amd import hcu
    cfg = workloads.make_config("tiny")
    cfg["ns"] = 24
    ctx = _ctx(cfg)
    D = _rand_D(1, ctx.nhub, 7)
    ctx.set_hubbard_occupation(D)
    X0, v0 = hcu.start_inputs(ctx, cfg)
    ctx.set_start(0, 0, X0, v0)
    ctx.lanczos_bounds(0, 0, 10)
    lam_old = None
    for _ in range(80):
        ctx.chfsi_pass(0, 0)
        ctx.update_occupations()
        lam = ctx.get_eigenvalues()[0, 0]
        if lam_old is not None and np.max(np.abs(lam - lam_old)) < 1e-13:
            break
        lam_old = lam
    ev = np.linalg.eigvalsh(_oracle_H(cfg, D[0]).dense())
    np.testing.assert_allclose(lam[:16], ev[:16], atol=1e-8)


def test_scf_c1_matches_oracle():
    """Full SCF on the 6-atom cell (36x36x24, 32 states, degree 20) against
    the oracle's SCF from the same seeded inputs."""
    torch = _torch()
    from oracle import scf as oscf
    from paper_2507_23612_amd import hcu
    cfg = workloads.make_config("c1")
    print("[gpu] scf c1", flush=True)
    ctx = _ctx(cfg)
    ctx.set_hubbard_occupation(hcu.initial_occupation(ctx, cfg))
    X0, v0 = hcu.start_inputs(ctx, cfg)
    ctx.set_start(0, 0, X0, v0)
    rep = ctx.scf(verbose=True)
    assert rep["converged"]
    ref = oscf.scf(cfg)
    natom = len(cfg["atom_species"])
    e = ctx.get_energies()
    print(f"[gpu] scf c1 F gpu {e['F']:.12f} oracle {ref['F']:.12f} iters {rep['iterations']} vs {ref['iterations']}",
          flush=True)
    assert abs(e["F"] - ref["F"]) / natom < 1e-8
    assert abs(e["E_U"] - ref["E_U"]) < 1e-7
    lam = ctx.get_eigenvalues()[0, 0]
    nocc = int(cfg["nelec"] / 2)
    np.testing.assert_allclose(lam[:nocc + 4], ref["eigs"][0, 0, :nocc + 4], atol=1e-8)
    Dg = ctx.get_hubbard_occupation()[0]
    for h in range(ctx.nhub):
        np.testing.assert_allclose(Dg[h], ref["D"][0][h], atol=1e-6)
    rho = ctx.get_density()[0]
    dv = float(np.prod(cfg["L"] / cfg["n"]))
    assert abs(rho.sum() * dv - cfg["nelec"]) < 1e-8
    np.testing.assert_allclose(rho, ref["rho"][0], atol=1e-6 * rho.max())


@pytest.mark.parametrize("ns", [16, 70])
def test_gram_and_rotate_match_numpy(ns):
    """Rayleigh-Ritz contractions against numpy (ragged tile counts)."""
    torch = _torch()
    cfg = workloads.make_config("tiny")
    cfg["ns"] = ns
    ctx = _ctx(cfg)
    dv = float(np.prod(cfg["L"] / cfg["n"]))
    Y = workloads.random_block(ctx.nd, ns, 21)
    Z = workloads.random_block(ctx.nd, ns, 22)
    S, Hs = ctx.gram(torch.from_numpy(Y).cuda(), torch.from_numpy(Z).cuda())
    Sw = dv * Y @ Y.T
    np.testing.assert_allclose(S, Sw, atol=1e-12 * np.abs(Sw).max())
    # Hs is computed on upper tiles and mirrored, diagonal tiles symmetrised
    Hw = dv * Y @ Z.T
    t = 64
    for i in range(ns):
        for j in range(i, ns):
            want = 0.5 * (Hw[i, j] + Hw[j, i]) if i // t == j // t else Hw[i, j]
            assert abs(Hs[i, j] - want) < 1e-12 * np.abs(Hw).max()
            assert Hs[j, i] == Hs[i, j]
    Cm = np.random.default_rng(3).normal(size=(ns, ns))
    Xd = torch.empty((ns, ctx.nd), dtype=torch.float64, device="cuda")
    ctx.rotate(torch.from_numpy(Y).cuda(), Cm, Xd)
    np.testing.assert_allclose(Xd.cpu().numpy(), (Y.T @ Cm).T, atol=1e-12 * np.abs(Y).max() * ns)


@pytest.mark.parametrize("kind", ["f64", "c64"])
def test_gram_fewer_columns_than_states(kind):
    """hcu_gram on the first ncol < ns states where ncol spans fewer output
    tiles than ns (the tile list built for ns must serve ncol): every entry
    of S and Hs against numpy."""
    torch = _torch()
    cfg = workloads.make_config("tiny")
    cfg["ns"] = 200
    cp = kind == "c64"
    if cp:
        cfg["kpts"] = np.array([KPT])
    ctx = _ctx(cfg, "fp64" if kind == "f64" else "mixed")
    dv = float(np.prod(cfg["L"] / cfg["n"]))
    ncol = 130
    Y = workloads.random_block(ctx.nd, 200, 23, complex_=cp)
    Z = workloads.random_block(ctx.nd, 200, 24, complex_=cp)
    Yd = torch.from_numpy(Y).cuda().to(ctx.dtype)
    Zd = torch.from_numpy(Z).cuda().to(ctx.dtype)
    S, Hs = ctx.gram(Yd, Zd, ncol=ncol, ld=ctx.nd)
    Yr = Yd.cpu().numpy().astype(np.complex128 if cp else np.float64)[:ncol]
    Zr = Zd.cpu().numpy().astype(np.complex128 if cp else np.float64)[:ncol]
    Sw = dv * Yr.conj() @ Yr.T
    Hw = dv * Yr.conj() @ Zr.T
    bar = 1e-12 if kind == "f64" else 1e-5
    assert np.max(np.abs(S - Sw)) < bar * np.abs(Sw).max()
    t = 32 if cp else 64
    for i in range(ncol):
        for j in range(i, ncol):
            want = 0.5 * (Hw[i, j] + np.conj(Hw[j, i])) if i // t == j // t else Hw[i, j]
            assert abs(Hs[i, j] - want) < bar * np.abs(Hw).max()


def test_apply_h_mixed_c1():
    """Mixed mode: FP32 blocks and tables (FP32 stencil, FP32 MFMA scatter)
    against the FP64 oracle; bound ~ a few FP32 ulps of the largest term."""
    torch = _torch()
    cfg = workloads.make_config("c1")
    ctx = _ctx(cfg, "mixed")
    D = _rand_D(1, ctx.nhub, 10)
    ctx.set_hubbard_occupation(D)
    X = workloads.random_block(ctx.nd, ctx.ns, 17)
    Xd = torch.from_numpy(X).float().cuda()
    Yd = torch.empty_like(Xd)
    ctx.apply_h(Xd, Yd)
    torch.cuda.synchronize()
    want = _oracle_H(cfg, D[0]).apply(X.astype(np.float32).astype(np.float64))
    err = np.max(np.abs(Yd.cpu().numpy() - want)) / np.max(np.abs(want))
    print(f"[gpu] apply_h mixed c1 rel err {err:.2e}", flush=True)
    assert err < 2e-6


def test_scf_mixed_c1_energy_error():
    """Mixed-precision SCF on the 6-atom cell: free energy within 1e-5 Ha/atom
    of the FP64 oracle (the stated target), occupied eigenvalues within 1e-5 Ha."""
    torch = _torch()
    from oracle import scf as oscf
    from paper_2507_23612_amd import hcu
    cfg = workloads.make_config("c1")
    ctx = _ctx(cfg, "mixed")
    ctx.set_hubbard_occupation(hcu.initial_occupation(ctx, cfg))
    X0, v0 = hcu.start_inputs(ctx, cfg)
    ctx.set_start(0, 0, X0, v0)
    rep = ctx.scf(tol_d=1e-5, tol_f=1e-7, verbose=True, raise_on_nonconv=False)
    ref = oscf.scf(cfg)
    natom = len(cfg["atom_species"])
    e = ctx.get_energies()
    dF = abs(e["F"] - ref["F"]) / natom
    lam = ctx.get_eigenvalues()[0, 0]
    nocc = int(cfg["nelec"] / 2)
    dl = np.max(np.abs(lam[:nocc] - ref["eigs"][0, 0, :nocc]))
    dEU = abs(e["E_U"] - ref["E_U"])
    print(f"[gpu] mixed c1: iters {rep['iterations']} conv {rep['converged']} |dF|/atom {dF:.2e} "
          f"max|dlam| {dl:.2e} |dE_U| {dEU:.2e}", flush=True)
    assert dF < 1e-5
    assert dl < 1e-5


KPT = (0.18, -0.18, 0.28)


@pytest.mark.parametrize("precision,ring", [("fp64", 0), ("mixed", 0), ("fp64", 1), ("mixed", 1)])
def test_apply_h_bloch_kpoint(precision, ring):
    """Complex (Bloch) path at a general k-point: stencil wrap phases, complex
    projectors and scatter, against the oracle (complex128); with the halo
    ring, z chunks of 5 planes (their ring loads clamped at the chunk end)."""
    torch = _torch()
    cfg = _ragged()
    cfg["kpts"] = np.array([KPT])
    ctx = _ctx(cfg, precision)
    if ring:
        ctx.set_tuning(20, 4, 2, 5, 1)
    D = _rand_D(1, ctx.nhub, 11)
    ctx.set_hubbard_occupation(D)
    X = workloads.random_block(ctx.nd, ctx.ns, 18, complex_=True)
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    Xd = torch.from_numpy(X).to(dt).cuda()
    Yd = torch.empty_like(Xd)
    ctx.apply_h(Xd, Yd)
    torch.cuda.synchronize()
    Xr = Xd.cpu().numpy().astype(np.complex128)
    want = _oracle_H(cfg, D[0], KPT).apply(Xr)
    err = np.max(np.abs(Yd.cpu().numpy() - want)) / np.max(np.abs(want))
    print(f"[gpu] apply_h k-point {precision} rel err {err:.2e}", flush=True)
    assert err < (1e-12 if precision == "fp64" else 3e-6)


@pytest.mark.parametrize("kind", ["fp64", "mixed", "c128", "c64"])
def test_apply_h_odd_grid_unaligned_rows(kind):
    """A 15x13x11 grid (2145 points: rows of the block not 16-byte aligned,
    so the brick kernels take their element-wise load path; last brick
    ragged) with 9 states, real and complex, against the oracle."""
    torch = _torch()
    cfg = workloads.make_config("tiny", seed=3)
    cfg["n"] = np.array([15, 13, 11], np.int32)
    cfg["ns"] = 9
    cplx = kind in ("c128", "c64")
    if cplx:
        cfg["kpts"] = np.array([KPT])
    precision = "fp64" if kind in ("fp64", "c128") else "mixed"
    ctx = _ctx(cfg, precision)
    D = _rand_D(1, ctx.nhub, 12)
    ctx.set_hubbard_occupation(D)
    X = workloads.random_block(ctx.nd, ctx.ns, 19, complex_=cplx)
    Xd = torch.from_numpy(X).to(ctx.dtype).cuda()
    Yd = torch.empty_like(Xd)
    ctx.apply_h(Xd, Yd)
    torch.cuda.synchronize()
    Xr = Xd.cpu().numpy().astype(np.complex128 if cplx else np.float64)
    want = _oracle_H(cfg, D[0], KPT if cplx else (0.0, 0.0, 0.0)).apply(Xr)
    err = np.max(np.abs(Yd.cpu().numpy() - want)) / np.max(np.abs(want))
    print(f"[gpu] apply_h odd grid {kind} rel err {err:.2e}", flush=True)
    assert err < (1e-12 if precision == "fp64" else 3e-6)


def test_scf_spin_polarised_kpoints_tiny():
    """Spin-polarised SCF with the shifted 2x2x2 k-point set (16 complex
    problems in one context) against the oracle's SCF."""
    torch = _torch()
    from oracle import scf as oscf
    from paper_2507_23612_amd import hcu
    cfg = workloads.with_kpoints(workloads.make_config("tiny"))
    ctx = _ctx(cfg)
    ctx.set_hubbard_occupation(hcu.initial_occupation(ctx, cfg))
    for s in range(2):
        for ik in range(8):
            X0, v0 = hcu.start_inputs(ctx, cfg, s, ik)
            ctx.set_start(s, ik, X0, v0)
    rep = ctx.scf(verbose=True)
    ref = oscf.scf(cfg)
    e = ctx.get_energies()
    natom = len(cfg["atom_species"])
    print(f"[gpu] spin+k tiny: F gpu {e['F']:.12f} oracle {ref['F']:.12f} iters {rep['iterations']} "
          f"vs {ref['iterations']}", flush=True)
    assert rep["converged"] and ref["converged"]
    assert abs(e["F"] - ref["F"]) / natom < 1e-8
    lam = ctx.get_eigenvalues()
    np.testing.assert_allclose(lam[:, :, :8], ref["eigs"][:, :, :8], atol=1e-8)
    Dg = ctx.get_hubbard_occupation()
    for s in range(2):
        for h in range(ctx.nhub):
            np.testing.assert_allclose(Dg[s, h], np.real(ref["D"][s][h]), atol=1e-6)


def test_scf_spin_polarised_kpoints_tiny_mixed():
    """The same spin-polarised 8-k-point SCF with complex FP32 blocks
    (projections, scatters, Gram matrices and rotations of complex FP32 on
    the matrix cores; Cholesky, eigensolve and D in FP64) against the
    oracle's FP64 SCF: free energy within 1e-5 Ha/atom."""
    torch = _torch()
    from oracle import scf as oscf
    from paper_2507_23612_amd import hcu
    cfg = workloads.with_kpoints(workloads.make_config("tiny"))
    ctx = _ctx(cfg, "mixed")
    ctx.set_hubbard_occupation(hcu.initial_occupation(ctx, cfg))
    for s in range(2):
        for ik in range(8):
            X0, v0 = hcu.start_inputs(ctx, cfg, s, ik)
            ctx.set_start(s, ik, X0, v0)
    rep = ctx.scf(tol_d=1e-5)
    ref = oscf.scf(cfg)
    e = ctx.get_energies()
    natom = len(cfg["atom_species"])
    dF = abs(e["F"] - ref["F"]) / natom
    lam = ctx.get_eigenvalues()
    dl = np.max(np.abs(lam[:, :, :8] - ref["eigs"][:, :, :8]))
    print(f"[gpu] spin+k tiny mixed: |dF|/atom {dF:.2e}, max |d eig| {dl:.2e}, iters {rep['iterations']}",
          flush=True)
    assert rep["converged"]
    assert dF < 1e-5
    assert dl < 1e-4

