"""The Rayleigh-Ritz eigensolve at the states counts of the benchmarks, for real
and complex (Bloch) blocks
(Sec. II.B: Chebyshev-filtered subspace iteration, Rayleigh-Ritz step),
where the Householder tridiagonalization runs in one workgroup.

One filter + Rayleigh-Ritz pass through the C ABI; the same filtered block Y
and H Y are rebuilt with hcu_cheb_filter / hcu_apply_h, their projected
matrices S = Y^T Y dV and H_s = Y^T H Y dV (hcu_gram) are solved on the CPU
with scipy's generalized symmetric eigensolver, and the pass's Ritz values
must match (1e-10 relative to the spectral width); the rotated block must be
dV-orthonormal and diagonalise H (1e-10).
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


@pytest.mark.parametrize("ns", [24, 256, 300, 512, 520])
def test_rayleigh_ritz_eigensolve_matches_scipy(ns):
    torch = _torch()
    import scipy.linalg
    from paper_2507_23612_amd import hcu
    cfg = workloads.make_config("c1")
    cfg["ns"] = ns
    print(f"[gpu] Rayleigh-Ritz eigensolve ns={ns}", flush=True)
    ctx = hcu.HcuContext(cfg)
    ctx.set_hubbard_occupation(hcu.initial_occupation(ctx, cfg))
    X0, v0 = hcu.start_inputs(ctx, cfg)
    ctx.set_start(0, 0, X0, v0)
    tmin, b = ctx.lanczos_bounds(0, 0, 10)
    a = tmin + (b - tmin) / 10.0
    Y = torch.empty_like(X0)
    ctx.cheb_filter(X0, Y, m=int(cfg["degree"]), a=a, b=b, aL=tmin)
    HY = torch.empty_like(Y)
    ctx.apply_h(Y, HY)
    S, Hs = ctx.gram(Y, HY)
    lam_ref = scipy.linalg.eigh(Hs, S, eigvals_only=True)
    ctx.chfsi_pass(0, 0)
    ctx.update_occupations()
    lam = ctx.get_eigenvalues()[0, 0]
    width = lam_ref[-1] - lam_ref[0]
    err = np.max(np.abs(lam - lam_ref)) / width
    X = ctx.get_orbitals(0, 0)
    HX = torch.empty_like(X)
    ctx.apply_h(X, HX)
    Sx, Hx = ctx.gram(X, HX)
    ctx.close()
    orth = np.max(np.abs(Sx - np.eye(ns)))
    diag = np.max(np.abs(Hx - np.diag(lam))) / width
    print(f"[gpu] ns={ns}: Ritz values rel err {err:.2e}, orthonormality {orth:.2e}, diagonalisation {diag:.2e}",
          flush=True)
    assert err < 1e-10 and orth < 1e-10 and diag < 1e-10


@pytest.mark.parametrize("ns", [24, 256, 300])
def test_rayleigh_ritz_eigensolve_complex_matches_scipy(ns):
    """Complex (Bloch) blocks, where the Hermitian reduction to tridiagonal
    form also runs in one workgroup: a +-k pair on the 6-atom cell, block
    (spin 0, k 0), against scipy's generalized Hermitian eigensolver, with
    the same bars as for real blocks."""
    torch = _torch()
    import scipy.linalg
    from paper_2507_23612_amd import hcu
    cfg = workloads.make_config("c1")
    cfg["ns"] = ns
    k = np.array([0.18, -0.18, 0.28])
    cfg["kpts"] = np.array([k, -k])
    cfg["kw"] = np.array([0.5, 0.5])
    print(f"[gpu] complex Rayleigh-Ritz eigensolve ns={ns}", flush=True)
    ctx = hcu.HcuContext(cfg)
    ctx.set_hubbard_occupation(hcu.initial_occupation(ctx, cfg))
    for ik in range(2):
        X0, v0 = hcu.start_inputs(ctx, cfg, 0, ik)
        ctx.set_start(0, ik, X0, v0)
    X0, _ = hcu.start_inputs(ctx, cfg, 0, 0)
    tmin, b = ctx.lanczos_bounds(0, 0, 10)
    a = tmin + (b - tmin) / 10.0
    Y = torch.empty_like(X0)
    ctx.cheb_filter(X0, Y, m=int(cfg["degree"]), a=a, b=b, aL=tmin, spin=0, ik=0)
    HY = torch.empty_like(Y)
    ctx.apply_h(Y, HY, spin=0, ik=0)
    S, Hs = ctx.gram(Y, HY)
    assert np.iscomplexobj(Hs) and np.max(np.abs(Hs.imag)) > 0
    lam_ref = scipy.linalg.eigh(Hs, S, eigvals_only=True)
    ctx.chfsi_pass(0, 0)
    ctx.lanczos_bounds(0, 1, 10)
    ctx.chfsi_pass(0, 1)
    ctx.update_occupations()
    lam = ctx.get_eigenvalues()[0, 0]
    width = lam_ref[-1] - lam_ref[0]
    err = np.max(np.abs(lam - lam_ref)) / width
    X = ctx.get_orbitals(0, 0)
    HX = torch.empty_like(X)
    ctx.apply_h(X, HX, spin=0, ik=0)
    Sx, Hx = ctx.gram(X, HX)
    ctx.close()
    orth = np.max(np.abs(Sx - np.eye(ns)))
    diag = np.max(np.abs(Hx - np.diag(lam))) / width
    print(f"[gpu] complex ns={ns}: Ritz values rel err {err:.2e}, orthonormality {orth:.2e}, "
          f"diagonalisation {diag:.2e}", flush=True)
    assert err < 1e-10 and orth < 1e-10 and diag < 1e-10
