"""Benchmark of the ChFSI hot path on one MI355X.

A step is one SCF iteration of real-space DFT+U over one block of orbitals:
degree-m Chebyshev filter (m applications of H = stencil + V_loc + KB +
Hubbard, fused with the three-term step), Rayleigh-Ritz (H Y, S and Hs
contractions, FP64 generalized eigensolve, rotation), Fermi level and
occupations, occupation matrices D, E_U and free energy, Pulay mixing.
Inputs are resident in HBM before the timed region; table setup is one-time
and not timed.

value = nd * ns * (m + 1) / seconds per step / 1e9  [Gpts.states/s]
(m filter applications plus the H Y of Rayleigh-Ritz).

Also reported: the stencil kernel's and the fused scatter + projection
kernel's achieved rates against the MI355X peaks (algorithmic bytes or
flops / event-timed average launch), the mixed-precision figure on the
108-atom cell beside the FP64 one (default run), the SCF wall time to
convergence, the time of one Hubbard force and one stress evaluation, and
the CPU oracle's throughput on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# dense matrix-core peaks of the MI355X (published): FP64 78.6, FP32 157.3 TFLOP/s
MFMA_PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3}
METRIC = "ChFSI H·X Gpts·states/s (FP64 vs mixed); SCF wall-time to 1e-5 Ha/atom"

WORKLOADS = {
    "c2": "48-atom TiO2-like cell (16 Ti + 32 O), 17.4x17.4x22.4 bohr, grid 72x72x96, 256 states, "
          "Chebyshev degree 16, 12th-order FD, Gamma, spin-unpolarised",
    "c3": "108-atom TiO2-like cell (36 Ti + 72 O), 26.1x26.1x22.4 bohr, grid 108x108x96, 640 states, "
          "Chebyshev degree 16, 12th-order FD, Gamma, spin-unpolarised",
    "c1": "6-atom TiO2-like cell, 8.7x8.7x5.6 bohr, grid 36x36x24, 32 states, Chebyshev degree 20",
    "c2k": "c2 cell spin-polarised with the shifted 2x2x2 k-point set: 16 complex (spin, k) blocks of "
           "497664 x 256 in one context, one persistent stencil launch per Chebyshev step over all of them",
}


def make_workload(name):
    import workloads
    if name == "c2k":
        cfg = workloads.with_kpoints(workloads.make_config("c2"))
        cfg["precision"] = "mixed"
        return cfg
    return workloads.make_config(name)


def stencil_bytes(cfg, elem):
    """Algorithmic HBM bytes of one fused Chebyshev-step stencil launch: read
    Y_i and Y_{i-1}, write Y_{i+1} (3 words per point-state) for every
    (spin, k) block of the launch, plus V_loc once per block."""
    nd = int(np.prod(cfg["n"]))
    ns = int(cfg["ns"])
    nsk = int(cfg["nspin"]) * len(cfg["kw"])
    return nsk * (3 * elem * nd * ns + elem * nd)


def parse_tile(text):
    """TX,TYt,RY,TZ[,ring] -> (TX, TYt, RY, TZ, halo_ring)."""
    parts = text.split(",")
    ring = 1 if len(parts) == 5 and parts[4] == "ring" else 0
    if len(parts) not in (4, 5) or (len(parts) == 5 and not ring):
        raise SystemExit(f"--tile: expected TX,TYt,RY,TZ[,ring], got {text!r}")
    return tuple(int(v) for v in parts[:4]) + (ring,)


def tile_name(t):
    """Tile shape as the counter records name it: TX,TYt,RY,TZ[,ring]."""
    name = f'{t["tile_x"]},{t["tile_yt"]},{t["ry"]},{t["tile_z"]}'
    return name + (",ring" if t.get("halo_ring") else "")


def measured_traffic(kernel, config, prec, tile, sources):
    """HBM bytes per launch of `kernel` from the committed counter summaries
    profiles/<kernel>_<config>_<prec>*.md (FETCH_SIZE and WRITE_SIZE runs,
    calibrated on a plain copy; one file per stencil tile shape, "any" for
    kernels that do not depend on it), or None if there is none for this
    tile shape or the kernel's sources changed since it was taken."""
    import glob
    from paper_2507_23612_amd.tracesum import kernel_source_digest
    digest = kernel_source_digest(sources)
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"{kernel}_{config}_{prec}*.md"))):
        rec = {}
        with open(path) as fh:
            for line in fh:
                if line.startswith("- record "):
                    k, _, v = line[len("- record "):].partition(":")
                    rec[k.strip()] = v.strip()
        try:
            if rec.get("source_sha256") == digest and rec.get("tile") in (tile, "any"):
                return int(float(rec["traffic_bytes_per_launch"]))
        except (KeyError, ValueError):
            continue
    return None


def cpu_baseline(cfg, nstates=24, degree=16):
    """The oracle's Chebyshev filter on a bounded sample of the workload:
    `nstates` states of the same grid and operator, degree-`degree` filter."""
    import psutil
    import workloads
    from oracle import chfsi
    from oracle.hamiltonian import Hamiltonian
    h = Hamiltonian(cfg, D=[0.2 * np.eye(5)] * sum(1 for s in cfg["atom_species"] if s == 0))
    X = workloads.random_block(h.nd, nstates, 1)
    proc = psutil.Process()
    c0 = proc.cpu_times()
    t0 = time.perf_counter()
    chfsi.cheb_filter(h.apply, X, degree, 20.0, 190.0, -0.1)
    dt = time.perf_counter() - t0
    c1 = proc.cpu_times()
    cores = max(1, int(round(((c1.user - c0.user) + (c1.system - c0.system)) / dt)))
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": h.nd * nstates * degree / dt / 1e9, "unit": "Gpts·states/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{nstates} of {cfg['ns']} states, one degree-{degree} Chebyshev filter "
                      f"({degree} H applications) on the full {cfg['n'][0]}x{cfg['n'][1]}x{cfg['n'][2]} grid, "
                      f"{dt:.1f} s on host cores",
            "cores_note": "threads actually used = process CPU time / wall time over the sample (numpy/BLAS "
                          "threads)",
            "nproc": os.cpu_count(), "cpu_model": model or None,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


MODEL = os.path.join(ROOT, "paper_2507_23612_amd", "models", "site_mlp_c5.npz")


def bench_scf_compare(args):
    """SCF wall time at equal accuracy on held-out c5 cells (seeds 3000..):
    FP64 and mixed precision, each from the isolated-atom start and from the
    learned start (BF16 inference, counted inside the timer), all four with
    the same stopping rule (|D_out - D_in|_F < 1e-5 and |dF|/atom < 1e-6 Ha)
    and the cells of one setting converged together in one batch.  The
    accuracy reached is checked against an FP64 reference converged to
    1e-9 (|F - F_ref|/atom, target 1e-5 Ha/atom)."""
    import torch
    import workloads
    from paper_2507_23612_amd import hcu, mlguess
    if not os.path.exists(MODEL):
        raise FileNotFoundError(f"{MODEL} missing: train it with python -m paper_2507_23612_amd.mlguess --save-model")
    seeds = list(range(mlguess.HELDOUT_SEED0, mlguess.HELDOUT_SEED0 + args.cells))
    cfgs = [workloads.make_config("c5", seed=s) for s in seeds]
    m = mlguess.load_model(MODEL)
    natom = len(cfgs[0]["atom_species"])
    tol_d, tol_f = 1e-5, 1e-6

    def run(precision, learned, td, tf):
        ctxs = [mlguess._context(c, precision) for c in cfgs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for ctx, cfg in zip(ctxs, cfgs):
            if learned:
                m.guess(ctx, bf16=True)
            else:
                ctx.set_hubbard_occupation(hcu.initial_occupation(ctx, cfg))
        b = hcu.HcuBatch(ctxs)
        reps = b.scf(max_iter=100, tol_d=td, tol_f=tf, raise_on_nonconv=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        b.close()
        for ctx in ctxs:
            ctx.close()
        return reps, dt

    ref, _ = run("fp64", False, 1e-9, 1e-10)
    Fref = [r["F"] for r in ref]
    table = {}
    for prec in ("fp64", "mixed"):
        for start in ("isolated_atom", "learned"):
            reps, dt = run(prec, start == "learned", tol_d, tol_f)
            err = [abs(r["F"] - f) / natom for r, f in zip(reps, Fref)]
            table[f"{prec}+{start}"] = {
                "seconds": round(dt, 3), "iterations": [int(r["iterations"]) for r in reps],
                "mean_iterations": round(float(np.mean([r["iterations"] for r in reps])), 2),
                "converged": all(bool(r["converged"]) for r in reps),
                "max_abs_F_minus_ref_per_atom_Ha": max(err), "within_1e-5": max(err) < 1e-5}
    base = table["fp64+isolated_atom"]["seconds"]
    best = table["mixed+learned"]["seconds"]
    return {"metric": "SCF wall-time to 1e-5 Ha/atom (mixed + learned start vs FP64 + isolated-atom start)",
            "value": round(best, 3), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": round(1e3 * best, 1), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{args.cells} held-out c5 cells (24 atoms, 72x72x24, 128 states, jitter 0.1), "
                                   "converged together in one batch per setting",
                       "stopping_rule": f"|D_out-D_in|_F < {tol_d:g} and |dF|/atom < {tol_f:g} Ha",
                       "reference": "FP64 SCF to |dD| < 1e-9, |dF|/atom < 1e-10"},
            "settings": table,
            "speedup_vs_fp64_isolated_atom": {k: round(base / v["seconds"], 3) for k, v in table.items()}}


def bench_batch(args):
    """Sixteen independent cells (4 each of 6, 12, 24 and 48 atoms), FP64,
    degree 16: a step is one ChFSI pass (filter + Rayleigh-Ritz) on every
    cell.  Timed batched (one persistent stencil launch per Chebyshev step
    over all 16 blocks) and sequential (each cell's own launches)."""
    import torch
    import workloads
    from paper_2507_23612_amd import hcu
    cells = workloads.batch_cells()
    ctxs = []
    tuned = {}
    for cfg in cells:
        ctx = hcu.HcuContext(cfg, "fp64")
        ctx.set_hubbard_occupation(hcu.initial_occupation(ctx, cfg))
        X0, v0 = hcu.start_inputs(ctx, cfg)
        ctx.set_start(0, 0, X0, v0)
        key = (tuple(int(v) for v in cfg["n"]), int(cfg["ns"]))
        if key not in tuned:                      # one autotuning per cell type
            tuned[key] = ctx.autotune()
        t = tuned[key]
        ctx.set_tuning(t["tile_x"], t["tile_yt"], t["ry"], t["tile_z"], t["halo_ring"])
        ctx.lanczos_bounds()
        ctxs.append(ctx)
    work = sum(int(np.prod(c["n"])) * int(c["ns"]) * (int(c["degree"]) + 1) for c in cells)
    b = hcu.HcuBatch(ctxs)
    for _ in range(args.warmup):
        b.chfsi_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.chfsi_pass()
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t0) / args.steps
    for _ in range(args.warmup):
        for ctx in ctxs:
            ctx.chfsi_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for ctx in ctxs:
            ctx.chfsi_pass()
    torch.cuda.synchronize()
    dt_s = (time.perf_counter() - t0) / args.steps
    b.close()
    for ctx in ctxs:
        ctx.close()
    return {"metric": "ChFSI H·X Gpts·states/s, 16 independent cells batched", "value": round(work / dt_b / 1e9, 3),
            "unit": "Gpts·states/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(dt_b * 1e3, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "batch16: 4 cells each of 6 atoms (36x36x24, 32 states), 12 atoms (36x36x48, 64), "
                                   "24 atoms (72x72x24, 128), 48 atoms (72x72x96, 256); degree 16, Gamma",
                       "precision": "fp64"},
            "sequential": {"ms_per_step": round(dt_s * 1e3, 3), "value": round(work / dt_s / 1e9, 3)},
            "batched_over_sequential": round(dt_s / dt_b, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--precision", default=None, help="fp64 | mixed (default: the config's)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-scf", action="store_true", help="skip the SCF wall-time run")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision (c3) figure of the default run")
    ap.add_argument("--no-c1", action="store_true", help="skip the c1 FP64 figure of the default run")
    ap.add_argument("--no-hxc", action="store_true",
                    help="skip the density-dependent Hamiltonian figure (Hartree + exchange + density mixing)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (calibrates hardware byte counters)")
    ap.add_argument("--tile", default=None,
                    help="stencil tile shape TX,TYt,RY,TZ[,ring] (skips the autotuner, e.g. for profiling; "
                         "ring: halo rows read with the queue head)")
    ap.add_argument("--scf-compare", action="store_true",
                    help="SCF wall time on held-out 24-atom cells: mixed precision with the learned start against "
                         "FP64 with the isolated-atom start (needs the trained site network)")
    ap.add_argument("--cells", type=int, default=8, help="cells for --scf-compare")
    ap.add_argument("--batch", action="store_true",
                    help="measure the 16-cell batched workload instead (one persistent stencil launch per "
                         "Chebyshev step over all cells) against the same cells run one after another")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU hot path "
              "(see the sharding design notes); --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_2507_23612_amd import hcu

    if args.calib_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.batch:
        print(json.dumps(bench_batch(args)), flush=True)
        return
    if args.scf_compare:
        print(json.dumps(bench_scf_compare(args)), flush=True)
        return
    out = measure(args, args.config, args.precision, hcu, torch, top=True)
    if not args.no_hxc:
        out["hxc"] = measure_hxc(args, args.config, args.precision, out["stencil_tuning"], hcu, torch)
    if args.config == "c2" and args.precision in (None, "fp64") and not args.no_mixed:
        # the mixed-precision half of the metric, on its own workload (c3)
        mixed = measure(args, "c3", "mixed", hcu, torch, top=False)
        out["mixed"] = mixed
    if args.config == "c2" and args.precision in (None, "fp64") and not args.no_c1:
        # the small FP64 configuration of the metric; its 8 MB block lives in the
        # Infinity Cache, so no HBM fraction is claimed for it
        c1 = measure(args, "c1", "fp64", hcu, torch, top=False)
        c1["note"] = "cache-resident block (31104 x 32 FP64, 8 MB): throughput only, no HBM roofline claim"
        out["c1"] = {k: c1[k] for k in ("value", "unit", "ms_per_step", "dtype", "config", "kernel_ms_per_step",
                                         "note")}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(make_workload(args.config))
    print(json.dumps(out), flush=True)


def fused_roofline(cfg, prec, sizes, kt, config, tile, complex_):
    """Roofline of the fused scatter + projection kernel of one Chebyshev
    step (the stage that follows the stencil): algorithmic HBM bytes = the
    block read and written once (2 words per point-state) + the function
    values once (nnz of the per-point table) + the projection partial sums
    written once; algorithmic flops = 2 per (point, function, state) for the
    scatter and 2 for the projection (x4 for complex blocks)."""
    nd, ns = sizes["nd"], int(cfg["ns"])
    nsk = int(cfg["nspin"]) * len(cfg["kw"])
    elem = (4 if prec == "mixed" else 8) * (2 if complex_ else 1)
    nbytes = nsk * (2 * elem * nd * ns + elem * sizes["table_nnz"] + elem * sizes["brick_slots"] * ns)
    flops = nsk * 4 * sizes["table_nnz"] * ns * (4 if complex_ else 1)
    if kt["fused_launches"] == 0:
        return None
    ms = kt["fused_ms"] / kt["fused_launches"]
    gbs = nbytes / (ms * 1e-3) / 1e9
    tf = flops / (ms * 1e-3) / 1e12
    peak_tf = MFMA_PEAK_TFLOPS["mixed" if prec == "mixed" else "fp64"]
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("k_scatter_project", config, prec, tile, ("proj.hip",)),
            "kernel": "k_scatter_project (projector scatter of a Chebyshev step fused with the projections of "
                      "its output)",
            "avg_launch_ms": round(ms, 4), "algorithmic_bytes_per_launch": int(nbytes),
            "algorithmic_flops_per_launch": int(flops), "achieved_tflops": round(tf, 2),
            "mfma_peak_tflops": peak_tf, "mfma_frac": round(tf / peak_tf, 4)}


def scf_reference(config):
    """The oracle's converged SCF of this configuration, if it was stored
    (tests/golden/scf_reference_<config>.json, written by
    tests/golden/make_scf_reference.py from the oracle alone)."""
    path = os.path.join(ROOT, "tests", "golden", f"scf_reference_{config}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh)


def measure_hxc(args, config, precision, tuning, hcu, torch):
    """SCF iterations of the same workload with the density-dependent
    Hamiltonian (V = V_loc + V_H[rho_in] + V_x[rho_in], the density mixed by
    the Kerker-preconditioned Pulay step, its coefficients mixing D): time
    per iteration and the share of the density, Hartree/exchange energies and
    mixing step (stream time of those phases, host solve included)."""
    cfg = make_workload(config)
    cfg["hxc"] = True
    prec = precision or cfg["precision"]
    nd, ns = int(np.prod(cfg["n"])), int(cfg["ns"])
    ctx = hcu.HcuContext(cfg, prec)
    ctx.set_tuning(tuning["tile_x"], tuning["tile_yt"], tuning["ry"], tuning["tile_z"], tuning["halo_ring"])
    ctx.set_hubbard_occupation(hcu.initial_occupation(ctx, cfg))
    for sp in range(ctx.nspin):
        for ik in range(ctx.nk):
            X0, v0 = hcu.start_inputs(ctx, cfg, sp, ik)
            ctx.set_start(sp, ik, X0, v0)
            del X0, v0
    ctx.scf_begin(first_passes=1)
    for _ in range(args.warmup):
        ctx.scf_step()
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info = ctx.scf_step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    kt = ctx.get_kernel_times()
    ctx.set_profiling(False)
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    m = int(cfg["degree"])
    elem = 4 if prec == "mixed" else 8
    hx_ms = kt["hxc_ms"] / args.steps
    # algorithmic bytes of the density-dependent phases per iteration: the
    # density reads the orbital block once; the grid passes (sums, FFTs,
    # window, combination, Kerker step, assembly) are ~(30 + 3 m) grid
    # vectors of doubles with a full mixing window of m = 7 differences
    hx_bytes = ns * nd * elem + (30 + 3 * 7) * nd * 8
    return {"ms_per_step": round(dt * 1e3, 3),
            "value": round(nd * ns * (m + 1) / dt / 1e9, 3), "unit": "Gpts·states/s",
            "hxc_ms_per_step": round(hx_ms, 3), "hxc_share": round(hx_ms / (dt * 1e3), 4),
            "hxc_algorithmic_bytes": int(hx_bytes),
            "hxc_achieved_GBs": round(hx_bytes / (hx_ms * 1e-3) / 1e9, 1) if hx_ms > 0 else None,
            "residual_rho_last": info["residual_rho"],
            "note": "density + FFT Hartree (stencil symbol) + LDA exchange + Kerker-preconditioned Pulay step on "
                    "the density; stream time of those phases per SCF iteration"}


def measure(args, config, precision, hcu, torch, top):
    """Throughput of K timed SCF iterations of one workload (inputs resident,
    setup and tuning untimed), with the stencil and fused-kernel rooflines
    from HIP events on the library's stream; the top-level line also gets
    the SCF wall time and the forces/stress timing."""
    cfg = make_workload(config)
    prec = precision or cfg["precision"]
    nd = int(np.prod(cfg["n"]))
    ns = int(cfg["ns"])
    m = int(cfg["degree"])
    nsk = int(cfg["nspin"]) * len(cfg["kw"])

    ctx = hcu.HcuContext(cfg, prec)
    ctx.set_hubbard_occupation(hcu.initial_occupation(ctx, cfg))
    for sp in range(ctx.nspin):
        for ik in range(ctx.nk):
            X0, v0 = hcu.start_inputs(ctx, cfg, sp, ik)
            ctx.set_start(sp, ik, X0, v0)
            del X0, v0
    torch.cuda.synchronize()
    if args.tile and top:
        tx, tyt, ry, tz, ring = parse_tile(args.tile)
        ctx.set_tuning(tx, tyt, ry, tz, ring)
        tuning = {"tile_x": tx, "tile_yt": tyt, "ry": ry, "tile_z": tz, "halo_ring": ring, "stencil_ms": None}
    else:
        tuning = ctx.autotune()
    ctx.scf_begin(first_passes=1)
    for _ in range(args.warmup):
        ctx.scf_step()
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.scf_step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = ctx.get_kernel_times()
    ctx.set_profiling(False)
    ms_step = dt / args.steps * 1e3
    value = nsk * nd * ns * (m + 1) / (dt / args.steps) / 1e9

    elem = (4 if prec == "mixed" else 8) * (2 if ctx.complex else 1)
    bytes_launch = stencil_bytes(cfg, elem)
    st_ms = kt["stencil_ms"] / max(kt["stencil_launches"], 1)
    achieved = bytes_launch / (st_ms * 1e-3) / 1e9
    tile = tile_name(tuning)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic("k_stencil", config, prec, tile, ("stencil.hip",)),
                "kernel": ("k_stencil_batch (persistent, all (spin, k) blocks)" if nsk > 1 else
                           "k_stencil_big" if tuning["tile_x"] * tuning["tile_yt"] > 512 else "k_stencil")
                          + " (12th-order FD stencil + V_loc + Chebyshev three-term step)",
                "avg_launch_ms": round(st_ms, 4), "algorithmic_bytes_per_launch": int(bytes_launch),
                "tile": tile}
    breakdown = {k: round(v / args.steps, 3) for k, v in kt.items() if k.endswith("_ms")}
    sizes = ctx.get_sizes()
    fused = fused_roofline(cfg, prec, sizes, kt, config, tile, ctx.complex)
    dtype = ("c64" if prec == "mixed" else "c128") if ctx.complex else ("f32" if prec == "mixed" else "f64")
    out = {"metric": METRIC, "value": round(value, 3), "unit": "Gpts·states/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic",
           "config": {"workload": f"{config}: {WORKLOADS.get(config, config)}",
                      "precision": prec, "nd": nd, "ns": ns, "degree": m},
           "roofline": roofline, "roofline_second": fused, "kernel_ms_per_step": breakdown,
           "stencil_tuning": tuning}
    # "roofline" describes the kernel that takes the most time per step
    if fused and kt["fused_ms"] > kt["stencil_ms"]:
        out["roofline"], out["roofline_second"] = fused, roofline
    if not top:
        out = {k: out[k] for k in ("value", "unit", "ms_per_step", "dtype", "config", "roofline", "roofline_second",
                                   "kernel_ms_per_step", "stencil_tuning")}
    # forces and stress of the state reached (one call each, outside the timed region)
    ctx.update_occupations()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.hubbard_forces()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.hubbard_stress()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out["forces_stress_ms"] = {"forces": round((t1 - t0) * 1e3, 2), "stress": round((t2 - t1) * 1e3, 2)}

    if top and not args.no_scf:
        ctx2 = hcu.HcuContext(cfg, prec)
        ctx2.set_tuning(tuning["tile_x"], tuning["tile_yt"], tuning["ry"], tuning["tile_z"], tuning["halo_ring"])
        ctx2.set_hubbard_occupation(hcu.initial_occupation(ctx2, cfg))
        for sp in range(ctx2.nspin):
            for ik in range(ctx2.nk):
                X0, v0 = hcu.start_inputs(ctx2, cfg, sp, ik)
                ctx2.set_start(sp, ik, X0, v0)
                del X0, v0
        torch.cuda.synchronize()
        tol_d = 1e-5 if prec == "mixed" else 1e-7
        ref = scf_reference(config)
        natom = len(cfg["atom_species"])
        # step-wise, timing every iteration (from the Lanczos bounds and the
        # first filter on; the one-time table setup is excluded)
        t0 = time.perf_counter()
        ctx2.scf_begin(max_iter=100, tol_d=tol_d)
        t_acc = None
        for _ in range(100):
            info = ctx2.scf_step()
            if ref is not None and t_acc is None and info["converged"] and \
                    abs(info["F"] - ref["F"]) / natom < 1e-5:
                t_acc = time.perf_counter() - t0
            if info["converged"]:
                break
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        e = ctx2.get_energies()
        out["scf"] = {"wall_s": round(wall, 3), "iterations": info["iteration"] + 1,
                      "converged": bool(info["converged"]), "F_Ha": e["F"], "E_U_Ha": e["E_U"],
                      "criterion": f"|D_out-D_in|_F < {tol_d:g} and |dF|/atom < 1e-7 Ha"}
        if ref is not None:
            out["scf"]["F_oracle_Ha"] = ref["F"]
            out["scf"]["dF_per_atom_vs_oracle"] = abs(e["F"] - ref["F"]) / natom
            out["scf"]["wall_s_to_1e-5_Ha_per_atom"] = round(t_acc, 3) if t_acc is not None else None
        ctx2.close()
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
