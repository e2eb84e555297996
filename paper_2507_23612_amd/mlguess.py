"""Learned start for the Hubbard occupation matrices, end to end on the GPU.

  1. data     converged SCF runs (isolated-atom start) of seeded cells; per
              Hubbard site the descriptor (hcu_descriptor) and the targets
              (hcu_site_targets: site-frame D and density shells);
  2. train    the site MLP with the library's forward/backward/Adam kernels
              on mini-batches drawn from a seeded permutation;
  3. compare  SCF from the learned start (BF16 inference, hcu_mlp_guess)
              against SCF from the isolated-atom start on held-out cells:
              iterations, wall time and the final free-energy difference.

Everything numeric runs in the library; this module moves arrays and
collects reports.  Command line (writes one JSON summary):

    python -m paper_2507_23612_amd.mlguess --train 2000 --heldout 200 \\
        --out mlguess.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DIMS = (64, 128, 128, 30)
TRAIN_SEED0 = 1000
HELDOUT_SEED0 = 3000


def _cell(seed):
    import workloads
    return workloads.make_config("c5", seed=seed)


def _context(cfg, precision="fp64"):
    from paper_2507_23612_amd import hcu
    ctx = hcu.HcuContext(cfg, precision)
    for s in range(ctx.nspin):
        for ik in range(ctx.nk):
            X0, v0 = hcu.start_inputs(ctx, cfg, s, ik)
            ctx.set_start(s, ik, X0, v0)
    return ctx


def _scf_group(ctxs, tol_d, tol_f, max_iter=100):
    """Converge a group of contexts together (one persistent stencil launch
    per Chebyshev step over all of them)."""
    from paper_2507_23612_amd import hcu
    b = hcu.HcuBatch(ctxs)
    t0 = time.perf_counter()
    reps = b.scf(max_iter=max_iter, tol_d=tol_d, tol_f=tol_f, raise_on_nonconv=False)
    dt = time.perf_counter() - t0
    b.close()
    return reps, dt


def generate(seeds, group=8, tol_d=1e-6, tol_f=1e-7, log=print):
    """Descriptors X [nsite, 64], targets T [nsite, 30], and per-cell SCF
    reports from the isolated-atom start."""
    from paper_2507_23612_amd import hcu
    Xs, Ts, cells = [], [], []
    t0 = time.perf_counter()
    for g0 in range(0, len(seeds), group):
        chunk = seeds[g0:g0 + group]
        cfgs = [_cell(s) for s in chunk]
        ctxs = [_context(c) for c in cfgs]
        for ctx, cfg in zip(ctxs, cfgs):
            ctx.set_hubbard_occupation(hcu.initial_occupation(ctx, cfg))
        reps, _ = _scf_group(ctxs, tol_d, tol_f)
        for seed, ctx, rep in zip(chunk, ctxs, reps):
            if not rep["converged"]:
                log(f"[mlguess] cell {seed} did not converge; skipped")
                ctx.close()
                continue
            d, _ = ctx.descriptor()
            Xs.append(d.cpu().numpy())
            Ts.append(ctx.site_targets())
            cells.append({"seed": int(seed), "iterations": int(rep["iterations"]), "F": rep["F"]})
            ctx.close()
        log(f"[mlguess] data {min(g0 + group, len(seeds))}/{len(seeds)} cells, "
            f"{time.perf_counter() - t0:.1f} s", flush=True)
    return np.concatenate(Xs).astype(np.float32), np.concatenate(Ts).astype(np.float32), cells


def standardised_error(m, X, T, chunk):
    """Per-output mean squared error of the network's FP32 predictions in
    the units of its own output scaling (the training loss's units); X is
    fed in chunks of at most the network's batch capacity."""
    import torch
    _, _, out_mean, out_sd = m.get_scaling()
    err = np.zeros(T.shape[1])
    for r0 in range(0, X.shape[0], chunk):
        Y = m.forward(torch.from_numpy(np.ascontiguousarray(X[r0:r0 + chunk])).cuda()).cpu().numpy()
        err += (((Y - T[r0:r0 + chunk]) / out_sd) ** 2).sum(0)
    return err / X.shape[0]


def train(X, T, epochs=200, batch=256, lr=2e-3, seed=7, val_frac=0.1, log=print):
    """Train a fresh MLP (seeded initial parameters and batch order, both
    drawn on the host) and return it with its loss history.  The last
    val_frac of the rows (the last cells) is held back as a validation
    split: the parameters of the epoch with the lowest validation loss are
    kept (early stopping; longer training fits noise in the occupation
    entries that the radial descriptor cannot predict)."""
    import torch
    import workloads
    from paper_2507_23612_amd import hcu
    n_all = X.shape[0]
    nv = int(round(n_all * val_frac)) // 8 * 8 if val_frac > 0 else 0   # whole cells (8 sites each)
    Xt, Tt, Xv, Tv = X[:n_all - nv], T[:n_all - nv], X[n_all - nv:], T[n_all - nv:]
    m = hcu.HcuMlp(DIMS, max(batch, 64))
    m.set_params(workloads.mlp_init_params(seed, DIMS))
    Xd = torch.from_numpy(np.ascontiguousarray(Xt)).cuda()
    Td = torch.from_numpy(np.ascontiguousarray(Tt)).cuda()
    m.fit_scaling(Xd, Td)
    rng = np.random.default_rng(seed)
    n = Xt.shape[0]
    hist, vhist = [], []
    best = (np.inf, None, -1)
    for ep in range(epochs):
        perm = rng.permutation(n).astype(np.int32)
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1 if n >= batch else 1, batch):
            idx = torch.from_numpy(perm[b0:b0 + min(batch, n)]).cuda()
            tot += m.train_step(Xd, Td, idx, lr=lr)
            cnt += 1
        hist.append(tot / max(cnt, 1))
        if nv:
            vl = float(standardised_error(m, Xv, Tv, max(batch, 64)).mean())
            vhist.append(vl)
            if vl < best[0]:
                best = (vl, m.get_params(), ep)
        if log and (ep % 50 == 0 or ep == epochs - 1):
            log(f"[mlguess] epoch {ep} loss {hist[-1]:.4e}" + (f" validation {vhist[-1]:.4e}" if nv else ""),
                flush=True)
    if nv:
        m.set_params(best[1])
        log(f"[mlguess] kept epoch {best[2]} (validation loss {best[0]:.4e})", flush=True)
    m.train_info = {"validation_rows": nv, "best_epoch": best[2], "best_validation_loss": best[0],
                    "validation_history": vhist}
    return m, hist


def compare(m, seeds, group=8, tol_d=1e-6, tol_f=1e-7, bf16=True, log=print):
    """SCF from the isolated-atom start and from the learned start on the
    given cells; per-cell iterations, seconds and free energies."""
    from paper_2507_23612_amd import hcu
    out = []
    for g0 in range(0, len(seeds), group):
        chunk = seeds[g0:g0 + group]
        cfgs = [_cell(s) for s in chunk]
        base = [_context(c) for c in cfgs]
        for ctx, cfg in zip(base, cfgs):
            ctx.set_hubbard_occupation(hcu.initial_occupation(ctx, cfg))
        rb, tb = _scf_group(base, tol_d, tol_f)
        learned = [_context(c) for c in cfgs]
        pred = []
        for ctx in learned:
            pred.append(m.guess(ctx, bf16=bf16))
        rl, tl = _scf_group(learned, tol_d, tol_f)
        for i, seed in enumerate(chunk):
            natom = len(cfgs[i]["atom_species"])
            targets = base[i].site_targets()
            shells_true = targets[:, 15:]
            out.append({"seed": int(seed), "it_atomic": int(rb[i]["iterations"]),
                        "it_learned": int(rl[i]["iterations"]),
                        "conv_atomic": bool(rb[i]["converged"]), "conv_learned": bool(rl[i]["converged"]),
                        "F_atomic": rb[i]["F"], "F_learned": rl[i]["F"],
                        "dF_per_atom": abs(rb[i]["F"] - rl[i]["F"]) / natom,
                        "pred": np.asarray(pred[i], np.float64).tolist(),
                        "target": np.asarray(targets, np.float64).tolist(),
                        "shell_rel_err": float(np.abs(pred[i][:, 15:] - shells_true).max()
                                               / np.abs(shells_true).max())})
        out[-1]["group_seconds_atomic"] = tb
        out[-1]["group_seconds_learned"] = tl
        for ctx in base + learned:
            ctx.close()
        log(f"[mlguess] compared {min(g0 + group, len(seeds))}/{len(seeds)} cells", flush=True)
    return out


def save_model(m, path):
    """Parameters and scaling of a trained site MLP, with its layer widths."""
    in_mean, in_sd, out_mean, out_sd = m.get_scaling()
    np.savez(path, dims=np.array(m.dims, np.int32), params=m.get_params(), in_mean=in_mean, in_sd=in_sd,
             out_mean=out_mean, out_sd=out_sd)


def load_model(path, max_batch=64):
    """A bound site MLP from a file written by save_model."""
    from paper_2507_23612_amd import hcu
    z = np.load(path)
    m = hcu.HcuMlp(tuple(int(d) for d in z["dims"]), max_batch)
    m.set_params(z["params"])
    m.set_scaling(z["in_mean"], z["in_sd"], z["out_mean"], z["out_sd"])
    return m


def fit_summary(rows):
    """Held-out fit of the BF16 predictions: R^2 per output group (against
    the held-out variance of each output, averaged over the group) and the
    rms error of the occupation-matrix entries."""
    P = np.concatenate([np.asarray(r["pred"]) for r in rows])
    T = np.concatenate([np.asarray(r["target"]) for r in rows])
    r2 = 1.0 - ((P - T) ** 2).mean(0) / T.var(0)
    diag = [0, 5, 9, 12, 14]                   # (m, m) entries of the row-major upper triangle of a 5x5 D
    pooled = 1.0 - ((P[:, :15] - T[:, :15]) ** 2).sum() / (T[:, :15].var(0).sum() * P.shape[0])
    return {"r2_D_mean": float(r2[:15].mean()), "r2_shells_mean": float(r2[15:].mean()),
            "r2_D_diagonal_mean": float(r2[diag].mean()), "r2_D_pooled": float(pooled),
            "r2_D": [float(v) for v in r2[:15]],
            "rms_err_D": float(np.sqrt(((P[:, :15] - T[:, :15]) ** 2).mean())),
            "rms_D_about_mean": float(np.sqrt(T[:, :15].var(0).mean()))}


def summarise(rows):
    ia = np.array([r["it_atomic"] for r in rows], float)
    il = np.array([r["it_learned"] for r in rows], float)
    ta = sum(r.get("group_seconds_atomic", 0.0) for r in rows)
    tl = sum(r.get("group_seconds_learned", 0.0) for r in rows)
    return {"cells": len(rows), "iterations_atomic_mean": float(ia.mean()),
            "iterations_learned_mean": float(il.mean()),
            "iterations_saved_fraction": float(1 - il.sum() / ia.sum()),
            "cells_fewer_iterations": int((il < ia).sum()), "cells_more_iterations": int((il > ia).sum()),
            "scf_seconds_atomic": ta, "scf_seconds_learned": tl,
            "max_dF_per_atom": float(max(r["dF_per_atom"] for r in rows)),
            "all_converged": bool(all(r["conv_atomic"] and r["conv_learned"] for r in rows)),
            "max_shell_rel_err": float(max(r["shell_rel_err"] for r in rows))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=2000, help="training cells")
    ap.add_argument("--seed0", type=int, default=TRAIN_SEED0, help="first training cell seed")
    ap.add_argument("--heldout", type=int, default=200, help="held-out cells (seeds 3000..)")
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--val-frac", type=float, default=0.1,
                    help="fraction of the training cells held back for early stopping (0: none)")
    ap.add_argument("--gen-only", action="store_true", help="generate and save training data, then stop")
    ap.add_argument("--data", default=None,
                    help="comma-separated npz files with X, T from earlier runs (skips generation)")
    ap.add_argument("--save-data", default=None)
    ap.add_argument("--save-model", default=None, help="write the trained network (npz)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    t0 = time.perf_counter()
    if args.data:
        zs = [np.load(f) for f in args.data.split(",")]
        X = np.concatenate([z["X"] for z in zs])
        T = np.concatenate([z["T"] for z in zs])
        gen = {"cells": int(sum(int(z["ncells"]) for z in zs)), "sites": int(X.shape[0]),
               "seconds": float(sum(float(z["seconds"]) for z in zs)),
               "iterations_mean": float(np.mean(np.concatenate([z["iterations"] for z in zs])))}
    else:
        X, T, cells = generate(list(range(args.seed0, args.seed0 + args.train)))
        its = np.array([c["iterations"] for c in cells])
        gen = {"cells": len(cells), "sites": int(X.shape[0]), "seconds": time.perf_counter() - t0,
               "iterations_mean": float(its.mean())}
        if args.save_data:
            np.savez(args.save_data, X=X, T=T, ncells=len(cells), seconds=gen["seconds"], iterations=its)
        if args.gen_only:
            print(json.dumps({"data": gen}), flush=True)
            return
    t1 = time.perf_counter()
    m, hist = train(X, T, epochs=args.epochs, val_frac=args.val_frac)
    t_train = time.perf_counter() - t1
    if args.save_model:
        save_model(m, args.save_model)
    rows = compare(m, list(range(HELDOUT_SEED0, HELDOUT_SEED0 + args.heldout))) if args.heldout > 0 else []
    info = getattr(m, "train_info", {})
    res = {"data": gen, "train": {"samples": int(X.shape[0]), "epochs": args.epochs, "seconds": t_train,
                                   "loss_first": hist[0], "loss_last": hist[-1],
                                   "validation_rows": info.get("validation_rows"),
                                   "best_epoch": info.get("best_epoch"),
                                   "best_validation_loss": info.get("best_validation_loss")},
           "heldout": summarise(rows) if rows else None,
           "heldout_fit": fit_summary(rows) if rows else None,
           "rows": [{k: v for k, v in r.items() if k not in ("pred", "target")} for r in rows]}
    print(json.dumps({k: v for k, v in res.items() if k != "rows"}), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
