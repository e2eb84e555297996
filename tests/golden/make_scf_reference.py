"""Write the oracle's self-consistent result for a benchmark configuration
(Sec. II.B: ChFSI + Pulay SCF of the model DFT+U problem) to
tests/golden/scf_reference_<config>.json.

Calls the oracle only (FP64 NumPy): the stored values are the oracle's, from
the seeded synthetic inputs of `workloads`.  The c2 run (48 atoms, 72x72x96,
256 states) takes several hours on 8 host cores (more than six when the cores
are shared with other work).

    python tests/golden/make_scf_reference.py c2
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import scf as oscf  # noqa: E402


def main(name):
    cfg = workloads.make_config(name)
    t0 = time.perf_counter()
    r = oscf.scf(cfg, verbose=True)
    sec = time.perf_counter() - t0
    out = {
        "config": name,
        "what": "oracle SCF (FP64, NumPy) of the seeded synthetic configuration; stopping rule "
                f"|D_out - D_in|_F < {cfg['scf_tol_d']} and |dF|/atom < {cfg['scf_tol_f']} Ha",
        "natom": int(len(cfg["atom_species"])),
        "converged": bool(r["converged"]),
        "iterations": int(r["iterations"]),
        "F": float(r["F"]),
        "E_U": float(r["E_U"]),
        "e_band": float(r["e_band"]),
        "mu": float(r["mu"]),
        "eigenvalues": [float(x) for x in np.asarray(r["eigs"])[0, 0]],
        "D": [[[float(v) for v in row] for row in np.real(np.asarray(d))] for d in r["D"][0]],
        "F_history": [float(h["F"]) for h in r["history"]],
        "oracle_seconds": sec,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"scf_reference_{name}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"wrote {path}: F = {out['F']:.12f} Ha after {out['iterations']} iterations, {sec:.0f} s")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c2")
