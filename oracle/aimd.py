"""Initial occupation matrices along an ab initio molecular-dynamics
trajectory (Sec. II.B: the occupation matrix is split into the isolated-atom
guess and a residual, and the residual at the next time step is a
second-order extrapolation, as for the electron density in the scheme the
paper cites).

TEST INFRASTRUCTURE ONLY (see the oracle package header).

The extrapolation coefficients come from the atomic trajectory:
    R(t+dt) - R(t) ~ a (R(t) - R(t-dt)) + b (R(t-dt) - R(t-2dt)),
fitted over all atoms by least squares (numpy's minimum-norm solver), and
the residual D - D_atomic is carried forward with the same a, b:
    D(t+dt) = D_atomic + r(t) + a (r(t) - r(t-dt)) + b (r(t-dt) - r(t-2dt)).
With fewer recorded steps the scheme drops to first order (b = 0) or keeps
the last residual (a = b = 0).

Pins (tests/test_oracle_aimd.py): a trajectory quadratic in time gives
a = 2, b = -1 and then reproduces any occupation matrix quadratic in time
exactly; a linear trajectory (the two steps parallel) gives the
minimum-norm a = b = 1/2, exact for linear D; the isolated-atom part cancels.
"""
from __future__ import annotations

import numpy as np


def extrapolation_coefficients(R_new, R_hist):
    """(a, b) from the new positions and the recorded ones (most recent
    first), each (natom, 3)."""
    nh = len(R_hist)
    if nh < 2:
        return 0.0, 0.0
    r = (np.asarray(R_new) - np.asarray(R_hist[0])).ravel()
    x1 = (np.asarray(R_hist[0]) - np.asarray(R_hist[1])).ravel()
    if nh < 3:
        sol, *_ = np.linalg.lstsq(x1[:, None], r, rcond=None)
        return float(sol[0]), 0.0
    x2 = (np.asarray(R_hist[1]) - np.asarray(R_hist[2])).ravel()
    sol, *_ = np.linalg.lstsq(np.stack([x1, x2], axis=1), r, rcond=None)
    return float(sol[0]), float(sol[1])


def extrapolate_occupation(D_hist, a, b, D_atomic=0.0):
    """D(t+dt) from the recorded occupation matrices (most recent first)."""
    r = [np.asarray(D) - D_atomic for D in D_hist]
    out = r[0].copy()
    if len(r) >= 2:
        out = out + a * (r[0] - r[1])
    if len(r) >= 3:
        out = out + b * (r[1] - r[2])
    return D_atomic + out
