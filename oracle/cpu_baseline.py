"""CPU baseline for the benchmark (``cpu_pcd.c``): CONCORD-PCD (Algorithm 1)
with the maintained product W = Omega S, serial or with the pairs of each
colour spread over OpenMP threads.  TEST INFRASTRUCTURE ONLY (the
benchmark's CPU-baseline leg and the tests); it is not the oracle, which
evaluates eqs. (2)-(3) by direct sums, and the tests pin it to the oracle.
"""
from __future__ import annotations

import numpy as np

from . import OracleError, _dp, _f64, _load


def pcd_wform(S, lam: float, tol: float, maxit: int, threads: int = 0,
              colour_limit: int = 0):
    """Returns (Omega, info): sweeps, delta, converged, steps, moved_pairs,
    moved_diag, threads."""
    S = _f64(S)
    p = S.shape[0]
    om = np.empty((p, p))
    info = np.zeros(7)
    rc = _load().cpu_pcd_wform(_dp(S), p, float(lam), float(tol), int(maxit), int(threads),
                               int(colour_limit), _dp(om), _dp(info))
    if rc:
        raise OracleError(f"cpu_pcd_wform returned {rc}")
    return om, dict(sweeps=int(info[0]), delta=float(info[1]), converged=bool(info[2]),
                    steps=int(info[3]), moved_pairs=int(info[4]), moved_diag=int(info[5]),
                    threads=int(info[6]))
