"""Active-set CONCORD-PCD.  TEST INFRASTRUCTURE ONLY.

Theorem 2's argument (Section 4) holds for any edge colouring of K_p.  The
active-set scheme alternates:

1. one full sweep of Algorithm 1 (the round-robin colouring, all pairs, then
   the diagonal); stop when its delta < tol (the paper's rule) or after
   maxit full sweeps;
2. the support A = {i < j : omega_ij != 0} of the result is coloured
   greedily -- pairs in lexicographic order, each taking the smallest colour
   that neither endpoint has used -- and sweeps over those colour classes
   (then the diagonal) run until their delta < tol or active_maxit of them;
   pairs outside A keep the value 0 meanwhile.

A colour class of A has far fewer colours than K_p when A is sparse, so an
active sweep is a short chain of parallel steps.  The result satisfies the
same stopping rule as Algorithm 1 (a full sweep that moved nothing by tol).
"""
from __future__ import annotations

import numpy as np

from . import pcd, pcd_colouring


def greedy_colouring(pairs):
    """Colour the edges (i, j), i < j, in lexicographic order: each edge takes
    the smallest colour used by neither endpoint.  Returns the classes."""
    used = {}
    classes = []
    for i, j in sorted((int(a), int(b)) for a, b in pairs):
        ui, uj = used.setdefault(i, set()), used.setdefault(j, set())
        c = 0
        while c in ui or c in uj:
            c += 1
        ui.add(c)
        uj.add(c)
        while len(classes) <= c:
            classes.append([])
        classes[c].append((i, j))
    return classes


def support(omega):
    om = np.asarray(omega)
    iu, ju = np.nonzero(np.triu(om != 0, 1))
    return list(zip(iu.tolist(), ju.tolist()))


def active_set_pcd(S, lam: float, tol: float, maxit: int, active_maxit: int, omega0=None):
    """Returns (Omega, info) with full_sweeps, active_sweeps, phases, converged,
    delta (of the last full sweep), nnz_upper."""
    om = None if omega0 is None else np.array(omega0, dtype=np.float64)
    full = act = phases = 0
    converged = False
    delta = float("inf")
    while full < maxit:
        om, info, _ = pcd(S, lam, tol, 1, omega0=om)
        full += 1
        delta = info["delta"]
        if delta < tol:
            converged = True
            break
        if full >= maxit:
            break
        classes = greedy_colouring(support(om))
        om, ainfo, _ = pcd_colouring(S, lam, tol, active_maxit, classes, omega0=om)
        act += ainfo["sweeps"]
        phases += 1
    nnz = int(np.count_nonzero(np.triu(om, 1)))
    return om, dict(full_sweeps=full, active_sweeps=act, phases=phases, converged=converged,
                    delta=delta, nnz_upper=nnz)
