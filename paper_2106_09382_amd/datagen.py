"""Seeded synthetic workloads for CONCORD-PCD.

This module draws inputs only. It holds none of the solver's arithmetic: it
builds a true precision matrix Omega0 and samples a data matrix Y whose rows
are iid N(0, Omega0^{-1}). Forming S = Y^T Y / n is the solver's first step
and is left to whoever consumes Y (the HIP path's Gram kernel, or the CPU
oracle's own Gram).

Workloads (the paper's simulations, Section 5, draw data from N_p(0, Omega^{-1});
its AR(2) and scale-free generators are replaced here by a chain graph and an
Erdos-Renyi graph):

* ``chain``: omega_ii = 1, omega_{i,i+1} = omega_{i+1,i} = 0.4.
* ``er``: each pair i<j is an edge with probability 3/p; an edge weight is
  U[0.3, 0.5] with a random sign. With A the weighted adjacency matrix,
  Omega0 = A + (0.1 - lambda_min(A)) I, then rescaled to unit diagonal.

Every draw comes from ``numpy.random.default_rng(seed)`` (PCG64) in a fixed
order, so a (config, replicate) pair always yields the same bytes.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import cholesky, eigh, solve_triangular

__all__ = [
    "chain_precision",
    "er_precision",
    "sample_y",
    "standardise_columns",
    "problem",
    "batched_problems",
    "joint_problem",
    "lambda_path",
    "CONFIGS",
]


def chain_precision(p: int, diag: float = 1.0, off: float = 0.4) -> np.ndarray:
    """Tridiagonal chain-graph precision matrix (positive definite for |off| < diag/2)."""
    om = np.zeros((p, p))
    om[np.arange(p), np.arange(p)] = diag
    if p > 1:
        k = np.arange(p - 1)
        om[k, k + 1] = off
        om[k + 1, k] = off
    return om


def er_precision(p: int, rng: np.random.Generator, edge_prob: float | None = None,
                 wlo: float = 0.3, whi: float = 0.5, lam_min: float = 0.1) -> np.ndarray:
    """Erdos-Renyi precision matrix with unit diagonal.

    Draw order: one uniform per pair i<j in row-major order (edge test), then
    one magnitude U[wlo, whi] and one fair sign per edge, in the same order.
    The diagonal shift puts lambda_min at ``lam_min`` before the rescale to
    unit diagonal; afterwards lambda_min is lam_min / d with d the shift.
    """
    return _unit_diagonal(_er_adjacency(p, rng, edge_prob, wlo, whi), lam_min)


def _er_adjacency(p, rng, edge_prob, wlo, whi):
    if edge_prob is None:
        edge_prob = 3.0 / p
    iu, ju = np.triu_indices(p, 1)
    mask = rng.random(iu.shape[0]) < edge_prob
    iu, ju = iu[mask], ju[mask]
    mag = rng.uniform(wlo, whi, size=iu.shape[0])
    sgn = np.where(rng.random(iu.shape[0]) < 0.5, -1.0, 1.0)
    a = np.zeros((p, p))
    a[iu, ju] = mag * sgn
    a[ju, iu] = mag * sgn
    return a


def _unit_diagonal(a, lam_min):
    p = a.shape[0]
    if p == 1:
        lmin = 0.0
    else:
        lmin = float(eigh(a, eigvals_only=True, subset_by_index=[0, 0])[0])
    d = lam_min - lmin
    om = a.copy()
    om[np.arange(p), np.arange(p)] += d
    return om / d


def sample_y(omega0: np.ndarray, n: int, rng: np.random.Generator) -> np.ndarray:
    """n iid rows from N(0, omega0^{-1}): Y = Z L^{-1} with omega0 = L L^T."""
    p = omega0.shape[0]
    low = cholesky(omega0, lower=True)
    z = rng.standard_normal((n, p))
    # Y^T = L^{-T} Z^T, so each row has covariance L^{-T} L^{-1} = omega0^{-1}.
    return np.ascontiguousarray(solve_triangular(low.T, z.T, lower=False).T)


def standardise_columns(y: np.ndarray) -> np.ndarray:
    """Centre every column and scale it to unit variance (1/n convention)."""
    y = y - y.mean(axis=0, keepdims=True)
    return y / np.sqrt((y * y).mean(axis=0, keepdims=True))


def lambda_path(hi: float = 0.5, lo: float = 0.05, k: int = 16) -> np.ndarray:
    """Descending log-spaced penalty path."""
    return np.geomspace(hi, lo, k)


# Named workloads. ``graph`` picks the true precision matrix; ``standardise``
# applies to the data matrix only (the solver never preprocesses).
CONFIGS = {
    1: dict(p=64, n=100, graph="chain", standardise=True, lam=0.3, tol=1e-8, maxit=500),
    2: dict(p=1001, n=500, graph="er", standardise=False, lam=0.2, tol=1e-7, maxit=500),
    3: dict(p=5000, n=2000, graph="er", standardise=False, lam=0.1, tol=1e-6, maxit=500),
    5: dict(p=2000, n=1000, graph="chain", standardise=False, lam=0.15, tol=1e-8, maxit=500),
}


def problem(config: int, replicate: int = 0, *, graph: str | None = None,
            p: int | None = None, n: int | None = None) -> dict:
    """Draw one workload. Seed = 1000 * config + replicate.

    ``graph``, ``p`` and ``n`` override the config's values (the config's
    seed is kept), which gives the small variants used by tests.
    Returns a dict with ``omega0``, ``y`` (n x p, C-contiguous float64) and
    the config's solver settings.
    """
    spec = dict(CONFIGS[config])
    if graph is not None:
        spec["graph"] = graph
    if p is not None:
        spec["p"] = p
    if n is not None:
        spec["n"] = n
    seed = 1000 * config + replicate
    rng = np.random.default_rng(seed)
    pp, nn = spec["p"], spec["n"]
    if spec["graph"] == "chain":
        om0 = chain_precision(pp)
    elif spec["graph"] == "er":
        om0 = er_precision(pp, rng)
    else:
        raise ValueError(f"unknown graph {spec['graph']!r}")
    y = sample_y(om0, nn, rng)
    if spec["standardise"]:
        y = standardise_columns(y)
    spec.update(seed=seed, omega0=om0, y=np.ascontiguousarray(y))
    return spec


def batched_problems(replicate: int = 0, count: int = 64, p_lo: int = 200,
                     p_hi: int = 3000) -> list[dict]:
    """Independent Erdos-Renyi problems with p ~ U{p_lo..p_hi} and n = round(p/2).

    The seed sequence 4000 + replicate is split into count + 1 children: the
    first draws the sizes, child b + 1 draws problem b.
    """
    ss = np.random.SeedSequence(4000 + replicate)
    kids = ss.spawn(count + 1)
    sizes = np.random.default_rng(kids[0]).integers(p_lo, p_hi + 1, size=count)
    out = []
    for b in range(count):
        rng = np.random.default_rng(kids[b + 1])
        pb = int(sizes[b])
        nb = int(round(0.5 * pb))
        om0 = er_precision(pb, rng)
        y = sample_y(om0, nb, rng)
        out.append(dict(p=pb, n=nb, graph="er", omega0=om0, y=y))
    return out


def joint_problem(replicate: int = 0, p: int = 5000, n: int = 2000, changed: float = 0.1,
                  wlo: float = 0.3, whi: float = 0.5) -> dict:
    """Two populations whose graphs differ in a few edges (a differential network).

    Population 1 is an Erdos-Renyi precision matrix as in ``er_precision``.
    Population 2 keeps its edges and weights except round(changed * |E|)
    edges, chosen uniformly, which are deleted, and as many new edges between
    unconnected pairs, with weights U[wlo, whi] and random signs.  Each
    adjacency matrix is shifted and rescaled to unit diagonal separately, and
    each population draws its own n rows.  Seed 6000 + replicate; draw order:
    population 1's graph, the deleted edges, the new pairs, their magnitudes
    and signs, then Y_1, then Y_2.
    """
    rng = np.random.default_rng(6000 + replicate)
    a1 = _er_adjacency(p, rng, None, wlo, whi)
    iu, ju = np.triu_indices(p, 1)
    edge = a1[iu, ju] != 0
    eidx = np.flatnonzero(edge)
    k = int(round(changed * eidx.size))
    gone = rng.choice(eidx, size=k, replace=False) if k else np.zeros(0, dtype=np.int64)
    free = np.flatnonzero(~edge)
    new = rng.choice(free, size=k, replace=False) if k else np.zeros(0, dtype=np.int64)
    mag = rng.uniform(wlo, whi, size=k)
    sgn = np.where(rng.random(k) < 0.5, -1.0, 1.0)
    a2 = a1.copy()
    a2[iu[gone], ju[gone]] = 0.0
    a2[ju[gone], iu[gone]] = 0.0
    a2[iu[new], ju[new]] = mag * sgn
    a2[ju[new], iu[new]] = mag * sgn
    om1, om2 = _unit_diagonal(a1, 0.1), _unit_diagonal(a2, 0.1)
    y1 = sample_y(om1, n, rng)
    y2 = sample_y(om2, n, rng)
    return dict(p=p, n=n, changed=changed, omega0=(om1, om2), y=(y1, y2),
                seed=6000 + replicate)
