"""Exhaustive minimiser of the CONCORD objective for tiny p (p <= 4).

Independent of the oracle's coordinate descent: F(Omega) = -sum log omega_ii
+ 1/2 tr(Omega S Omega) + lam sum_{i<j} |omega_ij| is smooth once the sign of
every off-diagonal is fixed.  For each of the 3^(p(p-1)/2) sign patterns
(negative, zero, positive) this solves the smooth restricted problem by a
damped Newton method, keeps the solutions whose signs agree with the pattern
and whose zero entries satisfy the subgradient bound |G_ij| <= lam, and
returns the one with the smallest F.  With S positive definite F is strictly
convex, so that is the unique minimiser.
"""
import itertools

import numpy as np


def _basis(p, free):
    mats = []
    for i in range(p):
        e = np.zeros((p, p))
        e[i, i] = 1.0
        mats.append(e)
    for (i, j) in free:
        e = np.zeros((p, p))
        e[i, j] = e[j, i] = 1.0
        mats.append(e)
    return mats


def _F(S, om, lam):
    d = np.diag(om)
    if np.any(d <= 0):
        return np.inf
    return -np.log(d).sum() + 0.5 * np.trace(om @ S @ om) + lam * np.abs(np.triu(om, 1)).sum()


def _solve_pattern(S, lam, pairs, signs):
    p = S.shape[0]
    free = [pr for pr, s in zip(pairs, signs) if s != 0]
    sg = np.array([s for s in signs if s != 0], dtype=float)
    E = _basis(p, free)
    nv = len(E)
    # Hessian of the quadratic part: tr(E_a S E_b).
    Hq = np.array([[np.trace(E[a] @ S @ E[b]) for b in range(nv)] for a in range(nv)])
    x = np.zeros(nv)
    x[:p] = 1.0 / np.sqrt(np.diag(S))

    def assemble(x):
        return sum(x[k] * E[k] for k in range(nv))

    def fsmooth(x):
        om = assemble(x)
        d = x[:p]
        if np.any(d <= 0):
            return np.inf
        return -np.log(d).sum() + 0.5 * np.trace(om @ S @ om) + lam * float(sg @ x[p:])

    for _ in range(200):
        om = assemble(x)
        so = om @ S
        g = np.array([np.trace(E[k] @ so) for k in range(nv)])   # tr(E_k Omega S)
        g[:p] += -1.0 / x[:p]
        g[p:] += lam * sg
        H = Hq.copy()
        H[np.arange(p), np.arange(p)] += 1.0 / x[:p] ** 2
        step = -np.linalg.solve(H, g)
        if np.max(np.abs(g)) < 1e-14:
            break
        f0, t = fsmooth(x), 1.0
        # Close to the minimiser take the full Newton step: F differences are
        # then below rounding and a sufficient-decrease test cannot see them.
        near = np.max(np.abs(g)) < 1e-6 and np.all(x[:p] + step[:p] > 0)
        while not near and t > 1e-12:
            xn = x + t * step
            if np.all(xn[:p] > 0) and fsmooth(xn) <= f0 + 1e-4 * t * float(g @ step):
                break
            t *= 0.5
        x = x + t * step
        if t * np.max(np.abs(step)) < 1e-16:
            break
    return assemble(x), x[p:], sg


def brute_force(S, lam):
    """Exact minimiser of F for p <= 4 (S positive definite)."""
    S = np.asarray(S, dtype=float)
    p = S.shape[0]
    assert p <= 4
    pairs = [(i, j) for i in range(p) for j in range(i + 1, p)]
    best, best_f = None, np.inf
    for signs in itertools.product((-1, 0, 1), repeat=len(pairs)):
        om, xo, sg = _solve_pattern(S, lam, pairs, signs)
        if np.any(xo * sg <= 0):
            continue
        so = S @ om
        G = so + so.T
        ok = True
        for (i, j), s in zip(pairs, signs):
            if s == 0 and abs(G[i, j]) > lam * (1 + 1e-9) + 1e-12:
                ok = False
                break
        if not ok:
            continue
        f = _F(S, om, lam)
        if f < best_f:
            best, best_f = om, f
    return best, best_f
