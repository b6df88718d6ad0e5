"""Joint estimation of two precision matrices (Section 6 of arXiv 2106.09382).
TEST INFRASTRUCTURE ONLY (see the package docstring).

The objective, divided by n (both populations on the S scale):

  F(Omega_1, Omega_2) = sum_m [ -sum_i log omega^m_ii + 1/2 tr(Omega_m S_m Omega_m) ]
                        + lam1 sum_m sum_{i<j} |omega^m_ij|
                        + lam2 sum_{i<=j} |omega^1_ij - omega^2_ij|.

``pcd`` runs block coordinate descent over (omega^1_ij, omega^2_ij) on
Algorithm 1's schedule (in ``concord_oracle.c``, direct sums); ``pair`` and
``diag`` are its exact block minimisers.  ``objective`` and ``kkt`` are plain
definitions written from the objective above, independent of the block
formulas: ``kkt`` measures how far zero is from the subdifferential of F.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import OracleError, _dp, _f64, _load


def pair(a1, b1, a2, b2, lam1, lam2):
    """Minimiser of sum_m [a_m x_m^2 / 2 + b_m x_m + lam1 |x_m|] + lam2 |x_1 - x_2|."""
    out = np.zeros(2)
    _load().oracle_joint_pair(float(a1), float(b1), float(a2), float(b2), float(lam1),
                              float(lam2), _dp(out))
    return float(out[0]), float(out[1])


def diag(s1, c1, s2, c2, lam2):
    """Minimiser over y_m > 0 of sum_m [-log y_m + s_m y_m^2 / 2 + c_m y_m] + lam2 |y_1 - y_2|."""
    out = np.zeros(2)
    _load().oracle_joint_diag(float(s1), float(c1), float(s2), float(c2), float(lam2), _dp(out))
    return float(out[0]), float(out[1])


def pcd(S1, S2, lam1: float, lam2: float, tol: float, maxit: int, omega0=(None, None)):
    """Joint CONCORD-PCD.  Returns (Omega_1, Omega_2, info, delta_trace)."""
    S1, S2 = _f64(S1), _f64(S2)
    p = S1.shape[0]
    if S2.shape != S1.shape:
        raise OracleError("joint pcd: S1 and S2 differ in shape")
    o1, o2 = np.empty((p, p)), np.empty((p, p))
    tr = np.zeros(maxit)
    info = np.zeros(6)
    s1 = None if omega0[0] is None else _f64(omega0[0])
    s2 = None if omega0[1] is None else _f64(omega0[1])
    rc = _load().oracle_joint_pcd(_dp(S1), _dp(S2), p, float(lam1), float(lam2), float(tol),
                                  int(maxit), _dp(s1), _dp(s2), _dp(o1), _dp(o2), _dp(tr),
                                  _dp(info))
    if rc:
        raise OracleError(f"oracle_joint_pcd returned {rc}")
    inf = dict(sweeps=int(info[0]), delta=float(info[1]), converged=bool(info[2]),
               nnz_upper=(int(info[3]), int(info[4])), differ_upper=int(info[5]))
    return o1, o2, inf, tr[: inf["sweeps"]].copy()


def objective(S1, S2, O1, O2, lam1: float, lam2: float) -> float:
    """F(Omega_1, Omega_2) as defined above."""
    tot = 0.0
    for S, O in ((S1, O1), (S2, O2)):
        S, O = _f64(S), _f64(O)
        d = np.diag(O)
        if np.any(d <= 0):
            return float("inf")
        tot += -np.log(d).sum() + 0.5 * float(np.sum((O @ S) * O.T))
        tot += lam1 * float(np.abs(np.triu(O, 1)).sum())
    tot += lam2 * float(np.abs(np.triu(_f64(O1) - _f64(O2))).sum())
    return float(tot)


def _gap(intervals):
    """Distance between the largest lower and the smallest upper end."""
    lo = max(iv[0] for iv in intervals)
    hi = min(iv[1] for iv in intervals)
    return max(0.0, lo - hi)


def kkt(S1, S2, O1, O2, lam1: float, lam2: float) -> dict:
    """How far zero is from the subdifferential of F at (Omega_1, Omega_2).

    Off-diagonal block (i < j), x_m = omega^m_ij: the smooth part has partial
    derivative G^m_ij = (Omega_m S_m + S_m Omega_m)_ij in x_m.  Zero is a
    subgradient iff some u in lam2 d|x_1 - x_2| has -G^1 - u in lam1 d|x_1|
    and -G^2 + u in lam1 d|x_2|: each condition is an interval for u.
    Diagonal block, y_m = omega^m_ii: the smooth part has derivative
    g_m = (S_m Omega_m)_ii - 1 / y_m, and the conditions are u = -g_1,
    u = g_2, u in lam2 d|y_1 - y_2|.  Returns the largest interval gap over
    the pairs and over the diagonal.
    """
    S1, S2, O1, O2 = _f64(S1), _f64(S2), _f64(O1), _f64(O2)
    p = S1.shape[0]
    so1, so2 = S1 @ O1, S2 @ O2
    G1, G2 = so1 + so1.T, so2 + so2.T

    def sub(x, scale):  # the interval scale * d|x|
        if x > 0:
            return (scale, scale)
        if x < 0:
            return (-scale, -scale)
        return (-scale, scale)

    worst_pair = 0.0
    for i in range(p):
        for j in range(i + 1, p):
            x1, x2 = O1[i, j], O2[i, j]
            fu = sub(x1 - x2, lam2)
            s1 = sub(x1, lam1)        # -G1 - u in s1  <=>  u in [-G1 - s1_hi, -G1 - s1_lo]
            s2 = sub(x2, lam1)        # -G2 + u in s2  <=>  u in [G2 + s2_lo, G2 + s2_hi]
            ivs = [fu, (-G1[i, j] - s1[1], -G1[i, j] - s1[0]), (G2[i, j] + s2[0], G2[i, j] + s2[1])]
            worst_pair = max(worst_pair, _gap(ivs))
    worst_diag = 0.0
    for i in range(p):
        y1, y2 = O1[i, i], O2[i, i]
        g1 = so1[i, i] - 1.0 / y1
        g2 = so2[i, i] - 1.0 / y2
        ivs = [sub(y1 - y2, lam2), (-g1, -g1), (g2, g2)]
        worst_diag = max(worst_diag, _gap(ivs))
    return dict(pairs=worst_pair, diag=worst_diag)


def borderline_pairs(S1, S2, O1, O2, lam1: float, lam2: float, rel: float) -> np.ndarray:
    """Pairs i < j whose block update at (Omega_1, Omega_2) takes a decision
    that rounding may flip (the joint analogue of the single solve's
    borderline filter, for reading R22's case order).

    From the eq. (3) numerators b_m and a_m = S^m_ii + S^m_jj of each pair,
    the block minimiser decides, in order: case x_1 > x_2 (the two thresholds
    |b_1 + lam2| and |b_2 - lam2| against lam1, then u_1 > u_2); if not, case
    x_1 < x_2 (|b_1 - lam2|, |b_2 + lam2| against lam1, then v_1 < v_2); if
    not, the fused value (|b_1 + b_2| against 2 lam1).  A pair is borderline
    when a decision it reaches is within rel (a_1 + a_2) of its threshold, or
    a comparison of candidate values within rel (two candidates that are both
    exactly 0 tie under any rounding and do not count).  Returns a (k, 2)
    index array.
    """
    S1, S2, O1, O2 = _f64(S1), _f64(S2), _f64(O1), _f64(O2)
    p = S1.shape[0]
    iu = np.triu_indices(p, 1)
    a, b = [], []
    for S, O in ((S1, O1), (S2, O2)):
        so = S @ O
        d = np.diag(S)
        am = (d[:, None] + d[None, :])[iu]
        a.append(am)
        b.append((so + so.T)[iu] - am * O[iu])
    a1, a2, b1, b2 = a[0], a[1], b[0], b[1]
    width = rel * (a1 + a2)

    def soft(x, t):
        return np.sign(x) * np.maximum(np.abs(x) - t, 0.0)

    def near(x, t):  # a threshold decision |x| vs t within the band
        return np.abs(np.abs(x) - t) < width

    ta1, ta2 = -(b1 + lam2), -(b2 - lam2)
    u1, u2 = soft(ta1, lam1) / a1, soft(ta2, lam1) / a2
    case_a = u1 > u2
    # two candidates that are both exactly 0 (both thresholds clear of their
    # bands) compare equal under any rounding: not a borderline tie
    def tie(x, y):
        return (np.abs(x - y) < rel) & ((x != 0.0) | (y != 0.0))

    flag = near(ta1, lam1) | near(ta2, lam1) | tie(u1, u2)
    tb1, tb2 = -(b1 - lam2), -(b2 + lam2)
    v1, v2 = soft(tb1, lam1) / a1, soft(tb2, lam1) / a2
    case_b = ~case_a & (v1 < v2)
    flag |= ~case_a & (near(tb1, lam1) | near(tb2, lam1) | tie(v1, v2))
    fused = ~case_a & ~case_b
    flag |= fused & near(-(b1 + b2), 2.0 * lam1)
    return np.stack([iu[0][flag], iu[1][flag]], axis=1)


def block_update_at(S1, S2, O1, O2, i: int, j: int, lam1: float, lam2: float):
    """The new (omega^1_ij, omega^2_ij) (i != j) or (omega^1_ii, omega^2_ii)
    (i == j) that one block update would give at (Omega_1, Omega_2): the eq.
    (3) numerators (or eq. (2) sums) as direct sums over rows i and j, then
    the block minimiser.  O(p) per call, for spot checks at any size."""
    S1, S2, O1, O2 = _f64(S1), _f64(S2), _f64(O1), _f64(O2)
    if i == j:
        c = []
        for S, O in ((S1, O1), (S2, O2)):
            row = O[i] * S[i]
            c.append(float(row.sum() - row[i]))
        return diag(S1[i, i], c[0], S2[i, i], c[1], lam2)
    ab = []
    for S, O in ((S1, O1), (S2, O2)):
        # sum_{u != j} omega_iu S_ju + sum_{u != i} omega_uj S_iu
        t1 = O[i] * S[j]
        t2 = O[j] * S[i]
        b = float(t1.sum() - t1[j] + t2.sum() - t2[i])
        ab += [S[i, i] + S[j, j], b]
    return pair(ab[0], ab[1], ab[2], ab[3], lam1, lam2)
