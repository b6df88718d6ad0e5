"""Pins for two oracle helpers that every parity test leans on.

* ``oracle.objective``: eq. (1) of Section 2.1 divided by n (the S scale),
  F(Omega) = -sum_i log omega_ii + 1/2 tr(Omega S Omega) + lam sum_{i<j} |omega_ij|.
  Pinned by values the definition fixes by hand (Omega = I, diagonal Omega,
  a 2 x 2 Omega with the trace written out), by the brute-force minimisers
  of ``bruteforce.py`` (no direction may lower F there), and by the
  symmetry of the penalty.
* ``oracle.borderline_pairs``: the pairs whose eq. (3) numerator sits within
  rel (S_ii + S_jj) of lam (reading R11: the support decision there is left to
  rounding).  Pinned on constructed S and Omega whose numerators are known by
  hand, and by the claim that the tested workloads have none in FP64.

Each pin set is a function that returns the list of pins an implementation
fails, so that planted mistakes (a dropped 1/2, the penalty on both
triangles, a missing log term, a dropped or doubled term in the numerator)
can be shown to fail them.
"""
import numpy as np
import pytest

import oracle
from bruteforce import brute_force
from paper_2106_09382_amd import datagen


# ---------------------------------------------------------------- objective

def _tiny_S(p, seed, n=40):
    rng = np.random.default_rng(100 + seed)
    a = rng.normal(size=(p, p))
    cov = a @ a.T + p * np.eye(p)
    y = rng.multivariate_normal(np.zeros(p), cov, size=n)
    return oracle.gram(y)


_BF_CASES = [(3, 1, 0.05), (3, 2, 0.3), (4, 3, 0.1), (4, 5, 0.02)]
_BF = {}


def _bf(case):
    if case not in _BF:
        p, seed, lam = case
        S = _tiny_S(p, seed)
        om, _ = brute_force(S, lam)
        _BF[case] = (S, om, lam)
    return _BF[case]


def _objective_failures(F) -> list:
    bad = []
    rng = np.random.default_rng(7)
    # Omega = I: the log terms and the penalty vanish, F = tr(S) / 2.
    S = _tiny_S(5, 9)
    if abs(F(S, np.eye(5), 0.3) - 0.5 * np.trace(S)) > 1e-13 * np.trace(S):
        bad.append("identity")
    # Omega = diag(d): F = -sum log d_i + 1/2 sum_i S_ii d_i^2, for any lam.
    d = rng.uniform(0.5, 2.0, size=5)
    want = -np.log(d).sum() + 0.5 * float((np.diag(S) * d * d).sum())
    if abs(F(S, np.diag(d), 0.7) - want) > 1e-13 * abs(want):
        bad.append("diagonal")
    # p = 2 written out: with S = [[s1, r], [r, s2]] and Omega = [[a, b], [b, c]],
    # (Omega S Omega)_11 = s1 a^2 + 2 r a b + s2 b^2 and
    # (Omega S Omega)_22 = s1 b^2 + 2 r b c + s2 c^2.
    for (s1, s2, r, a, b, c, lam) in [(1.3, 0.8, 0.4, 1.1, -0.3, 0.9, 0.2),
                                      (2.0, 1.0, -0.6, 0.7, 0.25, 1.4, 0.05),
                                      (1.0, 1.0, 0.0, 1.0, 0.5, 1.0, 1.0)]:
        S2 = np.array([[s1, r], [r, s2]])
        om = np.array([[a, b], [b, c]])
        tr = s1 * a * a + 2 * r * a * b + s2 * b * b + s1 * b * b + 2 * r * b * c + s2 * c * c
        want = -np.log(a) - np.log(c) + 0.5 * tr + lam * abs(b)
        if abs(F(S2, om, lam) - want) > 1e-14 * max(1.0, abs(want)):
            bad.append(f"p2 {s1, s2, r, a, b, c, lam}")
    # The penalty sees |omega_ij|: with r = 0 the sign of b cannot matter.
    S2 = np.diag([1.5, 0.7])
    om = np.array([[1.0, 0.4], [0.4, 1.2]])
    omn = np.array([[1.0, -0.4], [-0.4, 1.2]])
    if F(S2, om, 0.3) != pytest.approx(F(S2, omn, 0.3), rel=1e-15):
        bad.append("penalty sign")
    # A non-positive diagonal is outside the domain of -log.
    if not np.isinf(F(S2, np.diag([1.0, 0.0]), 0.1)):
        bad.append("domain")
    # The brute-force minimiser (found by an independent exhaustive search
    # over sign patterns) minimises F: no small symmetric change lowers it.
    for case in _BF_CASES:
        Sb, omb, lam = _bf(case)
        p = Sb.shape[0]
        f0 = F(Sb, omb, lam)
        for _ in range(40):
            E = rng.normal(size=(p, p))
            E = (E + E.T) / 2
            for eps in (1e-4, -1e-4):
                if F(Sb, omb + eps * E, lam) < f0 - 1e-13 * max(1.0, abs(f0)):
                    bad.append(f"not minimal at brute force {case}")
                    break
            else:
                continue
            break
    return bad


def _quad(S, om):
    return float(np.trace(om @ S @ om))


def test_objective_pins():
    assert _objective_failures(oracle.objective) == []


@pytest.mark.parametrize("name,mutant", [
    ("dropped 1/2", lambda S, om, lam: oracle.objective(S, om, lam) + 0.5 * _quad(S, om)),
    ("penalty on both triangles",
     lambda S, om, lam: oracle.objective(S, om, lam) + lam * np.abs(np.triu(om, 1)).sum()),
    ("missing log term",
     lambda S, om, lam: (oracle.objective(S, om, lam) + np.log(np.diag(om)).sum()
                         if np.all(np.diag(om) > 0) else np.inf)),
    ("penalty with sign",
     lambda S, om, lam: (oracle.objective(S, om, lam) - lam * np.abs(np.triu(om, 1)).sum()
                         + lam * np.triu(om, 1).sum())),
    ("Omega S instead of Omega S Omega",
     lambda S, om, lam: (oracle.objective(S, om, lam) - 0.5 * _quad(S, om)
                         + 0.5 * float(np.trace(om @ S)))),
])
def test_objective_planted_mistakes_fail_a_pin(name, mutant):
    assert _objective_failures(mutant) != [], name


def test_objective_equals_bruteforce_value():
    # bruteforce._F is a separate transcription (trace of the triple product);
    # the two agree at the minimisers the exhaustive search returns.
    from bruteforce import _F
    for case in _BF_CASES:
        Sb, omb, lam = _bf(case)
        assert oracle.objective(Sb, omb, lam) == pytest.approx(_F(Sb, omb, lam), rel=1e-14)


# ---------------------------------------------------------------- borderline pairs

def _numerator_by_sums(S, om, i, j):
    # eq. (3): b_ij = sum_{u != j} omega_iu S_ju + sum_{u != i} omega_uj S_iu
    p = S.shape[0]
    return (sum(om[i, u] * S[j, u] for u in range(p) if u != j)
            + sum(om[u, j] * S[i, u] for u in range(p) if u != i))


def _as_set(arr):
    return {(int(a), int(b)) for a, b in arr}


def _borderline_failures(fn) -> list:
    bad = []
    lam, rel = 0.2, 1e-9
    # Omega = I: b_ij = 2 S_ij.  Unit diagonal, so the band is 2 rel wide.
    S = np.eye(4)
    S[0, 1] = lam / 2 * (1 + 1e-12)       # |b| - lam = 2e-13: inside
    S[0, 2] = -lam / 2 * (1 - 1e-12)      # negative numerator, inside
    S[0, 3] = (lam + 3e-9) / 2            # 3e-9 > 2e-9: outside
    S[1, 2] = 0.3 * lam                   # far away
    S[1, 3] = (lam + 1e-9) / 2            # 1e-9 < 2e-9: inside
    S[2, 3] = 0.0
    S = np.triu(S, 1) + np.triu(S, 1).T + np.eye(4)
    if _as_set(fn(S, np.eye(4), lam, rel)) != {(0, 1), (0, 2), (1, 3)}:
        bad.append("identity")
    # With omega_01 = w the numerator of (0, 1) leaves out its own entry
    # (b_01 = 2 S_01 whatever w is), while b_02 = 2 S_02 + w S_12.
    w = 0.7
    om = np.eye(3)
    om[0, 1] = om[1, 0] = w
    S3 = np.eye(3)
    S3[0, 1] = S3[1, 0] = lam / 2 * (1 - 1e-13)
    S3[1, 2] = S3[2, 1] = 0.25
    S3[0, 2] = S3[2, 0] = (lam * (1 + 1e-13) - w * 0.25) / 2
    for (i, j) in [(0, 1), (0, 2)]:
        if abs(abs(_numerator_by_sums(S3, om, i, j)) - lam) > 1e-12:
            bad.append("construction")
    if _as_set(fn(S3, om, lam, rel)) != {(0, 1), (0, 2)}:
        bad.append("off-diagonal omega")
    # Omega = diag(d): b_ij = S_ij (d_i + d_j), so unequal d_i, d_j tell
    # W_ij + W_ji apart from 2 W_ij; and the band scales with S_ii + S_jj.
    d = np.array([1.0, 3.0, 0.5])
    S4 = np.diag([3.0, 1.0, 1.0])
    S4[0, 1] = S4[1, 0] = (lam + 3e-9) / (d[0] + d[1])    # 3e-9 < 4e-9 (S_00 + S_11 = 4)
    S4[1, 2] = S4[2, 1] = (lam + 3e-9) / (d[1] + d[2])    # 3e-9 > 2e-9: outside
    S4[0, 2] = S4[2, 0] = lam * (1 - 1e-13) / (d[0] + d[2])  # 4e-9 band: inside
    if _as_set(fn(S4, np.diag(d), lam, rel)) != {(0, 1), (0, 2)}:
        bad.append("diagonal omega")
    return bad


def test_borderline_pins():
    assert _borderline_failures(oracle.borderline_pairs) == []


def _bl_mutant(numerator, scale_by_diag=True):
    def fn(S, om, lam, rel):
        so = S @ om
        dS = np.diag(S)
        b = numerator(S, om, so, dS)
        band = rel * ((dS[:, None] + dS[None, :]) if scale_by_diag else 2.0)
        near = np.abs(np.abs(b) - lam) < band
        iu = np.triu_indices(S.shape[0], 1)
        sel = near[iu]
        return np.stack([iu[0][sel], iu[1][sel]], axis=1)
    return fn


_RIGHT = lambda S, om, so, dS: so + so.T - (dS[:, None] + dS[None, :]) * om  # noqa: E731


@pytest.mark.parametrize("name,mutant", [
    ("own entry not removed", _bl_mutant(lambda S, om, so, dS: so + so.T)),
    ("2 W_ij for W_ij + W_ji",
     _bl_mutant(lambda S, om, so, dS: 2 * so - (dS[:, None] + dS[None, :]) * om)),
    ("own entry added instead of removed",
     _bl_mutant(lambda S, om, so, dS: so + so.T + (dS[:, None] + dS[None, :]) * om)),
    ("band not scaled by S_ii + S_jj", _bl_mutant(_RIGHT, scale_by_diag=False)),
])
def test_borderline_planted_mistakes_fail_a_pin(name, mutant):
    # the correct numerator through the same harness passes
    assert _borderline_failures(_bl_mutant(_RIGHT)) == []
    assert _borderline_failures(mutant) != [], name


def test_no_borderline_pairs_on_small_workloads():
    # Reading R11's claim for FP64: no pair of the converged oracle solution
    # of workloads 1 and 2 sits within 1e-9 (S_ii + S_jj) of lam.
    for cfg in (1, 2):
        pr = datagen.problem(cfg)
        S = oracle.gram(pr["y"])
        om, info, _ = oracle.pcd(S, pr["lam"], pr["tol"], pr["maxit"])
        assert info["converged"]
        assert oracle.borderline_pairs(S, om, pr["lam"], 1e-9).shape[0] == 0, cfg
