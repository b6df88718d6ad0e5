"""Pins of the oracle's joint estimation of two precision matrices
(oracle/joint.py, Section 6's fused objective), each against something other
than the oracle's own block formulas:

* The block minimisers (a pair block and a diagonal block) against a
  numerical minimisation of the same 2-variable function, and against the
  subgradient conditions.
* lam2 = 0 decouples the populations: the joint sweeps are two independent
  runs of Algorithm 1 (bit for bit, at a fixed sweep count).
* A large lam2 fuses them: both estimates equal Algorithm 1 on
  (S_1 + S_2) / 2, since F then is twice the CONCORD objective of the mean.
* Identical populations give identical estimates, equal to Algorithm 1 on S.
* The converged estimates satisfy the optimality conditions of F (interval
  form of the subdifferential, written from the objective), and the check
  rejects a perturbed point.
* Block coordinate descent never increases F.
* Each sweep's delta is the largest entry change over both matrices,
  recomputed from successive iterates.
* At p <= 4 the converged estimates equal the minimiser a general convex
  solver (SLSQP on a reformulation with auxiliary variables for the absolute
  values) finds, with and without fused entries.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
from oracle import joint
from paper_2106_09382_amd import datagen


def _pair_f(x, a1, b1, a2, b2, l1, l2):
    return (0.5 * a1 * x[0] ** 2 + b1 * x[0] + 0.5 * a2 * x[1] ** 2 + b2 * x[1]
            + l1 * (abs(x[0]) + abs(x[1])) + l2 * abs(x[0] - x[1]))


def _numeric_min(f, starts):
    best = None
    for x0 in starts:
        r = minimize(f, np.asarray(x0, dtype=float), method="Nelder-Mead",
                     options=dict(xatol=1e-12, fatol=1e-15, maxiter=20000))
        if best is None or r.fun < best.fun:
            best = r
    return best


def _pair_cases():
    rng = np.random.default_rng(11)
    out = []
    for _ in range(60):
        a1, a2 = rng.uniform(0.5, 3.0, 2)
        b1, b2 = rng.normal(0, 1, 2)
        l1, l2 = rng.uniform(0, 0.6, 2)
        out.append((a1, b1, a2, b2, l1, l2))
    # each regime on purpose: both zero, fused nonzero, separated, lam2 = 0, lam1 = 0
    out += [(1.0, 0.1, 2.0, -0.1, 0.5, 0.1), (1.0, -1.0, 1.5, -1.1, 0.1, 0.5),
            (2.0, -3.0, 1.0, 2.0, 0.2, 0.3), (1.0, -0.7, 2.0, 0.4, 0.1, 0.0),
            (1.2, -0.7, 0.8, -0.2, 0.0, 0.3)]
    return out


@pytest.mark.parametrize("case", _pair_cases())
def test_pair_block_is_the_minimiser(case):
    a1, b1, a2, b2, l1, l2 = case
    x = np.array(joint.pair(*case))
    f = lambda z: _pair_f(z, *case)
    r = _numeric_min(f, [x + 0.3, x - 0.2, [0.0, 0.0], [1.0, -1.0]])
    assert f(x) <= r.fun + 1e-12
    # strong convexity (curvature >= min a) turns a value gap into a distance
    assert np.abs(x - r.x).max() < 1e-5
    # the subgradient conditions, as intervals for the fused term's subgradient u
    g1, g2 = a1 * x[0] + b1, a2 * x[1] + b2

    def sub(v, s):
        return (s, s) if v > 0 else (-s, -s) if v < 0 else (-s, s)
    s1, s2 = sub(x[0], l1), sub(x[1], l1)
    ivs = [sub(x[0] - x[1], l2), (-g1 - s1[1], -g1 - s1[0]), (g2 + s2[0], g2 + s2[1])]
    assert max(iv[0] for iv in ivs) - min(iv[1] for iv in ivs) < 1e-12


def _diag_cases():
    rng = np.random.default_rng(12)
    out = []
    for _ in range(40):
        s1, s2 = rng.uniform(0.3, 3.0, 2)
        c1, c2 = rng.normal(0, 1, 2)
        l2 = rng.uniform(0, 0.8)
        out.append((s1, c1, s2, c2, l2))
    out += [(1.0, 0.0, 1.0, 0.0, 0.1), (1.0, 0.5, 2.0, -0.5, 0.0), (0.5, -2.0, 3.0, 1.0, 5.0)]
    return out


@pytest.mark.parametrize("case", _diag_cases())
def test_diag_block_is_the_minimiser(case):
    s1, c1, s2, c2, l2 = case
    y = np.array(joint.diag(*case))
    assert (y > 0).all()

    def f(z):
        if z[0] <= 0 or z[1] <= 0:
            return np.inf
        return (-np.log(z[0]) + 0.5 * s1 * z[0] ** 2 + c1 * z[0] - np.log(z[1])
                + 0.5 * s2 * z[1] ** 2 + c2 * z[1] + l2 * abs(z[0] - z[1]))
    r = _numeric_min(f, [y * 1.2, y * 0.8, [1.0, 1.0]])
    assert f(y) <= r.fun + 1e-12
    assert np.abs(y - r.x).max() < 1e-5
    g1, g2 = s1 * y[0] + c1 - 1 / y[0], s2 * y[1] + c2 - 1 / y[1]
    if y[0] != y[1]:
        u = l2 if y[0] > y[1] else -l2
        assert abs(g1 + u) < 1e-12 and abs(g2 - u) < 1e-12
    else:
        assert abs(g1 + g2) < 1e-12 and abs(g1) <= l2 + 1e-12


def _pair_of_grams(p, n, seed, changed=0.2):
    jp = datagen.joint_problem(seed, p=p, n=n, changed=changed)
    return oracle.gram(jp["y"][0]), oracle.gram(jp["y"][1])


@pytest.mark.parametrize("p,sweeps", [(9, 3), (24, 5), (1, 2)])
def test_lam2_zero_is_two_independent_solves(p, sweeps):
    S1, S2 = _pair_of_grams(p, 2 * p + 5, 1)
    O1, O2, info, _ = joint.pcd(S1, S2, 0.12, 0.0, 1e-300, sweeps)
    want1, _, _ = oracle.pcd(S1, 0.12, 1e-300, sweeps)
    want2, _, _ = oracle.pcd(S2, 0.12, 1e-300, sweeps)
    assert info["sweeps"] == sweeps
    assert np.array_equal(O1, want1) and np.array_equal(O2, want2)


@pytest.mark.parametrize("p,n,lam1", [(20, 40, 0.1), (33, 20, 0.15)])
def test_large_lam2_is_concord_on_the_mean(p, n, lam1):
    S1, S2 = _pair_of_grams(p, n, 2)
    O1, O2, info, tr = joint.pcd(S1, S2, lam1, 1e3, 1e-12, 2000)
    want, winfo, wtr = oracle.pcd(0.5 * (S1 + S2), lam1, 1e-12, 2000)
    assert info["converged"] and winfo["converged"]
    assert np.array_equal(O1, O2)
    assert np.abs(O1 - want).max() < 1e-10
    assert np.array_equal(O1 != 0, want != 0)


def test_identical_populations():
    S1, _ = _pair_of_grams(30, 50, 3)
    O1, O2, info, _ = joint.pcd(S1, S1, 0.1, 0.05, 1e-12, 2000)
    want, _, _ = oracle.pcd(S1, 0.1, 1e-12, 2000)
    assert info["converged"] and info["differ_upper"] == 0
    assert np.array_equal(O1, O2)
    assert np.abs(O1 - want).max() < 1e-10


@pytest.mark.parametrize("p,n,lam1,lam2", [(25, 60, 0.1, 0.02), (40, 30, 0.15, 0.05),
                                           (31, 100, 0.05, 0.01), (16, 40, 0.3, 0.2)])
def test_converged_solution_is_optimal(p, n, lam1, lam2):
    S1, S2 = _pair_of_grams(p, n, 4)
    O1, O2, info, _ = joint.pcd(S1, S2, lam1, lam2, 1e-13, 20000)
    assert info["converged"]
    assert np.array_equal(O1, O1.T) and np.array_equal(O2, O2.T)
    r = joint.kkt(S1, S2, O1, O2, lam1, lam2)
    assert r["pairs"] < 1e-9 and r["diag"] < 1e-9, r
    # the fused penalty is doing something: some pairs are equal across the
    # populations, some differ
    iu = np.triu_indices(p, 1)
    assert 0 < info["differ_upper"] < iu[0].size
    # a perturbed point fails the check, so the check is not vacuous
    bad = O1.copy()
    i, j = np.argwhere(np.triu(O1 != 0, 1))[0]
    bad[i, j] = bad[j, i] = O1[i, j] * 1.01
    assert joint.kkt(S1, S2, bad, O2, lam1, lam2)["pairs"] > 1e-6
    bad = O2.copy()
    bad[3, 3] *= 1.001
    assert joint.kkt(S1, S2, O1, bad, lam1, lam2)["diag"] > 1e-6


def test_objective_never_increases():
    S1, S2 = _pair_of_grams(18, 30, 5)
    prev = joint.objective(S1, S2, np.eye(18), np.eye(18), 0.1, 0.05)
    for t in range(1, 9):
        O1, O2, _, _ = joint.pcd(S1, S2, 0.1, 0.05, 1e-300, t)
        f = joint.objective(S1, S2, O1, O2, 0.1, 0.05)
        assert f <= prev + 1e-12
        prev = f


def test_rejects_bad_input():
    S = np.eye(4)
    bad = S.copy()
    bad[2, 2] = 0.0
    with pytest.raises(oracle.OracleError):
        joint.pcd(S, bad, 0.1, 0.1, 1e-6, 10)
    with pytest.raises(oracle.OracleError):
        joint.pcd(S, S, 0.1, -1.0, 1e-6, 10)


def test_delta_is_the_largest_change_over_both_matrices():
    # population 2 moves more than population 1 (S_1 is near the identity)
    rng = np.random.default_rng(6)
    p = 14
    S1 = np.eye(p) + 0.01 * oracle.gram(rng.standard_normal((40, p)))
    _, S2 = _pair_of_grams(p, 30, 6)
    T = 6
    _, _, _, tr = joint.pcd(S1, S2, 0.05, 0.01, 1e-300, T)
    prev = (np.eye(p), np.eye(p))
    pop2_larger = False
    for t in range(1, T + 1):
        O1, O2, _, _ = joint.pcd(S1, S2, 0.05, 0.01, 1e-300, t)
        d1, d2 = np.abs(O1 - prev[0]).max(), np.abs(O2 - prev[1]).max()
        assert tr[t - 1] == max(d1, d2)
        pop2_larger |= d2 > d1
        prev = (O1, O2)
    assert pop2_larger


def test_block_update_at_a_fixed_point():
    # at the oracle's converged point every block update is (nearly) the identity
    S1, S2 = _pair_of_grams(20, 50, 7)
    O1, O2, info, _ = joint.pcd(S1, S2, 0.1, 0.03, 1e-14, 20000)
    assert info["converged"]
    worst = 0.0
    for i in range(20):
        for j in range(i, 20):
            x1, x2 = joint.block_update_at(S1, S2, O1, O2, i, j, 0.1, 0.03)
            worst = max(worst, abs(x1 - O1[i, j]), abs(x2 - O2[i, j]))
    assert worst < 1e-12
    # and away from it, not
    x1, _ = joint.block_update_at(S1, S2, np.eye(20), np.eye(20), 0, 0, 0.1, 0.03)
    assert abs(x1 - 1.0) > 1e-3


def _convex_reference(S1, S2, lam1, lam2):
    """Minimise F over (Omega_1, Omega_2) with a general solver: the absolute
    values become auxiliary variables bounded by linear constraints (t >= x,
    t >= -x), which leaves a smooth convex objective for SLSQP.  Written from
    the objective alone, sharing nothing with the block updates."""
    p = S1.shape[0]
    iu = list(zip(*np.triu_indices(p, 1)))
    q = len(iu)
    # layout: y1 (p), y2 (p), x1 (q), x2 (q), t1 (q), t2 (q), u (q), v (p)
    n_var = 3 * p + 5 * q
    Y1, Y2, X1, X2 = 0, p, 2 * p, 2 * p + q
    T1, T2, U, V = 2 * p + 2 * q, 2 * p + 3 * q, 2 * p + 4 * q, 2 * p + 5 * q

    def mats(z):
        O1, O2 = np.diag(z[Y1:Y1 + p]), np.diag(z[Y2:Y2 + p])
        for k, (i, j) in enumerate(iu):
            O1[i, j] = O1[j, i] = z[X1 + k]
            O2[i, j] = O2[j, i] = z[X2 + k]
        return O1, O2

    def f(z):
        O1, O2 = mats(z)
        val = 0.0
        for S, O, y in ((S1, O1, z[Y1:Y1 + p]), (S2, O2, z[Y2:Y2 + p])):
            if np.any(y <= 0):
                return 1e30
            val += -np.log(y).sum() + 0.5 * float(np.sum((O @ S) * O))
        return val + lam1 * (z[T1:T1 + q].sum() + z[T2:T2 + q].sum()) \
            + lam2 * (z[U:U + q].sum() + z[V:V + p].sum())

    A, rows = [], []
    for k in range(q):
        for src, dst in ((X1, T1), (X2, T2)):
            for sgn in (1.0, -1.0):          # t - sgn x >= 0
                a = np.zeros(n_var)
                a[dst + k], a[src + k] = 1.0, -sgn
                A.append(a)
        for sgn in (1.0, -1.0):              # u - sgn (x1 - x2) >= 0
            a = np.zeros(n_var)
            a[U + k], a[X1 + k], a[X2 + k] = 1.0, -sgn, sgn
            A.append(a)
    for i in range(p):
        for sgn in (1.0, -1.0):              # v - sgn (y1 - y2) >= 0
            a = np.zeros(n_var)
            a[V + i], a[Y1 + i], a[Y2 + i] = 1.0, -sgn, sgn
            A.append(a)
    A = np.array(A)
    z0 = np.zeros(n_var)
    z0[Y1:Y1 + p] = 1.0 / np.sqrt(np.diag(S1))
    z0[Y2:Y2 + p] = 1.0 / np.sqrt(np.diag(S2))
    z0[V:V + p] = np.abs(z0[Y1:Y1 + p] - z0[Y2:Y2 + p])
    bounds = [(1e-6, None)] * (2 * p) + [(None, None)] * (2 * q) + [(0, None)] * (3 * q + p)
    r = minimize(f, z0, method="SLSQP", bounds=bounds,
                 constraints=[dict(type="ineq", fun=lambda z: A @ z, jac=lambda z: A)],
                 options=dict(ftol=1e-15, maxiter=2000))
    O1, O2 = mats(r.x)
    return O1, O2, r


@pytest.mark.parametrize("p,seed,lam1,lam2,min_fused", [
    (2, 1, 0.1, 0.05, 0), (3, 2, 0.05, 0.02, 0), (3, 3, 0.2, 0.1, 1), (4, 4, 0.1, 0.03, 1),
    (3, 5, 0.05, 0.3, 2), (4, 6, 0.02, 0.15, 4)])
def test_joint_matches_a_general_convex_solver(p, seed, lam1, lam2, min_fused):
    rng = np.random.default_rng(300 + seed)
    a = rng.normal(size=(p, p))
    cov = a @ a.T + p * np.eye(p)
    S1 = oracle.gram(rng.multivariate_normal(np.zeros(p), cov, size=40))
    b = rng.normal(size=(p, p))
    S2 = oracle.gram(rng.multivariate_normal(np.zeros(p), cov + 0.3 * (b @ b.T), size=40))
    O1, O2, info, _ = joint.pcd(S1, S2, lam1, lam2, 1e-14, 100000)
    assert info["converged"]
    R1, R2, r = _convex_reference(S1, S2, lam1, lam2)
    f_or = joint.objective(S1, S2, O1, O2, lam1, lam2)
    f_ref = joint.objective(S1, S2, R1, R2, lam1, lam2)
    # the oracle is never worse than the general solver, and they agree
    assert f_or <= f_ref + 1e-10
    assert f_ref - f_or < 1e-7
    assert max(np.abs(O1 - R1).max(), np.abs(O2 - R2).max()) < 1e-4
    # entries on the fused line omega^1_ij = omega^2_ij (i <= j)
    iu = np.triu_indices(p)
    assert int((O1[iu] == O2[iu]).sum()) >= min_fused


# ---------------------------------------------------------------- borderline filter

def _two_by_two(r1, r2):
    """p = 2, unit diagonals, off-diagonals r_1, r_2, at Omega = I: a_m = 2 and
    the eq. (3) numerator b_m = 2 r_m (nothing else enters)."""
    S1 = np.array([[1.0, r1], [r1, 1.0]])
    S2 = np.array([[1.0, r2], [r2, 1.0]])
    return S1, S2, np.eye(2), np.eye(2)


@pytest.mark.parametrize("r1,r2,border,why", [
    # b = (-0.6, -0.5): |b_1 + lam2| = |b_2 - lam2| = 0.55, so u_1 = u_2 exactly
    (-0.3, -0.25, True, "u_1 = u_2: the x_1 > x_2 test is a tie"),
    # b_1 = -0.15: |b_1 + lam2| = lam1 in the case x_1 > x_2 that is taken
    (-0.075, 0.2, True, "threshold of x_1 in case x_1 > x_2"),
    # b_1 = b_2 = -0.1: fused, |b_1 + b_2| = 2 lam1
    (-0.05, -0.05, True, "fused threshold"),
    # b = (-0.6, 0.4): case x_1 > x_2 by 0.35, thresholds far
    (-0.3, 0.2, False, "clear case x_1 > x_2"),
    # b = (0.4, -0.6): case x_1 < x_2
    (0.2, -0.3, False, "clear case x_1 < x_2"),
    # b_1 = b_2 = -0.6: fused, far from every threshold
    (-0.3, -0.3, False, "clear fused pair"),
    # b = 0: every candidate is exactly 0, a tie no rounding can break
    (0.0, 0.0, False, "zero block"),
])
def test_joint_borderline_pairs_on_constructed_blocks(r1, r2, border, why):
    """Constructed blocks whose decisions sit exactly on (or clearly off) the
    case boundaries of the block minimiser, at lam1 = 0.1, lam2 = 0.05.  A
    missing or mis-signed lam2 shift, or the fused threshold taken at lam1
    instead of 2 lam1, moves one of the first three off its boundary."""
    S1, S2, O1, O2 = _two_by_two(r1, r2)
    got = joint.borderline_pairs(S1, S2, O1, O2, 0.1, 0.05, 1e-9)
    assert (len(got) == 1) == border, why
    if border:
        assert tuple(got[0]) == (0, 1)


def test_joint_borderline_pairs_agree_with_the_block_update():
    """Nudging the numerators of a flagged block by a few rounding units flips
    one of the block minimiser's decisions (fused or not, zero or not); for an
    unflagged block no such nudge changes any decision."""
    lam1, lam2 = 0.1, 0.05
    eps = (-1e-12, 0.0, 1e-12)

    def outcomes(r1, r2):
        b1, b2 = 2 * r1, 2 * r2
        seen = set()
        for e1 in eps:
            for e2 in eps:
                x1, x2 = joint.pair(2.0, b1 + e1, 2.0, b2 + e2, lam1, lam2)
                seen.add((x1 != x2, x1 != 0.0, x2 != 0.0))
        return seen

    for r1, r2 in ((-0.3, -0.25), (-0.075, 0.2), (-0.05, -0.05)):
        assert len(outcomes(r1, r2)) > 1, (r1, r2)
    for r1, r2 in ((-0.3, 0.2), (0.2, -0.3), (-0.3, -0.3), (0.0, 0.0)):
        assert len(outcomes(r1, r2)) == 1, (r1, r2)


@pytest.mark.parametrize("p,n,lam1,lam2,seed", [
    (17, 40, 0.1, 0.02, 3), (64, 120, 0.1, 0.01, 5), (130, 90, 0.15, 0.03, 7),
    (301, 150, 0.2, 0.1, 9),
])
def test_no_borderline_pairs_on_the_parity_workloads(p, n, lam1, lam2, seed):
    """Reading R22's claim for the GPU parity workloads: at the converged
    joint estimate no block decision is within rounding of its boundary, so
    the pair-by-pair comparisons exclude nothing."""
    jp = datagen.joint_problem(seed, p=p, n=n, changed=0.2)
    S1, S2 = oracle.gram(jp["y"][0]), oracle.gram(jp["y"][1])
    O1, O2, info, _ = joint.pcd(S1, S2, lam1, lam2, 1e-10, 3000)
    assert info["converged"]
    assert len(joint.borderline_pairs(S1, S2, O1, O2, lam1, lam2, 1e-9)) == 0
