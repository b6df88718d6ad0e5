"""Pins of the oracle's active-set scheme (oracle/active.py) and of PCD over
an arbitrary edge colouring (Section 4: Theorem 2's order extends to any
edge colouring of K_p).

* Given Algorithm 1's own colouring, PCD over a colouring reproduces
  Algorithm 1 bit for bit.
* The greedy colouring: every class is a matching, every support edge is
  coloured once, at most 2 Delta - 1 colours, and known small graphs.
* The active-set scheme stops on a full sweep of Algorithm 1 and reaches the
  minimiser: against brute force at p <= 4, against plain PCD (same support,
  within the tolerance) where n > p, and the stationarity conditions.
"""
import numpy as np
import pytest

import oracle
from oracle import active
from bruteforce import brute_force
from paper_2106_09382_amd import datagen


def _round_robin_classes(p):
    tab = oracle.round_robin(p)
    return [[(int(a), int(b)) if a < b else (int(b), int(a)) for a, b in colour
             if a != p and b != p] for colour in tab]


@pytest.mark.parametrize("p", [2, 5, 8, 31, 64])
def test_colouring_pcd_reproduces_algorithm_1(p):
    pr = datagen.problem(2, p=p, n=2 * p + 4)
    S = oracle.gram(pr["y"])
    want, winfo, wtr = oracle.pcd(S, 0.15, 1e-10, 300)
    got, ginfo, gtr = oracle.pcd_colouring(S, 0.15, 1e-10, 300, _round_robin_classes(p))
    assert np.array_equal(got, want)
    assert ginfo["sweeps"] == winfo["sweeps"]
    assert np.array_equal(gtr, wtr)


def test_colouring_pcd_leaves_uncoloured_pairs_alone():
    pr = datagen.problem(2, p=12, n=30)
    S = oracle.gram(pr["y"])
    om0 = np.eye(12)
    om0[2, 7] = om0[7, 2] = 0.05
    got, _, _ = oracle.pcd_colouring(S, 0.05, 1e-12, 1, [[(0, 1), (3, 4)], [(1, 5)]], omega0=om0)
    untouched = np.ones((12, 12), dtype=bool)
    for i, j in [(0, 1), (3, 4), (1, 5)]:
        untouched[i, j] = untouched[j, i] = False
    np.fill_diagonal(untouched, False)
    assert np.array_equal(got[untouched], om0[untouched])


def _check_colouring(pairs, classes):
    seen = set()
    for cls in classes:
        verts = [v for pr in cls for v in pr]
        assert len(verts) == len(set(verts)), "a class is not a matching"
        for pr in cls:
            assert pr not in seen
            seen.add(pr)
    assert seen == set(tuple(sorted(p)) for p in pairs)


def test_greedy_colouring_small_graphs():
    assert active.greedy_colouring([]) == []
    assert len(active.greedy_colouring([(0, 1), (1, 2), (2, 3)])) == 2        # path
    assert len(active.greedy_colouring([(0, 1), (0, 2), (1, 2)])) == 3        # triangle
    star = [(0, k) for k in range(1, 6)]
    assert len(active.greedy_colouring(star)) == 5                          # star: degree 5
    assert active.greedy_colouring([(2, 3), (0, 1)]) == [[(0, 1), (2, 3)]]   # one matching


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_greedy_colouring_invariants(seed):
    rng = np.random.default_rng(seed)
    p = 60
    mask = np.triu(rng.random((p, p)) < 0.1, 1)
    pairs = [tuple(x) for x in np.argwhere(mask).tolist()]
    classes = active.greedy_colouring(pairs)
    _check_colouring(pairs, classes)
    deg = mask.sum(0) + mask.sum(1)
    assert len(classes) <= max(1, 2 * deg.max() - 1)
    assert classes == active.greedy_colouring(list(reversed(pairs)))       # order-free input


@pytest.mark.parametrize("p,seed,lam", [(3, 1, 0.05), (4, 3, 0.1), (4, 5, 0.02)])
def test_active_set_matches_brute_force(p, seed, lam):
    rng = np.random.default_rng(100 + seed)
    a = rng.normal(size=(p, p))
    cov = a @ a.T + p * np.eye(p)
    S = oracle.gram(rng.multivariate_normal(np.zeros(p), cov, size=40))
    want, _ = brute_force(S, lam)
    got, info = active.active_set_pcd(S, lam, 1e-13, 1000, 10000)
    assert info["converged"]
    assert np.abs(got - want).max() < 1e-9


@pytest.mark.parametrize("p,n,lam", [(60, 150, 0.2), (120, 240, 0.2), (97, 300, 0.1)])
def test_active_set_reaches_the_pcd_minimiser(p, n, lam):
    pr = datagen.problem(2, p=p, n=n)
    S = oracle.gram(pr["y"])
    tol = 1e-10
    got, info = active.active_set_pcd(S, lam, tol, 500, 20000)
    want, winfo, _ = oracle.pcd(S, lam, tol, 500)
    assert info["converged"] and winfo["converged"]
    assert info["delta"] < tol
    assert np.array_equal(got != 0, want != 0)
    assert np.abs(got - want).max() < 1e3 * tol
    r = oracle.kkt(S, got, lam)
    assert max(r.values()) < 1e-7
    # the point of the scheme: far fewer parallel steps
    m = p + (p & 1) - 1
    ncol = len(active.greedy_colouring(active.support(got)))
    assert ncol < m
