"""The benchmark's CPU baseline (oracle/cpu_pcd.c: Algorithm 1 with a
maintained W, serial and OpenMP colour-parallel) against the oracle's
direct-sum PCD: the same iterates up to rounding, the same sweeps and
support, and the parallel run bit for bit the serial one."""
import numpy as np
import pytest

import oracle
from oracle import cpu_baseline
from paper_2106_09382_amd import datagen


@pytest.mark.parametrize("p,n,lam", [(1, 5, 0.1), (2, 8, 0.1), (17, 40, 0.2), (64, 100, 0.3),
                                     (101, 60, 0.15), (200, 400, 0.1)])
def test_wform_matches_the_oracle(p, n, lam):
    pr = datagen.problem(2, p=p, n=n)
    S = oracle.gram(pr["y"])
    want, winfo, _ = oracle.pcd(S, lam, 1e-10, 2000)
    got, info = cpu_baseline.pcd_wform(S, lam, 1e-10, 2000, threads=1)
    assert info["converged"] and winfo["converged"]
    assert info["sweeps"] == winfo["sweeps"]
    assert np.abs(got - want).max() < 1e-10
    assert np.array_equal(got != 0, want != 0)
    par, pinfo = cpu_baseline.pcd_wform(S, lam, 1e-10, 2000, threads=4)
    assert np.array_equal(par, got) and pinfo["sweeps"] == info["sweeps"]
    assert pinfo["moved_pairs"] == info["moved_pairs"] and pinfo["threads"] == 4


def test_colour_limit_and_counts():
    pr = datagen.problem(2, p=30, n=60)
    S = oracle.gram(pr["y"])
    want, _, _ = oracle.pcd(S, 0.2, 1e-300, 1, colour_limit=7)
    got, info = cpu_baseline.pcd_wform(S, 0.2, 1e-300, 1, threads=2, colour_limit=7)
    assert info["steps"] == 7 and info["moved_diag"] == 0
    assert np.abs(got - want).max() < 1e-12
    full, finfo = cpu_baseline.pcd_wform(S, 0.2, 1e-300, 1)
    assert finfo["steps"] == 29 and finfo["moved_diag"] == 30
    # the count of pairs that moved in the first sweep, from the iterate itself
    assert finfo["moved_pairs"] == int((np.triu(full, 1) != 0).sum())


def test_rejects_bad_input():
    with pytest.raises(oracle.OracleError):
        cpu_baseline.pcd_wform(np.diag([1.0, 0.0]), 0.1, 1e-6, 10)
    with pytest.raises(oracle.OracleError):
        cpu_baseline.pcd_wform(np.eye(3), -0.1, 1e-6, 10)
