"""Pins of the oracle's implicit gradient (oracle/backward.py).

Not pinned to itself: the gradient is checked against
* central finite differences of the oracle's own forward solve (Algorithm 1
  run to 1e-14), entry by entry of S and in lambda;
* the closed form above lambda_max, where Omega-hat = diag(S_ii^-1/2) and
  nothing off the diagonal depends on S;
* structure: J is symmetric with the denominators of eqs. (2)-(3) on its
  diagonal, and the residuals vanish at the optimum.
"""
import numpy as np
import pytest

import oracle
from oracle import backward as ob
from paper_2106_09382_amd import datagen


def _problem(p, n, lam, seed, graph="chain"):
    rng = np.random.default_rng(seed)
    om0 = datagen.chain_precision(p) if graph == "chain" else datagen.er_precision(p, rng)
    y = datagen.sample_y(om0, n, rng)
    S = oracle.gram(y)
    om, info, _ = oracle.pcd(S, lam, 1e-14, 20000)
    assert info["converged"]
    return S, om, om0


def _loss(om, om0):
    return float(((om - om0) ** 2).sum())


def _solve(S, lam, start):
    om, info, _ = oracle.pcd(S, lam, 1e-14, 20000, omega0=start)
    assert info["converged"]
    return om


CASES = [(32, 64, 0.15, 11, "chain"), (24, 12, 0.2, 12, "chain"), (20, 40, 0.1, 13, "er")]


@pytest.mark.parametrize("p,n,lam,seed,graph", CASES)
def test_residuals_vanish_and_jacobian_is_symmetric(p, n, lam, seed, graph):
    S, om, _ = _problem(p, n, lam, seed, graph)
    coords = ob.free_coordinates(om)
    assert np.abs(ob.residuals(S, om, lam, coords)).max() < 1e-10
    J = ob.jacobian(S, om, coords)
    assert np.allclose(J, J.T, rtol=0, atol=1e-14)
    d = np.diag(J)
    for r, c in enumerate(coords):
        if c[0] == "d":
            assert d[r] == pytest.approx(S[c[1], c[1]] + 1.0 / om[c[1], c[1]] ** 2)
        else:
            assert d[r] == pytest.approx(S[c[1], c[1]] + S[c[2], c[2]])
    assert np.linalg.eigvalsh(J).min() > 0


@pytest.mark.parametrize("p,n,lam,seed,graph", CASES)
def test_gradient_matches_central_differences(p, n, lam, seed, graph):
    S, om, om0 = _problem(p, n, lam, seed, graph)
    res = ob.backward(S, om, lam, 2.0 * (om - om0))
    G = res["grad_S"]
    rng = np.random.default_rng(seed + 100)
    act = [(int(i), int(j)) for i, j in zip(*np.nonzero(np.triu(om != 0, 1)))]
    ina = [(int(i), int(j)) for i, j in zip(*np.nonzero(np.triu(om == 0, 1)))]
    picks = [(i, i) for i in rng.choice(p, 6, replace=False)]
    picks += [act[k] for k in rng.choice(len(act), min(8, len(act)), replace=False)]
    picks += [ina[k] for k in rng.choice(len(ina), min(6, len(ina)), replace=False)]
    eps = 1e-6
    for a, b in picks:
        E = np.zeros_like(S)
        E[a, b] = 1.0
        E[b, a] = 1.0
        lp = _loss(_solve(S + eps * E, lam, om), om0)
        lm = _loss(_solve(S - eps * E, lam, om), om0)
        fd = (lp - lm) / (2 * eps)
        want = G[a, a] if a == b else 2.0 * G[a, b]
        assert fd == pytest.approx(want, abs=2e-6 * max(1.0, abs(want))), (a, b)
    eps = 1e-6
    fl = (_loss(_solve(S, lam + eps, om), om0) - _loss(_solve(S, lam - eps, om), om0)) / (2 * eps)
    assert fl == pytest.approx(res["grad_lambda"], abs=2e-6 * max(1.0, abs(fl)))


def test_gradient_above_lambda_max_is_closed_form():
    rng = np.random.default_rng(5)
    S = oracle.gram(rng.standard_normal((50, 9)))
    lam = 1.5 * oracle.lambda_max(S)
    om, info, _ = oracle.pcd(S, lam, 1e-14, 1000)
    d = 1.0 / np.sqrt(np.diag(S))
    assert np.allclose(om, np.diag(d), rtol=0, atol=1e-14)
    C = rng.standard_normal(S.shape)
    res = ob.backward(S, om, lam, C)
    # omega_ii = S_ii^-1/2 alone moves: dL/dS_ii = C_ii * (-1/2) S_ii^-3/2
    want = np.diag(np.diag(C) * -0.5 * np.diag(S) ** -1.5)
    assert np.allclose(res["grad_S"], want, rtol=1e-12, atol=1e-15)
    assert res["grad_lambda"] == 0.0


def test_adjoint_layout_and_lambda_gradient_identity():
    # dL/dlam = -sum_A v_ij sign(omega_ij): with V laid out symmetric, that is
    # -1/2 sum_{i != j} V_ij sign(omega_ij).
    S, om, om0 = _problem(32, 64, 0.15, 11)
    res = ob.backward(S, om, 0.15, 2.0 * (om - om0))
    V = res["V"]
    assert np.array_equal(V, V.T)
    assert np.all(V[(om == 0)] == 0)
    off = ~np.eye(32, dtype=bool)
    assert res["grad_lambda"] == pytest.approx(-0.5 * float((V * np.sign(om))[off].sum()),
                                               rel=1e-12)
