"""GPU parity of the implicit gradient (concord_backward) and the autograd
wrapper.

The reference is the oracle's dense solve of the stationarity system
(oracle/backward.py), fed the same Omega-hat the GPU solve produced, so the
comparison isolates the backward pass.  At the full size of the
differentiable workload (p = 2000) the oracle cannot run; there the gradient
is checked by central differences of the GPU's own forward solve along random
symmetric directions (a property that holds at any size).
"""
import warnings

import numpy as np
import pytest
import torch

import oracle
from oracle import backward as ob
from paper_2106_09382_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2106_09382_amd import _lib
    _lib.load()
    return _lib


_cache = {}


def _case(p, n, lam, seed, graph):
    key = (p, n, lam, seed, graph)
    if key not in _cache:
        rng = np.random.default_rng(seed)
        om0 = datagen.chain_precision(p) if graph == "chain" else datagen.er_precision(p, rng)
        S = oracle.gram(datagen.sample_y(om0, n, rng))
        _cache[key] = (S, om0)
    return _cache[key]


def _forward(lib, S, lam, dtype=torch.float64, tol=1e-13, maxit=50000):
    St = torch.tensor(S, dtype=dtype, device="cuda")
    om, info = lib.fit(St, lam, tol, maxit)
    torch.cuda.synchronize()
    return St, om, info


CASES = [
    (32, 64, 0.15, 11, "chain"),
    (24, 12, 0.2, 12, "chain"),
    (20, 40, 0.1, 13, "er"),
    (97, 150, 0.2, 14, "er"),
    (100, 50, 0.15, 1, "er"),
]


@pytest.mark.parametrize("p,n,lam,seed,graph", CASES)
def test_backward_fp64_matches_dense_solve(lib, p, n, lam, seed, graph):
    S, om0 = _case(p, n, lam, seed, graph)
    St, om, _ = _forward(lib, S, lam)
    omn = om.cpu().numpy()
    C = 2.0 * (omn - om0)
    gS, gl, info = lib.backward(St, om, torch.tensor(C, device="cuda"), 1e-13, 50000)
    torch.cuda.synchronize()
    assert info["code"] == 0
    want = ob.backward(S, omn, lam, C)
    scale = max(1.0, np.abs(want["grad_S"]).max())
    err = np.abs(gS.cpu().numpy() - want["grad_S"]).max()
    assert err <= 1e-8 * scale, err
    assert gl == pytest.approx(want["grad_lambda"], rel=1e-8, abs=1e-8)
    g = gS.cpu().numpy()
    assert np.array_equal(g, g.T)


def test_backward_independent_of_launch_shape(lib):
    S, om0 = _case(97, 150, 0.2, 14, "er")
    St, om, _ = _forward(lib, S, 0.2)
    Ct = torch.tensor(2.0 * (om.cpu().numpy() - om0), device="cuda")
    ref, gl, _ = lib.backward(St, om, Ct, 1e-13, 50000)
    ref = ref.cpu().numpy()
    for shape in (dict(row_groups=4, col_slices=2), dict(row_groups=8, col_slices=1, w_in_lds=2),
                  dict(row_groups=3, col_slices=3, block_threads=64, pending_depth=5)):
        g, gl2, _ = lib.backward(St, om, Ct, 1e-13, 50000, **shape)
        assert np.array_equal(g.cpu().numpy(), ref), shape
        # dL/dlam is a sum reduced with atomics: the order, not the terms, varies
        assert gl2 == pytest.approx(gl, rel=1e-14)


def test_backward_fp32_close_to_fp64(lib):
    S, om0 = _case(100, 50, 0.15, 1, "er")
    St, om, _ = _forward(lib, S, 0.15)
    omn = om.cpu().numpy()
    C = 2.0 * (omn - om0)
    want = ob.backward(S, omn, 0.15, C)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        g32, gl32, info = lib.backward(St.float(), om.float(), torch.tensor(C, device="cuda").float(),
                                       1e-7, 50000, check=False)
    assert info["code"] in (0, 1)
    scale = np.abs(want["grad_S"]).max()
    assert np.abs(g32.double().cpu().numpy() - want["grad_S"]).max() <= 1e-3 * scale
    assert gl32 == pytest.approx(want["grad_lambda"], rel=1e-3)


def test_backward_above_lambda_max_is_closed_form(lib):
    rng = np.random.default_rng(5)
    S = oracle.gram(rng.standard_normal((50, 9)))
    lam = 1.5 * oracle.lambda_max(S)
    St, om, _ = _forward(lib, S, lam)
    C = rng.standard_normal(S.shape)
    gS, gl, _ = lib.backward(St, om, torch.tensor(C, device="cuda"), 1e-14, 1000)
    want = np.diag(np.diag(C) * -0.5 * np.diag(S) ** -1.5)
    assert np.allclose(gS.cpu().numpy(), want, rtol=1e-12, atol=1e-15)
    assert gl == 0.0


def test_backward_rejects_bad_inputs(lib):
    from paper_2106_09382_amd._lib import ConcordError
    rng = np.random.default_rng(2)
    S = oracle.gram(rng.standard_normal((30, 8)))
    St, om, _ = _forward(lib, S, 0.2)
    C = torch.zeros_like(St)
    bad = om.clone()
    bad[3, 3] = -1.0
    with pytest.raises(ConcordError) as e:
        lib.backward(St, bad, C)
    assert e.value.code == -3
    Cn = C.clone()
    Cn[1, 2] = float("nan")
    with pytest.raises(ConcordError) as e:
        lib.backward(St, om, Cn)
    assert e.value.code == -2


def test_autograd_matches_backward_and_differences(lib):
    from paper_2106_09382_amd.autograd import concord
    S, om0 = _case(32, 64, 0.15, 11, "chain")
    St = torch.tensor(S, device="cuda", requires_grad=True)
    lam = torch.tensor(0.15, dtype=torch.float64, device="cuda", requires_grad=True)
    O0 = torch.tensor(om0, device="cuda")
    om = concord(St, lam, tol=1e-13, maxit=50000, backward_tol=1e-13)
    loss = ((om - O0) ** 2).sum()
    loss.backward()
    gS, gl, _ = lib.backward(St.detach(), om.detach(), (2.0 * (om - O0)).detach(), 1e-13, 50000)
    assert torch.equal(St.grad, gS)
    assert lam.grad.item() == gl
    # a symmetric direction: dL = <grad_S, D>
    rng = np.random.default_rng(9)
    D = rng.standard_normal(S.shape)
    D = D + D.T
    eps = 1e-6

    def L(Sx, lx):
        with torch.no_grad():
            o = concord(torch.tensor(Sx, device="cuda"), lx, tol=1e-14, maxit=50000)
            return float(((o - O0) ** 2).sum())

    fd = (L(S + eps * D, 0.15) - L(S - eps * D, 0.15)) / (2 * eps)
    assert fd == pytest.approx(float((St.grad.cpu().numpy() * D).sum()), rel=1e-5)
    fl = (L(S, 0.15 + eps) - L(S, 0.15 - eps)) / (2 * eps)
    assert fl == pytest.approx(lam.grad.item(), rel=1e-5)


@pytest.mark.slow
def test_backward_p200_matches_dense_solve(lib):
    S, om0 = _case(200, 100, 0.15, 1, "chain")
    St, om, _ = _forward(lib, S, 0.15)
    omn = om.cpu().numpy()
    C = 2.0 * (omn - om0)
    gS, gl, info = lib.backward(St, om, torch.tensor(C, device="cuda"), 1e-13, 50000)
    want = ob.backward(S, omn, 0.15, C)
    scale = max(1.0, np.abs(want["grad_S"]).max())
    assert np.abs(gS.cpu().numpy() - want["grad_S"]).max() <= 1e-8 * scale
    assert gl == pytest.approx(want["grad_lambda"], rel=1e-8)


@pytest.mark.slow
def test_config5_gradient_by_directional_differences(lib):
    # p = 2000, n = 1000, chain Omega_0, lam = 0.15, L = |Omega-hat - Omega_0|_F^2.
    pr = datagen.problem(5)
    p, lam = pr["p"], pr["lam"]
    S, om0 = oracle.gram(pr["y"]), pr["omega0"]
    St, om, finfo = _forward(lib, S, lam, tol=1e-12)
    O0 = torch.tensor(om0, device="cuda")
    gS, gl, info = lib.backward(St, om, 2.0 * (om - O0), 1e-12, 50000)
    assert info["code"] == 0
    g = gS.cpu().numpy()

    def L(Sx, lx):
        _, o, _ = _forward(lib, Sx, lx, tol=1e-13)
        return float(((o - O0) ** 2).sum())

    rng = np.random.default_rng(17)
    eps = 1e-7
    for _ in range(2):
        D = np.zeros((p, p))
        idx = rng.integers(0, p, size=(400, 2))
        D[idx[:, 0], idx[:, 1]] = rng.standard_normal(400)
        D = D + D.T
        fd = (L(S + eps * D, lam) - L(S - eps * D, lam)) / (2 * eps)
        assert fd == pytest.approx(float((g * D).sum()), rel=1e-4, abs=1e-6)
    fl = (L(S, lam + eps) - L(S, lam - eps)) / (2 * eps)
    assert fl == pytest.approx(gl, rel=1e-4)
