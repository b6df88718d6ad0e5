"""GPU parity: the HIP CONCORD-PCD path against the CPU oracle.

Bar (per element, same seeded inputs):
* FP64: max |Omega_gpu - Omega_oracle| <= 1e-8, identical support, identical
  sweep count.
* FP32: max |Omega_gpu - Omega_oracle(FP64)| <= 1e-4, identical support
  outside borderline pairs (numerator within 1e-4 (S_ii + S_jj) of lambda).
The oracle runs the same schedule from the same start with the same stopping
rule, so both produce the same iterates up to rounding (Theorem 2's
reordering argument does not even come into play).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2106_09382_amd import datagen

pytestmark = pytest.mark.gpu

TOL64 = 1e-8
TOL32 = 1e-4


@pytest.fixture(scope="module")
def lib():
    from paper_2106_09382_amd import _lib
    _lib.load()
    return _lib


def _gpu_fit(lib, S, lam, tol, maxit, dtype=torch.float64, check=True, **kw):
    St = torch.tensor(S, dtype=dtype, device="cuda")
    om, info = lib.fit(St, lam, tol, maxit, check=check, **kw)
    torch.cuda.synchronize()
    return om.double().cpu().numpy(), info


def _support_mismatch(S, got, want, lam, rel):
    bad = (got != 0) != (want != 0)
    np.fill_diagonal(bad, False)
    if rel > 0 and bad.any():
        for i, j in oracle.borderline_pairs(S, want, lam, rel):
            bad[i, j] = bad[j, i] = False
    return int(np.triu(bad, 1).sum())


def _assert_parity64(S, got, ginfo, want, winfo, lam):
    err = np.abs(got - want).max()
    assert err <= TOL64, f"max abs error {err:.3e}"
    assert _support_mismatch(S, got, want, lam, 1e-9) == 0
    assert ginfo["sweeps"] == winfo["sweeps"]
    assert np.array_equal(got, got.T)


_cache = {}


def _problem(config, **kw):
    key = (config, tuple(sorted(kw.items())))
    if key not in _cache:
        pr = datagen.problem(config, **kw)
        pr["S"] = oracle.gram(pr["y"])
        _cache[key] = pr
    return _cache[key]


def _oracle(pr, lam=None, tol=None, maxit=None):
    lam = pr["lam"] if lam is None else lam
    tol = pr["tol"] if tol is None else tol
    maxit = pr["maxit"] if maxit is None else maxit
    key = ("oracle", id(pr), lam, tol, maxit)
    if key not in _cache:
        _cache[key] = oracle.pcd(pr["S"], lam, tol, maxit)
    return _cache[key]


# ------------------------------------------------------------------ config 1

SHAPES = [
    dict(),                                           # one workgroup, W in LDS
    dict(row_groups=4, col_slices=2),                 # grid, W blocks in LDS
    dict(row_groups=8, col_slices=1, w_in_lds=2),     # grid, W in HBM
    dict(row_groups=2, col_slices=4, w_in_lds=2),
    dict(row_groups=16, col_slices=4, block_threads=256),
    dict(row_groups=64, col_slices=1),                # one row per workgroup
    dict(row_groups=8, col_slices=2, w_in_lds=2, pending_depth=4),
    dict(row_groups=4, col_slices=4, w_in_lds=2, pending_depth=8),
    dict(row_groups=1, col_slices=3, block_threads=64, pending_depth=6),
]


@pytest.mark.parametrize("shape", SHAPES, ids=[str(s) for s in SHAPES])
def test_config1_fp64_parity(lib, shape):
    pr = _problem(1)
    want, winfo, wtr = _oracle(pr)
    got, ginfo = _gpu_fit(lib, pr["S"], 0.3, 1e-8, 500, trace=True, **shape)
    _assert_parity64(pr["S"], got, ginfo, want, winfo, 0.3)
    np.testing.assert_allclose(ginfo["delta_trace"], wtr, rtol=1e-6, atol=1e-12)
    assert ginfo["nnz_upper"] == winfo["nnz_upper"]
    assert ginfo["objective"] == pytest.approx(oracle.objective(pr["S"], want, 0.3), rel=1e-12)


def test_config1_bitwise_identical_across_shapes_and_runs(lib):
    # Every W entry receives its updates in an order fixed by the schedule,
    # so the result does not depend on the launch shape.
    pr = _problem(1)
    ref, _ = _gpu_fit(lib, pr["S"], 0.3, 1e-8, 500)
    for shape in SHAPES[1:]:
        got, _ = _gpu_fit(lib, pr["S"], 0.3, 1e-8, 500, **shape)
        assert np.array_equal(got, ref), shape
    again, _ = _gpu_fit(lib, pr["S"], 0.3, 1e-8, 500)
    assert np.array_equal(again, ref)


W_SHAPES = [
    dict(),
    dict(pending_depth=2),
    dict(pending_depth=5),
    dict(row_groups=4, col_slices=2, pending_depth=6),
    dict(row_groups=8, col_slices=1, w_in_lds=2, pending_depth=8),
    dict(row_groups=1, col_slices=2, block_threads=128, w_in_lds=2, pending_depth=3),
]


@pytest.mark.parametrize("maxit", [1, 3, 500])
@pytest.mark.parametrize("shape", W_SHAPES, ids=[str(s) for s in W_SHAPES])
def test_stored_product_is_omega_s(lib, shape, maxit):
    # The kernel keeps W = Omega S with deferred row updates; after the last
    # sweep every pending update must be in the stored rows.  Exact up to the
    # rounding of the accumulated fused multiply-adds.
    pr = _problem(1)
    S = pr["S"]
    St = torch.tensor(S, device="cuda")
    Wt = torch.full_like(St, float("nan"))
    om, info = lib.fit(St, 0.3, 1e-8, maxit, check=False, w_out=Wt, **shape)
    torch.cuda.synchronize()
    got = om.cpu().numpy()
    W = Wt.cpu().numpy()
    assert info["code"] in (0, 1)
    scale = (np.abs(got) @ np.abs(S)).max()
    assert np.abs(W - got @ S).max() <= 1e-13 * scale * max(info["sweeps"], 1)


# Background row rewrites (the default whenever W is in HBM, some wave holds
# no rows and the pending depth is at least 4) against rewrites right after
# each step: the same updates in the same order, so the same bits in Omega and
# in the stored product W.
BG_CASES = [
    (1, dict(w_in_lds=2)),
    (1, dict(w_in_lds=2, pending_depth=4)),
    (1, dict(w_in_lds=2, pending_depth=5, block_threads=128)),
    (2, dict(w_in_lds=2)),
    (2, dict(w_in_lds=2, row_groups=16, col_slices=4, pending_depth=6)),
    (2, dict(w_in_lds=2, row_groups=64, col_slices=2, block_threads=256, pending_depth=4)),
]


@pytest.mark.parametrize("config,shape", BG_CASES, ids=[f"{c}-{s}" for c, s in BG_CASES])
def test_background_rewrites_match_synchronous_bit_for_bit(lib, config, shape):
    pr = _problem(config)
    S = pr["S"]
    lam, tol = (0.3, 1e-8) if config == 1 else (0.2, 1e-7)
    St = torch.tensor(S, device="cuda")
    outs = []
    for sync in (False, True):
        Wt = torch.full_like(St, float("nan"))
        om, info = lib.fit(St, lam, tol, 500, w_out=Wt, sync_rewrites=sync, **shape)
        torch.cuda.synchronize()
        outs.append((om.cpu().numpy(), Wt.cpu().numpy(), info))
    (a, wa, ia), (b, wb, ib) = outs
    assert ia["w_in_lds"] == 0 and ia["code"] == 0
    assert np.array_equal(a, b)
    assert np.array_equal(wa, wb)
    assert ia["sweeps"] == ib["sweeps"] and ia["moved_pairs"] == ib["moved_pairs"]


# Workgroups wider than 512 threads (W in HBM, one row per thread, the waves
# without rows rewriting in the background): the same bits as 512 threads, in
# plain, active-set and adjoint sweeps.
WIDE_CASES = [
    (1, "f64", dict(w_in_lds=2, block_threads=768)),
    (2, "f64", dict(w_in_lds=2, block_threads=768)),
    (2, "f64", dict(w_in_lds=2, block_threads=640, sync_rewrites=True)),
    (2, "f64", dict(block_threads=768, active_set=True)),
    (2, "f32", dict(w_in_lds=2, block_threads=1024)),
    (2, "f32", dict(w_in_lds=2, block_threads=1024, row_groups=16, col_slices=4,
                    pending_depth=6)),
]


@pytest.mark.parametrize("config,dt,shape", WIDE_CASES,
                         ids=[f"{c}-{d}-{s}" for c, d, s in WIDE_CASES])
def test_wide_workgroups_match_512_threads_bit_for_bit(lib, config, dt, shape):
    pr = _problem(config)
    lam, tol = (0.3, 1e-8) if config == 1 else (0.2, 1e-7)
    St = torch.tensor(pr["S"], device="cuda",
                      dtype=torch.float64 if dt == "f64" else torch.float32)
    outs = []
    for threads in (shape["block_threads"], 512):
        kw = dict(shape, block_threads=threads, w_in_lds=2)
        Wt = torch.full_like(St, float("nan"))
        om, info = lib.fit(St, lam, tol, 500, w_out=Wt, **kw)
        torch.cuda.synchronize()
        outs.append((om.cpu().numpy(), Wt.cpu().numpy(), info))
    (a, wa, ia), (b, wb, ib) = outs
    assert ia["block_threads"] == shape["block_threads"] and ib["block_threads"] == 512
    assert ia["w_in_lds"] == 0 and ia["code"] == 0
    assert np.array_equal(a, b)
    assert np.array_equal(wa, wb)
    assert ia["sweeps"] == ib["sweeps"] and ia["moved_pairs"] == ib["moved_pairs"]
    assert ia["active_sweeps"] == ib["active_sweeps"]


def test_wide_adjoint_sweeps_match_512_threads_bit_for_bit(lib):
    pr = _problem(2)
    St = torch.tensor(pr["S"], device="cuda")
    om, _ = lib.fit(St, 0.2, 1e-10, 2000)
    G = torch.tensor(np.random.default_rng(11).standard_normal(St.shape), device="cuda")
    G = G + G.T
    outs = []
    for threads in (768, 512):
        gS, glam, info = lib.backward(St, om, G, 1e-10, 2000, w_in_lds=2, block_threads=threads)
        torch.cuda.synchronize()
        outs.append((gS.cpu().numpy(), glam, info))
    (a, la, ia), (b, lb, ib) = outs
    assert ia["block_threads"] == 768 and ib["block_threads"] == 512
    assert np.array_equal(a, b) and ia["sweeps"] == ib["sweeps"]
    # dL/dlam sums the active set's terms with atomics: the order of the
    # additions varies from call to call (a few units in the 14th digit at
    # p = 1001), the terms do not
    assert la == pytest.approx(lb, rel=1e-12)


# ------------------------------------------------------------------ ragged sizes

RAGGED = [1, 2, 3, 4, 5, 6, 7, 16, 31, 33, 64, 65, 96, 97, 128, 129, 200, 257, 300]


@pytest.mark.parametrize("p", RAGGED)
def test_ragged_p_fp64(lib, p):
    pr = _problem(2, p=p, n=max(2 * p, 8))
    lam, tol = 0.15, 1e-9
    want, winfo, _ = _oracle(pr, lam, tol, 2000)
    got, ginfo = _gpu_fit(lib, pr["S"], lam, tol, 2000)
    _assert_parity64(pr["S"], got, ginfo, want, winfo, lam)
    if p >= 8:
        g2, i2 = _gpu_fit(lib, pr["S"], lam, tol, 2000, row_groups=min(p, 7), col_slices=3)
        assert np.array_equal(g2, got)
        g3, i3 = _gpu_fit(lib, pr["S"], lam, tol, 2000, row_groups=3, col_slices=2,
                          block_threads=64, w_in_lds=2, pending_depth=5)
        assert np.array_equal(g3, got)


@pytest.mark.parametrize("wl", [1, 2])
def test_two_rows_per_thread(lib, wl):
    # 100 rows in one row group on 64 threads: each thread carries two rows.
    pr = _problem(2, p=100, n=150)
    want, winfo, _ = _oracle(pr, 0.15, 1e-9, 2000)
    got, ginfo = _gpu_fit(lib, pr["S"], 0.15, 1e-9, 2000, row_groups=1, col_slices=2,
                          block_threads=64, w_in_lds=wl, pending_depth=3)
    _assert_parity64(pr["S"], got, ginfo, want, winfo, 0.15)


@pytest.mark.parametrize("wl", [1, 2])
def test_rows_spread_over_waves(lib, wl):
    # 100 rows in one row group on two waves of 50 rows each.
    pr = _problem(2, p=100, n=150)
    want, winfo, _ = _oracle(pr, 0.15, 1e-9, 2000)
    got, ginfo = _gpu_fit(lib, pr["S"], 0.15, 1e-9, 2000, row_groups=1, col_slices=2,
                          block_threads=128, w_in_lds=wl, pending_depth=3)
    _assert_parity64(pr["S"], got, ginfo, want, winfo, 0.15)


def test_long_logs_many_chunks(lib):
    # W in HBM, one column slice (many column chunks per row rewrite) and a
    # deep list of pending row updates.
    pr = _problem(2, p=300, n=150)
    want, winfo, _ = _oracle(pr, 0.05, 1e-9, 3000)
    got, ginfo = _gpu_fit(lib, pr["S"], 0.05, 1e-9, 3000, row_groups=8, col_slices=1,
                          block_threads=64, w_in_lds=2, pending_depth=6)
    _assert_parity64(pr["S"], got, ginfo, want, winfo, 0.05)


@pytest.mark.parametrize("p", [5, 64, 129, 257])
def test_ragged_p_n_less_than_p(lib, p):
    # n < p: S singular.  Parity still holds against the same-schedule oracle.
    pr = _problem(2, p=p, n=max(p // 2, 2))
    lam, tol = 0.2, 1e-9
    want, winfo, _ = _oracle(pr, lam, tol, 3000)
    got, ginfo = _gpu_fit(lib, pr["S"], lam, tol, 3000)
    _assert_parity64(pr["S"], got, ginfo, want, winfo, lam)


# ------------------------------------------------------------------ config 2

def test_config2_fp64_parity(lib):
    pr = _problem(2)
    want, winfo, wtr = _oracle(pr)
    got, ginfo = _gpu_fit(lib, pr["S"], pr["lam"], pr["tol"], pr["maxit"], trace=True)
    _assert_parity64(pr["S"], got, ginfo, want, winfo, pr["lam"])
    np.testing.assert_allclose(ginfo["delta_trace"], wtr, rtol=1e-5, atol=1e-12)


def test_config2_fp32_parity(lib):
    pr = _problem(2)
    want, winfo, _ = _oracle(pr)
    got, ginfo = _gpu_fit(lib, pr["S"], pr["lam"], pr["tol"], pr["maxit"], dtype=torch.float32,
                          check=False)
    assert ginfo["code"] == 0, ginfo
    err = np.abs(got - want).max()
    assert err <= TOL32, f"{err:.3e}"
    assert _support_mismatch(pr["S"], got, want, pr["lam"], 1e-4) == 0


# ------------------------------------------------------------------ inputs and paths

def test_gram_matches_oracle(lib):
    for (n, p) in [(100, 64), (37, 129), (500, 1001), (3, 70)]:
        rng = np.random.default_rng(n * 7 + p)
        y = rng.normal(size=(n, p))
        want = oracle.gram(y)
        got64 = lib.gram(torch.tensor(y, device="cuda")).cpu().numpy()
        np.testing.assert_allclose(got64, want, rtol=0, atol=1e-13 * np.abs(want).max())
        assert np.array_equal(got64, got64.T)
        got32 = lib.gram(torch.tensor(y, dtype=torch.float32, device="cuda")).double().cpu().numpy()
        np.testing.assert_allclose(got32, want, rtol=0, atol=2e-5 * np.abs(want).max())


def test_y_input_matches_oracle_on_its_gram(lib):
    pr = _problem(1)
    want, winfo, _ = _oracle(pr)
    Yt = torch.tensor(pr["y"], device="cuda")
    om, ginfo = lib.fit(Yt, 0.3, 1e-8, 500, kind="Y")
    got = om.cpu().numpy()
    _assert_parity64(pr["S"], got, ginfo, want, winfo, 0.3)


def test_warm_start_matches_oracle(lib):
    pr = _problem(2, p=150, n=120)
    lam = 0.25
    start, _, _ = oracle.pcd(pr["S"], 0.35, 1e-10, 2000)
    want, winfo, _ = oracle.pcd(pr["S"], lam, 1e-10, 2000, omega0=start)
    St = torch.tensor(pr["S"], device="cuda")
    om, ginfo = lib.fit(St, lam, 1e-10, 2000, omega0=torch.tensor(start, device="cuda"))
    _assert_parity64(pr["S"], om.cpu().numpy(), ginfo, want, winfo, lam)


def test_warm_start_at_solution_one_sweep(lib):
    pr = _problem(1)
    want, _, _ = oracle.pcd(pr["S"], 0.3, 1e-13, 5000)
    St = torch.tensor(pr["S"], device="cuda")
    om, info = lib.fit(St, 0.3, 1e-9, 50, omega0=torch.tensor(want, device="cuda"))
    assert info["sweeps"] == 1
    assert np.abs(om.cpu().numpy() - want).max() < 1e-11


def test_maxit_exhaustion_returns_last_iterate(lib):
    pr = _problem(2, p=90, n=60)
    want, winfo, _ = oracle.pcd(pr["S"], 0.1, 1e-300, 3)
    got, ginfo = _gpu_fit(lib, pr["S"], 0.1, 1e-300, 3, check=False)
    assert ginfo["code"] == 1 and ginfo["sweeps"] == 3
    assert np.abs(got - want).max() <= TOL64


def test_lambda_above_lambda_max_gives_diagonal(lib):
    pr = _problem(1)
    lam = oracle.lambda_max(pr["S"]) * 1.01
    got, info = _gpu_fit(lib, pr["S"], lam, 1e-10, 500)
    assert info["nnz_upper"] == 0
    off = got - np.diag(np.diag(got))
    assert np.all(off == 0)
    np.testing.assert_allclose(np.diag(got), 1 / np.sqrt(np.diag(pr["S"])), rtol=1e-13)


def test_nonpositive_diagonal_rejected(lib):
    S = np.eye(20)
    S[7, 7] = 0.0
    _, info = _gpu_fit(lib, S, 0.1, 1e-6, 10, check=False)
    assert info["code"] == -3


def test_nonfinite_input_rejected(lib):
    S = np.eye(130)
    S[3, 9] = S[9, 3] = np.nan
    _, info = _gpu_fit(lib, S, 0.1, 1e-6, 10, check=False)
    assert info["code"] == -2
