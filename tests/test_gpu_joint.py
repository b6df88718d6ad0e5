"""GPU parity of the joint two-population solve (concord_fit_joint, Section 6)
against the oracle (oracle/joint.py), through the C ABI.

* FP64: every element within 1e-8 of the oracle's joint PCD on the same S
  bytes; pair by pair the same support in each population and the same
  fused pattern (which pairs differ between the populations), leaving out
  only blocks whose case decision is within rounding; the same sweep count; one
  workgroup per population and several, odd and even p, W in LDS and in
  HBM, ragged row groups and column slices.
* lam2 = 0 and a fixed sweep count: bit for bit two independent GPU solves.
* A large lam2: both outputs identical, equal to the GPU solve on (S_1 + S_2)/2.
* FP32 against the FP64 oracle within 1e-4; the Y path equals the S path;
  the reported objective, supports and delta trace; a warm start.
* The full-size workload (p = 5000, n = 2000, two ER populations that differ
  in 10 % of their edges, lam1 = 0.1, lam2 = 0.05), in the launch shape the
  benchmark times: sampled blocks are fixed points of the block updates
  (computed by the oracle with direct sums) and the output does not depend
  on the launch shape.
"""
import warnings

import numpy as np
import pytest
import torch

import oracle
from oracle import joint
from paper_2106_09382_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2106_09382_amd import _lib
    _lib.load()
    return _lib


_cache = {}


def _grams(p, n, seed, changed=0.2):
    key = (p, n, seed, changed)
    if key not in _cache:
        jp = datagen.joint_problem(seed, p=p, n=n, changed=changed)
        _cache[key] = (oracle.gram(jp["y"][0]), oracle.gram(jp["y"][1]), jp)
    return _cache[key]


def _gpu(lib, S1, S2, lam1, lam2, tol, maxit, dtype=torch.float64, **kw):
    a = torch.tensor(S1, dtype=dtype, device="cuda")
    b = torch.tensor(S2, dtype=dtype, device="cuda")
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        o1, o2, info = lib.fit_joint(a, b, lam1, lam2, tol, maxit, check=False, **kw)
    torch.cuda.synchronize()
    return o1.double().cpu().numpy(), o2.double().cpu().numpy(), info


def _patterns_equal(S1, S2, g1, g2, w1, w2, lam1, lam2, rel):
    """Pair by pair (i < j): the support of each population and the fused
    pattern (omega^1_ij != omega^2_ij) agree, leaving out only the blocks
    whose case decision at the oracle's estimate is within rounding
    (oracle.joint.borderline_pairs, reading R22).  Returns the mismatches."""
    p = S1.shape[0]
    iu = np.triu_indices(p, 1)
    keep = np.ones(iu[0].size, dtype=bool)
    bl = joint.borderline_pairs(S1, S2, w1, w2, lam1, lam2, rel)
    if len(bl):
        lin = {int(i) * p + int(j) for i, j in bl}
        keep = np.array([int(i) * p + int(j) not in lin for i, j in zip(*iu)])
    out = {}
    for name, a, b in (("support 1", g1[iu] != 0, w1[iu] != 0),
                       ("support 2", g2[iu] != 0, w2[iu] != 0),
                       ("fused pattern", g1[iu] != g2[iu], w1[iu] != w2[iu])):
        out[name] = int(((a != b) & keep).sum())
    return out


CASES = [
    # p, n, lam1, lam2, seed, launch options
    (1, 10, 0.1, 0.05, 1, {}),
    (2, 10, 0.1, 0.05, 2, {}),
    (17, 40, 0.1, 0.02, 3, {}),
    (40, 30, 0.15, 0.05, 4, {}),
    (64, 120, 0.1, 0.01, 5, {}),
    (97, 150, 0.2, 0.05, 6, {}),
    (130, 90, 0.15, 0.03, 7, {}),
    (130, 90, 0.15, 0.03, 7, dict(row_groups=5, col_slices=3)),
    (130, 90, 0.15, 0.03, 7, dict(row_groups=4, col_slices=2, w_in_lds=2, pending_depth=3)),
    (211, 300, 0.1, 0.02, 8, dict(row_groups=16, col_slices=4, block_threads=64)),
    # two rows per thread, W in HBM and in LDS
    (300, 150, 0.15, 0.05, 16, dict(row_groups=2, col_slices=2, block_threads=128, w_in_lds=2)),
    (160, 200, 0.1, 0.03, 17, dict(row_groups=2, col_slices=2, block_threads=64, w_in_lds=1)),
    (301, 150, 0.2, 0.1, 9, {}),
    # wide workgroups: one row per thread, W in HBM, rewrites in the background
    (211, 300, 0.1, 0.02, 8, dict(row_groups=16, col_slices=4, block_threads=768, w_in_lds=2)),
    (300, 150, 0.15, 0.05, 16, dict(row_groups=4, col_slices=2, block_threads=640, w_in_lds=2,
                                    pending_depth=5)),
]


@pytest.mark.parametrize("p,n,lam1,lam2,seed,opts", CASES)
def test_joint_fp64_matches_oracle(lib, p, n, lam1, lam2, seed, opts):
    print(f"joint parity p={p} n={n} lam1={lam1} lam2={lam2} opts={opts}", flush=True)
    S1, S2, _ = _grams(p, n, seed)
    tol = 1e-10
    g1, g2, info = _gpu(lib, S1, S2, lam1, lam2, tol, 3000, **opts)
    w1, w2, winfo, wtr = joint.pcd(S1, S2, lam1, lam2, tol, 3000)
    assert info["code"] == 0 and winfo["converged"]
    assert info["sweeps"] == winfo["sweeps"]
    assert np.abs(g1 - w1).max() <= 1e-8 and np.abs(g2 - w2).max() <= 1e-8
    assert np.array_equal(g1, g1.T) and np.array_equal(g2, g2.T)
    mism = _patterns_equal(S1, S2, g1, g2, w1, w2, lam1, lam2, 1e-9)
    assert all(v == 0 for v in mism.values()), mism
    assert info["nnz_upper"] == tuple(int((np.triu(g, 1) != 0).sum()) for g in (g1, g2))
    iu = np.triu_indices(p, 1)
    assert info["differ_upper"] == int((g1[iu] != g2[iu]).sum())
    if opts.get("row_groups"):
        assert info["row_groups"] == min(opts["row_groups"], p)


@pytest.mark.parametrize("p,sweeps", [(9, 4), (130, 3), (300, 2)])
def test_lam2_zero_is_two_independent_gpu_solves(lib, p, sweeps):
    S1, S2, _ = _grams(p, p + 20, 10)
    g1, g2, info = _gpu(lib, S1, S2, 0.12, 0.0, 1e-300, sweeps)
    assert info["sweeps"] == sweeps
    for S, g in ((S1, g1), (S2, g2)):
        St = torch.tensor(S, device="cuda")
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            want, _ = lib.fit(St, 0.12, 1e-300, sweeps, check=False)
        assert np.array_equal(g, want.cpu().numpy())


def test_large_lam2_fuses_the_populations(lib):
    S1, S2, _ = _grams(150, 200, 11)
    g1, g2, info = _gpu(lib, S1, S2, 0.15, 1e3, 1e-12, 3000)
    assert info["code"] == 0 and info["differ_upper"] == 0
    assert np.array_equal(g1, g2)
    want, _ = lib.fit(torch.tensor(0.5 * (S1 + S2), device="cuda"), 0.15, 1e-12, 3000)
    assert np.abs(g1 - want.cpu().numpy()).max() < 1e-10


def test_fp32_close_to_fp64_oracle(lib):
    S1, S2, _ = _grams(97, 150, 12)
    g1, g2, info = _gpu(lib, S1, S2, 0.2, 0.05, 1e-7, 3000, dtype=torch.float32)
    assert info["code"] in (0, 1)
    w1, w2, _, _ = joint.pcd(S1, S2, 0.2, 0.05, max(info["tol_eff"], 1e-12), 3000)
    assert np.abs(g1 - w1).max() <= 1e-4 and np.abs(g2 - w2).max() <= 1e-4
    mism = _patterns_equal(S1, S2, g1, g2, w1, w2, 0.2, 0.05, 1e-4)
    assert all(v == 0 for v in mism.values()), mism


def test_y_input_equals_s_input(lib):
    _, _, jp = _grams(120, 80, 13)
    Y1 = torch.tensor(jp["y"][0], device="cuda")
    Y2 = torch.tensor(jp["y"][1], device="cuda")
    a1, a2, ia = lib.fit_joint(Y1, Y2, 0.15, 0.03, 1e-10, 3000, kind="Y")
    S1, S2 = lib.gram(Y1), lib.gram(Y2)
    b1, b2, ib = lib.fit_joint(S1, S2, 0.15, 0.03, 1e-10, 3000)
    assert torch.equal(a1, b1) and torch.equal(a2, b2)
    assert ia["sweeps"] == ib["sweeps"] and ia["gram_ms"] > 0


def test_objective_trace_and_warm_start(lib):
    S1, S2, _ = _grams(64, 100, 14)
    St1, St2 = torch.tensor(S1, device="cuda"), torch.tensor(S2, device="cuda")
    o1, o2, info = lib.fit_joint(St1, St2, 0.1, 0.02, 1e-11, 3000, trace=True)
    g1, g2 = o1.cpu().numpy(), o2.cpu().numpy()
    assert info["objective"] == pytest.approx(joint.objective(S1, S2, g1, g2, 0.1, 0.02),
                                              rel=1e-10)
    tr = info["delta_trace"]
    assert len(tr) == info["sweeps"] and tr[-1] < 1e-11 <= tr[-2]
    assert tr[-1] == info["delta"]
    r = joint.kkt(S1, S2, g1, g2, 0.1, 0.02)
    assert r["pairs"] < 1e-8 and r["diag"] < 1e-8
    # warm start at the solution: one sweep, same point
    w1, w2, winfo = lib.fit_joint(St1, St2, 0.1, 0.02, 1e-9, 3000, omega0=(o1, o2))
    assert winfo["sweeps"] == 1
    assert (w1 - o1).abs().max().item() < 1e-9 and (w2 - o2).abs().max().item() < 1e-9
    # one population warm, the other from the identity
    h1, h2, _ = lib.fit_joint(St1, St2, 0.1, 0.02, 1e-11, 3000, omega0=(o1, None))
    assert (h1 - o1).abs().max().item() < 1e-8 and (h2 - o2).abs().max().item() < 1e-8


def test_rejects_bad_input(lib):
    from paper_2106_09382_amd._lib import ConcordError
    S1, S2, _ = _grams(30, 50, 15)
    bad = S2.copy()
    bad[4, 4] = -1.0
    with pytest.raises(ConcordError) as e:
        lib.fit_joint(torch.tensor(S1, device="cuda"), torch.tensor(bad, device="cuda"), 0.1, 0.1)
    assert e.value.code == -3
    bad = S1.copy()
    bad[2, 3] = float("nan")
    with pytest.raises(ConcordError) as e:
        lib.fit_joint(torch.tensor(bad, device="cuda"), torch.tensor(S2, device="cuda"), 0.1, 0.1)
    assert e.value.code == -2


@pytest.fixture(scope="module")
def fullsize():
    jp = datagen.joint_problem(0)
    return oracle.gram(jp["y"][0]), oracle.gram(jp["y"][1])


@pytest.mark.slow
def test_fullsize_fixed_point_and_shape_independence(lib, fullsize):
    S1, S2 = fullsize
    p, lam1, lam2, tol = S1.shape[0], 0.1, 0.05, 1e-6
    print(f"joint full size p={p}", flush=True)
    g1, g2, info = _gpu(lib, S1, S2, lam1, lam2, tol, 500)
    assert info["code"] == 0
    rng = np.random.default_rng(21)
    nz = np.argwhere(np.triu((g1 != 0) | (g2 != 0), 1))
    picks = [tuple(nz[k]) for k in rng.choice(len(nz), 200, replace=False)]
    zz = rng.integers(0, p, size=(200, 2))
    picks += [tuple(x) for x in zz if x[0] != x[1]]
    picks += [(i, i) for i in rng.choice(p, 100, replace=False)]
    worst = 0.0
    for i, j in picks:
        x1, x2 = joint.block_update_at(S1, S2, g1, g2, int(i), int(j), lam1, lam2)
        worst = max(worst, abs(x1 - g1[i, j]), abs(x2 - g2[i, j]))
    assert worst < 50 * tol, worst
    assert info["differ_upper"] > 0 and info["differ_upper"] < min(info["nnz_upper"])
    h1, h2, hinfo = _gpu(lib, S1, S2, lam1, lam2, tol, 500, row_groups=32, col_slices=4)
    assert hinfo["sweeps"] == info["sweeps"]
    assert np.array_equal(h1, g1) and np.array_equal(h2, g2)


def test_y_input_with_different_sample_sizes(lib):
    # n_1 != n_2: each population's S is its own Y^T Y / n_m (the S-scale
    # objective weighs the two losses equally)
    jp1 = datagen.joint_problem(18, p=90, n=60)
    jp2 = datagen.joint_problem(18, p=90, n=200)
    Y1 = torch.tensor(jp1["y"][0], device="cuda")
    Y2 = torch.tensor(jp2["y"][1], device="cuda")
    a1, a2, ia = lib.fit_joint(Y1, Y2, 0.15, 0.03, 1e-11, 3000, kind="Y")
    b1, b2, ib = lib.fit_joint(lib.gram(Y1), lib.gram(Y2), 0.15, 0.03, 1e-11, 3000)
    assert torch.equal(a1, b1) and torch.equal(a2, b2) and ia["sweeps"] == ib["sweeps"]
    S1, S2 = oracle.gram(jp1["y"][0]), oracle.gram(jp2["y"][1])
    w1, w2, winfo, _ = joint.pcd(S1, S2, 0.15, 0.03, 1e-11, 3000)
    assert winfo["converged"]
    assert np.abs(a1.cpu().numpy() - w1).max() < 1e-8 and np.abs(a2.cpu().numpy() - w2).max() < 1e-8
