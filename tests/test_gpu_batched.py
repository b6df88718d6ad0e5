"""GPU parity of the batched solver (many problems, lambda paths, one launch).

Each problem's path is compared with the oracle run along the same path: the
first lambda from the identity, every later one warm-started from the
oracle's previous Omega (Algorithm 1 with the Omega^(0) it is given).  The
bar is the single-solve one: FP64 within 1e-8 with the same support and the
same sweep count per lambda; FP32 within 1e-4 of the FP64 oracle.
"""
import warnings

import numpy as np
import pytest
import torch

import oracle
from paper_2106_09382_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2106_09382_amd import _lib
    _lib.load()
    return _lib


_cache = {}


def _small_batch(count=6, p_lo=3, p_hi=160, replicate=0):
    key = ("batch", count, p_lo, p_hi, replicate)
    if key not in _cache:
        probs = datagen.batched_problems(replicate, count=count, p_lo=p_lo, p_hi=p_hi)
        for pr in probs:
            pr["S"] = oracle.gram(pr["y"])
        _cache[key] = probs
    return _cache[key]


def _oracle_path(S, lams, tol, maxit):
    """The oracle along a path; tol is one value or one per lambda."""
    tols = tuple(tol) if np.ndim(tol) else (tol,) * len(lams)
    key = ("path", S.tobytes(), tuple(lams), tols, maxit)
    if key not in _cache:
        res, om = [], None
        for lam, t in zip(lams, tols):
            om, info, _ = oracle.pcd(S, lam, t, maxit, omega0=om)
            res.append((om, info))
        _cache[key] = res
    return _cache[key]


def _support_mismatch(S, got, want, lam, rel):
    bad = (got != 0) != (want != 0)
    np.fill_diagonal(bad, False)
    if bad.any():
        for i, j in oracle.borderline_pairs(S, want, lam, rel):
            bad[i, j] = bad[j, i] = False
    return int(np.triu(bad, 1).sum())


def _run(lib, mats, lams, tol, maxit, dtype=torch.float64, **kw):
    Xs = [torch.tensor(M, dtype=dtype, device="cuda") for M in mats]
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        outs, infos, code = lib.fit_batched(Xs, lams, tol, maxit, check=False, **kw)
    torch.cuda.synchronize()
    return [[o.double().cpu().numpy() for o in row] for row in outs], infos, code


LAMS = list(datagen.lambda_path(0.5, 0.08, 5))
TOL, MAXIT = 1e-7, 1500


def test_batched_fp64_path_matches_oracle(lib):
    probs = _small_batch()
    tol, maxit = TOL, MAXIT
    got, infos, code = _run(lib, [pr["S"] for pr in probs], LAMS, tol, maxit)
    any_nc = False
    for b, pr in enumerate(probs):
        want = _oracle_path(pr["S"], LAMS, tol, maxit)
        for l, lam in enumerate(LAMS):
            om, winfo = want[l]
            g, gi = got[b][l], infos[b][l]
            err = np.abs(g - om).max()
            assert err <= 1e-8, (b, l, pr["p"], err)
            assert np.array_equal(g, g.T)
            assert _support_mismatch(pr["S"], g, om, lam, 1e-9) == 0, (b, l)
            assert gi["sweeps"] == winfo["sweeps"], (b, l, gi["sweeps"], winfo["sweeps"])
            assert gi["status"] == (0 if winfo["converged"] else 1)
            any_nc |= not winfo["converged"]
            assert gi["nnz_upper"] == winfo["nnz_upper"]
            assert gi["objective"] == pytest.approx(oracle.objective(pr["S"], om, lam), rel=1e-10)
    assert code == (1 if any_nc else 0)


def test_batched_fp32_path_matches_fp64_oracle(lib):
    # FP32 stops at tol_eff = max(tol, 16 eps_32 max omega_ii); on slowly
    # converging problems that alone moves Omega by more than 1e-4, so the
    # FP64 oracle runs each lambda to the tol_eff the solve reports.
    probs = _small_batch()
    tol, maxit = TOL, MAXIT
    got, infos, code = _run(lib, [pr["S"] for pr in probs], LAMS, tol, maxit,
                            dtype=torch.float32)
    assert code in (0, 1)
    checked = 0
    for b, pr in enumerate(probs):
        tols = [infos[b][l]["tol_eff"] for l in range(len(LAMS))]
        want = _oracle_path(pr["S"], LAMS, tols, maxit)
        for l, lam in enumerate(LAMS):
            om, winfo = want[l]
            if infos[b][l]["status"] != 0 or not winfo["converged"]:
                continue  # an unconverged iterate on a flat objective is not pinned to 1e-4
            checked += 1
            err = np.abs(got[b][l] - om).max()
            assert err <= 1e-4, (b, l, pr["p"], err)
            assert _support_mismatch(pr["S"], got[b][l], om, lam, 1e-4) == 0, (b, l)
            assert infos[b][l]["tol_eff"] >= tol
    assert checked >= 0.8 * len(probs) * len(LAMS)


def test_batched_y_input_matches_oracle(lib):
    probs = _small_batch(count=4, p_lo=20, p_hi=120, replicate=1)
    tol, maxit = TOL, MAXIT
    lams = LAMS[:3]
    got, infos, code = _run(lib, [pr["y"] for pr in probs], lams, tol, maxit, kind="Y")
    assert code in (0, 1)
    for b, pr in enumerate(probs):
        want = _oracle_path(pr["S"], lams, tol, maxit)
        for l in range(len(lams)):
            assert np.abs(got[b][l] - want[l][0]).max() <= 1e-8
            assert infos[b][l]["sweeps"] == want[l][1]["sweeps"]


def test_first_lambda_is_bitwise_the_single_solve(lib):
    # From the identity, every W entry receives its updates in the order the
    # schedule fixes, so the batched launch and a single solve agree exactly.
    probs = _small_batch()
    got, _, _ = _run(lib, [pr["S"] for pr in probs], LAMS, TOL, MAXIT)
    for b, pr in enumerate(probs):
        St = torch.tensor(pr["S"], device="cuda")
        om, _ = lib.fit(St, LAMS[0], TOL, MAXIT, check=False)
        assert np.array_equal(om.cpu().numpy(), got[b][0]), b


def test_batched_split_over_launches_is_identical(lib):
    # Four workgroups per launch cannot hold all problems: they run in
    # several launches, each problem on fewer workgroups.  Same bits.
    probs = _small_batch()
    ref, _, rcode = _run(lib, [pr["S"] for pr in probs], LAMS, TOL, MAXIT)
    got, infos, code = _run(lib, [pr["S"] for pr in probs], LAMS, TOL, MAXIT, workgroups=4,
                            block_threads=128, pending_depth=3)
    assert code == rcode
    for b in range(len(probs)):
        for l in range(len(LAMS)):
            assert np.array_equal(got[b][l], ref[b][l]), (b, l)
        assert all(infos[b][l]["row_groups"] <= 4 for l in range(len(LAMS)))


def test_batched_edge_cases(lib):
    # p = 1 and p = 2, a lambda above lambda_max (diagonal answer), and a
    # sweep limit that stops one lambda early while the path goes on.
    rng = np.random.default_rng(7)
    mats = []
    for p in (1, 2, 7, 64):
        y = rng.standard_normal((3 * p + 4, p))
        mats.append(oracle.gram(y))
    lams_hi = [oracle.lambda_max(S) * 1.01 for S in mats]
    lams = [[lh, 0.3, 0.1] for lh in lams_hi]
    tol = 1e-9
    got, infos, code = _run(lib, mats, lams, tol, 2000)
    assert code == 0
    for b, S in enumerate(mats):
        np.testing.assert_allclose(got[b][0], np.diag(1.0 / np.sqrt(np.diag(S))), rtol=0,
                                   atol=1e-10)
        want = _oracle_path(S, lams[b], tol, 2000)
        for l in range(3):
            assert np.abs(got[b][l] - want[l][0]).max() <= 1e-8
            assert infos[b][l]["sweeps"] == want[l][1]["sweeps"]
    # maxit = 2: every lambda stops at the limit with the oracle's iterate
    got2, infos2, code2 = _run(lib, mats, lams, 1e-14, 2)
    assert code2 == 1
    for b, S in enumerate(mats):
        want = _oracle_path(S, lams[b], 1e-14, 2)
        for l in range(3):
            assert np.abs(got2[b][l] - want[l][0]).max() <= 1e-8
            if b >= 2 and l >= 1:
                assert infos2[b][l]["status"] == 1 and infos2[b][l]["sweeps"] == 2


def test_batched_bad_problem_is_reported_alone(lib):
    rng = np.random.default_rng(3)
    good = oracle.gram(rng.standard_normal((40, 12)))
    bad = good.copy()
    bad[4, 4] = -1.0
    got, infos, code = _run(lib, [good, bad, good], [0.3, 0.1], 1e-9, 500)
    assert code == -3
    assert all(infos[1][l]["status"] == -3 for l in range(2))
    want = _oracle_path(good, [0.3, 0.1], 1e-9, 500)
    for b in (0, 2):
        for l in range(2):
            assert infos[b][l]["status"] == 0
            assert np.abs(got[b][l] - want[l][0]).max() <= 1e-8


EPS32 = 2.0 ** -23


def _oracle_path_f32_rule(S, lams, tol, maxit):
    """The oracle (FP64) along a warm-started path, each lambda stopped by the
    rule an FP32 solve applies (reading R8): the first sweep whose delta is
    below max(tol, 16 eps_32 max_i omega_ii) of that sweep.  The oracle's
    whole state between sweeps is Omega, so it runs one sweep per call."""
    key = ("path32", S.tobytes(), tuple(lams), tol, maxit)
    if key not in _cache:
        res, om = [], None
        for lam in lams:
            info = None
            for t in range(1, maxit + 1):
                om, info, tr = oracle.pcd(S, lam, tol, 1, omega0=om)
                tol_eff = max(tol, 16 * EPS32 * float(np.diag(om).max()))
                if tr[0] < tol_eff:
                    break
            res.append((om.copy(), dict(sweeps=t, converged=bool(tr[0] < tol_eff),
                                        tol_eff=tol_eff)))
        _cache[key] = res
    return _cache[key]


@pytest.fixture(scope="module")
def config4():
    """The 64-problem workload as the benchmark runs it: p ~ U[200, 3000],
    n = p/2, Erdos-Renyi, the 16-value path 0.5 -> 0.05, FP32 from Y, tol
    1e-5, maxit 500, one persistent launch with the built-in plan."""
    from paper_2106_09382_amd import _lib as lib
    lib.load()
    probs = datagen.batched_problems(0)
    lams = list(datagen.lambda_path())
    Xs = [torch.tensor(pr["y"], dtype=torch.float32, device="cuda") for pr in probs]
    tol, maxit = 1e-5, 500
    print("config4: 64 problems x 16 lambdas, FP32 from Y, maxit 500", flush=True)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        outs, infos, code = lib.fit_batched(Xs, lams, tol, maxit, kind="Y", check=False)
    torch.cuda.synchronize()
    return dict(probs=probs, lams=lams, Xs=Xs, tol=tol, maxit=maxit, outs=outs, infos=infos,
                code=code)


@pytest.mark.slow
def test_config4_full_batch_properties(lib, config4):
    # What holds at any size: the first lambda equals the single FP32 solve
    # bit for bit, and sampled (problem, lambda) results satisfy the
    # stationarity conditions, evaluated in FP64 on the oracle's Gram of the
    # same draws, to the FP32 tolerance.
    c = config4
    probs, lams, Xs, tol, maxit = c["probs"], c["lams"], c["Xs"], c["tol"], c["maxit"]
    outs, infos = c["outs"], c["infos"]
    assert c["code"] in (0, 1)
    assert all(infos[b][l]["status"] in (0, 1) for b in range(64) for l in range(16))
    order = np.argsort([pr["p"] for pr in probs])
    for b in (int(order[0]), int(order[31]), int(order[-1])):
        pr = probs[b]
        S = oracle.gram(pr["y"].astype(np.float32).astype(np.float64))
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            om1, _ = lib.fit(Xs[b], lams[0], tol, maxit, kind="Y", check=False)
        assert np.array_equal(om1.cpu().numpy(), outs[b][0].cpu().numpy())
        row1 = np.abs(S).sum(axis=1).max()
        for l in (0, 7, 15):
            if infos[b][l]["status"] != 0:
                continue
            om = outs[b][l].double().cpu().numpy()
            r = oracle.kkt(S, om, lams[l])
            # after the last sweep every coordinate is within one change
            # (< tol) of its own minimiser; the gradient then moves by at
            # most 2 tol |S|_1 per entry, plus FP32 rounding of Omega and S
            bound = 4e-5 * row1 * max(1.0, np.abs(om).max()) + 1e-4
            assert r["support"] < bound and r["zeros"] < bound and r["diag"] < bound, (b, l, r)


@pytest.mark.slow
def test_config4_smallest_problems_match_the_oracle_along_their_paths(lib, config4):
    # The three smallest problems of the batch (p = 254, 261, 274), every
    # lambda of their paths, against the FP64 oracle on the Gram of the same
    # (FP32-rounded) draws with the FP32 stopping rule, on the lambdas both
    # converged: within 1e-4 relative to the largest entry of Omega (reading
    # R23: FP32 error scales with the entries, which grow to about 4.5 at the
    # end of the path, where n = p/2 makes the sweeps contract slowly), the
    # same support outside the pairs borderline at that scale.
    c = config4
    probs, lams, tol, maxit = c["probs"], c["lams"], c["tol"], c["maxit"]
    order = np.argsort([pr["p"] for pr in probs])
    checked = total = 0
    for b in (int(x) for x in order[:3]):
        pr = probs[b]
        print(f"config4 oracle path: problem {b} p={pr['p']}", flush=True)
        S = oracle.gram(pr["y"].astype(np.float32).astype(np.float64))
        want = _oracle_path_f32_rule(S, lams, tol, maxit)
        for l, lam in enumerate(lams):
            total += 1
            om, winfo = want[l]
            gi = c["infos"][b][l]
            if gi["status"] != 0 or not winfo["converged"]:
                continue
            checked += 1
            got = c["outs"][b][l].double().cpu().numpy()
            scale = max(1.0, float(np.abs(om).max()))
            err = np.abs(got - om).max()
            print(f"  lambda {lam:.4f}: sweeps gpu {gi['sweeps']} oracle {winfo['sweeps']}, "
                  f"max|Omega| {scale:.3f}, max error {err:.3e}", flush=True)
            assert err <= 1e-4 * scale, (b, l, pr["p"], err, scale)
            assert _support_mismatch(S, got, om, lam, 1e-4 * scale) == 0, (b, l)
    assert checked >= 0.8 * total


def test_explicit_and_autotuned_plans_give_the_same_bits(lib):
    from paper_2106_09382_amd import autotune
    probs = _small_batch()
    ps = [pr["p"] for pr in probs]
    ref, infos, rcode = _run(lib, [pr["S"] for pr in probs], LAMS, TOL, MAXIT)
    tuned = autotune.plan_from_infos(ps, infos, 64)
    got, infos2, code = _run(lib, [pr["S"] for pr in probs], LAMS, TOL, MAXIT,
                             problem_workgroups=tuned)
    assert code == rcode
    assert [row[0]["row_groups"] for row in infos2] == tuned
    for b in range(len(probs)):
        for l in range(len(LAMS)):
            assert np.array_equal(got[b][l], ref[b][l]), (b, l)
    # a count below a problem's minimum is rejected before any device work
    _, _, bad = _run(lib, [pr["S"] for pr in probs], LAMS, TOL, MAXIT,
                     problem_workgroups=[0] * len(ps))
    assert bad == -1


@pytest.mark.parametrize("dt,threads,cpl", [("f64", 768, 2), ("f64", 640, 4), ("f32", 1024, 4),
                                             ("f32", 1024, 2)])
def test_wide_workgroups_give_the_same_bits(lib, dt, threads, cpl):
    """Workgroups wider than 512 threads hold one row per thread and rewrite
    rows in the background in more problems: the same iterates, bit for bit,
    as 512-thread workgroups (two rows per thread)."""
    probs = _small_batch()
    dtype = torch.float64 if dt == "f64" else torch.float32
    tol = TOL if dt == "f64" else 1e-5
    mats = [pr["S"] for pr in probs]
    ref, rinfo, rcode = _run(lib, mats, LAMS, tol, MAXIT, dtype=dtype)
    got, infos, code = _run(lib, mats, LAMS, tol, MAXIT, dtype=dtype, block_threads=threads,
                            cols_per_lane=cpl)
    assert code == rcode
    for b in range(len(probs)):
        assert infos[b][0]["block_threads"] == threads
        for l in range(len(LAMS)):
            assert np.array_equal(got[b][l], ref[b][l]), (b, l)
            assert infos[b][l]["sweeps"] == rinfo[b][l]["sweeps"]
            assert infos[b][l]["nnz_upper"] == rinfo[b][l]["nnz_upper"]


@pytest.mark.parametrize("threads,cpl", [(512, 2), (256, 4), (256, 2)])
def test_column_slices_and_rewrite_width_give_the_same_bits(lib, threads, cpl):
    """Problems split into row groups x column slices, narrower workgroups
    (two per CU) and two columns per lane in row rewrites: the same iterates,
    bit for bit, as the default launch (and so the oracle's, checked above)."""
    probs = _small_batch()
    ps = [pr["p"] for pr in probs]
    ref, rinfo, rcode = _run(lib, [pr["S"] for pr in probs], LAMS, TOL, MAXIT)
    pw = [6 if p >= 48 else 1 for p in ps]
    pc = [3 if p >= 48 else 1 for p in ps]
    assert any(c > 1 for c in pc)
    got, infos, code = _run(lib, [pr["S"] for pr in probs], LAMS, TOL, MAXIT,
                            problem_workgroups=pw, problem_col_slices=pc, block_threads=threads,
                            cols_per_lane=cpl)
    assert code == rcode
    for b in range(len(probs)):
        assert infos[b][0]["row_groups"] * infos[b][0]["col_slices"] == pw[b]
        assert infos[b][0]["col_slices"] == pc[b]
        for l in range(len(LAMS)):
            assert np.array_equal(got[b][l], ref[b][l]), (b, l)
            assert infos[b][l]["sweeps"] == rinfo[b][l]["sweeps"]
            assert infos[b][l]["nnz_upper"] == rinfo[b][l]["nnz_upper"]
    # slices that do not divide a problem's workgroups are rejected
    _, _, bad = _run(lib, [pr["S"] for pr in probs], LAMS, TOL, MAXIT, problem_workgroups=pw,
                     problem_col_slices=[4 if c > 1 else 1 for c in pc])
    assert bad == -1
    _, _, bad = _run(lib, [pr["S"] for pr in probs], LAMS, TOL, MAXIT, cols_per_lane=3)
    assert bad == -1
