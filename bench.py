#!/usr/bin/env python3
"""Benchmark: CONCORD-PCD time-to-tolerance and sweep bandwidth on one MI355X.

Workload (default): p = 5000 variables, n = 2000 samples, Erdos-Renyi true
precision matrix (edge probability 3/p, weights U[0.3, 0.5] with random sign,
unit diagonal), Y ~ N(0, Omega0^{-1}) drawn with seed 3000, lambda = 0.1,
tol = 1e-6, FP64.  One step = one whole solve from Y already resident in HBM:
MFMA Gram S = Y^T Y / n, set-up, all sweeps to the tolerance, dense Omega out.

Reported value: sweep GB/s = algorithmic bytes of all sweeps / wall time of
the timed solves.  Algorithmic bytes of one sweep (maintained-product form):
  e * (1.5 p m + 6 p N_pairs + 3 p N_diag)
with e the element size, m = p_even - 1 colours (each colour reads p numerator
entries and p/2 omegas), N_pairs the pairs whose omega_ij moved (each moves
two rows of W: read S row, read and write W row, twice) and N_diag the
diagonals that moved (one row each).

Also printed: the sweep kernel's own bandwidth (event-timed, `roofline`) and
the CPU oracle timed on a bounded sample of the same problem (`cpu_baseline`),
and two side measurements on their own workloads:

* `batched`: 64 independent Erdos-Renyi problems, p ~ U[200, 3000], n = p/2,
  each on a 16-value lambda path 0.5 -> 0.05 with warm starts, FP32, tol 1e-5,
  in one persistent launch (concord_fit_batched), timed once with the built-in
  workgroup plan and once with the plan the autotuner builds from that run's
  per-problem device times (the reported rate); solves/s against a loop of
  plain single-solve fits along the same paths at the same tolerance, timed
  on all 64 problems (--plain-sample times every 4th problem by size and
  interpolates linearly in p instead).
* `floor`: the sweep's two floors.  Bandwidth: B_sweep / 8 TB/s.  Sync: m
  dependent colour steps x the cost of one step with nothing to move, measured
  as a solve at lambda = 1000 lambda_max-scale (no pair ever moves; two sweeps
  of pure dependency chain, same launch shape).  T_floor = max of the two per
  sweep, `frac` = T_floor / t_sweep, `binds` names the larger.
* `fp32`: the same solve in FP32 (S 100 MB + W 100 MB, the cache-resident
  regime), with a cache-resident copy bandwidth (a 64 MiB device copy,
  repeated) beside the HBM peak.
* `active_set`: time to tolerance of the same workload at lambda 0.1 and 0.2,
  plain Algorithm 1 against the active-set sweeps (full round-robin sweeps
  decide convergence; between them, sweeps over a greedy colouring of the
  support).
* `backward`: the implicit gradient (concord_backward) at p = 2000, n = 1000,
  chain Omega_0, lambda = 0.15, L = |Omega-hat - Omega_0|_F^2, FP64, against the
  forward solve at the same tolerance.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sweep_bytes(p: int, elem: int, sweeps: int, moved_pairs: int, moved_diag: int) -> float:
    m = p + (p & 1) - 1
    return float(elem) * (1.5 * p * m * sweeps + 6.0 * p * moved_pairs + 3.0 * p * moved_diag)


def cpu_oracle_baseline(S, p: int, lam: float, elem: int, gpu_sweeps: int, bytes_per_sweep: float,
                        budget_s: float) -> dict:
    """Time the CPU oracle (serial, FP64, direct sums) on a bounded sample:
    the first c colour steps of sweep 1, extrapolated to one sweep."""
    import oracle

    m = p + (p & 1) - 1
    # time per colour from two short runs (their difference leaves out the
    # call's fixed set-up), then as many colours as fill the budget
    ts = []
    for cl in (2, 6):
        t0 = time.perf_counter()
        oracle.pcd(S, lam, 1e-300, 1, colour_limit=cl)
        ts.append(time.perf_counter() - t0)
    per = max((ts[1] - ts[0]) / 4, 1e-9)
    c = int(max(2, min(m, (budget_s - max(ts[0] - 2 * per, 0.0)) / per)))
    t0 = time.perf_counter()
    oracle.pcd(S, lam, 1e-300, 1, colour_limit=c)
    dt = time.perf_counter() - t0
    t_sweep = dt / c * m
    return {
        "value": bytes_per_sweep / t_sweep / 1e9,
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"first {c} of {m} colour steps of sweep 1 of the oracle's serial direct-sum "
                   f"PCD on the same S ({dt:.1f} s), extrapolated to a sweep"),
        "t_sweep_s": t_sweep,
        "time_to_tol_s_extrapolated": t_sweep * gpu_sweeps,
        "host_cpu": _cpu_model(),
        "host_threads": os.cpu_count(),
    }


def cpu_wform_baseline(S, p: int, lam: float, gpu_bytes: float, budget_s: float) -> dict:
    """Time the CPU baseline with a maintained W (FP64): the whole first sweep
    on all host threads, and a bounded sample of sweep 1 on one thread.  Each
    rate is algorithmic bytes / time; time to tolerance is extrapolated as
    the GPU solve's algorithmic bytes / that rate."""
    from oracle import cpu_baseline

    m = p + (p & 1) - 1
    t0 = time.perf_counter()
    _, info = cpu_baseline.pcd_wform(S, lam, 1e-300, 1)
    dt = time.perf_counter() - t0
    b = sweep_bytes(p, 8, 1, info["moved_pairs"], info["moved_diag"])
    par = {"GBps": b / dt / 1e9, "cores": info["threads"], "t_sweep1_s": dt,
           "time_to_tol_s_extrapolated": gpu_bytes / (b / dt),
           "sample": f"sweep 1 ({info['moved_pairs']} pair changes), OpenMP over a colour's pairs"}
    # per-colour cost from the difference of two runs (each also copies S into W)
    t0 = time.perf_counter()
    cpu_baseline.pcd_wform(S, lam, 1e-300, 1, threads=1, colour_limit=2)
    t1 = time.perf_counter()
    cpu_baseline.pcd_wform(S, lam, 1e-300, 1, threads=1, colour_limit=42)
    per = max(time.perf_counter() - t1 - (t1 - t0), 1e-6) / 40
    c = int(max(2, min(m, budget_s / per)))
    t0 = time.perf_counter()
    _, info = cpu_baseline.pcd_wform(S, lam, 1e-300, 1, threads=1, colour_limit=c)
    dt = time.perf_counter() - t0
    b = float(8) * (1.5 * p * c + 6.0 * p * info["moved_pairs"])
    ser = {"GBps": b / dt / 1e9, "cores": 1, "time_to_tol_s_extrapolated": gpu_bytes / (b / dt),
           "sample": f"first {c} of {m} colour steps of sweep 1 ({dt:.1f} s)"}
    return {"kind": "Algorithm 1 with a maintained W = Omega S, FP64 (oracle/cpu_pcd.c)",
            "parallel": par, "serial": ser, "host_cpu": _cpu_model(),
            "host_threads": os.cpu_count()}


def measured_traffic(p: int, n: int, lam: float, dtype: str, kernel: str):
    """HBM bytes per sweep-kernel launch from the committed rocprofv3 counter
    runs, or None when they were taken on another workload, kernel or kernel
    source."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "pcd_sweep_traffic.json")))
        src = b"".join(open(os.path.join(ROOT, "paper_2106_09382_amd", "csrc", f), "rb").read()
                       for f in ("sweep_solve.hpp", "sweep.hip"))
    except (OSError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest()[:16] != rec.get("sweep_src_sha256_16"):
        return None
    if rec.get("kernel") != kernel:
        return None
    if (p, n, lam, dtype) != (5000, 2000, 0.1, "f64"):
        return None
    return float(rec["bytes_per_launch"])


def batched_measurement(plain_all: bool) -> dict:
    """Config-4 batch in one launch against the plain single-solve loop."""
    import warnings

    import numpy as np
    import torch

    from paper_2106_09382_amd import _lib, datagen

    t0 = time.perf_counter()
    probs = datagen.batched_problems(0)
    lams = [float(x) for x in datagen.lambda_path()]
    log(f"bench: batched workload ready in {time.perf_counter() - t0:.1f} s")
    Xs = [torch.tensor(q["y"], dtype=torch.float32, device="cuda") for q in probs]
    ps = np.array([q["p"] for q in probs])
    tol, maxit = 1e-5, 500
    B, L = len(probs), len(lams)

    from paper_2106_09382_amd import autotune

    last = {}

    def run_batch(pw=None, pc=None, cpl=0, threads=0):
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            outs, infos, code = _lib.fit_batched(Xs, lams, tol, maxit, kind="Y", check=False,
                                                 problem_workgroups=pw, problem_col_slices=pc,
                                                 cols_per_lane=cpl, block_threads=threads)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        if code < 0:
            raise RuntimeError(f"batched solve failed with status {code}")
        last[(None if pw is None else tuple(pw), None if pc is None else tuple(pc), cpl,
              infos[0][0]["block_threads"])] = (infos, code)
        return infos, wall

    total = torch.cuda.get_device_properties(0).multi_processor_count
    # FP32 batch: the library's default workgroups are the wide ones, 1024
    # threads with one row each
    best = autotune.search(run_batch, [int(x) for x in ps], total, threads=1024, log=log)
    wall_default = best["trials"][0]["wall_s"]
    tuned = best["problem_workgroups"]
    infos, code = last[(tuple(tuned), tuple(best["problem_col_slices"]), best["cols_per_lane"],
                        best["block_threads"])]
    wall = best["wall_s"]
    sweeps = sum(i["sweeps"] for row in infos for i in row)
    moved = np.array([sum(i["moved_pairs"] for i in row) for row in infos], dtype=float)
    mdiag = np.array([sum(i["moved_diag"] for i in row) for row in infos], dtype=float)
    sw = np.array([sum(i["sweeps"] for i in row) for row in infos], dtype=float)
    m = ps + (ps & 1) - 1
    byt = float((4.0 * (1.5 * ps * m * sw + 6.0 * ps * moved + 3.0 * ps * mdiag)).sum())
    log(f"bench: batched {B} x {L} solves in {wall:.2f} s (code {code})")

    order = np.argsort(ps)
    subset = list(range(B)) if plain_all else [int(b) for b in order[::4]]
    times = {}
    for b in subset:
        om = None
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            for lam in lams:
                om, _ = _lib.fit(Xs[b], lam, tol, maxit, kind="Y", omega0=om, check=False)
        torch.cuda.synchronize()
        times[b] = time.perf_counter() - t1
    if plain_all:
        plain_total = sum(times.values())
        how = "measured on all 64 problems"
    else:
        xp = np.array([ps[b] for b in subset], dtype=float)
        fp = np.array([times[b] for b in subset])
        plain_total = float(np.interp(ps.astype(float), xp, fp).sum())
        how = (f"measured on {len(subset)} problems (every 4th by p, "
               f"{sum(times.values()):.1f} s), linearly interpolated in p over all 64")
    log(f"bench: plain loop {plain_total:.1f} s ({how})")
    return {
        "workload": ("64 ER problems p~U[200,3000] (seed 4000), n=p/2, 16-value lambda path "
                     "0.5->0.05 with warm starts, FP32, tol 1e-5, maxit 500 per lambda, from Y"),
        "solves": B * L,
        "wall_s": wall,
        "wall_s_builtin_plan": wall_default,
        "plan": ("autotuned: workgroups dealt by measured per-problem work, each problem's "
                 "split into row groups x column slices, the columns per lane in row "
                 "rewrites and the workgroup width picked from measured runs"),
        "tuned_plan": {"problem_workgroups": [int(x) for x in tuned],
                       "problem_col_slices": [int(x) for x in best["problem_col_slices"]],
                       "cols_per_lane": int(best["cols_per_lane"]),
                       "block_threads": int(best["block_threads"]),
                       "work_model_exponent": best["work_model_exponent"]},
        "autotune_trials": [{"tag": t["tag"], "wall_s": t["wall_s"]} for t in best["trials"]],
        "solves_per_s": B * L / wall,
        "plain_loop_s": plain_total,
        "plain_solves_per_s": B * L / plain_total,
        "speedup_vs_plain": plain_total / wall,
        "plain_loop_how": how,
        "status": code,
        "setup_ms": float(infos[0][0]["gram_ms"]),
        "launch_ms": float(infos[0][0]["elapsed_ms"]),
        "sweeps_total": int(sweeps),
        "algorithmic_GBs": byt / wall / 1e9,
        "workgroups": int(sum(row[0]["row_groups"] * row[0]["col_slices"] for row in infos)),
    }


def floor_measurement(Y, shape: dict, bytes_per_sweep: float, t_sweep_ms: float, m: int) -> dict:
    """Bandwidth and synchronisation floors of one sweep (see the module doc)."""
    import torch

    from paper_2106_09382_amd import _lib

    ts = []
    for _ in range(3):
        _, info = _lib.fit(Y, 1000.0, 1e-6, 10, kind="Y", check=False, **shape)
        torch.cuda.synchronize()
        ts.append(info["sweep_ms"] * 1e3 / (max(info["sweeps"], 1) * m))
    t_step = float(min(ts))
    t_bw = bytes_per_sweep / (HBM_PEAK_GBS * 1e9) * 1e3
    t_sync = t_step * m / 1e3
    t_floor = max(t_bw, t_sync)
    return {
        "us_per_step_no_moves": t_step,
        "sweeps_no_moves": info["sweeps"],
        "t_bandwidth_ms": t_bw,
        "t_sync_ms": t_sync,
        "t_floor_ms": t_floor,
        "t_sweep_ms": t_sweep_ms,
        "frac": t_floor / t_sweep_ms,
        "binds": "sync" if t_sync >= t_bw else "bandwidth",
    }


def active_measurement(Y, tol: float, shape: dict) -> dict:
    """Plain Algorithm 1 against the active-set sweeps, time to tolerance."""
    import torch

    from paper_2106_09382_amd import _lib

    out = {}
    for lam in (0.1, 0.2):
        row = {}
        for mode in ("plain", "active"):
            best = None
            for _ in range(2):
                _, info = _lib.fit(Y, lam, tol, 500, kind="Y", check=False,
                                   active_set=(mode == "active"), **shape)
                torch.cuda.synchronize()
                if best is None or info["elapsed_ms"] < best["elapsed_ms"]:
                    best = info
            row[mode] = {"ms": best["elapsed_ms"], "full_sweeps": best["sweeps"],
                         "active_sweeps": best["active_sweeps"], "nnz_upper": best["nnz_upper"],
                         "code": best["code"]}
        row["speedup"] = row["plain"]["ms"] / row["active"]["ms"]
        out[f"lambda_{lam}"] = row
    return out


def chain_measurement(p: int, n: int, tol: float, shape: dict) -> dict:
    """The chain-graph workload at the same size (omega_ii = 1, omega_{i,i+1} =
    0.4), FP64 from Y: time to tolerance and algorithmic bandwidth."""
    import torch

    from paper_2106_09382_amd import _lib, datagen

    pr = datagen.problem(3, graph="chain", p=p, n=n)
    Y = torch.tensor(pr["y"], device="cuda")
    m = p + (p & 1) - 1
    out = {"workload": f"chain Omega0, p={p}, n={n}, tol={tol}, f64, from Y"}
    for lam in (0.1, 0.2):
        best = None
        for _ in range(2):
            _, info = _lib.fit(Y, lam, tol, 500, kind="Y", check=False, **shape)
            torch.cuda.synchronize()
            if best is None or info["sweep_ms"] < best["sweep_ms"]:
                best = info
        b = sweep_bytes(p, 8, best["sweeps"], best["moved_pairs"], best["moved_diag"])
        gbs = b / (best["sweep_ms"] * 1e-3) / 1e9
        out[f"lambda_{lam}"] = {"ms": best["elapsed_ms"], "sweep_ms": best["sweep_ms"],
                                "sweeps": best["sweeps"], "code": best["code"],
                                "nnz_upper": best["nnz_upper"], "algorithmic_GBps": gbs,
                                "frac_of_8TBps": gbs / 8000.0,
                                "us_per_colour_step": best["sweep_ms"] * 1e3 / (best["sweeps"] * m)}
    return out


def fp32_measurement(Y, lam: float, tol: float, shape: dict) -> dict:
    """The benchmark solve in FP32 and a cache-resident copy bandwidth."""
    import numpy as np
    import torch

    from paper_2106_09382_amd import _lib

    Y32 = Y.float()
    p = Y.shape[1]
    m = p + (p & 1) - 1
    infos = []
    for _ in range(3):
        _, info = _lib.fit(Y32, lam, tol, 500, kind="Y", check=False, **shape)
        torch.cuda.synchronize()
        infos.append(info)
    last = infos[-1]
    byt = sweep_bytes(p, 4, last["sweeps"], last["moved_pairs"], last["moved_diag"])
    t = float(np.mean([i["sweep_ms"] for i in infos[1:]]))
    # cache-resident copy: 64 MiB in, 64 MiB out, repeated
    a = torch.empty(16 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    reps = 50
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * a.numel() * 4 * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    return {
        "sweep_kernel_ms": t,
        "sweeps": last["sweeps"],
        "code": last["code"],
        "tol_eff": last["tol_eff"],
        "algorithmic_GBs": byt / (t / 1e3) / 1e9,
        "us_per_colour_step": t * 1e3 / max(last["sweeps"] * m, 1),
        "cache_copy_GBs": copy_gbs,
        "frac_of_cache_copy": byt / (t / 1e3) / 1e9 / copy_gbs,
    }


def cache_fp64_measurement(tol: float, shape: dict) -> dict:
    """FP64 in the Infinity-Cache-resident regime: ER p = 3500, n = 1400
    (S and W together 196 MB, under the 256 MB cache), lambda = 0.1."""
    import numpy as np
    import torch

    from paper_2106_09382_amd import _lib, datagen

    p, n = 3500, 1400
    pr = datagen.problem(3, p=p, n=n)
    Y = torch.tensor(pr["y"], device="cuda")
    m = p + (p & 1) - 1
    infos = []
    for _ in range(3):
        _, info = _lib.fit(Y, 0.1, tol, 500, kind="Y", check=False, **shape)
        torch.cuda.synchronize()
        infos.append(info)
    last = infos[-1]
    byt = sweep_bytes(p, 8, last["sweeps"], last["moved_pairs"], last["moved_diag"])
    t = float(np.mean([i["sweep_ms"] for i in infos[1:]]))
    gbs = byt / (t / 1e3) / 1e9
    return {"workload": f"ER p={p}, n={n}, lambda=0.1, tol={tol}, f64, from Y (S + W = "
                        f"{2 * 8 * p * p / 1e6:.0f} MB)",
            "sweep_kernel_ms": t, "sweeps": last["sweeps"], "code": last["code"],
            "algorithmic_GBs": gbs, "frac_of_8TBps": gbs / 8000.0,
            "us_per_colour_step": t * 1e3 / max(last["sweeps"] * m, 1)}


def lds_measurement(shape: dict) -> dict:
    """ER p = 1001 (odd: 1001 colours), n = 500, lambda = 0.2, tol 1e-7: W in
    LDS, the sync-bound regime; FP64 and FP32."""
    import numpy as np
    import torch

    from paper_2106_09382_amd import _lib, datagen

    pr = datagen.problem(2)
    p = pr["p"]
    m = p + (p & 1) - 1
    out = {"workload": f"ER p={p}, n={pr['n']}, lambda={pr['lam']}, tol={pr['tol']}, from Y"}
    for dt, name in ((torch.float64, "f64"), (torch.float32, "f32")):
        Y = torch.tensor(pr["y"], dtype=dt, device="cuda")
        infos = []
        for _ in range(4):
            _, info = _lib.fit(Y, pr["lam"], pr["tol"], pr["maxit"], kind="Y", check=False, **shape)
            torch.cuda.synchronize()
            infos.append(info)
        t = float(np.mean([i["sweep_ms"] for i in infos[1:]]))
        last = infos[-1]
        out[name] = {"sweep_kernel_ms": t, "sweeps": last["sweeps"], "code": last["code"],
                     "w_in_lds": last["w_in_lds"], "workgroups": last["row_groups"] * last["col_slices"],
                     "us_per_colour_step": t * 1e3 / max(last["sweeps"] * m, 1)}
    return out


def joint_measurement() -> dict:
    """Joint estimation of two populations (p = 5000, n = 2000 each, ER graphs
    differing in 10 % of their edges) against estimating them separately."""
    import torch

    from paper_2106_09382_amd import _lib, datagen

    t0 = time.perf_counter()
    jp = datagen.joint_problem(0)
    log(f"bench: joint workload ready in {time.perf_counter() - t0:.1f} s")
    p = jp["p"]
    Y1 = torch.tensor(jp["y"][0], device="cuda")
    Y2 = torch.tensor(jp["y"][1], device="cuda")
    lam1, lam2, tol = 0.1, 0.05, 1e-6

    def best_joint(l2):
        best = None
        for _ in range(2):
            _, _, info = _lib.fit_joint(Y1, Y2, lam1, l2, tol, 500, kind="Y", check=False)
            torch.cuda.synchronize()
            if best is None or info["elapsed_ms"] < best["elapsed_ms"]:
                best = info
        return best

    def summary(info):
        b = sweep_bytes(p, 8, 2 * info["sweeps"], info["moved_pairs"], info["moved_diag"])
        gbs = b / (info["sweep_ms"] * 1e-3) / 1e9
        return {"ms": info["elapsed_ms"], "sweep_ms": info["sweep_ms"], "sweeps": info["sweeps"],
                "code": info["code"], "nnz_upper": list(info["nnz_upper"]),
                "differ_upper": info["differ_upper"], "algorithmic_GBps": gbs,
                "frac_of_8TBps": gbs / 8000.0,
                "workgroups": 2 * info["row_groups"] * info["col_slices"]}

    joint = summary(best_joint(lam2))
    log(f"bench: joint solve {joint['ms']:.1f} ms, {joint['sweeps']} sweeps, "
        f"{joint['differ_upper']} pairs differ")
    decoupled = summary(best_joint(0.0))
    sep = []
    for Y in (Y1, Y2):
        best = None
        for _ in range(2):
            _, info = _lib.fit(Y, lam1, tol, 500, kind="Y", check=False)
            torch.cuda.synchronize()
            if best is None or info["elapsed_ms"] < best["elapsed_ms"]:
                best = info
        sep.append(best)
    return {
        "workload": (f"two populations, ER Omega0 differing in 10 % of edges, p={p}, n=2000 "
                     f"each, lambda1={lam1}, lambda2={lam2}, tol={tol}, f64, from Y"),
        "joint": joint,
        "lambda2_0_one_launch": decoupled,
        "separate_solves": {"ms": sum(i["elapsed_ms"] for i in sep),
                            "sweeps": [i["sweeps"] for i in sep],
                            "nnz_upper": [i["nnz_upper"] for i in sep]},
    }


def backward_measurement() -> dict:
    """Config-5 implicit gradient against its forward solve."""
    import numpy as np
    import torch

    from paper_2106_09382_amd import _lib, datagen

    pr = datagen.problem(5)
    S = _lib.gram(torch.tensor(pr["y"], device="cuda"))
    O0 = torch.tensor(pr["omega0"], device="cuda")
    tol, maxit = pr["tol"], 5000
    fw, bw = [], []
    for rep in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        om, fi = _lib.fit(S, pr["lam"], tol, maxit)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gS, gl, bi = _lib.backward(S, om, 2.0 * (om - O0), tol, maxit)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if rep:
            fw.append(t1 - t0)
            bw.append(t2 - t1)
    return {
        "workload": "p=2000 n=1000 chain Omega_0, lambda=0.15, L=|Omega-hat - Omega_0|_F^2, FP64, tol 1e-8",
        "forward_ms": 1e3 * float(np.mean(fw)),
        "backward_ms": 1e3 * float(np.mean(bw)),
        "backward_over_forward": float(np.mean(bw) / np.mean(fw)),
        "forward_sweeps": fi["sweeps"],
        "backward_sweeps": bi["sweeps"],
        "nnz_upper": fi["nnz_upper"],
        "grad_lambda": gl,
    }


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--graph", choices=["er", "chain"], default="er")
    ap.add_argument("--lam", type=float, default=0.1)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--p", type=int, default=5000)
    ap.add_argument("--n", type=int, default=2000)
    ap.add_argument("--row-groups", type=int, default=0)
    ap.add_argument("--col-slices", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched measurement")
    ap.add_argument("--no-backward", action="store_true", help="skip the backward measurement")
    ap.add_argument("--no-joint", action="store_true", help="skip the joint measurement")
    ap.add_argument("--plain-sample", action="store_true",
                    help="time the plain single-solve loop on every 4th batched problem only and "
                         "interpolate (default: all 64, about two minutes)")
    ap.add_argument("--dump-y", metavar="PATH",
                    help="write the workload's Y (raw float64, n x p) to PATH and exit; "
                         "input for the native driver concord_bench")
    ap.add_argument("--only", choices=["batched", "backward", "joint", "active", "chain"],
                    help="run one side measurement alone and print its JSON (for profiling)")
    ap.add_argument("--dump-config", type=int, default=3,
                    help="workload whose Y --dump-y writes (3: the benchmark solve; 5: the "
                         "gradient workload, p=2000 n=1000 chain)")
    ap.add_argument("--dump-batched", metavar="DIR",
                    help="write the batched workload (DIR/y_<b>.bin raw float64 n_b x p_b, "
                         "DIR/problems.txt 'p n' per line, DIR/lambdas.txt) and exit")
    ap.add_argument("--dump-joint-y", metavar="PREFIX",
                    help="write the joint workload's Y_1 and Y_2 (raw float64, 2000 x 5000) to "
                         "PREFIX1.bin and PREFIX2.bin and exit")
    args = ap.parse_args()

    if args.dump_batched:
        from paper_2106_09382_amd import datagen
        os.makedirs(args.dump_batched, exist_ok=True)
        probs = datagen.batched_problems(0)
        with open(os.path.join(args.dump_batched, "problems.txt"), "w") as fh:
            for b, q in enumerate(probs):
                q["y"].astype("<f8").tofile(os.path.join(args.dump_batched, f"y_{b}.bin"))
                fh.write(f"{q['p']} {q['n']}\n")
        with open(os.path.join(args.dump_batched, "lambdas.txt"), "w") as fh:
            fh.write("\n".join(repr(float(x)) for x in datagen.lambda_path()) + "\n")
        log(f"bench: wrote {len(probs)} batched problems to {args.dump_batched}")
        return 0

    if args.dump_joint_y:
        from paper_2106_09382_amd import datagen
        jp = datagen.joint_problem(0)
        for m in (0, 1):
            jp["y"][m].astype("<f8").tofile(f"{args.dump_joint_y}{m + 1}.bin")
        log(f"bench: wrote Y_1, Y_2 ({jp['n']} x {jp['p']}, seed {jp['seed']}) to "
            f"{args.dump_joint_y}{{1,2}}.bin")
        return 0

    if args.dump_y:
        from paper_2106_09382_amd import datagen
        if args.dump_config == 5:
            pr = datagen.problem(5)
        else:
            pr = datagen.problem(3, graph=args.graph, p=args.p, n=args.n)
        pr["y"].astype("<f8").tofile(args.dump_y)
        log(f"bench: wrote Y ({pr['n']} x {pr['p']}, seed {pr['seed']}) to {args.dump_y}")
        return 0

    if args.only:
        import torch
        if not torch.cuda.is_available():
            log("bench.py: no GPU visible")
            return 1
        from paper_2106_09382_amd import _lib
        _lib.load()
        if args.only == "batched":
            r = batched_measurement(not args.plain_sample)
        elif args.only == "backward":
            r = backward_measurement()
        elif args.only == "joint":
            r = joint_measurement()
        elif args.only == "chain":
            r = chain_measurement(args.p, args.n, args.tol, {})
        else:
            from paper_2106_09382_amd import datagen
            pr = datagen.problem(3, graph=args.graph, p=args.p, n=args.n)
            r = active_measurement(torch.tensor(pr["y"], device="cuda"), args.tol, {})
        print(json.dumps({"only": args.only, args.only: r}), flush=True)
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        log("bench.py: this solver runs one problem per GPU and is measured on one GPU only; "
            "run it with --gpus 1 (independent problems shard across GPUs with no exchange).")
        return 2

    import numpy as np
    import torch

    from paper_2106_09382_amd import _lib, datagen

    _lib.load()
    dt = torch.float64 if args.dtype == "f64" else torch.float32
    elem = 8 if args.dtype == "f64" else 4
    log(f"bench: drawing workload p={args.p} n={args.n} graph={args.graph} (seed 3000)")
    t0 = time.perf_counter()
    pr = datagen.problem(3, graph=args.graph, p=args.p, n=args.n)
    log(f"bench: workload ready in {time.perf_counter() - t0:.1f} s")
    y = pr["y"]
    Y = torch.tensor(y, dtype=dt, device="cuda")
    shape = dict(row_groups=args.row_groups, col_slices=args.col_slices,
                 block_threads=args.threads)
    out = torch.empty((args.p, args.p), dtype=dt, device="cuda")
    maxit = 500

    def solve():
        _, info = _lib.fit(Y, args.lam, args.tol, maxit, kind="Y", out=out, check=False, **shape)
        if info["code"] not in (0, 1):
            raise RuntimeError(f"solve failed: {info}")
        return info

    for w in range(args.warmup):
        info = solve()
        log(f"bench: warmup {w + 1}/{args.warmup}: sweeps={info['sweeps']} "
            f"sweep_ms={info['sweep_ms']:.1f} total_ms={info['elapsed_ms']:.1f}")
    torch.cuda.synchronize()
    infos = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        infos.append(solve())
        log(f"bench: step {k + 1}/{args.steps}: sweeps={infos[-1]['sweeps']} "
            f"sweep_ms={infos[-1]['sweep_ms']:.1f}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    bytes_total = sum(sweep_bytes(args.p, elem, i["sweeps"], i["moved_pairs"], i["moved_diag"])
                      for i in infos)
    sweep_ms = [i["sweep_ms"] for i in infos]
    bytes_launch = bytes_total / len(infos)
    achieved = bytes_launch / (np.mean(sweep_ms) / 1e3) / 1e9
    sweeps = infos[-1]["sweeps"]
    m = args.p + (args.p & 1) - 1
    last = infos[-1]
    # measured HBM bytes of one sweep-kernel launch (rocprofv3 FETCH_SIZE +
    # WRITE_SIZE on this source), beside the algorithmic account above
    # workgroups of more than 512 threads run the wide form of the sweep kernel
    kernel = "pcd_sweep_wide_kernel" if last["block_threads"] > 512 else "pcd_sweep_kernel"
    traffic = measured_traffic(args.p, args.n, args.lam, args.dtype, kernel)
    res = {
        "metric": "sweep GB/s (algorithmic) of a CONCORD-PCD solve to tolerance at p=5000, n=2000",
        "value": bytes_total / wall / 1e9,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": (f"CONCORD-PCD solve from Y, {args.graph.upper()} Omega0, p={args.p}, "
                         f"n={args.n}, lambda={args.lam}, tol={args.tol}"),
            "p": args.p, "n": args.n, "graph": args.graph, "lambda": args.lam, "tol": args.tol,
            "seed": pr["seed"], "maxit": maxit,
            "launch": {"row_groups": last["row_groups"], "col_slices": last["col_slices"],
                       "w_in_lds": last["w_in_lds"], "block_threads": last["block_threads"]},
        },
        "time_to_tol_ms": wall / args.steps * 1e3,
        "sweeps": sweeps,
        "converged": last["code"] == 0,
        "nnz_upper": last["nnz_upper"],
        "sweep_kernel_ms": float(np.mean(sweep_ms)),
        "gram_ms": float(np.mean([i["gram_ms"] for i in infos])),
        "t_sweep_ms": float(np.mean(sweep_ms)) / max(sweeps, 1),
        "sweeps_per_s": max(sweeps, 1) / (float(np.mean(sweep_ms)) / 1e3),
        "us_per_colour_step": float(np.mean(sweep_ms)) * 1e3 / max(sweeps * m, 1),
        "moved_pairs_per_sweep": last["moved_pairs"] / max(sweeps, 1),
        "bytes_per_sweep": bytes_launch / max(sweeps, 1),
        "roofline": {
            "kernel": kernel,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "hbm_GBs_measured": (traffic / (np.mean(sweep_ms) / 1e3) / 1e9) if traffic else None,
            "hbm_frac_measured": ((traffic / (np.mean(sweep_ms) / 1e3) / 1e9) / HBM_PEAK_GBS
                                  if traffic else None),
        },
    }
    res["paper_context"] = {
        "note": ("arXiv 2106.09382 Table 2, AR(2) network, n=2000, p=5000, lambda=0.1: the "
                 "paper's own data, tolerance 1e-5 and hardware (GTX 1080 Ti FP32 for PCD-GPU, "
                 "a Xeon W-2175 in FP64 for the CPU columns); context, not a like-for-like "
                 "comparison with this workload"),
        "pcd_gpu_s": 386.23, "pcd_cpu_s": 3929.09, "cd_naive_s": 3440.95, "cd_blas_s": 1389.95,
        "iterations_pcd": 26.0,
    }
    if not args.no_cpu_baseline:
        log(f"bench: timing the CPU oracle on a ~{args.cpu_seconds:.0f} s sample")
        import oracle
        S_cpu = oracle.gram(y)
        res["cpu_baseline"] = cpu_oracle_baseline(S_cpu, args.p, args.lam, elem, sweeps,
                                                  bytes_launch / max(sweeps, 1), args.cpu_seconds)
        if args.dtype == "f64":
            log("bench: timing the CPU baseline with a maintained W")
            res["cpu_wform"] = cpu_wform_baseline(S_cpu, args.p, args.lam, bytes_launch,
                                                  args.cpu_seconds / 2)
    if args.p == 5000 and args.dtype == "f64":
        res["floor"] = floor_measurement(Y, shape, bytes_launch / max(sweeps, 1),
                                         float(np.mean(sweep_ms)) / max(sweeps, 1), m)
        res["fp32"] = fp32_measurement(Y, args.lam, args.tol, shape)
        res["cache_fp64"] = cache_fp64_measurement(args.tol, shape)
        res["lds_p1001"] = lds_measurement(shape)
        res["active_set"] = active_measurement(Y, args.tol, shape)
        if args.graph == "er":
            res["chain"] = chain_measurement(args.p, args.n, args.tol, shape)
    if not args.no_batched:
        res["batched"] = batched_measurement(not args.plain_sample)
    if not args.no_backward:
        res["backward"] = backward_measurement()
    if not args.no_joint:
        res["joint"] = joint_measurement()
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
