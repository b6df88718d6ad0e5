"""Launch plans for batched solves from measured work.

A batched launch gives every problem its own group of workgroups; the launch
ends when the slowest problem ends, so a good plan balances the problems'
finishing times.  The built-in plan deals workgroups by a size model.  After
one run, the info records hold each problem's own device time per lambda
(`sweep_ms`) and its launch shape (`row_groups` x `col_slices` workgroups):
their product estimates the problem's work, and dealing workgroups in
proportion to it balances the next run of the same (or similar) problems,
e.g. the replicates of a bootstrap or a repeated path.

`search` goes further: besides the workgroup counts it picks, from measured
runs, each problem's split of its workgroups into row groups x column slices
(the tile each workgroup holds: its rows of W over a slice of the columns)
and the batch's columns per lane in row rewrites (how many loads each lane
keeps in flight, i.e. how many waves a row rewrite occupies).
"""
from __future__ import annotations

import math


def max_rows(threads: int) -> int:
    """Rows of W one workgroup holds: two per thread, one per thread in a
    wide workgroup (more than 512 threads)."""
    return threads if threads > 512 else 2 * threads


def min_workgroups(p: int, threads: int = 512, col_slices: int = 1) -> int:
    """Fewest workgroups a problem of size p needs (max_rows(threads) rows in
    each row group), for a given number of column slices."""
    return max(1, -(-p // max_rows(threads))) * col_slices


def plan(ps, work, total: int, threads: int = 512, slices=None) -> list[int]:
    """Deal `total` workgroups: every problem its minimum, then one step at a
    time to the problem with the largest work per workgroup (keeping at least
    8 rows per row group).  With `slices`, problem b's count stays a multiple
    of slices[b] (its workgroups form row groups x slices[b])."""
    cs = [1] * len(ps) if slices is None else [int(c) for c in slices]
    G = [min_workgroups(p, threads, c) for p, c in zip(ps, cs)]
    if sum(G) > total:
        raise ValueError("the problems' minimum workgroup counts exceed the launch")
    w = [max(float(x), 1e-12) for x in work]
    left = total - sum(G)
    while left > 0:
        best, bc = -1, -1.0
        for b, p in enumerate(ps):
            c = cs[b]
            if c > left or (G[b] // c + 1) * 8 > p:
                continue
            v = w[b] / G[b]
            if v > bc:
                best, bc = b, v
        if best < 0:
            break
        G[best] += cs[best]
        left -= cs[best]
    return G


def problem_times(infos) -> list[float]:
    """Each problem's device time over its whole path (ms)."""
    return [sum(i["sweep_ms"] for i in row) for row in infos]


def problem_work(infos) -> list[float]:
    """Work estimate per problem: device time x workgroups it had."""
    return [t * row[0]["row_groups"] * row[0]["col_slices"]
            for t, row in zip(problem_times(infos), infos)]


def plan_from_infos(ps, infos, total: int, threads: int = 512, slices=None) -> list[int]:
    """Plan from the info records (B x L dicts) of a previous batched run of
    problems with sizes ps: work_b = (device time of problem b) x (its
    workgroups)."""
    return plan(ps, problem_work(infos), total, threads, slices)


def _slices_ok(p: int, G: int, c: int, threads: int) -> bool:
    if c < 1 or c > p or G % c:
        return False
    gr = G // c
    return -(-p // gr) <= max_rows(threads) and gr * 8 <= p


def search(run, ps, total: int, threads: int = 512, cpls=(4, 2), slice_options=(2,),
           wide_threads: int | None = None, log=None) -> dict:
    """Measured search for the batch's launch plan.

    run(problem_workgroups, problem_col_slices, cols_per_lane[, threads])
    runs the whole batch once and returns (infos, wall_seconds);
    problem_workgroups None means the built-in plan, and threads (passed
    only for the wide trials) the workgroup width, else `threads`.  The
    search:

    1. runs the built-in plan and deals the workgroups by its measured work;
    2. for each candidate number of column slices, deals the workgroups
       again in multiples of it, runs the problems large enough with that
       split (the heaviest first, while every problem's minimum count still
       fits the launch) and keeps, problem by problem, the split with the
       smaller work
       (device time x workgroups, so that problems whose counts moved are
       compared fairly);
    3. re-deals the workgroups by the work measured at the chosen splits,
       then runs that plan with each candidate columns-per-lane and keeps the
       faster batch;
    4. with `wide_threads`, runs wide workgroups (one row per thread, so that
       more problems rewrite rows in the background) with the best columns
       per lane, dealt by the measured work and then re-dealt by the work
       measured in the wide run.

    Returns {"problem_workgroups", "problem_col_slices", "cols_per_lane",
    "block_threads", "wall_s", "trials"}: the best plan found and a record
    of every run.
    """
    say = log or (lambda *a: None)
    trials = []

    def trial(tag, pw, pc, cpl, th=None):
        infos, wall = run(pw, pc, cpl) if th is None else run(pw, pc, cpl, th)
        trials.append({"tag": tag, "cols_per_lane": cpl, "wall_s": wall,
                       "block_threads": threads if th is None else th,
                       "problem_workgroups": None if pw is None else list(pw),
                       "problem_col_slices": None if pc is None else list(pc)})
        say(f"autotune: {tag}: {wall:.2f} s")
        return infos, wall

    B = len(ps)
    cpl0 = cpls[0]
    infos, wall = trial("built-in plan", None, None, cpl0)
    G = plan_from_infos(ps, infos, total, threads)
    C = [1] * B
    infos, wall = trial("dealt by measured work", G, C, cpl0)
    best = {"problem_workgroups": list(G), "problem_col_slices": list(C), "cols_per_lane": cpl0,
            "block_threads": threads, "wall_s": wall}
    work = problem_work(infos)
    for c in slice_options:
        # problems large enough for c slices of at least 8 rows per row group,
        # the heaviest first, as long as every problem's minimum still fits
        cand = [1] * B
        need = sum(min_workgroups(p, threads) for p in ps)
        for b in sorted(range(B), key=lambda b: -work[b]):
            extra = min_workgroups(ps[b], threads, c) - min_workgroups(ps[b], threads)
            if ps[b] >= 16 * c and need + extra <= total:
                cand[b], need = c, need + extra
        Gc = plan(ps, work, total, threads, cand)
        cand = [x if _slices_ok(p, g, x, threads) else 1 for p, g, x in zip(ps, Gc, cand)]
        if all(x == 1 for x in cand):
            continue
        infos_c, _ = trial(f"{c} column slices where the counts allow", Gc, cand, cpl0)
        work_c = problem_work(infos_c)
        for b in range(B):
            if cand[b] != 1 and work_c[b] < work[b]:
                C[b], work[b] = cand[b], work_c[b]
    # re-deal by the work at the chosen splits; a count must stay a multiple
    # of its problem's slices and keep their shape valid
    G2 = plan(ps, work, total, threads, C)
    C2 = [c if _slices_ok(p, g, c, threads) else 1 for p, g, c in zip(ps, G2, C)]
    for cpl in cpls:
        infos_f, wall_f = trial(f"re-dealt at the chosen splits, {cpl} columns per lane",
                                G2, C2, cpl)
        if wall_f < best["wall_s"]:
            best = {"problem_workgroups": list(G2), "problem_col_slices": list(C2),
                    "cols_per_lane": cpl, "block_threads": threads, "wall_s": wall_f}
    if wide_threads and sum(min_workgroups(p, wide_threads) for p in ps) <= total:
        cpl = best["cols_per_lane"]
        C1 = [1] * B
        Gw = plan(ps, work, total, wide_threads)
        infos_w, wall_w = trial(f"{wide_threads}-thread workgroups, dealt by measured work", Gw,
                                C1, cpl, wide_threads)
        cands = [(wall_w, Gw)]
        Gw2 = plan(ps, problem_work(infos_w), total, wide_threads)
        if Gw2 != Gw:
            _, wall_w2 = trial(f"{wide_threads}-thread workgroups, re-dealt by their own work",
                               Gw2, C1, cpl, wide_threads)
            cands.append((wall_w2, Gw2))
        for wall_c, Gc_ in cands:
            if wall_c < best["wall_s"]:
                best = {"problem_workgroups": list(Gc_), "problem_col_slices": list(C1),
                        "cols_per_lane": cpl, "block_threads": wide_threads, "wall_s": wall_c}
    best["trials"] = trials
    best["slices_used"] = sorted({int(c) for c in best["problem_col_slices"]})
    best["work_model_exponent"] = _fit_exponent(ps, problem_work(infos))
    return best


def _fit_exponent(ps, work) -> float | None:
    """Least-squares slope of log(work) against log(p): how the measured
    work grows with problem size (the built-in plan assumes 1.55)."""
    pts = [(math.log(p), math.log(w)) for p, w in zip(ps, work) if w > 0]
    if len(pts) < 2:
        return None
    mx = sum(x for x, _ in pts) / len(pts)
    my = sum(y for _, y in pts) / len(pts)
    sxx = sum((x - mx) ** 2 for x, _ in pts)
    if sxx == 0:
        return None
    return sum((x - mx) * (y - my) for x, y in pts) / sxx
