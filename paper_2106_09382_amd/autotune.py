"""Workgroup plans for batched solves from measured work.

A batched launch gives every problem its own group of workgroups; the launch
ends when the slowest problem ends, so a good plan balances the problems'
finishing times.  The built-in plan deals workgroups by a size model.  After
one run, the info records hold each problem's own device time per lambda
(`sweep_ms`) and its workgroup count (`row_groups`): their product estimates
the problem's work, and dealing workgroups in proportion to it balances the
next run of the same (or similar) problems, e.g. the replicates of a
bootstrap or a repeated path.
"""
from __future__ import annotations


def min_workgroups(p: int, threads: int = 512) -> int:
    """Fewest workgroups a problem of size p needs (two rows per thread)."""
    return max(1, -(-p // (2 * threads)))


def plan(ps, work, total: int, threads: int = 512) -> list[int]:
    """Deal `total` workgroups: every problem its minimum, then one at a time
    to the problem with the largest work per workgroup (keeping at least 8
    rows per workgroup)."""
    G = [min_workgroups(p, threads) for p in ps]
    if sum(G) > total:
        raise ValueError("the problems' minimum workgroup counts exceed the launch")
    w = [max(float(x), 1e-12) for x in work]
    for _ in range(total - sum(G)):
        best, bc = -1, -1.0
        for b, p in enumerate(ps):
            if (G[b] + 1) * 8 > p:
                continue
            c = w[b] / G[b]
            if c > bc:
                best, bc = b, c
        if best < 0:
            break
        G[best] += 1
    return G


def plan_from_infos(ps, infos, total: int, threads: int = 512) -> list[int]:
    """Plan from the info records (B x L dicts) of a previous batched run of
    problems with sizes ps: work_b = (device time of problem b) x (its
    workgroups)."""
    work = [sum(i["sweep_ms"] for i in row) * row[0]["row_groups"] for row in infos]
    return plan(ps, work, total, threads)
