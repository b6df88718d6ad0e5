"""Per-colour-step device timestamps of a solve, summarised.

concord_fit_ex can record, for each of the first timestamp_steps colour
steps, the 100 MHz device clock of every workgroup at the step's start, when
its rows are done (after the step's workgroup barrier) and when its
synchronous row rewrites are done.  `step_times` runs one solve with all
steps recorded and summarises them: the time from one step's start to the
next (per workgroup, then averaged over workgroups), the row phase, the
spread of the workgroups' start times, and the percentiles of the step time.

    python -m paper_2106_09382_amd.steptimes      # the p = 5000 solves of bench.py
"""
from __future__ import annotations

import json

import numpy as np
import torch

from . import _lib

CLOCK_HZ = 100e6  # s_memrealtime


def step_times(X: torch.Tensor, lam: float, tol: float = 1e-6, maxit: int = 500,
               kind: str = "Y", skip_sweeps: int = 4, **opts) -> dict:
    """One solve of X (as for _lib.fit) with every colour step time-stamped.

    The first `skip_sweeps` sweeps (fewer if the solve is shorter) are left
    out of the summary, so that it describes the steady state.  The steps
    that cross a sweep barrier are left out too."""
    _, info = _lib.fit(X, lam, tol, maxit, kind=kind, **opts)
    G = info["row_groups"] * info["col_slices"]
    p = X.shape[1] if kind == "Y" else X.shape[0]
    m = p - 1 if p % 2 == 0 else p
    steps = info["sweeps"] * m
    ts = torch.zeros((G, steps, 3), dtype=torch.int64, device=X.device)
    _, info2 = _lib.fit(X, lam, tol, maxit, kind=kind, timestamps=ts, **opts)
    torch.cuda.synchronize()
    a = ts.cpu().numpy().astype(np.float64) * (1e6 / CLOCK_HZ)  # microseconds
    del ts
    sw = info2["sweeps"]
    first = skip_sweeps if sw > skip_sweeps else (1 if sw > 1 else 0)
    t0 = a[:, :, 0]
    step = np.diff(t0, axis=1)
    row = a[:, :, 1] - a[:, :, 0]
    # the steps of each sweep but its last (whose successor follows the barrier)
    keep = np.zeros(steps - 1, dtype=bool)
    for s in range(first, sw):
        keep[s * m:(s + 1) * m - 1] = True
    per_step = step[:, keep].mean(axis=0)
    spread = (t0.max(axis=0) - t0.min(axis=0))[:-1][keep]
    return {
        "p": int(p), "lambda": float(lam), "dtype": str(X.dtype).replace("torch.", ""),
        "sweeps": int(sw), "sweeps_summarised": int(sw - first),
        "launch": [info["row_groups"], info["col_slices"], info["block_threads"]],
        "sweep_ms": float(info2["sweep_ms"]), "sweep_ms_untimed": float(info["sweep_ms"]),
        "step_us_mean": float(per_step.mean()),
        "step_us_percentiles": {str(q): float(np.percentile(per_step, q))
                                for q in (10, 50, 90, 99, 99.9)},
        "row_phase_us_mean": float(row[:, :-1][:, keep].mean()),
        "start_spread_us_median": float(np.median(spread)),
    }


def main() -> int:
    from . import datagen
    pr = datagen.problem(3)
    Y = torch.from_numpy(pr["y"]).cuda()
    out = []
    for dt, lam in ((torch.float64, 0.1), (torch.float64, 0.2), (torch.float64, 1000.0),
                    (torch.float32, 0.1)):
        r = step_times(Y.to(dt), lam)
        out.append(r)
        print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
