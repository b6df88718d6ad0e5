"""Writes the converged reference solutions of the p = 5000 workload.

The workload: Erdos-Renyi Omega0, p = 5000, n = 2000, seed 3000 (workload 3 of
``paper_2106_09382_amd.datagen``), S = Y^T Y / n by ``oracle.gram``.  For each
lambda this runs the oracle's Algorithm 1 (serial direct sums, FP64) from the
identity with tol 1e-6, one sweep per call so that every iterate is seen (the
oracle's whole state between sweeps is Omega, so a sweep started from the
previous Omega is the same sweep), and stores:

* the sweep count, the delta of every sweep and the stopping sweep;
* the converged Omega: its nonzeros above the diagonal (linear indices,
  delta-coded, and values) and its diagonal;
* the pairs whose eq. (3) numerator lies within 1e-9 (S_ii + S_jj) of lambda
  (the support decisions that rounding may flip);
* for FP32 comparisons: the iterate at the first sweep whose delta is below
  max(tol, 16 eps_f32 max_i omega_ii) of that sweep (the stopping rule an FP32
  solve applies), with its own borderline pairs at 1e-4;
* the SHA-256 of the bytes of S, so a reader can tell whether their S is
  bit-identical to the one used here.

It calls only ``oracle`` and ``datagen``.  About three minutes of CPU per sweep
on an 8-core Xeon, so an hour per lambda; both lambdas can run at once:

    python tests/golden/make_fullsize.py 0.1
    python tests/golden/make_fullsize.py 0.2

Output: tests/golden/fullsize_er5000_lam<lambda>.npz
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2106_09382_amd import datagen  # noqa: E402

TOL = 1e-6
MAXIT = 500
EPS32 = 2.0 ** -23


def _upper(om):
    p = om.shape[0]
    iu = np.triu_indices(p, 1)
    v = om[iu]
    nz = np.flatnonzero(v != 0)
    lin = (iu[0][nz].astype(np.int64) * p + iu[1][nz]).astype(np.int64)
    return lin, v[nz]


def _delta_code(lin):
    d = np.diff(lin, prepend=0)
    return d.astype(np.uint32)


def path_for(lam: float) -> str:
    return os.path.join(HERE, f"fullsize_er5000_lam{lam:g}.npz")


def main(lam: float) -> None:
    t0 = time.time()
    pr = datagen.problem(3)
    S = oracle.gram(pr["y"])
    p = S.shape[0]
    sha = hashlib.sha256(np.ascontiguousarray(S).tobytes()).hexdigest()
    print(f"make_fullsize: lam={lam} p={p} n={pr['n']} S sha256={sha[:16]} "
          f"({time.time() - t0:.1f} s)", flush=True)
    om = None
    trace = []
    t32 = 0
    om32 = None
    tol32 = 0.0
    for t in range(1, MAXIT + 1):
        ts = time.time()
        om, info, tr = oracle.pcd(S, lam, TOL, 1, omega0=om)
        d = float(tr[0])
        trace.append(d)
        gmax = float(np.diag(om).max())
        tol_eff32 = max(TOL, 16 * EPS32 * gmax)
        if t32 == 0 and d < tol_eff32:
            t32, om32, tol32 = t, om.copy(), tol_eff32
        print(f"make_fullsize: lam={lam} sweep {t} delta={d:.6e} nnz={info['nnz_upper']} "
              f"({time.time() - ts:.0f} s)", flush=True)
        if d < TOL:
            break
    sweeps = len(trace)
    converged = trace[-1] < TOL
    lin, val = _upper(om)
    lin32, val32 = _upper(om32)
    bl = oracle.borderline_pairs(S, om, lam, 1e-9)
    bl32 = oracle.borderline_pairs(S, om32, lam, 1e-4)
    np.savez_compressed(
        path_for(lam),
        p=p, n=pr["n"], seed=pr["seed"], lam=lam, tol=TOL, maxit=MAXIT,
        sweeps=sweeps, converged=converged, delta_trace=np.array(trace),
        s_sha256=np.array(sha),
        upper_dlin=_delta_code(lin), upper_val=val, diag=np.diag(om).copy(),
        borderline=bl.astype(np.int32),
        f32_sweeps=t32, f32_tol_eff=tol32,
        f32_upper_dlin=_delta_code(lin32), f32_upper_val=val32.astype(np.float32),
        f32_diag=np.diag(om32).copy(), f32_borderline=bl32.astype(np.int32),
    )
    print(f"make_fullsize: lam={lam} wrote {path_for(lam)}: {sweeps} sweeps, "
          f"{lin.size} nonzeros, {bl.shape[0]} borderline; FP32 rule stops at sweep {t32} "
          f"(tol_eff {tol32:.4e}, {bl32.shape[0]} borderline); {time.time() - t0:.0f} s",
          flush=True)


def load(lam: float) -> dict:
    """Reads a stored reference back: dense upper support, values, diagonals."""
    z = np.load(path_for(lam), allow_pickle=False)
    out = {k: z[k] for k in z.files}
    for pre in ("", "f32_"):
        lin = np.cumsum(out[pre + "upper_dlin"].astype(np.int64))
        out[pre + "upper_lin"] = lin
    return out


if __name__ == "__main__":
    main(float(sys.argv[1]))
