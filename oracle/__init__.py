"""CPU oracle for CONCORD-PCD.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path and
imports nothing from it.

The coordinate-descent sweeps live in ``concord_oracle.c`` (plain serial C,
double precision, direct sums exactly as eqs. (2)-(3) of arXiv 2106.09382
write them).  The helpers here are plain NumPy definitions:

* ``gram``: S = Y^T Y / n (the Gram matrix T = X^T X of Algorithm 1's
  initialisation, on the S scale; a library matmul is the whole step).
* ``objective``: the CONCORD objective, eq. (1), divided by n:
  F(Omega) = -sum_i log omega_ii + 1/2 tr(Omega S Omega) + lam sum_{i<j} |omega_ij|.
* ``kkt``: stationarity of F.  With G = Omega S + S Omega, an optimum has
  omega_ii (S Omega)_ii = 1, G_ij + lam sign(omega_ij) = 0 where omega_ij != 0,
  and |G_ij| <= lam where omega_ij = 0.

``oracle.active`` holds the active-set scheme (greedy edge colouring of the
support, sweeps over it, full sweeps to decide convergence).
``oracle.backward`` holds the implicit gradient of the estimate (dL/dS and
dL/dlam from the stationarity system on the active set, by a dense solve).
``oracle.cpu_baseline`` is not part of the oracle: it is the benchmark's
CPU baseline (Algorithm 1 with a maintained W = Omega S, serial or
colour-parallel with OpenMP), pinned against the oracle in the tests.
``oracle.joint`` holds the joint estimation of two precision matrices with a
fused penalty (Section 6): block coordinate descent on Algorithm 1's schedule,
its objective and its optimality conditions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "concord_oracle.c")
_SRC_CPU = os.path.join(_HERE, "cpu_pcd.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile the C oracle and the CPU baseline (OpenMP) with gcc into
    oracle/liboracle.so."""
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-o", tmp, _SRC,
                    _SRC_CPU, "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                                                 os.path.getmtime(_SRC_CPU)):
        build()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_round_robin.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int32)]
    lib.oracle_round_robin.restype = ctypes.c_int
    lib.oracle_pcd.argtypes = [dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                               dp, dp, ctypes.c_longlong, ctypes.c_int, dp, dp]
    lib.oracle_pcd.restype = ctypes.c_int
    lib.oracle_cd.argtypes = [dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                              dp, dp, dp, dp]
    lib.oracle_cd.restype = ctypes.c_int
    ip = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_pcd_colouring.argtypes = [dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, dp, dp, ip, ip, ctypes.c_int, dp, dp]
    lib.oracle_pcd_colouring.restype = ctypes.c_int
    lib.oracle_offdiag_update.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double]
    lib.oracle_offdiag_update.restype = ctypes.c_double
    lib.oracle_diag_update.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int]
    lib.oracle_diag_update.restype = ctypes.c_double
    cd_ = ctypes.c_double
    lib.oracle_joint_pair.argtypes = [cd_, cd_, cd_, cd_, cd_, cd_, dp]
    lib.oracle_joint_pair.restype = None
    lib.oracle_joint_diag.argtypes = [cd_, cd_, cd_, cd_, cd_, dp]
    lib.oracle_joint_diag.restype = None
    lib.oracle_joint_pcd.argtypes = [dp, dp, ctypes.c_int, cd_, cd_, cd_, ctypes.c_int, dp, dp,
                                     dp, dp, dp, dp]
    lib.oracle_joint_pcd.restype = ctypes.c_int
    lib.cpu_pcd_wform.argtypes = [dp, ctypes.c_int, cd_, cd_, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_longlong, dp, dp]
    lib.cpu_pcd_wform.restype = ctypes.c_int
    _lib = lib
    return lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def round_robin(p: int) -> np.ndarray:
    """Literal round-robin table (Section 3.2): int32 array (m, p_even/2, 2).

    Entry [k, q] is the 0-based pair of slot q at step k; for odd p the value
    p stands for the dummy index p+1.
    """
    pe = p + (p & 1)
    m, h = pe - 1, pe // 2
    out = np.zeros((max(m, 0), h, 2), dtype=np.int32)
    rc = _load().oracle_round_robin(p, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc < 0:
        raise OracleError(f"round_robin: invalid p={p}")
    return out


def _info(a):
    return dict(sweeps=int(a[0]), delta=float(a[1]), converged=bool(a[2]),
                nnz_upper=int(a[3]), steps=int(a[4]))


def pcd(S, lam: float, tol: float, maxit: int, omega0=None, colour_limit: int = 0,
        serial: bool = False):
    """CONCORD-PCD, Algorithm 1.  Returns (Omega, info, delta_trace)."""
    S = _f64(S)
    p = S.shape[0]
    om = np.empty((p, p))
    tr = np.zeros(maxit)
    info = np.zeros(5)
    o0 = None if omega0 is None else _f64(omega0)
    rc = _load().oracle_pcd(_dp(S), p, float(lam), float(tol), int(maxit), _dp(o0), _dp(om),
                            int(colour_limit), int(bool(serial)), _dp(tr), _dp(info))
    if rc:
        raise OracleError(f"oracle_pcd returned {rc}")
    inf = _info(info)
    return om, inf, tr[: inf["sweeps"]].copy()


def pcd_colouring(S, lam: float, tol: float, maxit: int, classes, omega0=None):
    """CONCORD-PCD over a given edge colouring (a list of colour classes, each
    a list of 0-based pairs (i, j) forming a matching).  Returns (Omega, info,
    delta_trace)."""
    S = _f64(S)
    p = S.shape[0]
    flat = [x for cls in classes for pr in cls for x in pr]
    starts = [0]
    for cls in classes:
        starts.append(starts[-1] + len(cls))
    pairs = np.ascontiguousarray(np.array(flat if flat else [0], dtype=np.int32))
    cst = np.ascontiguousarray(np.array(starts, dtype=np.int32))
    om = np.empty((p, p))
    tr = np.zeros(maxit)
    info = np.zeros(5)
    o0 = None if omega0 is None else _f64(omega0)
    ip = ctypes.POINTER(ctypes.c_int32)
    rc = _load().oracle_pcd_colouring(_dp(S), p, float(lam), float(tol), int(maxit), _dp(o0),
                                      _dp(om), pairs.ctypes.data_as(ip), cst.ctypes.data_as(ip),
                                      len(classes), _dp(tr), _dp(info))
    if rc:
        raise OracleError(f"oracle_pcd_colouring returned {rc}")
    inf = _info(info)
    return om, inf, tr[: inf["sweeps"]].copy()


def cd(S, lam: float, tol: float, maxit: int, omega0=None):
    """CONCORD-CD (Section 2.1).  Returns (Omega, info, delta_trace)."""
    S = _f64(S)
    p = S.shape[0]
    om = np.empty((p, p))
    tr = np.zeros(maxit)
    info = np.zeros(5)
    o0 = None if omega0 is None else _f64(omega0)
    rc = _load().oracle_cd(_dp(S), p, float(lam), float(tol), int(maxit), _dp(o0), _dp(om),
                           _dp(tr), _dp(info))
    if rc:
        raise OracleError(f"oracle_cd returned {rc}")
    inf = _info(info)
    return om, inf, tr[: inf["sweeps"]].copy()


def offdiag_update(S, omega, i: int, j: int, lam: float) -> float:
    """New value of omega_ij by eq. (3), from the given Omega (direct sums)."""
    S, omega = _f64(S), _f64(omega)
    return _load().oracle_offdiag_update(_dp(S), _dp(omega), S.shape[0], int(i), int(j),
                                         float(lam))


def diag_update(S, omega, i: int) -> float:
    """New value of omega_ii by eq. (2), from the given Omega (direct sums)."""
    S, omega = _f64(S), _f64(omega)
    return _load().oracle_diag_update(_dp(S), _dp(omega), S.shape[0], int(i))


def gram(Y) -> np.ndarray:
    """S = Y^T Y / n in double precision."""
    Y = _f64(Y)
    return (Y.T @ Y) / Y.shape[0]


def objective(S, omega, lam: float) -> float:
    """CONCORD objective (eq. (1) divided by n)."""
    S, om = _f64(S), _f64(omega)
    d = np.diag(om)
    if np.any(d <= 0):
        return float("inf")
    quad = 0.5 * float(np.sum((om @ S) * om.T))
    pen = lam * float(np.abs(np.triu(om, 1)).sum())
    return float(-np.log(d).sum() + quad + pen)


def kkt(S, omega, lam: float) -> dict:
    """Stationarity residuals of F at Omega (all zero at the optimum)."""
    S, om = _f64(S), _f64(omega)
    p = S.shape[0]
    so = S @ om
    G = so + so.T
    iu = np.triu_indices(p, 1)
    g = G[iu]
    w = om[iu]
    nz = w != 0
    res_nz = np.abs(g[nz] + lam * np.sign(w[nz]))
    res_z = np.maximum(np.abs(g[~nz]) - lam, 0.0)
    res_d = np.abs(np.diag(om) * np.diag(so) - 1.0)
    return dict(
        support=float(res_nz.max()) if res_nz.size else 0.0,
        zeros=float(res_z.max()) if res_z.size else 0.0,
        diag=float(res_d.max()) if res_d.size else 0.0,
    )


def lambda_max(S) -> float:
    """Smallest threshold at which diag(1/sqrt(S_ii)) is optimal.

    At Omega = diag(1/sqrt(S_ii)) the diagonal condition holds exactly and
    G_ij = S_ij (1/sqrt(S_ii) + 1/sqrt(S_jj)), so the point is optimal iff
    lam >= max_{i<j} |G_ij|.
    """
    S = _f64(S)
    r = 1.0 / np.sqrt(np.diag(S))
    G = np.abs(S) * (r[:, None] + r[None, :])
    np.fill_diagonal(G, 0.0)
    return float(G.max()) if S.shape[0] > 1 else 0.0


def borderline_pairs(S, omega, lam: float, rel: float) -> np.ndarray:
    """Pairs i<j whose eq. (3) numerator sits within rel*(S_ii+S_jj) of lam.

    At such a pair the support decision is decided by rounding; support
    comparisons leave them out.  Returns an (k, 2) index array.
    """
    S, om = _f64(S), _f64(omega)
    so = S @ om
    d = np.diag(S)
    b = so + so.T - (d[:, None] + d[None, :]) * om
    near = np.abs(np.abs(b) - lam) < rel * (d[:, None] + d[None, :])
    iu = np.triu_indices(S.shape[0], 1)
    sel = near[iu]
    return np.stack([iu[0][sel], iu[1][sel]], axis=1)
