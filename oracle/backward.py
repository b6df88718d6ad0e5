"""Implicit gradient of the CONCORD estimate.  TEST INFRASTRUCTURE ONLY.

The estimate Omega-hat(S, lam) minimises F of eq. (1) (S scale, as in the
rest of the oracle).  On its active set A = {i < j : omega_ij != 0} plus the
diagonal it satisfies the stationarity conditions, written here with
W = Omega S (so that (S Omega)_ij = W_ji):

    R_ii = W_ii - 1 / omega_ii                          = 0   (every i)
    R_ij = W_ij + W_ji + lam * sign(omega_ij)           = 0   ((i, j) in A)

while the entries outside A stay 0 under small changes of S and lam (strict
complementarity).  The implicit function theorem gives, for a loss L with
gradient C = dL/dOmega-hat,

    J^T v = dL/dtheta,     dL/dS = -sum_r v_r dR_r/dS,     dL/dlam = -sum_r v_r dR_r/dlam,

with theta the free entries (omega_ii, and omega_ij = omega_ji for (i,j) in
A) and J = dR/dtheta.  Everything below is that definition written out:
J column by column from dR/dtheta, then one dense solve (a library routine).
The returned dL/dS is the symmetric gradient (dL = sum_ab G_ab dS_ab for every
symmetric dS).
"""
from __future__ import annotations

import numpy as np


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def free_coordinates(omega):
    """theta's coordinates: ('d', i) for every diagonal entry, then ('o', i, j)
    for every i < j with omega_ij != 0 (row-major order)."""
    om = _f64(omega)
    p = om.shape[0]
    coords = [("d", i) for i in range(p)]
    iu, ju = np.nonzero(np.triu(om != 0, 1))
    coords += [("o", int(i), int(j)) for i, j in zip(iu, ju)]
    return coords


def residuals(S, omega, lam: float, coords=None) -> np.ndarray:
    """The stationarity residuals R_r at Omega, in the order of coords."""
    S, om = _f64(S), _f64(omega)
    coords = free_coordinates(om) if coords is None else coords
    W = om @ S
    out = np.empty(len(coords))
    for r, c in enumerate(coords):
        if c[0] == "d":
            i = c[1]
            out[r] = W[i, i] - 1.0 / om[i, i]
        else:
            i, j = c[1], c[2]
            out[r] = W[i, j] + W[j, i] + lam * np.sign(om[i, j])
    return out


def _unit_times_S(c, S):
    """E_c S: E_c has ones at (k, l) and (l, k) (at (k, k) for a diagonal
    coordinate), so row k of E_c S is S_l., row l is S_k., the rest is 0."""
    dW = np.zeros_like(S)
    if c[0] == "d":
        dW[c[1]] = S[c[1]]
    else:
        dW[c[1]] += S[c[2]]
        dW[c[2]] += S[c[1]]
    return dW


def jacobian(S, omega, coords=None) -> np.ndarray:
    """J[r, t] = dR_r / dtheta_t.  Moving theta_t by one changes W by E_t S
    and, for a diagonal coordinate, 1/omega_ii by -1/omega_ii^2."""
    S, om = _f64(S), _f64(omega)
    coords = free_coordinates(om) if coords is None else coords
    N = len(coords)
    # residual r reads W at (ri, rj) and (rj, ri); a diagonal one has ri = rj
    # and counts the entry once
    ri = np.array([c[1] for c in coords])
    rj = np.array([c[1] if c[0] == "d" else c[2] for c in coords])
    isd = np.array([c[0] == "d" for c in coords])
    J = np.zeros((N, N))
    for t, ct in enumerate(coords):
        dW = _unit_times_S(ct, S)
        col = dW[ri, rj] + np.where(isd, 0.0, dW[rj, ri])
        if ct[0] == "d":
            col[t] += 1.0 / om[ct[1], ct[1]] ** 2
        J[:, t] = col
    return J


def backward(S, omega, lam: float, grad_omega) -> dict:
    """dL/dS (symmetric, p x p) and dL/dlam at Omega-hat for dL/dOmega-hat =
    grad_omega, by a dense solve of the stationarity system.

    Also returns v (the adjoint, laid out as a symmetric p x p matrix V with
    V_ii = v_ii, V_ij = V_ji = v_ij on A and 0 elsewhere) and J."""
    S, om, C = _f64(S), _f64(omega), _f64(grad_omega)
    p = S.shape[0]
    coords = free_coordinates(om)
    J = jacobian(S, om, coords)
    g = np.array([C[c[1], c[1]] if c[0] == "d" else C[c[1], c[2]] + C[c[2], c[1]]
                  for c in coords])
    v = np.linalg.solve(J.T, g)
    # dR_r/dS_ab as a general (unsymmetric) matrix: d W_ij / d S_ab = omega_ia [b == j]
    G = np.zeros((p, p))
    glam = 0.0
    V = np.zeros((p, p))
    for r, c in enumerate(coords):
        if c[0] == "d":
            i = c[1]
            G[:, i] -= v[r] * om[i, :]
            V[i, i] = v[r]
        else:
            i, j = c[1], c[2]
            G[:, j] -= v[r] * om[i, :]
            G[:, i] -= v[r] * om[j, :]
            glam -= v[r] * np.sign(om[i, j])
            V[i, j] = V[j, i] = v[r]
    return dict(grad_S=0.5 * (G + G.T), grad_lambda=float(glam), V=V, J=J, coords=coords)
