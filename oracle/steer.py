"""Cost(u, v): the optimal double-integrator connection (oracle, FP64).

Sec. II takes the trajectory cost as elapsed time plus a quadratic control
effort, c = tau + int_0^tau u^T R u dt; Sec. IV defines Cost(u, v) as the cost of
the optimal trajectory between two states.  Reading: R = r_u * I.

For a fixed duration tau the minimum-effort control of x'' = u between
(p0, v0) and (p1, v1) is linear in time, the position is the cubic Hermite
interpolant, and per axis (P = p1 - p0) the effort is

    J_a(tau) = 12 P^2 / tau^3 - 12 P (v0 + v1) / tau^2 + 4 (v0^2 + v0 v1 + v1^2) / tau

(the controllability-Gramian form d^T G(tau)^-1 d with G = [[tau^3/3, tau^2/2],
[tau^2/2, tau]] and d = (P - v0 tau, v1 - v0), expanded).  Summed over axes with
S_PP = sum P^2, S_Pv = sum P (v0 + v1), S_vv = sum (v0^2 + v0 v1 + v1^2):

    c(tau) = tau + r_u (12 S_PP / tau^3 - 12 S_Pv / tau^2 + 4 S_vv / tau).

The optimal duration minimises c over tau > 0; its stationary points are the
positive real roots of tau^4 - 4 r_u S_vv tau^2 + 24 r_u S_Pv tau - 36 r_u S_PP,
and c -> +inf at both ends, so the global minimum is the least c over those
roots (reading: ties go to the smaller tau).
"""

from __future__ import annotations

import numpy as np


def boundary_sums(x0, x1):
    """S_PP, S_Pv, S_vv for state pairs (..., 6)."""
    x0 = np.asarray(x0, np.float64)
    x1 = np.asarray(x1, np.float64)
    P = x1[..., :3] - x0[..., :3]
    v0 = x0[..., 3:]
    v1 = x1[..., 3:]
    S_PP = np.sum(P * P, axis=-1)
    S_Pv = np.sum(P * (v0 + v1), axis=-1)
    S_vv = np.sum(v0 * v0 + v0 * v1 + v1 * v1, axis=-1)
    return S_PP, S_Pv, S_vv


def cost_of_duration(tau, S_PP, S_Pv, S_vv, r_u):
    """c(tau) above."""
    tau = np.asarray(tau, np.float64)
    return tau + r_u * (12.0 * S_PP / tau ** 3 - 12.0 * S_Pv / tau ** 2
                        + 4.0 * S_vv / tau)


def optimal_duration(S_PP, S_Pv, S_vv, r_u):
    """(tau*, c*) for arrays of boundary sums.

    The quartic's roots come from the eigenvalues of its companion matrix (a
    library eigen-solver); every root with a positive real part and a small
    imaginary part is a candidate, polished by two Newton steps, and tau* is the
    candidate of least cost.  Evaluating c at a point that is not a minimiser
    can only give a larger value, so generous candidate acceptance is safe.
    Pairs with S_PP = S_vv = 0 (identical states) get tau* = 0, c* = 0."""
    S_PP = np.atleast_1d(np.asarray(S_PP, np.float64))
    S_Pv = np.atleast_1d(np.asarray(S_Pv, np.float64))
    S_vv = np.atleast_1d(np.asarray(S_vv, np.float64))
    n = S_PP.shape[0]
    a2 = -4.0 * r_u * S_vv
    a1 = 24.0 * r_u * S_Pv
    a0 = -36.0 * r_u * S_PP
    comp = np.zeros((n, 4, 4))
    comp[:, 0, 1] = -a2
    comp[:, 0, 2] = -a1
    comp[:, 0, 3] = -a0
    comp[:, 1, 0] = 1.0
    comp[:, 2, 1] = 1.0
    comp[:, 3, 2] = 1.0
    roots = np.linalg.eigvals(comp) if n else np.zeros((0, 4), complex)
    re = roots.real
    ok = (re > 0) & (np.abs(roots.imag) <= 1e-4 * np.maximum(1.0, np.abs(re)))
    t = np.where(ok, re, 1.0)
    for _ in range(2):
        f = t ** 4 + a2[:, None] * t ** 2 + a1[:, None] * t + a0[:, None]
        fp = 4.0 * t ** 3 + 2.0 * a2[:, None] * t + a1[:, None]
        step = np.where(fp != 0, f / np.where(fp != 0, fp, 1.0), 0.0)
        tn = t - step
        t = np.where(ok & (tn > 0), tn, t)
    c = np.where(ok, cost_of_duration(t, S_PP[:, None], S_Pv[:, None],
                                      S_vv[:, None], r_u), np.inf)
    # least cost; ties to the smaller tau
    order = np.lexsort((np.where(ok, t, np.inf), c), axis=-1)
    best = order[:, 0]
    tau = t[np.arange(n), best]
    cst = c[np.arange(n), best]
    degenerate = (S_PP == 0) & (S_vv == 0)
    tau = np.where(degenerate, 0.0, tau)
    cst = np.where(degenerate, 0.0, cst)
    return tau, cst


def steer(x0, x1, r_u):
    """Cost(x0, x1) for state pairs: returns (tau*, c*)."""
    return optimal_duration(*boundary_sums(x0, x1), r_u)


def hermite(x0, x1, tau):
    """Per-axis cubic p(t) = p0 + v0 t + c2 t^2 + c3 t^3 with p(tau) = p1 and
    p'(tau) = v1 (the minimum-effort nominal trajectory).
    Returns coefficients [..., 3, 4] = (p0, v0, c2, c3)."""
    x0 = np.asarray(x0, np.float64)
    x1 = np.asarray(x1, np.float64)
    tau = np.asarray(tau, np.float64)[..., None]
    p0 = x0[..., :3]
    v0 = x0[..., 3:]
    v1 = x1[..., 3:]
    P = x1[..., :3] - p0
    c2 = (3.0 * P - (2.0 * v0 + v1) * tau) / tau ** 2
    c3 = (-2.0 * P + (v0 + v1) * tau) / tau ** 3
    return np.stack([p0, v0, c2, c3], axis=-1)


def hermite_eval(coef, t):
    """Position at times t; coef [..., 3, 4], t broadcast against [...]."""
    t = np.asarray(t, np.float64)[..., None]
    return coef[..., 0] + t * (coef[..., 1] + t * (coef[..., 2] + t * coef[..., 3]))


def waypoint_count(tau, dt):
    """K_e = max(1, ceil(tau / dt)) waypoints on an edge (reading: the tracking
    grid of eq. (2) laid over the edge, spacing tau / K_e <= dt)."""
    return np.maximum(1, np.ceil(np.asarray(tau, np.float64) / float(dt))).astype(np.int64)
