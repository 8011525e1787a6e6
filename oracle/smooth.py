"""Smooth(p, alpha): the post-processing step of PlanSelection (oracle, FP64).

Test infrastructure only: it checks the HIP path and is never called by it.

Alg. 5 returns Smooth(p*, alpha) rather than p* itself: a local improvement of
the selected plan that keeps the CP constraint (Sec. IV, the definition of
Smooth after the primitives; Sec. IV's description of the final phase).  The
paper defers the method to a cited work and states its shape: a bisection
search over plans formed as a combination of p* and the unconstrained optimal
trajectory from x_init to p*.head, each re-certified.

Readings (the paper gives no formulas):
  * the plan p is its concatenated edge trajectories (the Hermite cubics of
    Cost, durations tau_e, total T_p); q is the optimal connection
    x_init -> p.head (duration tau_q = tau*, cost c*);
  * blend with weight beta in [0, 1] over normalised time s in [0, 1]:
    duration T = (1 - beta) T_p + beta tau_q and position
    P(s) = (1 - beta) p(s T_p) + beta q(s tau_q).  At s = 0 and s = 1 both
    terms share position and (scaled) velocity, so the blend keeps x_init and
    p.head exactly, velocities included;
  * its cost is T + r_u int_0^T |d^2P/dt^2|^2 dt = T + r_u N / T^3 with
    N = int_0^1 |P''(s)|^2 ds; P'' is linear in s between the plan's edge
    breakpoints, so N is a sum of exact Simpson rules;
  * its tracking grid: K = max(1, ceil(T / dt)) waypoints at s_k = k / K (one
    trajectory), certified by MC over those waypoints with the same M
    particles (same noise) as MC(p); a grid longer than the certification
    noise (K > S_max) is not certified;
  * search: beta = 1 first; if it is not certified, BISECT_STEPS bisection
    steps on [lo, hi] = [0, 1] (the midpoint becomes lo if certified, else
    hi); the result is the blend at the final lo when lo > 0 and its cost is
    below p's, otherwise p itself (beta = 0);
  * certified means count / M <= alpha, as in Alg. 5.
"""

from __future__ import annotations

import math

import numpy as np

from . import steer as st

BISECT_STEPS = 9


def plan_edges(V, nodes, r_u):
    """(tau [E], cost [E], coef [E, 3, 4], t0 [E + 1]) of the plan's edges;
    t0 holds the edge start times, t0[E] = T_p (summed edge by edge)."""
    V = np.asarray(V, np.float64)
    u = np.array(nodes[:-1], np.int64)
    v = np.array(nodes[1:], np.int64)
    tau, cost = st.steer(V[u], V[v], r_u)
    coef = st.hermite(V[u], V[v], tau)
    t0 = np.zeros(len(tau) + 1)
    for e in range(len(tau)):
        t0[e + 1] = t0[e] + tau[e]
    return tau, cost, coef, t0


def optimal_connection(V, nodes, r_u):
    """(tau_q, c_q, coef [3, 4]) of the optimal trajectory x_init -> head."""
    V = np.asarray(V, np.float64)
    a, b = V[nodes[0]][None], V[nodes[-1]][None]
    tau, cost = st.steer(a, b, r_u)
    return float(tau[0]), float(cost[0]), st.hermite(a, b, tau)[0]


def _edge_at(t0, t):
    """Edge index holding plan time t (the last edge holds T_p)."""
    E = t0.shape[0] - 1
    return np.clip(np.searchsorted(t0, t, side="right") - 1, 0, E - 1)


def blend_positions(s, beta, edges, q):
    """P(s) [len(s), 3] of the blend with weight beta."""
    _, _, coef, t0 = edges
    tau_q, _, qc = q
    s = np.asarray(s, np.float64)
    T_p = t0[-1]
    t = s * T_p
    e = _edge_at(t0, t)
    p = st.hermite_eval(coef[e], t - t0[e])
    r = st.hermite_eval(qc[None], s * tau_q)
    return (1.0 - beta) * p + beta * r


def _second(beta, coef_e, loc_p, tau_q, qc, t_q, T_p):
    """P''(s) [3] from edge coefficients at local plan time loc_p and optimal
    time t_q (derivatives with respect to s)."""
    pdd = 2.0 * coef_e[:, 2] + 6.0 * coef_e[:, 3] * loc_p
    qdd = 2.0 * qc[:, 2] + 6.0 * qc[:, 3] * t_q
    return (1.0 - beta) * T_p * T_p * pdd + beta * tau_q * tau_q * qdd


def blend_effort(beta, edges, q):
    """N(beta) = int_0^1 |P''(s)|^2 ds, exact (Simpson on each edge piece)."""
    _, _, coef, t0 = edges
    tau_q, _, qc = q
    T_p = t0[-1]
    total = 0.0
    for e in range(coef.shape[0]):
        sa, sb = t0[e] / T_p, t0[e + 1] / T_p
        sm = 0.5 * (sa + sb)
        f = []
        for s in (sa, sm, sb):
            P2 = _second(beta, coef[e], s * T_p - t0[e], tau_q, qc, s * tau_q, T_p)
            f.append(float(P2 @ P2))
        total += (sb - sa) / 6.0 * (f[0] + 4.0 * f[1] + f[2])
    return total


def blend_cost(beta, edges, q, r_u):
    """T + r_u N / T^3 of the blend."""
    T = (1.0 - beta) * edges[3][-1] + beta * q[0]
    return T + r_u * blend_effort(beta, edges, q) / T ** 3


def blend_waypoints(beta, edges, q, dt):
    """Tracking waypoints [K + 1, 3] of the blend (K = max(1, ceil(T / dt)))."""
    T = (1.0 - beta) * edges[3][-1] + beta * q[0]
    K = max(1, int(math.ceil(T / dt)))
    s = np.arange(K + 1, dtype=np.float64) / K
    return blend_positions(s, beta, edges, q)


def bisect_beta(certified):
    """The search over the blend weight: beta = 1 if certified(1), else
    BISECT_STEPS halvings of [0, 1] keeping the certified side low."""
    if certified(1.0):
        return 1.0
    lo, hi = 0.0, 1.0
    for _ in range(BISECT_STEPS):
        m = 0.5 * (lo + hi)
        if certified(m):
            lo = m
        else:
            hi = m
    return lo


def smooth(V, nodes, plan_cost, plan_steps, plan_count, alpha, M, S_max, count_fn, r_u, dt):
    """Smooth(p, alpha).  count_fn(W) is the MC count over waypoints W.
    Returns dict(beta, cost, count, steps, W, evals {beta: count or None})."""
    keep = dict(beta=0.0, cost=plan_cost, count=plan_count, steps=plan_steps, W=None, evals={})
    if len(nodes) < 2:
        return keep
    edges = plan_edges(V, nodes, r_u)
    q = optimal_connection(V, nodes, r_u)
    evals = keep["evals"]

    def certified(beta):
        W = blend_waypoints(beta, edges, q, dt)
        if W.shape[0] - 1 > S_max:
            evals[beta] = None
            return False
        c = count_fn(W)
        evals[beta] = c
        return not (c / M > alpha)

    beta = bisect_beta(certified)
    if beta > 0.0:
        cost = blend_cost(beta, edges, q, r_u)
        if cost < plan_cost:
            W = blend_waypoints(beta, edges, q, dt)
            return dict(beta=beta, cost=cost, count=evals[beta], steps=W.shape[0] - 1, W=W,
                        evals=evals)
    return keep
