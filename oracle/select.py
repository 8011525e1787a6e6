"""MC(p) and PlanSelection (Alg. 5) (oracle, FP64).

Sec. IV defines MC(p) as an asymptotically exact Monte Carlo CP estimate of a
plan with full collision checking; Alg. 5 sorts P_goal by cp_hat and runs a
bisection on MC(P_m) <= alpha.

Readings: MC draws M fresh particles (their own noise, passed in) through the
same closed-loop deviation model, from a zero deviation at x_init, over the
plan's full tracking grid; a particle's workspace path is the polyline through
its waypoint positions, and it collides iff some segment meets a closed box;
MC(p) = colliding / M (no variance reduction).  Before sorting, P_goal is
reduced to its Pareto front across goal nodes (same dominance as
RemoveDominated); ties in cp_hat are broken by cost descending, then by node
sequence.  Smooth(p, alpha) is in smooth.py.
"""

from __future__ import annotations


import numpy as np

from . import steer as st


def plan_waypoints(V, nodes, r_u, dt):
    """Nominal positions of a plan's tracking waypoints, step 0 = x_init:
    an array [S+1, 3].  Each edge (u, v) contributes K_e waypoints at
    t_k = k tau*/K_e, k = 1..K_e."""
    V = np.asarray(V, np.float64)
    pts = [V[nodes[0], :3][None, :]]
    for u, v in zip(nodes[:-1], nodes[1:]):
        tau, _ = st.steer(V[u][None], V[v][None], r_u)
        K = int(st.waypoint_count(tau, dt)[0])
        coef = st.hermite(V[u][None], V[v][None], tau)[0]
        k = np.arange(1, K + 1)
        t = (k * tau[0]) / K
        pts.append(st.hermite_eval(coef[None, :, :], t))
    return np.concatenate(pts, axis=0)


def segments_hit_box(a, b, lo, hi):
    """Closed-box test of segments a -> b ([M, 3] each) by slab clipping."""
    t0 = np.zeros(a.shape[0])
    t1 = np.ones(a.shape[0])
    miss = np.zeros(a.shape[0], bool)
    for ax in range(3):
        d = b[:, ax] - a[:, ax]
        flat = d == 0
        out = flat & ((a[:, ax] < lo[ax]) | (a[:, ax] > hi[ax]))
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = (lo[ax] - a[:, ax]) / d
            tb = (hi[ax] - a[:, ax]) / d
        lo_t = np.where(flat, -np.inf, np.minimum(ta, tb))
        hi_t = np.where(flat, np.inf, np.maximum(ta, tb))
        t0 = np.maximum(t0, lo_t)
        t1 = np.minimum(t1, hi_t)
        miss |= out
    return (~miss) & (t0 <= t1)


def mc_count(V, nodes, boxes, A_cl, L, noise_mc, r_u, dt):
    """Number of the M certification particles whose path meets an obstacle."""
    return mc_count_waypoints(plan_waypoints(V, nodes, r_u, dt), boxes, A_cl, L, noise_mc)


def mc_count_waypoints(W, boxes, A_cl, L, noise_mc):
    """MC count over given nominal waypoints W [S+1, 3] (step 0 = start)."""
    S = W.shape[0] - 1
    xi = np.asarray(noise_mc, np.float64)
    M = xi.shape[2]
    if S > xi.shape[0]:
        raise ValueError("plan longer than the certification noise")
    b = np.asarray(boxes, np.float64)
    dev = np.zeros((3, 2, M))
    prev = np.broadcast_to(W[0][:, None], (3, M)).T.copy()
    hit = np.zeros(M, bool)
    for s in range(S):
        for a in range(3):
            dev[a] = A_cl @ dev[a] + L @ xi[s, 2 * a:2 * a + 2, :]
        cur = (W[s + 1][:, None] + dev[:, 0, :]).T
        for j in range(b.shape[0]):
            hit |= segments_hit_box(prev, cur, b[j, :3], b[j, 3:])
        prev = cur
    return int(hit.sum())


def mc_count_lqg(V, nodes, boxes, M_cl, E, noise_mc, noise_mc_meas, r_u, dt):
    """mc_count with LQG tracking (dynamics.lqg_closed_loop): each
    certification particle carries (dx, x_hat) per axis, driven by its process
    and measurement noise; its position is the waypoint plus dx's position."""
    return mc_count_lqg_waypoints(plan_waypoints(V, nodes, r_u, dt), boxes, M_cl, E, noise_mc,
                                  noise_mc_meas)


def mc_count_lqg_waypoints(W, boxes, M_cl, E, noise_mc, noise_mc_meas):
    """mc_count_lqg over given nominal waypoints W [S+1, 3]."""
    S = W.shape[0] - 1
    xi = np.asarray(noise_mc, np.float64)
    xm = np.asarray(noise_mc_meas, np.float64)
    M = xi.shape[2]
    if S > xi.shape[0]:
        raise ValueError("plan longer than the certification noise")
    b = np.asarray(boxes, np.float64)
    z = np.zeros((3, 4, M))
    prev = np.broadcast_to(W[0][:, None], (3, M)).T.copy()
    hit = np.zeros(M, bool)
    for s in range(S):
        for a in range(3):
            nz = np.concatenate([xi[s, 2 * a:2 * a + 2, :], xm[s, a:a + 1, :]], axis=0)
            z[a] = M_cl @ z[a] + E @ nz
        cur = (W[s + 1][:, None] + z[:, 0, :]).T
        for j in range(b.shape[0]):
            hit |= segments_hit_box(prev, cur, b[j, :3], b[j, 3:])
        prev = cur
    return int(hit.sum())


def pareto_front(plans):
    """Plans of the list not dominated by another of the list:
    d dominates p iff p.cost > d.cost and p.pop >= d.pop."""
    return [p for p in plans
            if not any(p.cost > d.cost and p.pop >= d.pop for d in plans)]


def plan_selection(goal_plans, alpha, mc):
    """Alg. 5.  `mc(plan)` returns the certification count; MC(P_m) is that
    count over M.  Returns (chosen plan or None, sorted front, evaluations)."""
    front = pareto_front(goal_plans)
    if not front:
        return None, [], {}
    P = sorted(front, key=lambda p: (p.pop, -p.cost, p.nodes))
    evals = {}

    def MC(m):
        if m not in evals:
            evals[m] = mc(P[m - 1])
        return evals[m]

    # Alg. 5 bisects the risk-sorted front for the riskiest plan whose MC
    # estimate is within alpha, premised on MC growing along the order.
    # `good` is the plan the search stands on (it starts on the safest plan,
    # not yet evaluated); plans from `bad` on are ruled out.  A probe in the
    # middle of the open range moves `good` up when within alpha and `bad`
    # down otherwise; when nothing lies strictly between them, `good` gets
    # one last evaluation (it may never have been probed) before it is
    # returned, and the query is infeasible if it fails.
    good, bad = 1, len(P) + 1
    while bad - good > 1:
        mid = (good + bad) // 2
        if MC(mid)[1] <= alpha:
            good = mid
        else:
            bad = mid
    if MC(good)[1] > alpha:
        return None, P, evals
    return P[good - 1], P, evals
