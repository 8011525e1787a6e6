"""PUMP main (Alg. 2) and the parameters the paper leaves open (oracle).

Alg. 2: build the graph, set alpha_min = alpha/eta and alpha_max = eta*alpha,
explore, select.  Real-valued parameters arrive as FP32 (as the library's
configuration does) and are used exactly, widened to FP64.

Readings: eta = 2 for alpha >= 1%, eta = 10 for alpha <= 0.1% (Sec. V-A) and
log-linear in between; lambda = 0.5 (Sec. V-A); r_n = 1.0; steering effort
weight r_u = 0.1; tracking step dt = 0.05; LQR weights Q = diag(100, 10),
R = 1 per axis; goal nodes are samples whose position lies in the closed goal
box (velocity free); x_init is node 0.
"""

from __future__ import annotations

import dataclasses
import math
import time

import numpy as np

from . import dynamics, explore as ex, graph as gr, select as sel, smooth as sm


def f32(x) -> float:
    return float(np.float32(x))


@dataclasses.dataclass
class Config:
    dt: float = f32(0.05)
    q_pos: float = f32(100.0)
    q_vel: float = f32(10.0)
    r_track: float = f32(1.0)
    r_steer: float = f32(0.1)
    r_conn: float = f32(1.0)
    eta: float = 0.0          # 0: the rule above
    lam: float = f32(0.5)
    cp_model: str = "box"     # exploration collision model: "box" or "hsmc"
    estimator: str = "lqr"    # tracking: "lqr" (full state) or "lqg" (Kalman estimate)
    smooth: bool = False      # Smooth(p*, alpha) after selection (smooth.py); off: identity


def eta_rule(alpha: float) -> float:
    """Sec. V-A: eta = 2 above 1%, 10 at 0.1%; log-linear between (reading)."""
    if alpha >= 0.01:
        return 2.0
    if alpha <= 0.001:
        return 10.0
    w = (math.log(0.01) - math.log(alpha)) / (math.log(0.01) - math.log(0.001))
    return math.exp(math.log(2.0) + w * (math.log(10.0) - math.log(2.0)))


def thresholds(alpha: float, eta: float):
    """Alg. 2: alpha_min = alpha / eta, alpha_max = eta * alpha (FP64)."""
    return alpha / eta, eta * alpha


def run(scene, cfg: Config = Config(), record=False, with_selection=True):
    """PUMP on one scene.  Returns a dict with the graph, plans, P_goal front,
    the chosen plan, statistics and (optionally) per-round snapshots."""
    t0 = time.perf_counter()
    V = np.concatenate([scene.x_init[None, :], scene.samples], axis=0).astype(np.float64)
    alpha = float(scene.alpha)
    eta = cfg.eta if cfg.eta > 0 else eta_rule(alpha)
    alpha_min, alpha_max = thresholds(alpha, eta)
    A_cl, L, K = dynamics.closed_loop(cfg.dt, scene.sigma, cfg.q_pos, cfg.q_vel, cfg.r_track)
    S_max = scene.S_max
    if cfg.estimator == "lqg":
        M_cl, E_cl, _, _ = dynamics.lqg_closed_loop(cfg.dt, scene.sigma, scene.sigma_meas,
                                                    cfg.q_pos, cfg.q_vel, cfg.r_track)
        D = dynamics.lqg_deviation_table(M_cl, E_cl, scene.noise, scene.noise_meas, S_max)
    else:
        D = dynamics.deviation_table(A_cl, L, scene.noise, S_max)
    g = gr.build_graph(V, scene.obstacles, cfg.r_conn, cfg.r_steer)
    t1 = time.perf_counter()
    gl = scene.goal.astype(np.float64)
    in_goal = np.all((V[:, :3] >= gl[:3]) & (V[:, :3] <= gl[3:]), axis=1) & g["valid"]
    goal_nodes = np.nonzero(in_goal)[0]
    plans, P, stats, rounds = ex.explore(V, g, D, scene.obstacles, goal_nodes, alpha_min,
                                         alpha_max, cfg.lam, cfg.r_conn, cfg.dt, S_max,
                                         record=record, cp_model=cfg.cp_model)
    t2 = time.perf_counter()
    Pg = ex.goal_plans(plans, P, goal_nodes)
    out = dict(V=V, graph=g, D=D, A_cl=A_cl, L=L, K=K, eta=eta, alpha_min=alpha_min,
               alpha_max=alpha_max, goal_nodes=goal_nodes, plans=plans, P=P,
               stats=stats, rounds=rounds, goal_plans=Pg,
               ms_build=1e3 * (t1 - t0), ms_explore=1e3 * (t2 - t1))
    if not with_selection:
        return out
    M = scene.M

    def mc(plan):
        if cfg.estimator == "lqg":
            c = sel.mc_count_lqg(V, plan.nodes, scene.obstacles, M_cl, E_cl, scene.noise_mc,
                                 scene.noise_mc_meas, cfg.r_steer, cfg.dt)
        else:
            c = sel.mc_count(V, plan.nodes, scene.obstacles, A_cl, L, scene.noise_mc,
                             cfg.r_steer, cfg.dt)
        return c, c / M

    best, front, evals = sel.plan_selection(Pg, alpha, mc)
    t3 = time.perf_counter()
    if not Pg:
        status = 2            # no goal plan
    elif best is None:
        status = 1            # infeasible: no plan certified
    else:
        status = 0
    out.update(best=best, front=front, evals=evals, status=status,
               ms_select=1e3 * (t3 - t2))
    if cfg.smooth and best is not None:
        def count_w(W):
            if cfg.estimator == "lqg":
                return sel.mc_count_lqg_waypoints(W, scene.obstacles, M_cl, E_cl, scene.noise_mc,
                                                  scene.noise_mc_meas)
            return sel.mc_count_waypoints(W, scene.obstacles, A_cl, L, scene.noise_mc)
        k = front.index(best) + 1
        out["smooth"] = sm.smooth(V, best.nodes, best.cost, best.step, evals[k][0], alpha, M,
                                  S_max, count_w, cfg.r_steer, cfg.dt)
    return out
