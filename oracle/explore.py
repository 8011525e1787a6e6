"""Explore (Alg. 4): the bucketed multiobjective search (oracle, FP64).

Plans are records (head, path, cost, cp_hat) (Sec. IV); cp_hat is the particle
estimate: N particle trajectories follow the plan, and a particle counts as
invalid once any of its waypoint positions lies in an obstacle; cp_hat is the
number of invalid particles over N (Sec. III-B: per-particle checks, an OR
over the trajectory, a count).  A plan carries its particles' invalid bits, so
extending it by one edge ORs in the new edge's hits.

Readings used here:
  * particles: the deviation of particle j at plan step s is the shared table
    D[s][.][j] (plan-independent; see dynamics.py); an edge of duration tau* gets
    K_e = max(1, ceil(tau*/dt)) waypoints at t_k = k tau*/K_e, k = 1..K_e, at
    plan steps s_p + k, and particle j's position there is nominal(t_k) + D[s_p+k].
  * the per-waypoint predicate is "position inside a closed box";
  * a candidate whose step count exceeds S_max is dropped (and counted);
  * RemoveDominated acts on every plan still open at that point, including
    the group just expanded, against all plans with the same head; closed
    plans are never removed; dominance is strict on cost and non-strict on
    cp_hat, so plans with equal (cost, cp_hat) coexist;
  * every (p in B, x in N(p.head)) pair formed counts as one partial plan.
"""

from __future__ import annotations

import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np

from . import steer as st

EPS_FLAG = 1e-5


@dataclasses.dataclass
class Plan:
    nodes: tuple        # path + head (node indices from x_init)
    cost: float
    step: int           # tracking steps covered so far
    mask: np.ndarray    # bool [N]: particle j invalid
    parent: int
    # bool [N]: particles whose bit was decided within EPS_FLAG of a face
    # somewhere along the plan while still valid (None: not tracked)
    fmask: Optional[np.ndarray] = None
    pop: int = dataclasses.field(init=False)   # number of invalid particles

    def __post_init__(self):
        self.pop = int(self.mask.sum())

    @property
    def head(self) -> int:
        return self.nodes[-1]


def extend_batch(V, graph, D, boxes, dt, S_max, parents: List[Plan], edges: np.ndarray,
                 chunk=256, cp_model="box", hs_cache=None):
    """q = (x, p.path + p.head, p.cost + Cost(p.head, x), CP_hat(x, p)) for many
    (p, edge) pairs (Alg. 4, the line that forms q).

    cp_model "box": a particle collides at a waypoint when its position lies in
    a closed box; "hsmc": when its deviation violates one of the waypoint's
    half-spaces (hsmc.py).  hs_cache (dict) keeps the half-spaces of each
    (edge, waypoint).

    A (pair, particle) decision is flagged when the parent's bit is 0, the
    particle comes within EPS_FLAG of a face (or a half-space boundary) at one
    of the edge's waypoints and nowhere lies EPS_FLAG or more inside.

    Returns (x, cost, step, mask [m, N], over_steps [m], flagged [m, N])."""
    if cp_model == "hsmc":
        return _extend_hsmc(V, graph, D, boxes, dt, S_max, parents, edges,
                            {} if hs_cache is None else hs_cache)
    V = np.asarray(V, np.float64)
    b = np.asarray(boxes, np.float64)
    m = len(parents)
    N = D.shape[2]
    x = graph["col"][edges]
    tau = graph["tau"][edges]
    cst = graph["cost"][edges]
    K = st.waypoint_count(tau, dt)
    s_p = np.array([p.step for p in parents], np.int64)
    heads = np.array([p.head for p in parents], np.int64)
    cost = np.array([p.cost for p in parents]) + cst
    step = s_p + K
    over = step > S_max
    mask = np.stack([p.mask for p in parents]) if m else np.zeros((0, N), bool)
    mask = mask.copy()
    flagged = np.zeros((m, N), bool)
    Dd = np.asarray(D, np.float64)
    for c0 in range(0, m, chunk):
        sl = slice(c0, min(m, c0 + chunk))
        idx = np.arange(sl.start, sl.stop)
        idx = idx[~over[idx]]
        if idx.shape[0] == 0:
            continue
        coef = st.hermite(V[heads[idx]], V[x[idx]], tau[idx])
        Kmax = int(K[idx].max())
        k = np.arange(1, Kmax + 1)
        live = k[None, :] <= K[idx][:, None]                       # [c, Kmax]
        t = (k[None, :] * tau[idx][:, None]) / K[idx][:, None]
        nom = st.hermite_eval(coef[:, None, :, :], t)              # [c, Kmax, 3]
        srow = np.minimum(s_p[idx][:, None] + k[None, :], S_max)
        y = nom[..., None] + Dd[srow]                               # [c, Kmax, 3, N]
        hit = np.zeros((idx.shape[0], N), bool)
        best = np.full((idx.shape[0], N), -np.inf)                  # max depth
        near = np.zeros((idx.shape[0], N), bool)
        for j in range(b.shape[0]):
            lo = b[j, :3][None, None, :, None]
            hi = b[j, 3:][None, None, :, None]
            inside = np.all((y >= lo) & (y <= hi), axis=2)         # [c, Kmax, N]
            inside &= live[..., None]
            hit |= inside.any(axis=1)
            depth = np.minimum(y - lo, hi - y).min(axis=2)         # [c, Kmax, N]
            depth = np.where(live[..., None], depth, -np.inf)
            best = np.maximum(best, depth.max(axis=1))
            near |= ((np.abs(depth) < EPS_FLAG) & live[..., None]).any(axis=1)
        par = mask[idx]
        flagged[idx] = (~par) & near & (best < EPS_FLAG)
        mask[idx] = par | hit
    return x, cost, step, mask, over, flagged


def _extend_hsmc(V, graph, D, boxes, dt, S_max, parents, edges, cache):
    """extend_batch with the HSMC predicate (one pair at a time)."""
    from . import hsmc
    V = np.asarray(V, np.float64)
    m = len(parents)
    N = D.shape[2]
    x = graph["col"][edges]
    tau = graph["tau"][edges]
    cst = graph["cost"][edges]
    K = st.waypoint_count(tau, dt)
    s_p = np.array([p.step for p in parents], np.int64)
    heads = np.array([p.head for p in parents], np.int64)
    cost = np.array([p.cost for p in parents]) + cst
    step = s_p + K
    over = step > S_max
    mask = np.stack([p.mask for p in parents]) if m else np.zeros((0, N), bool)
    mask = mask.copy()
    flagged = np.zeros((m, N), bool)
    Dd = np.asarray(D, np.float64)
    for q in range(m):
        if over[q]:
            continue
        e = int(edges[q])
        regions = cache.get(e)
        if regions is None:
            coef = st.hermite(V[heads[q]][None], V[x[q]][None], tau[q:q + 1])[0]   # [3, 4]
            regions = []
            for k in range(1, int(K[q]) + 1):
                t = k * tau[q] / K[q]
                pos = coef[:, 0] + t * (coef[:, 1] + t * (coef[:, 2] + t * coef[:, 3]))
                vel = coef[:, 1] + t * (2.0 * coef[:, 2] + t * 3.0 * coef[:, 3])
                regions.append(hsmc.halfspaces(pos, vel, boxes))
            cache[e] = regions
        hit = np.zeros(N, bool)
        best = np.full(N, -np.inf)
        near = np.zeros(N, bool)
        for k, (a, b) in enumerate(regions, start=1):
            if a.shape[0] == 0:
                continue
            dy = Dd[min(int(s_p[q]) + k, S_max)]                       # [3, N]
            hit |= hsmc.violations(a, b, dy)
            na = np.sqrt(b)
            with np.errstate(divide="ignore", invalid="ignore"):
                mg = np.where(na[:, None] > 0, ((a @ dy) - b[:, None]) / na[:, None], -np.inf)
            best = np.maximum(best, mg.max(axis=0))
            near |= (np.abs(mg) < EPS_FLAG).any(axis=0)
        par = mask[q]
        flagged[q] = (~par) & near & (best < EPS_FLAG)
        mask[q] = par | hit
    return x, cost, step, mask, over, flagged


def row_range(graph, u):
    """Edge-id range of N(u): a CSR row, or a row built on demand
    (graph.RowsOnDemand)."""
    rows = getattr(graph, "rows", None)
    if rows is not None:
        return rows(u)
    return int(graph["row_ptr"][u]), int(graph["row_ptr"][u + 1])


# Worker state of the process pool that splits a round's pairs (set by
# pool_init in each worker process).
_POOL_ARGS = None


def pool_init(V, D, boxes, dt, S_max):
    global _POOL_ARGS
    _POOL_ARGS = (np.asarray(V, np.float64), D, boxes, dt, S_max)


def _pool_extend(job):
    parents, col, tau, cost = job
    V, D, boxes, dt, S_max = _POOL_ARGS
    g = dict(col=col, tau=tau, cost=cost)
    return extend_batch(V, g, D, boxes, dt, S_max, parents, np.arange(col.shape[0]))


def extend_split(pool, V, graph, D, boxes, dt, S_max, parents, edges, pieces):
    """extend_batch over the pairs of one round split into `pieces`
    contiguous slices, each run by a worker of `pool` (pool_init), the results
    concatenated in slice order: the same arrays as one call."""
    m = len(parents)
    cuts = np.linspace(0, m, pieces + 1).astype(np.int64)
    jobs = [(parents[a:b], graph["col"][edges[a:b]], graph["tau"][edges[a:b]],
             graph["cost"][edges[a:b]]) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    outs = pool.map(_pool_extend, jobs)
    if not outs:
        return extend_batch(V, graph, D, boxes, dt, S_max, parents, edges)
    return tuple(np.concatenate([o[k] for o in outs]) for k in range(6))


def dominates(d: Plan, p: Plan) -> bool:
    """d dominates p (Sec. IV, RemoveDominated): d is strictly cheaper and its
    particle CP estimate is no larger (cp_hat = pop / N with the same N, so
    comparing pops is comparing cp_hat)."""
    return d.cost < p.cost and d.pop <= p.pop


def remove_dominated(plans: List[Plan], P: Dict[int, List[int]], P_open: set) -> set:
    """RemoveDominated(P, P_open) (Sec. IV primitives; called once per round in
    Alg. 4 after every candidate of the group has been inserted).

    Only plans of P_open are candidates for removal -- the group just expanded
    is still in P_open at this point -- and each is tested against every plan
    of P(head) (open or closed), all tests taking the sets as they are on entry.
    A removed plan leaves both P(head) and P_open; closed plans are never
    removed.  Returns the set of removed plan ids."""
    removed = set()
    for p in P_open:
        pp = plans[p]
        if any(dominates(plans[d], pp) for d in P[pp.head] if d != p):
            removed.add(p)
    for p in removed:
        P[plans[p].head].remove(p)
        P_open.discard(p)
    return removed


def explore(V, graph, D, boxes, goal_nodes, alpha_min, alpha_max, lam, r_n, dt,
            S_max, record=False, cp_model="box", time_budget=None, pool=None, pieces=1):
    """Alg. 4.  Returns (plans, P, stats, rounds) where P maps head -> plan ids
    still in P(head) at exit and `rounds` holds per-round snapshots if `record`.

    For timing runs only: with `time_budget` (seconds) the loop also ends
    after the first round that finishes past the budget (stats["truncated"]);
    with a process pool (pool_init) each round's pairs are split into
    `pieces` slices that workers extend side by side."""
    N = D.shape[2]
    root = Plan(nodes=(0,), cost=0.0, step=0, mask=np.zeros(N, bool), parent=-1,
                fmask=np.zeros(N, bool))
    plans: List[Plan] = [root]
    P: Dict[int, List[int]] = {0: [0]}
    P_open = {0}
    B = [0]
    i = 0
    h = float(lam) * float(r_n)
    goal = np.zeros(V.shape[0], bool)
    goal[np.asarray(goal_nodes, np.int64)] = True
    stats = dict(partial_plans=0, inserted=0, rounds=0, iterations=0,
                 dropped_steps=0, flagged_particles=0, flagged_below_cut=0)
    hs_cache = {}
    rounds = []
    t_start = time.perf_counter()
    stats["truncated"] = False

    def stop_now():
        return any(goal[plans[g].head] and plans[g].pop / N < alpha_min for g in B)

    while P_open and not stop_now():
        stats["iterations"] += 1
        snap = dict(i=i, B=[plans[p].nodes for p in B]) if record else None
        parents, edges, parent_ids = [], [], []
        for p in sorted(B):
            u = plans[p].head
            e0, e1 = row_range(graph, u)
            for e in range(e0, e1):
                parents.append(plans[p])
                parent_ids.append(p)
                edges.append(e)
        edges = np.asarray(edges, np.int64)
        if B:
            stats["rounds"] += 1
        if pool is not None and cp_model == "box" and len(parents) > pieces:
            x, cost, step, mask, over, flagged = extend_split(
                pool, V, graph, D, boxes, dt, S_max, parents, edges, pieces)
        else:
            x, cost, step, mask, over, flagged = extend_batch(
                V, graph, D, boxes, dt, S_max, parents, edges, cp_model=cp_model,
                hs_cache=hs_cache)
        stats["partial_plans"] += len(parents)
        stats["dropped_steps"] += int(over.sum())
        stats["flagged_particles"] += int(flagged.sum())
        inserted = []
        for q in range(len(parents)):
            if over[q]:
                continue
            cp_hat = mask[q].sum() / N
            if cp_hat < alpha_max:                      # CP cutoff
                # flagged decisions of the pairs that pass the cutoff (a
                # diagnostic count only; the rest of the run ignores it)
                stats["flagged_below_cut"] += int(flagged[q].sum())
                pf = parents[q].fmask
                plan = Plan(nodes=parents[q].nodes + (int(x[q]),), cost=float(cost[q]),
                            step=int(step[q]), mask=mask[q].copy(), parent=parent_ids[q],
                            fmask=flagged[q] if pf is None else (pf | flagged[q]))
                plans.append(plan)
                pid = len(plans) - 1
                P.setdefault(int(x[q]), []).append(pid)
                P_open.add(pid)
                inserted.append(pid)
        stats["inserted"] += len(inserted)
        dominated = remove_dominated(plans, P, P_open)
        P_open -= set(B)
        if record:
            snap["candidates"] = {plans[p].nodes: (plans[p].cost, plans[p].pop,
                                                   np.packbits(plans[p].mask, bitorder="little"))
                                  for p in inserted}
            snap["survivors"] = sorted(plans[p].nodes for p in inserted if p not in dominated)
            snap["removed"] = sorted(plans[p].nodes for p in dominated)
            snap["open"] = sorted(plans[p].nodes for p in P_open)
            snap["pairs"] = len(parents)
            # per formed pair: cost, pop (-2: past S_max), packed bits and the
            # packed bits whose decisions are flagged along the whole plan
            snap["pairs_all"] = {
                parents[q].nodes + (int(x[q]),): (
                    float(cost[q]), -2 if over[q] else int(mask[q].sum()),
                    np.packbits(mask[q], bitorder="little"),
                    np.packbits(flagged[q] if parents[q].fmask is None
                                else (parents[q].fmask | flagged[q]), bitorder="little"))
                for q in range(len(parents))}
            rounds.append(snap)
        i += 1
        B = sorted(p for p in P_open if plans[p].cost <= i * h)
        if time_budget is not None and time.perf_counter() - t_start > time_budget:
            stats["truncated"] = True
            break
    stats["final_i"] = i
    stats["stopped_at_goal"] = bool(P_open) and stop_now()
    return plans, P, stats, rounds


def goal_plans(plans, P, goal_nodes):
    """P_goal = {p in P(v) : v in X_goal} (Alg. 4 return)."""
    out = []
    for v in goal_nodes:
        out.extend(P.get(int(v), []))
    return [plans[p] for p in out]
