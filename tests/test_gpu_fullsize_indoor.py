"""The indoor workload at its full size (Sec. V-C's indoor experiment: a 4x4
room grid of 60 thin walls with doorways 0.08 wide, 20,000 samples, N = 256,
sigma 0.02, alpha 0.01, M = 10^4, S_max = 512), with the bench's capacities
and device-resident inputs, checked on outputs the oracle can compute one by
one: sampled graph rows (node 0 among them), the whole deviation table,
sampled plan records re-simulated edge by edge, the dominance invariant,
the selection order of the front and the certification count of every
front plan (the query's outcome: on this map no front plan certifies at
alpha = 0.01, which the oracle's counts confirm)."""

import numpy as np
import pytest

from oracle import dynamics, explore as oex, graph as ogr, pump as opump, select as osel
from paper_1607_06886_amd import _lib, scenes
from tests._gpu import (assert_bits_except_flagged, assert_table_is_fp32_of, gpu_plans,
                        print_case, unpack_mask)
from tests.test_gpu_fullsize import _resimulate

pytestmark = pytest.mark.gpu

CFG = opump.Config()
REL = 1e-12


@pytest.fixture(scope="module")
def run():
    import torch
    sc = scenes.make_scene("cfg3", scenes.workload_seed(3, 0), M=10_000, S_max=512)
    print_case("fullsize_indoor", n=sc.n, n_obs=sc.n_obs, N=sc.N, M=sc.M)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    pl = _lib.Planner(n_particles=sc.N, max_nodes=sc.n + 1, max_obstacles=sc.n_obs,
                      max_steps=sc.S_max, mc_particles=sc.M, cap_plans=1 << 22,
                      cap_pairs=1 << 25, cap_edges=1 << 25)
    pr = pl.problem(dev(sc.samples), dev(sc.obstacles), sc.x_init, sc.goal, sc.alpha, sc.sigma,
                    dev(sc.noise), dev(sc.noise_mc))
    res = pl.plan(pr)
    ids, mc = pl.front()
    print("  gpu", {k: res[k] for k in ("status", "partial_plans", "rounds", "n_front",
                                        "n_edges", "flagged", "ms_total")}, flush=True)
    out = dict(sc=sc, res=res, graph=pl.graph(sc.n + 1), D=pl.deviation(), st=gpu_plans(pl),
               front=(ids, mc))
    pl.close()
    return out


def test_sampled_graph_rows(run):
    sc, g = run["sc"], run["graph"]
    V = np.concatenate([sc.x_init[None], sc.samples]).astype(np.float64)
    valid = ~ogr.points_in_boxes(V[:, :3], sc.obstacles)
    np.testing.assert_array_equal(g["valid"].astype(bool), valid)
    rows = [0] + list(np.random.default_rng(4).choice(np.arange(1, sc.n + 1), 7, replace=False))
    src, dst, tau, cost = ogr.graph_rows(V, valid, sc.obstacles, CFG.r_conn, CFG.r_steer, rows)
    for v in rows:
        a, b = g["row_ptr"][v], g["row_ptr"][v + 1]
        sel = src == v
        np.testing.assert_array_equal(g["col"][a:b], dst[sel])
        np.testing.assert_allclose(g["tau"][a:b], tau[sel], rtol=REL)
        np.testing.assert_allclose(g["cost"][a:b], cost[sel], rtol=REL)
    assert sum(int((src == v).sum()) for v in rows) > 500


def test_deviation_table(run):
    sc, D = run["sc"], run["D"]
    A_cl, L, _ = dynamics.closed_loop(CFG.dt, sc.sigma, CFG.q_pos, CFG.q_vel, CFG.r_track)
    Dref = dynamics.deviation_table(A_cl, L, sc.noise, sc.S_max)
    print("  entries one FP32 ulp from the rounded FP64 value:",
          assert_table_is_fp32_of(D, Dref, tol=1e-6), flush=True)


def test_sampled_plans_resimulated(run):
    sc, st = run["sc"], run["st"]
    A_cl, L, _ = dynamics.closed_loop(CFG.dt, sc.sigma, CFG.q_pos, CFG.q_vel, CFG.r_track)
    D = dynamics.deviation_table(A_cl, L, sc.noise, sc.S_max)
    alive = np.nonzero(st["state"] != 2)[0]
    assert alive.shape[0] > 1000
    picks = np.random.default_rng(5).choice(alive[alive > 0], 120, replace=False)
    flagged, flagged_diff = 0, 0
    for pid in picks:
        nodes = st["paths"][pid]
        ref = _resimulate(sc, nodes, D)
        assert st["step"][pid] == ref.step, pid
        assert abs(st["cost"][pid] - ref.cost) <= REL * max(1.0, ref.cost), pid
        nf = assert_bits_except_flagged(unpack_mask(st["mask"][pid], sc.N), ref.mask, ref.fmask,
                                        nodes)
        assert st["pop"][pid] == ref.pop or abs(int(st["pop"][pid]) - ref.pop) <= nf
        flagged += int(ref.fmask.sum())
        flagged_diff += nf
    print("  flagged particle bits on the sampled plans:", flagged, "differing:", flagged_diff,
          flush=True)


def test_no_open_plan_dominated_at_its_head(run):
    st = run["st"]
    alive = np.nonzero(st["state"] != 2)[0]
    heads = st["head"][alive]
    for h in np.random.default_rng(6).choice(np.unique(heads), 300, replace=False):
        ids = alive[heads == h]
        c, k = st["cost"][ids], st["pop"][ids]
        dom = (c[:, None] > c[None, :]) & (k[:, None] >= k[None, :])
        open_ = st["state"][ids] == 0
        assert not (dom.any(axis=1) & open_).any(), h


def test_front_order_and_certification_counts(run):
    """The front in selection order (cp_hat ascending, cost descending), no
    member dominated by another goal plan, and every member's MC count equal
    to the oracle's segment-swept count on the same certification particles;
    the outcome follows Alg. 5 on those counts."""
    sc, res, st = run["sc"], run["res"], run["st"]
    ids, mc = run["front"]
    assert len(ids) == res["n_front"] > 0
    pops, costs = st["pop"][ids], st["cost"][ids]
    assert all((pops[i], -costs[i]) < (pops[i + 1], -costs[i + 1]) for i in range(len(ids) - 1))
    V = np.concatenate([sc.x_init[None], sc.samples]).astype(np.float64)
    A_cl, L, _ = dynamics.closed_loop(CFG.dt, sc.sigma, CFG.q_pos, CFG.q_vel, CFG.r_track)
    counts = [osel.mc_count(V, st["paths"][p], sc.obstacles, A_cl, L, sc.noise_mc, CFG.r_steer,
                            CFG.dt) for p in ids]
    print("  front pops", pops.tolist(), "MC counts", counts, flush=True)
    assert list(mc) == counts
    # Alg. 5 on the oracle's counts gives the query's outcome
    plans = [oex.Plan(nodes=st["paths"][p], cost=float(st["cost"][p]), step=0,
                      mask=np.arange(sc.N) < st["pop"][p], parent=-1) for p in ids]
    count_of = {pl.nodes: c for pl, c in zip(plans, counts)}
    best, front, _ = osel.plan_selection(plans, sc.alpha,
                                         lambda pl: (count_of[pl.nodes], count_of[pl.nodes] / sc.M))
    assert [f.nodes for f in front] == [pl.nodes for pl in plans]
    if best is None:
        assert res["status"] == 1
    else:
        assert res["status"] == 0 and res["best"] == front.index(best)


def test_front_is_the_pareto_front_of_the_goal_plans(run):
    """P_goal and its Pareto front recomputed on the host from the plan
    store: the goal plans are the plans not removed whose head is a goal
    sample, and the front keeps those no other goal plan dominates (strictly
    cheaper with cp_hat no larger).  At this size (2^14 plans or more) the
    library gathers P_goal over the whole device; the smaller queries of the
    other tests take the one-workgroup gather."""
    sc, res, st = run["sc"], run["res"], run["st"]
    ids, _ = run["front"]
    n_plans = len(st["cost"])
    assert n_plans == res["n_plans"] >= 1 << 14
    V = np.concatenate([sc.x_init[None], sc.samples]).astype(np.float64)
    gl = sc.goal.astype(np.float64)
    valid = ~ogr.points_in_boxes(V[:, :3], sc.obstacles)
    is_goal = np.all((V[:, :3] >= gl[:3]) & (V[:, :3] <= gl[3:]), axis=1) & valid
    goal = np.nonzero((st["state"] != 2) & is_goal[st["head"]])[0]
    assert res["n_goal_plans"] == len(goal)
    c, k = st["cost"][goal], st["pop"][goal]
    dominated = np.array([np.any((c < c[i]) & (k <= k[i])) for i in range(len(goal))])
    assert sorted(goal[~dominated].tolist()) == sorted(int(i) for i in ids)

