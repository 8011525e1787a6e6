"""BuildGraph over a cached roadmap (pump_roadmap_create / pump_set_roadmap):
the graph, and so every result, equals the one built from scratch; one
roadmap serves several obstacle sets; mismatched inputs are rejected."""

import dataclasses

import numpy as np
import pytest

from oracle import graph as ogr, pump as opump
from paper_1607_06886_amd import _lib, scenes
from tests._gpu import planner_for, print_case, scene

pytestmark = pytest.mark.gpu

SAME = ("status", "n_goal_plans", "n_front", "best_plan", "best_pop", "best_mc_count",
        "best_cost", "partial_plans", "simulated", "rounds", "final_i", "n_edges", "n_plans")


def _graph_and_result(sc, rm=None):
    pl = planner_for(sc)
    if rm is not None:
        pl.set_roadmap(rm)
    res = pl.plan(pl.scene_problem(sc))
    g = pl.graph(sc.n + 1)
    path = pl.path(res["best_plan"]) if res["status"] == 0 else None
    pl.close()
    return g, res, path


@pytest.mark.parametrize("kind,seed", [("cfg1", 0), ("boxes20", 1), ("indoor", 2)])
def test_roadmap_graph_equals_scratch_graph(kind, seed):
    print_case("roadmap", kind=kind, seed=seed)
    sc = scene(kind, seed)
    rm = _lib.Roadmap(sc.samples, max_nodes=sc.n + 1, cap_edges=1 << 24)
    info = rm.info()
    g0, r0, p0 = _graph_and_result(sc)
    g1, r1, p1 = _graph_and_result(sc, rm)
    print("  roadmap", info, "edges", r0["n_edges"], flush=True)
    assert info["n"] == sc.n and info["n_edges"] >= r0["n_edges"] - 2 * sc.n
    for k in ("valid", "row_ptr", "col", "tau", "cost"):
        np.testing.assert_array_equal(g1[k], g0[k])
    for k in SAME:
        assert r1[k] == r0[k], k
    assert p1 == p0
    rm.close()


def test_one_roadmap_for_several_obstacle_sets():
    print_case("roadmap_maps")
    base = scenes.make_scene(dict(n=500, n_obs=10, side=(0.05, 0.25), N=64, sigma=0.02,
                                  alpha=0.05, indoor=False), 1200, M=2000, S_max=256)
    rm = _lib.Roadmap(base.samples, max_nodes=base.n + 1, cap_edges=1 << 24)
    rng = np.random.default_rng(5)
    for m in range(3):
        lo = rng.uniform(0.2, 0.7, (12, 3))
        boxes = np.concatenate([lo, lo + rng.uniform(0.05, 0.2, (12, 3))], 1).astype(np.float32)
        start = np.array([0.05 + 0.03 * m, 0.1, 0.1, 0, 0, 0], np.float32)
        sc = dataclasses.replace(base, obstacles=boxes, x_init=start)
        g0, r0, p0 = _graph_and_result(sc)
        g1, r1, p1 = _graph_and_result(sc, rm)
        for k in ("row_ptr", "col", "tau", "cost"):
            np.testing.assert_array_equal(g1[k], g0[k])
        for k in SAME:
            assert r1[k] == r0[k], (m, k)
        if m == 0:
            V = np.concatenate([sc.x_init[None], sc.samples]).astype(np.float64)
            ref = ogr.build_graph(V, sc.obstacles, opump.Config().r_conn, opump.Config().r_steer)
            np.testing.assert_array_equal(g1["col"], ref["col"])
            np.testing.assert_array_equal(g1["row_ptr"], ref["row_ptr"])
    rm.close()


def test_roadmap_mismatches_are_rejected():
    print_case("roadmap_args")
    sc = scene("cfg1", 1)
    rm = _lib.Roadmap(sc.samples, max_nodes=sc.n + 1)
    pl = planner_for(sc)
    pl.set_roadmap(rm)
    other = sc.samples.copy()
    other[7, 2] += np.float32(1e-3)
    pr = pl.problem(other, sc.obstacles, sc.x_init, sc.goal, sc.alpha, sc.sigma, sc.noise,
                    sc.noise_mc)
    with pytest.raises(_lib.PumpError) as e:
        pl.plan(pr)
    assert e.value.code == _lib.PUMP_E_ARG
    pr = pl.problem(sc.samples[:-1], sc.obstacles, sc.x_init, sc.goal, sc.alpha, sc.sigma,
                    sc.noise, sc.noise_mc)
    with pytest.raises(_lib.PumpError):
        pl.plan(pr)
    # the right samples work after the failures, and None goes back to scratch
    assert pl.plan(pl.scene_problem(sc))["status"] in (0, 1, 2)
    pl.set_roadmap(None)
    pl.close()
    pl2 = planner_for(sc, r_conn=0.9)
    with pytest.raises(_lib.PumpError):
        pl2.set_roadmap(rm)
    pl2.close()
    rm.close()


def test_batched_queries_with_roadmaps():
    """The batched engine with per-query roadmaps (two queries share one,
    one has none, one has samples that differ from its roadmap's) equals the
    scratch build query by query."""
    import torch
    print_case("roadmap_batch")
    base = scene("n64", 4)
    other = scene("cfg1", 0)
    rng = np.random.default_rng(9)
    lo = rng.uniform(0.2, 0.7, (6, 3))
    boxes2 = np.concatenate([lo, lo + 0.1], 1).astype(np.float32)
    scs = [base, dataclasses.replace(base, obstacles=boxes2), other, base]
    rm_a = _lib.Roadmap(base.samples, max_nodes=base.n + 1, cap_edges=1 << 24)
    rm_b = _lib.Roadmap(other.samples, max_nodes=other.n + 1, cap_edges=1 << 24)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    qs = [(t(s.samples), t(np.asarray(s.obstacles, np.float32).reshape(-1, 6)), s.x_init, s.goal,
           s.alpha, s.sigma, t(s.noise), t(s.noise_mc)) for s in scs]
    bad = list(qs[3])
    smp = base.samples.copy()
    smp[3, 0] += np.float32(1e-3)
    bad[0] = t(smp)
    qs[3] = tuple(bad)
    b = _lib.Batch(len(scs), n_particles=max(s.N for s in scs),
                   max_nodes=max(s.n for s in scs) + 1,
                   max_obstacles=max(s.n_obs for s in scs), max_steps=base.S_max,
                   mc_particles=base.M, cap_plans=1 << 20, cap_pairs=1 << 22, cap_edges=1 << 24)
    b.set_roadmaps([rm_a, rm_a, None, rm_a])
    res = b.plan(qs, raise_on_error=False)
    for i in range(3):
        _, ref, path = _graph_and_result(scs[i])
        for k in SAME:
            assert res[i][k] == ref[k], (i, k)
        if path is not None:
            assert b.path(i, res[i]["best_plan"]) == path
    assert res[3]["status"] == _lib.PUMP_E_ARG
    b.set_roadmaps([None, None, rm_b])
    res2 = b.plan(qs[:3])
    for i in range(3):
        for k in SAME:
            assert res2[i][k] == res[i][k], (i, k)
    b.close()
    rm_a.close()
    rm_b.close()
