"""The batched engine (many queries of uneven size, one graph launch) through
the C ABI: per-query results equal the oracle's, and equal the single-query
path's bit for bit under every persistent-kernel shape."""

import dataclasses
import json
import os

import numpy as np
import pytest

from paper_1607_06886_amd import _lib, scenes
from tests._gpu import oracle_run, opump, planner_for, print_case, scene, small_spec

pytestmark = pytest.mark.gpu

REL = 1e-12
KINDS = [("cfg1", 0), ("cfg1", 3), ("boxes20", 1), ("n64", 4), ("n256", 5), ("indoor", 2)]
# fields that must agree exactly between the batched and single-query paths
SAME = ("status", "n_goal_plans", "n_front", "best", "best_plan", "best_pop", "best_mc_count",
        "best_len", "best_cost", "best_cp_mc", "partial_plans", "simulated", "preprune",
        "inserted", "survivors", "dropped_steps", "flagged", "rounds", "final_i", "n_plans",
        "n_edges", "c_cut", "c_min", "sim_waypoints", "sim_box_tests")


def _dev(sc):
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return (t(sc.samples), t(np.asarray(sc.obstacles, np.float32).reshape(-1, 6)), sc.x_init,
            sc.goal, sc.alpha, sc.sigma, t(sc.noise), t(sc.noise_mc))


def _batch_for(scs, **over):
    kw = dict(n_particles=max(s.N for s in scs), max_nodes=max(s.n for s in scs) + 1,
              max_obstacles=max(max(s.n_obs for s in scs), 1), max_steps=scs[0].S_max,
              mc_particles=scs[0].M, cap_plans=1 << 20, cap_pairs=1 << 22, cap_edges=1 << 24)
    kw.update(over)
    return _lib.Batch(len(scs), **kw)


def _single(sc, **over):
    pl = planner_for(sc, **over)
    res = pl.plan(pl.scene_problem(sc, device=True))
    path = pl.path(res["best_plan"]) if res["status"] == 0 else None
    pl.close()
    return res, path


def _edge_scenes():
    """Degenerate queries: start inside the goal box, a goal no sample lies in,
    no obstacles, and a start inside an obstacle (an argument error)."""
    base = scene("cfg1", 1)
    in_goal = dataclasses.replace(base, goal=np.array([0.05, 0.05, 0.05, 0.15, 0.15, 0.15],
                                                      np.float32))
    far_goal = dataclasses.replace(base, goal=np.array([0.995, 0.995, 0.995, 1.0, 1.0, 1.0],
                                                       np.float32))
    free = dataclasses.replace(scene("cfg1", 2), obstacles=np.zeros((0, 6), np.float32))
    blocked = dataclasses.replace(scene("cfg1", 4), obstacles=np.concatenate(
        [scene("cfg1", 4).obstacles, np.array([[0.05, 0.05, 0.05, 0.15, 0.15, 0.15]],
                                              np.float32)]))
    return [("in_goal", in_goal), ("far_goal", far_goal), ("no_obstacles", free),
            ("start_blocked", blocked)]


def test_batch_matches_oracle():
    print_case("batch_oracle", kinds=KINDS)
    scs = [scene(k, s) for k, s in KINDS]
    b = _batch_for(scs)
    res = b.plan([_dev(s) for s in scs])
    for i, (kind, seed) in enumerate(KINDS):
        ref = oracle_run(kind, seed)
        r = res[i]
        print("  ", kind, seed, {k: r[k] for k in ("status", "partial_plans", "rounds")},
              flush=True)
        assert r["status"] == ref["status"]
        assert r["partial_plans"] == ref["stats"]["partial_plans"]
        assert r["rounds"] == ref["stats"]["rounds"]
        assert r["final_i"] == ref["stats"]["final_i"]
        assert r["dropped_steps"] == ref["stats"]["dropped_steps"]
        assert r["n_goal_plans"] == len(ref["goal_plans"])
        assert r["n_front"] == len(ref["front"])
        if ref["status"] == 0:
            assert b.path(i, r["best_plan"]) == ref["best"].nodes
            assert r["best_pop"] == ref["best"].pop
            assert abs(r["best_cost"] - ref["best"].cost) <= REL * ref["best"].cost
            k = ref["front"].index(ref["best"]) + 1
            assert r["best_mc_count"] == ref["evals"][k][0]
    b.close()


# shapes of the persistent kernel, including teams of several workgroups per
# query (team_scale > 0) and scales that give even the small queries teams
TUNINGS = [dict(explore_threads=t, blocks_per_cu=c, order=o, use_graph=g, team_scale=k)
           for t, c, o, g, k in [(256, 2, 1, 1, 0), (256, 1, 0, 1, 0), (256, 4, 1, 1, 4),
                                 (256, 1, 0, 0, 4), (256, 8, 1, 0, 8), (256, 2, 1, 1, 64),
                                 (256, 2, 1, 1, 256)]]


def test_batch_equals_single_query_path_under_every_shape():
    print_case("batch_vs_single", kinds=KINDS, tunings=len(TUNINGS))
    scs = [scene(k, s) for k, s in KINDS]
    single = [_single(s) for s in scs]
    b = _batch_for(scs)
    qs = [_dev(s) for s in scs]
    for t in TUNINGS:
        res = b.plan(qs, tuning=t)
        for i in range(len(scs)):
            for k in SAME:
                assert res[i][k] == single[i][0][k], (t, i, k)
            if single[i][1] is not None:
                assert b.path(i, res[i]["best_plan"]) == single[i][1]
    b.close()


def test_batch_uneven_random_queries():
    """Uneven sizes: samples, particles, obstacles and alpha differ per query."""
    rng = np.random.default_rng(31)
    scs = []
    for q in range(10):
        spec = small_spec(n=int(rng.integers(100, 700)), N=int(rng.choice([64, 128, 256])),
                          sigma=0.02, alpha=float(rng.choice([0.01, 0.05])),
                          n_obs=int(rng.integers(5, 61)), side=(0.05, 0.2))
        scs.append(scenes.make_scene(spec, 4000 + q, M=2000, S_max=256))
    print_case("batch_uneven", n=[s.n for s in scs], N=[s.N for s in scs],
               n_obs=[s.n_obs for s in scs])
    b = _batch_for(scs)
    res = b.plan([_dev(s) for s in scs])
    for i, sc in enumerate(scs):
        ref, path = _single(sc)
        for k in SAME:
            assert res[i][k] == ref[k], (i, k)
        if path is not None:
            assert b.path(i, res[i]["best_plan"]) == path
    # the oracle on the two smallest queries
    for i in np.argsort([s.n * s.N for s in scs])[:2]:
        o = opump.run(scs[i], opump.Config(), record=False)
        assert res[i]["status"] == o["status"]
        assert res[i]["partial_plans"] == o["stats"]["partial_plans"]
        if o["status"] == 0:
            assert b.path(int(i), res[i]["best_plan"]) == o["best"].nodes
    b.close()


def test_batch_degenerate_queries():
    cases = _edge_scenes()
    print_case("batch_degenerate", cases=[c for c, _ in cases])
    scs = [s for _, s in cases]
    b = _batch_for(scs)
    res = b.plan([_dev(s) for s in scs], raise_on_error=False)
    got = {name: res[i] for i, (name, _) in enumerate(cases)}
    assert got["start_blocked"]["status"] == _lib.PUMP_E_ARG
    for name, sc in cases:
        if name == "start_blocked":
            continue
        ref, path = _single(sc)
        o = opump.run(sc, opump.Config(), record=False)
        assert got[name]["status"] == ref["status"] == o["status"], name
        for k in SAME:
            assert got[name][k] == ref[k], (name, k)
        if path is not None:
            i = [c for c, _ in cases].index(name)
            assert b.path(i, got[name]["best_plan"]) == path == o["best"].nodes
    assert got["in_goal"]["status"] == 0 and got["in_goal"]["best_len"] == 1
    assert got["far_goal"]["status"] == _lib.PUMP_NO_GOAL_PLAN
    b.close()


def test_batch_repeat_and_smaller_second_call():
    """Same batch twice gives identical results; a shorter batch on the same
    workspaces equals its own first results."""
    print_case("batch_repeat")
    scs = [scene(k, s) for k, s in KINDS]
    b = _batch_for(scs)
    qs = [_dev(s) for s in scs]
    r1 = b.plan(qs)
    r2 = b.plan(qs)
    r3 = b.plan(qs[3:])
    for i in range(len(scs)):
        for k in SAME:
            assert r1[i][k] == r2[i][k]
    for i in range(3, len(scs)):
        for k in SAME:
            assert r3[i - 3][k] == r1[i][k]
    b.close()


def test_autotuner_picks_a_shape_and_writes_json(tmp_path):
    print_case("autotune")
    scs = [scene(k, s) for k, s in KINDS[:4]]
    b = _batch_for(scs)
    out = os.path.join(str(tmp_path), "tune.json")
    best, ms = b.tune([_dev(s) for s in scs], json_path=out)
    rec = json.load(open(out))
    assert len(rec["candidates"]) == 9
    assert best["explore_threads"] == 256 and ms > 0
    assert rec["best"]["threads"] == best["explore_threads"]
    b.close()


def test_batch_hsmc_equals_single_query_path():
    """The half-space exploration model in the batched engine (teams and one
    workgroup per query) equals the single-query path."""
    kinds = [("cfg1", 0), ("n64", 4), ("cfg1", 3)]
    print_case("batch_hsmc", kinds=kinds)
    scs = [scene(k, s) for k, s in kinds]
    single = [_single(s, cp_model=1) for s in scs]
    b = _batch_for(scs, cp_model=1)
    qs = [_dev(s) for s in scs]
    for t in (TUNINGS[0], TUNINGS[2]):
        res = b.plan(qs, tuning=t)
        for i in range(len(scs)):
            for k in SAME:
                assert res[i][k] == single[i][0][k], (t, i, k)
    b.close()
