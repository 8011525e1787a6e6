"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bit-exact for particle bitmasks, graph adjacency, plan sets, Pareto fronts,
the selected plan and Monte Carlo counts; costs and durations within 1e-12
relative (both sides decide in FP64; the HIP particle test runs in FP32 with
an FP64 re-test inside a 2^-14 guard band, so its decisions equal the FP64
ones).  Flagged decisions (a particle within 1e-5 of a face) are counted and
printed; the tests require exact agreement regardless.
"""

import functools
import math

import numpy as np
import pytest

from oracle import dynamics, graph as ogr, pump as opump, select as osel
from paper_1607_06886_amd import _lib, scenes
from tests._gpu import (assert_bits_except_flagged, assert_table_is_fp32_of, gpu_plans,
                        oracle_mask_bool, oracle_run, planner_for, print_case, scene, small_spec,
                        unpack_mask)

pytestmark = pytest.mark.gpu

CFG = opump.Config()
REL = 1e-12


_scene = scene
_oracle = oracle_run


@pytest.mark.parametrize("N", [32, 64, 128, 256])
def test_deviation_table(N):
    print_case("deviation_table", N=N)
    sc = scenes.make_scene(small_spec(n=20, N=N, sigma=0.02), 11, M=64, S_max=300)
    pl = planner_for(sc)
    pl.setup(pl.scene_problem(sc))
    D = pl.deviation()
    A_cl, L, _ = dynamics.closed_loop(CFG.dt, sc.sigma, CFG.q_pos, CFG.q_vel, CFG.r_track)
    Dref = dynamics.deviation_table(A_cl, L, sc.noise, sc.S_max)
    print("  entries one FP32 ulp from the rounded FP64 value:", assert_table_is_fp32_of(D, Dref),
          flush=True)
    pl.close()


@pytest.mark.parametrize("kind,seed", [("cfg1", 0), ("boxes20", 1), ("indoor", 2)])
def test_graph(kind, seed):
    print_case("graph", kind=kind, seed=seed)
    sc = _scene(kind, seed)
    pl = planner_for(sc)
    pl.setup(pl.scene_problem(sc))
    g = pl.graph(sc.n + 1)
    V = np.concatenate([sc.x_init[None], sc.samples]).astype(np.float64)
    ref = ogr.build_graph(V, sc.obstacles, CFG.r_conn, CFG.r_steer)
    np.testing.assert_array_equal(g["valid"], ref["valid"])
    np.testing.assert_array_equal(g["row_ptr"], ref["row_ptr"])
    np.testing.assert_array_equal(g["col"], ref["col"])
    np.testing.assert_allclose(g["tau"], ref["tau"], rtol=REL)
    np.testing.assert_allclose(g["cost"], ref["cost"], rtol=REL)
    assert g["col"].shape[0] > 1000
    pl.close()


def _compare_end_state(pl, ref, sc):
    st = gpu_plans(pl)
    N = sc.N
    alive = st["state"] != 2
    gpu_P = {st["paths"][p]: p for p in np.nonzero(alive)[0]}
    ref_P = {ref["plans"][q].nodes: ref["plans"][q] for ids in ref["P"].values() for q in ids}
    assert set(gpu_P) == set(ref_P)
    flagged_diff = 0
    for nodes, p in gpu_P.items():
        rp = ref_P[nodes]
        assert abs(st["cost"][p] - rp.cost) <= REL * max(1.0, rp.cost)
        assert st["step"][p] == rp.step
        nf = assert_bits_except_flagged(unpack_mask(st["mask"][p], N), rp.mask, rp.fmask, nodes)
        assert st["pop"][p] == rp.pop or abs(int(st["pop"][p]) - rp.pop) <= nf
        flagged_diff += nf
    # plans created per group index
    by_round = {}
    for p in range(1, st["head"].shape[0]):
        by_round.setdefault(int(st["round"][p]), set()).add(st["paths"][p])
    for snap in ref["rounds"]:
        assert by_round.get(snap["i"], set()) == set(snap["survivors"]), snap["i"]
    print("  flagged particle bits that differ from the oracle:", flagged_diff, flush=True)
    return st


@pytest.mark.parametrize("preprune", [0, 1])
@pytest.mark.parametrize("kind,seed", [("cfg1", 0), ("cfg1", 3), ("boxes20", 1), ("n64", 4),
                                       ("n256", 5), ("indoor", 2)])
def test_plan_end_to_end(kind, seed, preprune):
    print_case("plan", kind=kind, seed=seed, preprune=preprune)
    sc = _scene(kind, seed)
    ref = _oracle(kind, seed)
    pl = planner_for(sc, preprune=preprune)
    res = pl.plan(pl.scene_problem(sc))
    print("  gpu", {k: res[k] for k in ("status", "partial_plans", "simulated", "preprune",
                                        "rounds", "flagged", "ms_total")},
          "oracle flagged", ref["stats"]["flagged_below_cut"], flush=True)
    assert res["partial_plans"] == ref["stats"]["partial_plans"]
    assert res["rounds"] == ref["stats"]["rounds"]
    assert res["final_i"] == ref["stats"]["final_i"]
    assert res["dropped_steps"] == ref["stats"]["dropped_steps"]
    if preprune == 0:
        assert res["inserted"] == ref["stats"]["inserted"]
        assert res["flagged"] == ref["stats"]["flagged_below_cut"]
    st = _compare_end_state(pl, ref, sc)
    assert res["status"] == ref["status"]
    assert res["n_goal_plans"] == len(ref["goal_plans"])
    ids, mc = pl.front()
    assert [st["paths"][p] for p in ids] == [p.nodes for p in ref["front"]]
    for m, cnt in ref["evals"].items():
        assert mc[m - 1] == cnt[0]
    if ref["status"] == 0:
        assert pl.path(res["best_plan"]) == ref["best"].nodes
        assert res["best_pop"] == ref["best"].pop
        assert abs(res["best_cost"] - ref["best"].cost) <= REL * ref["best"].cost
        k = ref["front"].index(ref["best"]) + 1
        assert res["best_mc_count"] == ref["evals"][k][0]
    pl.close()


def test_rounds_candidate_by_candidate():
    """Round by round with pre-pruning off: every formed pair's particle
    count (for a cut pair, a count at or past c_cut), and every kept pair's
    cost and bits, equal the oracle's."""
    print_case("rounds", kind="cfg1", seed=0)
    sc = _scene("cfg1", 0)
    ref = _oracle("cfg1", 0)
    c_cut = math.ceil(ref["alpha_max"] * sc.N)
    snaps = [s for s in ref["rounds"] if s["B"]]
    pl = planner_for(sc, preprune=0)
    pl.setup(pl.scene_problem(sc))
    pl.explore_begin()
    done = False
    r = 0
    flagged_diff = 0
    while not done:
        done = pl.explore_round()
        cand = pl.candidates()
        st = gpu_plans(pl)
        snap = snaps[r]
        assert cand["flag"].shape[0] == snap["pairs"]
        seen = set()
        for q in range(cand["flag"].shape[0]):
            nodes = st["paths"][cand["parent"][q]] + (int(cand["head"][q]),)
            seen.add(nodes)
            cost, pop, packed, fpacked = snap["pairs_all"][nodes]
            fl = oracle_mask_bool(fpacked, sc.N)
            got, nf = int(cand["pop"][q]), int(fl.sum())
            if pop >= c_cut:
                # a cut pair stops once its count reaches c_cut: any count
                # from there up to the full one
                assert c_cut - nf <= got <= pop + nf, (r, nodes, got, pop)
            else:
                assert got == pop or abs(got - pop) <= nf, (r, nodes)
            if cand["flag"][q]:
                assert abs(cand["cost"][q] - cost) <= REL * max(1.0, cost)
                flagged_diff += assert_bits_except_flagged(
                    unpack_mask(cand["mask"][q], sc.N), oracle_mask_bool(packed, sc.N), fl, nodes)
        assert seen == set(snap["pairs_all"])
        r += 1
    assert r == len(snaps)
    print("  flagged particle bits that differ from the oracle:", flagged_diff, flush=True)
    pl.close()


def test_mc_on_given_paths():
    print_case("mc_path")
    sc = _scene("cfg1", 0)
    ref = _oracle("cfg1", 0)
    pl = planner_for(sc)
    pl.setup(pl.scene_problem(sc))
    V = ref["V"]
    rng = np.random.default_rng(5)
    plans = [p for p in ref["plans"] if len(p.nodes) >= 3]
    picks = [plans[i] for i in rng.choice(len(plans), 12, replace=False)]
    for p in picks:
        c_ref = osel.mc_count(V, p.nodes, sc.obstacles, ref["A_cl"], ref["L"], sc.noise_mc,
                              CFG.r_steer, CFG.dt)
        assert pl.mc_path(p.nodes) == c_ref, p.nodes
    pl.close()


def test_mc_near_obstacle_counts():
    """A path that grazes a box: a substantial count, equal to the oracle's."""
    print_case("mc_near")
    samples = np.array([[0.9, 0.5, 0.5, 0.0, 0.0, 0.0]], np.float32)
    boxes = np.array([[0.45, 0.515, 0.0, 0.55, 0.8, 1.0]], np.float32)
    rng = np.random.default_rng(8)
    N, M, S = 32, 4000, 64
    noise = rng.standard_normal((S, 6, N), dtype=np.float32)
    noise_mc = rng.standard_normal((S, 6, M), dtype=np.float32)
    x0 = np.array([0.1, 0.5, 0.5, 0, 0, 0], np.float32)
    pl = _lib.Planner(n_particles=N, max_nodes=2, max_obstacles=1, max_steps=S, mc_particles=M,
                      cap_plans=1024, cap_pairs=1024, cap_edges=1024, r_conn=1.5)
    pl.setup(pl.problem(samples, boxes, x0, [0.8, 0.4, 0.4, 1, 0.6, 0.6], 0.05, 0.02, noise,
                        noise_mc))
    got = pl.mc_path([0, 1])
    V = np.concatenate([x0[None], samples]).astype(np.float64)
    A_cl, L, _ = dynamics.closed_loop(CFG.dt, float(np.float32(0.02)), CFG.q_pos, CFG.q_vel,
                                      CFG.r_track)
    want = osel.mc_count(V, (0, 1), boxes, A_cl, L, noise_mc, CFG.r_steer, CFG.dt)
    assert want > 100
    assert got == want
    pl.close()


def test_determinism():
    print_case("determinism")
    sc = _scene("boxes20", 1)
    pl = planner_for(sc)
    pr = pl.scene_problem(sc)
    a = pl.plan(pr)
    sa = pl.plans()
    b = pl.plan(pr)
    sb = pl.plans()
    for k in ("status", "partial_plans", "best_plan", "best_cost", "best_mc_count", "n_plans"):
        assert a[k] == b[k]
    for k in sa:
        np.testing.assert_array_equal(sa[k], sb[k])
    pl.close()


def test_device_inputs_match_host_inputs():
    print_case("device_inputs")
    sc = _scene("cfg1", 3)
    pl = planner_for(sc)
    a = pl.plan(pl.scene_problem(sc))
    sa = pl.plans()
    b = pl.plan(pl.scene_problem(sc, device=True))
    sb = pl.plans()
    assert a["best_plan"] == b["best_plan"] and a["best_cost"] == b["best_cost"]
    for k in sa:
        np.testing.assert_array_equal(sa[k], sb[k])
    pl.close()


@pytest.mark.parametrize("kind,seed", [("cfg1", 0), ("boxes20", 1), ("n64", 4), ("n256", 5),
                                       ("indoor", 2)])
def test_single_launch_explore_equals_per_phase_launches(kind, seed):
    """Explore as one cooperative launch and as one launch per phase build the
    same plan store, counters and selection (and both equal the oracle's)."""
    print_case("explore_modes", kind=kind, seed=seed)
    sc = _scene(kind, seed)
    ref = _oracle(kind, seed)
    pl = planner_for(sc)
    mode, blocks = pl.explore_mode()
    print("  single-launch workgroups", blocks, flush=True)
    assert mode == 2 and blocks > 0       # by graph size; these graphs take the single launch
    pr = pl.scene_problem(sc, device=True)
    pl.set_explore_mode(1)
    a = pl.plan(pr)
    sa = pl.plans()
    pl.set_explore_mode(0)
    b = pl.plan(pr)
    sb = pl.plans()
    for k in ("status", "partial_plans", "simulated", "preprune", "inserted", "survivors",
              "dropped_steps", "flagged", "rounds", "final_i", "n_plans", "best_plan",
              "best_cost", "best_mc_count", "n_front", "n_goal_plans", "sim_waypoints",
              "sim_box_tests"):
        assert a[k] == b[k], k
    for k in sa:
        np.testing.assert_array_equal(sa[k], sb[k])
    assert a["partial_plans"] == ref["stats"]["partial_plans"]
    assert a["rounds"] == ref["stats"]["rounds"]
    pl.close()


HSMC_SCENES = [("cfg1", 0), ("n64", 4)]


@functools.lru_cache(maxsize=None)
def _oracle_hsmc(kind, seed):
    import dataclasses
    return opump.run(_scene(kind, seed), dataclasses.replace(CFG, cp_model="hsmc"), record=True)


@pytest.mark.parametrize("mode,preprune", [(1, 0), (0, 1)])
@pytest.mark.parametrize("kind,seed", HSMC_SCENES)
def test_hsmc_plan_end_to_end(kind, seed, mode, preprune):
    """Half-space exploration model: plan sets, counters, the front and p*
    equal the oracle's, in both Explore modes (flag counts with pre-pruning
    off, since pre-pruned pairs are never simulated)."""
    print_case("hsmc_plan", kind=kind, seed=seed, mode=mode, preprune=preprune)
    sc = _scene(kind, seed)
    ref = _oracle_hsmc(kind, seed)
    pl = planner_for(sc, cp_model=1, preprune=preprune)
    pl.set_explore_mode(mode)
    res = pl.plan(pl.scene_problem(sc))
    print("  gpu", {k: res[k] for k in ("status", "partial_plans", "simulated", "rounds",
                                        "flagged", "sim_box_tests")},
          "oracle flagged", ref["stats"]["flagged_below_cut"], flush=True)
    assert res["partial_plans"] == ref["stats"]["partial_plans"]
    assert res["rounds"] == ref["stats"]["rounds"]
    assert res["final_i"] == ref["stats"]["final_i"]
    if preprune == 0:
        assert res["flagged"] == ref["stats"]["flagged_below_cut"]
        assert res["inserted"] == ref["stats"]["inserted"]
    _compare_end_state(pl, ref, sc)
    assert res["status"] == ref["status"]
    assert res["n_goal_plans"] == len(ref["goal_plans"])
    if ref["status"] == 0:
        assert pl.path(res["best_plan"]) == ref["best"].nodes
        assert res["best_pop"] == ref["best"].pop
        k = ref["front"].index(ref["best"]) + 1
        assert res["best_mc_count"] == ref["evals"][k][0]
    pl.close()


def test_single_launch_timeout_falls_back_to_per_phase():
    """A single-launch barrier wait that runs out of patience (forced from the
    host with a one-tick patience) makes every workgroup leave the launch;
    pump_plan then redoes Explore per phase and returns the same result."""
    print_case("explore_fallback", kind="boxes20", seed=1)
    sc = _scene("boxes20", 1)
    pl = planner_for(sc)
    pr = pl.scene_problem(sc, device=True)
    a = pl.plan(pr)
    sa = pl.plans()
    assert pl.explore_fallbacks() == 0
    pl.set_barrier_patience(1e-5)      # one tick of the 100 MHz counter
    b = pl.plan(pr)
    sb = pl.plans()
    print("  fallbacks", pl.explore_fallbacks(), flush=True)
    assert pl.explore_fallbacks() == 1
    for k in ("status", "partial_plans", "inserted", "rounds", "final_i", "n_plans", "best_plan",
              "best_cost", "best_mc_count", "n_front"):
        assert a[k] == b[k], k
    for k in sa:
        np.testing.assert_array_equal(sa[k], sb[k])
    # the step-by-step entry points fall back the same way
    pl.setup(pr)
    pl.explore_begin()
    pl.explore_run()
    assert pl.explore_fallbacks() == 2
    c = pl.select()
    assert c["best_plan"] == a["best_plan"] and c["partial_plans"] == a["partial_plans"]
    pl.set_barrier_patience(4000.0)
    d = pl.plan(pr)
    assert pl.explore_fallbacks() == 2 and d["best_plan"] == a["best_plan"]
    pl.close()
