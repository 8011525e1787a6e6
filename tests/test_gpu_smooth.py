"""Smooth(p*, alpha) (Alg. 5's last step) on the HIP path, through the C ABI,
against the oracle: the blend weight the bisection settles on, the cost, the
certification count, the tracking steps and the waypoints, for the
single-query path (both tracking controllers) and the batched engine."""

import numpy as np
import pytest

from oracle import pump as opump, select as osel
from paper_1607_06886_amd import _lib
from tests._gpu import SIGMA_MEAS, planner_for, print_case, scene

pytestmark = pytest.mark.gpu

REL = 1e-12
# (kind, seed): beta = 1 at once for cfg1/0 and cfg1/3; the bisection runs
# for n64/0, n64/4, cfg1/1 and cfg1/6
CASES = [("cfg1", 0), ("cfg1", 1), ("cfg1", 6), ("n64", 0), ("n64", 4), ("cfg1", 3)]


def _check(res, pl, ref, sc):
    s = ref["smooth"]
    print("  gpu", {k: res[k] for k in ("status", "smooth_beta", "smooth_cost", "smooth_mc_count",
                                        "smooth_steps")},
          "oracle", {k: s[k] for k in ("beta", "cost", "count", "steps")}, flush=True)
    assert res["status"] == ref["status"] == 0
    assert pl.path(res["best_plan"]) == ref["best"].nodes
    assert res["smooth_beta"] == s["beta"]
    assert abs(res["smooth_cost"] - s["cost"]) <= REL * s["cost"]
    assert res["smooth_mc_count"] == s["count"]
    assert res["smooth_steps"] == s["steps"]
    assert res["smooth_cost"] <= res["best_cost"]
    W = pl.smooth_path()
    assert W.shape == (s["steps"] + 1, 3)
    if s["beta"] > 0:
        np.testing.assert_allclose(W, s["W"], rtol=0, atol=1e-12)
    else:
        Wp = osel.plan_waypoints(ref["V"], ref["best"].nodes, opump.Config().r_steer,
                                 opump.Config().dt)
        np.testing.assert_allclose(W, Wp, rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind,seed", CASES)
def test_smooth_matches_oracle(kind, seed):
    print_case("smooth", kind=kind, seed=seed)
    sc = scene(kind, seed)
    ref = opump.run(sc, opump.Config(smooth=True))
    pl = planner_for(sc, smooth=1)
    res = pl.plan(pl.scene_problem(sc))
    _check(res, pl, ref, sc)
    pl.close()


def test_smooth_with_lqg_tracking_matches_oracle():
    print_case("smooth_lqg", kind="n64", seed=4)
    sc = scene("n64", 4, SIGMA_MEAS)
    ref = opump.run(sc, opump.Config(smooth=True, estimator="lqg"))
    pl = planner_for(sc, smooth=1, estimator=1)
    res = pl.plan(pl.scene_problem(sc))
    _check(res, pl, ref, sc)
    pl.close()


def test_smooth_off_is_the_identity():
    print_case("smooth_off", kind="n64", seed=4)
    sc = scene("n64", 4)
    pl = planner_for(sc)
    res = pl.plan(pl.scene_problem(sc))
    assert res["status"] == 0
    assert res["smooth_beta"] == 0.0 and res["smooth_cost"] == res["best_cost"]
    assert res["smooth_mc_count"] == res["best_mc_count"]
    nodes = pl.path(res["best_plan"])
    V = np.concatenate([sc.x_init[None], sc.samples]).astype(np.float64)
    Wp = osel.plan_waypoints(V, nodes, opump.Config().r_steer, opump.Config().dt)
    assert res["smooth_steps"] == Wp.shape[0] - 1
    np.testing.assert_allclose(pl.smooth_path(), Wp, rtol=0, atol=1e-12)
    pl.close()


def test_smooth_without_a_certified_plan():
    """No plan certified: status 1, the smoothing fields stay zero and the
    path reader reports a state error."""
    print_case("smooth_infeasible", kind="indoor", seed=2)
    sc = scene("indoor", 2)
    pl = planner_for(sc, smooth=1)
    res = pl.plan(pl.scene_problem(sc))
    assert res["status"] == _lib.PUMP_INFEASIBLE
    assert res["smooth_beta"] == 0.0 and res["smooth_steps"] == 0
    with pytest.raises(_lib.PumpError) as e:
        pl.smooth_path()
    assert e.value.code == _lib.PUMP_E_STATE
    pl.close()


def test_batched_smooth_equals_single_query_path():
    import torch
    kinds = [("n64", 4), ("cfg1", 0), ("cfg1", 6), ("indoor", 2)]
    print_case("smooth_batch", kinds=kinds)
    scs = [scene(k, s) for k, s in kinds]
    single = []
    for sc in scs:
        pl = planner_for(sc, smooth=1)
        single.append(pl.plan(pl.scene_problem(sc, device=True)))
        pl.close()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    qs = [(t(s.samples), t(np.asarray(s.obstacles, np.float32).reshape(-1, 6)), s.x_init, s.goal,
           s.alpha, s.sigma, t(s.noise), t(s.noise_mc)) for s in scs]
    b = _lib.Batch(len(scs), n_particles=max(s.N for s in scs),
                   max_nodes=max(s.n for s in scs) + 1,
                   max_obstacles=max(s.n_obs for s in scs), max_steps=scs[0].S_max,
                   mc_particles=scs[0].M, cap_plans=1 << 20, cap_pairs=1 << 22,
                   cap_edges=1 << 24, smooth=1)
    for tuning in (dict(team_scale=0, use_graph=1), dict(team_scale=8, use_graph=0)):
        res = b.plan(qs, tuning=tuning)
        for i in range(len(scs)):
            for k in ("status", "best_plan", "best_cost", "best_mc_count", "smooth_beta",
                      "smooth_cost", "smooth_mc_count", "smooth_steps"):
                assert res[i][k] == single[i][k], (tuning, i, k)
    b.close()
    assert single[0]["smooth_beta"] == 0.20703125
