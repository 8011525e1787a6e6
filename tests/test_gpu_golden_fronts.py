"""Whole-query parity at full size against stored oracle results.

tests/golden/front_*.json are written by tests/golden/make_fronts.py, which
runs only the CPU oracle on the seeded inputs: the 4000-sample, 20-box,
128-particle workload (single queries through pump_plan, with the bench's
capacities and device-resident inputs) and large queries of the uneven
256-query batch (through the batched engine, in one batch together).  The
Pareto front of P_goal in selection order (node sequences, costs, cp_hat
counts), the certification count of every front plan and the selected plan
must equal the oracle's; costs within 1e-12 relative.  The number of
(plan, particle) decisions the oracle flags (within 1e-5 of a face) is
printed: a run whose front plans carry no flagged bit must match exactly, and
the fixtures record the flagged bits of each front plan."""

import glob
import json
import os

import numpy as np
import pytest

from paper_1607_06886_amd import _lib, scenes
from tests._gpu import gpu_plans, print_case

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
REL = 1e-12


def _fixtures(kind):
    out = []
    for p in sorted(glob.glob(os.path.join(HERE, "front_*.json"))):
        rec = json.load(open(p))
        if rec["query"].split(":")[0] == kind:
            out.append(rec)
    return out


def _scene(key):
    parts = key.split(":")
    if parts[0] == "cfg2":
        return scenes.make_scene("cfg2", scenes.workload_seed(2, int(parts[1])), M=10_000,
                                 S_max=512)
    return scenes.batch_scene(int(parts[1]), int(parts[2]), M=10_000, S_max=512)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _check_front(rec, nodes_of, costs, pops, mc, res):
    assert res["status"] == rec["status"]
    assert res["partial_plans"] == rec["stats"]["partial_plans"]
    assert res["rounds"] == rec["stats"]["rounds"]
    assert res["final_i"] == rec["stats"]["final_i"]
    assert res["dropped_steps"] == rec["stats"]["dropped_steps"]
    assert res["n_goal_plans"] == rec["n_goal_plans"]
    assert res["n_front"] == len(rec["front"])
    for k, f in enumerate(rec["front"]):
        assert nodes_of(k) == tuple(f["nodes"]), k
        assert abs(costs[k] - f["cost"]) <= REL * max(1.0, f["cost"]), k
        assert pops[k] == f["pop"], k
        if mc is not None:
            assert mc[k] == rec["front_mc_counts"][k], k
    b = rec["best"]
    if b is None:
        assert res["best_plan"] < 0
    else:
        assert res["best"] == b["index"]
        assert res["best_pop"] == b["pop"]
        assert abs(res["best_cost"] - b["cost"]) <= REL * b["cost"]
        assert res["best_mc_count"] == rec["front_mc_counts"][b["index"]]


@pytest.mark.parametrize("rec", _fixtures("cfg2"), ids=lambda r: r["query"])
def test_single_query_front_equals_oracle(rec):
    sc = _scene(rec["query"])
    print_case("golden_front", query=rec["query"], n=sc.n, N=sc.N)
    pl = _lib.Planner(n_particles=sc.N, max_nodes=sc.n + 1, max_obstacles=max(1, sc.n_obs),
                      max_steps=sc.S_max, mc_particles=sc.M, cap_plans=1 << 21,
                      cap_pairs=1 << 23, cap_edges=1 << 24)
    res = pl.plan(pl.problem(_dev(sc.samples), _dev(sc.obstacles), sc.x_init, sc.goal, sc.alpha,
                             sc.sigma, _dev(sc.noise), _dev(sc.noise_mc)))
    ids, mc = pl.front()
    st = gpu_plans(pl)
    print("  gpu", {k: res[k] for k in ("status", "partial_plans", "n_front", "best_cost",
                                        "best_mc_count", "flagged")},
          "oracle flagged", rec["stats"]["flagged_particles"],
          "flagged bits on the front", [f["flagged_bits"] for f in rec["front"]], flush=True)
    _check_front(rec, lambda k: st["paths"][ids[k]], st["cost"][ids], st["pop"][ids], mc, res)
    if rec["best"] is not None:
        assert pl.path(res["best_plan"]) == tuple(rec["best"]["nodes"])
    pl.close()


def test_batched_queries_equal_oracle():
    recs = _fixtures("batch")
    if not recs:
        pytest.skip("no batched fixtures")
    scs = [_scene(r["query"]) for r in recs]
    print_case("golden_batch", queries=[r["query"] for r in recs])
    b = _lib.Batch(len(scs), n_particles=max(s.N for s in scs),
                   max_nodes=max(s.n for s in scs) + 1, max_obstacles=60, max_steps=512,
                   mc_particles=10_000, cap_plans=1 << 20, cap_pairs=1 << 21, cap_edges=1 << 22)
    qs = [(_dev(s.samples), _dev(s.obstacles), s.x_init, s.goal, s.alpha, s.sigma, _dev(s.noise),
           _dev(s.noise_mc)) for s in scs]
    out = b.plan(qs)
    for i, (rec, res) in enumerate(zip(recs, out)):
        print("  gpu", rec["query"], {k: res[k] for k in ("status", "partial_plans", "n_front",
                                                           "best_cost", "best_mc_count")},
              flush=True)
        assert res["status"] == rec["status"]
        assert res["partial_plans"] == rec["stats"]["partial_plans"]
        assert res["rounds"] == rec["stats"]["rounds"]
        assert res["n_goal_plans"] == rec["n_goal_plans"]
        assert res["n_front"] == len(rec["front"])
        best = rec["best"]
        if best is not None:
            assert b.path(i, res["best_plan"]) == tuple(best["nodes"])
            assert res["best"] == best["index"]
            assert res["best_pop"] == best["pop"]
            assert abs(res["best_cost"] - best["cost"]) <= REL * best["cost"]
            assert res["best_mc_count"] == rec["front_mc_counts"][best["index"]]
    b.close()
