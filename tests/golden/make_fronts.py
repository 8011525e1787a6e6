"""Writes the oracle's result for full-size planning queries to JSON fixtures.

For each query the fixture holds what the plain CPU oracle (oracle/) computes
on the seeded synthetic inputs of paper_1607_06886_amd.scenes: Explore's
counters (Alg. 4), the Pareto front of P_goal in selection order (Alg. 5
sorting: cp_hat ascending, cost descending, node sequence), the certification
count MC(p) of every front plan (Sec. IV, MC with M fresh particles), the
indices Alg. 5's bisection evaluated, and the selected plan p*.

Nothing here reads the HIP library; the GPU tests compare the library's
results with these files.  Usage:
    python tests/golden/make_fronts.py cfg2:0 [batch:<seed>:<query> ...]
"""

from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import pump as opump, select as osel  # noqa: E402
from paper_1607_06886_amd import scenes  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def scene_for(key):
    """Inputs of a named query: "cfg2:<seed>" (the 20-box, 4000-sample,
    128-particle workload) or "batch:<seed>:<i>" (query i of the uneven
    256-query batch with batch seed <seed>, host-drawn noise)."""
    parts = key.split(":")
    if parts[0] == "cfg2":
        return scenes.make_scene("cfg2", scenes.workload_seed(2, int(parts[1])), M=10_000,
                                 S_max=512)
    if parts[0] == "batch":
        return scenes.batch_scene(int(parts[1]), int(parts[2]), M=10_000, S_max=512)
    raise ValueError(key)


def record(key):
    sc = scene_for(key)
    cfg = opump.Config()
    t0 = time.perf_counter()
    out = opump.run(sc, cfg)
    mc_all = [osel.mc_count(out["V"], p.nodes, sc.obstacles, out["A_cl"], out["L"], sc.noise_mc,
                            cfg.r_steer, cfg.dt) for p in out["front"]]
    for m, (c, _) in out["evals"].items():
        assert mc_all[m - 1] == c
    best = out["best"]
    st = out["stats"]
    return {
        "query": key,
        "inputs": {"n": sc.n, "n_obs": sc.n_obs, "N": sc.N, "M": sc.M, "S_max": sc.S_max,
                   "alpha": float(sc.alpha), "sigma": float(sc.sigma), "seed": sc.seed},
        "status": out["status"],
        "stats": {k: int(st[k]) for k in ("partial_plans", "inserted", "rounds", "final_i",
                                          "dropped_steps", "flagged_particles")},
        "n_goal_plans": len(out["goal_plans"]),
        "front": [{"nodes": list(p.nodes), "cost": p.cost, "pop": p.pop, "step": p.step,
                   "flagged_bits": int(p.fmask.sum())} for p in out["front"]],
        "front_mc_counts": [int(c) for c in mc_all],
        "bisection_evaluated": sorted(int(m) for m in out["evals"]),
        "best": None if best is None else {"index": out["front"].index(best), "nodes":
                                           list(best.nodes), "cost": best.cost, "pop": best.pop},
        "oracle_seconds": time.perf_counter() - t0,
    }


def main(keys):
    for key in keys:
        rec = record(key)
        path = os.path.join(HERE, "front_" + key.replace(":", "_") + ".json")
        with open(path, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(key, rec["status"], rec["stats"], len(rec["front"]),
              f"{rec['oracle_seconds']:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["cfg2:0"])
