"""Benchmark: PUMP planning queries on one MI355X.

One step = one whole pump_plan call (deviation table, BuildGraph, every
Explore round, PlanSelection with MC certification) on the 20-box, 4000-sample,
128-particle workload (alpha = 0.01, sigma = 0.02), inputs resident in HBM.
Prints one JSON line.  `value` is partial plans evaluated per second over the
whole timed job; the line also carries the time to a certified plan, the
per-kernel roofline of the dominant kernel and the CPU oracle timed on a
bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TFLOPS = 78.6        # 256 CU x 64 lanes x 2.4 GHz x 2 (FMA)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--batch-queries", type=int, default=256,
                    help="queries in the batched-engine leg (0 skips the leg)")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--tune-queries", type=int, default=256)
    return ap.parse_args()


def make_inputs(seed):
    from paper_1607_06886_amd import scenes
    return scenes.make_scene("cfg2", scenes.workload_seed(2, seed), M=10_000, S_max=512)


VALU_PEAK_TLANEOPS = 39.3          # 256 CU x 64 lanes x 2.4 GHz (one lane-op per lane per clock)

# Algorithmic lane-ops of Explore, per unit of work:
OPS_PAIR = 40          # locate the pair in the group, its edge, cost, steps, cutoff, pre-prune lookup
OPS_GEOM = 150         # + Hermite coefficients, three cubic ranges, per-waypoint cloud boxes ...
OPS_GEOM_PER_BOX = 12  # ... and one box-overlap test per obstacle (pairs past the pre-prune)
OPS_PARTICLE_WP = 3    # particle position at a tested waypoint
OPS_PARTICLE_BOX = 12  # inner and outer box test of a particle (6 compares each)


def kernel_models(sc, res, rounds_pairs, N):
    """Algorithmic work per launch for the kernels the roofline may name.

    graph_mark (BuildGraph pass 1): one ordered pair per unit; it reads two
    24-byte states (one from cache) and writes one bit, so it is bound by
    FP64 arithmetic: the closed-form parts of the connection cost (boundary
    sums, quartic coefficients, two cost evaluations) plus the root solves
    modelled at 2 roots x 8 Newton steps x 9 flops: 230 FP64 flops per pair.
    expand (per-phase path): one (plan, neighbour) pair per unit; algorithmic
    HBM bytes per pair = edge record (col 4 + tau 8 + cost 8) + pair identity,
    flag and count (4 + 4 + 1 + 4) + kept fraction x (edge 4 + step 4 + cost 8
    + N/8 mask) + parent record (head, cost, step, pop 20 + N/8) / mean degree.
    explore_single (all rounds in one launch): lane-operations, counted from
    the library's counters: every pair OPS_PAIR, every pair past the
    pre-prune OPS_GEOM + OPS_GEOM_PER_BOX x n_obs, and per particle
    OPS_PARTICLE_WP at each tested waypoint and OPS_PARTICLE_BOX per
    waypoint-box test.
    """
    n1 = sc.n + 1
    pairs = n1 * (n1 - 1)
    kept = res["inserted"] / max(1, res["partial_plans"])
    deg = res["n_edges"] / max(1, res["n_valid_nodes"])
    per_pair = 20 + 13 + kept * (16 + N / 8) + (20 + N / 8) / max(1.0, deg)
    lane_ops = (OPS_PAIR * res["partial_plans"]
                + (OPS_GEOM + OPS_GEOM_PER_BOX * sc.n_obs) * res["simulated"]
                + N * (OPS_PARTICLE_WP * res["sim_waypoints"]
                       + OPS_PARTICLE_BOX * res["sim_box_tests"]))
    return {
        "graph_mark": dict(bound="alu", unit="TFLOP/s", peak=FP64_VALU_PEAK_TFLOPS,
                           work=230.0 * pairs, scale=1e12),
        "expand": dict(bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS,
                       work=per_pair * (res["partial_plans"] / max(1, rounds_pairs)), scale=1e9,
                       per_pair_bytes=per_pair),
        "explore_single": dict(bound="alu", unit="T lane-ops/s", peak=VALU_PEAK_TLANEOPS,
                               work=lane_ops, scale=1e12, lane_ops=lane_ops,
                               hbm_bytes_model=per_pair * res["partial_plans"]),
    }


def cpu_baseline(seconds):
    """The oracle on a bounded sample of the same workload: BuildGraph rows for
    a random subset of source nodes, then Alg. 4's pair expansion (cost plus
    particle CP estimate) for plans at those nodes to every neighbour, with
    step offsets drawn over the plan lengths seen in the workload."""
    from oracle import dynamics, explore as ex, graph as gr, pump as opump
    sc = make_inputs(0)
    cfg = opump.Config()
    V = np.concatenate([sc.x_init[None], sc.samples]).astype(np.float64)
    A_cl, L, _ = dynamics.closed_loop(cfg.dt, sc.sigma, cfg.q_pos, cfg.q_vel, cfg.r_track)
    D = dynamics.deviation_table(A_cl, L, sc.noise, sc.S_max)
    valid = ~gr.points_in_boxes(V[:, :3], sc.obstacles)
    rng = np.random.default_rng(1)
    rows = rng.choice(np.nonzero(valid)[0], 56, replace=False)
    c0 = time.process_time()
    t0 = time.perf_counter()
    src, dst, tau, cost = gr.graph_rows(V, valid, sc.obstacles, cfg.r_conn, cfg.r_steer, rows)
    t1 = time.perf_counter()
    graph_pairs = len(rows) * (int(valid.sum()) - 1)
    graph = dict(col=dst, tau=tau, cost=cost)
    # parents: one plan per sampled head, mid-length step offsets
    pairs_done = 0
    t_ex = 0.0
    e = 0
    while t_ex < seconds and e < dst.shape[0]:
        idx = np.arange(e, min(dst.shape[0], e + 2048))
        parents = [ex.Plan(nodes=(0, int(src[k])), cost=1.0, step=int(rng.integers(0, 60)),
                           mask=np.zeros(sc.N, bool), parent=0) for k in idx]
        ta = time.perf_counter()
        ex.extend_batch(V, graph, D, sc.obstacles, cfg.dt, sc.S_max, parents, idx)
        t_ex += time.perf_counter() - ta
        pairs_done += idx.shape[0]
        e += idx.shape[0]
    wall = (t1 - t0) + t_ex
    cpu = time.process_time() - c0
    return {
        "value": pairs_done / t_ex,
        "unit": "partial plans/s",
        "cores": max(1, int(round(cpu / max(wall, 1e-9)))),
        "kind": "oracle",
        "sample": (f"cfg2 seed 0: Alg. 4 pair expansion (cost + {sc.N}-particle CP estimate) "
                   f"for {pairs_done} pairs out of {len(rows)} sampled heads "
                   f"({t_ex:.1f} s); BuildGraph rows for the same heads: "
                   f"{graph_pairs} pairs in {t1 - t0:.1f} s = {graph_pairs / (t1 - t0):.3g} pairs/s"),
        "graph_pairs_per_s": graph_pairs / (t1 - t0),
    }


# HBM traffic of the dominant kernel, from two rocprofv3 --pmc runs (FETCH_SIZE,
# then WRITE_SIZE) recorded in profiles/ together with a hash of the sources
# that define the kernel; it is reported only while those sources are unchanged.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "explore_single_cfg2_traffic.txt")
TRAFFIC_SOURCES = ["paper_1607_06886_amd/csrc/" + f for f in (
    "kernels_coop.hip", "explore_team.hpp", "explore_ops.hpp", "device_math.hpp",
    "pump_internal.hpp")]


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel):
    """Bytes per launch of `kernel` measured by the counters, or None."""
    try:
        rec = dict(line.strip().split("=", 1) for line in open(TRAFFIC_FILE)
                   if "=" in line and not line.startswith("#"))
    except OSError:
        return None
    if rec.get("bench_kernel") != kernel or rec.get("sources_sha256") != sources_digest():
        return None
    kib = (float(rec["fetch_kib"]) * float(rec["fetch_scale"])
           + float(rec["write_kib"]) * float(rec["write_scale"]))
    return kib * 1024.0


def batched_inputs(q, seed, S_max=512, M=10_000):
    """q uneven queries (scenes.batch_specs) with device-resident inputs; the
    particle noise is drawn on the device from a per-query seed."""
    import torch

    from paper_1607_06886_amd import scenes
    specs = scenes.batch_specs(seed, q)
    g = torch.Generator(device="cuda")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = []
    for i, sp in enumerate(specs):
        qs = scenes.workload_seed(4, 1000 * seed + i)
        x0, goal, boxes, smp = scenes.batch_map(sp, qs)
        g.manual_seed(qs)
        noise = torch.randn((S_max, 6, sp["N"]), generator=g, device="cuda")
        noise_mc = torch.randn((S_max, 6, M), generator=g, device="cuda")
        out.append((dev(smp), dev(boxes), x0, goal, float(np.float32(sp["alpha"])),
                    float(np.float32(sp["sigma"])), noise, noise_mc))
    return specs, out


def batched_leg(q, seed, steps, tune_q, S_max=512, M=10_000):
    """The batched engine on q uneven queries: the autotuner picks the
    persistent kernel's shape on the first tune_q queries, then whole batches
    are timed (device inputs resident, one graph launch per batch)."""
    import torch

    from paper_1607_06886_amd import _lib
    specs, queries = batched_inputs(q, seed, S_max, M)
    b = _lib.Batch(q, n_particles=256, max_nodes=max(s["n"] for s in specs) + 1,
                   max_obstacles=60, max_steps=S_max, mc_particles=M, cap_plans=1 << 20,
                   cap_pairs=1 << 21, cap_edges=1 << 22)
    t0 = time.perf_counter()
    best, tune_ms = b.tune(queries[:tune_q])
    t_tune = time.perf_counter() - t0
    best["use_graph"] = 1
    # warm-up (and the reference results); a query that fails reports its
    # status and the others complete
    res = b.plan(queries, tuning=best, raise_on_error=False)
    times = []
    for _ in range(steps):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        r = b.plan(queries, tuning=best, raise_on_error=False)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ta)
        assert [x["partial_plans"] for x in r] == [x["partial_plans"] for x in res]
    b.close()
    total = sum(times)
    pairs = sum(x["partial_plans"] for x in res)
    st = [x["status"] for x in res]
    return {
        "workload": f"{q} queries: samples U{{1000..8000}}, particles {{64,128,256}}, "
                    "boxes U{5..60} (sides U[0.05,0.25]), alpha {0.01,0.05}, sigma 0.02, "
                    f"M {M}, S_max {S_max}",
        "queries": q,
        "steps": steps,
        "ms_per_batch": 1e3 * total / steps,
        "queries_per_s": q * steps / total,
        "partial_plans_per_s": pairs * steps / total,
        "partial_plans_per_batch": pairs,
        "status_counts": {str(k): st.count(k) for k in sorted(set(st))},
        "tuning": best,
        "tune_queries": tune_q,
        "tune_best_ms": tune_ms,
        "tune_s": t_tune,
    }


def roadmap_leg(pl, samples, pr, r0, steps):
    """The same query with the graph built over a cached roadmap (Near and the
    optimal connections of the samples computed once, as the paper caches them
    offline): build time, then per-query times with the cache."""
    import torch

    from paper_1607_06886_amd import _lib
    cfg = pl.cfg
    rm = _lib.Roadmap(samples, max_nodes=cfg.max_nodes, cap_edges=cfg.cap_edges,
                      r_steer=cfg.r_steer, r_conn=cfg.r_conn)
    pl.set_roadmap(rm)
    pl.plan(pr)
    torch.cuda.synchronize()
    res = [pl.plan(pr) for _ in range(steps)]
    pl.set_roadmap(None)
    info = rm.info()
    rm.close()
    same = all(r["partial_plans"] == r0["partial_plans"] and r["best_plan"] == r0["best_plan"]
               and r["best_cost"] == r0["best_cost"] for r in res)
    return {"ms_build": info["ms_build"], "cached_connections": info["n_edges"],
            "ms_to_certified_plan": statistics.median(r["ms_total"] for r in res),
            "setup_ms": statistics.median(r["ms_setup"] for r in res),
            "partial_plans_per_s": r0["partial_plans"] / (statistics.median(
                r["ms_total"] for r in res) / 1e3),
            "same_result_as_scratch_graph": same}


def smooth_leg(sc, stream, samples, obstacles, noise, noise_mc):
    """Smooth(p*, alpha) on the same query: the blend weight, cost and time."""
    from paper_1607_06886_amd import _lib
    pl = _lib.Planner(stream=stream, n_particles=sc.N, max_nodes=sc.n + 1,
                      max_obstacles=max(1, sc.n_obs), max_steps=sc.S_max, mc_particles=sc.M,
                      cap_plans=1 << 21, cap_pairs=1 << 23, cap_edges=1 << 24, smooth=1)
    pr = pl.problem(samples, obstacles, sc.x_init, sc.goal, sc.alpha, sc.sigma, noise, noise_mc)
    pl.plan(pr)
    pl.set_timing(True)
    r = pl.plan(pr)
    kt = pl.timing()
    pl.close()
    return {"beta": r["smooth_beta"], "cost": r["smooth_cost"], "plan_cost": r["best_cost"],
            "mc_count": r["smooth_mc_count"], "steps": r["smooth_steps"],
            "ms": kt["smooth"][0], "ms_to_certified_smoothed_plan": r["ms_total"]}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested); "
              "this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1607_06886_amd import _lib

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    sc = make_inputs(args.seed)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    samples, obstacles, noise, noise_mc = (dev(sc.samples), dev(sc.obstacles), dev(sc.noise),
                                           dev(sc.noise_mc))
    stream = torch.cuda.current_stream()
    pl = _lib.Planner(stream=stream, n_particles=sc.N, max_nodes=sc.n + 1,
                      max_obstacles=max(1, sc.n_obs), max_steps=sc.S_max, mc_particles=sc.M,
                      cap_plans=1 << 21, cap_pairs=1 << 23, cap_edges=1 << 24)
    pr = pl.problem(samples, obstacles, sc.x_init, sc.goal, sc.alpha, sc.sigma, noise, noise_mc)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        pl.plan(pr)
    pl.set_timing(True)
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        results.append(pl.plan(pr))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = pl.timing()
    pl.set_timing(False)
    total_s = t1 - t0
    pairs = sum(r["partial_plans"] for r in results)
    r0 = results[0]
    assert all(r["partial_plans"] == r0["partial_plans"] and r["best_plan"] == r0["best_plan"]
               for r in results), "non-deterministic results across steps"
    models = kernel_models(sc, r0, max(1, kt["expand"][1] // args.steps), sc.N)
    dom = max(models, key=lambda k: kt[k][0])
    m = models[dom]
    ms_total, launches = kt[dom]
    avg_s = ms_total / 1e3 / max(1, launches)
    achieved = m["work"] / avg_s / m["scale"]
    roofline = {"bound": m["bound"], "kernel": dom, "achieved": achieved, "peak": m["peak"],
                "unit": m["unit"], "frac": achieved / m["peak"], "traffic": recorded_traffic(dom),
                "avg_launch_us": avg_s * 1e6, "launches": launches}
    if "hbm_bytes_model" in m:
        roofline["algorithmic_hbm_bytes"] = m["hbm_bytes_model"]
        roofline["algorithmic_hbm_gbs"] = m["hbm_bytes_model"] / avg_s / 1e9
    line = {
        "metric": "partial plans evaluated/s; ms to certified plan at CP<=alpha, plain vs learned",
        "value": pairs / total_s,
        "unit": "partial plans/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total_s / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "plain PUMP, 20 random boxes (sides U[0.05,0.25]), 4000 samples, "
                               "128 particles, sigma 0.02, alpha 0.01, M 10000",
                   "n": sc.n, "n_obs": sc.n_obs, "N": sc.N, "alpha": sc.alpha, "sigma": sc.sigma,
                   "M": sc.M, "S_max": sc.S_max, "parallelism": "1 GPU"},
        "ms_to_certified_plan": statistics.median(r["ms_total"] for r in results),
        "explore_partial_plans_per_s": r0["partial_plans"] / (statistics.median(
            r["ms_explore"] for r in results) / 1e3),
        "partial_plans_per_query": r0["partial_plans"],
        "simulated_per_query": r0["simulated"],
        "preprune_per_query": r0["preprune"],
        "sim_waypoints_per_query": r0["sim_waypoints"],
        "sim_box_tests_per_query": r0["sim_box_tests"],
        "rounds": r0["rounds"],
        "status": r0["status"],
        "best_cost": r0["best_cost"],
        "best_cp_mc": r0["best_cp_mc"],
        "stage_ms": {"setup": statistics.median(r["ms_setup"] for r in results),
                     "explore": statistics.median(r["ms_explore"] for r in results),
                     "select": statistics.median(r["ms_select"] for r in results)},
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kt.items()},
        "roofline": roofline,
    }
    line["roadmap"] = roadmap_leg(pl, samples, pr, r0, args.steps)
    line["smooth"] = smooth_leg(sc, stream, samples, obstacles, noise, noise_mc)
    pl.close()
    if args.batch_queries > 0:
        line["batched"] = batched_leg(args.batch_queries, args.seed, args.batch_steps,
                                      min(args.tune_queries, args.batch_queries))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
