"""Benchmark: PUMP planning queries on one MI355X.

One step = one whole pump_plan call (deviation table, BuildGraph, every
Explore round, PlanSelection with MC certification) on the indoor workload:
a 4x4 room grid of 60 thin walls with doorways 0.08 wide, 20,000 samples,
256 particles, sigma 0.02, alpha 0.01, M = 10^4, inputs resident in HBM.
Prints one JSON line.  `value` is partial plans evaluated per second over the
whole timed job; the line also carries the query's outcome (time to Alg. 5's
result and, where a plan is certified, to the certified plan), the roofline of
the dominant kernel, the 4000-sample query (time to its certified plan), the
same indoor query over a cached roadmap, the batched engine on 256 uneven
queries, and the CPU oracle timed on the indoor query's own first rounds.
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
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="oracle time per CPU-baseline run (one process, then all)")
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="worker processes of the all-core oracle run (0: host cores, <= 16)")
    ap.add_argument("--batch-queries", type=int, default=256,
                    help="queries in the batched-engine leg (0 skips the leg)")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--tune-queries", type=int, default=256)
    ap.add_argument("--legs", default="cfg2,roadmap,batch,learned,hsmc",
                    help="comma list of the extra legs to run (cfg2, roadmap, batch, learned, hsmc)")
    ap.add_argument("--learned-maps", type=int, default=20)
    return ap.parse_args()


def indoor_inputs(seed):
    """The headline query: indoor map, 20,000 samples, N = 256."""
    from paper_1607_06886_amd import scenes
    return scenes.make_scene("cfg3", scenes.workload_seed(3, seed), M=10_000, S_max=512)


def boxes_inputs(seed):
    """The 4000-sample, 20-box, N = 128 query."""
    from paper_1607_06886_amd import scenes
    return scenes.make_scene("cfg2", scenes.workload_seed(2, seed), M=10_000, S_max=512)


VALU_PEAK_TLANEOPS = 39.3          # 256 CU x 64 lanes x 2.4 GHz (one lane-op per lane per clock)

# The hot-path scope table's per-pair work of the expansion (A3-A7) at the
# three single-query workloads (3 / 20 / 60 boxes; N = 32 / 128 / 256):
# steer + K (18 + 12 n_obs) + K N (3 + 6 n_near) + K N / 64 with K ~ 10.
SCOPE_OPS_PER_PAIR = {3: 1.9e3, 20: 8.2e3, 60: 31e3}

# Executed lane-operations of the particle stage, per unit:
OPS_SIM_PAIR = 50      # Hermite coefficients of the queued pair's edge
OPS_SIM_WP_UNIFORM = 18    # nominal point and cloud box of a tested waypoint ...
OPS_SIM_WP_PER_BOX = 12    # ... and its overlap test with each obstacle
OPS_PARTICLE_WP = 3    # particle position at a tested waypoint
OPS_PARTICLE_BOX = 6   # point-in-box test of a particle (6 compares)
# ... and of the pair stage / the single launch, per pair:
OPS_PAIR = 40          # locate the pair in its group, edge, cost, steps, cutoff, pre-prune lookup
OPS_GEOM = 150         # + Hermite coefficients, three cubic ranges, cloud boxes per waypoint ...
OPS_GEOM_PER_BOX = 12  # ... and one box-overlap test per obstacle (pairs past the pre-prune)


def kernel_models(sc, res, N):
    """Algorithmic lane-operations per query of the kernels the roofline may
    name (all VALU-bound: see the design doc), from the library's counters of that
    query:

    expand_sim (particle stage, per-phase mode): per simulated pair
      OPS_SIM_PAIR, per tested waypoint OPS_SIM_WP_UNIFORM + OPS_SIM_WP_PER_BOX
      x n_obs + N x OPS_PARTICLE_WP, per waypoint-box test N x OPS_PARTICLE_BOX
      (the scope table's terms, with the measured waypoints and box tests);
    expand (pair stage, per-phase mode): every pair OPS_PAIR, every pair past
      the pre-prune OPS_GEOM + OPS_GEOM_PER_BOX x n_obs;
    explore_single (every phase in one launch): the sum of the two.
    """
    sim = (OPS_SIM_PAIR * res["simulated"]
           + res["sim_waypoints"] * (OPS_SIM_WP_UNIFORM + OPS_SIM_WP_PER_BOX * sc.n_obs
                                     + N * OPS_PARTICLE_WP)
           + res["sim_box_tests"] * N * OPS_PARTICLE_BOX)
    # pairs past the pair stage's pre-prune (the particle stage's own
    # pre-prunes are counted with them, so this is a slight undercount)
    geom = max(res["simulated"], res["partial_plans"] - res["preprune"] - res["dropped_steps"])
    pairs = OPS_PAIR * res["partial_plans"] + (OPS_GEOM + OPS_GEOM_PER_BOX * sc.n_obs) * geom
    return {"expand_sim": sim, "expand": pairs, "explore_single": sim + pairs}


def cpu_baseline(seconds, procs):
    """The oracle, as written, on the headline query's own first rounds.

    Round 0 (the root's pairs) runs through the oracle's Explore with the
    graph rows built on demand by its BuildGraph row function; then the pairs
    of round 1's group, head by head in group order, until about `seconds` of
    work: extended once in this process and once split over `procs` worker
    processes (each round's pairs cut into contiguous slices, results joined
    in order).  Rates count partial plans over the time spent extending them;
    the row builds are timed separately."""
    import multiprocessing as mp

    from oracle import dynamics, explore as ex, graph as gr, pump as opump
    sc = indoor_inputs(0)
    cfg = opump.Config()
    V = np.concatenate([sc.x_init[None], sc.samples]).astype(np.float64)
    A_cl, L, _ = dynamics.closed_loop(cfg.dt, sc.sigma, cfg.q_pos, cfg.q_vel, cfg.r_track)
    D = dynamics.deviation_table(A_cl, L, sc.noise, sc.S_max)
    g = gr.RowsOnDemand(V, sc.obstacles, cfg.r_conn, cfg.r_steer)
    gl = sc.goal.astype(np.float64)
    goal = np.nonzero(np.all((V[:, :3] >= gl[:3]) & (V[:, :3] <= gl[3:]), axis=1) & g["valid"])[0]
    amin, amax = opump.thresholds(float(sc.alpha), opump.eta_rule(float(sc.alpha)))
    t0 = time.perf_counter()
    plans, P, stats, rounds = ex.explore(V, g, D, sc.obstacles, goal, amin, amax, cfg.lam,
                                         cfg.r_conn, cfg.dt, sc.S_max, record=True,
                                         time_budget=0.0)
    t_r0 = time.perf_counter() - t0 - g.seconds
    pairs_r0 = stats["partial_plans"]
    # round 1's group: open plans with cost <= 1 * lambda * r_n, in id order
    open_nodes = set(rounds[-1]["open"])
    h = float(cfg.lam) * float(cfg.r_conn)
    B = [k for k, p in enumerate(plans) if p.nodes in open_nodes and p.cost <= h]
    parents, edges = [], []
    est = 0.0
    per_pair = t_r0 / max(1, pairs_r0)
    n_heads = 0
    for k in B:
        e0, e1 = ex.row_range(g, plans[k].head)
        parents += [plans[k]] * (e1 - e0)
        edges += list(range(e0, e1))
        n_heads += 1
        est += (e1 - e0) * per_pair
        if est >= seconds:
            break
    edges = np.asarray(edges, np.int64)
    ta = time.perf_counter()
    one = ex.extend_batch(V, g, D, sc.obstacles, cfg.dt, sc.S_max, parents, edges)
    t_one = time.perf_counter() - ta
    rate_one = len(parents) / t_one
    procs = procs or min(16, os.cpu_count() or 1)
    rate_all, t_all = None, None
    if procs > 1:
        with mp.get_context("fork").Pool(procs, initializer=ex.pool_init,
                                         initargs=(V, D, sc.obstacles, cfg.dt, sc.S_max)) as pool:
            ta = time.perf_counter()
            par = ex.extend_split(pool, V, g, D, sc.obstacles, cfg.dt, sc.S_max, parents, edges,
                                  procs)
            t_all = time.perf_counter() - ta
        assert all((a == b).all() for a, b in zip(one, par)), "split run differs"
        rate_all = len(parents) / t_all
    try:
        cpu_model = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo")
                     if l.startswith("model name")][0]
    except (OSError, IndexError):
        cpu_model = "unknown"
    use_all = rate_all is not None and rate_all > rate_one
    return {
        "value": rate_all if use_all else rate_one,
        "unit": "partial plans/s",
        "cores": procs if use_all else 1,
        "kind": "oracle",
        "sample": (f"indoor 20000-sample N=256 query, seed 0: Alg. 4 round 0 ({pairs_r0} pairs "
                   f"from the root, {t_r0:.1f} s) and the first {n_heads} of the {len(B)} "
                   f"plans of round 1's group ({len(parents)} pairs): {t_one:.1f} s in one process"
                   + (f", {t_all:.1f} s over {procs} processes" if t_all else "")
                   + f"; {len(g._range)} BuildGraph rows built on demand in {g.seconds:.1f} s"),
        "single_process": {"partial_plans_per_s": rate_one, "seconds": t_one},
        "all_cores": None if rate_all is None else {"partial_plans_per_s": rate_all,
                                                    "processes": procs, "seconds": t_all},
        "round0_partial_plans_per_s": pairs_r0 / max(t_r0, 1e-9),
        "graph_rows_per_s": len(g._range) / max(g.seconds, 1e-9),
        "host": {"cpu_model": cpu_model, "os_cpu_count": os.cpu_count()},
    }


# HBM traffic of the dominant kernel, from two rocprofv3 --pmc runs (FETCH_SIZE,
# then WRITE_SIZE) recorded in profiles/ together with a hash of the sources
# that define the kernel; it is reported only while those sources are unchanged.
TRAFFIC_FILES = {
    "expand_sim": os.path.join(ROOT, "profiles", "expand_sim_indoor_traffic.txt"),
    "explore_single": os.path.join(ROOT, "profiles", "explore_single_indoor_traffic.txt"),
}
TRAFFIC_SOURCES = ["paper_1607_06886_amd/csrc/" + f for f in (
    "kernels_coop.hip", "kernels_explore.hip", "explore_team.hpp", "explore_ops.hpp",
    "device_math.hpp", "pump_internal.hpp")]


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel):
    """Bytes per launch of `kernel` measured by the counters, or None."""
    path = TRAFFIC_FILES.get(kernel)
    try:
        rec = dict(line.strip().split("=", 1) for line in open(path)
                   if "=" in line and not line.startswith("#"))
    except (OSError, TypeError):
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


def hsmc_leg(stream, seed, warmup, steps):
    """The paper's own exploration model (Half-Space Monte Carlo, Sec. III-B,
    eq. (7); run there with N = 128) on the 4000-sample, 20-box, N = 128
    query: time to the certified plan and partial plans per second."""
    import torch
    sc = boxes_inputs(seed)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    pl = planner_for(sc, stream, cap_pairs=1 << 23, cap_edges=1 << 24, cp_model=1)
    pr = pl.problem(dev(sc.samples), dev(sc.obstacles), sc.x_init, sc.goal, sc.alpha, sc.sigma,
                    dev(sc.noise), dev(sc.noise_mc))
    results, total, _ = timed_queries(pl, pr, warmup, steps)
    pl.close()
    r0 = results[0]
    return {"workload": "HSMC exploration model, 20 random boxes, 4000 samples, 128 particles, "
                        "sigma 0.02, alpha 0.01, M 10000",
            "status": STATUS[r0["status"]],
            "ms_to_certified_plan": statistics.median(r["ms_total"] for r in results),
            "partial_plans_per_s": r0["partial_plans"] * steps / total,
            "partial_plans_per_query": r0["partial_plans"], "best_cost": r0["best_cost"],
            "best_cp_mc": r0["best_cp_mc"]}


# Trained weights of the learned proposal (FP32, the library's flat layout),
# written by `python -m paper_1607_06886_amd.learned --params <file>`.
WEIGHTS = os.path.join(ROOT, "paper_1607_06886_amd", "weights", "proposal_params.npy")


def learned_leg(n_maps, sizes=(2000, 4000, 8000)):
    """The learned proposal at its evaluation size (8000 samples, 256
    particles, alpha 0.01, M 10^4) on held-out maps, half random boxes and
    half indoor: plain PUMP on n uniform samples against n/2 samples from the
    trained mixture + n/2 uniform, every plan certified by MC(p) <= alpha.
    Times are pump_plan's (plus the network's sampling for learned)."""
    from paper_1607_06886_amd import _lib, learned
    if not os.path.exists(WEIGHTS):
        return {"skipped": f"no trained weights at {os.path.relpath(WEIGHTS, ROOT)}"}
    params = np.load(WEIGHTS, allow_pickle=False)
    mlp = _lib.MLP(64)
    mlp.set_params(params)
    sizes = list(sizes)
    rows = learned.evaluate(mlp, n_maps, ["boxes", "indoor"], sizes, 256, 0.01, 0.02, 900_000)
    mlp.close()
    summ = learned.summarise(rows, sizes)
    top = max(sizes)
    per = summ["per_n"][top]
    by = {(r["map"], r["n"]): r for r in rows}
    vs_plain = {}
    for n in sizes:
        wins, ratio = [], []
        for m in sorted({r["map"] for r in rows}):
            a, b = by[(m, n)], by[(m, top)]
            cl = a["learned_cost"] if a["learned_status"] == 0 else math.inf
            cp = b["plain_cost"] if b["plain_status"] == 0 else math.inf
            if math.isinf(cl) and math.isinf(cp):
                continue
            wins.append(cl <= cp + 1e-12)
            ratio.append(a["learned_ms"] / b["plain_ms"])
        vs_plain[f"learned@{n}"] = {"maps": len(wins),
                                    "cost_le_plain@%d" % top: float(np.mean(wins)) if wins else None,
                                    "median_time_ratio": float(np.median(ratio)) if ratio else None}
    return {
        "workload": f"{n_maps} held-out maps (random boxes and indoor), 256 particles, alpha 0.01, "
                    f"sigma 0.02, M 10000; learned = n/2 network + n/2 uniform samples",
        "plain_ms_to_certified_plan": per["median_plain_ms"],
        "learned_ms_to_certified_plan": per["median_learned_ms"],
        "plain_certified": per["plain_certified"], "learned_certified": per["learned_certified"],
        "mean_cost_where_both_certify": {"plain": per["mean_plain_cost"],
                                         "learned": per["mean_learned_cost"]},
        "learned_le_plain_share": per["learned_le_plain"],
        "vs_plain_at_%d" % top: vs_plain,
        "per_n": summ["per_n"],
    }


STATUS = {0: "certified", 1: "infeasible (no front plan certified)", 2: "no goal plan"}


def planner_for(sc, stream, **over):
    from paper_1607_06886_amd import _lib
    kw = dict(stream=stream, n_particles=sc.N, max_nodes=sc.n + 1, max_obstacles=max(1, sc.n_obs),
              max_steps=sc.S_max, mc_particles=sc.M, cap_plans=1 << 22, cap_pairs=1 << 25,
              cap_edges=1 << 25)
    kw.update(over)
    return _lib.Planner(**kw)


def timed_queries(pl, pr, warmup, steps, timing=False):
    """warmup untimed pump_plan calls, then `steps` timed back to back."""
    import torch
    for _ in range(warmup):
        pl.plan(pr)
    if timing:
        pl.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [pl.plan(pr) for _ in range(steps)]
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    kt = pl.timing() if timing else None
    if timing:
        pl.set_timing(False)
    r0 = results[0]
    assert all(r["partial_plans"] == r0["partial_plans"] and r["best_plan"] == r0["best_plan"]
               and r["status"] == r0["status"] for r in results), "results differ across steps"
    return results, total, kt


def boxes_leg(stream, seed, warmup, steps):
    """The 4000-sample, 20-box, N = 128 query: time to its certified plan,
    throughput, and Smooth(p*) on it."""
    import torch
    sc = boxes_inputs(seed)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    samples, obstacles, noise, noise_mc = (dev(sc.samples), dev(sc.obstacles), dev(sc.noise),
                                           dev(sc.noise_mc))
    pl = planner_for(sc, stream, cap_pairs=1 << 23, cap_edges=1 << 24)
    pr = pl.problem(samples, obstacles, sc.x_init, sc.goal, sc.alpha, sc.sigma, noise, noise_mc)
    results, total, _ = timed_queries(pl, pr, warmup, steps)
    pl.close()
    r0 = results[0]
    return {
        "workload": "plain PUMP, 20 random boxes (sides U[0.05,0.25]), 4000 samples, 128 particles, "
                    "sigma 0.02, alpha 0.01, M 10000",
        "status": STATUS[r0["status"]],
        "ms_to_certified_plan": statistics.median(r["ms_total"] for r in results),
        "partial_plans_per_s": r0["partial_plans"] * steps / total,
        "partial_plans_per_query": r0["partial_plans"],
        "best_cost": r0["best_cost"], "best_cp_mc": r0["best_cp_mc"],
        "stage_ms": {"setup": statistics.median(r["ms_setup"] for r in results),
                     "explore": statistics.median(r["ms_explore"] for r in results),
                     "select": statistics.median(r["ms_select"] for r in results)},
        "smooth": smooth_leg(sc, stream, samples, obstacles, noise, noise_mc),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested); "
              "the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    # the CPU oracle first: its worker processes are forked before this
    # process touches the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.cpu_seconds, args.cpu_procs)
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    legs = set(x for x in args.legs.split(",") if x)
    sc = indoor_inputs(args.seed)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    samples, obstacles, noise, noise_mc = (dev(sc.samples), dev(sc.obstacles), dev(sc.noise),
                                           dev(sc.noise_mc))
    stream = torch.cuda.current_stream()
    pl = planner_for(sc, stream)
    pr = pl.problem(samples, obstacles, sc.x_init, sc.goal, sc.alpha, sc.sigma, noise, noise_mc)
    torch.cuda.synchronize()
    results, total_s, kt = timed_queries(pl, pr, args.warmup, args.steps, timing=True)
    pairs = sum(r["partial_plans"] for r in results)
    r0 = results[0]
    ids, mc = pl.front()
    st = pl.plans()
    front = [{"pop": int(st["pop"][i]), "cost": float(st["cost"][i]), "mc_count": int(c)}
             for i, c in zip(ids, mc)]
    mode, _ = pl.explore_mode()
    # roofline of the dominant kernel (largest time per step among the
    # Explore kernels the library times with HIP events on its stream)
    work = kernel_models(sc, r0, sc.N)
    cands = [k for k in work if kt[k][1] > 0]
    dom = max(cands, key=lambda k: kt[k][0])
    ms_total, launches = kt[dom]
    avg_s = ms_total / 1e3 / launches
    work_launch = work[dom] * args.steps / launches
    achieved = work_launch / avg_s / 1e12
    # algorithmic HBM bytes of the particle stage per simulated pair: queue
    # record 32, parent bits N/8, cost 8, count and flag 5, the kept bits N/8,
    # the head's staircase entries c_cut x 8
    sim_bytes = r0["simulated"] * (32 + sc.N / 8 + 8 + 5 + sc.N / 8 + 8 * r0["c_cut"])
    expl_ms = sum(kt[k][0] for k in ("expand", "expand_sim", "explore_single")) / args.steps
    roofline = {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": VALU_PEAK_TLANEOPS,
                "unit": "T lane-ops/s", "frac": achieved / VALU_PEAK_TLANEOPS,
                "traffic": recorded_traffic(dom), "avg_launch_us": avg_s * 1e6,
                "launches": launches, "work_per_launch": work_launch,
                "algorithmic_hbm_bytes_per_launch": sim_bytes * args.steps / launches
                if dom == "expand_sim" else None,
                "scope_model": {
                    "ops_per_pair": SCOPE_OPS_PER_PAIR[60],
                    "pairs_per_query": r0["partial_plans"],
                    "expansion_kernel_ms_per_query": expl_ms,
                    "achieved": SCOPE_OPS_PER_PAIR[60] * r0["partial_plans"] / (expl_ms / 1e3) / 1e12,
                    "frac": SCOPE_OPS_PER_PAIR[60] * r0["partial_plans"] / (expl_ms / 1e3) / 1e12
                    / VALU_PEAK_TLANEOPS,
                    "note": "credits every (plan, neighbour) pair with the full per-pair particle work, "
                            "including the pairs settled by the staircase before simulation and those cut "
                            "early; it can exceed 1 for that reason, the executed-work frac above is the "
                            "measure of the kernel"}}
    ms_q = statistics.median(r["ms_total"] for r in results)
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
        "config": {"workload": "plain PUMP, indoor map: 4x4 room grid of 60 thin walls, doorways "
                               "0.08 wide, 20000 samples, 256 particles, sigma 0.02, alpha 0.01, "
                               "goal a 0.05 box in the far room, M 10000",
                   "n": sc.n, "n_obs": sc.n_obs, "N": sc.N, "alpha": sc.alpha, "sigma": sc.sigma,
                   "M": sc.M, "S_max": sc.S_max, "seed": args.seed, "parallelism": "1 GPU"},
        "outcome": STATUS[r0["status"]],
        "ms_to_outcome": ms_q,
        "ms_to_certified_plan": ms_q if r0["status"] == 0 else None,
        "front": front,
        "explore_mode": {0: "per phase", 1: "single launch", 2: "by graph size"}[mode],
        "explore_partial_plans_per_s": r0["partial_plans"] / (statistics.median(
            r["ms_explore"] for r in results) / 1e3),
        "simulated_partial_plans_per_s": r0["simulated"] * args.steps / total_s,
        "partial_plans_per_query": r0["partial_plans"],
        "simulated_per_query": r0["simulated"],
        "preprune_per_query": r0["preprune"],
        "inserted_per_query": r0["inserted"],
        "sim_waypoints_per_query": r0["sim_waypoints"],
        "sim_box_tests_per_query": r0["sim_box_tests"],
        "flagged_per_query": r0["flagged"],
        "n_edges": r0["n_edges"],
        "rounds": r0["rounds"],
        "stage_ms": {"setup": statistics.median(r["ms_setup"] for r in results),
                     "explore": statistics.median(r["ms_explore"] for r in results),
                     "select": statistics.median(r["ms_select"] for r in results)},
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kt.items() if v[1]},
        "roofline": roofline,
    }
    if "roadmap" in legs:
        line["roadmap"] = roadmap_leg(pl, samples, pr, r0, min(args.steps, 10))
    pl.close()
    if "cfg2" in legs:
        line["boxes_4000"] = boxes_leg(stream, args.seed, args.warmup, args.steps)
    if "batch" in legs and args.batch_queries > 0:
        line["batched"] = batched_leg(args.batch_queries, args.seed, args.batch_steps,
                                      min(args.tune_queries, args.batch_queries))
    if "hsmc" in legs:
        line["hsmc_4000"] = hsmc_leg(stream, args.seed, args.warmup, min(args.steps, 10))
    if "learned" in legs:
        line["learned"] = learned_leg(args.learned_maps)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
