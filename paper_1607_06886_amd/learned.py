"""Learned sampling proposal driver: data from plain PUMP, training on the
device, and plain-vs-learned evaluation.

Every numerical step runs in libpump kernels (planning, condition vectors,
MLP forward/backward/Adam, mixture sampling); this module only moves arrays
and keeps score.  A learned query draws half of its n samples from the
network's mixture and half uniformly (with the usual goal-box share), then
runs plain PUMP on them; the plan it returns is certified by MC(p) exactly as
in the plain method (Alg. 5), so the CP guarantee is unchanged.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

from . import _lib, scenes

MAX_BOXES = 64


def _torch():
    import torch
    return torch


def device_noise(S, N, M, seed):
    """Standard normals for the exploration and certification particles."""
    torch = _torch()
    g = torch.Generator(device="cuda")
    g.manual_seed(int(seed))
    noise = torch.randn((S, 6, N), generator=g, device="cuda", dtype=torch.float32)
    noise_mc = torch.randn((S, 6, M), generator=g, device="cuda", dtype=torch.float32)
    return noise, noise_mc


class Runner:
    """A planner context plus shared device noise for many queries."""

    def __init__(self, n_max, N, S_max=256, M=2000, seed=0, n_obs_max=64, cap_pairs=1 << 23):
        self.N, self.S_max, self.M = N, S_max, M
        self.pl = _lib.Planner(n_particles=N, max_nodes=n_max + 1, max_obstacles=n_obs_max,
                               max_steps=S_max, mc_particles=M, cap_plans=1 << 21,
                               cap_pairs=cap_pairs, cap_edges=1 << 25)
        self.noise, self.noise_mc = device_noise(S_max, N, M, seed)

    def plan(self, x_init, goal, boxes, samples, alpha, sigma):
        torch = _torch()
        s = samples if not isinstance(samples, np.ndarray) else torch.from_numpy(samples).cuda()
        b = torch.from_numpy(np.ascontiguousarray(boxes, np.float32)).cuda()
        pr = self.pl.problem(s, b, x_init, goal, alpha, sigma, self.noise, self.noise_mc)
        t0 = time.perf_counter()
        try:
            res = self.pl.plan(pr)
        except _lib.PumpError as e:
            # a workspace limit: the query counts as not certified
            return dict(status=e.code, best_cost=math.inf, best_cp_mc=math.nan,
                        ms_total=1e3 * (time.perf_counter() - t0), partial_plans=0), None
        path = self.pl.path(res["best_plan"]) if res["status"] == 0 else None
        return res, path

    def close(self):
        self.pl.close()


def condition_batch(mlp, maps):
    """Condition vectors [q, 396] (device) for a list of (x_init, goal, boxes)."""
    torch = _torch()
    q = len(maps)
    x0 = np.stack([m[0] for m in maps]).astype(np.float32)
    g = np.stack([m[1] for m in maps]).astype(np.float32)
    bx = np.zeros((q, MAX_BOXES, 6), np.float32)
    nb = np.zeros(q, np.int32)
    for i, m in enumerate(maps):
        k = min(MAX_BOXES, m[2].shape[0])
        bx[i, :k] = m[2][:k]
        nb[i] = k
    t = lambda a: torch.from_numpy(a).cuda()
    return mlp.condition(t(x0), t(g), t(bx), t(nb))


def generate(n_queries, kinds, n_samples, N, alpha, sigma, seed0, log=None):
    """Certified plans of plain PUMP on random maps: returns the maps, and per
    certified plan its map index and node states (x_init excluded)."""
    run = Runner(n_samples, N, seed=seed0)
    maps, plans = [], []
    t0 = time.time()
    for q in range(n_queries):
        kind = kinds[q % len(kinds)]
        x0, g, b = scenes.random_map(kind, seed0 + q)
        smp = scenes.uniform_samples(seed0 + q, n_samples, b, g)
        res, path = run.plan(x0, g, b, smp, alpha, sigma)
        maps.append((x0, g, b))
        if path is not None and len(path) > 1:
            plans.append((q, smp[np.asarray(path[1:]) - 1]))
        if log and (q + 1) % 500 == 0:
            log(f"generated {q + 1}/{n_queries} queries, {len(plans)} certified plans, "
                f"{time.time() - t0:.0f} s")
    run.close()
    return maps, plans


def _map_and_samples(args):
    """One training map and its uniform samples (worker of generate_batched)."""
    kind, seed, n = args
    x0, g, b = scenes.random_map(kind, seed)
    return x0, g, b, scenes.uniform_samples(seed, n, b, g)


def map_pool(procs=0):
    """Worker processes that draw maps and samples.  Create it before the
    process first touches the GPU: the workers are forked copies."""
    import multiprocessing as mp
    return mp.get_context("fork").Pool(procs or min(16, os.cpu_count() or 1))


def generate_batched(pool, n_queries, kinds, n_samples, N, alpha, sigma, seed0, want_plans=None,
                     batch=256, log=None):
    """generate() through the batched engine: maps are drawn by `pool`
    (map_pool) and planned `batch` at a time in one graph launch each (shared
    particle noise, as Runner does).  Stops early once `want_plans` certified
    plans are in hand.  Returns (maps, plans) like generate()."""
    torch = _torch()
    S_max, M = 256, 2000
    noise, noise_mc = device_noise(S_max, N, M, seed0)
    b = _lib.Batch(batch, n_particles=N, max_nodes=n_samples + 1, max_obstacles=MAX_BOXES,
                   max_steps=S_max, mc_particles=M, cap_plans=1 << 20, cap_pairs=1 << 21,
                   cap_edges=1 << 22)
    maps, plans = [], []
    t0 = time.time()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    for q0 in range(0, n_queries, batch):
        jobs = [(kinds[q % len(kinds)], seed0 + q, n_samples)
                for q in range(q0, min(n_queries, q0 + batch))]
        drawn = pool.map(_map_and_samples, jobs, chunksize=8)
        queries = [(dev(smp), dev(bx), x0, g, alpha, sigma, noise, noise_mc)
                   for x0, g, bx, smp in drawn]
        res = b.plan(queries, raise_on_error=False)
        for i, (r, (x0, g, bx, smp)) in enumerate(zip(res, drawn)):
            maps.append((x0, g, bx))
            if r["status"] == 0:
                path = b.path(i, r["best_plan"])
                if len(path) > 1:
                    plans.append((q0 + i, smp[np.asarray(path[1:]) - 1]))
        if log:
            log(f"generated {len(maps)}/{n_queries} queries, {len(plans)} certified plans, "
                f"{time.time() - t0:.0f} s")
        if want_plans and len(plans) >= want_plans:
            break
    b.close()
    return maps, plans


def train(mlp, maps, plans, steps, batch, lr, seed, log=None):
    """Adam on the mean mixture NLL of certified-plan node states given their
    map's condition vector."""
    torch = _torch()
    cond_all = condition_batch(mlp, maps)                    # [n_maps, 396] device
    idx = np.concatenate([np.full(len(st), q, np.int64) for q, st in plans])
    tgt = torch.from_numpy(np.concatenate([st for _, st in plans]).astype(np.float32)).cuda()
    idx_t = torch.from_numpy(idx).cuda()
    rng = np.random.default_rng(seed)
    losses = []
    for s in range(steps):
        sel = torch.from_numpy(rng.integers(0, idx.shape[0], batch)).cuda()
        c = cond_all.index_select(0, idx_t.index_select(0, sel)).contiguous()
        z = tgt.index_select(0, sel).contiguous()
        losses.append(mlp.train_step(c, z, lr))
        if log and (s + 1) % 500 == 0:
            log(f"step {s + 1}: loss {np.mean(losses[-100:]):.3f}")
    return losses


def learned_samples(mlp, x0, g, b, n, seed):
    """n states: n // 2 from the mixture, the rest uniform (with the goal
    share).  Returns a device tensor [n, 6] and the sampling time in ms."""
    torch = _torch()
    n_l = n // 2
    uni = scenes.uniform_samples(seed, n - n_l, b, g)
    rng = np.random.default_rng(seed + 17)
    u = torch.from_numpy(rng.uniform(0, 1, (1, n_l)).astype(np.float32)).cuda()
    eps = torch.from_numpy(rng.standard_normal((1, n_l, 6)).astype(np.float32)).cuda()
    uni_t = torch.from_numpy(uni).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cond = condition_batch(mlp, [(x0, g, b)])
    z = mlp.sample(cond, u, eps)[0]
    out = torch.cat([z, uni_t], 0).contiguous()
    torch.cuda.synchronize()
    return out, 1e3 * (time.perf_counter() - t0)


def evaluate(mlp, n_maps, kinds, sizes, N, alpha, sigma, seed0, log=None, M=10_000, S_max=512):
    """Plain (n uniform) vs learned (n/2 mixture + n/2 uniform) on held-out maps,
    certified with M particles over S_max steps."""
    run = Runner(max(sizes), N, S_max=S_max, M=M, seed=seed0 + 99, cap_pairs=1 << 24)
    rows = []
    for q in range(n_maps):
        kind = kinds[q % len(kinds)]
        x0, g, b = scenes.random_map(kind, seed0 + q)
        for n in sizes:
            smp = scenes.uniform_samples(seed0 + q, n, b, g)
            rp, _ = run.plan(x0, g, b, smp, alpha, sigma)
            ls, ms_s = learned_samples(mlp, x0, g, b, n, seed0 + q)
            rl, _ = run.plan(x0, g, b, ls, alpha, sigma)
            rows.append(dict(map=q, kind=kind, n=n,
                             plain_status=rp["status"], plain_cost=rp["best_cost"],
                             plain_cp=rp["best_cp_mc"], plain_ms=rp["ms_total"],
                             plain_pairs=rp["partial_plans"],
                             learned_status=rl["status"], learned_cost=rl["best_cost"],
                             learned_cp=rl["best_cp_mc"], learned_ms=rl["ms_total"] + ms_s,
                             learned_pairs=rl["partial_plans"]))
        if log and (q + 1) % 10 == 0:
            log(f"evaluated {q + 1}/{n_maps} maps")
    run.close()
    return rows


def summarise(rows, sizes):
    """Per sample count: certification rates, costs where both certify, CP and
    median times.  Across counts: for learned at n_l against plain at n_p, the
    share of maps where learned certifies a plan at least as cheap as plain's
    (plain uncertified counts as infinite cost) and the ratio of median times."""
    out = {}
    for n in sizes:
        r = [x for x in rows if x["n"] == n]
        ok_p = [x for x in r if x["plain_status"] == 0]
        ok_l = [x for x in r if x["learned_status"] == 0]
        both = [x for x in r if x["plain_status"] == 0 and x["learned_status"] == 0]
        out[n] = dict(
            maps=len(r), plain_certified=len(ok_p), learned_certified=len(ok_l),
            mean_plain_cost=float(np.mean([x["plain_cost"] for x in both])) if both else None,
            mean_learned_cost=float(np.mean([x["learned_cost"] for x in both])) if both else None,
            learned_le_plain=float(np.mean([x["learned_cost"] <= x["plain_cost"] + 1e-12
                                           for x in both])) if both else None,
            max_cp_plain=max([x["plain_cp"] for x in ok_p], default=None),
            max_cp_learned=max([x["learned_cp"] for x in ok_l], default=None),
            median_plain_ms=float(np.median([x["plain_ms"] for x in r])),
            median_learned_ms=float(np.median([x["learned_ms"] for x in r])),
            median_plain_pairs=float(np.median([x["plain_pairs"] for x in r])),
            median_learned_pairs=float(np.median([x["learned_pairs"] for x in r])),
        )
    cross = {}
    by = {(x["map"], x["n"]): x for x in rows}
    maps = sorted({x["map"] for x in rows})
    for nl in sizes:
        for np_ in sizes:
            wins, tl, tp = [], [], []
            for m in maps:
                a, b = by.get((m, nl)), by.get((m, np_))
                if a is None or b is None:
                    continue
                cl = a["learned_cost"] if a["learned_status"] == 0 else math.inf
                cp = b["plain_cost"] if b["plain_status"] == 0 else math.inf
                if math.isinf(cl) and math.isinf(cp):
                    continue
                wins.append(cl <= cp + 1e-12)
                tl.append(a["learned_ms"])
                tp.append(b["plain_ms"])
            if wins:
                cross[f"learned@{nl} vs plain@{np_}"] = dict(
                    maps=len(wins), learned_le_plain=float(np.mean(wins)),
                    median_ms_ratio=float(np.median(tl) / max(1e-9, np.median(tp))))
    return dict(per_n=out, cross=cross)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--queries", type=int, default=72000)
    ap.add_argument("--want-plans", type=int, default=50000)
    ap.add_argument("--n-train", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=2048)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-maps", type=int, default=100)
    ap.add_argument("--sizes", type=str, default="1000,2000,4000,8000")
    ap.add_argument("--out", type=str, default="learned.json")
    ap.add_argument("--state", type=str, default="", help="save the training state (.npz)")
    ap.add_argument("--params", type=str, default="",
                    help="save the trained FP32 parameters (.npy) for inference")
    args = ap.parse_args()
    pool = map_pool()                 # before the GPU is touched: forked workers
    torch = _torch()
    torch.cuda.set_device(0)
    log = lambda m: print(m, flush=True)
    kinds = ["boxes", "indoor"]
    t0 = time.time()
    maps, plans = generate_batched(pool, args.queries, kinds, args.n_train, 128, 0.01, 0.02,
                                   10_000, want_plans=args.want_plans, log=log)
    pool.close()
    t_gen = time.time() - t0
    log(f"data: {len(plans)} certified plans of {len(maps)} queries in {t_gen:.0f} s")
    mlp = _lib.MLP(max(args.batch, 64))
    mlp.set_params(init_params(7))
    t1 = time.time()
    losses = train(mlp, maps, plans, args.steps, args.batch, args.lr, 8, log)
    t_train = time.time() - t1
    log(f"trained {args.steps} steps in {t_train:.1f} s: "
        f"loss {np.mean(losses[:50]):.3f} -> {np.mean(losses[-50:]):.3f}")
    if args.state:
        mlp.save(args.state)
    if args.params:
        os.makedirs(os.path.dirname(args.params) or ".", exist_ok=True)
        np.save(args.params, mlp.get_params())
    sizes = [int(x) for x in args.sizes.split(",")]
    rows = evaluate(mlp, args.eval_maps, kinds, sizes, 256, 0.01, 0.02, 900_000, log)
    summary = dict(queries=len(maps), certified_plans=len(plans),
                   targets=int(sum(len(st) for _, st in plans)), generate_s=t_gen,
                   steps=args.steps, batch=args.batch, lr=args.lr, train_s=t_train,
                   loss_first=float(np.mean(losses[:50])),
                   loss_last=float(np.mean(losses[-50:])), eval=summarise(rows, sizes))
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(dict(summary=summary, rows=rows), f)
    log(json.dumps(summary))
    mlp.close()


def init_params(seed):
    """He-uniform weights and zero biases, flat in the library's layout."""
    rng = np.random.default_rng(seed)
    dims = [(396, 256), (256, 256), (256, 256), (256, 256), (256, 208)]
    parts = []
    for fi, fo in dims:
        lim = math.sqrt(6.0 / fi)
        parts.append(rng.uniform(-lim, lim, fo * fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


if __name__ == "__main__":
    main()
