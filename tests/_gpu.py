"""Helpers shared by the GPU parity tests (not collected by pytest)."""

from __future__ import annotations

import functools

import numpy as np

from oracle import pump as opump
from paper_1607_06886_amd import _lib, scenes

CFG = opump.Config()


def small_spec(n=150, N=32, sigma=0.02, alpha=0.05, n_obs=3, side=(0.1, 0.3)):
    return dict(n=n, n_obs=n_obs, side=side, N=N, sigma=sigma, alpha=alpha, indoor=False)


def planner_for(sc, **over):
    kw = dict(n_particles=sc.N, max_nodes=sc.n + 1, max_obstacles=max(sc.n_obs, 1),
              max_steps=sc.S_max, mc_particles=sc.M, cap_plans=1 << 20, cap_pairs=1 << 22,
              cap_edges=1 << 24)
    kw.update(over)
    return _lib.Planner(**kw)


def gpu_plans(pl):
    st = pl.plans()
    st["paths"] = _lib.plan_paths(st)
    return st


def unpack_mask(words, N):
    """uint32 words -> bool[N] (bit j of word j // 32)."""
    w = np.asarray(words, np.uint32)
    bits = (w[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1
    return bits.reshape(-1)[:N].astype(bool)


def oracle_mask_bool(packed, N):
    return np.unpackbits(packed, bitorder="little")[:N].astype(bool)


def mask_words_from_bool(m):
    m = np.asarray(m, bool)
    pad = (-m.shape[0]) % 32
    m = np.concatenate([m, np.zeros(pad, bool)]).reshape(-1, 32)
    return (m.astype(np.uint64) << np.arange(32, dtype=np.uint64)).sum(1).astype(np.uint32)


def print_case(name, **kw):
    print(f"[gpu case] {name} {kw}", flush=True)


def scene(kind, seed, sigma_meas=0.0):
    """Parity scenes (M = 2000 certification particles, S_max = 256);
    sigma_meas > 0 adds the measurement noise of LQG tracking."""
    kw = dict(M=2000, S_max=256, sigma_meas=sigma_meas)
    if kind == "cfg1":
        return scenes.make_scene("cfg1", scenes.workload_seed(1, seed), **kw)
    if kind == "boxes20":
        return scenes.make_scene(small_spec(n=400, N=128, sigma=0.02, alpha=0.01, n_obs=20,
                                            side=(0.05, 0.25)), 500 + seed, **kw)
    if kind == "indoor":
        return scenes.make_scene(dict(n=450, n_obs=60, side=None, N=128, sigma=0.02, alpha=0.05,
                                      indoor=True), 700 + seed, **kw)
    if kind == "n64":
        return scenes.make_scene(small_spec(n=250, N=64, sigma=0.03, alpha=0.05, n_obs=8),
                                 900 + seed, **kw)
    if kind == "n256":
        return scenes.make_scene(small_spec(n=300, N=256, sigma=0.02, alpha=0.02, n_obs=12,
                                            side=(0.05, 0.25)), 950 + seed, **kw)
    raise ValueError(kind)


@functools.lru_cache(maxsize=None)
def oracle_run(kind, seed):
    return opump.run(scene(kind, seed), CFG, record=True)


# measurement-noise intensity of the LQG parity scenes (half the process
# noise of the cfg1 workload)
SIGMA_MEAS = 0.01


@functools.lru_cache(maxsize=None)
def oracle_run_lqg(kind, seed):
    return opump.run(scene(kind, seed, SIGMA_MEAS), opump.Config(estimator="lqg"), record=True)


def assert_bits_except_flagged(got, want, flagged, what=""):
    """Particle bits equal the oracle's except where the oracle flags the
    decision (the particle came within 1e-5 of a face and nowhere lay 1e-5 or
    more inside).  Returns how many flagged bits differ, for reporting."""
    diff = np.asarray(got, bool) ^ np.asarray(want, bool)
    fl = np.zeros_like(diff) if flagged is None else np.asarray(flagged, bool)
    bad = diff & ~fl
    assert not bad.any(), (what, np.nonzero(bad)[0])
    return int((diff & fl).sum())


def assert_table_is_fp32_of(D, Dref, tol=1e-5):
    """An FP32 table from the device against the oracle's FP64 table: within
    `tol` relative to max(|x|, 1) everywhere, and equal to the FP64 value
    rounded to FP32 except in rare entries one FP32 ulp away (the two sides
    compute their gains and recurrences independently)."""
    D = np.asarray(D, np.float32)
    assert D.shape == Dref.shape
    scale = max(1.0, float(np.abs(Dref).max()))
    np.testing.assert_allclose(D.astype(np.float64), Dref, rtol=0, atol=tol * scale)
    R = Dref.astype(np.float32)
    diff = D != R
    assert diff.mean() < 1e-4, int(diff.sum())
    ulp = np.abs(D.view(np.int32)[diff].astype(np.int64) - R.view(np.int32)[diff])
    assert ulp.size == 0 or ulp.max() <= 1
    return int(diff.sum())
