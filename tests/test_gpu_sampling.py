"""Halton SampleFree on the device (pump_sample_halton) against the oracle's
exact radical inverses, bit for bit, and a query planned on Halton samples."""

import dataclasses

import numpy as np
import pytest

from oracle import pump as opump, sampling as osmp
from paper_1607_06886_amd import _lib, scenes
from tests._gpu import planner_for, print_case, small_spec

pytestmark = pytest.mark.gpu

LO = [0.0, 0.0, 0.0, -0.5, -0.5, -0.5]
HI = [1.0, 1.0, 1.0, 0.5, 0.5, 0.5]
GOAL = [0.85, 0.85, 0.85, 0.95, 0.95, 0.95]


def test_halton_equals_oracle_bit_for_bit():
    print_case("halton", n=5000)
    got = _lib.sample_halton(5000, LO, HI, goal=GOAL).cpu().numpy()
    want = osmp.sample_free_halton(5000, LO, HI, GOAL[:3], GOAL[3:])
    np.testing.assert_array_equal(got, want)
    # an odd box, no goal block, a later start
    lo = [-0.3, 0.1, 2.0, -1.0, 0.0, -0.25]
    hi = [0.7, 0.35, 2.5, 1.0, 0.125, 0.25]
    got = _lib.sample_halton(3000, lo, hi, start=123456).cpu().numpy()
    np.testing.assert_array_equal(got, osmp.halton(123456, 3000, lo, hi))


def test_halton_near_the_index_limit():
    start = (1 << 31) - 2001
    print_case("halton_limit", start=start)
    got = _lib.sample_halton(2000, LO, HI, start=start).cpu().numpy()
    np.testing.assert_array_equal(got, osmp.halton(start, 2000, LO, HI))
    with pytest.raises(_lib.PumpError):
        _lib.sample_halton(2000, LO, HI, start=start + 1)
    with pytest.raises(_lib.PumpError):
        _lib.sample_halton(10, LO, HI, goal=GOAL, n_goal=11)
    with pytest.raises(_lib.PumpError):
        _lib.sample_halton(10, HI, LO)


def test_plan_on_halton_samples_matches_oracle():
    print_case("halton_plan")
    sc = scenes.make_scene(small_spec(n=600, N=64, sigma=0.02, alpha=0.05, n_obs=8), 77, M=2000,
                           S_max=256)
    smp = _lib.sample_halton(600, LO, HI, goal=sc.goal)
    sc = dataclasses.replace(sc, samples=smp.cpu().numpy())
    np.testing.assert_array_equal(sc.samples, osmp.sample_free_halton(600, LO, HI, sc.goal[:3],
                                                                      sc.goal[3:]))
    ref = opump.run(sc, opump.Config())
    pl = planner_for(sc)
    res = pl.plan(pl.scene_problem(sc))
    assert res["status"] == ref["status"]
    assert res["partial_plans"] == ref["stats"]["partial_plans"]
    assert res["n_edges"] == int(ref["graph"]["col"].shape[0])
    if ref["status"] == 0:
        assert pl.path(res["best_plan"]) == ref["best"].nodes
    pl.close()
