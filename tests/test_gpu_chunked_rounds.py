"""Rounds of Explore with more pairs than candidate slots (cap_pairs) run in
chunks, in two passes (RemoveDominated depends only on each node's final
staircase): the plan store, the front and p* must equal those of the round
in one piece, bit for bit, plan ids included, in the per-phase mode and
through the single launch's fallback to it.  The round in one piece is itself
compared with the oracle plan by plan in tests/test_gpu_parity.py."""

import re

import numpy as np
import pytest

from paper_1607_06886_amd import _lib, scenes
from tests._gpu import planner_for, print_case, scene, small_spec

pytestmark = pytest.mark.gpu

KEYS = ("status", "partial_plans", "rounds", "final_i", "n_plans", "n_front", "best_plan",
        "best_cost", "best_mc_count", "best_pop")
STORE = ("head", "parent", "edge", "cost", "step", "pop", "round", "state", "mask")


def _scene(kind):
    if kind == "free":
        # obstacle-free: no exact box tests share cap_pairs
        return scenes.make_scene(small_spec(n=300, N=32, n_obs=0), 31, M=256, S_max=128)
    return scene(kind, 2)


def _round_pairs(sc):
    """Pairs of every round of the query in one piece (roomy context)."""
    pl = planner_for(sc)
    pl.set_explore_mode(0)
    pl.setup(pl.scene_problem(sc))
    pl.explore_begin()
    pairs = []
    done = False
    while not done:
        done = pl.explore_round()
        pairs.append(len(pl.candidates()["flag"]))
    pl.close()
    return pairs


def _run(sc, mode, **caps):
    pl = planner_for(sc, **caps)
    pl.set_explore_mode(mode)
    r = pl.plan(pl.scene_problem(sc))
    st = pl.plans()
    ids, mc = pl.front()
    out = dict(res=r, store=st, front=(ids.copy(), mc.copy()), chunked=pl.chunked_rounds(),
               fallbacks=pl.explore_fallbacks())
    pl.close()
    return out


@pytest.mark.parametrize("kind", ["free", "boxes20", "indoor"])
@pytest.mark.parametrize("mode", [0, 1])
def test_round_in_chunks_equals_round_in_one_piece(kind, mode):
    sc = _scene(kind)
    pairs = _round_pairs(sc)
    big = max(pairs)
    cap = max(big // 5, 32)
    ref = _run(sc, 0)
    try:
        got = _run(sc, mode, cap_pairs=cap)
    except _lib.PumpError as e:
        # BuildGraph's exact queue shares cap_pairs; take what it needs
        m = re.search(r"exact box tests (\d+) exceed cap_pairs", str(e))
        assert m, str(e)
        cap = int(m.group(1))
        got = _run(sc, mode, cap_pairs=cap)
    n_chunked = sum(1 for p in pairs if p > cap)
    print_case("chunked rounds", kind=kind, mode=mode, cap_pairs=cap, max_round_pairs=big,
               rounds_over_cap=n_chunked, chunked=got["chunked"], fallbacks=got["fallbacks"])
    if kind == "free":
        assert n_chunked > 0
    assert got["chunked"] == n_chunked
    if mode == 1 and n_chunked:
        assert got["fallbacks"] == 1   # the single launch met a round over cap_pairs
    for k in KEYS:
        assert got["res"][k] == ref["res"][k], k
    for k in STORE:
        np.testing.assert_array_equal(got["store"][k], ref["store"][k], err_msg=k)
    for a, b in zip(got["front"], ref["front"]):
        np.testing.assert_array_equal(a, b)


def test_candidates_of_a_chunked_round_are_not_kept():
    sc = _scene("free")
    big = max(_round_pairs(sc))
    pl = planner_for(sc, cap_pairs=max(big // 5, 32))
    pl.set_explore_mode(0)
    pl.setup(pl.scene_problem(sc))
    pl.explore_begin()
    done = False
    saw = False
    while not done:
        before = pl.chunked_rounds()
        done = pl.explore_round()
        if pl.chunked_rounds() > before:
            saw = True
            with pytest.raises(_lib.PumpError) as ei:
                pl.candidates()
            assert "chunks" in str(ei.value)
        else:
            pl.candidates()
    assert saw
    pl.close()
