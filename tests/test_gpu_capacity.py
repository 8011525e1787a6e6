"""Capacity failures (failure detection): workspaces sized too small for a
query make pump_plan return PUMP_E_CAPACITY (-2) with the size it needed in
the message, never write past a buffer, and leave the context usable; a
context sized from the reported numbers then plans the query and matches a
roomy context.  Checked for the graph (cap_edges), BuildGraph's exact
queue (cap_pairs) and the plan store (cap_plans), in both Explore modes.
(A round with more pairs than cap_pairs runs in chunks instead:
tests/test_gpu_chunked_rounds.py.)"""

import re

import pytest

from paper_1607_06886_amd import _lib
from tests._gpu import planner_for, print_case, scene

pytestmark = pytest.mark.gpu

KEYS = ("status", "partial_plans", "rounds", "n_plans", "best_plan", "best_cost", "best_mc_count")


def _needed(err, pattern):
    m = re.search(pattern, str(err))
    assert m, str(err)
    return int(m.group(1))


@pytest.fixture(scope="module")
def ref():
    sc = scene("boxes20", 1)
    pl = planner_for(sc)
    r = pl.plan(pl.scene_problem(sc))
    pl.close()
    return sc, r


def _plan(sc, mode, **caps):
    pl = planner_for(sc, **caps)
    pl.set_explore_mode(mode)
    try:
        return pl, pl.plan(pl.scene_problem(sc))
    except _lib.PumpError:
        pl.close()
        raise


@pytest.mark.parametrize("mode", [1, 0])
def test_edges_pairs_and_plans_too_small(ref, mode):
    sc, r = ref
    print_case("capacity", mode=mode, partial_plans=r["partial_plans"], n_plans=r["n_plans"])
    # the graph
    with pytest.raises(_lib.PumpError) as ei:
        _plan(sc, mode, cap_edges=1000)
    assert ei.value.code == -2
    need_e = _needed(ei.value, r"(?:near connections|graph edges) (\d+) exceed cap_edges")
    assert need_e > 1000
    # BuildGraph's exact queue (connection, box) shares cap_pairs
    with pytest.raises(_lib.PumpError) as ei:
        _plan(sc, mode, cap_pairs=4)
    assert ei.value.code == -2
    need_q = _needed(ei.value, r"exact box tests (\d+) exceed cap_pairs")
    assert need_q > 4
    # the plan store
    with pytest.raises(_lib.PumpError) as ei:
        _plan(sc, mode, cap_plans=r["n_plans"] // 3)
    assert ei.value.code == -2
    need_p = _needed(ei.value, r"plan store needs (\d+) plans")
    assert need_p > r["n_plans"] // 3
    # sized from the numbers reported, the query runs as in a roomy context
    # (the cap_edges figure covers the near list; the plan store may still
    # need more in a later round, so it is raised to the final count)
    pl, got = _plan(sc, mode, cap_edges=need_e, cap_plans=max(need_p, r["n_plans"]))
    for k in KEYS:
        assert got[k] == r[k], k
    pl.close()
    # a failed call leaves the context as it was: the same call fails the
    # same way again
    pl = planner_for(sc, cap_plans=r["n_plans"] // 3)
    pl.set_explore_mode(mode)
    msgs = []
    for _ in range(2):
        with pytest.raises(_lib.PumpError) as ei:
            pl.plan(pl.scene_problem(sc))
        msgs.append(str(ei.value))
    assert msgs[0] == msgs[1]
    pl.close()
