"""The learned proposal at its evaluation size: 8000 samples, 256 particles,
alpha = 0.01, sigma = 0.02, M = 10^4, on held-out maps (half random boxes,
half indoor; seeds disjoint from the training maps), with the network that
`python -m paper_1607_06886_amd.learned` trained on the GPU on 50,000
certified plans of plain PUMP (paper_1607_06886_amd/weights).

What it must show: every plan either way is certified (MC <= alpha); at
8000 samples the learned samples (4000 network + 4000 uniform) reach a lower
mean certified cost than 8000 uniform samples where both certify; and the
learned proposal with 2000 samples (1000 + 1000) reaches a certified cost at
least as low as plain PUMP's with 8000 on most maps in less time."""

import math
import os

import numpy as np
import pytest

from paper_1607_06886_amd import _lib, learned
from tests._gpu import print_case

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1607_06886_amd", "weights", "proposal_params.npy")
ALPHA = 0.01


def test_learned_against_plain_at_8000_samples():
    print_case("learned_config5", maps=40)
    mlp = _lib.MLP(64)
    mlp.set_params(np.load(WEIGHTS, allow_pickle=False))
    log = lambda m: print("  " + m, flush=True)
    rows = learned.evaluate(mlp, 40, ["boxes", "indoor"], [2000, 8000], 256, ALPHA, 0.02,
                            900_000, log)
    mlp.close()
    for r in rows:
        if r["learned_status"] == 0:
            assert r["learned_cp"] <= ALPHA
        if r["plain_status"] == 0:
            assert r["plain_cp"] <= ALPHA
    by = {(r["map"], r["n"]): r for r in rows}
    maps = sorted({r["map"] for r in rows})
    both = [by[(m, 8000)] for m in maps
            if by[(m, 8000)]["plain_status"] == 0 and by[(m, 8000)]["learned_status"] == 0]
    mean_p = float(np.mean([r["plain_cost"] for r in both]))
    mean_l = float(np.mean([r["learned_cost"] for r in both]))
    print(f"  at 8000 samples: {len(both)} maps certified both ways, mean cost plain {mean_p:.4f},"
          f" learned {mean_l:.4f}", flush=True)
    assert len(both) >= 12 and mean_l < mean_p
    wins, ratios = [], []
    for m in maps:
        a, b = by[(m, 2000)], by[(m, 8000)]
        cl = a["learned_cost"] if a["learned_status"] == 0 else math.inf
        cp = b["plain_cost"] if b["plain_status"] == 0 else math.inf
        if math.isinf(cl) and math.isinf(cp):
            continue
        wins.append(cl <= cp + 1e-12)
        ratios.append(a["learned_ms"] / b["plain_ms"])
    share, ratio = float(np.mean(wins)), float(np.median(ratios))
    print(f"  learned@2000 vs plain@8000: cost <= plain on {share:.2f} of {len(wins)} maps, "
          f"median time ratio {ratio:.2f}", flush=True)
    assert share >= 0.6 and ratio < 1.0
