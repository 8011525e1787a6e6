"""SampleFree(n) with the Halton sequence (oracle, exact then FP32).

Test infrastructure only: it checks the HIP path and is never called by it.

The paper samples the state space with the deterministic low-dispersion
Halton sequence (Sec. V-A) for SampleFree (Alg. 3).  Halton point i (i >= 1)
has coordinate d equal to the radical inverse of i in the d-th prime base:
write i in base b, mirror its digits about the radix point.

Readings (the paper fixes none of them):
  * the six state coordinates (px, py, pz, vx, vy, vz) use the bases
    2, 3, 5, 7, 11, 13 in that order; point i maps to lo + (hi - lo) * phi
    per coordinate over the sampling box [lo, hi];
  * the sequence starts at index `start` (default 1: index 0 is the origin);
  * the radical inverse is the exact fraction R / b^k (R the mirrored digits,
    k the digit count) rounded once to FP64; lo + (hi - lo) * phi is rounded
    after each operation in FP64 and stored in FP32;
  * SampleFree(n) with a goal region ("including at least one from X_goal"):
    the first n - n_goal points cover the state box, the next n_goal
    points of the sequence (default max(1, n // 100), the 1% goal share of
    the uniform inputs) cover the goal box's positions (velocities over the
    state box's velocity range);
    samples that land in obstacles are kept as nodes without edges, as for
    uniform samples.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np

BASES = (2, 3, 5, 7, 11, 13)


def radical_inverse_fraction(i: int, b: int) -> Fraction:
    """phi_b(i) as an exact fraction."""
    num, den = 0, 1
    while i > 0:
        i, digit = divmod(i, b)
        num = num * b + digit
        den *= b
    return Fraction(num, den)


def radical_inverse(i: int, b: int) -> float:
    """phi_b(i) rounded once to FP64."""
    return float(radical_inverse_fraction(i, b))


def halton(start: int, n: int, lo, hi) -> np.ndarray:
    """Points start .. start + n - 1 of the 6-D Halton sequence over the box
    [lo, hi] (6 floats each), as FP32 [n, 6]."""
    lo = np.asarray(lo, np.float32).astype(np.float64)
    hi = np.asarray(hi, np.float32).astype(np.float64)
    out = np.zeros((n, 6), np.float32)
    for r in range(n):
        i = start + r
        for d, b in enumerate(BASES):
            phi = radical_inverse(i, b)
            out[r, d] = np.float32((lo[d] + (hi[d] - lo[d]) * phi))
    return out


def sample_free_halton(n: int, lo, hi, goal_lo, goal_hi, n_goal=None, start=1):
    """SampleFree(n) as in the module header: [n, 6] FP32."""
    if n_goal is None:
        n_goal = max(1, n // 100)
    n_box = n - n_goal
    a = halton(start, n_box, lo, hi)
    glo = np.array([*np.asarray(goal_lo, np.float32)[:3], *np.asarray(lo, np.float32)[3:]])
    ghi = np.array([*np.asarray(goal_hi, np.float32)[:3], *np.asarray(hi, np.float32)[3:]])
    g = halton(start + n_box, n_goal, glo, ghi)
    return np.concatenate([a, g], axis=0)
