"""Pins of the oracle's Halton SampleFree (oracle/sampling.py) against the
sequence's defining values and its stratification properties."""

from fractions import Fraction

import numpy as np
import pytest

from oracle import sampling as smp


def test_van_der_corput_values():
    assert [smp.radical_inverse_fraction(i, 2) for i in range(1, 8)] == [
        Fraction(1, 2), Fraction(1, 4), Fraction(3, 4), Fraction(1, 8), Fraction(5, 8),
        Fraction(3, 8), Fraction(7, 8)]
    assert [smp.radical_inverse_fraction(i, 3) for i in range(1, 7)] == [
        Fraction(1, 3), Fraction(2, 3), Fraction(1, 9), Fraction(4, 9), Fraction(7, 9),
        Fraction(2, 9)]
    # 1234 = 1*5^4 + 4*5^3 + 4*5^2 + 1*5 + 4 -> mirrored 4 1 4 4 1 over 5^5
    assert smp.radical_inverse_fraction(1234, 5) == Fraction(4 * 625 + 1 * 125 + 4 * 25 + 4 * 5 + 1,
                                                             5 ** 5)
    assert smp.radical_inverse_fraction(0, 7) == 0


@pytest.mark.parametrize("b", smp.BASES)
def test_each_coordinate_is_stratified(b):
    """Indices 0 .. b^k - 1 put exactly one point in each interval
    [j / b^k, (j + 1) / b^k)."""
    for k in (1, 2, 3):
        n = b ** k
        if n > 3000:
            continue
        cells = sorted(int(smp.radical_inverse_fraction(i, b) * n) for i in range(n))
        assert cells == list(range(n))


def test_pairs_of_coordinates_are_jointly_stratified():
    """Halton's elementary intervals: 2^a 3^c consecutive points from 0 put one
    point in each cell of a 2^a x 3^c grid (bases 2 and 3, coprime)."""
    for a, c in ((2, 1), (3, 2), (4, 2)):
        n = 2 ** a * 3 ** c
        cells = {(int(smp.radical_inverse_fraction(i, 2) * 2 ** a),
                  int(smp.radical_inverse_fraction(i, 3) * 3 ** c)) for i in range(n)}
        assert len(cells) == n


def test_box_mapping_and_goal_share():
    lo = [0, 0, 0, -0.5, -0.5, -0.5]
    hi = [1, 1, 1, 0.5, 0.5, 0.5]
    X = smp.halton(1, 500, lo, hi)
    assert X.dtype == np.float32 and X.shape == (500, 6)
    assert np.all(X >= np.float32(lo)) and np.all(X <= np.float32(hi))
    assert X[0, 0] == np.float32(0.5) and X[0, 1] == np.float32(1 / 3)
    assert X[0, 3] == np.float32(-0.5 + 1 / 7)
    # mean of a stratified sequence is close to the box centre
    np.testing.assert_allclose(X.mean(0), [0.5, 0.5, 0.5, 0, 0, 0], atol=0.02)
    S = smp.sample_free_halton(400, lo, hi, [0.85] * 3, [0.95] * 3)
    assert S.shape == (400, 6)
    g = S[-4:]
    assert np.all((g[:, :3] >= np.float32(0.85)) & (g[:, :3] <= np.float32(0.95)))
    np.testing.assert_array_equal(S[:396], smp.halton(1, 396, lo, hi))
    # the goal block continues the sequence where the box block stopped
    glo, ghi = float(np.float32(0.85)), float(np.float32(0.95))
    assert S[396, 1] == np.float32(glo + (ghi - glo) * float(smp.radical_inverse_fraction(397, 3)))
