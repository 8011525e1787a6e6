"""Pins of the oracle's Smooth(p, alpha) (oracle/smooth.py; Alg. 5's last
step) against closed forms, finite differences and a linear scan."""

import math

import numpy as np
import pytest

from oracle import dynamics, pump, select as sel, smooth as sm, steer as st
from tests._gpu import scene

CFG = pump.Config()
R_U, DT = CFG.r_steer, CFG.dt


def _random_plan(rng, k):
    """k + 1 states along a rough line from a start at rest."""
    V = np.zeros((k + 1, 6))
    V[0, :3] = [0.1, 0.1, 0.1]
    for i in range(1, k + 1):
        V[i, :3] = V[i - 1, :3] + rng.uniform(0.05, 0.25, 3)
        V[i, 3:] = rng.uniform(-0.5, 0.5, 3)
    return V, tuple(range(k + 1))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_blend_ends_cost_the_plan_and_the_optimal_connection(seed):
    rng = np.random.default_rng(seed)
    V, nodes = _random_plan(rng, 5)
    edges = sm.plan_edges(V, nodes, R_U)
    q = sm.optimal_connection(V, nodes, R_U)
    plan_cost = float(np.sum(edges[1]))
    assert abs(sm.blend_cost(0.0, edges, q, R_U) - plan_cost) <= 1e-12 * plan_cost
    tau, c = st.steer(V[0][None], V[-1][None], R_U)
    assert abs(sm.blend_cost(1.0, edges, q, R_U) - c[0]) <= 1e-12 * c[0]
    # the optimal connection is the cheapest trajectory between the two states
    assert c[0] <= plan_cost
    for beta in (0.25, 0.5, 0.75):
        assert sm.blend_cost(beta, edges, q, R_U) >= c[0] * (1 - 1e-12)


@pytest.mark.parametrize("seed", [4, 5])
def test_blend_effort_matches_finite_differences(seed):
    """N(beta) against Gauss-Legendre quadrature (3 nodes per piece, exact for
    the quadratic |P''|^2) of central second differences of P(s), which are
    exact for the cubic pieces when the stencil stays inside one piece."""
    rng = np.random.default_rng(seed)
    V, nodes = _random_plan(rng, 4)
    edges = sm.plan_edges(V, nodes, R_U)
    q = sm.optimal_connection(V, nodes, R_U)
    t0 = edges[3]
    gx, gw = np.polynomial.legendre.leggauss(3)
    for beta in (0.0, 0.3, 0.8, 1.0):
        total = 0.0
        for e in range(len(nodes) - 1):
            sa, sb = t0[e] / t0[-1], t0[e + 1] / t0[-1]
            h = 1e-3 * (sb - sa)
            for x, w in zip(gx, gw):
                s = 0.5 * (sa + sb) + 0.5 * (sb - sa) * x
                P = sm.blend_positions(np.array([s - h, s, s + h]), beta, edges, q)
                d2 = (P[0] - 2 * P[1] + P[2]) / h ** 2
                total += 0.5 * (sb - sa) * w * float(d2 @ d2)
        ref = sm.blend_effort(beta, edges, q)
        assert abs(total - ref) <= 1e-5 * ref, (beta, total, ref)


def test_blend_keeps_both_boundary_states():
    rng = np.random.default_rng(6)
    V, nodes = _random_plan(rng, 3)
    V[0, 3:] = [0.2, -0.1, 0.3]
    edges = sm.plan_edges(V, nodes, R_U)
    q = sm.optimal_connection(V, nodes, R_U)
    for beta in (0.0, 0.4, 1.0):
        T = (1 - beta) * edges[3][-1] + beta * q[0]
        P = sm.blend_positions(np.array([0.0, 1.0]), beta, edges, q)
        np.testing.assert_allclose(P[0], V[0, :3], atol=1e-14)
        np.testing.assert_allclose(P[1], V[-1, :3], atol=1e-13)
        h = 1e-7
        v0 = (sm.blend_positions(np.array([h]), beta, edges, q)[0] - P[0]) / (h * T)
        v1 = (P[1] - sm.blend_positions(np.array([1 - h]), beta, edges, q)[0]) / (h * T)
        np.testing.assert_allclose(v0, V[0, 3:], atol=1e-5)
        np.testing.assert_allclose(v1, V[-1, 3:], atol=1e-5)


def test_full_blend_is_the_direct_connection_on_its_grid():
    rng = np.random.default_rng(7)
    V, nodes = _random_plan(rng, 4)
    edges = sm.plan_edges(V, nodes, R_U)
    q = sm.optimal_connection(V, nodes, R_U)
    W = sm.blend_waypoints(1.0, edges, q, DT)
    direct = sel.plan_waypoints(np.stack([V[0], V[-1]]), (0, 1), R_U, DT)
    assert W.shape == direct.shape
    np.testing.assert_allclose(W, direct, atol=1e-13)
    W0 = sm.blend_waypoints(0.0, edges, q, DT)
    assert W0.shape[0] - 1 == max(1, math.ceil(edges[3][-1] / DT))


@pytest.mark.parametrize("thr", [0.0, 0.001, 0.3, 0.5, 0.61803, 0.999, 1.0])
def test_bisection_equals_a_linear_scan(thr):
    """For a monotone certificate (certified iff beta <= thr) the search
    returns the largest point k / 2^BISECT_STEPS not above thr (1 if thr = 1)."""
    calls = []

    def cert(b):
        calls.append(b)
        return b <= thr

    got = sm.bisect_beta(cert)
    n = 1 << sm.BISECT_STEPS
    want = 1.0 if thr >= 1.0 else max(k for k in range(n) if k / n <= thr) / n
    assert got == want
    assert len(calls) == (1 if thr >= 1.0 else 1 + sm.BISECT_STEPS)


def test_no_obstacles_gives_the_optimal_connection():
    sc = scene("cfg1", 2)
    sc.obstacles = np.zeros((0, 6), np.float32)
    out = pump.run(sc, pump.Config(smooth=True))
    assert out["status"] == 0
    s = out["smooth"]
    V = out["V"]
    _, c = st.steer(V[0][None], V[out["best"].head][None], R_U)
    assert s["beta"] == 1.0 and s["count"] == 0
    assert abs(s["cost"] - c[0]) <= 1e-12 * c[0]
    assert s["cost"] <= out["best"].cost


@pytest.mark.parametrize("kind,seed", [("cfg1", 0), ("n64", 4)])
def test_smoothed_plan_is_certified_and_cheaper(kind, seed):
    sc = scene(kind, seed)
    out = pump.run(sc, pump.Config(smooth=True))
    s = out["smooth"]
    best = out["best"]
    assert s["cost"] <= best.cost
    assert s["count"] / sc.M <= sc.alpha
    if s["beta"] > 0:
        A_cl, L, _ = dynamics.closed_loop(CFG.dt, sc.sigma, CFG.q_pos, CFG.q_vel, CFG.r_track)
        assert sel.mc_count_waypoints(s["W"], sc.obstacles, A_cl, L, sc.noise_mc) == s["count"]
        np.testing.assert_allclose(s["W"][0], out["V"][0, :3], atol=1e-14)
        np.testing.assert_allclose(s["W"][-1], out["V"][best.head, :3], atol=1e-13)
    # every probed weight above the result failed (or the result is beta = 1)
    for b, c in s["evals"].items():
        if b > s["beta"]:
            assert c is None or c / sc.M > sc.alpha
