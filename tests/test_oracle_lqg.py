"""Pins of the oracle's LQG tracking model (oracle/dynamics.py, eq. (2) with a
measurement and a Kalman estimate) against textbook forms and statistics."""

import math

import numpy as np
import scipy.linalg

from oracle import dynamics, select as sel

DT, SIG, SIGM = 0.05, 0.02, 0.01
QP, QV, RT = 100.0, 10.0, 1.0


def test_kalman_gain_matches_the_filter_riccati_equation():
    A, B, V = dynamics.discretize(DT, SIG)
    C = np.array([[1.0, 0.0]])
    W = np.array([[SIGM ** 2 / DT]])
    G, P = dynamics.kalman_gain(A, C, V, W)
    # predicted covariance of the steady-state filter: the dual control DARE
    P_ref = scipy.linalg.solve_discrete_are(A.T, C.T, V, W)
    np.testing.assert_allclose(P, P_ref, rtol=1e-10)
    G_ref = P_ref @ C.T @ np.linalg.inv(C @ P_ref @ C.T + W)
    np.testing.assert_allclose(G, G_ref, rtol=1e-10)
    # the estimation error dynamics are stable
    assert np.max(np.abs(np.linalg.eigvals((np.eye(2) - G @ C) @ A))) < 1.0


def test_joint_recursion_equals_a_direct_simulation_of_the_loop():
    """Predict with the applied control, correct with the measurement of the
    new state: the same trajectories as z' = M z + E xi."""
    M, E, K, G = dynamics.lqg_closed_loop(DT, SIG, SIGM, QP, QV, RT)
    A, B, V = dynamics.discretize(DT, SIG)
    L = np.linalg.cholesky(V)
    C = np.array([[1.0, 0.0]])
    sw = math.sqrt(SIGM ** 2 / DT)
    rng = np.random.default_rng(3)
    S, P = 40, 64
    noise = rng.standard_normal((S, 6, P))
    meas = rng.standard_normal((S, 3, P))
    z = dynamics.lqg_deviation_states(M, E, noise, meas, S)
    for a in range(3):
        x = np.zeros((2, P))
        xh = np.zeros((2, P))
        for s in range(S):
            u = -K @ xh
            x = A @ x + B @ u + L @ noise[s, 2 * a:2 * a + 2]
            y = C @ x + sw * meas[s, a:a + 1]
            pred = A @ xh + B @ u
            xh = pred + G @ (y - C @ pred)
            np.testing.assert_allclose(z[s + 1, a, :2], x, atol=1e-13)
            np.testing.assert_allclose(z[s + 1, a, 2:], xh, atol=1e-13)


def test_estimation_error_evolves_on_its_own():
    """Separation: e = dx - x_hat obeys e' = (I - GC) A e + (I - GC) L xi_p -
    G sqrt(W) xi_m, whatever the controller."""
    M, E, K, G = dynamics.lqg_closed_loop(DT, SIG, SIGM, QP, QV, RT)
    A, B, V = dynamics.discretize(DT, SIG)
    L = np.linalg.cholesky(V)
    C = np.array([[1.0, 0.0]])
    sw = math.sqrt(SIGM ** 2 / DT)
    rng = np.random.default_rng(4)
    S, P = 30, 16
    noise = rng.standard_normal((S, 6, P))
    meas = rng.standard_normal((S, 3, P))
    z = dynamics.lqg_deviation_states(M, E, noise, meas, S)
    F = (np.eye(2) - G @ C)
    for a in range(3):
        e = np.zeros((2, P))
        for s in range(S):
            e = F @ A @ e + F @ L @ noise[s, 2 * a:2 * a + 2] - G * sw @ meas[s, a:a + 1]
            np.testing.assert_allclose(z[s + 1, a, :2] - z[s + 1, a, 2:], e, atol=1e-13)


def test_deviation_covariance_follows_the_lyapunov_recursion():
    M, E, _, _ = dynamics.lqg_closed_loop(DT, SIG, SIGM, QP, QV, RT)
    rng = np.random.default_rng(5)
    S, P = 25, 100_000
    noise = rng.standard_normal((S, 6, P))
    meas = rng.standard_normal((S, 3, P))
    z = dynamics.lqg_deviation_states(M, E, noise, meas, S)
    Sig = np.zeros((4, 4))
    for s in range(S):
        Sig = M @ Sig @ M.T + E @ E.T
    samp = np.cov(z[S, 0])
    # position variance and the position-estimate covariance within 5 s.e.
    for (i, j) in ((0, 0), (0, 2), (1, 1), (2, 2)):
        se = math.sqrt((Sig[i, i] * Sig[j, j] + Sig[i, j] ** 2) / P)
        assert abs(samp[i, j] - Sig[i, j]) <= 5 * se, (i, j, samp[i, j], Sig[i, j])
    # the estimate adds variance relative to full-state feedback
    A_cl, L, _ = dynamics.closed_loop(DT, SIG, QP, QV, RT)
    S2 = np.zeros((2, 2))
    for s in range(S):
        S2 = A_cl @ S2 @ A_cl.T + L @ L.T
    assert Sig[0, 0] > S2[0, 0]


def test_certification_count_with_lqg_matches_direct_particles():
    """mc_count_lqg equals a count over particles propagated by the direct
    loop of the test above, each segment tested against the box."""
    M, E, K, G = dynamics.lqg_closed_loop(DT, SIG, SIGM, QP, QV, RT)
    V = np.array([[0.1, 0.5, 0.5, 0.0, 0.0, 0.0], [0.9, 0.5, 0.5, 0.0, 0.0, 0.0]])
    box = np.array([[0.45, 0.51, 0.0, 0.55, 0.8, 1.0]])
    rng = np.random.default_rng(6)
    Mp = 3000
    W = sel.plan_waypoints(V, (0, 1), 0.1, DT)
    S = W.shape[0] - 1
    noise = rng.standard_normal((S + 2, 6, Mp))
    meas = rng.standard_normal((S + 2, 3, Mp))
    got = sel.mc_count_lqg(V, (0, 1), box, M, E, noise, meas, 0.1, DT)
    z = dynamics.lqg_deviation_states(M, E, noise, meas, S)
    hit = np.zeros(Mp, bool)
    prev = np.repeat(W[0][None], Mp, 0)
    for s in range(S):
        cur = (W[s + 1][:, None] + z[s + 1, :, 0, :]).T
        hit |= sel.segments_hit_box(prev, cur, box[0, :3], box[0, 3:])
        prev = cur
    assert got == int(hit.sum())
    assert got > 50
