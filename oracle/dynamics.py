"""Dynamics, tracking controller and particle deviations (oracle, FP64).

Sec. II, eq. (1)-(2): linear dynamics with Gaussian process noise, discretised
with a zero-order hold at the tracking step dt; a linear-quadratic tracking
controller acts on the deviation from the nominal trajectory.  Sec. V-A fixes
the model: a 6-D double integrator (x'' = u) in a 3-D workspace, so every axis
is an independent 2-state (position, velocity) system and all matrices below
are per axis.

Readings (the paper leaves these open): the process noise intensity is
V_c = sigma^2 * I on the 6 state derivatives; the tracking law is the
steady-state discrete LQR gain with full-state feedback (du = -K dx),
Q = diag(q_pos, q_vel), R = r_track; the deviation process starts at zero at
the start state and its noise is indexed by (tracking step, particle), shared by
every plan, so the deviation at plan step s does not depend on the plan.  Every
quantity here stays in FP64.
"""

from __future__ import annotations

import math

import numpy as np


def discretize(dt: float, sigma: float):
    """Eq. (2) per axis for A_c = [[0,1],[0,0]], B_c = [0,1]^T, V_c = sigma^2 I.

    A = exp(A_c dt) = [[1, dt], [0, 1]]
    B = (int_0^dt exp(A_c s) ds) B_c = [dt^2/2, dt]^T
    V = int_0^dt exp(A_c s) V_c exp(A_c^T s) ds
      = sigma^2 [[dt + dt^3/3, dt^2/2], [dt^2/2, dt]]
    (exp(A_c s) exp(A_c^T s) = [[1 + s^2, s], [s, 1]], integrated term by term.)
    """
    dt = float(dt)
    s2 = float(sigma) ** 2
    A = np.array([[1.0, dt], [0.0, 1.0]])
    B = np.array([[dt * dt / 2.0], [dt]])
    V = s2 * np.array([[dt + dt ** 3 / 3.0, dt * dt / 2.0],
                       [dt * dt / 2.0, dt]])
    return A, B, V


def lqr_gain(A, B, Q, R, tol=1e-14, max_iter=1_000_000):
    """Steady-state discrete LQR gain (Sec. II tracking controller; reading:
    infinite-horizon, full-state feedback).

    Iterates the Riccati difference equation
        P <- Q + A^T P A - A^T P B (R + B^T P B)^-1 B^T P A
    from P = Q until the relative change is below `tol`; returns
    K = (R + B^T P B)^-1 B^T P A and P.  The control is du = -K dx."""
    A = np.asarray(A, float)
    B = np.asarray(B, float)
    Q = np.asarray(Q, float)
    R = np.atleast_2d(np.asarray(R, float))
    P = Q.copy()
    for _ in range(max_iter):
        G = R + B.T @ P @ B
        PB = P @ B
        Pn = Q + A.T @ P @ A - A.T @ PB @ np.linalg.solve(G, PB.T @ A)
        delta = np.max(np.abs(Pn - P)) / max(np.max(np.abs(Pn)), 1e-300)
        P = Pn
        if delta < tol:
            break
    K = np.linalg.solve(R + B.T @ P @ B, B.T @ P @ A)
    return K, P


def closed_loop(dt, sigma, q_pos, q_vel, r_track):
    """A_cl = A - B K and L = chol(V) for one axis."""
    A, B, V = discretize(dt, sigma)
    K, _ = lqr_gain(A, B, np.diag([q_pos, q_vel]), [[r_track]])
    A_cl = A - B @ K
    L = np.linalg.cholesky(V)
    return A_cl, L, K


def deviation_states(A_cl, L, noise, steps):
    """Particle deviations dx_s for s = 0..steps (FP64).

    noise: [>= steps, 6, P] standard normals; component 2a and 2a+1 drive axis a.
    dx_0 = 0 and dx_{s+1} = A_cl dx_s + L (xi_{s,2a}, xi_{s,2a+1})^T  (eq. (2)
    closed loop: dx_{t+1} = A dx_t + B du_t + v_t with du_t = -K dx_t and
    v_t ~ N(0, V) drawn as L xi).
    Returns an array [steps+1, 3, 2, P] of (position, velocity) deviations."""
    noise = np.asarray(noise, dtype=np.float64)
    P = noise.shape[2]
    out = np.zeros((steps + 1, 3, 2, P))
    for s in range(steps):
        for a in range(3):
            x = out[s, a]
            w = L @ noise[s, 2 * a:2 * a + 2, :]
            out[s + 1, a] = A_cl @ x + w
    return out


def deviation_table(A_cl, L, noise, steps):
    """Position part of the deviations, D[s][a][j] (FP64)."""
    dev = deviation_states(A_cl, L, noise, steps)
    return np.ascontiguousarray(dev[:, :, 0, :])


# ---------------------------------------------------------------------------
# LQG tracking (eq. (2) with the measurement y = C x + w and a Kalman
# estimate; the controller acts on the estimate).  Readings: C = [1, 0] per
# axis (the workspace output is the position); W = W_c / dt with
# W_c = sigma_meas^2 per axis; steady-state LQR gain on the estimate
# (certainty equivalence) and steady-state Kalman gain; the start state is
# known exactly (dx_0 = 0, estimate 0); the measurement taken after step s
# uses the s-th row of the measurement noise.
# ---------------------------------------------------------------------------
def kalman_gain(A, C, V, W, tol=1e-14, max_iter=1_000_000):
    """Steady-state Kalman gain G (update x_hat += G (y - C x_hat_pred)).

    Iterates the predicted covariance P <- A (P - P C^T S^-1 C P) A^T + V,
    S = C P C^T + W, from P = V to a relative change below `tol`;
    G = P C^T S^-1 with the converged predicted covariance P."""
    A = np.asarray(A, float)
    C = np.atleast_2d(np.asarray(C, float))
    V = np.asarray(V, float)
    W = np.atleast_2d(np.asarray(W, float))
    P = V.copy()
    for _ in range(max_iter):
        S = C @ P @ C.T + W
        Pu = P - P @ C.T @ np.linalg.solve(S, C @ P)
        Pn = A @ Pu @ A.T + V
        delta = np.max(np.abs(Pn - P)) / max(np.max(np.abs(Pn)), 1e-300)
        P = Pn
        if delta < tol:
            break
    G = P @ C.T @ np.linalg.inv(C @ P @ C.T + W)
    return G, P


def lqg_closed_loop(dt, sigma, sigma_meas, q_pos, q_vel, r_track):
    """Joint closed loop of (dx, x_hat) for one axis: z_{t+1} = M z_t + E xi_t
    with xi_t = (process normal 1, process normal 2, measurement normal).

        dx'    = A dx - B K x_hat + L xi_p
        x_hat' = G C A dx + ((I - G C) A - B K) x_hat + G C L xi_p + G sqrt(W) xi_m

    (predict with the applied control, then correct with the measurement of
    the new state).  Returns M [4, 4], E [4, 3], K [1, 2], G [2, 1]."""
    A, B, V = discretize(dt, sigma)
    K, _ = lqr_gain(A, B, np.diag([q_pos, q_vel]), [[r_track]])
    C = np.array([[1.0, 0.0]])
    W = np.array([[float(sigma_meas) ** 2 / float(dt)]])
    G, _ = kalman_gain(A, C, V, W)
    L = np.linalg.cholesky(V)
    I2 = np.eye(2)
    M = np.block([[A, -B @ K], [G @ C @ A, (I2 - G @ C) @ A - B @ K]])
    E = np.block([[L, np.zeros((2, 1))], [G @ C @ L, G * math.sqrt(W[0, 0])]])
    return M, E, K, G


def lqg_deviation_states(M, E, noise, noise_meas, steps):
    """Joint states z_s (s = 0..steps) [steps+1, 3, 4, P]; noise [>= steps, 6, P]
    (process, two per axis), noise_meas [>= steps, 3, P] (one per axis)."""
    noise = np.asarray(noise, np.float64)
    meas = np.asarray(noise_meas, np.float64)
    P = noise.shape[2]
    out = np.zeros((steps + 1, 3, 4, P))
    for s in range(steps):
        for a in range(3):
            xi = np.concatenate([noise[s, 2 * a:2 * a + 2, :], meas[s, a:a + 1, :]], axis=0)
            out[s + 1, a] = M @ out[s, a] + E @ xi
    return out


def lqg_deviation_table(M, E, noise, noise_meas, steps):
    """Position part of the true deviation, D[s][a][j] (FP64)."""
    return np.ascontiguousarray(lqg_deviation_states(M, E, noise, noise_meas, steps)[:, :, 0, :])
