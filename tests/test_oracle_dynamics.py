"""Pins for the oracle's dynamics and particle model (eq. (1)-(2), Sec. II)."""

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

from oracle import dynamics

AC = np.array([[0.0, 1.0], [0.0, 0.0]])
BC = np.array([[0.0], [1.0]])


@pytest.mark.parametrize("dt,sigma", [(0.05, 0.01), (0.05, 0.02), (0.1, 0.3), (0.013, 1.0)])
def test_zoh_matches_matrix_exponential(dt, sigma):
    """Eq. (2) by scipy's expm and numerical quadrature vs the closed form."""
    A, B, V = dynamics.discretize(dt, sigma)
    np.testing.assert_allclose(A, scipy.linalg.expm(AC * dt), rtol=0, atol=1e-15)
    Bq = scipy.integrate.quad_vec(lambda s: scipy.linalg.expm(AC * s) @ BC, 0, dt)[0]
    np.testing.assert_allclose(B, Bq, rtol=1e-12, atol=0)
    Vc = sigma ** 2 * np.eye(2)
    Vq = scipy.integrate.quad_vec(
        lambda s: scipy.linalg.expm(AC * s) @ Vc @ scipy.linalg.expm(AC * s).T, 0, dt)[0]
    np.testing.assert_allclose(V, Vq, rtol=1e-12, atol=0)
    # Van Loan: the noise covariance also equals F22^T F12 of exp([[-Ac, Vc],[0, Ac^T]] dt)
    Mv = np.block([[-AC, Vc], [np.zeros((2, 2)), AC.T]]) * dt
    F = scipy.linalg.expm(Mv)
    np.testing.assert_allclose(V, F[2:, 2:].T @ F[:2, 2:], rtol=1e-10, atol=1e-18)


@pytest.mark.parametrize("q", [(100.0, 10.0, 1.0), (1.0, 1.0, 1.0), (10.0, 0.1, 0.01)])
def test_lqr_matches_scipy_dare(q):
    A, B, _ = dynamics.discretize(0.05, 0.01)
    Q = np.diag(q[:2])
    R = np.array([[q[2]]])
    K, P = dynamics.lqr_gain(A, B, Q, R)
    Ps = scipy.linalg.solve_discrete_are(A, B, Q, R)
    Ks = np.linalg.solve(R + B.T @ Ps @ B, B.T @ Ps @ A)
    np.testing.assert_allclose(P, Ps, rtol=1e-9)
    np.testing.assert_allclose(K, Ks, rtol=1e-9)
    rho = np.max(np.abs(np.linalg.eigvals(A - B @ K)))
    assert rho < 1.0


def test_deviation_covariance_follows_lyapunov():
    """Sample covariance of the deviation process vs Sigma_{s+1} = A_cl Sigma_s
    A_cl^T + V (per axis), with 2e5 particles: every entry within 5 standard
    errors of its Wishart spread."""
    rng = np.random.default_rng(7)
    sigma = 0.02
    A_cl, L, _ = dynamics.closed_loop(0.05, sigma, 100.0, 10.0, 1.0)
    V = L @ L.T
    P = 200_000
    steps = 12
    noise = rng.standard_normal((steps, 6, P))
    dev = dynamics.deviation_states(A_cl, L, noise, steps)
    Sig = np.zeros((2, 2))
    for s in range(steps):
        Sig = A_cl @ Sig @ A_cl.T + V
        if s + 1 in (1, 5, 12):
            for a in range(3):
                x = dev[s + 1, a]
                C = x @ x.T / P
                se = np.sqrt((Sig ** 2 + np.outer(np.diag(Sig), np.diag(Sig))) / P)
                assert np.all(np.abs(C - Sig) < 5 * se), (s, a, C, Sig)


def test_deviation_table_is_fp64_position_part():
    rng = np.random.default_rng(3)
    A_cl, L, _ = dynamics.closed_loop(0.05, 0.01, 100.0, 10.0, 1.0)
    noise = rng.standard_normal((9, 6, 64)).astype(np.float32)
    dev = dynamics.deviation_states(A_cl, L, noise, 9)
    D = dynamics.deviation_table(A_cl, L, noise, 9)
    assert D.dtype == np.float64 and D.shape == (10, 3, 64)
    assert np.all(D[0] == 0)
    np.testing.assert_array_equal(D, dev[:, :, 0, :])
    # the first step is pure noise: dx_1 = L xi_0
    np.testing.assert_allclose(dev[1, 1, 0], L[0, 0] * noise[0, 2].astype(np.float64), rtol=1e-15)
