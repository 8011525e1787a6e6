"""Pins for Cost(u, v): the optimal double-integrator connection (Sec. II cost,
Sec. IV Cost primitive)."""

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

from oracle import steer as st

R_U = 0.1


def _rand_pairs(rng, m):
    x0 = np.concatenate([rng.uniform(0, 1, (m, 3)), rng.uniform(-0.5, 0.5, (m, 3))], 1)
    x1 = np.concatenate([rng.uniform(0, 1, (m, 3)), rng.uniform(-0.5, 0.5, (m, 3))], 1)
    return x0, x1


def _gramian_effort(x0, x1, tau):
    """Minimum effort d^T G(tau)^-1 d per axis, with G from scipy's expm and
    quadrature (independent of the closed form)."""
    Ac = np.array([[0.0, 1.0], [0.0, 0.0]])
    Bc = np.array([[0.0], [1.0]])
    G = scipy.integrate.quad_vec(
        lambda s: scipy.linalg.expm(Ac * s) @ Bc @ Bc.T @ scipy.linalg.expm(Ac * s).T, 0, tau)[0]
    eA = scipy.linalg.expm(Ac * tau)
    J = 0.0
    for a in range(3):
        d = np.array([x1[a], x1[3 + a]]) - eA @ np.array([x0[a], x0[3 + a]])
        J += d @ np.linalg.solve(G, d)
    return J


def test_effort_closed_form_equals_gramian_and_hermite_integral():
    rng = np.random.default_rng(11)
    x0, x1 = _rand_pairs(rng, 6)
    for i in range(6):
        for tau in (0.2, 0.7, 1.9):
            S = st.boundary_sums(x0[i], x1[i])
            c = st.cost_of_duration(tau, *S, 1.0)       # r_u = 1: c - tau = effort
            Jg = _gramian_effort(x0[i], x1[i], tau)
            coef = st.hermite(x0[i], x1[i], tau)
            # int_0^tau |p''(t)|^2 dt of the Hermite cubic
            Jh = scipy.integrate.quad(
                lambda t: float(np.sum((2 * coef[:, 2] + 6 * coef[:, 3] * t) ** 2)), 0, tau,
                epsabs=1e-14, epsrel=1e-13)[0]
            assert abs((c - tau) - Jg) <= 1e-9 * max(1.0, Jg)
            assert abs((c - tau) - Jh) <= 1e-9 * max(1.0, Jh)


def test_optimal_duration_is_global_minimum_on_a_dense_grid():
    rng = np.random.default_rng(12)
    x0, x1 = _rand_pairs(rng, 200)
    tau, c = st.steer(x0, x1, R_U)
    grid = np.geomspace(1e-3, 20.0, 400_001)
    S = st.boundary_sums(x0, x1)
    for i in range(200):
        cg = st.cost_of_duration(grid, S[0][i], S[1][i], S[2][i], R_U)
        j = int(np.argmin(cg))
        assert c[i] <= cg[j] + 1e-12
        assert abs(c[i] - cg[j]) <= 1e-6 * max(1.0, c[i])
        assert abs(tau[i] - grid[j]) <= 1e-3 * grid[j] + 1e-4
        # stationarity: the quartic vanishes at tau*
        a2, a1, a0 = -4 * R_U * S[2][i], 24 * R_U * S[1][i], -36 * R_U * S[0][i]
        f = tau[i] ** 4 + a2 * tau[i] ** 2 + a1 * tau[i] + a0
        scale = tau[i] ** 4 + abs(a2) * tau[i] ** 2 + abs(a1) * tau[i] + abs(a0)
        assert abs(f) <= 1e-12 * scale


@pytest.mark.parametrize("r_u", [1.0, 0.25, 0.1])
def test_rest_to_rest_closed_form(r_u):
    """v0 = v1 = 0: c = tau + 12 r |P|^2 / tau^3, so tau* = (36 r |P|^2)^(1/4)
    and c* = 4 tau* / 3."""
    rng = np.random.default_rng(13)
    p0 = rng.uniform(0, 1, (50, 3))
    p1 = rng.uniform(0, 1, (50, 3))
    x0 = np.concatenate([p0, np.zeros((50, 3))], 1)
    x1 = np.concatenate([p1, np.zeros((50, 3))], 1)
    tau, c = st.steer(x0, x1, r_u)
    P2 = np.sum((p1 - p0) ** 2, 1)
    t_ref = (36.0 * r_u * P2) ** 0.25
    np.testing.assert_allclose(tau, t_ref, rtol=1e-13)
    np.testing.assert_allclose(c, 4.0 * t_ref / 3.0, rtol=1e-13)


def test_two_local_minima_picks_the_global_one():
    """Pairs where c(tau) has two local minima (the quartic has three positive
    roots): coasting through a short displacement either quickly or slowly.
    The result is the lower minimum, as found on a dense grid."""
    found = 0
    for v in (0.8, 1.0, 1.5):
        for P in (0.05, 0.1, 0.15, 0.2):
            x0 = np.array([[0.2, 0.3, 0.4, v, 0.0, 0.0]])
            x1 = np.array([[0.2 + P, 0.3, 0.4, v, 0.0, 0.0]])
            S = st.boundary_sums(x0[0], x1[0])
            a2, a1, a0 = -4 * R_U * S[2], 24 * R_U * S[1], -36 * R_U * S[0]
            r = np.roots([1, 0, a2, a1, a0])
            pos = r[(np.abs(r.imag) < 1e-12) & (r.real > 0)].real
            if len(pos) != 3:
                continue
            found += 1
            tau, c = st.steer(x0, x1, R_U)
            grid = np.geomspace(1e-3, 20.0, 400_001)
            cg = st.cost_of_duration(grid, *S, R_U)
            assert abs(c[0] - cg.min()) <= 1e-6 * c[0]
            assert abs(tau[0] - grid[np.argmin(cg)]) <= 1e-3 * tau[0]
            mins = st.cost_of_duration(pos, *S, R_U)
            assert c[0] <= mins.min() + 1e-12
    assert found >= 4


def test_hermite_boundary_conditions():
    rng = np.random.default_rng(15)
    x0, x1 = _rand_pairs(rng, 100)
    tau, _ = st.steer(x0, x1, R_U)
    coef = st.hermite(x0, x1, tau)
    np.testing.assert_allclose(st.hermite_eval(coef, np.zeros(100)), x0[:, :3], atol=1e-15)
    np.testing.assert_allclose(st.hermite_eval(coef, tau), x1[:, :3], atol=1e-12)
    vel0 = coef[..., 1]
    vel1 = coef[..., 1] + 2 * coef[..., 2] * tau[:, None] + 3 * coef[..., 3] * tau[:, None] ** 2
    np.testing.assert_allclose(vel0, x0[:, 3:], atol=1e-15)
    np.testing.assert_allclose(vel1, x1[:, 3:], atol=1e-11)


def test_identical_states_give_no_connection():
    x = np.array([[0.3, 0.4, 0.5, 0.0, 0.0, 0.0]])
    tau, c = st.steer(x, x, R_U)
    assert tau[0] == 0.0 and c[0] == 0.0


def test_waypoint_count():
    assert list(st.waypoint_count(np.array([1e-9, 0.05, 0.0500001, 0.99, 1.0]), 0.05)) == [1, 1, 2, 20, 20]
