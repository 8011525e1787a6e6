"""Pins of the oracle's HSMC collision model (oracle/hsmc.py) against what the
paper's construction and plain geometry fix (Sec. III-B, eq. (7))."""

import math

import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.csgraph
import scipy.stats

from oracle import dynamics, explore as ex, graph as gr, hsmc, pump, steer as st
from paper_1607_06886_amd import scenes

CFG = pump.Config()


def _random_boxes(rng, k):
    lo = rng.uniform(0.0, 0.8, (k, 3))
    return np.concatenate([lo, lo + rng.uniform(0.05, 0.2, (k, 3))], axis=1)


def test_closest_point_matches_dense_search():
    rng = np.random.default_rng(1)
    for _ in range(20):
        box = _random_boxes(rng, 1)[0]
        y = rng.uniform(-0.2, 1.2, 3)
        g = [np.linspace(box[a], box[3 + a], 41) for a in range(3)]
        Z = np.stack(np.meshgrid(*g, indexing="ij"), -1).reshape(-1, 3)
        d_brute = np.sqrt(((Z - y) ** 2).sum(1)).min()
        d = np.linalg.norm(hsmc.closest_point(y, box) - y)
        assert d <= d_brute + 1e-12
        assert d >= d_brute - np.linalg.norm((box[3:] - box[:3]) / 40) - 1e-12


def test_single_box_gives_its_closest_point():
    box = np.array([0.4, 0.1, 0.2, 0.6, 0.3, 0.5])
    y = np.array([0.1, 0.2, 0.9])
    d = hsmc.local_region(y, box[None])
    np.testing.assert_allclose(d, [[0.3, 0.0, -0.4]], atol=1e-15)


def test_shadowed_box_is_pruned_and_side_box_is_not():
    y = np.zeros(3)
    front = [1.0, -0.5, -0.5, 2.0, 0.5, 0.5]       # closest, straight ahead
    behind = [3.0, -0.5, -0.5, 4.0, 0.5, 0.5]      # entirely beyond the first plane
    side = [-0.5, 1.5, -0.5, 0.5, 2.5, 0.5]        # off to the side
    d = hsmc.local_region(y, np.array([front, behind, side]))
    np.testing.assert_allclose(d, [[1.0, 0.0, 0.0], [0.0, 1.5, 0.0]], atol=1e-15)


@pytest.mark.parametrize("seed", [2, 3, 4])
def test_region_separates_every_box_and_contains_the_waypoint(seed):
    """Every box lies beyond one of the planes (so no box point is inside the
    region), the waypoint itself is inside, and the planes come in order of
    non-decreasing distance."""
    rng = np.random.default_rng(seed)
    boxes = _random_boxes(rng, 25)
    for _ in range(30):
        y = rng.uniform(0, 1, 3)
        if any(np.all((y >= b[:3]) & (y <= b[3:])) for b in boxes):
            continue
        d = hsmc.local_region(y, boxes)
        assert d.shape[0] >= 1
        norms = np.linalg.norm(d, axis=1)
        assert np.all(np.diff(norms) >= -1e-12)
        for b in boxes:
            # smallest d_i.(z - y) over the box, per plane; some plane must cut it off
            m = np.minimum(d * b[:3], d * b[3:]).sum(1) - d @ y
            assert np.any(m >= (d * d).sum(1) - 1e-12)
        # corners of every box are outside the region (violate some plane)
        for b in boxes:
            corners = np.array([[b[0 + 3 * i], b[1 + 3 * j], b[2 + 3 * k]]
                                for i in (0, 1) for j in (0, 1) for k in (0, 1)])
            assert np.all(((corners - y) @ d.T >= (d * d).sum(1) - 1e-12).any(axis=1))
        # the waypoint satisfies every plane strictly
        assert np.all(0.0 < (d * d).sum(1))


def test_projection_is_perpendicular_to_the_velocity():
    rng = np.random.default_rng(5)
    boxes = _random_boxes(rng, 10)
    y = np.array([0.95, 0.95, 0.95])
    v = np.array([0.3, -0.2, 0.1])
    a, b = hsmc.halfspaces(y, v, boxes)
    d = hsmc.local_region(y, boxes)
    np.testing.assert_allclose(a @ v, 0.0, atol=1e-15)
    np.testing.assert_allclose(b, (a * a).sum(1), rtol=1e-15)
    # at rest the planes are not projected
    a0, b0 = hsmc.halfspaces(y, np.zeros(3), boxes)
    np.testing.assert_allclose(a0, d, atol=0)
    # moving straight at the closest box makes its plane vanish
    a1, b1 = hsmc.halfspaces(y, d[0], boxes)
    assert np.linalg.norm(a1[0]) < 1e-12 and b1[0] < 1e-24


def test_single_waypoint_hsmc_cp_matches_gaussian_tail():
    """One waypoint next to a wall parallel to the motion: the half-space is
    the wall's normal (a = d, b = |d|^2), the particle deviation is Gaussian
    with the Lyapunov covariance, and the violation fraction is the normal
    tail probability 1 - Phi(|d| / sigma_pos), within a 4.5-sigma band."""
    N = 40_000
    sigma = 0.02
    A_cl, L, _ = dynamics.closed_loop(CFG.dt, sigma, CFG.q_pos, CFG.q_vel, CFG.r_track)
    rng = np.random.default_rng(32)
    noise = rng.standard_normal((12, 6, N)).astype(np.float32)
    D = dynamics.deviation_table(A_cl, L, noise, 12)
    Sig = np.zeros((2, 2))
    for _ in range(11):
        Sig = A_cl @ Sig @ A_cl.T + L @ L.T
    s = math.sqrt(Sig[0, 0])
    x0 = np.array([0.5, 0.5, 0.5, 0.25, 0.0, 0.0])      # coasting along x
    x1 = np.array([0.51, 0.5, 0.5, 0.25, 0.0, 0.0])
    tau, c = st.steer(x0[None], x1[None], CFG.r_steer)
    assert tau[0] <= CFG.dt
    V = np.stack([x0, x1])
    graph = dict(col=np.array([1]), tau=tau, cost=c, row_ptr=np.array([0, 1, 1]))
    gap = 1.2 * s
    wall = np.array([[0.0, 0.5 + gap, 0.0, 1.0, 0.9, 1.0]])   # y >= 0.5 + gap
    parent = ex.Plan(nodes=(0,), cost=0.0, step=10, mask=np.zeros(N, bool), parent=-1)
    _, _, step, mask, over, _ = ex.extend_batch(V, graph, D, wall, CFG.dt, 12, [parent],
                                                np.array([0]), cp_model="hsmc")
    assert step[0] == 11 and not over[0]
    coef = st.hermite(x0[None], x1[None], tau)[0]
    vel = coef[:, 1] + tau[0] * (2 * coef[:, 2] + tau[0] * 3 * coef[:, 3])
    assert abs(vel[1]) < 1e-12 and abs(vel[2]) < 1e-12     # motion along x only
    p = 1.0 - scipy.stats.norm.cdf(gap / s)
    frac = mask[0].mean()
    assert 0.05 < p < 0.5
    assert abs(frac - p) <= 4.5 * math.sqrt(p * (1 - p) / N), (frac, p)


def test_zero_noise_hsmc_reduces_to_dijkstra():
    """sigma = 0: no deviation violates a plane (b > 0 on collision-free
    waypoints), so HSMC exploration equals shortest paths, like the box model."""
    sc = scenes.make_scene(dict(n=100, n_obs=3, side=(0.1, 0.3), N=32, sigma=0.0, alpha=0.05,
                                indoor=False), 104, M=100, S_max=256)
    V = np.concatenate([sc.x_init[None], sc.samples]).astype(np.float64)
    D = np.zeros((sc.S_max + 1, 3, sc.N), np.float32)
    g = gr.build_graph(V, sc.obstacles, CFG.r_conn, CFG.r_steer)
    gl = sc.goal.astype(np.float64)
    goal_nodes = np.nonzero(np.all((V[:, :3] >= gl[:3]) & (V[:, :3] <= gl[3:]), 1))[0]
    plans, P, stats, _ = ex.explore(V, g, D, sc.obstacles, goal_nodes, 0.0, 0.1, CFG.lam,
                                    CFG.r_conn, CFG.dt, sc.S_max, cp_model="hsmc")
    assert all(p.pop == 0 for p in plans)
    n = V.shape[0]
    rows = np.repeat(np.arange(n), np.diff(g["row_ptr"]))
    Gm = scipy.sparse.csr_matrix((g["cost"], (rows, g["col"])), shape=(n, n))
    dist = scipy.sparse.csgraph.dijkstra(Gm, directed=True, indices=0)
    best = min(plans[q].cost for v in goal_nodes for q in P.get(int(v), []))
    assert abs(best - dist[goal_nodes].min()) <= 1e-9 * best


def test_hsmc_plans_grow_their_bits_and_match_a_resimulation():
    sc = scenes.make_scene(dict(n=90, n_obs=4, side=(0.1, 0.3), N=32, sigma=0.02, alpha=0.1,
                                indoor=False), 105, M=100, S_max=256)
    cfg = pump.Config(cp_model="hsmc")
    out = pump.run(sc, cfg, with_selection=False)
    plans, V, D = out["plans"], out["V"], out["D"]
    assert out["stats"]["partial_plans"] > 200
    checked = 0
    for pid, p in enumerate(plans[1:], start=1):
        par = plans[p.parent]
        assert np.all(p.mask >= par.mask)
        if pid % 5:
            continue
        # from scratch: every waypoint of the path, its own half-spaces
        hit = np.zeros(sc.N, bool)
        s = 0
        for u, v in zip(p.nodes[:-1], p.nodes[1:]):
            tau, c = st.steer(V[u][None], V[v][None], CFG.r_steer)
            K = int(st.waypoint_count(tau, CFG.dt)[0])
            coef = st.hermite(V[u][None], V[v][None], tau)[0]
            for k in range(1, K + 1):
                t = k * tau[0] / K
                pos = st.hermite_eval(coef, t)
                vel = coef[:, 1] + t * (2 * coef[:, 2] + t * 3 * coef[:, 3])
                a, b = hsmc.halfspaces(pos, vel, sc.obstacles)
                hit |= hsmc.violations(a, b, D[s + k].astype(np.float64))
            s += K
        np.testing.assert_array_equal(hit, p.mask)
        checked += 1
    assert checked > 10
