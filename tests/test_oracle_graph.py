"""Pins for BuildGraph (Alg. 3): Near, exact continuous Collision, validity."""

import numpy as np

from oracle import graph as gr
from oracle import steer as st

R_U = 0.1


def _dense_hits(coef, tau, box, n=20001):
    t = np.linspace(0.0, tau, n)
    p = st.hermite_eval(coef[None, :, :], t)
    inside = np.all((p >= box[:3]) & (p <= box[3:]), axis=1)
    # signed depth of the deepest sample (positive inside)
    depth = np.minimum(p - box[:3], box[3:] - p).min(axis=1)
    return inside.any(), depth.max()


def test_continuous_collision_matches_dense_sampling():
    rng = np.random.default_rng(21)
    m = 400
    x0 = np.concatenate([rng.uniform(0, 1, (m, 3)), rng.uniform(-0.5, 0.5, (m, 3))], 1)
    x1 = np.concatenate([rng.uniform(0, 1, (m, 3)), rng.uniform(-0.5, 0.5, (m, 3))], 1)
    tau, _ = st.steer(x0, x1, R_U)
    coef = st.hermite(x0, x1, tau)
    # boxes placed near a random point of each trajectory, so about half meet it
    tr = rng.uniform(0, 1, m) * tau
    ctr = st.hermite_eval(coef, tr) + rng.uniform(-0.1, 0.1, (m, 3))
    half = rng.uniform(0.01, 0.1, (m, 3))
    boxes = np.concatenate([ctr - half, ctr + half], 1)
    agree = 0
    hits = 0
    for i in range(m):
        exact = gr.trajectory_hits_boxes(coef[i:i + 1], tau[i:i + 1], boxes[i:i + 1])[0]
        dense, depth = _dense_hits(coef[i], tau[i], boxes[i])
        hits += exact
        if exact == dense:
            agree += 1
        else:
            # sampling can only miss a graze shallower than its resolution
            assert exact and not dense and depth > -1e-5, (i, depth)
    assert 100 < hits < m - 100 and agree >= m - 2


def test_straight_line_through_box_between_samples():
    """Constant-velocity pass (zero control) through a thin wall: both ends
    outside, the middle inside -- the continuous test must report it."""
    v = 1.0
    x0 = np.array([[0.2, 0.5, 0.5, v, 0.0, 0.0]])
    x1 = np.array([[0.8, 0.5, 0.5, v, 0.0, 0.0]])
    tau = np.array([0.6])                     # exactly the coasting time
    coef = st.hermite(x0, x1, tau)
    np.testing.assert_allclose(coef[0, :, 2:], 0.0, atol=1e-14)
    wall = np.array([[0.49, 0.0, 0.0, 0.51, 1.0, 1.0]])
    assert gr.trajectory_hits_boxes(coef, tau, wall)[0]
    # the ends are free
    assert not gr.points_in_boxes(x0[:, :3], wall)[0]
    assert not gr.points_in_boxes(x1[:, :3], wall)[0]
    # moved off to the side it misses
    side = np.array([[0.49, 0.6, 0.0, 0.51, 1.0, 1.0]])
    assert not gr.trajectory_hits_boxes(coef, tau, side)[0]


def test_touching_a_face_counts_as_collision():
    """Obstacles are closed: a trajectory running along the plane of a face
    touches the box."""
    x0 = np.array([[0.2, 0.25, 0.5, 0.0, 0.0, 0.0]])
    x1 = np.array([[0.8, 0.25, 0.5, 0.0, 0.0, 0.0]])
    tau, _ = st.steer(x0, x1, R_U)
    coef = st.hermite(x0, x1, tau)
    face = np.array([[0.4, 0.25, 0.0, 0.6, 0.5, 1.0]])      # lo_y == 0.25
    assert gr.trajectory_hits_boxes(coef, tau, face)[0]
    off = face + np.array([[0, 1e-9, 0, 0, 0, 0]])
    assert not gr.trajectory_hits_boxes(coef, tau, off)[0]


def test_overshoot_between_monotone_pieces():
    """A trajectory that leaves along +x, turns and comes back: the box sits
    beyond both endpoints in x and is reached only at the turn."""
    x0 = np.array([[0.3, 0.5, 0.5, 0.5, 0.0, 0.0]])
    x1 = np.array([[0.3, 0.5, 0.5, -0.5, 0.0, 0.0]])
    tau, _ = st.steer(x0, x1, R_U)
    coef = st.hermite(x0, x1, tau)
    t = np.linspace(0, tau[0], 100001)
    px = st.hermite_eval(coef[0], t)[:, 0]
    apex = px.max()
    assert apex > 0.3 + 1e-3
    box_hit = np.array([[apex - 1e-4, 0.4, 0.4, apex + 0.1, 0.6, 0.6]])
    box_miss = np.array([[apex + 1e-6, 0.4, 0.4, apex + 0.1, 0.6, 0.6]])
    assert gr.trajectory_hits_boxes(coef, tau, box_hit)[0]
    assert not gr.trajectory_hits_boxes(coef, tau, box_miss)[0]


def test_build_graph_matches_per_pair_brute_force():
    """Tiny scene: every ordered pair recomputed one at a time with numpy's
    polynomial root finder and a dense-sampling collision check."""
    rng = np.random.default_rng(22)
    n = 60
    V = np.concatenate([rng.uniform(0, 1, (n, 3)), rng.uniform(-0.5, 0.5, (n, 3))], 1)
    boxes = np.array([[0.3, 0.3, 0.0, 0.5, 0.5, 1.0], [0.6, 0.1, 0.2, 0.7, 0.4, 0.9]])
    g = gr.build_graph(V, boxes, 1.0, R_U)
    valid = ~gr.points_in_boxes(V[:, :3], boxes)
    np.testing.assert_array_equal(g["valid"], valid)
    for v in range(n):
        nbrs = []
        for u in range(n):
            if u == v or not valid[u] or not valid[v]:
                continue
            S = st.boundary_sums(V[v], V[u])
            r = np.roots([1, 0, -4 * R_U * S[2], 24 * R_U * S[1], -36 * R_U * S[0]])
            pos = r[(np.abs(r.imag) < 1e-9) & (r.real > 0)].real
            cs = st.cost_of_duration(pos, *S, R_U)
            tau, c = pos[np.argmin(cs)], cs.min()
            if not (c < 1.0):
                continue
            coef = st.hermite(V[v], V[u], tau)
            if any(_dense_hits(coef, tau, b, 4001)[0] for b in boxes):
                continue
            nbrs.append((u, tau, c))
        row = slice(g["row_ptr"][v], g["row_ptr"][v + 1])
        got = list(g["col"][row])
        exp = [u for u, _, _ in nbrs]
        # a dense check can miss only grazes; none expected on this scene
        assert got == exp, (v, got, exp)
        np.testing.assert_allclose(g["tau"][row], [t for _, t, _ in nbrs], rtol=1e-12)
        np.testing.assert_allclose(g["cost"][row], [c for _, _, c in nbrs], rtol=1e-12)
    assert g["col"].shape[0] > 100, g["col"].shape
