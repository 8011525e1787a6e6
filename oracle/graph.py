"""BuildGraph (Alg. 3) with Near and Collision (oracle, FP64).

Alg. 3: V = {x_init} U SampleFree(n); for every v, N(v) = Near(V \\ {v}, v, r_n)
minus the u whose connection v -> u collides.  Sec. IV: Near(V, u, r) =
{v : Cost(u, v) < r}; Collision(u, v) says whether the optimal trajectory from
u to v meets the obstacle set.

Readings: neighbours are out-neighbours with the strict test c* < r_n, and
connections with tau* <= 1e-6 are left out; obstacles are closed boxes;
Collision is exact in continuous time (the nominal cubic on [0, tau*] meets a
closed box); a sample whose position lies in a closed box is dropped (it keeps
its index but gets no edges).
"""

from __future__ import annotations

import time

import numpy as np

from . import steer as st

TAU_MIN = 1e-6


def points_in_boxes(p, boxes):
    """Closed-box membership of positions p (..., 3) in any of boxes [k, 6]."""
    p = np.asarray(p, np.float64)
    b = np.asarray(boxes, np.float64)
    if b.shape[0] == 0:
        return np.zeros(p.shape[:-1], dtype=bool)
    inside = np.all((p[..., None, :] >= b[:, :3]) & (p[..., None, :] <= b[:, 3:]), axis=-1)
    return inside.any(axis=-1)


def _monotone_breaks(c1, c2, c3, tau):
    """Interior stationary points of p(t) = c0 + c1 t + c2 t^2 + c3 t^3 on
    (0, tau): roots of c1 + 2 c2 t + 3 c3 t^2, as a [m, 2] array (nan = none),
    sorted."""
    A = 3.0 * c3
    Bq = 2.0 * c2
    C = c1
    r = np.full(c1.shape + (2,), np.nan)
    lin = np.abs(A) <= 1e-300
    # linear case
    with np.errstate(divide="ignore", invalid="ignore"):
        rl = np.where(np.abs(Bq) > 0, -C / np.where(Bq != 0, Bq, 1.0), np.nan)
    r[..., 0] = np.where(lin, rl, r[..., 0])
    disc = Bq * Bq - 4.0 * A * C
    quad = (~lin) & (disc >= 0)
    sq = np.sqrt(np.where(quad, disc, 0.0))
    qv = -0.5 * (Bq + np.where(Bq >= 0, sq, -sq))
    with np.errstate(divide="ignore", invalid="ignore"):
        x1 = np.where(quad & (qv != 0), qv / np.where(A != 0, A, 1.0), np.nan)
        x2 = np.where(quad & (qv != 0), C / np.where(qv != 0, qv, 1.0), np.nan)
        x1 = np.where(quad & (qv == 0), 0.0, x1)   # C = B = 0: double root at 0
    r[..., 0] = np.where(quad, x1, r[..., 0])
    r[..., 1] = np.where(quad, x2, r[..., 1])
    inside = (r > 0) & (r < tau[..., None])
    r = np.where(inside, r, np.nan)
    return np.sort(r, axis=-1)


def _cubic(c0, c1, c2, c3, t):
    return c0 + t * (c1 + t * (c2 + t * c3))


def _crossing(c, ta, tb, level, rising, iters=80):
    """On a monotone piece [ta, tb] where p(ta) and p(tb) bracket `level`, the
    time where p crosses it, by bisection."""
    lo = ta.copy()
    hi = tb.copy()
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        v = _cubic(c[0], c[1], c[2], c[3], mid)
        below = v < level
        go_right = np.where(rising, below, ~below)
        lo = np.where(go_right, mid, lo)
        hi = np.where(go_right, hi, mid)
    return lo, hi


def slab_intervals(c, tau, lo, hi):
    """For one axis of many (trajectory, box) combos: the set of t in [0, tau]
    with lo <= p(t) <= hi, as up to 3 closed intervals [m, 3, 2] (nan = empty).

    [0, tau] splits at the stationary points into <= 3 monotone pieces; on a
    monotone piece the in-slab set is a single interval whose ends are where p
    crosses lo or hi."""
    br = _monotone_breaks(c[1], c[2], c[3], tau)
    edges = np.concatenate([np.zeros(tau.shape + (1,)), br, tau[..., None]], axis=-1)
    # pieces: consecutive finite edges
    out = np.full(tau.shape + (3, 2), np.nan)
    # compact the finite edges in order
    fin = np.isfinite(edges)
    cnt = fin.sum(-1)
    order = np.argsort(~fin, axis=-1, kind="stable")
    e = np.take_along_axis(edges, order, axis=-1)
    for k in range(3):
        has = cnt > k + 1
        ta = np.where(has, e[..., k], 0.0)
        tb = np.where(has, e[..., np.minimum(k + 1, 3)], 0.0)
        tb = np.where(has, tb, 0.0)
        pa = _cubic(c[0], c[1], c[2], c[3], ta)
        pb = _cubic(c[0], c[1], c[2], c[3], tb)
        rising = pb >= pa
        pmin = np.minimum(pa, pb)
        pmax = np.maximum(pa, pb)
        nonempty = has & (pmax >= lo) & (pmin <= hi)
        # rising: enter at crossing of lo (or ta), leave at crossing of hi (or tb)
        lo_c, lo_c_hi = _crossing(c, ta, tb, lo, rising)
        hi_c, hi_c_hi = _crossing(c, ta, tb, hi, rising)
        # for a rising piece the in-slab set is [t(lo), t(hi)];
        # for a falling piece it is [t(hi), t(lo)].
        s_rise = np.where(pmin >= lo, ta, lo_c_hi)
        e_rise = np.where(pmax <= hi, tb, hi_c)
        s_fall = np.where(pmax <= hi, ta, hi_c_hi)
        e_fall = np.where(pmin >= lo, tb, lo_c)
        s = np.where(rising, s_rise, s_fall)
        en = np.where(rising, e_rise, e_fall)
        out[..., k, 0] = np.where(nonempty, s, np.nan)
        out[..., k, 1] = np.where(nonempty, en, np.nan)
    return out


def trajectory_hits_boxes(coef, tau, boxes):
    """Collision(u, v) for many edges: does the cubic with coefficients
    coef [m, 3, 4] on [0, tau[m]] meet any closed box in boxes [k, 6]?

    The trajectory is in a box at time t iff all three coordinates are in their
    slabs, so it meets the box iff the three per-axis in-slab sets intersect."""
    m = coef.shape[0]
    b = np.asarray(boxes, np.float64)
    hit = np.zeros(m, dtype=bool)
    for j in range(b.shape[0]):
        sets = []
        for a in range(3):
            c = [coef[:, a, q] for q in range(4)]
            sets.append(slab_intervals(c, tau, b[j, a], b[j, 3 + a]))
        X, Y, Z = sets
        any_j = np.zeros(m, dtype=bool)
        for i in range(3):
            for k in range(3):
                for l in range(3):
                    s = np.maximum(np.maximum(X[:, i, 0], Y[:, k, 0]), Z[:, l, 0])
                    e = np.minimum(np.minimum(X[:, i, 1], Y[:, k, 1]), Z[:, l, 1])
                    any_j |= np.isfinite(s) & np.isfinite(e) & (s <= e)
        hit |= any_j
    return hit


def graph_rows(V, valid, obstacles, r_n, r_u, rows):
    """N(v) for the source nodes `rows` (Alg. 3 inner loop): returns flat
    arrays (src, dst, tau, cost), each row's neighbours ascending."""
    V = np.asarray(V, np.float64)
    ids = np.nonzero(valid)[0]
    vs = np.asarray([v for v in rows if valid[v]], np.int64)
    src = np.repeat(vs, ids.shape[0])
    dst = np.tile(ids, vs.shape[0])
    keep = src != dst
    src, dst = src[keep], dst[keep]
    tau, c = st.steer(V[src], V[dst], r_u)
    near = (c < r_n) & (tau > TAU_MIN)
    src, dst, tau, c = src[near], dst[near], tau[near], c[near]
    if src.shape[0]:
        coef = st.hermite(V[src], V[dst], tau)
        free = ~trajectory_hits_boxes(coef, tau, obstacles)
        src, dst, tau, c = src[free], dst[free], tau[free], c[free]
    return src, dst, tau, c


def build_graph(V, obstacles, r_n, r_u, chunk=1 << 18):
    """Alg. 3.  V: [n+1, 6] states with V[0] = x_init.

    Returns CSR arrays (row_ptr, col, tau, cost) of the out-neighbour lists,
    each row sorted by neighbour index, and `valid` [n+1] (sample not in an
    obstacle).  All ordered pairs are evaluated, a chunk of rows at a time."""
    V = np.asarray(V, np.float64)
    nv = V.shape[0]
    valid = ~points_in_boxes(V[:, :3], obstacles)
    ids = np.nonzero(valid)[0]
    rows_per = max(1, chunk // max(1, ids.shape[0]))
    parts = [graph_rows(V, valid, obstacles, r_n, r_u, ids[r0:r0 + rows_per])
             for r0 in range(0, ids.shape[0], rows_per)]
    if parts:
        src, col, tau, cost = (np.concatenate([p[k] for p in parts]) for k in range(4))
    else:
        src, col, tau, cost = (np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0),
                               np.zeros(0))
    order = np.lexsort((col, src))
    src, col, tau, cost = src[order], col[order], tau[order], cost[order]
    row_ptr = np.zeros(nv + 1, np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return dict(valid=valid, row_ptr=row_ptr, col=col.astype(np.int64), tau=tau, cost=cost)


class RowsOnDemand(dict):
    """The graph of build_graph, each row N(v) built by graph_rows the first
    time Explore asks for it.  The rows are the same; a bounded run of Explore
    on a graph too large to build whole then builds only the rows it expands.
    `col`, `tau`, `cost` hold the rows built so far (edge ids in build order);
    rows(v) returns the edge-id range of N(v); `seconds` is the time spent
    building rows."""

    def __init__(self, V, obstacles, r_n, r_u):
        V = np.asarray(V, np.float64)
        super().__init__(valid=~points_in_boxes(V[:, :3], obstacles))
        self._args = (V, obstacles, r_n, r_u)
        self._range = {}
        self._buf = dict(col=np.zeros(1024, np.int64), tau=np.zeros(1024), cost=np.zeros(1024))
        self._size = 0
        self.seconds = 0.0
        self._publish()

    def _publish(self):
        for k, a in self._buf.items():
            self[k] = a[:self._size]

    def rows(self, v):
        r = self._range.get(int(v))
        if r is None:
            t0 = time.perf_counter()
            V, obs, r_n, r_u = self._args
            _, dst, tau, cost = graph_rows(V, self["valid"], obs, r_n, r_u, [int(v)])
            lo, hi = self._size, self._size + dst.shape[0]
            if hi > self._buf["col"].shape[0]:
                cap = max(hi, 2 * self._buf["col"].shape[0])
                for k in self._buf:
                    grown = np.zeros(cap, self._buf[k].dtype)
                    grown[:lo] = self._buf[k][:lo]
                    self._buf[k] = grown
            self._buf["col"][lo:hi] = dst
            self._buf["tau"][lo:hi] = tau
            self._buf["cost"][lo:hi] = cost
            self._size = hi
            self._publish()
            r = self._range[int(v)] = (lo, hi)
            self.seconds += time.perf_counter() - t0
        return r
