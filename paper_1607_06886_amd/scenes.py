"""Seeded synthetic planning problems (inputs only).

This module draws the inputs a planning query consumes -- obstacle boxes, state
samples, the start state, the goal box and the standard-normal noise that the
particle models use -- and nothing else.  It holds none of the planner's
arithmetic, so both the HIP path and the CPU oracle may take their inputs from
it.

Workload shapes follow the paper's experiments (Sec. V-A and V-C): a 6-D double
integrator flying in a unit-cube workspace cluttered with axis-aligned boxes
(obstacles are unions of AABBs, Sec. V-C), either a few random boxes or an
indoor map of thin walls with doorways.  The paper's own maps are not
published; these seeded scenes stand in for them with the stated sizes.

Random numbers that the method itself consumes (the exploration particles'
process noise and the Monte Carlo certification particles' noise) are drawn
here and handed to the planner as arrays, so both implementations see the same
values.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# Named workloads.  "cfg1".."cfg3" are single queries; the batched and learned
# workloads are assembled from these generators by their own callers.
WORKLOADS = {
    # 3 random boxes, sides U[0.1, 0.3]; 500 samples; 32 particles, sigma 0.01.
    "cfg1": dict(n=500, n_obs=3, side=(0.1, 0.3), N=32, sigma=0.01, alpha=0.05,
                 indoor=False),
    # 20 random boxes, sides U[0.05, 0.25]; 4000 samples; 128 particles.
    "cfg2": dict(n=4000, n_obs=20, side=(0.05, 0.25), N=128, sigma=0.02,
                 alpha=0.01, indoor=False),
    # Indoor map: 60 thin walls forming a 4x4 room grid, 20000 samples.
    "cfg3": dict(n=20000, n_obs=60, side=None, N=256, sigma=0.02, alpha=0.01,
                 indoor=True),
}

X_INIT = (0.1, 0.1, 0.1, 0.0, 0.0, 0.0)
GOAL_BOX = (0.85, 0.85, 0.85, 0.95, 0.95, 0.95)
VEL_HALF = 0.5            # sample velocities uniform in [-0.5, 0.5]^3
INDOOR_X_INIT = (0.125, 0.125, 0.3, 0.0, 0.0, 0.0)
INDOOR_GOAL_CENTRE = (0.875, 0.875, 0.3)
INDOOR_GOAL_HALF = 0.025  # a 0.05 box


def workload_seed(config_index: int, query: int) -> int:
    """Seed of query `query` of workload `config_index`."""
    return 1_000_003 * int(config_index) + int(query)


@dataclasses.dataclass
class Scene:
    """One planning query's inputs (all float32, C-contiguous)."""
    samples: np.ndarray      # [n, 6] states (px, py, pz, vx, vy, vz)
    obstacles: np.ndarray    # [n_obs, 6] closed boxes (lo xyz, hi xyz)
    x_init: np.ndarray       # [6]
    goal: np.ndarray         # [6] closed position box (lo xyz, hi xyz)
    alpha: float             # CP bound, stored as float32
    N: int                   # exploration particles
    sigma: float             # process-noise intensity
    noise: np.ndarray        # [S_max, 6, N] standard normals (exploration)
    noise_mc: np.ndarray     # [S_max, 6, M] standard normals (certification)
    name: str = ""
    seed: int = 0
    # measurement noise of LQG tracking (only with sigma_meas > 0)
    sigma_meas: float = 0.0
    noise_meas: Optional[np.ndarray] = None     # [S_max, 3, N] standard normals
    noise_mc_meas: Optional[np.ndarray] = None  # [S_max, 3, M] standard normals

    @property
    def n(self) -> int:
        return int(self.samples.shape[0])

    @property
    def n_obs(self) -> int:
        return int(self.obstacles.shape[0])

    @property
    def S_max(self) -> int:
        return int(self.noise.shape[0])

    @property
    def M(self) -> int:
        return int(self.noise_mc.shape[2])


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(stream)]))


def _in_boxes(p: np.ndarray, boxes: np.ndarray) -> np.ndarray:
    """Rows of p (…,3) lying in any closed box."""
    if boxes.shape[0] == 0:
        return np.zeros(p.shape[:-1], dtype=bool)
    lo = boxes[:, :3]
    hi = boxes[:, 3:]
    inside = np.all((p[..., None, :] >= lo) & (p[..., None, :] <= hi), axis=-1)
    return inside.any(axis=-1)


def _boxes_touch(a: np.ndarray, b_lo, b_hi) -> bool:
    return bool(np.all(a[:3] <= b_hi) and np.all(a[3:] >= b_lo))


def random_boxes(rng, n_obs: int, side, x_init, goal, margin=0.05) -> np.ndarray:
    """n_obs boxes with independent side lengths U[side] inside [0,1]^3.

    A box that comes within `margin` of the start position or of the goal box
    is drawn again."""
    out = []
    s_lo = np.asarray(x_init[:3], np.float64) - margin
    s_hi = np.asarray(x_init[:3], np.float64) + margin
    g_lo = np.asarray(goal[:3], np.float64) - margin
    g_hi = np.asarray(goal[3:], np.float64) + margin
    while len(out) < n_obs:
        sides = rng.uniform(side[0], side[1], size=3)
        lo = rng.uniform(0.0, 1.0 - sides)
        box = np.concatenate([lo, lo + sides])
        if _boxes_touch(box, s_lo, s_hi) or _boxes_touch(box, g_lo, g_hi):
            continue
        out.append(box)
    return np.asarray(out, dtype=np.float32).reshape(n_obs, 6)


def indoor_boxes(rng, thick=0.02, door=0.08, door_h=0.6) -> np.ndarray:
    """Indoor map: a 4x4 grid of rooms in the unit cube.

    Six interior wall lines (x = 0.25, 0.5, 0.75 and y = 0.25, 0.5, 0.75), each
    full height and `thick` thick, with one doorway per room side (`door` wide at
    a uniform offset, `door_h` high).  Each line yields 5 wall pieces and 4
    lintels; 6 boundary slabs (4 walls, floor, ceiling) close the map: 60 boxes.
    """
    boxes = []
    h = thick / 2.0
    for axis in (0, 1):                      # wall normal along x, then y
        for c in (0.25, 0.5, 0.75):
            # doorway intervals along the wall's length, one per room side
            doors = []
            for k in range(4):
                a0 = 0.25 * k + thick
                a1 = 0.25 * (k + 1) - thick - door
                d0 = rng.uniform(a0, a1)
                doors.append((d0, d0 + door))
            edges = [0.0]
            for d0, d1 in doors:
                edges += [d0, d1]
            edges.append(1.0)
            for k in range(5):               # solid pieces between doorways
                s0, s1 = edges[2 * k], edges[2 * k + 1]
                lo = [0.0, 0.0, 0.0]
                hi = [1.0, 1.0, 1.0]
                lo[axis], hi[axis] = c - h, c + h
                lo[1 - axis], hi[1 - axis] = s0, s1
                boxes.append(lo + hi)
            for d0, d1 in doors:             # lintels above the doorways
                lo = [0.0, 0.0, door_h]
                hi = [1.0, 1.0, 1.0]
                lo[axis], hi[axis] = c - h, c + h
                lo[1 - axis], hi[1 - axis] = d0, d1
                boxes.append(lo + hi)
    slabs = [
        [0.0, 0.0, 0.0, thick, 1.0, 1.0], [1.0 - thick, 0.0, 0.0, 1.0, 1.0, 1.0],
        [0.0, 0.0, 0.0, 1.0, thick, 1.0], [0.0, 1.0 - thick, 0.0, 1.0, 1.0, 1.0],
        [0.0, 0.0, 0.0, 1.0, 1.0, thick], [0.0, 0.0, 1.0 - thick, 1.0, 1.0, 1.0],
    ]
    boxes += slabs
    return np.asarray(boxes, dtype=np.float32)


def free_samples(rng, n: int, boxes: np.ndarray, goal, n_goal: int) -> np.ndarray:
    """n states: n_goal with positions in the goal box, the rest uniform in the
    unit cube; positions inside an obstacle are redrawn; velocities uniform in
    [-VEL_HALF, VEL_HALF]^3."""
    g_lo = np.asarray(goal[:3], np.float64)
    g_hi = np.asarray(goal[3:], np.float64)
    pos = []
    have = 0
    while have < n_goal:
        p = rng.uniform(g_lo, g_hi, size=(2 * (n_goal - have) + 8, 3))
        p = p[~_in_boxes(p.astype(np.float32), boxes)][: n_goal - have]
        pos.append(p)
        have += p.shape[0]
    rest = n - n_goal
    have = 0
    while have < rest:
        p = rng.uniform(0.0, 1.0, size=(int(1.5 * (rest - have)) + 64, 3))
        p = p[~_in_boxes(p.astype(np.float32), boxes)][: rest - have]
        pos.append(p)
        have += p.shape[0]
    pos = np.concatenate(pos, axis=0)
    vel = rng.uniform(-VEL_HALF, VEL_HALF, size=(n, 3))
    return np.ascontiguousarray(np.concatenate([pos, vel], axis=1).astype(np.float32))


def _map_of(p, seed: int):
    """x_init, goal box, obstacle boxes and samples of one query (stream 0)."""
    rng = _rng(seed, 0)
    if p.get("indoor"):
        x_init = np.asarray(INDOOR_X_INIT, np.float32)
        c = np.asarray(INDOOR_GOAL_CENTRE, np.float64)
        goal = np.concatenate([c - INDOOR_GOAL_HALF, c + INDOOR_GOAL_HALF]).astype(np.float32)
        boxes = indoor_boxes(rng)
    else:
        x_init = np.asarray(X_INIT, np.float32)
        goal = np.asarray(GOAL_BOX, np.float32)
        boxes = random_boxes(rng, int(p["n_obs"]), p["side"], x_init, goal)
    n_s = int(p["n"])
    n_goal = max(1, int(math.ceil(0.01 * n_s)))
    samples = free_samples(rng, n_s, boxes, goal, n_goal)
    return x_init, goal, np.ascontiguousarray(boxes, np.float32), samples


def make_scene(spec, seed: int, *, M: int = 10_000, S_max: int = 512,
               n: Optional[int] = None, N: Optional[int] = None,
               n_obs: Optional[int] = None, alpha: Optional[float] = None,
               sigma: Optional[float] = None, sigma_meas: float = 0.0) -> Scene:
    """Build one seeded query.  `spec` is a WORKLOADS key or a dict of the same
    fields; keyword arguments override individual fields."""
    p = dict(WORKLOADS[spec]) if isinstance(spec, str) else dict(spec)
    name = spec if isinstance(spec, str) else p.get("name", "custom")
    for k, v in (("n", n), ("N", N), ("n_obs", n_obs), ("alpha", alpha),
                 ("sigma", sigma)):
        if v is not None:
            p[k] = v
    x_init, goal, boxes, samples = _map_of(p, seed)
    Np = int(p["N"])
    noise = _rng(seed, 1).standard_normal((S_max, 6, Np), dtype=np.float32)
    noise_mc = _rng(seed, 2).standard_normal((S_max, 6, int(M)), dtype=np.float32)
    sc = Scene(samples=samples, obstacles=np.ascontiguousarray(boxes, np.float32),
               x_init=x_init, goal=goal, alpha=float(np.float32(p["alpha"])),
               N=Np, sigma=float(np.float32(p["sigma"])),
               noise=np.ascontiguousarray(noise), noise_mc=np.ascontiguousarray(noise_mc),
               name=name, seed=int(seed))
    if sigma_meas > 0.0:
        sc.sigma_meas = float(np.float32(sigma_meas))
        sc.noise_meas = np.ascontiguousarray(
            _rng(seed, 6).standard_normal((S_max, 3, Np), dtype=np.float32))
        sc.noise_mc_meas = np.ascontiguousarray(
            _rng(seed, 7).standard_normal((S_max, 3, int(M)), dtype=np.float32))
    return sc


# ---------------------------------------------------------------------------
# Maps for the learned-proposal workloads: random start and goal per map.
# ---------------------------------------------------------------------------
ROOM_CENTRES = [(0.125 + 0.25 * i, 0.125 + 0.25 * j) for i in range(4) for j in range(4)]


def random_map(kind: str, seed: int):
    """(x_init [6], goal [6], boxes [k, 6]) of one map.

    'boxes': n_obs ~ U{5..60} boxes with sides U[0.05, 0.25], a start uniform in
    [0.05, 0.95]^3 at rest and a 0.1-wide goal box at least 0.6 away.
    'indoor': the 4x4 room grid with random doorways, start and goal at the
    centres of two rooms at least two rooms apart (height 0.3), goal box 0.05."""
    rng = _rng(seed, 3)
    if kind == "indoor":
        boxes = indoor_boxes(rng)
        while True:
            a, b = rng.choice(16, 2, replace=False)
            (ax, ay), (bx, by) = ROOM_CENTRES[a], ROOM_CENTRES[b]
            if abs(ax - bx) + abs(ay - by) >= 0.5 - 1e-9:
                break
        x_init = np.array([ax, ay, 0.3, 0, 0, 0], np.float32)
        c = np.array([bx, by, 0.3])
        goal = np.concatenate([c - INDOOR_GOAL_HALF, c + INDOOR_GOAL_HALF]).astype(np.float32)
        return x_init, goal, boxes
    while True:
        s = rng.uniform(0.05, 0.95, 3)
        c = rng.uniform(0.1, 0.9, 3)
        if np.linalg.norm(c - s) >= 0.6:
            break
    x_init = np.concatenate([s, np.zeros(3)]).astype(np.float32)
    goal = np.concatenate([c - 0.05, c + 0.05]).astype(np.float32)
    boxes = random_boxes(rng, int(rng.integers(5, 61)), (0.05, 0.25), x_init, goal)
    return x_init, goal, boxes


def uniform_samples(seed: int, n: int, boxes, goal) -> np.ndarray:
    """SampleFree(n): 1% (at least one) in the goal box, the rest uniform in the
    unit cube, all outside the boxes; velocities uniform."""
    rng = _rng(seed, 4)
    return free_samples(rng, n, np.asarray(boxes, np.float32), goal, max(1, int(math.ceil(0.01 * n))))


# ---------------------------------------------------------------------------
# Batched workload: many independent queries of uneven size.
# ---------------------------------------------------------------------------
def batch_specs(seed: int, q: int = 256):
    """Shapes of q batched queries: n ~ U{1000..8000} samples, N in
    {64, 128, 256} particles, n_obs ~ U{5..60} random boxes with sides
    U[0.05, 0.25], alpha in {0.01, 0.05}, sigma 0.02."""
    rng = _rng(seed, 5)
    out = []
    for i in range(q):
        out.append(dict(n=int(rng.integers(1000, 8001)), N=int(rng.choice([64, 128, 256])),
                        n_obs=int(rng.integers(5, 61)), side=(0.05, 0.25), sigma=0.02,
                        alpha=float(rng.choice([0.01, 0.05])), indoor=False,
                        name=f"batch{i}"))
    return out


def batch_map(spec, seed: int):
    """(x_init, goal, boxes, samples) of one batched query; its noise arrays
    are drawn by the caller (on the device for large batches)."""
    return _map_of(spec, seed)


def batch_scene(seed: int, i: int, *, M: int = 10_000, S_max: int = 512) -> Scene:
    """Query i of the batch with batch seed `seed` (the shape batch_specs
    gives it and the map batch_map draws for it), with host-drawn noise
    arrays so that both implementations can consume the same values."""
    spec = batch_specs(seed, i + 1)[i]
    return make_scene(spec, workload_seed(4, 1000 * seed + i), M=M, S_max=S_max)
