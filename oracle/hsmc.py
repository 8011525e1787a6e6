"""Half-Space Monte Carlo (HSMC) collision model (oracle, FP64).

Test infrastructure only: it checks the HIP path and is never called by it.

The paper's exploration CP model (Sec. III-B, "Half-Space Monte Carlo"):
around each nominal waypoint position y (workspace = position) a local convex
region is built by a sequential process -- take the closest obstacle point,
keep the vector d from y to it, discard every obstacle that lies beyond the
plane through that point normal to d, repeat until no obstacle is left.  Each
d is then made perpendicular to the nominal velocity v at the waypoint
(eq. (7)): a = d - (d.v / v.v) v, b = a.a, and a particle whose deviation from
the nominal position is dy counts as colliding at that waypoint iff
a.dy > b for some of the waypoint's half-spaces.  As with the box model, a
particle is invalid once it collides at any waypoint of the plan (an OR over
the trajectory) and cp_hat is the invalid count over N.

Readings (the paper is silent on them):
  * obstacles are closed axis-aligned boxes; the closest point of a box to y
    is y clamped to the box; ties between boxes at the same distance go to the
    lowest box index;
  * a box is discarded when all of it lies in the closed half-space
    {z : d.(z - y) >= d.d} (the box that supplied d always is, through its
    closest point, so the loop ends after at most one step per box);
  * v = 0 (a waypoint at rest) leaves d unprojected: a = d;
  * a waypoint inside a box (d = 0) cannot occur on a collision-free edge; it
    would give a = 0, b = 0 and no particle collides there.
"""

from __future__ import annotations

import numpy as np


def closest_point(y, box):
    """Closest point of the closed box (lo xyz, hi xyz) to y."""
    b = np.asarray(box, np.float64)
    return np.minimum(np.maximum(np.asarray(y, np.float64), b[:3]), b[3:])


def local_region(y, boxes):
    """The d vectors of the local convex region around y, in the order the
    sequential process finds them."""
    y = np.asarray(y, np.float64)
    boxes = np.asarray(boxes, np.float64).reshape(-1, 6)
    remaining = list(range(boxes.shape[0]))
    ds = []
    while remaining:
        best, best_d2, best_d = None, np.inf, None
        for o in remaining:
            d = closest_point(y, boxes[o]) - y
            d2 = float(d @ d)
            if d2 < best_d2:
                best, best_d2, best_d = o, d2, d
        d = best_d
        ds.append(d)
        dd = float(d @ d)
        keep = []
        for o in remaining:
            lo, hi = boxes[o, :3], boxes[o, 3:]
            # smallest value of d.(z - y) over the box
            m = float(np.minimum(d * lo, d * hi).sum() - d @ y)
            if not (m >= dd or o == best):
                keep.append(o)
        remaining = keep
    return np.array(ds, np.float64).reshape(-1, 3)


def halfspaces(y, v, boxes):
    """(A [m, 3], b [m]) of eq. (7) at a waypoint with position y and velocity v."""
    d = local_region(y, boxes)
    v = np.asarray(v, np.float64)
    vv = float(v @ v)
    if vv > 0.0:
        a = d - np.outer(d @ v / vv, v)
    else:
        a = d.copy()
    b = np.einsum("ij,ij->i", a, a)
    return a, b


def violations(a, b, dy):
    """Per particle: does a.dy > b hold for some half-space?  dy [3, N]."""
    if a.shape[0] == 0:
        return np.zeros(dy.shape[1], bool)
    return ((a @ dy) > b[:, None]).any(axis=0)


def margins(a, b, dy):
    """Per particle: the largest signed distance (a.dy - b)/|a| beyond a plane
    (-inf without half-spaces or with a = 0)."""
    if a.shape[0] == 0:
        return np.full(dy.shape[1], -np.inf)
    na = np.sqrt(b)
    with np.errstate(divide="ignore", invalid="ignore"):
        m = np.where(na[:, None] > 0, ((a @ dy) - b[:, None]) / na[:, None], -np.inf)
    return m.max(axis=0)
