"""ctypes binding of libpump (include/pump.h): argument marshalling only.

Every step of the planner runs in the HIP library; this module converts numpy
arrays (host memory) or torch CUDA tensors (device memory) into the C
structures and reads results back.  It raises if the built library is absent.
"""

from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpump.so")

PUMP_OK = 0
PUMP_INFEASIBLE = 1
PUMP_NO_GOAL_PLAN = 2
PUMP_E_ARG = -1
PUMP_E_CAPACITY = -2
PUMP_E_HIP = -3
PUMP_E_STATE = -4
MEM_HOST = 0
MEM_DEVICE = 1

_f = ctypes.c_float
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_d = ctypes.c_double
_p = ctypes.c_void_p


class Config(ctypes.Structure):
    _fields_ = [("n_particles", _i32), ("max_nodes", _i32), ("max_obstacles", _i32),
                ("max_steps", _i32), ("mc_particles", _i32), ("preprune", _i32),
                ("dt", _f), ("q_pos", _f), ("q_vel", _f), ("r_track", _f), ("r_steer", _f),
                ("r_conn", _f), ("eta", _f), ("lambda_", _f), ("cp_model", _i32),
                ("estimator", _i32), ("smooth", _i32), ("reserved_", _i32), ("cap_edges", _i64), ("cap_plans", _i64),
                ("cap_pairs", _i64)]


class AABB(ctypes.Structure):
    _fields_ = [("lo", _f * 3), ("hi", _f * 3)]


class Problem(ctypes.Structure):
    _fields_ = [("samples", _p), ("n", _i32), ("obstacles", _p), ("n_obs", _i32),
                ("x_init", _f * 6), ("goal", AABB), ("alpha", _f), ("sigma", _f),
                ("noise", _p), ("noise_mc", _p), ("mem", _i32), ("sigma_meas", _f),
                ("noise_meas", _p), ("noise_mc_meas", _p)]


class Result(ctypes.Structure):
    _fields_ = [("status", _i32), ("n_goal_plans", _i32), ("n_front", _i32), ("best", _i32),
                ("best_plan", _i32), ("best_pop", _i32), ("best_mc_count", _i32),
                ("best_len", _i32), ("best_cost", _d), ("best_cp_mc", _d),
                ("partial_plans", _i64), ("simulated", _i64), ("preprune", _i64),
                ("inserted", _i64), ("survivors", _i64), ("dropped_steps", _i64),
                ("flagged", _i64), ("rounds", _i32), ("final_i", _i32), ("n_plans", _i32),
                ("n_edges", _i32), ("n_valid_nodes", _i32), ("c_cut", _i32), ("c_min", _i32),
                ("pad", _i32), ("ms_setup", _f), ("ms_explore", _f), ("ms_select", _f),
                ("ms_total", _f), ("sim_waypoints", _i64), ("sim_box_tests", _i64),
                ("smooth_beta", _d), ("smooth_cost", _d), ("smooth_mc_count", _i32),
                ("smooth_steps", _i32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class Tuning(ctypes.Structure):
    _fields_ = [("explore_threads", _i32), ("blocks_per_cu", _i32), ("order", _i32),
                ("use_graph", _i32), ("team_scale", _i32)]


class PumpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libpump status {code}: {msg}")
        self.code = code


_LIB = None

# exported symbols (must match include/pump.h)
EXPORTS = ["pump_config_default", "pump_create", "pump_destroy", "pump_plan", "pump_setup",
           "pump_explore_begin", "pump_explore_round", "pump_explore_run", "pump_select",
           "pump_get_deviation", "pump_get_graph", "pump_get_plans", "pump_get_candidates",
           "pump_get_front", "pump_get_path", "pump_mc_path", "pump_get_smooth_path",
           "pump_sample_halton", "pump_roadmap_create", "pump_roadmap_destroy",
           "pump_roadmap_info", "pump_set_roadmap", "pump_batch_set_roadmaps",
           "pump_set_timing",
           "pump_get_timing", "pump_set_explore_mode", "pump_get_explore_mode",
           "pump_set_barrier_patience", "pump_get_explore_fallbacks", "pump_get_chunked_rounds",
           "pump_status_str", "pump_last_error", "pump_mlp_create",
           "pump_mlp_destroy", "pump_mlp_num_params", "pump_mlp_set_params",
           "pump_mlp_get_params", "pump_mlp_get_state", "pump_mlp_set_state",
           "pump_mlp_adam_step", "pump_mlp_forward", "pump_mlp_loss_grad",
           "pump_mlp_train_step", "pump_mlp_condition", "pump_mlp_sample",
           "pump_mlp_sample_noalloc",
           "pump_mlp_last_error", "pump_batch_create", "pump_batch_destroy",
           "pump_batch_plan", "pump_batch_get_path", "pump_batch_tune",
           "pump_batch_last_error"]

TIMING_KINDS = ["deviation", "graph_mark", "graph_fill", "expand", "prune", "compact",
                "next_group", "select_front", "mc", "explore_single", "ph_expand",
                "ph_simulate", "ph_stair", "ph_mark", "ph_compact", "ph_next_group",
                "ph_group", "smooth", "expand_sim"]


# Contexts, roadmaps, batches and MLPs still open; closed by an exit handler
# registered after torch's (exit handlers run last-registered first), so the
# library frees its device memory, events and pinned buffers while the HIP
# runtime is whole rather than from object finalisers during interpreter
# teardown.
_LIVE = weakref.WeakSet()
_EXIT_HOOKED = False


def _close_all():
    for obj in list(_LIVE):
        try:
            obj.close()
        except Exception:
            pass


def _track(obj):
    global _EXIT_HOOKED
    if not _EXIT_HOOKED:
        atexit.register(_close_all)
        _EXIT_HOOKED = True
    _LIVE.add(obj)


def load(path: Optional[str] = None):
    """Load libpump (built in-tree); raises if it is missing."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise FileNotFoundError(f"{p} is not built; run __graft_entry__.build()")
    # Load torch's HIP runtime first so libpump binds to the same runtime
    # instance (same soname); device pointers and streams from torch are then
    # valid in the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(p)
    P = ctypes.POINTER
    sig = {
        "pump_config_default": (None, [P(Config)]),
        "pump_create": (_i32, [P(Config), _p, P(_p)]),
        "pump_destroy": (_i32, [_p]),
        "pump_plan": (_i32, [_p, P(Problem), P(Result)]),
        "pump_setup": (_i32, [_p, P(Problem)]),
        "pump_explore_begin": (_i32, [_p]),
        "pump_explore_round": (_i32, [_p, P(_i32)]),
        "pump_explore_run": (_i32, [_p]),
        "pump_select": (_i32, [_p, P(Result)]),
        "pump_get_deviation": (_i32, [_p, _p, _i64]),
        "pump_get_graph": (_i32, [_p, _p, _p, _p, _p, _p, _i64, P(_i64)]),
        "pump_get_plans": (_i32, [_p] + [_p] * 9 + [_i64, P(_i64)]),
        "pump_get_candidates": (_i32, [_p] + [_p] * 6 + [_i64, P(_i64)]),
        "pump_get_front": (_i32, [_p, _p, _p, _i32, P(_i32)]),
        "pump_get_path": (_i32, [_p, _i32, _p, _i32, P(_i32)]),
        "pump_mc_path": (_i32, [_p, _p, _i32, P(_i32)]),
        "pump_get_smooth_path": (_i32, [_p, _p, _i32, P(_i32)]),
        "pump_sample_halton": (_i32, [_i32, _i32, P(_f), P(_f), P(AABB), _i64, _p, _p]),
        "pump_roadmap_create": (_i32, [P(Config), _p, _i32, _i32, _p, P(_p)]),
        "pump_roadmap_destroy": (_i32, [_p]),
        "pump_roadmap_info": (_i32, [_p, P(_i32), P(_i64), P(_f)]),
        "pump_set_roadmap": (_i32, [_p, _p]),
        "pump_batch_set_roadmaps": (_i32, [_p, P(_p), _i32]),
        "pump_set_timing": (_i32, [_p, _i32]),
        "pump_get_timing": (_i32, [_p, _p, _p, _i32]),
        "pump_set_explore_mode": (_i32, [_p, _i32]),
        "pump_get_explore_mode": (_i32, [_p, P(_i32), P(_i32)]),
        "pump_set_barrier_patience": (_i32, [_p, _d]),
        "pump_get_explore_fallbacks": (_i32, [_p, P(_i64)]),
        "pump_get_chunked_rounds": (_i32, [_p, P(_i64)]),
        "pump_status_str": (ctypes.c_char_p, [_i32]),
        "pump_last_error": (ctypes.c_char_p, [_p]),
        "pump_mlp_create": (_i32, [_i32, _p, P(_p)]),
        "pump_mlp_destroy": (_i32, [_p]),
        "pump_mlp_num_params": (_i32, []),
        "pump_mlp_set_params": (_i32, [_p, _p, _i64]),
        "pump_mlp_get_params": (_i32, [_p, _p, _i64]),
        "pump_mlp_get_state": (_i32, [_p, _p, _p, _p, _i64, P(_i32)]),
        "pump_mlp_set_state": (_i32, [_p, _p, _p, _p, _i64, _i32]),
        "pump_mlp_adam_step": (_i32, [_p, _p, _i64, _f, _i32]),
        "pump_mlp_forward": (_i32, [_p, _p, _i32, _p, _i32]),
        "pump_mlp_loss_grad": (_i32, [_p, _p, _p, _i32, P(_f), _p, _i32]),
        "pump_mlp_train_step": (_i32, [_p, _p, _p, _i32, _f, P(_f), _i32]),
        "pump_mlp_condition": (_i32, [_p, _p, _p, _p, _p, _i32, _i32, _p]),
        "pump_mlp_sample": (_i32, [_p, _p, _i32, _p, _p, _i32, _p, _i32]),
        "pump_mlp_sample_noalloc": (_i32, [_p, _p, _i32, _p, _p, _i32, _p, _i32]),
        "pump_mlp_last_error": (ctypes.c_char_p, [_p]),
        "pump_batch_create": (_i32, [P(Config), _i32, _p, P(_p)]),
        "pump_batch_destroy": (_i32, [_p]),
        "pump_batch_plan": (_i32, [_p, P(Problem), P(_i32), _i32, P(Tuning), P(Result)]),
        "pump_batch_get_path": (_i32, [_p, _i32, _i32, _p, _i32, P(_i32)]),
        "pump_batch_tune": (_i32, [_p, P(Problem), P(_i32), _i32, P(Tuning), P(_d),
                                   ctypes.c_char_p]),
        "pump_batch_last_error": (ctypes.c_char_p, [_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _LIB = lib
    return lib


def default_config(**over) -> Config:
    lib = load()
    c = Config()
    lib.pump_config_default(ctypes.byref(c))
    for k, v in over.items():
        setattr(c, "lambda_" if k == "lam" else k, v)
    return c


def sample_halton(n, lo, hi, goal=None, n_goal=None, start=1, stream=None):
    """SampleFree(n) with the Halton sequence on the device (pump_sample_halton):
    a torch CUDA float32 tensor [n, 6].  n_goal defaults to max(1, n // 100)
    with a goal box (6 floats, lo xyz then hi xyz), else 0."""
    import torch
    lib = load()
    if n_goal is None:
        n_goal = max(1, n // 100) if goal is not None else 0
    out = torch.empty((n, 6), dtype=torch.float32, device="cuda")
    lo_a = (_f * 6)(*[float(v) for v in lo])
    hi_a = (_f * 6)(*[float(v) for v in hi])
    g = None
    if goal is not None:
        gb = np.asarray(goal, np.float32)
        g = AABB((_f * 3)(*gb[:3]), (_f * 3)(*gb[3:]))
    s = getattr(stream, "cuda_stream", stream) if stream is not None else \
        torch.cuda.current_stream().cuda_stream
    rc = lib.pump_sample_halton(int(n), int(n_goal), lo_a, hi_a,
                                ctypes.byref(g) if g is not None else None, int(start),
                                out.data_ptr(), s)
    if rc != 0:
        raise PumpError(rc, "pump_sample_halton failed")
    return out


def _ptr(a):
    """Data pointer of a numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _np(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


class Planner:
    """One libpump context.  Inputs may be numpy arrays (host) or torch CUDA
    tensors (device); `stream` is a torch.cuda.Stream or raw hipStream_t."""

    def __init__(self, stream=None, **cfg):
        self.lib = load()
        self.cfg = default_config(**cfg)
        s = None
        if stream is not None:
            s = getattr(stream, "cuda_stream", stream)
        self.ctx = _p()
        rc = self.lib.pump_create(ctypes.byref(self.cfg), s, ctypes.byref(self.ctx))
        if rc != 0:
            raise PumpError(rc, "pump_create failed")
        self._keep = []
        _track(self)

    def close(self):
        if self.ctx:
            self.lib.pump_destroy(self.ctx)
            self.ctx = _p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow_positive=False):
        if rc < 0 or (rc > 0 and not allow_positive):
            msg = self.lib.pump_last_error(self.ctx) or b""
            raise PumpError(rc, msg.decode())
        return rc

    # -- problem -------------------------------------------------------------
    def problem(self, samples, obstacles, x_init, goal, alpha, sigma, noise, noise_mc,
                sigma_meas=0.0, noise_meas=None, noise_mc_meas=None):
        """Build the C problem struct.  Array arguments are numpy (host) or
        torch CUDA tensors (device), all of the same kind.  The measurement
        noise is read only with estimator = 1 (LQG)."""
        dev = not isinstance(samples, np.ndarray)
        if not dev:
            samples = _np(samples, np.float32)
            obstacles = _np(obstacles, np.float32).reshape(-1, 6)
            noise = _np(noise, np.float32)
            noise_mc = _np(noise_mc, np.float32)
            if noise_meas is not None:
                noise_meas = _np(noise_meas, np.float32)
            if noise_mc_meas is not None:
                noise_mc_meas = _np(noise_mc_meas, np.float32)
        self._keep = [samples, obstacles, noise, noise_mc, noise_meas, noise_mc_meas]
        pr = Problem()
        pr.samples = _ptr(samples)
        pr.n = int(samples.shape[0])
        pr.obstacles = _ptr(obstacles) if int(obstacles.shape[0]) else None
        pr.n_obs = int(obstacles.shape[0])
        xi = np.asarray(x_init, np.float32)
        for k in range(6):
            pr.x_init[k] = float(xi[k])
        g = np.asarray(goal, np.float32)
        for k in range(3):
            pr.goal.lo[k] = float(g[k])
            pr.goal.hi[k] = float(g[3 + k])
        pr.alpha = float(alpha)
        pr.sigma = float(sigma)
        pr.noise = _ptr(noise)
        pr.noise_mc = _ptr(noise_mc)
        pr.mem = MEM_DEVICE if dev else MEM_HOST
        pr.sigma_meas = float(sigma_meas)
        pr.noise_meas = _ptr(noise_meas)
        pr.noise_mc_meas = _ptr(noise_mc_meas)
        return pr

    def scene_problem(self, sc, device=False):
        if device:
            import torch
            t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
            tm = lambda a: None if a is None else t(a)
            return self.problem(t(sc.samples), t(sc.obstacles), sc.x_init, sc.goal, sc.alpha,
                                sc.sigma, t(sc.noise), t(sc.noise_mc), sc.sigma_meas,
                                tm(sc.noise_meas), tm(sc.noise_mc_meas))
        return self.problem(sc.samples, sc.obstacles, sc.x_init, sc.goal, sc.alpha, sc.sigma,
                            sc.noise, sc.noise_mc, sc.sigma_meas, sc.noise_meas,
                            sc.noise_mc_meas)

    # -- whole query and stages ----------------------------------------------
    def plan(self, pr) -> dict:
        res = Result()
        rc = self.lib.pump_plan(self.ctx, ctypes.byref(pr), ctypes.byref(res))
        self._check(rc, allow_positive=True)
        return res.as_dict()

    def setup(self, pr):
        self._check(self.lib.pump_setup(self.ctx, ctypes.byref(pr)))

    def explore_begin(self):
        self._check(self.lib.pump_explore_begin(self.ctx))

    def explore_round(self) -> bool:
        d = _i32(0)
        self._check(self.lib.pump_explore_round(self.ctx, ctypes.byref(d)))
        return bool(d.value)

    def explore_run(self):
        self._check(self.lib.pump_explore_run(self.ctx))

    def select(self) -> dict:
        res = Result()
        rc = self.lib.pump_select(self.ctx, ctypes.byref(res))
        self._check(rc, allow_positive=True)
        return res.as_dict()

    # -- readers ---------------------------------------------------------------
    def deviation(self):
        N = self.cfg.n_particles
        S = self.cfg.max_steps
        out = np.zeros((S + 1, 3, N), np.float32)
        self._check(self.lib.pump_get_deviation(self.ctx, out.ctypes.data, out.size))
        return out

    def graph(self, n_nodes):
        ne = _i64(0)
        self._check(self.lib.pump_get_graph(self.ctx, None, None, None, None, None, 0,
                                            ctypes.byref(ne)))
        E = ne.value
        row = np.zeros(n_nodes + 1, np.int32)
        col = np.zeros(max(E, 1), np.int32)
        tau = np.zeros(max(E, 1), np.float64)
        cost = np.zeros(max(E, 1), np.float64)
        valid = np.zeros(n_nodes, np.uint8)
        self._check(self.lib.pump_get_graph(self.ctx, row.ctypes.data, col.ctypes.data,
                                            tau.ctypes.data, cost.ctypes.data, valid.ctypes.data,
                                            max(E, 1), ctypes.byref(ne)))
        return dict(row_ptr=row, col=col[:E], tau=tau[:E], cost=cost[:E], valid=valid.astype(bool))

    def plans(self):
        n = _i64(0)
        self._check(self.lib.pump_get_plans(self.ctx, *([None] * 9), 0, ctypes.byref(n)))
        n = n.value
        W = self.cfg.n_particles // 32
        out = dict(head=np.zeros(n, np.int32), parent=np.zeros(n, np.int32),
                   edge=np.zeros(n, np.int32), cost=np.zeros(n, np.float64),
                   step=np.zeros(n, np.int32), pop=np.zeros(n, np.int32),
                   round=np.zeros(n, np.int32), state=np.zeros(n, np.uint8),
                   mask=np.zeros((n, W), np.uint32))
        ks = ["head", "parent", "edge", "cost", "step", "pop", "round", "state", "mask"]
        self._check(self.lib.pump_get_plans(self.ctx, *[out[k].ctypes.data for k in ks], n,
                                            ctypes.byref(_i64(0))))
        return out

    def candidates(self):
        n = _i64(0)
        self._check(self.lib.pump_get_candidates(self.ctx, *([None] * 6), 0, ctypes.byref(n)))
        n = n.value
        W = self.cfg.n_particles // 32
        out = dict(flag=np.zeros(n, np.uint8), pop=np.zeros(n, np.int32),
                   parent=np.zeros(n, np.int32), head=np.zeros(n, np.int32),
                   cost=np.zeros(n, np.float64), mask=np.zeros((n, W), np.uint32))
        ks = ["flag", "pop", "parent", "head", "cost", "mask"]
        self._check(self.lib.pump_get_candidates(self.ctx, *[out[k].ctypes.data for k in ks],
                                                 n, ctypes.byref(_i64(0))))
        return out

    def front(self):
        n = _i32(0)
        self._check(self.lib.pump_get_front(self.ctx, None, None, 0, ctypes.byref(n)))
        ids = np.zeros(max(n.value, 1), np.int32)
        mc = np.zeros(max(n.value, 1), np.int32)
        self._check(self.lib.pump_get_front(self.ctx, ids.ctypes.data, mc.ctypes.data,
                                            ids.size, ctypes.byref(n)))
        return ids[:n.value], mc[:n.value]

    def path(self, plan):
        cap = self.cfg.max_steps + 1
        buf = np.zeros(cap, np.int32)
        ln = _i32(0)
        self._check(self.lib.pump_get_path(self.ctx, int(plan), buf.ctypes.data, cap,
                                           ctypes.byref(ln)))
        return tuple(int(v) for v in buf[:ln.value])

    def set_explore_mode(self, mode: int):
        """1: all rounds in one launch; 0: one launch per phase; 2: chosen
        per query from the graph's size (the default)."""
        self._check(self.lib.pump_set_explore_mode(self.ctx, int(mode)))

    def explore_mode(self):
        m, b = _i32(0), _i32(0)
        self._check(self.lib.pump_get_explore_mode(self.ctx, ctypes.byref(m), ctypes.byref(b)))
        return m.value, b.value

    def set_barrier_patience(self, ms: float):
        """Longest wait at a barrier of the single-launch Explore (ms)."""
        self._check(self.lib.pump_set_barrier_patience(self.ctx, ctypes.c_double(ms)))

    def explore_fallbacks(self) -> int:
        n = _i64(0)
        self._check(self.lib.pump_get_explore_fallbacks(self.ctx, ctypes.byref(n)))
        return int(n.value)

    def chunked_rounds(self) -> int:
        """Rounds of the current Explore that ran in chunks of cap_pairs."""
        n = _i64(0)
        self._check(self.lib.pump_get_chunked_rounds(self.ctx, ctypes.byref(n)))
        return int(n.value)

    def set_timing(self, on: bool):
        self._check(self.lib.pump_set_timing(self.ctx, 1 if on else 0))

    def timing(self) -> dict:
        n = len(TIMING_KINDS)
        ms = np.zeros(n, np.float64)
        cnt = np.zeros(n, np.int64)
        self._check(self.lib.pump_get_timing(self.ctx, ms.ctypes.data, cnt.ctypes.data, n))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(TIMING_KINDS)}

    def set_roadmap(self, rm):
        """Build later queries' graphs from a cached Roadmap (None: from
        scratch)."""
        self._check(self.lib.pump_set_roadmap(self.ctx, rm.rm if rm is not None else None))
        self._rm = rm

    def smooth_path(self):
        """Waypoints [steps + 1, 3] of the trajectory the last selection
        returned (the Smooth blend, or p* itself)."""
        cap = int(self.cfg.max_steps)
        buf = np.zeros((cap + 1, 3), np.float64)
        n = _i32(0)
        self._check(self.lib.pump_get_smooth_path(self.ctx, buf.ctypes.data, cap, ctypes.byref(n)))
        return buf[:n.value + 1].copy()

    def mc_path(self, nodes):
        nd = np.ascontiguousarray(np.asarray(nodes, np.int32))
        c = _i32(0)
        self._check(self.lib.pump_mc_path(self.ctx, nd.ctypes.data, int(nd.shape[0]),
                                          ctypes.byref(c)))
        return int(c.value)


def plan_paths(pl: dict):
    """Node sequences of every plan from the plan-store arrays (host side)."""
    head, parent = pl["head"], pl["parent"]
    paths = [None] * head.shape[0]
    for p in range(head.shape[0]):
        if parent[p] < 0:
            paths[p] = (int(head[p]),)
        else:
            paths[p] = paths[parent[p]] + (int(head[p]),)
    return paths


class MLP:
    """The learned proposal network (pump_mlp_*).  Arrays are numpy (host) or
    torch CUDA tensors (device)."""

    def __init__(self, max_batch, stream=None):
        self.lib = load()
        s = None if stream is None else getattr(stream, "cuda_stream", stream)
        self.m = _p()
        rc = self.lib.pump_mlp_create(int(max_batch), s, ctypes.byref(self.m))
        if rc != 0:
            raise PumpError(rc, "pump_mlp_create failed")
        self.n_params = self.lib.pump_mlp_num_params()
        self.max_batch = int(max_batch)
        _track(self)

    def close(self):
        if self.m:
            self.lib.pump_mlp_destroy(self.m)
            self.m = _p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise PumpError(rc, (self.lib.pump_mlp_last_error(self.m) or b"").decode())

    @staticmethod
    def _mem(a):
        return MEM_HOST if isinstance(a, np.ndarray) else MEM_DEVICE

    def set_params(self, flat):
        f = _np(flat, np.float32)
        self._check(self.lib.pump_mlp_set_params(self.m, f.ctypes.data, f.size))

    def get_params(self):
        f = np.zeros(self.n_params, np.float32)
        self._check(self.lib.pump_mlp_get_params(self.m, f.ctypes.data, f.size))
        return f

    def get_state(self) -> dict:
        """Parameters, Adam moments and step counter (a training checkpoint)."""
        st = {k: np.zeros(self.n_params, np.float32) for k in ("params", "m1", "m2")}
        t = _i32(0)
        self._check(self.lib.pump_mlp_get_state(self.m, st["params"].ctypes.data,
                                                st["m1"].ctypes.data, st["m2"].ctypes.data,
                                                self.n_params, ctypes.byref(t)))
        st["t"] = int(t.value)
        return st

    def set_state(self, st: dict):
        a = {k: _np(st[k], np.float32) for k in ("params", "m1", "m2")}
        self._check(self.lib.pump_mlp_set_state(self.m, a["params"].ctypes.data,
                                                a["m1"].ctypes.data, a["m2"].ctypes.data,
                                                self.n_params, int(st["t"])))

    def save(self, path):
        """The training state to an .npz file (plain arrays, no pickles)."""
        st = self.get_state()
        np.savez(path, params=st["params"], m1=st["m1"], m2=st["m2"],
                 t=np.array([st["t"]], np.int64))

    def load(self, path):
        with np.load(path, allow_pickle=False) as z:
            self.set_state(dict(params=z["params"], m1=z["m1"], m2=z["m2"], t=int(z["t"][0])))

    def adam_step(self, grads, lr):
        """One Adam update with the given gradient vector."""
        g = _np(grads, np.float32)
        self._check(self.lib.pump_mlp_adam_step(self.m, g.ctypes.data, g.size, float(lr), MEM_HOST))

    def forward(self, cond):
        if isinstance(cond, np.ndarray):
            cond = _np(cond, np.float32)
            out = np.zeros((cond.shape[0], 208), np.float32)
        else:
            import torch
            out = torch.empty((cond.shape[0], 208), dtype=torch.float32, device=cond.device)
        self._check(self.lib.pump_mlp_forward(self.m, _ptr(cond), int(cond.shape[0]), _ptr(out),
                                              self._mem(cond)))
        return out

    def loss_grad(self, cond, target):
        cond = _np(cond, np.float32)
        target = _np(target, np.float32)
        g = np.zeros(self.n_params, np.float32)
        loss = _f(0)
        self._check(self.lib.pump_mlp_loss_grad(self.m, cond.ctypes.data, target.ctypes.data,
                                                int(cond.shape[0]), ctypes.byref(loss),
                                                g.ctypes.data, MEM_HOST))
        return float(loss.value), g

    def train_step(self, cond, target, lr):
        if isinstance(cond, np.ndarray):
            cond = _np(cond, np.float32)
            target = _np(target, np.float32)
        loss = _f(0)
        self._check(self.lib.pump_mlp_train_step(self.m, _ptr(cond), _ptr(target),
                                                 int(cond.shape[0]), float(lr),
                                                 ctypes.byref(loss), self._mem(cond)))
        return float(loss.value)

    def condition(self, x_init, goal, boxes, n_obs):
        """Device tensors in, device tensor [q][396] out."""
        import torch
        q = int(x_init.shape[0])
        out = torch.empty((q, 396), dtype=torch.float32, device=x_init.device)
        self._check(self.lib.pump_mlp_condition(self.m, _ptr(x_init), _ptr(goal), _ptr(boxes),
                                                _ptr(n_obs), q, int(boxes.shape[1]), _ptr(out)))
        return out

    def sample(self, cond, u, eps):
        q, n = int(u.shape[0]), int(u.shape[1])
        if isinstance(cond, np.ndarray):
            cond, u, eps = _np(cond, np.float32), _np(u, np.float32), _np(eps, np.float32)
            out = np.zeros((q, n, 6), np.float32)
        else:
            import torch
            out = torch.empty((q, n, 6), dtype=torch.float32, device=cond.device)
        self._check(self.lib.pump_mlp_sample(self.m, _ptr(cond), q, _ptr(u), _ptr(eps), n,
                                             _ptr(out), self._mem(cond)))
        return out

    def sample_noalloc(self, cond, u, eps):
        """sample() through pump_mlp_sample_noalloc (no allocation per call;
        host arrays are staged through the library's static per-GPU array)."""
        q, n = int(u.shape[0]), int(u.shape[1])
        if isinstance(cond, np.ndarray):
            cond, u, eps = _np(cond, np.float32), _np(u, np.float32), _np(eps, np.float32)
            out = np.zeros((q, n, 6), np.float32)
        else:
            import torch
            out = torch.empty((q, n, 6), dtype=torch.float32, device=cond.device)
        self._check(self.lib.pump_mlp_sample_noalloc(self.m, _ptr(cond), q, _ptr(u), _ptr(eps),
                                                     n, _ptr(out), self._mem(cond)))
        return out


class Roadmap:
    """BuildGraph's obstacle-independent part over a fixed sample set
    (pump_roadmap_create).  `samples` is a numpy array (host) or a torch CUDA
    tensor (device); cfg keywords as for Planner (r_steer, r_conn, max_nodes,
    cap_edges matter)."""

    def __init__(self, samples, stream=None, **cfg):
        self.lib = load()
        self.cfg = default_config(**cfg)
        dev = not isinstance(samples, np.ndarray)
        if not dev:
            samples = _np(samples, np.float32)
        s = getattr(stream, "cuda_stream", stream) if stream is not None else None
        self.rm = _p()
        rc = self.lib.pump_roadmap_create(ctypes.byref(self.cfg), _ptr(samples),
                                          int(samples.shape[0]), MEM_DEVICE if dev else MEM_HOST,
                                          s, ctypes.byref(self.rm))
        if rc != 0:
            raise PumpError(rc, "pump_roadmap_create failed")
        _track(self)

    def info(self):
        n, e, ms = _i32(0), _i64(0), _f(0.0)
        self.lib.pump_roadmap_info(self.rm, ctypes.byref(n), ctypes.byref(e), ctypes.byref(ms))
        return dict(n=n.value, n_edges=e.value, ms_build=ms.value)

    def close(self):
        if self.rm:
            self.lib.pump_roadmap_destroy(self.rm)
            self.rm = _p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """The batched engine: many device-resident queries in one graph launch.
    Queries are (samples, obstacles, x_init, goal, alpha, sigma, noise,
    noise_mc) with torch CUDA tensors for the arrays, optionally followed by
    (sigma_meas, noise_meas, noise_mc_meas) for LQG tracking; N is taken from
    noise.shape[2]."""

    def __init__(self, max_queries, stream=None, **cfg):
        self.lib = load()
        self.cfg = default_config(**cfg)
        s = getattr(stream, "cuda_stream", stream) if stream is not None else None
        self.b = _p()
        rc = self.lib.pump_batch_create(ctypes.byref(self.cfg), int(max_queries), s,
                                        ctypes.byref(self.b))
        if rc != 0:
            raise PumpError(rc, "pump_batch_create failed")
        self._keep = []
        _track(self)

    def close(self):
        if self.b:
            self.lib.pump_batch_destroy(self.b)
            self.b = _p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, rc):
        msg = self.lib.pump_batch_last_error(self.b) or b""
        raise PumpError(rc, msg.decode())

    def _problems(self, queries):
        q = len(queries)
        arr = (Problem * q)()
        ns = (_i32 * q)()
        keep = []
        for i, qu in enumerate(queries):
            smp, obs, x0, goal, alpha, sigma, noise, noise_mc = qu[:8]
            sm, nm, nmc = (tuple(qu[8:11]) + (0.0, None, None)[len(qu[8:11]):])
            keep += [smp, obs, noise, noise_mc, nm, nmc]
            pr = arr[i]
            pr.samples = _ptr(smp)
            pr.n = int(smp.shape[0])
            pr.obstacles = _ptr(obs) if int(obs.shape[0]) else None
            pr.n_obs = int(obs.shape[0])
            xi = np.asarray(x0, np.float32)
            for k in range(6):
                pr.x_init[k] = float(xi[k])
            g = np.asarray(goal, np.float32)
            for k in range(3):
                pr.goal.lo[k] = float(g[k])
                pr.goal.hi[k] = float(g[3 + k])
            pr.alpha = float(alpha)
            pr.sigma = float(sigma)
            pr.noise = _ptr(noise)
            pr.noise_mc = _ptr(noise_mc)
            pr.mem = MEM_DEVICE
            pr.sigma_meas = float(sm)
            pr.noise_meas = _ptr(nm)
            pr.noise_mc_meas = _ptr(nmc)
            ns[i] = int(noise.shape[2])
        self._keep = keep
        return arr, ns

    @staticmethod
    def _sync_torch():
        # inputs written on torch's stream must be complete before the
        # library's stream reads them
        import torch
        torch.cuda.current_stream().synchronize()

    def plan(self, queries, tuning=None, raise_on_error=True):
        arr, ns = self._problems(queries)
        self._sync_torch()
        q = len(queries)
        out = (Result * q)()
        t = None
        if tuning is not None:
            t = Tuning(*[int(tuning.get(k, d)) for k, d in (
                ("explore_threads", 256), ("blocks_per_cu", 2), ("order", 1), ("use_graph", 1),
                ("team_scale", 64))])
        rc = self.lib.pump_batch_plan(self.b, arr, ns, q, ctypes.byref(t) if t else None, out)
        if rc < 0 and raise_on_error:
            self._err(rc)
        return [r.as_dict() for r in out]

    def set_roadmaps(self, rms):
        """Per-query cached roadmaps (Roadmap or None each) for later plans."""
        arr = (_p * max(1, len(rms)))(*[r.rm if r is not None else None for r in rms])
        rc = self.lib.pump_batch_set_roadmaps(self.b, arr, len(rms))
        if rc != 0:
            self._err(rc)
        self._rms = list(rms)

    def path(self, query, plan):
        cap = self.cfg.max_steps + 1
        buf = np.zeros(cap, np.int32)
        n = _i32(0)
        rc = self.lib.pump_batch_get_path(self.b, int(query), int(plan), buf.ctypes.data, cap,
                                          ctypes.byref(n))
        if rc != 0:
            self._err(rc)
        return tuple(int(v) for v in buf[:n.value])

    def tune(self, queries, json_path=None):
        arr, ns = self._problems(queries)
        self._sync_torch()
        best = Tuning()
        ms = _d(0.0)
        rc = self.lib.pump_batch_tune(self.b, arr, ns, len(queries), ctypes.byref(best),
                                      ctypes.byref(ms),
                                      json_path.encode() if json_path else None)
        if rc != 0:
            self._err(rc)
        return dict(explore_threads=best.explore_threads, blocks_per_cu=best.blocks_per_cu,
                    order=best.order, use_graph=best.use_graph,
                    team_scale=best.team_scale), ms.value
