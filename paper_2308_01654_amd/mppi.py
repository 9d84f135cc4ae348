"""ctypes binding of the C ABI in ``include/mppi.h``.

The functions ``mppi_*`` below have the names and arguments of the C entry
points (argument marshalling only; every step of the iteration runs in the
HIP library).  ``Planner`` wraps one handle for convenience.  The library is
loaded from this package directory (``libmppi.so``, built by
``paper_2308_01654_amd.build``); if it is missing, loading raises: there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmppi.so")

OK = 0
E_INVALID = -1
E_NOMEM = -2
E_DEVICE = -3
E_NONFINITE = -4
E_BUSY = -5
E_NOT_READY = -6


class MppiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("mppi status %d: %s" % (status, msg))
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_int32), ("T", ctypes.c_int32),
        ("dt", ctypes.c_double), ("wheelbase", ctypes.c_double),
        ("lam", ctypes.c_double), ("gamma", ctypes.c_double),
        ("sigma", ctypes.c_double * 2), ("u_min", ctypes.c_double * 2),
        ("u_max", ctypes.c_double * 2), ("v_max", ctypes.c_double),
        ("w_track", ctypes.c_double), ("w_speed", ctypes.c_double),
        ("w_effort", ctypes.c_double), ("w_coll", ctypes.c_double),
        ("d_safe_c", ctypes.c_double), ("d_safe_0", ctypes.c_double),
        ("n_ego", ctypes.c_int32), ("ego_r", ctypes.c_double),
        ("ego_off", ctypes.c_double * 4),
        ("seed", ctypes.c_uint64),
        ("max_waypoints", ctypes.c_int32), ("max_circles", ctypes.c_int32),
        ("smoothing", ctypes.c_int32),
        ("w_target", ctypes.c_double), ("w_yaw", ctypes.c_double),
        ("collision_only", ctypes.c_int32),
        ("model", ctypes.c_int32),
        ("per_step_weights", ctypes.c_int32),
    ]


class Scene(ctypes.Structure):
    _fields_ = [
        ("waypoints", ctypes.POINTER(ctypes.c_double)), ("n_waypoints", ctypes.c_int32),
        ("circles", ctypes.POINTER(ctypes.c_double)), ("n_circles", ctypes.c_int32),
    ]


class IterStats(ctypes.Structure):
    _fields_ = [
        ("s_min", ctypes.c_double), ("log_z", ctypes.c_double), ("ess", ctypes.c_double),
        ("n_iter", ctypes.c_uint64), ("status", ctypes.c_int32),
        ("lanes_per_sample", ctypes.c_int32),
    ]


class Profile(ctypes.Structure):
    _fields_ = [
        ("iter_ms", ctypes.c_double), ("iter_launches", ctypes.c_int64),
        ("aux_ms", ctypes.c_double), ("aux_launches", ctypes.c_int64),
        ("rollout_ms", ctypes.c_double), ("rollout_launches", ctypes.c_int64),
    ]


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("hbm_budget_bytes", ctypes.c_uint64), ("n_streams", ctypes.c_int32),
        ("max_batch", ctypes.c_int32), ("queue_cap", ctypes.c_int32), ("plain", ctypes.c_int32),
        ("deadline_ms", ctypes.c_double),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
        ("rejected", ctypes.c_uint64), ("failed", ctypes.c_uint64),
        ("launches", ctypes.c_uint64), ("mean_batch", ctypes.c_double),
        ("mean_ms", ctypes.c_double), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
        ("p999_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
        ("hbm_peak_bytes", ctypes.c_uint64), ("max_queue", ctypes.c_int32),
        ("deadline_misses", ctypes.c_uint64),
    ]


class ReplayPlan(ctypes.Structure):
    _fields_ = [
        ("n_requests", ctypes.c_int32), ("vid", ctypes.POINTER(ctypes.c_int32)),
        ("x0", ctypes.POINTER(ctypes.c_double)), ("scene", ctypes.POINTER(ctypes.c_int32)),
        ("scenes", ctypes.POINTER(Scene)), ("n_scenes", ctypes.c_int32),
        ("arrival_ns", ctypes.POINTER(ctypes.c_uint64)),
    ]


# (name, restype, argtypes) of every exported entry point
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_sz = ctypes.c_size_t
_i32 = ctypes.c_int32
SIGNATURES = [
    ("mppi_create", _i32, [ctypes.POINTER(Config), _vp, ctypes.POINTER(_vp)]),
    ("mppi_destroy", _i32, [_vp]),
    ("mppi_step", _i32, [_vp, _dp, ctypes.POINTER(Scene)]),
    ("mppi_set_scene", _i32, [_vp, _dp, ctypes.POINTER(Scene)]),
    ("mppi_step_resident", _i32, [_vp, _dp]),
    ("mppi_step_batch", _i32, [ctypes.POINTER(_vp), _dp, ctypes.POINTER(Scene), _i32]),
    ("mppi_sync", _i32, [_vp]),
    ("mppi_get_controls", _i32, [_vp, _dp, _sz]),
    ("mppi_set_controls", _i32, [_vp, _dp, _sz]),
    ("mppi_shift", _i32, [_vp, _i32]),
    ("mppi_get_state", _i32, [_vp, _dp, _sz, _u64p, _u64p]),
    ("mppi_set_state", _i32, [_vp, _dp, _sz, ctypes.c_uint64]),
    ("mppi_get_costs", _i32, [_vp, _fp, _sz]),
    ("mppi_get_weights", _i32, [_vp, _dp, _sz]),
    ("mppi_get_noise", _i32, [_vp, _fp, _sz]),
    ("mppi_get_trajectory", _i32, [_vp, _dp, _sz, _dp, _sz]),
    ("mppi_set_steering", _i32, [_vp, ctypes.c_double]),
    ("mppi_get_stage_costs", _i32, [_vp, _fp, _sz]),
    ("mppi_get_iter_stats", _i32, [_vp, ctypes.POINTER(IterStats)]),
    ("mppi_set_lanes_per_sample", _i32, [_vp, _i32]),
    ("mppi_set_staging", _i32, [_vp, _i32]),
    ("mppi_set_occupancy", _i32, [_vp, _i32]),
    ("mppi_set_culling", _i32, [_vp, _i32]),
    ("mppi_get_stream", _i32, [_vp, ctypes.POINTER(_vp)]),
    ("mppi_set_profiling", _i32, [_vp, _i32]),
    ("mppi_get_profile", _i32, [_vp, ctypes.POINTER(Profile)]),
    ("mppi_step_static", _i32, [ctypes.POINTER(Config), _dp, ctypes.POINTER(Scene), _vp,
                                ctypes.c_uint64, _vp, _vp]),
    ("mppi_debug_philox", _i32, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                 ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _u32p, _sz]),
    ("mppi_bench_copy", _i32, [_sz, _i32]),
    ("mppi_server_now_ns", ctypes.c_uint64, []),
    ("mppi_server_create", _i32, [ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)]),
    ("mppi_server_destroy", _i32, [_vp]),
    ("mppi_server_add_vehicle", _i32, [_vp, ctypes.POINTER(Config), ctypes.POINTER(_i32)]),
    ("mppi_server_submit", _i32, [_vp, _i32, _dp, ctypes.POINTER(Scene), ctypes.c_uint64, _u64p]),
    ("mppi_server_poll", _i32, [_vp, ctypes.c_uint64, _dp, _sz, _u64p]),
    ("mppi_server_wait_idle", _i32, [_vp]),
    ("mppi_server_get_stats", _i32, [_vp, ctypes.POINTER(ServerStats)]),
    ("mppi_server_reset_stats", _i32, [_vp]),
    ("mppi_server_get_vehicle_state", _i32, [_vp, _i32, _dp, _sz, _u64p, _u64p]),
    ("mppi_server_set_vehicle_state", _i32, [_vp, _i32, _dp, _sz, ctypes.c_uint64, ctypes.c_uint64]),
    ("mppi_server_replay", _i32, [_vp, ctypes.POINTER(ReplayPlan), _dp]),
    ("mppi_status_str", ctypes.c_char_p, [_i32]),
    ("mppi_last_error", ctypes.c_char_p, []),
    ("mppi_version", ctypes.c_char_p, []),
]

_lib = None
_lock = threading.Lock()


def load(path: str = LIB_PATH):
    """Load libmppi.so (raises OSError if it is not built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise OSError("HIP library %s is not built; run "
                              "`python -m paper_2308_01654_amd.build`" % path)
            L = ctypes.CDLL(path)
            for name, res, args in SIGNATURES:
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


def check(status):
    if status != OK:
        raise MppiError(status, load().mppi_last_error().decode(errors="replace"))
    return status


def config_from_params(p, max_waypoints=2048, max_circles=1024) -> Config:
    c = Config()
    c.K, c.T = int(p["K"]), int(p["T"])
    c.dt, c.wheelbase = float(p["dt"]), float(p["wheelbase"])
    c.lam, c.gamma = float(p["lam"]), float(p["gamma"])
    for i in range(2):
        c.sigma[i] = float(p["sigma"][i])
        c.u_min[i] = float(p["u_min"][i])
        c.u_max[i] = float(p["u_max"][i])
    c.v_max = float(p["v_max"])
    c.w_track, c.w_speed = float(p["w_track"]), float(p["w_speed"])
    c.w_effort, c.w_coll = float(p["w_effort"]), float(p["w_coll"])
    c.d_safe_c, c.d_safe_0 = float(p["d_safe_c"]), float(p["d_safe_0"])
    offs = list(p["ego_off"])
    c.n_ego = len(offs)
    c.ego_r = float(p["ego_r"])
    for i, o in enumerate(offs):
        c.ego_off[i] = float(o)
    c.seed = int(p["seed"])
    c.max_waypoints = int(max_waypoints)
    c.max_circles = int(max_circles)
    c.smoothing = int(p.get("smoothing", 0))
    c.w_target = float(p.get("w_target", 0.0))
    c.w_yaw = float(p.get("w_yaw", 0.0))
    c.collision_only = int(p.get("collision_only", 0))
    c.model = int(p.get("model", 0))
    c.per_step_weights = int(p.get("per_step", 0))
    return c


def make_scene(waypoints, circles):
    """Returns (Scene, keepalive) for float64 arrays [n][4] and [n][5]."""
    wp = np.ascontiguousarray(np.asarray(waypoints, dtype=np.float64).reshape(-1, 4))
    ci = np.ascontiguousarray(np.asarray(circles, dtype=np.float64).reshape(-1, 5))
    s = Scene()
    s.waypoints = wp.ctypes.data_as(_dp)
    s.n_waypoints = wp.shape[0]
    s.circles = ci.ctypes.data_as(_dp) if ci.shape[0] else None
    s.n_circles = ci.shape[0]
    return s, (wp, ci)


# ---- thin wrappers with the C names (return the status) ----------------------

def mppi_create(cfg: Config, hip_stream=None):
    h = _vp()
    st = load().mppi_create(ctypes.byref(cfg), hip_stream, ctypes.byref(h))
    return st, h


def mppi_destroy(h):
    return load().mppi_destroy(h)


def mppi_step(h, x0, scene: Scene):
    x = np.ascontiguousarray(np.asarray(x0, dtype=np.float64))
    return load().mppi_step(h, x.ctypes.data_as(_dp), ctypes.byref(scene))


def mppi_set_scene(h, x0, scene: Scene):
    x = np.ascontiguousarray(np.asarray(x0, dtype=np.float64))
    return load().mppi_set_scene(h, x.ctypes.data_as(_dp), ctypes.byref(scene))


def mppi_step_resident(h, x0):
    x = np.ascontiguousarray(np.asarray(x0, dtype=np.float64))
    return load().mppi_step_resident(h, x.ctypes.data_as(_dp))


def mppi_sync(h):
    return load().mppi_sync(h)


def mppi_get_controls(h, out: np.ndarray):
    return load().mppi_get_controls(h, out.ctypes.data_as(_dp), out.size)


def mppi_set_controls(h, U: np.ndarray):
    U = np.ascontiguousarray(U, dtype=np.float64)
    return load().mppi_set_controls(h, U.ctypes.data_as(_dp), U.size)


def mppi_shift(h, steps: int):
    return load().mppi_shift(h, int(steps))


def mppi_step_static(cfg: Config, x0, scene: Scene, U_dev, n_iter, stats_dev=None,
                     hip_stream=None):
    """Allocation-free iteration; U_dev and stats_dev are device addresses
    (int) owned by the caller."""
    x = np.ascontiguousarray(np.asarray(x0, dtype=np.float64))
    return load().mppi_step_static(ctypes.byref(cfg), x.ctypes.data_as(_dp), ctypes.byref(scene),
                                   U_dev, int(n_iter), stats_dev, hip_stream)


def mppi_debug_philox(seed, n_iter, k0, nk, j0, nj):
    out = np.zeros((nk, nj, 4), dtype=np.uint32)
    st = load().mppi_debug_philox(int(seed), int(n_iter), int(k0), int(nk), int(j0), int(nj),
                                  out.ctypes.data_as(_u32p), out.size)
    check(st)
    return out


def mppi_step_batch(hs, x0s, scenes):
    """hs: list of handles; x0s: [n][4]; scenes: list of Scene or None."""
    n = len(hs)
    arr = (_vp * n)(*[h.value if isinstance(h, _vp) else h for h in hs])
    x = np.ascontiguousarray(np.asarray(x0s, dtype=np.float64).reshape(n, 4))
    sc = None
    if scenes is not None:
        sc = (Scene * n)(*scenes)
    return load().mppi_step_batch(arr, x.ctypes.data_as(_dp), sc, n)


def step_batch(planners, x0s, scene_arrays=None):
    """One batched iteration of several Planners (same stream).  scene_arrays:
    list of (waypoints, circles) or None for the resident scenes."""
    keep = []
    scenes = None
    if scene_arrays is not None:
        scenes = []
        for wp, ci in scene_arrays:
            s, k = make_scene(wp, ci)
            scenes.append(s)
            keep.append(k)
    check(mppi_step_batch([p.h for p in planners], x0s, scenes))
    del keep


class Planner:
    """One planning instance (owns an mppi_t handle)."""

    def __init__(self, params, max_waypoints=2048, max_circles=1024, lanes=0, hip_stream=None):
        """hip_stream: a hipStream_t (int) to enqueue on, or None for a new one."""
        self.cfg = config_from_params(params, max_waypoints, max_circles)
        self.K, self.T = self.cfg.K, self.cfg.T
        st, h = mppi_create(self.cfg, hip_stream)
        check(st)
        self.h = h
        if lanes:
            self.set_lanes(lanes)

    def close(self):
        if getattr(self, "h", None):
            load().mppi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_culling(self, on):
        check(load().mppi_set_culling(self.h, 1 if on else 0))

    def set_lanes(self, lanes):
        check(load().mppi_set_lanes_per_sample(self.h, int(lanes)))

    def set_staging(self, mode):
        """-1: tuning table, 0: no LDS copy of the perturbations, 1: when it fits."""
        check(load().mppi_set_staging(self.h, int(mode)))

    def set_occupancy(self, mode):
        """-1: tuning table, 0: default kernel, 1: the five-waves-per-SIMD kernel."""
        check(load().mppi_set_occupancy(self.h, int(mode)))

    def step(self, x0, waypoints, circles):
        scene, keep = make_scene(waypoints, circles)
        check(mppi_step(self.h, x0, scene))
        del keep

    def set_scene(self, x0, waypoints, circles):
        scene, keep = make_scene(waypoints, circles)
        check(mppi_set_scene(self.h, x0, scene))
        del keep

    def step_resident(self, x0):
        check(mppi_step_resident(self.h, x0))

    def sync(self):
        check(mppi_sync(self.h))

    def controls(self):
        out = np.zeros((self.T, 2))
        check(mppi_get_controls(self.h, out))
        return out

    def set_controls(self, U):
        check(mppi_set_controls(self.h, np.asarray(U, dtype=np.float64).reshape(self.T, 2)))

    def shift(self, steps=1):
        check(mppi_shift(self.h, steps))

    def costs(self):
        out = np.zeros(self.K, dtype=np.float32)
        check(load().mppi_get_costs(self.h, out.ctypes.data_as(_fp), out.size))
        return out

    def weights(self):
        out = np.zeros(self.K)
        check(load().mppi_get_weights(self.h, out.ctypes.data_as(_dp), out.size))
        return out

    def trajectory(self):
        """Optimal trajectory after the last step: (states [T+1][4], applied
        controls [T][2])."""
        xs = np.zeros((self.T + 1, 5 if self.cfg.model else 4))
        us = np.zeros((self.T, 2))
        check(load().mppi_get_trajectory(self.h, xs.ctypes.data_as(_dp), xs.size,
                                         us.ctypes.data_as(_dp), us.size))
        return xs, us

    def stage_costs(self):
        """Per-step stage costs [T][K] of the last step (per-step weights)."""
        out = np.zeros((self.T, self.K), dtype=np.float32)
        check(load().mppi_get_stage_costs(self.h, out.ctypes.data_as(_fp), out.size))
        return out

    def set_steering(self, delta0):
        """Initial steering angle of the 5-state model for the next steps."""
        check(load().mppi_set_steering(self.h, float(delta0)))

    def noise(self):
        out = np.zeros((self.T, self.K, 2), dtype=np.float32)
        check(load().mppi_get_noise(self.h, out.ctypes.data_as(_fp), out.size))
        return out

    def stats(self):
        s = IterStats()
        check(load().mppi_get_iter_stats(self.h, ctypes.byref(s)))
        return dict(s_min=s.s_min, log_z=s.log_z, ess=s.ess, n_iter=s.n_iter, status=s.status,
                    lanes=s.lanes_per_sample)

    def get_state(self):
        U = np.zeros((self.T, 2))
        n = ctypes.c_uint64()
        seed = ctypes.c_uint64()
        check(load().mppi_get_state(self.h, U.ctypes.data_as(_dp), U.size, ctypes.byref(n),
                                    ctypes.byref(seed)))
        return U, n.value, seed.value

    def set_state(self, U, n_iter):
        U = np.ascontiguousarray(np.asarray(U, dtype=np.float64).reshape(self.T, 2))
        check(load().mppi_set_state(self.h, U.ctypes.data_as(_dp), U.size, int(n_iter)))

    def stream(self):
        s = _vp()
        check(load().mppi_get_stream(self.h, ctypes.byref(s)))
        return s.value

    def set_profiling(self, on):
        check(load().mppi_set_profiling(self.h, 1 if on else 0))

    def profile(self):
        p = Profile()
        check(load().mppi_get_profile(self.h, ctypes.byref(p)))
        return dict(iter_ms=p.iter_ms, iter_launches=p.iter_launches, aux_ms=p.aux_ms,
                    aux_launches=p.aux_launches, rollout_ms=p.rollout_ms,
                    rollout_launches=p.rollout_launches)


class Server:
    """Continuous-batching replanning server (mppi_server_* of the C ABI)."""

    def __init__(self, hbm_budget_bytes=2 << 30, n_streams=3, max_batch=256, queue_cap=1 << 20,
                 plain=False, deadline_ms=50.0):
        c = ServerConfig(int(hbm_budget_bytes), int(n_streams), int(max_batch), int(queue_cap),
                         1 if plain else 0, float(deadline_ms))
        h = _vp()
        check(load().mppi_server_create(ctypes.byref(c), ctypes.byref(h)))
        self.h = h
        self.T = {}

    def close(self):
        if getattr(self, "h", None):
            load().mppi_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def add_vehicle(self, params, max_waypoints=2048, max_circles=1024):
        cfg = config_from_params(params, max_waypoints, max_circles)
        vid = _i32()
        check(load().mppi_server_add_vehicle(self.h, ctypes.byref(cfg), ctypes.byref(vid)))
        self.T[vid.value] = cfg.T
        return vid.value

    def submit(self, vid, x0, waypoints, circles, t_arrival_ns=0, keep=True):
        scene, keepalive = make_scene(waypoints, circles)
        x = np.ascontiguousarray(np.asarray(x0, dtype=np.float64))
        t = ctypes.c_uint64()
        check(load().mppi_server_submit(self.h, int(vid), x.ctypes.data_as(_dp),
                                        ctypes.byref(scene), int(t_arrival_ns),
                                        ctypes.byref(t) if keep else None))
        del keepalive
        return t.value

    def poll(self, ticket, vid):
        """Returns (controls [T][2], t_done_ns) or None while not ready."""
        U = np.zeros((self.T[vid], 2))
        td = ctypes.c_uint64()
        st = load().mppi_server_poll(self.h, int(ticket), U.ctypes.data_as(_dp), U.size,
                                     ctypes.byref(td))
        if st == E_NOT_READY:
            return None
        check(st)
        return U, td.value

    def wait(self, ticket, vid):
        while True:
            r = self.poll(ticket, vid)
            if r is not None:
                return r
            check(load().mppi_server_wait_idle(self.h))

    def wait_idle(self):
        check(load().mppi_server_wait_idle(self.h))

    def stats(self):
        s = ServerStats()
        check(load().mppi_server_get_stats(self.h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def reset_stats(self):
        check(load().mppi_server_reset_stats(self.h))

    def vehicle_state(self, vid):
        U = np.zeros((self.T[vid], 2))
        n = ctypes.c_uint64()
        r = ctypes.c_uint64()
        check(load().mppi_server_get_vehicle_state(self.h, int(vid), U.ctypes.data_as(_dp), U.size,
                                                   ctypes.byref(n), ctypes.byref(r)))
        return U, n.value, r.value

    def set_vehicle_state(self, vid, U, n_iter, requests):
        U = np.ascontiguousarray(np.asarray(U, dtype=np.float64))
        check(load().mppi_server_set_vehicle_state(self.h, int(vid), U.ctypes.data_as(_dp), U.size,
                                                   int(n_iter), int(requests)))

    def replay(self, vids, x0s, scene_idx, scene_pool, arrival_ns):
        """Open-loop load.  scene_pool: list of (waypoints, circles).
        Returns latency_ms [n] (NaN for refused requests)."""
        n = len(vids)
        vid = np.ascontiguousarray(np.asarray(vids, dtype=np.int32))
        x = np.ascontiguousarray(np.asarray(x0s, dtype=np.float64).reshape(n, 4))
        si = np.ascontiguousarray(np.asarray(scene_idx, dtype=np.int32))
        arr = np.ascontiguousarray(np.asarray(arrival_ns, dtype=np.uint64))
        keep = []
        scs = (Scene * len(scene_pool))()
        for i, (wp, ci) in enumerate(scene_pool):
            s_, k = make_scene(wp, ci)
            scs[i] = s_
            keep.append(k)
        plan = ReplayPlan(n, vid.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          x.ctypes.data_as(_dp), si.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          scs, len(scene_pool), arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
        lat = np.zeros(n)
        check(load().mppi_server_replay(self.h, ctypes.byref(plan), lat.ctypes.data_as(_dp)))
        del keep
        return lat
