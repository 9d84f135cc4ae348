"""FP64 CPU oracle for one MPPI iteration -- Python wrapper.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg use this module; the product package never imports it.  The
arithmetic lives in ``mppi_oracle.c`` (plain C, binary64) next to this file,
which shares no code with the HIP library.

Every entry point takes plain parameters: a ``params`` mapping (the keys
produced by the seeded scene generator: K, T, dt, wheelbase, lam, gamma,
sigma, u_min, u_max, v_max, w_track, w_speed, w_effort, w_coll, d_safe_c,
d_safe_0, ego_r, ego_off, seed) and float64 numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mppi_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

OK, E_INVALID, E_NONFINITE = 0, -1, -4


class OrcCfg(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_int32), ("T", ctypes.c_int32),
        ("dt", ctypes.c_double), ("wheelbase", ctypes.c_double),
        ("lam", ctypes.c_double), ("gamma", ctypes.c_double),
        ("sigma_a", ctypes.c_double), ("sigma_d", ctypes.c_double),
        ("a_min", ctypes.c_double), ("a_max", ctypes.c_double),
        ("d_min", ctypes.c_double), ("d_max", ctypes.c_double),
        ("v_max", ctypes.c_double),
        ("w_track", ctypes.c_double), ("w_speed", ctypes.c_double),
        ("w_effort", ctypes.c_double), ("w_coll", ctypes.c_double),
        ("d_safe_c", ctypes.c_double), ("d_safe_0", ctypes.c_double),
        ("n_ego", ctypes.c_int32), ("ego_r", ctypes.c_double),
        ("ego_off", ctypes.c_double * 4),
        ("seed", ctypes.c_uint64),
        ("smoothing", ctypes.c_int32),
        ("w_target", ctypes.c_double), ("w_yaw", ctypes.c_double),
        ("collision_only", ctypes.c_int32),
        ("model", ctypes.c_int32), ("steer0", ctypes.c_double),
        ("per_step", ctypes.c_int32),
    ]


def build(force: bool = False) -> str:
    """Compile ``mppi_oracle.c`` into ``liboracle.so`` (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            cp = ctypes.POINTER(OrcCfg)
            u32p = ctypes.POINTER(ctypes.c_uint32)
            L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
            L.orc_max_threads.restype = ctypes.c_int
            L.orc_set_threads.argtypes = [ctypes.c_int]
            L.orc_philox_batch.argtypes = [u32p, ctypes.c_int64, u32p, u32p]
            L.orc_uniform.argtypes = [ctypes.c_uint32]
            L.orc_uniform.restype = ctypes.c_double
            L.orc_box_muller.argtypes = [ctypes.c_double, ctypes.c_double, dp]
            L.orc_noise.argtypes = [cp, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, dp]
            L.orc_apply_limits.argtypes = [cp, dp, dp, ctypes.c_double, dp]
            L.orc_dynamics.argtypes = [cp, dp, dp, dp]
            L.orc_stage_cost.argtypes = [cp, dp, ctypes.c_int, dp, ctypes.c_int, dp, dp, dp,
                                         ctypes.c_int, dp, dp]
            L.orc_stage_cost.restype = ctypes.c_double
            L.orc_rollout.argtypes = [cp, dp, dp, ctypes.c_int, dp, ctypes.c_int, dp,
                                      ctypes.c_uint64, dp, dp, dp, dp]
            L.orc_update_per_step.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, dp,
                                              ctypes.c_double, dp, dp, dp, dp]
            L.orc_rollout_samples.argtypes = [cp, dp, dp, ctypes.c_int, dp, ctypes.c_int, dp,
                                              ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.c_int, dp, dp, dp]
            L.orc_simulate.argtypes = [cp, dp, dp, ctypes.c_int, dp, ctypes.c_int, dp, dp,
                                       dp, dp, dp]
            L.orc_weights.argtypes = [dp, ctypes.c_int, ctypes.c_double, dp, dp, dp]
            L.orc_update.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, dp]
            L.orc_iteration.argtypes = [cp, dp, dp, ctypes.c_int, dp, ctypes.c_int, dp,
                                        ctypes.c_uint64, dp, dp, dp, dp, dp]
            L.orc_sg_smooth.argtypes = [dp, ctypes.c_int, dp]
            L.orc_optimal_trajectory.argtypes = [cp, dp, dp, dp, dp]
            _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def make_cfg(p) -> OrcCfg:
    c = OrcCfg()
    c.K, c.T = int(p["K"]), int(p["T"])
    c.dt, c.wheelbase = float(p["dt"]), float(p["wheelbase"])
    c.lam, c.gamma = float(p["lam"]), float(p["gamma"])
    c.sigma_a, c.sigma_d = float(p["sigma"][0]), float(p["sigma"][1])
    c.a_min, c.d_min = float(p["u_min"][0]), float(p["u_min"][1])
    c.a_max, c.d_max = float(p["u_max"][0]), float(p["u_max"][1])
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
    c.smoothing = int(p.get("smoothing", 0))
    c.w_target = float(p.get("w_target", 0.0))
    c.w_yaw = float(p.get("w_yaw", 0.0))
    c.collision_only = int(p.get("collision_only", 0))
    c.model = int(p.get("model", 0))
    c.steer0 = float(p.get("steer0", 0.0))
    c.per_step = int(p.get("per_step", 0))
    return c


def philox(ctr, key):
    """Philox4x32-10 of one 128-bit counter under a 64-bit key -> 4 uint32."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def philox_batch(ctrs, key):
    """Philox of many counters: ctrs uint32 [n][4] -> uint32 [n][4]."""
    c = np.ascontiguousarray(np.asarray(ctrs, dtype=np.uint32).reshape(-1, 4))
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    out = np.zeros_like(c)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib().orc_philox_batch(c.ctypes.data_as(u32p), c.shape[0], k, out.ctypes.data_as(u32p))
    return out


def max_threads() -> int:
    return int(lib().orc_max_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops over samples."""
    lib().orc_set_threads(int(n))


def uniform(r: int) -> float:
    return lib().orc_uniform(int(r) & 0xFFFFFFFF)


def box_muller(u1: float, u2: float):
    z = np.zeros(2)
    lib().orc_box_muller(float(u1), float(u2), _dp(z))
    return z


def noise(p, n_iter: int, k: int, t: int):
    """Raw (unclamped) perturbation of step t of sample k at iteration n_iter."""
    c = make_cfg(p)
    e = np.zeros(2)
    lib().orc_noise(ctypes.byref(c), int(n_iter), int(k), int(t), _dp(e))
    return e


def apply_limits(p, U_t, eps, v):
    c = make_cfg(p)
    U_t, eps = _f64(U_t), _f64(eps)
    out = np.zeros(2)
    lib().orc_apply_limits(ctypes.byref(c), _dp(U_t), _dp(eps), float(v), _dp(out))
    return out


def dynamics(p, x, u):
    """One Euler step: x is (x, y, theta, v) or, for the 5-state model,
    (x, y, theta, v, delta); returns the same length."""
    c = make_cfg(p)
    x, u = _f64(x), _f64(u)
    x5 = np.zeros(5)
    x5[:x.shape[0]] = x
    out = np.zeros(5)
    lib().orc_dynamics(ctypes.byref(c), _dp(x5), _dp(u), _dp(out))
    return out[:x.shape[0]]


def stage_cost(p, waypoints, circles, x_new, U_t, eps, t, x_prev=None):
    """Stage cost on the new state reached from x_prev (default: x_new, so
    c_target = 0); returns (cost, (c_dist, c_speed, q_u, c_safe, c_target,
    c_yaw))."""
    c = make_cfg(p)
    wp = _f64(waypoints, (-1, 4))
    ci = _f64(circles, (-1, 5)) if len(circles) else np.zeros((0, 5))
    xn, U_t, eps = _f64(x_new), _f64(U_t), _f64(eps)
    xp = xn if x_prev is None else _f64(x_prev)
    parts = np.zeros(6)
    v = lib().orc_stage_cost(ctypes.byref(c), _dp(wp), wp.shape[0], _dp(ci), ci.shape[0],
                             _dp(xn), _dp(U_t), _dp(eps), int(t), _dp(xp), _dp(parts))
    return v, parts


def simulate(p, x0, waypoints, circles, U, eps=None):
    """Deterministic rollout of one control sequence U (+ optional eps).
    Returns (states [T+1][4], stage costs [T], parts [T][6])."""
    c = make_cfg(p)
    T = c.T
    wp = _f64(waypoints, (-1, 4))
    ci = _f64(circles, (-1, 5)) if len(circles) else np.zeros((0, 5))
    U = _f64(U, (T, 2))
    e = None if eps is None else _f64(eps, (T, 2))
    x0 = _f64(x0)
    states = np.zeros((T + 1, 4 + (1 if c.model else 0)))
    costs = np.zeros(T)
    parts = np.zeros((T, 6))
    rc = lib().orc_simulate(ctypes.byref(c), _dp(x0), _dp(wp), wp.shape[0], _dp(ci),
                            ci.shape[0], _dp(U), _dp(e), _dp(states), _dp(costs), _dp(parts))
    if rc != OK:
        raise ValueError("orc_simulate: status %d" % rc)
    return states, costs, parts


def rollout(p, x0, waypoints, circles, U, n_iter=0, eps_in=None, stage_costs=False):
    """All K rollouts.  Returns (S [K], eps_eff [T][K][2]) and, with
    stage_costs, the per-step costs q [T][K] as a third element."""
    c = make_cfg(p)
    K, T = c.K, c.T
    wp = _f64(waypoints, (-1, 4))
    ci = _f64(circles, (-1, 5)) if len(circles) else np.zeros((0, 5))
    U = _f64(U, (T, 2))
    x0 = _f64(x0)
    ein = None if eps_in is None else _f64(eps_in, (T, K, 2))
    S = np.zeros(K)
    eps = np.zeros((T, K, 2))
    q = np.zeros((T, K)) if stage_costs else None
    rc = lib().orc_rollout(ctypes.byref(c), _dp(x0), _dp(wp), wp.shape[0], _dp(ci), ci.shape[0],
                           _dp(U), int(n_iter), _dp(ein), _dp(S), _dp(eps), _dp(q))
    if rc != OK:
        raise ValueError("orc_rollout: status %d" % rc)
    return (S, eps, q) if stage_costs else (S, eps)


def rollout_samples(p, x0, waypoints, circles, U, ks, n_iter=0, eps_in=None):
    """Rollouts of the sample indices ``ks`` only.  Returns (S [nk], eps [T][nk][2])."""
    c = make_cfg(p)
    T = c.T
    ks = np.ascontiguousarray(np.asarray(ks, dtype=np.int32))
    nk = ks.shape[0]
    wp = _f64(waypoints, (-1, 4))
    ci = _f64(circles, (-1, 5)) if len(circles) else np.zeros((0, 5))
    U = _f64(U, (T, 2))
    x0 = _f64(x0)
    ein = None if eps_in is None else _f64(eps_in, (T, nk, 2))
    S = np.zeros(nk)
    eps = np.zeros((T, nk, 2))
    rc = lib().orc_rollout_samples(ctypes.byref(c), _dp(x0), _dp(wp), wp.shape[0], _dp(ci),
                                   ci.shape[0], _dp(U), int(n_iter),
                                   ks.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), nk,
                                   _dp(ein), _dp(S), _dp(eps))
    if rc != OK:
        raise ValueError("orc_rollout_samples: status %d" % rc)
    return S, eps


def weights(S, lam):
    """Normalised weights, S_min and log Z.  Raises on all-non-finite."""
    S = _f64(S)
    w = np.zeros(S.shape[0])
    smin = ctypes.c_double()
    logz = ctypes.c_double()
    rc = lib().orc_weights(_dp(S), S.shape[0], float(lam), _dp(w), ctypes.byref(smin),
                           ctypes.byref(logz))
    if rc == E_NONFINITE:
        raise FloatingPointError("every sample cost is non-finite")
    if rc != OK:
        raise ValueError("orc_weights: status %d" % rc)
    return w, smin.value, logz.value


def update(U, w, eps):
    """Returns U + sum_k w_k eps[:, k, :] (a new array)."""
    U = _f64(U).copy()
    T = U.shape[0]
    w = _f64(w)
    K = w.shape[0]
    eps = _f64(eps, (T, K, 2))
    lib().orc_update(_dp(U), T, K, _dp(w), _dp(eps))
    return U


def iteration(p, x0, waypoints, circles, U, n_iter=0):
    """One MPPI iteration.  Returns dict(U, S, w, eps, s_min, log_z)."""
    c = make_cfg(p)
    K, T = c.K, c.T
    wp = _f64(waypoints, (-1, 4))
    ci = _f64(circles, (-1, 5)) if len(circles) else np.zeros((0, 5))
    Un = _f64(U, (T, 2)).copy()
    x0 = _f64(x0)
    S = np.zeros(K)
    w = np.zeros(K)
    eps = np.zeros((T, K, 2))
    smin = ctypes.c_double()
    logz = ctypes.c_double()
    rc = lib().orc_iteration(ctypes.byref(c), _dp(x0), _dp(wp), wp.shape[0], _dp(ci),
                             ci.shape[0], _dp(Un), int(n_iter), _dp(S), _dp(w), _dp(eps),
                             ctypes.byref(smin), ctypes.byref(logz))
    if rc == E_NONFINITE:
        raise FloatingPointError("every sample cost is non-finite")
    if rc != OK:
        raise ValueError("orc_iteration: status %d" % rc)
    return dict(U=Un, S=S, w=w, eps=eps, s_min=smin.value, log_z=logz.value)


def sg_smooth(U):
    """Savitzky-Golay smoothing of eq. (sg) with repeated end values: [T][2]."""
    U = _f64(U).reshape(-1, 2)
    out = np.zeros_like(U)
    lib().orc_sg_smooth(_dp(U), U.shape[0], _dp(out))
    return out


def optimal_trajectory(p, x0, Us):
    """Optimal rollout of Alg. 1 from x0 under controls Us (each through the
    noise check with zero noise).  Returns (states [T+1][4], applied [T][2])."""
    c = make_cfg(p)
    Us = _f64(Us, (c.T, 2))
    x0 = _f64(x0)
    states = np.zeros((c.T + 1, 4 + (1 if c.model else 0)))
    applied = np.zeros((c.T, 2))
    lib().orc_optimal_trajectory(ctypes.byref(c), _dp(x0), _dp(Us), _dp(states), _dp(applied))
    return states, applied


def update_per_step(U, q, eps, lam):
    """Per-step update from stage costs q [T][K] and applied perturbations
    eps [T][K][2]: returns (U_new, S_tk [T][K] cost-to-go, w0 [K] weights of
    t = 0).  Raises when some step has no finite cost-to-go."""
    U = _f64(U).copy()
    T = U.shape[0]
    q = _f64(q).reshape(T, -1)
    K = q.shape[1]
    eps = _f64(eps, (T, K, 2))
    S = np.zeros((T, K))
    w0 = np.zeros(K)
    smin = ctypes.c_double()
    logz = ctypes.c_double()
    rc = lib().orc_update_per_step(_dp(U), T, K, _dp(q), _dp(eps), float(lam), _dp(S), _dp(w0),
                                   ctypes.byref(smin), ctypes.byref(logz))
    if rc == E_NONFINITE:
        raise FloatingPointError("a step has no finite cost-to-go")
    if rc != OK:
        raise ValueError("orc_update_per_step: status %d" % rc)
    return U, S, w0
