"""Seeded synthetic driving scenes and planner parameters.

This module only builds *inputs*: reference waypoints, obstacle circles, the
initial state and the planner parameters.  It holds none of the planner's
arithmetic and is shared by the tests, the benchmark and the smoke check so
that the HIP path and the CPU oracle always see the same inputs.

The paper validates on a real track with virtual objects and publishes no
dataset, so these scenes stand in for its scenarios.  Sizes and value
distributions follow the workload table of the planner:

* ``c0`` -- straight lane y = 0, one static obstacle of 3 circles at x = 30.
* ``c1`` -- sine lane y = 5 sin(2 pi x / 150), 20 obstacles x 3 circles, half
  of them moving along the lane.
* ``c2_instance(i)`` -- one of 256 uneven instances (K, T, circle count drawn
  per instance) on the sine lane.
* ``c3_vehicle(v)`` / ``c3_request(v, i)`` -- served vehicles and requests.
* ``c4`` -- 5 clothoid segments (300 m), 512 circles of which 128 move.
* ``paper_table1`` -- the paper's own workload shape (Table I: M = 2560,
  T = 16, dt = 0.25 s, lambda = 150) on the sine-lane scene.

Arrays are float64: waypoints [n][4] = (x, y, yaw, v_ref), circles [n][5] =
(x, y, r, vx, vy) at request time.  Everything is in world coordinates.
"""
from __future__ import annotations

import math

import numpy as np

# Planner defaults shared by every scene (the values of the plain single
# iteration; the larger scenes inherit them).
BASE = dict(
    dt=0.1, wheelbase=2.7, lam=1.0, gamma=1.0,
    sigma=(1.0, 0.3),                  # std dev of (accel m/s^2, steer rad)
    u_min=(-2.5, -0.5), u_max=(1.1, 0.5),
    v_max=10.0,
    w_track=1.0, w_speed=0.5, w_effort=0.1, w_coll=1.0e4,
    d_safe_c=0.0, d_safe_0=0.5,
    ego_r=1.0, ego_off=(0.0, 1.35, 2.7),
    seed=0,
)

SINE_AMP, SINE_LEN = 5.0, 150.0


def params(**over):
    p = dict(BASE)
    p.update(over)
    return p


def straight_lane(x_lo, x_hi, v_ref):
    xs = np.arange(x_lo, x_hi + 0.5, 1.0)
    wp = np.zeros((xs.size, 4))
    wp[:, 0] = xs
    wp[:, 3] = v_ref
    return wp


def _sine_y(x):
    return SINE_AMP * np.sin(2.0 * np.pi * x / SINE_LEN)


def _sine_slope(x):
    return SINE_AMP * 2.0 * np.pi / SINE_LEN * np.cos(2.0 * np.pi * x / SINE_LEN)


def sine_lane(x_lo=-20.0, x_hi=200.0, v_ref=15.0):
    xs = np.arange(x_lo, x_hi + 0.5, 1.0)
    wp = np.zeros((xs.size, 4))
    wp[:, 0] = xs
    wp[:, 1] = _sine_y(xs)
    wp[:, 2] = np.arctan(_sine_slope(xs))
    wp[:, 3] = v_ref
    return wp


def _sine_frame(x):
    """Point, unit tangent and unit left normal of the sine lane at abscissa x."""
    y = _sine_y(x)
    s = _sine_slope(x)
    n = math.hypot(1.0, s)
    tx, ty = 1.0 / n, s / n
    return (x, y), (tx, ty), (-ty, tx)


def sine_obstacles(rng, n_obst, x_lo=10.0, x_hi=150.0, n_dynamic=None):
    """Obstacles of 3 circles each: radius r ~ U(0.8, 1.5) per obstacle, centre
    x ~ U[x_lo, x_hi], lateral offset N(0, 2) along the lane normal, circles at
    {-r, 0, +r} along the lane tangent; the last ``n_dynamic`` obstacles move
    along the tangent at U(0, 8) m/s."""
    if n_dynamic is None:
        n_dynamic = n_obst // 2
    out = []
    for i in range(n_obst):
        r = rng.uniform(0.8, 1.5)
        cx = rng.uniform(x_lo, x_hi)
        lat = rng.normal(0.0, 2.0)
        (px, py), (tx, ty), (nx, ny) = _sine_frame(cx)
        ox, oy = px + lat * nx, py + lat * ny
        speed = rng.uniform(0.0, 8.0) if i >= n_obst - n_dynamic else 0.0
        for off in (-r, 0.0, r):
            out.append((ox + off * tx, oy + off * ty, r, speed * tx, speed * ty))
    return np.array(out, dtype=np.float64).reshape(-1, 5)


def sine_circles(rng, n_c, x_lo=10.0, x_hi=150.0):
    """Independent circles placed as the obstacles above; floor(n_c/2) move."""
    out = []
    n_dyn = n_c // 2
    for i in range(n_c):
        r = rng.uniform(0.8, 1.5)
        cx = rng.uniform(x_lo, x_hi)
        lat = rng.normal(0.0, 2.0)
        (px, py), (tx, ty), (nx, ny) = _sine_frame(cx)
        speed = rng.uniform(0.0, 8.0) if i >= n_c - n_dyn else 0.0
        out.append((px + lat * nx, py + lat * ny, r, speed * tx, speed * ty))
    return np.array(out, dtype=np.float64).reshape(-1, 5)


def _sine_x0(x=0.0, v=12.0):
    return np.array([x, float(_sine_y(x)), math.atan(float(_sine_slope(x))), v])


def c0():
    """Plain single iteration, oracle-sized: K=1024, T=50, dt=0.1."""
    p = params(K=1024, T=50, dt=0.1, v_max=10.0, seed=0)
    wp = straight_lane(-20.0, 120.0, 10.0)
    circ = np.array([[30.0, y, 1.0, 0.0, 0.0] for y in (-1.0, 0.0, 1.0)])
    x0 = np.array([0.0, 0.0, 0.0, 8.0])
    return dict(name="c0", params=p, x0=x0, waypoints=wp, circles=circ, iterations=1)


def c1(K=8192, T=100):
    """Single instance, sine lane, 20 obstacles x 3 circles (half moving),
    10 warm-started iterations."""
    rng = np.random.Generator(np.random.PCG64(1))
    p = params(K=K, T=T, dt=0.05, v_max=15.0, seed=1)
    wp = sine_lane(v_ref=15.0)
    circ = sine_obstacles(rng, 20)
    return dict(name="c1", params=p, x0=_sine_x0(), waypoints=wp, circles=circ, iterations=10)


C2_KS = (1024, 2048, 4096, 8192, 16384)


def c2_shapes(n=256):
    """(K, T, n_circles) per batched instance, drawn from PCG64(2)."""
    rng = np.random.Generator(np.random.PCG64(2))
    Ks = rng.choice(C2_KS, size=n)
    Ts = rng.integers(30, 151, size=n)
    Ns = rng.integers(0, 65, size=n)
    return [(int(a), int(b), int(c)) for a, b, c in zip(Ks, Ts, Ns)]


def c2_instance(i, shape=None):
    K, T, n_c = shape if shape is not None else c2_shapes()[i]
    rng = np.random.Generator(np.random.PCG64(2000 + i))
    p = params(K=K, T=T, dt=0.05, v_max=15.0, seed=2000 + i)
    wp = sine_lane(v_ref=15.0)
    circ = sine_circles(rng, n_c)
    return dict(name="c2[%d]" % i, params=p, x0=_sine_x0(), waypoints=wp, circles=circ,
                iterations=1)


def c2(n=256):
    shapes = c2_shapes(n)
    return [c2_instance(i, shapes[i]) for i in range(n)]


def c3_vehicle(v):
    """Per-vehicle fixed shape (K, T), seed and start abscissa."""
    rng = np.random.Generator(np.random.PCG64(3000 + v))
    K = int(rng.choice((2048, 4096, 8192)))
    T = int(rng.choice((50, 100)))
    x_start = float(rng.uniform(-10.0, 40.0))
    p = params(K=K, T=T, dt=0.05, v_max=15.0, seed=3000 + v)
    return dict(vehicle=v, params=p, x_start=x_start)


def c3_request(v, i, veh=None):
    """Request i of vehicle v: the vehicle advances open-loop along the lane
    at 15 m/s (one 50 ms period per request); 0-48 circles drawn per request."""
    veh = veh or c3_vehicle(v)
    rng = np.random.Generator(np.random.PCG64([3000 + v, i]))
    x = veh["x_start"] + 15.0 * 0.05 * i
    n_c = int(rng.integers(0, 49))
    circ = sine_circles(rng, n_c, x_lo=x + 5.0, x_hi=x + 120.0)
    wp = sine_lane(x_lo=math.floor(x) - 20.0, x_hi=math.floor(x) + 200.0, v_ref=15.0)
    return dict(name="c3[%d,%d]" % (v, i), params=veh["params"], x0=_sine_x0(x, 15.0),
                waypoints=wp, circles=circ)


def _clothoid_path(rng, n_seg=5, seg_len=60.0, step=0.01, spacing=1.0):
    """Concatenated clothoid segments: curvature linear in arc length on each
    segment between knots drawn U[-0.02, 0.02]; integrated in float64 with a
    midpoint rule at ``step`` metres, sampled every ``spacing`` metres."""
    knots = rng.uniform(-0.02, 0.02, size=n_seg + 1)
    total = n_seg * seg_len
    n = int(round(total / step))
    x = y = th = 0.0
    every = int(round(spacing / step))
    pts = [(0.0, 0.0, 0.0)]
    for i in range(n):
        s_mid = (i + 0.5) * step
        seg = min(int(s_mid // seg_len), n_seg - 1)
        f = (s_mid - seg * seg_len) / seg_len
        kap = knots[seg] * (1.0 - f) + knots[seg + 1] * f
        th_mid = th + 0.5 * step * kap
        x += step * math.cos(th_mid)
        y += step * math.sin(th_mid)
        th += step * kap
        if (i + 1) % every == 0:
            pts.append((x, y, th))
    return np.array(pts)


def c4(K=262144, T=200):
    """Stress single instance: 5 clothoids, 512 circles (128 moving)."""
    rng = np.random.Generator(np.random.PCG64(4))
    path = _clothoid_path(rng)
    wp = np.zeros((path.shape[0], 4))
    wp[:, :3] = path
    wp[:, 3] = 15.0
    circ = []
    n_c, n_dyn = 512, 128
    for i in range(n_c):
        s = rng.uniform(25.0, 290.0)
        j = int(round(s))
        px, py, th = path[j]
        tx, ty = math.cos(th), math.sin(th)
        lat = rng.normal(0.0, 2.0)
        r = rng.uniform(0.8, 1.5)
        speed = rng.uniform(0.0, 8.0) if i >= n_c - n_dyn else 0.0
        circ.append((px - lat * ty, py + lat * tx, r, speed * tx, speed * ty))
    x0 = np.array([path[10, 0], path[10, 1], path[10, 2], 12.0])
    p = params(K=K, T=T, dt=0.05, v_max=15.0, seed=4)
    return dict(name="c4", params=p, x0=x0, waypoints=wp, circles=np.array(circ),
                iterations=1)


def paper_table1():
    """The paper's own workload shape (Table I) on the sine-lane scene:
    M = 2560 samples, T = 16, dt = 0.25 s, lambda = 150, sigma_a = 0.85,
    steering noise 0.05, a in [-2.5, 1.1], v_G = 30 km/h."""
    rng = np.random.Generator(np.random.PCG64(1))
    p = params(K=2560, T=16, dt=0.25, lam=150.0, sigma=(0.85, 0.05), v_max=30.0 / 3.6,
               seed=5)
    wp = sine_lane(v_ref=30.0 / 3.6)
    circ = sine_obstacles(rng, 20)
    return dict(name="paper_table1", params=p, x0=_sine_x0(v=8.0), waypoints=wp, circles=circ,
                iterations=1)


# ---- the paper's three scenarios (Sec. IV-A) with its full Sec. IV-C cost
# and Table I parameters, on synthetic straight roads: lane merge, object
# avoidance (collision-only obstacle cost, a 0.7 m margin around the object)
# and vehicle following (velocity-dependent safe distance).

V_G = 30.0 / 3.6                       # target speed of Table I


def paper_params(**over):
    """Table I and the Sec. IV-C weights 15 / 7 / 120 / 5 / 25 (the paper's
    total has no input cost term), Savitzky-Golay smoothing on."""
    p = params(K=2560, T=16, dt=0.25, lam=150.0, sigma=(0.85, 0.05), v_max=V_G,
               u_min=(-2.5, -0.5), u_max=(1.1, 0.5),
               w_track=15.0, w_target=7.0, w_yaw=120.0, w_speed=5.0, w_coll=25.0,
               w_effort=0.0, d_safe_c=1.36, d_safe_0=11.0, smoothing=1, seed=11)
    p.update(over)
    return p


def car_circles(x, y, r=1.0, vx=0.0, vy=0.0, margin=0.0):
    """A car-sized object (4.5 m x 1.8 m) as three circles along x."""
    return np.array([[x + dx, y, r + margin, vx, vy] for dx in (-1.5, 0.0, 1.5)])


def paper_merge():
    """Lane merge: the path is the lane y = 0; the vehicle starts on the
    parallel lane 3.5 m to the left at 5 m/s."""
    p = paper_params(seed=21)
    wp = straight_lane(-10.0, 200.0, V_G)
    return dict(name="paper_merge", params=p, x0=np.array([0.0, 3.5, 0.0, 5.0]), waypoints=wp,
                circles=np.zeros((0, 5)), iterations=1)


def paper_avoid():
    """Object avoidance: a stopped car on the path 40 m ahead; obstacle
    cost only on contact (collision-only mode), the object inflated by the
    prescribed 0.7 m margin."""
    p = paper_params(seed=22, collision_only=1)
    wp = straight_lane(-10.0, 200.0, V_G)
    return dict(name="paper_avoid", params=p, x0=np.array([0.0, 0.0, 0.0, V_G]), waypoints=wp,
                circles=car_circles(40.0, 0.0, margin=0.7), iterations=1)


def paper_follow(lead_speed=4.0):
    """Vehicle following: a car 30 m ahead on the path at lead_speed; the
    safe distance 1.36 v + 11 m of Table I keeps the follower behind it."""
    p = paper_params(seed=23)
    wp = straight_lane(-10.0, 400.0, V_G)
    return dict(name="paper_follow", params=p, x0=np.array([0.0, 0.0, 0.0, V_G]), waypoints=wp,
                circles=car_circles(30.0, 0.0, vx=lead_speed), iterations=1)


def paper_model5(sc, steer0=0.0):
    """A copy of scene sc planned with the 5-state model of eq. (5): the
    steering angle is state (initially steer0) and the second control is the
    steering rate, with Table I's noise 0.05 rad/s and bound 0.11 rad/s."""
    out = dict(sc)
    p = dict(sc["params"])
    p.update(model=1, steer0=steer0, u_min=(p["u_min"][0], -0.11), u_max=(p["u_max"][0], 0.11),
             sigma=(p["sigma"][0], 0.05))
    out["params"] = p
    out["name"] = sc["name"] + "_m5"
    return out


def tiny(K=8, T=4, n_c=3, seed=7):
    """A small random scene for exhaustive checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = params(K=K, T=T, dt=0.1, v_max=15.0, seed=seed)
    wp = sine_lane(-5.0, 30.0, 15.0)
    circ = sine_circles(rng, n_c, 3.0, 20.0)
    return dict(name="tiny", params=p, x0=_sine_x0(v=10.0), waypoints=wp, circles=circ,
                iterations=1)


def speed_profile(sc, seed=0, n_dup=12):
    """A copy of scene sc whose waypoints carry a varying reference speed (a
    smooth profile along x) and n_dup exactly repeated waypoints: the repeat
    follows the original at the next index, with a reference speed 10 m/s
    higher, so the closest index must be the lower of the two.  Repeats are
    forced at indices that end a chunk of 8 consecutive waypoints."""
    rng = np.random.Generator(np.random.PCG64(seed))
    wp = np.array(sc["waypoints"], dtype=np.float64)
    wp[:, 3] = 12.0 + np.sin(wp[:, 0] / 15.0)
    pick = set(rng.choice(len(wp), size=min(n_dup, len(wp)), replace=False).tolist())
    rows = []
    for j in range(len(wp)):
        rows.append(wp[j])
        if j in pick or len(rows) % 8 == 0:
            dup = wp[j].copy()
            dup[3] += 10.0
            rows.append(dup)
    out = dict(sc)
    out["waypoints"] = np.array(rows)
    out["name"] = sc["name"] + "_speed"
    return out


def by_name(name):
    return {"c0": c0, "c1": c1, "c4": c4, "paper_table1": paper_table1, "tiny": tiny,
            "paper_merge": paper_merge, "paper_avoid": paper_avoid,
            "paper_follow": paper_follow}[name]()
