"""Closed-loop driving of the paper's scenarios (shared by the oracle and
GPU tests): every planner period the vehicle takes the first step of the
optimal trajectory, the obstacles move on, and the nominal controls are
shifted by one step for the next replan (Alg. 1's warm start)."""
import numpy as np

STEER_10_DEG = np.deg2rad(10.0)


def clearance(p, x, circ):
    """d_obj of Sec. IV-C for state x (ego circles vs obstacle circles)."""
    if len(circ) == 0:
        return np.inf
    d = np.inf
    for o in p["ego_off"]:
        ex, ey = x[0] + o * np.cos(x[2]), x[1] + o * np.sin(x[2])
        for c in circ:
            d = min(d, np.hypot(ex - c[0], ey - c[1]) - c[2] - p["ego_r"])
    return d


def moved(circles, t):
    c = np.array(circles, dtype=np.float64).reshape(-1, 5).copy()
    c[:, 0] += c[:, 3] * t
    c[:, 1] += c[:, 4] * t
    return c


def drive(sc, plan, ticks):
    """plan(k, x, circles) -> (states [T+1][4], applied controls [T][2]) of
    the optimal trajectory after replanning at tick k.  Returns the driven
    states [ticks][4], first controls [ticks][2] and clearances [ticks]."""
    p = sc["params"]
    dt = p["dt"]
    x = np.array(sc["x0"], dtype=np.float64)
    if p.get("model", 0):
        x = np.append(x, p.get("steer0", 0.0))   # the steering angle is state
    xs, us, ds = [], [], []
    for k in range(ticks):
        traj, ctl = plan(k, x, moved(sc["circles"], k * dt))
        x = np.array(traj[1], dtype=np.float64)
        xs.append(x)
        us.append(np.array(ctl[0]))
        ds.append(clearance(p, x, moved(sc["circles"], (k + 1) * dt)))
    return np.array(xs), np.array(us), np.array(ds)


def check_outcomes(name, p, xs, us, ds, lead_speed=4.0):
    """The paper's observations: the speed never exceeds the target speed,
    the steering angle stays within 10 degrees, no object is hit (for the
    avoidance: the car itself, inside the 0.7 m margin its circles carry);
    the merge ends on the lane, the avoidance passes the object and
    returns, the follower settles at the lead's speed behind it."""
    steer = xs[:, 4] if p.get("model", 0) else us[:, 1]
    assert np.all(xs[:, 3] <= p["v_max"] + 1e-9), xs[:, 3].max()
    assert np.all(np.abs(steer) <= STEER_10_DEG), np.abs(steer).max()
    assert np.all(ds > (-0.7 if name == "paper_avoid" else 0.0)), ds.min()
    n = len(xs)
    if name == "paper_merge":
        assert np.all(np.abs(xs[n // 2:, 1]) < 0.3), xs[:, 1]
    elif name == "paper_avoid":
        assert xs[-1, 0] > 60.0 and abs(xs[-1, 1]) < 0.5, xs[-1]
    elif name == "paper_follow":
        assert abs(xs[-1, 3] - lead_speed) < 0.5 and ds.min() > 5.0, (xs[-1], ds.min())
