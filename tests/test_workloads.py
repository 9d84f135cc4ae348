"""The synthetic workloads (no GPU): shapes, sizes and structure of each
input recipe, and that every generator is deterministic."""
import math
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2308_01654_amd import scenes  # noqa: E402

# circles: (x, y, r, vx, vy); waypoints: (x, y, heading, reference speed)


def _moving(c):
    c = np.asarray(c)
    return int(np.sum(np.hypot(c[:, 3], c[:, 4]) > 0))


def test_plain_instance():
    sc = scenes.c0()
    p = sc["params"]
    assert (p["K"], p["T"], p["dt"], p["seed"]) == (1024, 50, 0.1, 0)
    w = np.asarray(sc["waypoints"])
    assert w.shape == (141, 4) and np.all(w[:, 1] == 0.0) and np.all(np.diff(w[:, 0]) == 1.0)
    c = np.asarray(sc["circles"])
    assert c.shape == (3, 5) and np.all(c[:, 0] == 30.0) and list(c[:, 1]) == [-1.0, 0.0, 1.0]
    assert np.all(c[:, 2] == 1.0) and _moving(c) == 0
    assert list(sc["x0"]) == [0.0, 0.0, 0.0, 8.0]


def test_sine_lane_instance():
    sc = scenes.c1()
    p = sc["params"]
    assert (p["K"], p["T"], p["dt"]) == (8192, 100, 0.05)
    w = np.asarray(sc["waypoints"])
    assert w.shape == (221, 4) and w[0, 0] == -20.0 and w[-1, 0] == 200.0
    assert np.allclose(w[:, 1], 5.0 * np.sin(2 * np.pi * w[:, 0] / 150.0), atol=1e-12)
    assert np.all(w[:, 3] == 15.0)
    c = np.asarray(sc["circles"])
    assert c.shape == (60, 5) and _moving(c) == 30          # 20 obstacles of 3 circles, 10 moving
    assert 0.8 <= c[:, 2].min() and c[:, 2].max() <= 1.5
    assert len(p["ego_off"]) == 3
    x0 = sc["x0"]
    assert x0[0] == 0.0 and x0[1] == 0.0 and x0[3] == 12.0
    assert math.isclose(x0[2], math.atan(5.0 * 2 * math.pi / 150.0), rel_tol=1e-12)


def test_stress_instance():
    sc = scenes.c4()
    p = sc["params"]
    assert (p["K"], p["T"]) == (262144, 200)
    assert np.asarray(sc["waypoints"]).shape == (301, 4)
    c = np.asarray(sc["circles"])
    assert c.shape == (512, 5) and _moving(c) == 128


def test_paper_table1_shape():
    p = scenes.paper_table1()["params"]
    assert (p["K"], p["T"], p["dt"], p["lam"]) == (2560, 16, 0.25, 150.0)
    assert tuple(p["sigma"]) == (0.85, 0.05)
    assert math.isclose(p["v_max"], 30.0 / 3.6)


def test_batched_instances():
    insts = scenes.c2(256)
    assert len(insts) == 256
    K = np.array([s["params"]["K"] for s in insts])
    T = np.array([s["params"]["T"] for s in insts])
    C = np.array([np.asarray(s["circles"]).shape[0] for s in insts])
    assert K.min() >= 1024 and K.max() <= 16384
    assert T.min() >= 30 and T.max() <= 150
    assert C.min() >= 0 and C.max() <= 64
    assert len(set(K.tolist())) > 1 and len(set(T.tolist())) > 10   # uneven shapes


@pytest.mark.parametrize("make", [scenes.c0, scenes.c1, scenes.c4, scenes.paper_table1,
                                  lambda: scenes.c2(8)[5]])
def test_generators_are_deterministic(make):
    a, b = make(), make()
    a = a if isinstance(a, dict) else a[0]
    b = b if isinstance(b, dict) else b[0]
    assert np.array_equal(np.asarray(a["waypoints"]), np.asarray(b["waypoints"]))
    assert np.array_equal(np.asarray(a["circles"]), np.asarray(b["circles"]))
    assert np.array_equal(np.asarray(a["x0"]), np.asarray(b["x0"]))
    assert a["params"] == b["params"]
