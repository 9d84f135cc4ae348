"""The 5-state vehicle model of eq. (5) on MI355X: the steering angle is
part of the state and the second control is the steering rate, clamped to
+-omega_max (Table I).  Staged parity with the oracle, culled = full scans
bit for bit, the optimal trajectory with its steering-angle column, batches
mixing both models, and the paper's closed-loop scenarios."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2308_01654_amd import scenes
from tests import _closed_loop as CL
from tests import _parity as P

pytestmark = pytest.mark.gpu


def _mppi():
    from paper_2308_01654_amd import mppi
    mppi.load()
    return mppi


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _c0_m5(steer0=0.08):
    return scenes.paper_model5(scenes.c0(), steer0=steer0)


@pytest.mark.parametrize("name", ["c0", "paper_merge", "paper_avoid", "paper_follow"])
@pytest.mark.parametrize("lanes", [1, 8, 16])
def test_model5_staged_parity(name, lanes):
    mppi = _mppi()
    sc = _c0_m5() if name == "c0" else scenes.paper_model5(scenes.by_name(name), steer0=-0.03)
    p = sc["params"]
    _say("5-state staged", name, lanes)
    with mppi.Planner(p, lanes=lanes) as pl:
        pl.set_steering(p["steer0"])
        pl.set_controls(np.tile([0.2, 0.01], (p["T"], 1)))
        for it in range(2):
            g = P.gpu_step(pl, sc)
            rep = P.staged(p, sc, g, n_iter=it)
            P.assert_staged(rep)


def test_model5_culled_equals_full_scan():
    mppi = _mppi()
    sc = scenes.paper_model5(scenes.c1(), steer0=0.05)
    p = sc["params"]
    outs = []
    for cull in (True, False):
        with mppi.Planner(p, lanes=8) as pl:
            pl.set_steering(0.05)
            pl.set_culling(cull)
            for _ in range(2):
                pl.step(sc["x0"], sc["waypoints"], sc["circles"])
            outs.append((pl.costs(), pl.noise(), pl.controls()))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_model5_trajectory_matches_oracle():
    mppi = _mppi()
    sc = scenes.paper_model5(scenes.paper_merge(), steer0=0.04)
    p = sc["params"]
    with mppi.Planner(p) as pl:
        pl.set_steering(0.04)
        for _ in range(2):
            pl.step(sc["x0"], sc["waypoints"], sc["circles"])
        xs, us = pl.trajectory()
        ref_x, ref_u = O.optimal_trajectory(p, sc["x0"], pl.controls())
    assert xs.shape == (p["T"] + 1, 5) and xs[0, 4] == 0.04
    assert np.max(np.abs(us - ref_u)) <= 1e-12
    assert np.max(np.abs(xs - ref_x)) <= 1e-9
    assert np.all(np.abs(us[:, 1]) <= 0.11 + 1e-15)


def test_batch_mixing_models_equals_alone():
    mppi = _mppi()
    scs = [_c0_m5(0.02), scenes.c0(), scenes.paper_model5(scenes.paper_follow(), 0.0),
           scenes.paper_follow()]
    ref = []
    for sc in scs:
        with mppi.Planner(sc["params"]) as pl:
            if sc["params"].get("model"):
                pl.set_steering(sc["params"]["steer0"])
            pl.step(sc["x0"], sc["waypoints"], sc["circles"])
            ref.append(pl.controls())
    pls = [mppi.Planner(scs[0]["params"])]
    try:
        s0 = pls[0].stream()
        pls += [mppi.Planner(sc["params"], hip_stream=s0) for sc in scs[1:]]
        for pl, sc in zip(pls, scs):
            if sc["params"].get("model"):
                pl.set_steering(sc["params"]["steer0"])
        mppi.step_batch(pls, [sc["x0"] for sc in scs], [(sc["waypoints"], sc["circles"]) for sc in scs])
        for i, pl in enumerate(pls):
            assert np.array_equal(pl.controls(), ref[i]), i
    finally:
        for pl in reversed(pls):
            pl.close()


def test_server_rejects_the_steering_rate_model():
    mppi = _mppi()
    with mppi.Server(n_streams=1) as srv:
        with pytest.raises(mppi.MppiError):
            srv.add_vehicle(_c0_m5()["params"])


@pytest.mark.parametrize("name", ["paper_merge", "paper_avoid", "paper_follow"])
def test_model5_paper_scenarios_closed_loop(name):
    mppi = _mppi()
    sc = scenes.paper_model5(scenes.by_name(name))
    p = sc["params"]
    with mppi.Planner(p) as pl:
        def plan(k, x, circ):
            if k:
                pl.shift(1)
            pl.set_steering(float(x[4]))
            pl.step(x[:4], sc["waypoints"], circ)
            return pl.trajectory()

        xs, us, ds = CL.drive(sc, plan, 60)
    _say(name, "final", np.round(xs[-1], 3), "max |delta|", float(np.abs(xs[:, 4]).max()),
         "min clearance", float(ds.min()))
    CL.check_outcomes(name, p, xs, us, ds)
