"""Per-step weights on MI355X: the update of U_t weights the samples by their
cost-to-go from t, S_t,k = sum_{s>=t} q_s,k, with its own minimum per step
(eq. (update-input) indexed by t).

Gates, in the style of the total-cost path:
  Q   stage costs q_t,k vs the oracle rollout fed the GPU's applied
      perturbations (|dq| <= 1e-3 of the sample's total cost);
  G3  controls vs the oracle's per-step update fed the GPU's stage costs and
      perturbations, to the control tolerance (1e-4 relative, floored at
      sigma);
  W   step-0 weights and statistics vs the oracle normaliser of the same
      float64 cost-to-go;
and the end-to-end comparison against the fully independent oracle
iteration, bit identity of batched / served runs with runs alone, and of
culled with full scans."""
import json
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2308_01654_amd import scenes
from tests import _parity as P

pytestmark = pytest.mark.gpu


def _mppi():
    from paper_2308_01654_amd import mppi
    mppi.load()
    return mppi


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# parity reports are written as JSON when MPPI_PARITY_OUT names a folder
OUT = os.environ.get("MPPI_PARITY_OUT")


def _dump(name, obj):
    if not OUT:
        return
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "parity_per_step_%s.json" % name), "w") as f:
        json.dump(obj, f, indent=1, default=float)


def _per_step(sc, **kw):
    sc = dict(sc)
    sc["params"] = dict(sc["params"], per_step=1, **kw)
    return sc


def _step(pl, sc):
    U_prev = pl.controls()
    pl.step(sc["x0"], sc["waypoints"], sc["circles"])
    pl.sync()
    return dict(U_prev=U_prev, U=pl.controls(), S=pl.costs().astype(np.float64),
                q=pl.stage_costs().astype(np.float64), w=pl.weights(),
                eps=pl.noise().astype(np.float64), stats=pl.stats())


def _staged(p, sc, g, n_iter):
    sig = np.asarray(p["sigma"], dtype=np.float64)
    S_inj, _, q_inj = O.rollout(p, sc["x0"], sc["waypoints"], sc["circles"], g["U_prev"],
                                n_iter=n_iter, eps_in=g["eps"], stage_costs=True)
    rep = {}
    rep["Q_max"] = float(np.max(np.abs(g["q"] - q_inj) / np.maximum(np.abs(S_inj), 1e-30)[None, :]))
    rep["S_vs_sum_q"] = float(np.max(np.abs(g["q"].sum(axis=0) - g["S"]) /
                                     np.maximum(np.abs(g["S"]), 1e-30)))
    U_ref, Stk, w0 = O.update_per_step(g["U_prev"], g["q"], g["eps"], p["lam"])
    if p.get("smoothing", 0):
        U_ref = O.sg_smooth(U_ref)
    rep["G3_max_over_tol"] = float(np.max(np.abs(g["U"] - U_ref) / P.u_tol(U_ref, sig)))
    _, smin, logz = O.weights(Stk[0], p["lam"])
    rep["W_max_abs"] = float(np.max(np.abs(g["w"] - w0)))
    rep["s_min"] = (g["stats"]["s_min"], smin)
    rep["log_z"] = (g["stats"]["log_z"], logz)
    rep["status"] = g["stats"]["status"]
    return rep


def _assert_staged(rep):
    assert rep["status"] == 0, rep
    assert rep["Q_max"] <= P.S_REL, rep
    assert rep["S_vs_sum_q"] <= 1e-5, rep
    assert rep["G3_max_over_tol"] <= 1.0, rep
    assert rep["W_max_abs"] <= P.W_TOL, rep
    assert abs(rep["s_min"][0] - rep["s_min"][1]) <= 1e-12 * max(1.0, abs(rep["s_min"][1])), rep
    assert abs(rep["log_z"][0] - rep["log_z"][1]) <= 1e-9, rep


@pytest.mark.parametrize("name", ["c0", "paper_merge", "paper_avoid"])
@pytest.mark.parametrize("lanes", [1, 4, 16])
def test_per_step_staged_parity(name, lanes):
    mppi = _mppi()
    sc = _per_step(scenes.by_name(name))
    p = sc["params"]
    _say("per-step staged", name, lanes)
    reps = []
    with mppi.Planner(p, lanes=lanes) as pl:
        pl.set_controls(np.tile([0.3, -0.01], (p["T"], 1)))
        for it in range(2):
            g = _step(pl, sc)
            rep = _staged(p, sc, g, it)
            _say(" ", it, rep)
            reps.append(rep)
            _assert_staged(rep)
    _dump("%s_lanes%d" % (name, lanes), reps)


@pytest.mark.parametrize("K,T", [(1, 1), (37, 3), (300, 1), (1000, 23), (4099, 130)])
def test_per_step_ragged_shapes(K, T):
    mppi = _mppi()
    sc = _per_step(scenes.tiny(K=K, T=T, n_c=9, seed=K + T))
    p = sc["params"]
    _say("per-step ragged", K, T)
    with mppi.Planner(p) as pl:
        g = _step(pl, sc)
        _assert_staged(_staged(p, sc, g, 0))


@pytest.mark.parametrize("smoothing", [0, 1])
def test_per_step_above_the_direct_limit(smoothing):
    """600 tiles of 16 samples: the per-step combine walks more tile rows
    than the total-cost combine takes in one pass."""
    mppi = _mppi()
    sc = _per_step(scenes.tiny(K=9600, T=20, n_c=5, seed=31), smoothing=smoothing)
    p = sc["params"]
    with mppi.Planner(p, lanes=16) as pl:
        for it in range(2):
            g = _step(pl, sc)
            _assert_staged(_staged(p, sc, g, it))


def test_per_step_with_smoothing_and_model5():
    mppi = _mppi()
    sc = _per_step(scenes.paper_model5(scenes.paper_follow(), steer0=0.02), smoothing=1)
    p = sc["params"]
    with mppi.Planner(p, lanes=8) as pl:
        pl.set_steering(0.02)
        for it in range(2):
            g = _step(pl, sc)
            _assert_staged(_staged(p, sc, g, it))


def test_per_step_end_to_end_c0():
    mppi = _mppi()
    sc = _per_step(scenes.c0())
    p = sc["params"]
    with mppi.Planner(p) as pl:
        g = _step(pl, sc)
    r = O.iteration(p, sc["x0"], sc["waypoints"], sc["circles"], g["U_prev"], n_iter=0)
    sig = np.asarray(p["sigma"], dtype=np.float64)
    du = float(np.max(np.abs(g["U"] - r["U"]) / P.u_tol(r["U"], sig)))
    dw = float(np.max(np.abs(g["w"] - r["w"])))
    beta = float(np.max(np.abs(g["S"] - r["S"])))
    _say("per-step e2e", dict(U_max_over_tol=du, w_max_abs=dw, beta=beta, lam=p["lam"]))
    _dump("c0_e2e", dict(U_max_over_tol=du, w_max_abs=dw, beta=beta, lam=p["lam"]))
    assert du <= 1.0 and dw <= P.W_TOL


def test_one_step_horizon_matches_total_cost_update():
    """T = 1: the cost-to-go is the total cost, so both weightings give the
    same update up to the rounding of their sums."""
    mppi = _mppi()
    base = scenes.tiny(K=2000, T=1, n_c=5, seed=21)
    outs = []
    for ps in (0, 1):
        sc = _per_step(base) if ps else base
        with mppi.Planner(sc["params"]) as pl:
            pl.set_controls([[0.2, 0.03]])
            pl.step(sc["x0"], sc["waypoints"], sc["circles"])
            outs.append((pl.controls(), pl.weights()))
    sig = np.asarray(base["params"]["sigma"], dtype=np.float64)
    assert np.max(np.abs(outs[0][0] - outs[1][0]) / P.u_tol(outs[0][0], sig)) <= 1.0
    assert np.max(np.abs(outs[0][1] - outs[1][1])) <= P.W_TOL


def test_per_step_culled_equals_full_scan():
    mppi = _mppi()
    sc = _per_step(scenes.c1())
    p = sc["params"]
    outs = []
    for cull in (True, False):
        with mppi.Planner(p, lanes=8) as pl:
            pl.set_culling(cull)
            for _ in range(2):
                pl.step(sc["x0"], sc["waypoints"], sc["circles"])
            outs.append((pl.costs(), pl.stage_costs(), pl.controls(), pl.weights()))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_batch_mixing_weightings_equals_alone():
    mppi = _mppi()
    scs = [_per_step(scenes.c0()), scenes.c0(), _per_step(scenes.paper_merge()),
           scenes.paper_avoid(), _per_step(scenes.tiny(K=77, T=5, n_c=2, seed=3))]
    ref = []
    for sc in scs:
        with mppi.Planner(sc["params"]) as pl:
            for i in range(2):
                if i:
                    pl.shift(1)
                pl.step(sc["x0"], sc["waypoints"], sc["circles"])
            ref.append((pl.controls(), pl.stats()))
    pls = [mppi.Planner(scs[0]["params"])]
    try:
        s0 = pls[0].stream()
        pls += [mppi.Planner(sc["params"], hip_stream=s0) for sc in scs[1:]]
        for i in range(2):
            if i:
                for pl in pls:
                    pl.shift(1)
            mppi.step_batch(pls, [sc["x0"] for sc in scs],
                            [(sc["waypoints"], sc["circles"]) for sc in scs])
        for i, pl in enumerate(pls):
            assert np.array_equal(pl.controls(), ref[i][0]), i
            st = pl.stats()
            for key in ("s_min", "log_z", "ess", "n_iter", "status"):
                assert st[key] == ref[i][1][key], (i, key)
    finally:
        for pl in reversed(pls):
            pl.close()


def test_served_per_step_equals_alone():
    mppi = _mppi()
    rng = np.random.Generator(np.random.PCG64(11))
    vehs = []
    for v in range(4):
        p = dict(scenes.params(K=int(rng.choice([256, 1000, 2048])), T=int(rng.choice([20, 50])),
                               dt=0.05, v_max=15.0, seed=900 + v), per_step=v % 2)
        x = float(rng.uniform(-5, 20))
        reqs = []
        for i in range(3):
            circ = scenes.sine_circles(rng, int(rng.integers(0, 20)), x + 5, x + 80)
            wp = scenes.sine_lane(np.floor(x) - 20, np.floor(x) + 120, 15.0)
            reqs.append((scenes._sine_x0(x, 12.0), wp, circ))
            x += 0.75
        vehs.append((p, reqs))
    ref = []
    for p, reqs in vehs:
        out = []
        with mppi.Planner(p) as pl:
            for i, (x0, wp, ci) in enumerate(reqs):
                if i:
                    pl.shift(1)
                pl.step(x0, wp, ci)
                out.append(pl.controls())
        ref.append(out)
    with mppi.Server(n_streams=2, max_batch=16) as srv:
        vids = [srv.add_vehicle(p) for p, _ in vehs]
        tickets = []
        for i in range(3):
            for vid, (p, reqs) in zip(vids, vehs):
                tickets.append((vid, i, srv.submit(vid, *reqs[i])))
        res = {(vid, i): srv.wait(t, vid)[0] for vid, i, t in tickets}
    for v, vid in enumerate(vids):
        for i in range(3):
            assert np.array_equal(res[(vid, i)], ref[v][i]), (v, i)


def test_stage_costs_rejected_without_per_step():
    mppi = _mppi()
    sc = scenes.tiny(K=64, T=4, n_c=1, seed=1)
    with mppi.Planner(sc["params"]) as pl:
        pl.step(sc["x0"], sc["waypoints"], sc["circles"])
        with pytest.raises(mppi.MppiError):
            pl.stage_costs()
