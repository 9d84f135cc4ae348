"""Batched iterations: many uneven instances in one persistent launch replayed
as a HIP graph.  Every instance must compute exactly the bits it computes
alone; graph replays are checked one by one against eager single-instance
runs of the same work interleaved between them."""
import sys

import numpy as np
import pytest

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


SHAPES = [(1024, 30, 0), (2048, 150, 64), (4096, 77, 13), (8192, 100, 60), (1024, 45, 1),
          (16384, 31, 40), (3000, 64, 7), (512, 150, 64), (2048, 99, 33), (1, 40, 5)]


def _instances():
    out = []
    for i, shp in enumerate(SHAPES):
        sc = scenes.c2_instance(i, shp)
        out.append(sc)
    return out


def _run_alone(mppi, sc, iters, U0=None, lanes=0):
    with mppi.Planner(sc["params"], lanes=lanes) as pl:
        if U0 is not None:
            pl.set_controls(U0)
        res = []
        for _ in range(iters):
            pl.step(sc["x0"], sc["waypoints"], sc["circles"])
            res.append((pl.controls(), pl.costs(), pl.weights()))
        return res


def test_batch_equals_alone_bitwise_with_graph_replays():
    mppi = _mppi()
    insts = _instances()
    iters = 3
    _say("alone runs")
    alone = [_run_alone(mppi, sc, iters) for sc in insts]
    _say("batched runs")
    lead = mppi.Planner(insts[0]["params"])
    pls = [lead] + [mppi.Planner(sc["params"], hip_stream=lead.stream()) for sc in insts[1:]]
    try:
        x0s = np.array([sc["x0"] for sc in insts])
        arrays = [(sc["waypoints"], sc["circles"]) for sc in insts]
        for it in range(iters):
            mppi.step_batch(pls, x0s, arrays)
            # eager single-instance work on another handle between replays
            _run_alone(mppi, insts[3], 1)
            bad = []
            for k, pl in enumerate(pls):
                U, S, w = alone[k][it]
                Ub, Sb, wb = pl.controls(), pl.costs(), pl.weights()
                if not (np.array_equal(Ub, U) and np.array_equal(Sb, S) and np.array_equal(wb, w)):
                    bad.append((it, k, float(np.max(np.abs(Ub - U))), float(np.max(np.abs(Sb - S))),
                                int(np.sum(Sb != S)), pl.stats()))
                assert pl.stats()["n_iter"] == it + 1
            for b in bad:
                _say("mismatch", b)
            assert not bad
    finally:
        for pl in pls:
            pl.close()


def test_batch_resident_scenes_and_subset_order():
    """Resident scenes (no per-call scene copy) and a batch that lists the
    handles in a different order give the same bits."""
    mppi = _mppi()
    insts = _instances()[:6]
    alone = [_run_alone(mppi, sc, 2) for sc in insts]
    lead = mppi.Planner(insts[0]["params"])
    pls = [lead] + [mppi.Planner(sc["params"], hip_stream=lead.stream()) for sc in insts[1:]]
    try:
        for pl, sc in zip(pls, insts):
            pl.set_scene(sc["x0"], sc["waypoints"], sc["circles"])
        perm = [4, 1, 5, 0, 3, 2]
        x0s = np.array([insts[k]["x0"] for k in perm])
        for it in range(2):
            mppi.step_batch([pls[k] for k in perm], x0s, None)
            for k in range(len(insts)):
                assert np.array_equal(pls[k].controls(), alone[k][it][0]), (it, k)
    finally:
        for pl in pls:
            pl.close()


def test_batch_staged_parity_against_oracle():
    mppi = _mppi()
    insts = [scenes.c2_instance(i, shp) for i, shp in enumerate([(1024, 40, 9), (2048, 33, 0), (777, 61, 20)])]
    lead = mppi.Planner(insts[0]["params"])
    pls = [lead] + [mppi.Planner(sc["params"], hip_stream=lead.stream()) for sc in insts[1:]]
    try:
        prev = [pl.controls() for pl in pls]
        mppi.step_batch(pls, np.array([sc["x0"] for sc in insts]),
                        [(sc["waypoints"], sc["circles"]) for sc in insts])
        for pl, sc, U_prev in zip(pls, insts, prev):
            g = dict(U_prev=U_prev, U=pl.controls(), S=pl.costs().astype(np.float64),
                     w=pl.weights(), eps=pl.noise().astype(np.float64), stats=pl.stats())
            P.assert_staged(P.staged(sc["params"], sc, g, n_iter=0))
    finally:
        for pl in pls:
            pl.close()


def test_batch_rejects_mixed_streams_and_duplicates():
    mppi = _mppi()
    a = scenes.tiny(K=64, T=8)
    with mppi.Planner(a["params"]) as p1, mppi.Planner(a["params"]) as p2:
        with pytest.raises(mppi.MppiError):
            mppi.step_batch([p1, p2], np.array([a["x0"], a["x0"]]),
                            [(a["waypoints"], a["circles"])] * 2)
        with pytest.raises(mppi.MppiError):
            mppi.step_batch([p1, p1], np.array([a["x0"], a["x0"]]),
                            [(a["waypoints"], a["circles"])] * 2)
        assert p1.stats()["n_iter"] == 0


def test_c2_full_draw_staged_parity():
    """The 256 uneven instances of the batched workload (K in {1024..16384},
    T in [30, 150], 0-64 circles, each its own seeded scene) stepped as one
    batch: per instance the applied perturbations and costs of 32 sampled
    samples (the cheapest and dearest four among them) against the oracle
    fed the GPU's perturbations, the weights on every sample against the
    oracle normaliser fed the GPU's costs and the controls against the
    oracle update fed the GPU's weights and perturbations; four instances
    (the largest K, the longest T, the most circles and one without circles)
    end to end against fully independent oracle iterations."""
    mppi = _mppi()
    insts = scenes.c2()
    _say("c2 full draw: %d instances" % len(insts))
    lead = mppi.Planner(insts[0]["params"])
    pls = [lead] + [mppi.Planner(sc["params"], hip_stream=lead.stream()) for sc in insts[1:]]
    try:
        prev = [pl.controls() for pl in pls]
        mppi.step_batch(pls, np.array([sc["x0"] for sc in insts]),
                        [(sc["waypoints"], sc["circles"]) for sc in insts])
        shapes = [(sc["params"]["K"], sc["params"]["T"], len(sc["circles"])) for sc in insts]
        e2e_ids = {int(np.argmax([s[0] * 1000 + s[1] for s in shapes])),
                   int(np.argmax([s[1] * 100000 + s[0] for s in shapes])),
                   int(np.argmax([s[2] for s in shapes])),
                   int(np.argmin([s[2] for s in shapes]))}
        worst = dict(D1=0.0, D2=0.0, G2=0.0, G3=0.0)
        rng = np.random.Generator(np.random.PCG64(77))
        for i, (pl, sc, U_prev) in enumerate(zip(pls, insts, prev)):
            p = sc["params"]
            g = dict(U_prev=U_prev, U=pl.controls(), S=pl.costs().astype(np.float64),
                     w=pl.weights(), eps=pl.noise().astype(np.float64), stats=pl.stats())
            order = np.argsort(g["S"])
            ks = np.unique(np.concatenate([rng.integers(0, p["K"], size=24), order[:4], order[-4:]]))
            rep = P.staged(p, sc, g, n_iter=0, ks=ks)
            worst["D1"] = max(worst["D1"], rep["D1_max_abs_over_sigma"])
            worst["D2"] = max(worst["D2"], rep["D2_max_rel"])
            worst["G2"] = max(worst["G2"], rep["G2_max_abs"])
            worst["G3"] = max(worst["G3"], rep["G3_max_over_tol"])
            P.assert_staged(rep)
            if i in e2e_ids:
                e2e, ok, _ = P.end_to_end(p, sc, g, 0)
                _say("  e2e instance", i, shapes[i], e2e)
                assert ok, (i, e2e)
        _say("c2 worst gates", worst)
    finally:
        for pl in reversed(pls):
            pl.close()


@pytest.mark.parametrize("K", [32784, 16 * 2049 + 5])
def test_batched_tile_tree_equals_alone_tile_tree(K):
    """Above 2048 tiles the iteration kernel first merges an instance's
    tiles by its ticket tree (one and two levels here), alone and inside a
    batch: the groups depend on the instance only, so a batch with a small
    instance alongside gives the big instance its alone bits."""
    mppi = _mppi()
    big = scenes.tiny(K=K, T=20, n_c=9, seed=K % 997)
    small = scenes.c2_instance(0, SHAPES[0])
    insts = [big, small]
    alone = [_run_alone(mppi, big, 2, lanes=16), _run_alone(mppi, small, 2)]
    lead = mppi.Planner(insts[0]["params"], lanes=16)
    pls = [lead, mppi.Planner(small["params"], hip_stream=lead.stream())]
    try:
        x0s = np.array([sc["x0"] for sc in insts])
        arrays = [(sc["waypoints"], sc["circles"]) for sc in insts]
        for it in range(2):
            mppi.step_batch(pls, x0s, arrays)
            for k, pl in enumerate(pls):
                U, S, w = alone[k][it]
                assert np.array_equal(pl.costs(), S), (it, k)
                assert np.array_equal(pl.weights(), w), (it, k)
                assert np.array_equal(pl.controls(), U), (it, k)
    finally:
        for pl in pls:
            pl.close()


def test_batch_with_high_occupancy_instances():
    """Instances set to the other compilations of the iteration kernel form
    launch classes of their own in a batch; every instance keeps its alone
    bits."""
    mppi = _mppi()
    insts = _instances()[:5]
    occ = [1, 0, 1, 1, 0]
    alone = []
    for sc, o in zip(insts, occ):
        with mppi.Planner(sc["params"]) as pl:
            pl.set_occupancy(o)
            pl.step(sc["x0"], sc["waypoints"], sc["circles"])
            alone.append((pl.costs(), pl.controls()))
    lead = mppi.Planner(insts[0]["params"])
    pls = [lead] + [mppi.Planner(sc["params"], hip_stream=lead.stream()) for sc in insts[1:]]
    try:
        for pl, o in zip(pls, occ):
            pl.set_occupancy(o)
        mppi.step_batch(pls, np.array([sc["x0"] for sc in insts]),
                        [(sc["waypoints"], sc["circles"]) for sc in insts])
        for k, pl in enumerate(pls):
            assert np.array_equal(pl.costs(), alone[k][0]), k
            assert np.array_equal(pl.controls(), alone[k][1]), k
    finally:
        for pl in reversed(pls):
            pl.close()


@pytest.mark.parametrize("T", [60, 64, 65, 128, 132])
def test_combine_step_group_runs(T):
    """Horizons whose number of 4-step combine groups is just below, at and
    just past a whole run of 16 (15, 16, 17, 32, 33 groups).  Alone, the
    combine grid is padded to whole runs and paired workgroups share an
    XCD; in a batch with a longer horizon (38 groups) the grid is not padded
    and a short last run maps one to one.  Staged parity alone, and the
    batched instance computes the alone bits over two iterations."""
    mppi = _mppi()
    sc = scenes.c2_instance(3, (2048, T, 12))
    other = scenes.c2_instance(5, (1024, 150, 5))
    p = sc["params"]
    _say("group runs", T)
    with mppi.Planner(p) as pl:
        g = P.gpu_step(pl, sc)
    P.assert_staged(P.staged(p, sc, g, n_iter=0))
    alone = _run_alone(mppi, sc, 2)
    lead = mppi.Planner(other["params"])
    pls = [lead, mppi.Planner(p, hip_stream=lead.stream())]
    try:
        x0s = np.array([other["x0"], sc["x0"]])
        arrays = [(other["waypoints"], other["circles"]), (sc["waypoints"], sc["circles"])]
        for it in range(2):
            mppi.step_batch(pls, x0s, arrays)
            U, S, w = alone[it]
            assert np.array_equal(pls[1].controls(), U), (T, it)
            assert np.array_equal(pls[1].costs(), S), (T, it)
            assert np.array_equal(pls[1].weights(), w), (T, it)
    finally:
        for q in reversed(pls):
            q.close()
