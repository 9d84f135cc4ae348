"""Parity of the HIP path (through the C ABI) with the FP64 oracle on MI355X.

Every case prints its name before it runs.  Sizes: the plain single
iteration (K=1024, T=50), ragged shapes that span several tiles with a
partial last tile and a partial last block of steps, the sine-lane instance
(K=8192, T=100, 10 warm-started iterations) and the stress instance
(K=262144, T=200, 512 circles) at full size with sampled checks.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2308_01654_amd import scenes
from tests import _parity as P

pytestmark = pytest.mark.gpu

# parity reports are written as JSON when MPPI_PARITY_OUT names a folder
OUT = os.environ.get("MPPI_PARITY_OUT")


def _mppi():
    from paper_2308_01654_amd import mppi
    mppi.load()  # raises if the HIP library is not built
    return mppi


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dump(name, obj):
    if not OUT:
        return
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "parity_%s.json" % name), "w") as f:
        json.dump(obj, f, indent=1, default=float)


def test_philox_words_bit_exact_full_stream_c0():
    """G0: the device Philox (same function the rollout calls) equals the
    oracle's for every counter of the plain iteration (K=1024, T=50 -> 25
    counters per sample) at iterations 0 and 7."""
    mppi = _mppi()
    for n_iter in (0, 7, (3 << 32) + 5):
        _say("philox c0 n_iter", n_iter)
        got = mppi.mppi_debug_philox(0, n_iter, 0, 1024, 0, 25)
        ctr = np.zeros((1024, 25, 4), dtype=np.uint32)
        ctr[..., 0] = np.arange(1024)[:, None]
        ctr[..., 1] = np.arange(25)[None, :]
        ctr[..., 2] = n_iter & 0xFFFFFFFF
        ctr[..., 3] = n_iter >> 32
        ref = O.philox_batch(ctr.reshape(-1, 4), [0, 0]).reshape(1024, 25, 4)
        assert np.array_equal(got, ref)


def test_philox_words_sampled_large():
    """G0 at the stress size: 2^20 counters (k < 262144, j < 100) bit-exact."""
    mppi = _mppi()
    seed = 0x0123456789ABCDEF
    got = mppi.mppi_debug_philox(seed, 9, 262144 - 10486, 10486, 0, 100)
    ctr = np.zeros((10486, 100, 4), dtype=np.uint32)
    ctr[..., 0] = (262144 - 10486 + np.arange(10486))[:, None]
    ctr[..., 1] = np.arange(100)[None, :]
    ctr[..., 2] = 9
    ref = O.philox_batch(ctr.reshape(-1, 4), [seed & 0xFFFFFFFF, seed >> 32]).reshape(got.shape)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16])
def test_c0_staged_parity_all_launch_shapes(lanes):
    """Plain single iteration, every lanes-per-sample shape."""
    mppi = _mppi()
    sc = scenes.c0()
    p = sc["params"]
    _say("c0 lanes", lanes)
    with mppi.Planner(p, lanes=lanes) as pl:
        g = P.gpu_step(pl, sc)
        assert g["stats"]["lanes"] == lanes
        assert g["stats"]["n_iter"] == 1 and g["stats"]["status"] == 0
        rep = P.staged(p, sc, g, n_iter=0)
        _dump("c0_lanes%d" % lanes, rep)
        P.assert_staged(rep)


@pytest.mark.parametrize("ego_off", [(0.0,), (0.0, 2.0), (0.0, 1.0, 2.7), (-0.5, 0.5, 1.5, 2.5),
                                     (0.0, 1.35, 2.7)])
@pytest.mark.parametrize("lanes", [4, 16])
def test_ego_circle_sets(ego_off, lanes):
    """One to four ego circles, equally spaced or not, on a scene where many
    samples come close to the obstacles: staged gates and culled == full."""
    mppi = _mppi()
    sc = scenes.tiny(K=2048, T=40, n_c=48, seed=11)
    p = dict(sc["params"], ego_off=ego_off)
    sc = dict(sc, params=p)
    _say("ego circles", ego_off, lanes)
    outs = []
    for cull in (1, 0):
        with mppi.Planner(p, lanes=lanes) as pl:
            pl.set_culling(cull)
            g = P.gpu_step(pl, sc)
            outs.append(g)
    P.assert_staged(P.staged(p, sc, outs[0], n_iter=0))
    for key in ("S", "w", "U"):
        assert np.array_equal(outs[0][key], outs[1][key]), key


def test_c0_end_to_end():
    """Plain single iteration against a fully independent oracle iteration
    (its own noise and rollouts): weights within 1e-5, controls within the
    1e-4 relative tolerance."""
    mppi = _mppi()
    sc = scenes.c0()
    p = sc["params"]
    with mppi.Planner(p) as pl:
        g = P.gpu_step(pl, sc)
    rep, ok, _ = P.end_to_end(p, sc, g, 0)
    _dump("c0_e2e", rep)
    _say("c0 e2e", rep)
    assert ok, rep


@pytest.mark.parametrize("K,T,n_c,lanes", [
    (1000, 37, 7, 16), (1000, 37, 7, 1), (777, 13, 0, 4), (1, 5, 3, 0), (300, 1, 2, 8),
    (4097, 64, 33, 2)])
def test_ragged_shapes(K, T, n_c, lanes):
    """Partial last tile, partial last block of steps, no circles, K = 1, T = 1."""
    mppi = _mppi()
    sc = scenes.tiny(K=K, T=T, n_c=n_c, seed=K + T)
    p = sc["params"]
    _say("ragged", K, T, n_c, lanes)
    with mppi.Planner(p, lanes=lanes) as pl:
        U0 = np.tile([0.1, -0.02], (T, 1))
        pl.set_controls(U0)
        g = P.gpu_step(pl, sc)
        rep = P.staged(p, sc, g, n_iter=0)
        P.assert_staged(rep)
        if K == 1:
            assert g["w"][0] == 1.0
            assert np.allclose(g["U"], U0 + g["eps"][:, 0, :], rtol=0, atol=1e-12)


@pytest.mark.parametrize("lanes", [1, 16])
def test_maximum_sizes(lanes):
    """Horizon, waypoint and circle counts at their maxima (2048, 2048, 1024):
    the workgroup's LDS then holds more than 64 KB; a ragged K; the costs of
    every tenth sample against the oracle."""
    mppi = _mppi()
    rng = np.random.Generator(np.random.PCG64(5))
    p = scenes.params(K=300, T=2048, dt=0.05, v_max=15.0, seed=3)
    sc = dict(params=p, x0=scenes._sine_x0(), waypoints=scenes.sine_lane(-20.0, 2027.0, 15.0),
              circles=scenes.sine_circles(rng, 1024, 10.0, 1500.0))
    assert len(sc["waypoints"]) == 2048 and len(sc["circles"]) == 1024
    _say("maximum sizes", lanes)
    with mppi.Planner(p, max_waypoints=2048, max_circles=1024, lanes=lanes) as pl:
        g = P.gpu_step(pl, sc)
    rep = P.staged(p, sc, g, n_iter=0, ks=np.arange(0, 300, 10))
    _say(" ", rep)
    # one lane walks all 2048 steps sequentially in float32: the position
    # rounding grows with the horizon (about seven times the 300-step bound;
    # measured 2.8e-4), while 16 lanes sum 128 blocks of prefix sums
    P.assert_staged(rep, s_rel=1.5e-3 if lanes == 1 else P.S_REL)


def test_single_waypoint_and_unbounded_controls():
    mppi = _mppi()
    sc = scenes.tiny(K=512, T=20, n_c=4)
    inf = float("inf")
    p = dict(sc["params"], u_min=(-inf, -inf), u_max=(inf, inf), v_max=inf)
    sc = dict(sc, params=p, waypoints=sc["waypoints"][5:6])
    with mppi.Planner(p) as pl:
        g = P.gpu_step(pl, sc)
        P.assert_staged(P.staged(p, sc, g, n_iter=0))


@pytest.mark.parametrize("lanes", [1, 4, 16])
def test_initial_speed_above_cap_and_binding_cap(lanes):
    """The speed cap of the noise check in both regimes of the walk: a start
    above v_max (the braking bound binds, the step-by-step recursion runs)
    and a start just under it with acceleration noise that keeps hitting the
    cap (the closed form with its prefix maximum)."""
    mppi = _mppi()
    base = scenes.c0()
    for v0, U0 in ((13.0, 0.5), (9.9, 1.0)):
        x0 = np.array(base["x0"], dtype=np.float64)
        x0[3] = v0
        sc = dict(base, x0=x0)
        p = sc["params"]
        _say("speed cap", lanes, v0)
        with mppi.Planner(p, lanes=lanes) as pl:
            pl.set_controls(np.tile([U0, 0.0], (p["T"], 1)))
            for it in range(2):
                g = P.gpu_step(pl, sc)
                P.assert_staged(P.staged(p, sc, g, n_iter=it))


@pytest.mark.parametrize("K,smoothing", [(8192, 0), (8208, 0), (32768, 0), (32784, 0),
                                         (16 * 32769, 0), (8208, 1), (32784, 1)])
def test_combine_at_the_direct_limit_and_above(K, smoothing):
    """Up to 512 tiles of 16 samples go to the narrow combine kernel, up to
    2048 to the wide one (513 and 2048 tiles); 2049 tiles and 32769 tiles
    are first merged by one and two levels of the in-kernel tree (down to
    129 and 2049 -> 129 nodes); with smoothing the combine reads the
    controls the first tile kept."""
    mppi = _mppi()
    sc = scenes.tiny(K=K, T=12, n_c=6, seed=K % 1000)
    p = dict(sc["params"], smoothing=smoothing)
    sc = dict(sc, params=p)
    _say("combine limit", K, smoothing)
    ks = None if K <= 32784 else np.arange(0, K, 257)
    with mppi.Planner(p, lanes=16) as pl:
        pl.set_controls(np.tile([0.1, -0.02], (12, 1)))
        for it in range(2):
            g = P.gpu_step(pl, sc)
            rep = P.staged(p, sc, g, n_iter=it, ks=ks)
            P.assert_staged(rep)


def test_zero_noise_gives_uniform_weights_and_no_update():
    mppi = _mppi()
    sc = scenes.tiny(K=2048, T=30, n_c=5)
    p = dict(sc["params"], sigma=(0.0, 0.0))
    with mppi.Planner(p) as pl:
        U0 = np.tile([0.3, 0.01], (30, 1))
        pl.set_controls(U0)
        g = P.gpu_step(pl, sc)
        assert np.all(g["S"] == g["S"][0])
        assert np.all(g["w"] == 1.0 / 2048)
        assert np.array_equal(g["U"], U0)
        assert g["stats"]["ess"] == pytest.approx(2048.0, rel=1e-12)


def test_small_lambda_selects_argmin():
    mppi = _mppi()
    sc = scenes.tiny(K=1024, T=25, n_c=6)
    p = dict(sc["params"], lam=1e-6)
    with mppi.Planner(p) as pl:
        g = P.gpu_step(pl, sc)
    k = int(np.argmin(g["S"]))
    assert g["w"][k] == 1.0
    assert np.allclose(g["U"], g["U_prev"] + g["eps"][:, k, :], rtol=0, atol=1e-12)


def test_all_costs_nonfinite_leaves_state_unchanged():
    """Forced from the host: a huge tracking weight makes every cost +inf."""
    mppi = _mppi()
    sc = scenes.tiny(K=256, T=10, n_c=2)
    p = dict(sc["params"], w_track=1e38)
    wp = np.array([[1e6, 1e6, 0.0, 15.0]])
    with mppi.Planner(p) as pl:
        U0 = np.tile([0.2, 0.0], (10, 1))
        pl.set_controls(U0)
        pl.step(sc["x0"], wp, sc["circles"])
        with pytest.raises(mppi.MppiError) as ei:
            pl.sync()
        assert ei.value.status == mppi.E_NONFINITE
        U, n, _ = pl.get_state()
        assert np.array_equal(U, U0) and n == 0
        # the next good step proceeds from the unchanged state
        pl.step(sc["x0"], sc["waypoints"], sc["circles"])
        pl.sync()
        assert pl.stats()["n_iter"] == 1


def test_invalid_arguments_are_rejected():
    mppi = _mppi()
    sc = scenes.tiny(K=64, T=8)
    with mppi.Planner(sc["params"], max_waypoints=64, max_circles=4) as pl:
        with pytest.raises(mppi.MppiError):
            pl.step([0, 0, float("nan"), 1.0], sc["waypoints"][:10], sc["circles"])
        with pytest.raises(mppi.MppiError):
            pl.step(sc["x0"], sc["waypoints"][:10], np.zeros((5, 5)))   # > max_circles
        with pytest.raises(mppi.MppiError):
            pl.step(sc["x0"], np.zeros((0, 4)), sc["circles"])
        with pytest.raises(mppi.MppiError):
            pl.shift(-1)
        # the handle still works
        pl.step(sc["x0"], sc["waypoints"][:10], sc["circles"])
        pl.sync()


def test_deterministic_and_checkpoint_restore():
    """Repeated runs are bit-identical; restoring a checkpoint continues the
    Philox stream bit-identically."""
    mppi = _mppi()
    sc = scenes.c1(K=2048, T=60)
    p = sc["params"]
    outs = []
    for rep in range(2):
        with mppi.Planner(p) as pl:
            for i in range(3):
                pl.step(sc["x0"], sc["waypoints"], sc["circles"])
            U_ck, n_ck, _ = pl.get_state()
            for i in range(2):
                pl.step(sc["x0"], sc["waypoints"], sc["circles"])
            U_end = pl.controls()
            pl.set_state(U_ck, n_ck)
            for i in range(2):
                pl.step(sc["x0"], sc["waypoints"], sc["circles"])
            assert np.array_equal(pl.controls(), U_end)
            outs.append(U_end)
    assert np.array_equal(outs[0], outs[1])


def test_shift_warm_start():
    mppi = _mppi()
    sc = scenes.tiny(K=64, T=6)
    with mppi.Planner(sc["params"]) as pl:
        U = np.arange(12, dtype=np.float64).reshape(6, 2)
        pl.set_controls(U)
        pl.shift(2)
        got = pl.controls()
        assert np.array_equal(got, np.vstack([U[2:], U[5:6], U[5:6]]))


def test_c1_ten_warm_iterations_staged():
    """Sine-lane instance, K=8192, T=100: 10 warm-started iterations.  Per
    iteration, every staged gate with the oracle re-synced to the GPU's
    previous controls, and the end-to-end tolerances (weights within 1e-5,
    controls within 1e-4 relative) against a fully independent oracle
    iteration from the same previous controls.  After the 10 iterations the
    GPU's controls are within the control tolerance of 10 free-running
    oracle iterations (which never see a GPU value)."""
    mppi = _mppi()
    sc = scenes.c1()
    p = sc["params"]
    reps = []
    U_free = np.zeros((p["T"], 2))
    with mppi.Planner(p) as pl:
        for i in range(sc["iterations"]):
            g = P.gpu_step(pl, sc)
            rep = P.staged(p, sc, g, n_iter=i)
            e2e, ok, _ = P.end_to_end(p, sc, g, i)
            rep["e2e"] = e2e
            rep["e2e_ok"] = ok
            reps.append(rep)
            _say("c1 iteration", i, "D2 %.2e" % rep["D2_max_rel"], "e2e", e2e)
            P.assert_staged(rep)
            assert ok, (i, e2e)
            U_free = O.iteration(p, sc["x0"], sc["waypoints"], sc["circles"], U_free, n_iter=i)["U"]
        U_gpu = pl.controls()
    free = float(np.max(np.abs(U_gpu - U_free) / P.u_tol(U_free, p["sigma"])))
    _say("c1 free-running controls, error / tolerance", free)
    _dump("c1", dict(iterations=reps, free_running_U_max_over_tol=free))
    assert free <= 1.0, free


def test_c4_stress_sampled():
    """Stress instance at full size (K=262144, T=200, 512 circles): weights
    and update checked on every sample, costs on 192 sampled rollouts."""
    mppi = _mppi()
    sc = scenes.c4()
    p = sc["params"]
    _say("c4 stress")
    with mppi.Planner(p) as pl:
        g = P.gpu_step(pl, sc)
    ks = np.unique(np.concatenate([
        np.random.Generator(np.random.PCG64(44)).integers(0, p["K"], size=160),
        np.argsort(g["S"])[:16], np.argsort(g["S"])[-16:]]))
    rep = P.staged(p, sc, g, n_iter=0, ks=ks)
    _dump("c4", rep)
    P.assert_staged(rep)


def test_c4_stress_end_to_end():
    """Stress instance at full size (K=262144, T=200, 512 circles) against a
    fully independent oracle iteration (52.4 M float64 rollout steps on the
    host cores): weights within 1e-5 on every sample and controls within the
    1e-4 relative tolerance; the report carries the cost error of the
    samples that carry weight (beta_near), the top-2 gap and the ESS."""
    mppi = _mppi()
    sc = scenes.c4()
    p = sc["params"]
    _say("c4 stress end to end: GPU iteration")
    with mppi.Planner(p) as pl:
        g = P.gpu_step(pl, sc)
    _say("c4 stress end to end: oracle iteration on %d threads" % O.max_threads())
    rep, ok, _ = P.end_to_end(p, sc, g, 0)
    _say("c4 e2e", rep)
    _dump("c4_e2e", rep)
    assert ok, rep


@pytest.mark.parametrize("lanes", [1, 4, 16])
def test_positive_braking_bound(lanes):
    """A positive lower acceleration bound (u_min = (0.3, -0.5)) with the
    start just under v_max: the noise check applies a >= a_min last, so the
    speed rises above v_max whenever the cap falls below a_min (the walk then
    runs step by step); staged gates over two iterations."""
    mppi = _mppi()
    base = scenes.c0()
    p = dict(base["params"], u_min=(0.3, -0.5))
    x0 = np.array(base["x0"], dtype=np.float64)
    x0[3] = p["v_max"] - 0.02
    sc = dict(base, params=p, x0=x0)
    _say("positive a_min", lanes)
    with mppi.Planner(p, lanes=lanes) as pl:
        pl.set_controls(np.tile([0.5, 0.0], (p["T"], 1)))
        for it in range(2):
            g = P.gpu_step(pl, sc)
            P.assert_staged(P.staged(p, sc, g, n_iter=it))


@pytest.mark.parametrize("name,lanes", [("c0", 16), ("c0", 1), ("c1", 8), ("c1", 2), ("paper_table1", 4),
                                        ("tiny", 16), ("c4small", 2)])
def test_culled_scans_bit_identical_to_full_scans(name, lanes):
    """The wave-level culling of waypoint chunks and obstacle circles changes
    no bit of the costs, the applied noise or the updated controls."""
    mppi = _mppi()
    if name == "c4small":
        sc = scenes.c4(K=4096, T=200)
    elif name == "tiny":
        sc = scenes.tiny(K=3000, T=45, n_c=40, seed=5)
    else:
        sc = scenes.by_name(name)
    p = sc["params"]
    _say("culling", name, lanes)
    outs = []
    for cull in (True, False):
        with mppi.Planner(p, lanes=lanes) as pl:
            pl.set_culling(cull)
            for _ in range(2):
                pl.step(sc["x0"], sc["waypoints"], sc["circles"])
            outs.append((pl.costs(), pl.noise(), pl.controls()))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("lanes,n_c", [(1, 0), (8, 0), (16, 0), (8, 40)])
def test_varying_reference_speed_and_repeated_waypoints(lanes, n_c):
    """Per-waypoint reference speeds with exactly repeated waypoint positions
    (the repeat has a reference speed 10 m/s higher, some repeats straddle
    chunks of 8): the closest index, lowest on ties, picks the reference
    speed.  The culled scan (minimum first, index resolved afterwards)
    equals the full scan bit for bit, and both meet the staged gates."""
    mppi = _mppi()
    # without circles the costs are tracking and speed terms of order 1e3, so
    # a wrong pick among repeated waypoints (10 m/s apart) fails gate D2
    sc = scenes.speed_profile(scenes.tiny(K=3000, T=45, n_c=n_c, seed=5), seed=9)
    p = sc["params"]
    _say("speed profile lanes", lanes, "circles", n_c, "waypoints", len(sc["waypoints"]))
    outs = []
    for cull in (True, False):
        with mppi.Planner(p, lanes=lanes) as pl:
            pl.set_culling(cull)
            g = P.gpu_step(pl, sc)
            rep = P.staged(p, sc, g, n_iter=0)
            P.assert_staged(rep)
            outs.append((g["S"], g["eps"], g["U"]))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("name,lanes", [("c1", 16), ("c4", 16), ("c0", 4), ("tiny", 1),
                                        ("tiny", 8)])
def test_occupancy_choice_bit_identical(name, lanes):
    """The iteration kernel compiled for five waves per SIMD (tuned per
    shape) computes the same bits as the default compilation (below 8 lanes
    the request falls back to the default)."""
    mppi = _mppi()
    sc = scenes.tiny(K=3000, T=45, n_c=40, seed=5) if name == "tiny" else scenes.by_name(name)
    p = sc["params"]
    outs = []
    for occ in (1, 0):
        _say("occupancy", name, lanes, occ)
        with mppi.Planner(p, lanes=lanes) as pl:
            pl.set_occupancy(occ)
            for _ in range(1 if name == "c4" else 2):
                pl.step(sc["x0"], sc["waypoints"], sc["circles"])
            outs.append((pl.costs(), pl.noise(), pl.controls(), pl.weights()))
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("name,lanes", [("c1", 16), ("c0", 4), ("tiny", 1)])
def test_staging_choice_bit_identical(name, lanes):
    """The tiles' LDS copy of their perturbations (tuned per shape) and the
    read-back from L2 give the same bits: the weighted sums run in the same
    order over the same values."""
    mppi = _mppi()
    sc = scenes.tiny(K=3000, T=45, n_c=40, seed=5) if name == "tiny" else scenes.by_name(name)
    p = sc["params"]
    outs = []
    for stage in (1, 0):
        with mppi.Planner(p, lanes=lanes) as pl:
            pl.set_staging(stage)
            for _ in range(2):
                pl.step(sc["x0"], sc["waypoints"], sc["circles"])
            outs.append((pl.costs(), pl.noise(), pl.controls(), pl.weights()))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)
