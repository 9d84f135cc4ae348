#!/usr/bin/env python3
"""Benchmark of one MPPI iteration on one MI355X.

A step is one MPPI iteration (noise generation, rollouts, costs, weights and
the control update) of the sine-lane single instance: K = 8192 samples,
T = 100 steps, dt = 0.05 s, 221 waypoints, 20 obstacles x 3 circles (half
moving), warm-started (U and the Philox counter carry over between steps).
The scene is staged in HBM before the timed region (``mppi_set_scene``) and
every timed step is ``mppi_step_resident``.

Prints one JSON line: throughput in rollout-steps/s (K*T per iteration over
the HIP-event time of the timed region), the roofline of the fused iteration
kernel (algorithmic FP32 flops per launch over its HIP-event duration, and
the FP32 work it executes from committed hardware counters), the plain
one-at-a-time replan latency percentiles, the host-buffer (PCIe inclusive)
rate, the served and plain paths under the 20 Hz fleet load, the other
workloads' iteration times, and the FP64 CPU oracle timed on the host on
bounded samples of the same workloads (all cores and one core).

Usage: python bench.py [--gpus 1] [--steps 200] [--warmup 20]
       python bench.py --serve-sweep [--sweep-seconds 60] [--served-fleets
           1000,2000,4000] [--plain-fleets 250,500,750,1000]   (served and
           plain paths at several offered loads; one JSON line per run)
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2308_01654_amd.hip_events import HipEvents, time_steps  # noqa: E402

PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak
METRIC = "rollout-steps/s (K=8192,T=100) + p99 replan latency, served vs plain MPPI"
KERNEL_SRC = os.path.join(ROOT, "paper_2308_01654_amd", "csrc", "mppi_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_iteration_c1.json")


def flops_per_rollout_step(n_wp, n_c, n_ego):
    """Algorithmic FP32 flops of one rollout step (FMA = 2, transcendental = 1):
    73 for noise, noise check, dynamics, speed/effort/obstacle post-processing
    and the compensated sum; 6 per waypoint; 7 per ego-circle x obstacle-circle
    pair."""
    return 73 + 6 * n_wp + 7 * n_ego * n_c


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(n_launch_units):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters_iteration_c1.json")
TRACE_FILE = os.path.join(ROOT, "profiles", "trace_iteration_c1.json")


def load_trace():
    """Kernel-trace statistics of the iteration and combine kernels at the
    benchmark workload (rocprofv3 --kernel-trace --stats of bench.py --probe),
    if they were taken on the current kernel source."""
    try:
        with open(TRACE_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t


def load_counters():
    """SQ counters of the iteration kernel (one dispatch at the benchmark
    workload) from the committed rocprofv3 summary, if it was taken on the
    current kernel source."""
    try:
        with open(COUNTERS_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_iterations(O, sc, seconds):
    """Warm-started full oracle iterations until `seconds` have passed."""
    p = sc["params"]
    U = np.zeros((p["T"], 2))
    n = 0
    t0 = time.perf_counter()
    while True:
        U = O.iteration(p, sc["x0"], sc["waypoints"], sc["circles"], U, n_iter=n)["U"]
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return p["K"] * p["T"] * n / el, "%d full iteration(s) in %.2f s" % (n, el)


def _oracle_rollouts(O, sc, n_samples):
    """Rollouts (noise, dynamics, stage costs) of the first n_samples samples
    of the instance: the bulk of an iteration's work."""
    p = sc["params"]
    ks = np.arange(min(n_samples, p["K"]))
    t0 = time.perf_counter()
    O.rollout_samples(p, sc["x0"], sc["waypoints"], sc["circles"], np.zeros((p["T"], 2)), ks)
    el = time.perf_counter() - t0
    return ks.size * p["T"] / el, "rollouts of %d of the %d samples in %.2f s" % (ks.size, p["K"], el)


def cpu_baseline(sc, seconds, mean_request_steps):
    """The FP64 oracle, unchanged, on the host cores.  Headline: full
    warm-started iterations of the benchmark workload for `seconds` on every
    core.  Rows: the plain, stress and paper-shaped workloads on every core
    and on one (bounded samples: full iterations where they take a fraction
    of a second, else the rollouts of a subset of the samples), and the
    request rate of the served fleet's mix that the all-core rate implies."""
    from oracle import oracle as O
    from paper_2308_01654_amd import scenes
    p = sc["params"]
    n_all = O.max_threads()
    value, what = _oracle_iterations(O, sc, seconds)
    out = dict(value=value, unit="rollout-steps/s", cores=n_all, kind="oracle",
               sample="%s of the K=%d, T=%d sine-lane instance (warm-started FP64 oracle)"
                      % (what, p["K"], p["T"]),
               cpu_model=cpu_model(), rows=[])
    cases = [("plain K=1024 T=50", scenes.c0(), "iter", 1.0, 1.0),
             ("sine lane K=8192 T=100", sc, "roll", None, 2048),
             ("stress K=262144 T=200", scenes.c4(), "roll", 16384, 512),
             ("paper Table I shape K=2560 T=16", scenes.paper_table1(), "iter", 1.0, 1.0)]
    try:
        for threads in (n_all, 1):
            O.set_threads(threads)
            for name, c, kind, a_all, a_one in cases:
                arg = a_all if threads == n_all else a_one
                if arg is None:
                    rate, what = value, "the headline sample"
                elif kind == "iter":
                    rate, what = _oracle_iterations(O, c, arg)
                else:
                    rate, what = _oracle_rollouts(O, c, arg)
                out["rows"].append(dict(workload=name, threads=threads,
                                        rollout_steps_per_s=round(rate, 1), sample=what))
    finally:
        O.set_threads(n_all)
    out["served_mix_requests_per_s"] = round(value / mean_request_steps, 1)
    out["served_mix_mean_steps_per_request"] = mean_request_steps
    return out


def workload_rows(steps=20):
    """Iteration time of the other workloads on the GPU (library's launch
    shape, HIP events, resident scenes): the plain single iteration, the
    stress instance, the paper's Table I shape, and the share of one GPU in
    an eight-GPU split of a stress-sized instance (K = 32768 of 262144)."""
    from paper_2308_01654_amd import scenes
    rows = []
    cases = [("plain K=1024 T=50", scenes.c0()), ("stress K=262144 T=200", scenes.c4()),
             ("paper Table I shape K=2560 T=16", scenes.paper_table1()),
             ("one GPU's share of the stress instance, K=32768 T=200", scenes.c4(K=32768))]
    for name, sc in cases:
        p = sc["params"]
        F = flops_per_rollout_step(len(sc["waypoints"]), len(sc["circles"]), len(p["ego_off"]))
        ms = _iteration_ms(p, sc["x0"], sc["waypoints"], sc["circles"], 3, steps)
        rate = p["K"] * p["T"] / (ms * 1e-3)
        rows.append(dict(workload=name, iteration_ms=ms, rollout_steps_per_s=round(rate, 1),
                         full_scan_equivalent_tflops=round(F * rate / 1e12, 2)))
    return rows


def probe(steps, workload="c1"):
    """Dispatches for hardware-counter and kernel-trace runs: a 256 MiB
    streaming copy (the calibration reference, 3 dispatches), then `steps`
    warm-started iterations of one workload: "c1" the sine-lane benchmark
    instance, "c4" the stress instance, "c2" the 256 uneven instances of the
    batched workload stepped by mppi_step_batch."""
    from paper_2308_01654_amd import mppi, scenes
    mppi.check(mppi.load().mppi_bench_copy(256 << 20, 3))
    if workload == "c2":
        insts = scenes.c2(256)
        pls = [mppi.Planner(insts[0]["params"])]
        st = pls[0].stream()
        pls += [mppi.Planner(sc["params"], hip_stream=st) for sc in insts[1:]]
        for pl, sc in zip(pls, insts):
            pl.set_scene(sc["x0"], sc["waypoints"], sc["circles"])
        x0s = [sc["x0"] for sc in insts]
        for _ in range(steps):
            mppi.step_batch(pls, x0s)
        pls[0].sync()
        for pl in reversed(pls):
            pl.close()
    else:
        sc = scenes.c1() if workload == "c1" else scenes.by_name(workload)
        pl = mppi.Planner(sc["params"])
        pl.set_scene(sc["x0"], sc["waypoints"], sc["circles"])
        for _ in range(steps):
            pl.step_resident(sc["x0"])
        pl.sync()
        pl.close()
    print("probe: copy calibration + %d iterations of %s done" % (steps, workload), flush=True)


def sweep():
    """Kernel time of one iteration for every lanes-per-sample shape on the
    plain, sine-lane, stress and paper-shaped workloads (HIP events)."""
    from paper_2308_01654_amd import mppi, scenes
    for sc in (scenes.c0(), scenes.c1(), scenes.c4(), scenes.paper_table1(),
               scenes.paper_merge(), scenes.paper_avoid(), scenes.paper_follow()):
        p = sc["params"]
        K, T = p["K"], p["T"]
        F = flops_per_rollout_step(len(sc["waypoints"]), len(sc["circles"]), len(p["ego_off"]))
        for lanes in (1, 2, 4, 8, 16):
            pl = mppi.Planner(p, lanes=lanes)
            pl.set_scene(sc["x0"], sc["waypoints"], sc["circles"])
            for _ in range(3):
                pl.step_resident(sc["x0"])
            pl.sync()
            n = 40 if K * T < 10**7 else 3
            ms = time_steps(pl, sc["x0"], n)
            print("%-13s K=%-7d T=%-4d lanes=%-2d kernel %.4f ms  %.3e steps/s  %.1f TFLOP/s"
                  % (sc["name"], K, T, lanes, ms, K * T / (ms * 1e-3), F * K * T / (ms * 1e-3) / 1e12),
                  flush=True)
            pl.close()


def _iteration_ms(p, x0, wp, circ, warmup, steps):
    """Average device time of one iteration (one HIP event pair around
    `steps` back-to-back steps)."""
    from paper_2308_01654_amd import mppi
    pl = mppi.Planner(p)
    pl.set_scene(x0, wp, circ)
    for _ in range(warmup):
        pl.step_resident(x0)
    pl.sync()
    ms = time_steps(pl, x0, steps)
    pl.close()
    return round(ms, 5)


def alg1_output(p, x0, wp, circ, warmup, steps):
    """The last steps of Alg. 1 on the same workload: iteration time with
    Savitzky-Golay smoothing in the combine, the latency of one
    optimal-trajectory call (device rollout + copies, host clock), and the
    iteration time with per-step (cost-to-go) weights."""
    from paper_2308_01654_amd import mppi
    ps = dict(p)
    ps["smoothing"] = 1
    smooth_ms = _iteration_ms(ps, x0, wp, circ, warmup, steps)
    pl = mppi.Planner(ps)
    pl.set_scene(x0, wp, circ)
    pl.step_resident(x0)
    pl.sync()
    lat = []
    for _ in range(50):
        a = time.perf_counter()
        pl.trajectory()
        lat.append((time.perf_counter() - a) * 1e3)
    pl.close()
    return {"smoothing_iteration_ms": smooth_ms,
            "trajectory_call_ms_p50": round(float(np.percentile(lat, 50)), 4),
            "trajectory_call_ms_p99": round(float(np.percentile(lat, 99)), 4),
            "per_step_weights_iteration_ms": _iteration_ms(dict(p, per_step=1), x0, wp, circ,
                                                           warmup, steps)}


def paper_cost_kernels(steps=50):
    """Iteration time (HIP events, tuned launch shape) of the paper's
    full-cost scenarios at the Table I shape (K=2560, T=16, dt=0.25), with
    the 4-state model and with the 5-state model of eq. (5)."""
    from paper_2308_01654_amd import mppi, scenes
    out = {}
    cases = [f() for f in (scenes.paper_merge, scenes.paper_avoid, scenes.paper_follow)]
    cases += [scenes.paper_model5(sc) for sc in list(cases)]
    for sc in cases:
        out[sc["name"] + "_iteration_ms"] = _iteration_ms(sc["params"], sc["x0"], sc["waypoints"],
                                                          sc["circles"], 5, steps)
    return out


def batched(n=256, steps=10):
    """The batched workload: n uneven sine-lane instances (K, T and circle
    counts drawn per instance) stepped together by mppi_step_batch (one
    graph replay per step, resident scenes), against the same instances
    stepped one at a time on the same stream.  Total rollout-steps/s of
    each, HIP events around `steps` warm-started steps."""
    from paper_2308_01654_amd import mppi, scenes
    insts = scenes.c2(n)
    pls = [mppi.Planner(insts[0]["params"])]
    try:
        st = pls[0].stream()
        pls += [mppi.Planner(sc["params"], hip_stream=st) for sc in insts[1:]]
        for pl, sc in zip(pls, insts):
            pl.set_scene(sc["x0"], sc["waypoints"], sc["circles"])
        x0s = [sc["x0"] for sc in insts]
        work = sum(sc["params"]["K"] * sc["params"]["T"] for sc in insts)
        ev = HipEvents()

        def timed(fn):
            for _ in range(2):
                fn()
            pls[0].sync()
            e0, e1 = ev.event(), ev.event()
            ev.record(e0, st)
            for _ in range(steps):
                fn()
            ev.record(e1, st)
            ms = ev.elapsed_ms(e0, e1) / steps
            ev.destroy(e0)
            ev.destroy(e1)
            return ms

        def alone():
            for pl, x0 in zip(pls, x0s):
                pl.step_resident(x0)

        ms_b = timed(lambda: mppi.step_batch(pls, x0s))
        ms_a = timed(alone)
    finally:
        for pl in reversed(pls):
            pl.close()
    return {"instances": n, "rollout_steps_per_batch": int(work),
            "batch_ms": round(ms_b, 4), "batch_rollout_steps_per_s": round(work / (ms_b * 1e-3), 1),
            "one_at_a_time_ms": round(ms_a, 4),
            "one_at_a_time_rollout_steps_per_s": round(work / (ms_a * 1e-3), 1)}


def c3_load(n_vehicles, duration_s, pool_size=512, seed=33):
    """Served load: vehicles with their own (K, T) and seeds replanning at
    20 Hz with exponential inter-arrival times (mean 50 ms) and a random
    phase; each request draws a scene from a pool of sine-lane windows with
    0-48 circles ahead of the vehicle."""
    from paper_2308_01654_amd import scenes
    rng = np.random.Generator(np.random.PCG64(seed))
    pool, pool_x0 = [], []
    for j in range(pool_size):
        x = float(rng.uniform(-10.0, 100.0))
        n_c = int(rng.integers(0, 49))
        pool.append((scenes.sine_lane(np.floor(x) - 20.0, np.floor(x) + 200.0, 15.0),
                     scenes.sine_circles(rng, n_c, x + 5.0, x + 120.0)))
        pool_x0.append(scenes._sine_x0(x, 15.0))
    vehicles = [scenes.c3_vehicle(v)["params"] for v in range(n_vehicles)]
    vid, sidx, arr = [], [], []
    for v in range(n_vehicles):
        t = rng.uniform(0.0, 0.05)
        while t < duration_s:
            vid.append(v)
            sidx.append(int(rng.integers(0, pool_size)))
            arr.append(int(t * 1e9))
            t += rng.exponential(0.05)
    order = np.argsort(np.asarray(arr), kind="stable")
    vid = np.asarray(vid)[order]
    sidx = np.asarray(sidx)[order]
    arr = np.asarray(arr, dtype=np.uint64)[order]
    x0 = np.asarray(pool_x0)[sidx]
    steps = np.array([vehicles[v]["K"] * vehicles[v]["T"] for v in vid], dtype=np.float64)
    return vehicles, pool, vid, x0, sidx, arr, steps


def _replay(mode, n_vehicles, duration_s, warmup_s, deadline_ms=50.0):
    """One open-loop run of the fleet load on the served (continuous
    batching) or plain (one request at a time) path; statistics over the
    requests that arrive after the first warmup_s seconds."""
    from paper_2308_01654_amd import mppi
    vehicles, pool, vid, x0, sidx, arr, steps = c3_load(n_vehicles, warmup_s + duration_s)
    srv = mppi.Server(hbm_budget_bytes=8 << 30, n_streams=3, max_batch=512,
                      plain=(mode == "plain"), deadline_ms=deadline_ms)
    try:
        vids = [srv.add_vehicle(p) for p in vehicles]
        t0 = time.perf_counter()
        lat = srv.replay([vids[v] for v in vid], x0, sidx, pool, arr)
        wall = time.perf_counter() - t0
        st = srv.stats()
    finally:
        srv.close()
    meas = arr >= np.uint64(int(warmup_s * 1e9))
    ok = np.isfinite(lat) & meas
    done = np.isfinite(lat)
    return dict(
        path=mode, vehicles=n_vehicles, requests=int(meas.sum()), warmup_s=warmup_s,
        measured_s=duration_s, offered_rps=round(int(meas.sum()) / duration_s, 1),
        completed_rps=round(int(done.sum()) / wall, 1), wall_s=round(wall, 3),
        p50=round(float(np.percentile(lat[ok], 50)), 3),
        p99=round(float(np.percentile(lat[ok], 99)), 3),
        p999=round(float(np.percentile(lat[ok], 99.9)), 3), max=round(float(lat[ok].max()), 3),
        deadline_ms=deadline_ms, deadline_misses=int(np.sum(lat[ok] > deadline_ms)),
        rollout_steps_per_s=round(float(steps[done].sum()) / wall, 1),
        mean_batch=round(st["mean_batch"], 2), hbm_peak_bytes=int(st["hbm_peak_bytes"]),
        rejected=int(st["rejected"]))


def served(n_vehicles=1000, duration_s=10.0, plain_duration_s=3.0, warmup_s=2.0):
    """p50/p99/p99.9 replan latency of the continuous-batching server and of
    the plain one-at-a-time path under the same open-loop 20 Hz fleet load
    (1000 vehicles, ~20k requests/s).  The load runs warmup_s + duration
    seconds without a break; requests arriving in the first warmup_s
    seconds (first launches of every kernel variant, arena growth) are left
    out of the statistics.  The plain path cannot keep up with this load:
    its queue grows for as long as the run lasts, and its completed rate is
    its capacity."""
    out = {}
    for mode, dur in (("served", duration_s), ("plain", plain_duration_s)):
        r = _replay(mode, n_vehicles, dur, warmup_s)
        r.pop("path")
        out[mode] = r
    return out


def serve_sweep(seconds, warmup_s=5.0, served_fleets=(1000, 2000, 4000),
                plain_fleets=(250, 500, 750, 1000)):
    """Served path at 1000, 2000 and 4000 vehicles (offered ~20k, 40k and
    80k requests/s) and the plain path at 250, 500, 750 and 1000 vehicles
    (~5k to 20k requests/s) by default: one JSON line per run."""
    for mode, fleets in (("served", served_fleets), ("plain", plain_fleets)):
        for n in fleets:
            r = _replay(mode, n, seconds, warmup_s)
            print(json.dumps(r), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per sample (0 = library choice)")
    ap.add_argument("--latency-iters", type=int, default=200)
    ap.add_argument("--probe", type=int, default=0, metavar="N",
                    help="only dispatch the counter-calibration copy and N iterations")
    ap.add_argument("--probe-workload", default="c1", choices=("c1", "c4", "c2", "paper_table1"),
                    help="workload of --probe (sine lane, stress, batched, Table I shape)")
    ap.add_argument("--sweep", action="store_true", help="only run the lanes-per-sample sweep")
    ap.add_argument("--served-seconds", type=float, default=10.0,
                    help="duration of the served load (0 skips the served comparison)")
    ap.add_argument("--plain-seconds", type=float, default=3.0)
    ap.add_argument("--serve-sweep", action="store_true",
                    help="only run the served and plain paths at several offered loads")
    ap.add_argument("--sweep-seconds", type=float, default=60.0)
    ap.add_argument("--served-fleets", default="1000,2000,4000",
                    help="vehicle counts of the served runs of --serve-sweep (20 requests/s each)")
    ap.add_argument("--plain-fleets", default="250,500,750,1000",
                    help="vehicle counts of the plain runs of --serve-sweep")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the smoothing, trajectory, per-step, paper-scenario and batched timings")
    args = ap.parse_args(argv)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the iteration runs on a single MI355X "
              "(--gpus 1); runs on several GPUs are not supported.", file=sys.stderr)
        return 2

    if args.probe:
        probe(args.probe, args.probe_workload)
        return 0
    if args.sweep:
        sweep()
        return 0
    if args.serve_sweep:
        fl = lambda v: tuple(int(x) for x in v.split(",") if x)
        serve_sweep(args.sweep_seconds, served_fleets=fl(args.served_fleets),
                    plain_fleets=fl(args.plain_fleets))
        return 0

    from paper_2308_01654_amd import mppi, scenes
    sc = scenes.c1()
    p = sc["params"]
    K, T = p["K"], p["T"]
    n_wp, n_c, n_ego = len(sc["waypoints"]), len(sc["circles"]), len(p["ego_off"])
    x0, wp, circ = sc["x0"], sc["waypoints"], sc["circles"]

    pl = mppi.Planner(p, lanes=args.lanes)
    ev = HipEvents()
    stream = pl.stream()
    pl.set_scene(x0, wp, circ)
    for _ in range(args.warmup):
        pl.step_resident(x0)
    pl.sync()

    # ---- timed region: inputs resident in HBM, one iteration per step ----
    e0, e1 = ev.event(), ev.event()
    ev.record(e0, stream)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pl.step_resident(x0)
    ev.record(e1, stream)
    pl.sync()
    t1 = time.perf_counter()
    ms = ev.elapsed_ms(e0, e1)
    ms_per_step = ms / args.steps
    value = K * T * args.steps / (ms * 1e-3)
    # ---- kernel times: the same steps again with the library's per-launch
    # HIP events on the handle's stream (kept out of the timed region: the
    # extra event records between the two kernels of a step cost host time)
    pl.set_profiling(True)
    for _ in range(args.steps):
        pl.step_resident(x0)
    prof = pl.profile()
    pl.set_profiling(False)
    st = pl.stats()

    # the dominant kernel: the iteration kernel alone (its own event pair);
    # an iteration is that kernel and the combine kernel (the timed region)
    kern_ms = prof["rollout_ms"] / max(prof["rollout_launches"], 1)
    iter_ms = ms_per_step
    F = flops_per_rollout_step(n_wp, n_c, n_ego)
    achieved = F * K * T / (kern_ms * 1e-3) / 1e12
    counters = load_counters()
    executed = None
    if counters:
        ef = counters.get("executed_fp32_flop_per_dispatch")
        pw = counters.get("per_wave", {})
        executed = dict(
            source="profiles/counters_iteration_c1.json (rocprofv3 SQ counters, one dispatch)",
            fp32_tflops=round(ef / (kern_ms * 1e-3) / 1e12, 3) if ef else None,
            fp32_frac_of_157_3=round(ef / (kern_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4) if ef else None,
            algorithmic_over_executed_flops=round(F * K * T / ef, 2) if ef else None,
            valu_instructions_per_wave=round(pw.get("SQ_INSTS_VALU", 0.0), 1),
            salu_instructions_per_wave=round(pw.get("SQ_INSTS_SALU", 0.0), 1),
            wave_quad_cycles=round(pw.get("SQ_WAVE_CYCLES", 0.0), 1),
            waiting_quad_cycles=round(pw.get("SQ_WAIT_INST_ANY", 0.0), 1))
    tr = load_trace()
    kernel_trace = None
    if tr:
        kt = tr["iteration"]["average_ns"] * 1e-9
        kernel_trace = dict(
            source="profiles/trace_iteration_c1.json (rocprofv3 --kernel-trace, %d dispatches)"
                   % tr["iteration"]["calls"],
            kernel_ms=round(kt * 1e3, 5), achieved=round(F * K * T / kt / 1e12, 3),
            frac=round(F * K * T / kt / 1e12 / PEAK_FP32_TFLOPS, 4),
            combine_ms=round(tr["combine"]["average_ns"] * 1e-6, 5))
    roofline = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP32_TFLOPS,
                    unit="TFLOP/s", frac=round(achieved / PEAK_FP32_TFLOPS, 4),
                    traffic=load_traffic(K * T), executed=executed, kernel_trace=kernel_trace,
                    achieved_counts="algorithmic flops of full scans (the kernel culls them "
                                    "exactly; executed holds what the hardware counted)",
                    kernel="k_batch<G,NE,M5> (sampling, rollouts, costs, tile partials)",
                    kernel_ms=round(kern_ms, 5), iteration_ms=round(iter_ms, 5),
                    combine_ms=round(iter_ms - kern_ms, 5), flops_per_rollout_step=F,
                    lanes_per_sample=st["lanes"])

    # ---- plain one-at-a-time replan latency (host call to controls on host) ----
    lat = []
    for _ in range(args.latency_iters):
        a = time.perf_counter()
        pl.step_resident(x0)
        pl.controls()
        lat.append((time.perf_counter() - a) * 1e3)
    lat = np.array(lat)
    # ---- host-buffer rate: scene converted and copied on every step ----
    pl.sync()
    a = time.perf_counter()
    for _ in range(50):
        pl.step(x0, wp, circ)
    pl.sync()
    pcie_value = K * T * 50 / (time.perf_counter() - a)
    pl.close()
    smooth = bat = rows = None
    if not args.no_extras:
        smooth = alg1_output(p, x0, wp, circ, args.warmup, args.steps)
        smooth.update(paper_cost_kernels())
        bat = batched()
        rows = workload_rows()

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "rollout-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sine-lane single instance, K=8192, T=100, dt=0.05, 221 waypoints, "
                               "20 obstacles x 3 circles (10 moving), 3 ego circles, warm-started",
                   "K": K, "T": T, "n_waypoints": n_wp, "n_circles": n_c},
        "roofline": roofline,
        "latency_ms": {"one_at_a_time_unloaded_p50": round(float(np.percentile(lat, 50)), 4),
                       "one_at_a_time_unloaded_p99": round(float(np.percentile(lat, 99)), 4),
                       "one_at_a_time_unloaded_p999": round(float(np.percentile(lat, 99.9)), 4)},
        "wall_s_timed": round(t1 - t0, 4),
        "host_staged_value": round(pcie_value, 1),
        "alg1_output": smooth,
        "batched": bat,
        "workloads": rows,
    }
    if args.served_seconds > 0:
        sv = served(duration_s=args.served_seconds, plain_duration_s=args.plain_seconds)
        out["latency_ms"].update({"served_p50": sv["served"]["p50"], "served_p99": sv["served"]["p99"],
                                  "served_p999": sv["served"]["p999"],
                                  "plain_p50": sv["plain"]["p50"], "plain_p99": sv["plain"]["p99"],
                                  "plain_p999": sv["plain"]["p999"]})
        out["served"] = sv
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_seconds, 358400)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
