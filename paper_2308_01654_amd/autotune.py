"""Autotuner of the iteration kernel's launch shape.

For every shape bucket -- K in powers of two, T buckets (<=16, <=32, <=64,
<=128, <=256, >256) and circle-count buckets (0, <=16, <=64, <=256, >256) -- it runs
a representative sine-lane instance with every lanes-per-sample shape
(1, 2, 4, 8, 16), then, for the fastest of them, with and without the tiles'
LDS copy of their perturbations and -- at 8 or 16 lanes -- with the
iteration kernel compiled for five waves per SIMD, times whole iterations
with HIP events, and
writes the fastest choice as a line "k_log2 t_bucket c_bucket lanes stage
occupancy" of ``tuning.txt``.
The library reads that file at its first launch (next to libmppi.so, or the
file named by MPPI_TUNING_FILE).  A bucket's choice depends only on the
instance's own shape, so an instance computes the same bits alone and inside
any batch.

Usage (on the GPU): python -m paper_2308_01654_amd.autotune [--out PATH] [--quick]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

T_REPS = {0: 16, 1: 30, 2: 60, 3: 100, 4: 200, 5: 400}
C_REPS = {0: 0, 1: 12, 2: 60, 3: 200, 4: 512}
LANES = (1, 2, 4, 8, 16)


def shape_scene(K, T, n_c):
    from paper_2308_01654_amd import scenes
    rng = np.random.Generator(np.random.PCG64(K * 1000 + T * 7 + n_c))
    p = scenes.params(K=K, T=T, dt=0.05, v_max=15.0, seed=17)
    return dict(params=p, x0=scenes._sine_x0(), waypoints=scenes.sine_lane(v_ref=15.0),
                circles=scenes.sine_circles(rng, n_c))


def time_shape(sc, lanes, reps, rounds=3, stage=1, occ=0):
    """Best of `rounds` HIP-event timings of `reps` back-to-back iterations
    (the best filters out the other work of a shared GPU)."""
    from paper_2308_01654_amd import mppi
    from paper_2308_01654_amd.hip_events import time_steps
    pl = mppi.Planner(sc["params"], lanes=lanes)
    try:
        pl.set_staging(stage)
        pl.set_occupancy(occ)
        pl.set_scene(sc["x0"], sc["waypoints"], sc["circles"])
        pl.step_resident(sc["x0"])
        pl.sync()
        return min(time_steps(pl, sc["x0"], reps) for _ in range(rounds))
    finally:
        pl.close()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=os.path.join(HERE, "tuning.txt"))
    ap.add_argument("--k-min", type=int, default=10)
    ap.add_argument("--k-max", type=int, default=18)
    ap.add_argument("--t-buckets", default="0,1,2,3,4,5")
    ap.add_argument("--c-buckets", default="0,1,2,3,4")
    args = ap.parse_args(argv)
    lines = ["# launch-shape tuning table of the MPPI iteration kernel",
             "# written by: python -m paper_2308_01654_amd.autotune (HIP-event iteration time, "
             "best of 3 rounds, fastest of lanes 1/2/4/8/16, then LDS staging of the "
             "perturbations on (1) or off (0) at that shape, then at 8 or 16 lanes the "
             "compilation: default (0) or five waves per SIMD (1))",
             "# columns: k_log2 t_bucket c_bucket lanes stage occupancy   (t: <=16,<=32,<=64,"
             "<=128,<=256,>256; c: 0,<=16,<=64,<=256,>256)"]
    t0 = time.time()
    tmp = args.out + ".partial"
    with open(tmp, "w") as f:  # rows are appended as they are measured
        f.write("\n".join(lines) + "\n")
    for kb in range(args.k_min, args.k_max + 1):
        K = 1 << kb
        for tb in [int(v) for v in args.t_buckets.split(",")]:
            T = T_REPS[tb]
            for cb in [int(v) for v in args.c_buckets.split(",")]:
                sc = shape_scene(K, T, C_REPS[cb])
                reps = 20 if K * T < 2_000_000 else 3
                times = {g: time_shape(sc, g, reps) for g in LANES if g <= T}
                best = min(times, key=times.get)
                off = time_shape(sc, best, reps, stage=0)
                stage = 0 if off < times[best] else 1
                occ_t = {0: min(off, times[best])}
                if best >= 8:
                    for o in (1,):
                        occ_t[o] = time_shape(sc, best, reps, stage=stage, occ=o)
                occ = min(occ_t, key=occ_t.get)
                lines.append("%d %d %d %d %d %d" % (kb, tb, cb, best, stage, occ))
                with open(tmp, "a") as f:
                    f.write(lines[-1] + "\n")
                print("K=%-7d T=%-4d circles=%-4d " % (K, T, C_REPS[cb]) +
                      " ".join("g%d=%.4fms" % (g, ms) for g, ms in times.items()) +
                      " g%d-unstaged=%.4fms" % (best, off) +
                      "".join(" g%d-occ%d=%.4fms" % (best, o, ms) for o, ms in occ_t.items() if o) +
                      "  -> %d %d %d  (%.0fs)" % (best, stage, occ, time.time() - t0), flush=True)
    os.replace(tmp, args.out)
    print("wrote", args.out, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
