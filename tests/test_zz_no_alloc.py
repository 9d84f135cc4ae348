"""The allocation-free iteration (mppi_step_static) against mppi_step on
MI355X, through the C ABI.

The caller allocates its controls and statistics in device memory once (here
with the HIP runtime the library links); the entry point allocates nothing
and keeps its intermediates in the library's file-scope device array.  Its
results must equal, bit for bit, those of a handle stepped from the same
controls and iteration counter: same kernels, same launch shape.  Calls in a
row share the array: a large instance, then smaller ones (total-cost and
per-step weights with smoothing), then the large one again."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2308_01654_amd import scenes

pytestmark = pytest.mark.gpu

H2D, D2H = 1, 2  # hipMemcpyKind


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _libs():
    from paper_2308_01654_amd import mppi
    mppi.load()  # raises if the HIP library is not built
    hip = ctypes.CDLL("libamdhip64.so.7")  # the runtime libmppi.so is linked against
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    return mppi, hip


class _DevBuf:
    def __init__(self, hip, nbytes):
        self.hip = hip
        self.p = ctypes.c_void_p()
        assert hip.hipMalloc(ctypes.byref(self.p), nbytes) == 0
        self.nbytes = nbytes

    def put(self, arr):
        arr = np.ascontiguousarray(arr)
        assert arr.nbytes <= self.nbytes
        assert self.hip.hipMemcpy(self.p, arr.ctypes.data, arr.nbytes, H2D) == 0

    def get(self, arr):
        assert self.hip.hipMemcpy(arr.ctypes.data, self.p, arr.nbytes, D2H) == 0
        return arr

    def free(self):
        if self.p:
            self.hip.hipFree(self.p)
            self.p = ctypes.c_void_p()


def _with_handle(mppi, p, sc, U0, n_iter):
    with mppi.Planner(p) as pl:
        pl.set_state(U0, n_iter)
        pl.step(sc["x0"], sc["waypoints"], sc["circles"])
        pl.sync()
        return pl.controls(), pl.stats()


def _static(mppi, hip, p, sc, U0, n_iter, U_dev, st_dev):
    cfg = mppi.config_from_params(p)
    scene, keep = mppi.make_scene(sc["waypoints"], sc["circles"])
    U_dev.put(np.asarray(U0, dtype=np.float64))
    st = mppi.mppi_step_static(cfg, sc["x0"], scene, U_dev.p, n_iter, st_dev.p, None)
    assert st == mppi.OK, mppi.load().mppi_last_error()
    assert hip.hipDeviceSynchronize() == 0
    del keep
    U = U_dev.get(np.zeros((p["T"], 2)))
    stats = mppi.IterStats()
    assert hip.hipMemcpy(ctypes.addressof(stats), st_dev.p, ctypes.sizeof(stats), D2H) == 0
    return U, stats


def _cases():
    c1 = scenes.c1()
    tiny = scenes.tiny(K=1000, T=37, n_c=7, seed=11)
    ps = scenes.tiny(K=700, T=23, n_c=5, seed=12)
    ps = dict(ps, params=dict(ps["params"], per_step=1, smoothing=1))
    rng = np.random.Generator(np.random.PCG64(4))
    out = []
    for sc, n_iter in ((c1, 3), (tiny, 0), (ps, 7), (c1, 4)):
        T = sc["params"]["T"]
        U0 = np.column_stack([rng.normal(0.0, 0.3, T), rng.normal(0.0, 0.05, T)])
        out.append((sc, U0, n_iter))
    return out


def test_static_iteration_equals_handle_iteration():
    mppi, hip = _libs()
    T_max = max(sc["params"]["T"] for sc, _, _ in _cases())
    U_dev = _DevBuf(hip, 16 * T_max)
    st_dev = _DevBuf(hip, ctypes.sizeof(mppi.IterStats))
    try:
        for sc, U0, n_iter in _cases():
            p = sc["params"]
            _say("static vs handle", p["K"], p["T"], len(sc["circles"]),
                 "per_step" if p.get("per_step") else "total", "n_iter", n_iter)
            U_ref, st_ref = _with_handle(mppi, p, sc, U0, n_iter)
            U, st = _static(mppi, hip, p, sc, U0, n_iter, U_dev, st_dev)
            assert np.array_equal(U, U_ref), float(np.max(np.abs(U - U_ref)))
            assert not np.array_equal(U, U0)
            assert st.status == 0 and st.n_iter == n_iter + 1
            assert st.s_min == st_ref["s_min"] and st.log_z == st_ref["log_z"]
            assert st.ess == st_ref["ess"]
            assert st.lanes_per_sample == st_ref["lanes"]
    finally:
        U_dev.free()
        st_dev.free()


def test_static_iteration_rejects_oversize_and_host_pointers():
    """Nothing is enqueued for an instance beyond the array (the stress size
    needs 419 MB of perturbations) or for controls in host memory."""
    mppi, hip = _libs()
    sc = scenes.c0()
    U_dev = _DevBuf(hip, 16 * 200)
    try:
        big = dict(scenes.c0()["params"], K=262144, T=200)
        scene, keep = mppi.make_scene(sc["waypoints"], sc["circles"])
        U0 = np.full((200, 2), 0.25)
        U_dev.put(U0)
        st = mppi.mppi_step_static(mppi.config_from_params(big), sc["x0"], scene, U_dev.p, 0,
                                   None, None)
        assert st == mppi.E_INVALID
        assert b"scratch" in mppi.load().mppi_last_error()
        assert np.array_equal(U_dev.get(np.zeros((200, 2))), U0)
        host_U = np.zeros((sc["params"]["T"], 2))
        st = mppi.mppi_step_static(mppi.config_from_params(sc["params"]), sc["x0"], scene,
                                   host_U.ctypes.data, 0, None, None)
        assert st == mppi.E_INVALID
        del keep
    finally:
        U_dev.free()
