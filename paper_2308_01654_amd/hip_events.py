"""HIP event timing on a given stream, through the HIP runtime that the
library itself links (found in this process's memory map).  Used to time
runs of iterations as a whole (one event pair around many steps), which
unlike per-launch events adds nothing between the kernels of a step."""
import ctypes


class HipEvents:
    """hipEvent timing on a given stream through the HIP runtime the library
    itself links (found in this process's memory map)."""

    def __init__(self):
        paths = [l.split()[-1] for l in open("/proc/self/maps") if "libamdhip64" in l]
        if not paths:
            raise RuntimeError("HIP runtime not loaded")
        H = ctypes.CDLL(paths[0])
        vp = ctypes.c_void_p
        H.hipEventCreate.argtypes = [ctypes.POINTER(vp)]
        H.hipEventRecord.argtypes = [vp, vp]
        H.hipEventSynchronize.argtypes = [vp]
        H.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), vp, vp]
        H.hipEventDestroy.argtypes = [vp]
        self.H = H

    def event(self):
        e = ctypes.c_void_p()
        assert self.H.hipEventCreate(ctypes.byref(e)) == 0
        return e

    def record(self, e, stream):
        assert self.H.hipEventRecord(e, ctypes.c_void_p(stream)) == 0

    def elapsed_ms(self, a, b):
        assert self.H.hipEventSynchronize(b) == 0
        ms = ctypes.c_float()
        assert self.H.hipEventElapsedTime(ctypes.byref(ms), a, b) == 0
        return float(ms.value)

    def destroy(self, e):
        self.H.hipEventDestroy(e)


def time_steps(planner, x0, n):
    """Average device time of one iteration over n back-to-back
    single-instance steps on resident inputs (ms)."""
    ev = HipEvents()
    st = planner.stream()
    e0, e1 = ev.event(), ev.event()
    ev.record(e0, st)
    for _ in range(n):
        planner.step_resident(x0)
    ev.record(e1, st)
    ms = ev.elapsed_ms(e0, e1) / n
    ev.destroy(e0)
    ev.destroy(e1)
    return ms
