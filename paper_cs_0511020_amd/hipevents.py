"""HIP events through the HIP runtime (ctypes), for timing work queued by
libpbit on a given stream."""
from __future__ import annotations

import ctypes
import ctypes.util

_hip = None


def hip():
    global _hip
    if _hip is None:
        for name in ("libamdhip64.so", "/opt/rocm/lib/libamdhip64.so"):
            try:
                _hip = ctypes.CDLL(name)
                break
            except OSError:
                continue
        if _hip is None:
            raise RuntimeError("libamdhip64.so not found")
        _hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        _hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        _hip.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        _hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        _hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                             ctypes.c_void_p]
    return _hip


class EventPool:
    """A fixed array of hipEvent_t handles usable as ``void**``."""

    def __init__(self, count: int):
        self.count = count
        self.handles = (ctypes.c_void_p * count)()
        h = hip()
        for i in range(count):
            ev = ctypes.c_void_p()
            if h.hipEventCreate(ctypes.byref(ev)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.handles[i] = ev
        self.ids = (ctypes.c_int32 * count)()

    def ptr(self):
        return ctypes.cast(self.handles, ctypes.c_void_p)

    def ids_ptr(self):
        return ctypes.cast(self.ids, ctypes.c_void_p)

    def record(self, i: int, stream_handle: int):
        hip().hipEventRecord(self.handles[i], ctypes.c_void_p(stream_handle))

    def elapsed_ms(self, i: int, j: int) -> float:
        out = ctypes.c_float()
        h = hip()
        h.hipEventSynchronize(self.handles[j])
        if h.hipEventElapsedTime(ctypes.byref(out), self.handles[i], self.handles[j]) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(out.value)

    def close(self):
        h = hip()
        for i in range(self.count):
            if self.handles[i]:
                h.hipEventDestroy(self.handles[i])
                self.handles[i] = None
