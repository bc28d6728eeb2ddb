"""HIP events, device synchronisation and a plain device copy through the
HIP runtime that libstringfdtd itself is linked against (ctypes; used for
timing, and the copy to calibrate HBM byte counters)."""
from __future__ import annotations

import ctypes as C

from . import binding

_hip = None


def hip():
    global _hip
    if _hip is None:
        binding.load()                          # the library pulls in /opt/rocm's runtime first
        lib = C.CDLL("libamdhip64.so.7")       # ... and this resolves to that same loaded copy
        lib.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        lib.hipEventRecord.argtypes = [C.c_void_p, C.c_void_p]
        lib.hipEventSynchronize.argtypes = [C.c_void_p]
        lib.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        lib.hipEventDestroy.argtypes = [C.c_void_p]
        lib.hipDeviceSynchronize.argtypes = []
        lib.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        lib.hipFree.argtypes = [C.c_void_p]
        lib.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip = lib
    return _hip


def _ok(rc, what):
    if rc != 0:
        raise RuntimeError("%s failed with HIP error %d" % (what, rc))


class Event:
    def __init__(self):
        self.ev = C.c_void_p()
        _ok(hip().hipEventCreate(C.byref(self.ev)), "hipEventCreate")

    def record(self, stream=0):
        _ok(hip().hipEventRecord(self.ev, C.c_void_p(stream or 0)), "hipEventRecord")

    def synchronize(self):
        _ok(hip().hipEventSynchronize(self.ev), "hipEventSynchronize")

    def elapsed_ms(self, end: "Event") -> float:
        ms = C.c_float()
        _ok(hip().hipEventElapsedTime(C.byref(ms), self.ev, end.ev), "hipEventElapsedTime")
        return float(ms.value)

    def __del__(self):
        try:
            hip().hipEventDestroy(self.ev)
        except Exception:
            pass


def synchronize():
    _ok(hip().hipDeviceSynchronize(), "hipDeviceSynchronize")


def copy_probe(nbytes: int) -> None:
    """One device-to-device copy of nbytes (a reference for byte counters)."""
    h = hip()
    src, dst = C.c_void_p(), C.c_void_p()
    _ok(h.hipMalloc(C.byref(src), nbytes), "hipMalloc")
    try:
        _ok(h.hipMalloc(C.byref(dst), nbytes), "hipMalloc")
        try:
            _ok(h.hipMemcpy(dst, src, nbytes, 3), "hipMemcpy")   # hipMemcpyDeviceToDevice
            synchronize()
        finally:
            h.hipFree(dst)
    finally:
        h.hipFree(src)
