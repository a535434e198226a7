"""Minimal ctypes access to HIP events (for stage timing with the library's
profiling hook; torch events do not expose their raw handle)."""
from __future__ import annotations

import ctypes
import ctypes.util

_hip = None


def hip():
    global _hip
    if _hip is None:
        for name in ("libamdhip64.so", "libamdhip64.so.7", "/opt/rocm/lib/libamdhip64.so"):
            try:
                _hip = ctypes.CDLL(name)
                break
            except OSError:
                continue
        if _hip is None:
            raise RuntimeError("libamdhip64 not found")
        _hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        _hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        _hip.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        _hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        _hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        _hip.hipGetLastError.restype = ctypes.c_int
    return _hip


class Event:
    def __init__(self):
        h = ctypes.c_void_p()
        if hip().hipEventCreate(ctypes.byref(h)) != 0:
            raise RuntimeError("hipEventCreate failed")
        self.handle = h.value

    def record(self, stream: int) -> None:
        if hip().hipEventRecord(ctypes.c_void_p(self.handle), ctypes.c_void_p(stream)) != 0:
            raise RuntimeError("hipEventRecord failed")

    def synchronize(self) -> None:
        hip().hipEventSynchronize(ctypes.c_void_p(self.handle))

    def elapsed_ms(self, later: "Event") -> float:
        ms = ctypes.c_float(0.0)
        if hip().hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(self.handle), ctypes.c_void_p(later.handle)) != 0:
            # e.g. an event that was never recorded; clear the runtime's last
            # error so that the next HIP call (torch's included) does not report it
            hip().hipGetLastError()
            raise RuntimeError("hipEventElapsedTime failed")
        return float(ms.value)

    def __del__(self):
        try:
            if self.handle:
                hip().hipEventDestroy(ctypes.c_void_p(self.handle))
        except Exception:
            pass
