"""ctypes declarations of libamber.so (the C ABI in include/amber.h)."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libamber.so")

AMBER_MAX_WIDTHS = 16

c_i32p = ctypes.POINTER(ctypes.c_int32)
c_f64p = ctypes.POINTER(ctypes.c_double)


class Geometry(ctypes.Structure):
    _fields_ = [("n_chan", ctypes.c_int32), ("freq_mhz", c_f64p), ("t_samp_s", ctypes.c_double),
                ("n_dm", ctypes.c_int32), ("dm_first", ctypes.c_double), ("dm_step", ctypes.c_double)]


class DelayInfo(ctypes.Structure):
    _fields_ = [("n_dm", ctypes.c_int32), ("n_chan", ctypes.c_int32), ("max_delay", ctypes.c_int32),
                ("max_step", ctypes.c_int32)]

    def __repr__(self):
        return "DelayInfo(n_dm=%d, n_chan=%d, max_delay=%d, max_step=%d)" % (
            self.n_dm, self.n_chan, self.max_delay, self.max_step)


class Tiles(ctypes.Structure):
    _fields_ = [("threads_per_dm", ctypes.c_int32), ("samples_per_thread", ctypes.c_int32),
                ("dms_per_block", ctypes.c_int32), ("channel_unroll", ctypes.c_int32),
                ("snr_threads", ctypes.c_int32), ("boxcar_step", ctypes.c_int32 * AMBER_MAX_WIDTHS)]

    def as_dict(self):
        return {"threads_per_dm": self.threads_per_dm, "samples_per_thread": self.samples_per_thread,
                "dms_per_block": self.dms_per_block, "channel_unroll": self.channel_unroll,
                "snr_threads": self.snr_threads, "boxcar_step": list(self.boxcar_step)}

    def __repr__(self):
        d = self.as_dict()
        d["boxcar_step"] = d["boxcar_step"][:8]
        return "Tiles(%s)" % ", ".join("%s=%s" % kv for kv in d.items())


# (name, restype, argtypes) of every exported symbol the header declares.
SIGNATURES = [
    ("amber_last_error", ctypes.c_char_p, []),
    ("amber_version", ctypes.c_char_p, []),
    ("amber_default_tiles", ctypes.c_int, [ctypes.POINTER(Tiles)]),
    ("amber_auto_tiles", ctypes.c_int, [ctypes.POINTER(DelayInfo), ctypes.POINTER(Tiles)]),
    ("amber_validate_tiles", ctypes.c_int, [ctypes.POINTER(Tiles), ctypes.POINTER(DelayInfo), ctypes.c_int32]),
    ("amber_delay_table", ctypes.c_int, [ctypes.POINTER(Geometry), c_i32p, ctypes.POINTER(DelayInfo)]),
    ("amber_dedisperse", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(DelayInfo), ctypes.c_void_p,
                                        ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.POINTER(Tiles), ctypes.c_void_p]),
    ("amber_integrate", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                       c_i32p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.POINTER(Tiles), ctypes.c_void_p]),
    ("amber_snr", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, c_i32p,
                                 ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Tiles),
                                 ctypes.c_void_p]),
    ("amber_integrate_snr", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                           c_i32p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.POINTER(Tiles), ctypes.c_void_p]),
]

_lib = None


class AmberError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("amber status %d: %s" % (status, message))
        self.status = status


def load():
    """Load libamber.so from the package directory; raise if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libamber.so is not built (run __graft_entry__.build() or "
                              "python paper_1811_04165_amd/build.py)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def check(status: int) -> None:
    if status != 0:
        msg = load().amber_last_error().decode()
        raise AmberError(status, msg)
