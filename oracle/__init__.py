"""TEST INFRASTRUCTURE ONLY: the CPU oracle for the single-pulse search hot path.

Only ``tests/``, the smoke entry point and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it.

The arithmetic lives in ``amber_oracle.c`` (plain C, FP64 where floating point
is involved); this module compiles it with gcc on first use and wraps it with
numpy in / numpy out functions:

* ``delay_table``  -- dispersion delay per (DM trial, channel) (Section 1:
  dedispersion as shift-and-sum of channels; textbook cold-plasma delay).
* ``dedisperse``   -- brute-force one-step dedispersion (Section 5 names the
  one-step scheme; Section 2 the dedispersion kernel).
* ``dedisperse_masked`` -- the same with zapped (RFI) channels excluded.
* ``subband_delays``, ``subband_dedisperse`` -- the two-step subband scheme
  (Section 2 footnote, Table 2).
* ``boxcar``       -- sliding boxcar "smoothing" of each series (Section 2).
* ``downsample``   -- decimating downsampling by a factor (Section 2, Table 2).
* ``snr``          -- (max - mean) / population std per series (Section 2's
  S/N kernel; the paper prints no formula).
* ``search``       -- the four steps in order, for every width.
* ``best_candidate`` -- argmax over (DM, width) of the S/N table.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "amber_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


# No -march: the library may be built on one host and run on another.
BUILD_FLAGS = ["-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile amber_oracle.c into liboracle.so (gcc with BUILD_FLAGS)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc"] + BUILD_FLAGS + ["-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            i32p = ctypes.POINTER(ctypes.c_int32)
            i64p = ctypes.POINTER(ctypes.c_int64)
            f64p = ctypes.POINTER(ctypes.c_double)
            u8p = ctypes.POINTER(ctypes.c_uint8)
            lib.oracle_delay_table.argtypes = [ctypes.c_int, f64p, ctypes.c_double, ctypes.c_int,
                                               ctypes.c_double, ctypes.c_double, i32p, i32p]
            lib.oracle_dedisperse.argtypes = [i32p, ctypes.c_int, ctypes.c_int, u8p, ctypes.c_int64,
                                              ctypes.c_int64, ctypes.c_int64, i32p, ctypes.c_int]
            lib.oracle_dedisperse_masked.argtypes = [i32p, ctypes.c_int, ctypes.c_int, u8p, ctypes.c_int64,
                                                     ctypes.c_int64, ctypes.c_int64, u8p, i32p, ctypes.c_int]
            lib.oracle_subband_delays.argtypes = [ctypes.c_int, f64p, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                                  ctypes.c_double, i32p, i32p, i32p, i32p]
            lib.oracle_subband_dedisperse.argtypes = [i32p, i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                      ctypes.c_int, u8p, ctypes.c_int64, ctypes.c_int64,
                                                      ctypes.c_int64, i32p, ctypes.c_int]
            lib.oracle_boxcar.argtypes = [i32p, ctypes.c_int, ctypes.c_int64, ctypes.c_int, i64p,
                                          ctypes.c_int]
            lib.oracle_downsample.argtypes = [i32p, ctypes.c_int, ctypes.c_int64, ctypes.c_int, i64p,
                                              ctypes.c_int]
            lib.oracle_snr.argtypes = [i64p, ctypes.c_int, ctypes.c_int64, f64p, i32p, ctypes.c_int]
            for f in (lib.oracle_delay_table, lib.oracle_dedisperse, lib.oracle_dedisperse_masked,
                      lib.oracle_subband_delays, lib.oracle_subband_dedisperse, lib.oracle_boxcar,
                      lib.oracle_downsample,
                      lib.oracle_snr):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def delay_table(freq_mhz, t_samp_s: float, n_dm: int, dm_first: float, dm_step: float):
    """Return (delays int32 [n_dm, n_chan], max_delay)."""
    f = np.ascontiguousarray(freq_mhz, dtype=np.float64)
    out = np.empty((n_dm, f.size), dtype=np.int32)
    mx = ctypes.c_int32(0)
    rc = _load().oracle_delay_table(f.size, _ptr(f, ctypes.c_double), float(t_samp_s), int(n_dm),
                                    float(dm_first), float(dm_step), _ptr(out, ctypes.c_int32),
                                    ctypes.byref(mx))
    if rc != 0:
        raise ValueError("oracle_delay_table rejected its arguments")
    return out, int(mx.value)


def dedisperse(delays: np.ndarray, x: np.ndarray, n_in: int, n_out: int, threads: int = 0) -> np.ndarray:
    """dd[i][t] = sum_c x[c][t + delays[i][c]] for t < n_out.  x is uint8 [n_chan, stride]."""
    d = np.ascontiguousarray(delays, dtype=np.int32)
    xa = np.ascontiguousarray(x, dtype=np.uint8)
    n_dm, n_chan = d.shape
    if xa.shape[0] != n_chan:
        raise ValueError("channel count of x and delays differ")
    out = np.empty((n_dm, n_out), dtype=np.int32)
    rc = _load().oracle_dedisperse(_ptr(d, ctypes.c_int32), n_dm, n_chan, _ptr(xa, ctypes.c_uint8),
                                   xa.shape[1], int(n_in), int(n_out), _ptr(out, ctypes.c_int32),
                                   int(threads))
    if rc != 0:
        raise ValueError("oracle_dedisperse: a delay reads outside [0, n_in)")
    return out


def dedisperse_masked(delays: np.ndarray, x: np.ndarray, n_in: int, n_out: int, keep, threads: int = 0) -> np.ndarray:
    """dd[i][t] = sum over channels with keep[c] != 0 of x[c][t + delays[i][c]] (zapped channels excluded)."""
    d = np.ascontiguousarray(delays, dtype=np.int32)
    xa = np.ascontiguousarray(x, dtype=np.uint8)
    k = np.ascontiguousarray(keep, dtype=np.uint8)
    n_dm, n_chan = d.shape
    if xa.shape[0] != n_chan or k.shape != (n_chan,):
        raise ValueError("channel count of x, delays and keep differ")
    out = np.empty((n_dm, n_out), dtype=np.int32)
    rc = _load().oracle_dedisperse_masked(_ptr(d, ctypes.c_int32), n_dm, n_chan, _ptr(xa, ctypes.c_uint8),
                                          xa.shape[1], int(n_in), int(n_out), _ptr(k, ctypes.c_uint8),
                                          _ptr(out, ctypes.c_int32), int(threads))
    if rc != 0:
        raise ValueError("oracle_dedisperse_masked: a delay reads outside [0, n_in)")
    return out


def subband_delays(freq_mhz, t_samp_s: float, n_sub: int, n_coarse: int, coarse_first: float, coarse_step: float,
                   n_fine: int, fine_first: float, fine_step: float):
    """Two-step subband delay tables: (delay1 int32 [n_sub, n_coarse, n_chan / n_sub] (within each subband,
    at the coarse DM), delay2 int32 [n_coarse, n_fine, n_sub] (subband references at the trial DM), max1, max2)."""
    f = np.ascontiguousarray(freq_mhz, dtype=np.float64)
    n_chan = f.shape[0]
    if n_sub < 1 or n_chan % n_sub:
        raise ValueError("n_sub must divide n_chan")
    d1 = np.empty((n_sub, n_coarse, n_chan // n_sub), dtype=np.int32)
    d2 = np.empty((n_coarse, n_fine, n_sub), dtype=np.int32)
    m1, m2 = ctypes.c_int32(), ctypes.c_int32()
    rc = _load().oracle_subband_delays(n_chan, _ptr(f, ctypes.c_double), float(t_samp_s), int(n_sub), int(n_coarse),
                                       float(coarse_first), float(coarse_step), int(n_fine), float(fine_first),
                                       float(fine_step), _ptr(d1, ctypes.c_int32), _ptr(d2, ctypes.c_int32),
                                       ctypes.byref(m1), ctypes.byref(m2))
    if rc != 0:
        raise ValueError("oracle_subband_delays: bad arguments")
    return d1, d2, m1.value, m2.value


def subband_dedisperse(delay1: np.ndarray, delay2: np.ndarray, x: np.ndarray, n_in: int, n_out: int,
                       threads: int = 0) -> np.ndarray:
    """dd[j n_fine + k][t] = sum over subbands s and their channels c of x[c][t + delay2[j,k,s] + delay1[s,j,c']]."""
    d1 = np.ascontiguousarray(delay1, dtype=np.int32)
    d2 = np.ascontiguousarray(delay2, dtype=np.int32)
    xa = np.ascontiguousarray(x, dtype=np.uint8)
    n_sub, n_coarse, m = d1.shape
    n_fine = d2.shape[1]
    if d2.shape != (n_coarse, n_fine, n_sub) or xa.shape[0] != n_sub * m:
        raise ValueError("inconsistent subband tables and input")
    out = np.empty((n_coarse * n_fine, n_out), dtype=np.int32)
    rc = _load().oracle_subband_dedisperse(_ptr(d1, ctypes.c_int32), _ptr(d2, ctypes.c_int32), n_sub * m, n_sub,
                                           n_coarse, n_fine, _ptr(xa, ctypes.c_uint8), xa.shape[1], int(n_in),
                                           int(n_out), _ptr(out, ctypes.c_int32), int(threads))
    if rc != 0:
        raise ValueError("oracle_subband_dedisperse: a delay reads outside [0, n_in)")
    return out


def boxcar(dd: np.ndarray, w: int, threads: int = 0) -> np.ndarray:
    """box[i][t] = sum_{k<w} dd[i][t+k] for t < n_out - w + 1 (int64)."""
    a = np.ascontiguousarray(dd, dtype=np.int32)
    n_dm, n_out = a.shape
    out = np.empty((n_dm, n_out - w + 1), dtype=np.int64)
    rc = _load().oracle_boxcar(_ptr(a, ctypes.c_int32), n_dm, n_out, int(w), _ptr(out, ctypes.c_int64),
                               int(threads))
    if rc != 0:
        raise ValueError("oracle_boxcar: width outside [1, n_out]")
    return out


def downsample(dd: np.ndarray, f: int, threads: int = 0) -> np.ndarray:
    """y[i][j] = sum_{k<f} dd[i][j*f + k] for j < n_out // f (int64): decimation by f."""
    a = np.ascontiguousarray(dd, dtype=np.int32)
    n_dm, n_out = a.shape
    out = np.empty((n_dm, n_out // int(f) if f >= 1 else 0), dtype=np.int64)
    rc = _load().oracle_downsample(_ptr(a, ctypes.c_int32), n_dm, n_out, int(f), _ptr(out, ctypes.c_int64),
                                   int(threads))
    if rc != 0:
        raise ValueError("oracle_downsample: factor outside [1, n_out]")
    return out


def snr(x: np.ndarray, threads: int = 0):
    """Per row: ((max - mean) / population std, first argmax).  Returns (float64, int32)."""
    a = np.ascontiguousarray(x, dtype=np.int64)
    if a.ndim == 1:
        a = a[None, :]
    n_rows, n = a.shape
    s = np.empty(n_rows, dtype=np.float64)
    p = np.empty(n_rows, dtype=np.int32)
    rc = _load().oracle_snr(_ptr(a, ctypes.c_int64), n_rows, n, _ptr(s, ctypes.c_double),
                            _ptr(p, ctypes.c_int32), int(threads))
    if rc != 0:
        raise ValueError("oracle_snr: empty series")
    return s, p


def search(delays: np.ndarray, x: np.ndarray, n_in: int, n_out: int, widths, threads: int = 0):
    """The hot path in order: dedisperse, then boxcar + S/N for every width.

    Returns (dd int32 [n_dm, n_out], snr float64 [n_w, n_dm], peak int32 [n_w, n_dm]).
    """
    dd = dedisperse(delays, x, n_in, n_out, threads)
    n_dm = dd.shape[0]
    s = np.empty((len(widths), n_dm), dtype=np.float64)
    p = np.empty((len(widths), n_dm), dtype=np.int32)
    for k, w in enumerate(widths):
        s[k], p[k] = snr(boxcar(dd, w, threads), threads)
    return dd, s, p


def best_candidate(snr_table: np.ndarray):
    """Argmax over (width index, DM index) of an S/N table [n_w, n_dm].

    Ties go to the smallest DM index, then the smallest width index.
    Returns (dm_index, width_index, snr).
    """
    s = np.asarray(snr_table)
    best = None
    for i in range(s.shape[1]):
        for k in range(s.shape[0]):
            v = s[k, i]
            if best is None or v > best[2]:
                best = (i, k, v)
    return best
