"""MI355X (gfx950) single-pulse search hot path: Python binding of libamber.so.

Argument marshalling only: every step runs in the library's HIP kernels (or,
for the delay table, in its FP64 host code).  Device buffers are torch CUDA
(HIP) tensors passed by pointer; work is enqueued on the current torch stream
unless a stream is given.  Importing this package without a built
libamber.so raises ImportError: there is no fallback path.

Steps (see include/amber.h for the exact contracts):
    delay_table    -> (int32 [n_dm, n_chan] host array, DelayInfo)
    dedisperse     -> int32 [n_dm, n_out]      dd[i][t] = sum_c x[c][t + delay[i][c]]
    integrate      -> int32 [n_w, n_dm, n_out] sliding boxcars (valid prefix per width)
    snr            -> (float32 [n_w, n_dm], int32 [n_w, n_dm]) from boxcar series
    integrate_snr  -> the previous two fused
    downsample     -> int32 [n_f, n_dm, n_out // f] decimated sums of f samples
    downsample_snr -> S/N of each decimated series, fused
    Batch          -> beams of uneven sizes in shared launches / one HIP graph
    Server         -> streaming chunks with continuous batching
"""
from __future__ import annotations

import atexit
import ctypes
import sys
import weakref
from typing import Optional, Sequence

import numpy as np

from ._lib import (AMBER_E_TIMEOUT, AMBER_MAX_WIDTHS, FITNESS_FN, Beam, ChunkResult, PendingChunk, SEARCH_KINDS,
                   SUBBAND_FITNESS_FN, AmberError, DelayInfo, Geometry, ServerConfig, ServerStats, StreamBeam,
                   SubbandGeometry, SubbandInfo, SubbandTuneResult, SubbandTuneSpace, Tiles, TuneParams, TuneResult,
                   TuneSpace, check, load)

__all__ = ["AmberError", "DelayInfo", "Tiles", "TuneSpace", "TuneParams", "TuneResult", "default_space",
           "space_size", "tune_params", "search_tiles", "tune", "Batch", "default_tiles", "make_tiles", "delay_table", "dedisperse",
           "integrate", "snr", "integrate_snr", "downsample", "downsample_snr", "validate_tiles", "auto_tiles", "version", "Search", "Server",
           "chunk_span", "admit", "server_config", "server_clock", "SubbandInfo", "subband_delay_tables",
           "subband_dedisperse", "subband_dedisperse_noalloc", "subband_static_bytes", "genes", "default_subband_space",
           "subband_space_size", "search_subband_tiles", "tune_subband"]

load()  # fail loudly at import if the native library is missing

# gene indices of a tune space (the dedispersion kernel's genes, then the
# boxcar / S/N kernel's): genes.GENE_SNR_THREADS, ...
from . import _lib as _l  # noqa: E402
import types as _types  # noqa: E402
genes = _types.SimpleNamespace(**{k: getattr(_l, k) for k in dir(_l) if k.startswith(("GENE_", "SB_GENE"))},
                               AMBER_GENES_K1=_l.AMBER_GENES_K1)


def version() -> str:
    return load().amber_version().decode()


def default_tiles() -> Tiles:
    t = Tiles()
    check(load().amber_default_tiles(ctypes.byref(t)))
    return t


def make_tiles(threads_per_dm=None, samples_per_thread=None, dms_per_block=None, channel_unroll=None,
               snr_threads=None, boxcar_step=None, dms_per_thread=None, direct_reads=None) -> Tiles:
    """Default tiles with the given fields replaced; boxcar_step is an int or a per-width list."""
    t = default_tiles()
    for name, v in (("threads_per_dm", threads_per_dm), ("samples_per_thread", samples_per_thread),
                    ("dms_per_block", dms_per_block), ("channel_unroll", channel_unroll),
                    ("snr_threads", snr_threads), ("dms_per_thread", dms_per_thread),
                    ("direct_reads", direct_reads)):
        if v is not None:
            setattr(t, name, int(v))
    if boxcar_step is not None:
        steps = [boxcar_step] * AMBER_MAX_WIDTHS if np.isscalar(boxcar_step) else list(boxcar_step)
        for k in range(AMBER_MAX_WIDTHS):
            t.boxcar_step[k] = int(steps[k] if k < len(steps) else steps[-1])
    return t


def auto_tiles(info: DelayInfo, n_out: int = 0) -> Tiles:
    """The default tiles adapted to this delay table and, when n_out > 0, made
    smaller until the dedispersion grid fills the chip (what tiles=None uses)."""
    t = Tiles()
    check(load().amber_auto_tiles(ctypes.byref(info), int(n_out), ctypes.byref(t)))
    return t


def validate_tiles(tiles: Tiles, info: DelayInfo, n_widths: int) -> None:
    check(load().amber_validate_tiles(ctypes.byref(tiles), ctypes.byref(info), int(n_widths)))


def delay_table(freq_mhz, t_samp_s: float, n_dm: int, dm_first: float, dm_step: float):
    """FP64 host delay table.  Returns (int32 [n_dm, n_chan], DelayInfo)."""
    f = np.ascontiguousarray(freq_mhz, dtype=np.float64)
    g = Geometry(n_chan=f.size, freq_mhz=f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                 t_samp_s=float(t_samp_s), n_dm=int(n_dm), dm_first=float(dm_first), dm_step=float(dm_step))
    out = np.empty((int(n_dm), f.size), dtype=np.int32)
    info = DelayInfo()
    check(load().amber_delay_table(ctypes.byref(g), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   ctypes.byref(info)))
    return out, info


# --- device steps -------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _stream_handle(stream) -> ctypes.c_void_p:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_dev(t, dtype, name: str, ndim: int):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if t.dim() != ndim or t.stride(-1) != 1:
        raise ValueError("%s must be %d-D with unit stride along its last dimension" % (name, ndim))


def _check_table(t, dtype, name: str, n_w: int, n_dm: int, device):
    """An output table [n_w, n_dm]: contiguous, on `device`."""
    _check_dev(t, dtype, name, 2)
    if tuple(t.shape) != (n_w, n_dm) or not t.is_contiguous():
        raise ValueError("%s must be a contiguous [%d, %d] tensor" % (name, n_w, n_dm))
    if t.device != device:
        raise ValueError("%s must be on %s" % (name, device))


def _table_out(out, n_w: int, n_dm: int, device):
    """(snr float32, peak int32) output tables, allocated or checked."""
    torch = _torch()
    if out is None:
        return (torch.empty((n_w, n_dm), dtype=torch.float32, device=device),
                torch.empty((n_w, n_dm), dtype=torch.int32, device=device))
    s, p = out
    _check_table(s, torch.float32, "snr out", n_w, n_dm, device)
    _check_table(p, torch.int32, "peak out", n_w, n_dm, device)
    return s, p


def _tiles_ref(tiles: Optional[Tiles]):
    return ctypes.byref(tiles) if tiles is not None else None


def dedisperse(delays, info: DelayInfo, x, n_in: int, n_out: int, tiles: Optional[Tiles] = None, out=None,
               stream=None, keep=None):
    """delays: int32 CUDA [n_dm, n_chan]; x: uint8 CUDA [n_chan, stride].  Returns int32 [n_dm, n_out].
    keep: optional uint8 CUDA [n_chan], 0 = zapped channel (excluded from the sums)."""
    torch = _torch()
    _check_dev(delays, torch.int32, "delays", 2)
    _check_dev(x, torch.uint8, "x", 2)
    if not delays.is_contiguous() or tuple(delays.shape) != (info.n_dm, info.n_chan):
        raise ValueError("delays must be contiguous [n_dm, n_chan] matching info")
    if x.shape[0] != info.n_chan or x.shape[1] < n_in:
        raise ValueError("x must be [n_chan, >= n_in]")
    if out is None:
        out = torch.empty((info.n_dm, n_out), dtype=torch.int32, device=x.device)
    _check_dev(out, torch.int32, "out", 2)
    if out.shape[0] != info.n_dm or out.shape[1] < n_out:
        raise ValueError("out must be [n_dm, >= n_out]")
    if delays.device != x.device or out.device != x.device:
        raise ValueError("delays, x and out must be on one device")
    if keep is not None:
        _check_dev(keep, torch.uint8, "keep", 1)
        if keep.shape[0] != info.n_chan or not keep.is_contiguous():
            raise ValueError("keep must be a contiguous uint8 [n_chan] tensor")
        check(load().amber_dedisperse_masked(delays.data_ptr(), ctypes.byref(info), x.data_ptr(), x.stride(0),
                                             int(n_in), out.data_ptr(), out.stride(0), int(n_out), keep.data_ptr(),
                                             _tiles_ref(tiles), _stream_handle(stream)))
        return out
    check(load().amber_dedisperse(delays.data_ptr(), ctypes.byref(info), x.data_ptr(), x.stride(0), int(n_in),
                                  out.data_ptr(), out.stride(0), int(n_out), _tiles_ref(tiles),
                                  _stream_handle(stream)))
    return out


def subband_delay_tables(freq_mhz, t_samp_s: float, n_subbands: int, n_coarse: int, coarse_first: float,
                         coarse_step: float, n_fine: int, fine_first: float, fine_step: float):
    """FP64 host tables of the two-step subband scheme, with each coarse DM's k = 0 step-two shift
    moved into step one.  Returns (delay1 int32 [n_sub, n_coarse, m], delay2 int32 [n_coarse, n_fine, n_sub],
    SubbandInfo)."""
    f = np.ascontiguousarray(freq_mhz, dtype=np.float64)
    g = SubbandGeometry(n_chan=f.size, freq_mhz=f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        t_samp_s=float(t_samp_s), n_subbands=int(n_subbands), n_coarse=int(n_coarse),
                        coarse_first=float(coarse_first), coarse_step=float(coarse_step), n_fine=int(n_fine),
                        fine_first=float(fine_first), fine_step=float(fine_step))
    m = f.size // max(int(n_subbands), 1)
    d1 = np.empty((max(int(n_subbands), 0), max(int(n_coarse), 0), m), dtype=np.int32)
    d2 = np.empty((max(int(n_coarse), 0), max(int(n_fine), 0), max(int(n_subbands), 0)), dtype=np.int32)
    info = SubbandInfo()
    i32 = ctypes.POINTER(ctypes.c_int32)
    check(load().amber_subband_delay_tables(ctypes.byref(g), d1.ctypes.data_as(i32), d2.ctypes.data_as(i32),
                                            ctypes.byref(info)))
    return d1, d2, info


def subband_dedisperse(delay1, delay2, info: SubbandInfo, x, n_in: int, n_out: int, tiles1: Optional[Tiles] = None,
                       tiles2: Optional[Tiles] = None, out=None, work=None, keep=None, stream=None):
    """Two-step subband dedispersion.  delay1/delay2: int32 CUDA tables from subband_delay_tables; x: uint8 CUDA
    [n_chan, stride].  work: optional uint16 CUDA [n_sub * n_coarse, >= n_out + max_delay2] (even row stride) for
    step one's sums.  Returns int32 [n_coarse * n_fine, n_out] (trial j * n_fine + k)."""
    torch = _torch()
    _check_dev(delay1, torch.int32, "delay1", 3)
    _check_dev(delay2, torch.int32, "delay2", 3)
    _check_dev(x, torch.uint8, "x", 2)
    n_sub, nc, nf = info.n_subbands, info.n_coarse, info.n_fine
    if n_sub < 1 or info.n_chan % n_sub:
        raise ValueError("info has an invalid subband count")
    m = info.n_chan // n_sub
    if not delay1.is_contiguous() or tuple(delay1.shape) != (n_sub, nc, m):
        raise ValueError("delay1 must be contiguous [n_sub, n_coarse, n_chan / n_sub]")
    if not delay2.is_contiguous() or tuple(delay2.shape) != (nc, nf, n_sub):
        raise ValueError("delay2 must be contiguous [n_coarse, n_fine, n_sub]")
    if x.shape[0] != info.n_chan or x.shape[1] < n_in:
        raise ValueError("x must be [n_chan, >= n_in]")
    n1 = int(n_out) + info.max_delay2
    if work is None:
        work = torch.empty((n_sub * nc, (n1 + 63) // 64 * 64), dtype=torch.uint16, device=x.device)
    _check_dev(work, torch.uint16, "work", 2)
    if work.shape[0] != n_sub * nc or work.shape[1] < n1 or work.stride(0) % 2:
        raise ValueError("work must be uint16 [n_sub * n_coarse, >= n_out + max_delay2] with an even row stride")
    if out is None:
        out = torch.empty((nc * nf, n_out), dtype=torch.int32, device=x.device)
    _check_dev(out, torch.int32, "out", 2)
    if out.shape[0] != nc * nf or out.shape[1] < n_out:
        raise ValueError("out must be [n_coarse * n_fine, >= n_out]")
    kp = None
    if keep is not None:
        _check_dev(keep, torch.uint8, "keep", 1)
        if keep.shape[0] != info.n_chan or not keep.is_contiguous():
            raise ValueError("keep must be a contiguous uint8 [n_chan] tensor")
        kp = keep.data_ptr()
    check(load().amber_subband_dedisperse(delay1.data_ptr(), delay2.data_ptr(), ctypes.byref(info), x.data_ptr(),
                                          x.stride(0), int(n_in), work.data_ptr(), work.stride(0), out.data_ptr(),
                                          out.stride(0), int(n_out), kp, _tiles_ref(tiles1), _tiles_ref(tiles2),
                                          _stream_handle(stream)))
    return out


def subband_dedisperse_noalloc(delay1, delay2, info: SubbandInfo, x, n_in: int, n_out: int,
                               tiles1: Optional[Tiles] = None, tiles2: Optional[Tiles] = None, out=None, keep=None,
                               stream=None):
    """subband_dedisperse without a work buffer: step one's sums go to the library's own device array
    (subband_static_bytes(); no allocation by the library).  `out` may be given to keep the call free of any
    allocation on the Python side too.  Returns int32 [n_coarse * n_fine, n_out]."""
    torch = _torch()
    _check_dev(delay1, torch.int32, "delay1", 3)
    _check_dev(delay2, torch.int32, "delay2", 3)
    _check_dev(x, torch.uint8, "x", 2)
    n_sub, nc, nf = info.n_subbands, info.n_coarse, info.n_fine
    if n_sub < 1 or info.n_chan % n_sub:
        raise ValueError("info has an invalid subband count")
    m = info.n_chan // n_sub
    if not delay1.is_contiguous() or tuple(delay1.shape) != (n_sub, nc, m):
        raise ValueError("delay1 must be contiguous [n_sub, n_coarse, n_chan / n_sub]")
    if not delay2.is_contiguous() or tuple(delay2.shape) != (nc, nf, n_sub):
        raise ValueError("delay2 must be contiguous [n_coarse, n_fine, n_sub]")
    if x.shape[0] != info.n_chan or x.shape[1] < n_in:
        raise ValueError("x must be [n_chan, >= n_in]")
    if out is None:
        out = torch.empty((nc * nf, n_out), dtype=torch.int32, device=x.device)
    _check_dev(out, torch.int32, "out", 2)
    if out.shape[0] != nc * nf or out.shape[1] < n_out:
        raise ValueError("out must be [n_coarse * n_fine, >= n_out]")
    kp = None
    if keep is not None:
        _check_dev(keep, torch.uint8, "keep", 1)
        if keep.shape[0] != info.n_chan or not keep.is_contiguous():
            raise ValueError("keep must be a contiguous uint8 [n_chan] tensor")
        kp = keep.data_ptr()
    check(load().amber_subband_dedisperse_noalloc(delay1.data_ptr(), delay2.data_ptr(), ctypes.byref(info),
                                                  x.data_ptr(), x.stride(0), int(n_in), out.data_ptr(),
                                                  out.stride(0), int(n_out), kp, _tiles_ref(tiles1),
                                                  _tiles_ref(tiles2), _stream_handle(stream)))
    return out


def subband_static_bytes() -> int:
    """Bytes of the device array subband_dedisperse_noalloc uses (one per GPU)."""
    return int(load().amber_subband_static_bytes())


def _widths_arr(widths: Sequence[int]):
    w = np.ascontiguousarray(list(widths), dtype=np.int32)
    return w, w.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def integrate(dd, n_out: int, widths: Sequence[int], tiles: Optional[Tiles] = None, out=None, stream=None):
    """dd: int32 CUDA [n_dm, >= n_out].  Returns int32 [n_w, n_dm, n_out] (row k valid up to n_out - w_k + 1)."""
    torch = _torch()
    _check_dev(dd, torch.int32, "dd", 2)
    if dd.shape[1] < int(n_out):
        raise ValueError("dd must be [n_dm, >= n_out]")
    w, wp = _widths_arr(widths)
    n_dm = dd.shape[0]
    if out is None:
        out = torch.empty((len(w), n_dm, n_out), dtype=torch.int32, device=dd.device)
    _check_dev(out, torch.int32, "out", 3)
    if out.device != dd.device or out.shape[0] != len(w) or out.shape[1] != n_dm or out.shape[2] < n_out \
            or out.stride(0) != n_dm * out.stride(1):
        raise ValueError("out must be int32 [n_w, n_dm, >= n_out] with packed rows on %s" % dd.device)
    check(load().amber_integrate(dd.data_ptr(), n_dm, dd.stride(0), int(n_out), wp, len(w), out.data_ptr(),
                                 out.stride(1), _tiles_ref(tiles), _stream_handle(stream)))
    return out


def snr(box, n_out: int, widths: Sequence[int], tiles: Optional[Tiles] = None, stream=None):
    """box: int32 CUDA [n_w, n_dm, stride] as written by integrate.  Returns (float32 [n_w, n_dm], int32 [n_w, n_dm])."""
    torch = _torch()
    _check_dev(box, torch.int32, "box", 3)
    w, wp = _widths_arr(widths)
    n_dm = box.shape[1]
    if box.shape[0] != len(w) or box.stride(0) != n_dm * box.stride(1):
        raise ValueError("box must be [n_w, n_dm, stride] with packed rows")
    s = torch.empty((len(w), n_dm), dtype=torch.float32, device=box.device)
    p = torch.empty((len(w), n_dm), dtype=torch.int32, device=box.device)
    check(load().amber_snr(box.data_ptr(), n_dm, box.stride(1), int(n_out), wp, len(w), s.data_ptr(), p.data_ptr(),
                           _tiles_ref(tiles), _stream_handle(stream)))
    return s, p


def integrate_snr(dd, n_out: int, widths: Sequence[int], tiles: Optional[Tiles] = None, stream=None, out=None):
    """Fused boxcar + S/N.  dd: int32 CUDA [n_dm, >= n_out].  Returns (snr float32, peak int32), [n_w, n_dm] each."""
    torch = _torch()
    _check_dev(dd, torch.int32, "dd", 2)
    if dd.shape[1] < int(n_out):
        raise ValueError("dd must be [n_dm, >= n_out]")
    w, wp = _widths_arr(widths)
    n_dm = dd.shape[0]
    s, p = _table_out(out, len(w), n_dm, dd.device)
    check(load().amber_integrate_snr(dd.data_ptr(), n_dm, dd.stride(0), int(n_out), wp, len(w), s.data_ptr(),
                                     p.data_ptr(), _tiles_ref(tiles), _stream_handle(stream)))
    return s, p


def downsample(dd, n_out: int, factors: Sequence[int], tiles: Optional[Tiles] = None, out=None, stream=None):
    """Decimation: int32 [n_f, n_dm, max_j] with row k valid up to n_out // factors[k]."""
    torch = _torch()
    _check_dev(dd, torch.int32, "dd", 2)
    if dd.shape[1] < int(n_out):
        raise ValueError("dd must be [n_dm, >= n_out]")
    f, fp = _widths_arr(factors)
    n_dm = dd.shape[0]
    if len(f) == 0 or int(f.min()) < 1:
        raise ValueError("factors must be >= 1")
    n_y = int(n_out) // int(f.min())
    if out is None:
        out = torch.empty((len(f), n_dm, n_y), dtype=torch.int32, device=dd.device)
    _check_dev(out, torch.int32, "out", 3)
    if out.device != dd.device or out.shape[0] != len(f) or out.shape[1] != n_dm or out.shape[2] < n_y \
            or out.stride(0) != n_dm * out.stride(1):
        raise ValueError("out must be int32 [n_f, n_dm, >= n_out // min f] with packed rows on %s" % dd.device)
    check(load().amber_downsample(dd.data_ptr(), n_dm, dd.stride(0), int(n_out), fp, len(f), out.data_ptr(),
                                  out.stride(1), _tiles_ref(tiles), _stream_handle(stream)))
    return out


def downsample_snr(dd, n_out: int, factors: Sequence[int], tiles: Optional[Tiles] = None, stream=None, out=None):
    """Decimation + S/N fused.  Returns (snr float32, peak int32), [n_f, n_dm] each; peaks in decimated samples."""
    torch = _torch()
    _check_dev(dd, torch.int32, "dd", 2)
    if dd.shape[1] < int(n_out):
        raise ValueError("dd must be [n_dm, >= n_out]")
    f, fp = _widths_arr(factors)
    n_dm = dd.shape[0]
    s, p = _table_out(out, len(f), n_dm, dd.device)
    check(load().amber_downsample_snr(dd.data_ptr(), n_dm, dd.stride(0), int(n_out), fp, len(f), s.data_ptr(),
                                      p.data_ptr(), _tiles_ref(tiles), _stream_handle(stream)))
    return s, p


class Search:
    """One beam geometry with its delay table resident on the device.

    run(x) executes dedispersion and the fused boxcar + S/N on x (uint8 CUDA
    [n_chan, stride]) and returns (dd, snr, peak).
    """

    def __init__(self, freq_mhz, t_samp_s, n_dm, dm_first, dm_step, n_out, widths, tiles=None, device="cuda"):
        torch = _torch()
        self.delays_host, self.info = delay_table(freq_mhz, t_samp_s, n_dm, dm_first, dm_step)
        self.delays = torch.from_numpy(self.delays_host).to(device)
        self.n_out = int(n_out)
        self.n_in = self.n_out + self.info.max_delay
        self.widths = tuple(int(w) for w in widths)
        self.tiles = tiles
        self.dd = torch.empty((self.info.n_dm, self.n_out), dtype=torch.int32, device=device)
        self.snr = torch.empty((len(self.widths), self.info.n_dm), dtype=torch.float32, device=device)
        self.peak = torch.empty((len(self.widths), self.info.n_dm), dtype=torch.int32, device=device)

    def run(self, x, stream=None):
        dedisperse(self.delays, self.info, x, self.n_in, self.n_out, self.tiles, out=self.dd, stream=stream)
        integrate_snr(self.dd, self.n_out, self.widths, self.tiles, stream=stream, out=(self.snr, self.peak))
        return self.dd, self.snr, self.peak


# --- tile search --------------------------------------------------------------------

def default_space(info: DelayInfo, widths: Sequence[int], n_out: int) -> TuneSpace:
    """The library's gene arrays for a problem (powers of two within the kernels' bounds)."""
    w, wp = _widths_arr(widths)
    sp = TuneSpace()
    check(load().amber_default_space(ctypes.byref(info), wp, len(w), int(n_out), ctypes.byref(sp)))
    return sp


def space_size(space: TuneSpace) -> int:
    n = ctypes.c_int64(0)
    check(load().amber_space_size(ctypes.byref(space), ctypes.byref(n)))
    return int(n.value)


def tune_params(search: str = "ga", **kw) -> TuneParams:
    """Default GA parameters with overrides; search is ga | exhaustive | random | per_kernel."""
    p = TuneParams()
    check(load().amber_default_tune_params(ctypes.byref(p)))
    p.search = SEARCH_KINDS[search]
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError("TuneParams has no field %r" % k)
        setattr(p, k, v)
    return p


def search_tiles(space: TuneSpace, params: TuneParams, fitness, log_path: Optional[str] = None) -> TuneResult:
    """Host-only search with a Python fitness(tiles) -> seconds (raise or return None for a failure)."""
    errors = []

    def cb(tiles_p, user, out_p):
        try:
            v = fitness(tiles_p.contents)
            if v is None:
                return 1
            out_p[0] = float(v)
            return 0
        except Exception as e:  # surfaced after the call
            errors.append(e)
            return 1

    cfn = FITNESS_FN(cb)
    res = TuneResult()
    rc = load().amber_search_tiles(ctypes.byref(space), ctypes.byref(params), cfn, None, ctypes.byref(res),
                                   log_path.encode() if log_path else None)
    check(rc)
    return res


def tune(space: TuneSpace, delays, x, n_in: int, params: TuneParams, log_path: Optional[str] = None, stream=None,
         buffers=None) -> TuneResult:
    """Device search: fitness = GPU time of dedisperse + fused boxcar/S/N on x."""
    torch = _torch()
    _check_dev(delays, torch.int32, "delays", 2)
    _check_dev(x, torch.uint8, "x", 2)
    info, n_out, n_w = space.info, space.n_out, space.n_widths
    if buffers is None:
        dd = torch.empty((info.n_dm, n_out), dtype=torch.int32, device=x.device)
        s = torch.empty((n_w, info.n_dm), dtype=torch.float32, device=x.device)
        p = torch.empty((n_w, info.n_dm), dtype=torch.int32, device=x.device)
    else:
        dd, s, p = buffers
    res = TuneResult()
    check(load().amber_tune(ctypes.byref(space), delays.data_ptr(), x.data_ptr(), x.stride(0), int(n_in),
                            dd.data_ptr(), dd.stride(0), s.data_ptr(), p.data_ptr(), ctypes.byref(params),
                            ctypes.byref(res), log_path.encode() if log_path else None, _stream_handle(stream)))
    return res


def default_subband_space(info: SubbandInfo, widths: Sequence[int], n_out: int) -> SubbandTuneSpace:
    """The default search space of the subband pipeline (both steps' genes and the boxcar / S/N genes)."""
    w, wp = _widths_arr(widths)
    sp = SubbandTuneSpace()
    check(load().amber_default_subband_space(ctypes.byref(info), wp, len(w), int(n_out), ctypes.byref(sp)))
    return sp


def subband_space_size(space: SubbandTuneSpace) -> int:
    n = ctypes.c_int64()
    check(load().amber_subband_space_size(ctypes.byref(space), ctypes.byref(n)))
    return n.value


def search_subband_tiles(space: SubbandTuneSpace, params: TuneParams, fitness,
                         log_path: Optional[str] = None) -> SubbandTuneResult:
    """Host-only subband search with a Python fitness(step1_tiles, step2_tiles) -> seconds (None: failure)."""
    def cb(t1, t2, user, out_p):
        try:
            v = fitness(t1.contents, t2.contents)
            if v is None:
                return 1
            out_p[0] = float(v)
            return 0
        except Exception:
            return 1

    cfn = SUBBAND_FITNESS_FN(cb)
    res = SubbandTuneResult()
    check(load().amber_search_subband_tiles(ctypes.byref(space), ctypes.byref(params), cfn, None, ctypes.byref(res),
                                            log_path.encode() if log_path else None))
    return res


def tune_subband(space: SubbandTuneSpace, delay1, delay2, x, n_in: int, params: TuneParams, work=None, out=None,
                 snr=None, peak=None, log_path: Optional[str] = None, stream=None) -> SubbandTuneResult:
    """Device search: fitness = GPU time of subband dedispersion + fused boxcar/S/N on x."""
    torch = _torch()
    _check_dev(delay1, torch.int32, "delay1", 3)
    _check_dev(delay2, torch.int32, "delay2", 3)
    _check_dev(x, torch.uint8, "x", 2)
    info, n_out, n_w = space.info, space.n_out, space.n_widths
    n_dm = info.n_coarse * info.n_fine
    n1 = n_out + info.max_delay2
    if work is None:
        work = torch.empty((info.n_subbands * info.n_coarse, (n1 + 63) // 64 * 64), dtype=torch.uint16,
                           device=x.device)
    if out is None:
        out = torch.empty((n_dm, n_out), dtype=torch.int32, device=x.device)
    if snr is None:
        snr = torch.empty((n_w, n_dm), dtype=torch.float32, device=x.device)
    if peak is None:
        peak = torch.empty((n_w, n_dm), dtype=torch.int32, device=x.device)
    res = SubbandTuneResult()
    check(load().amber_tune_subband(ctypes.byref(space), delay1.data_ptr(), delay2.data_ptr(), x.data_ptr(),
                                    x.stride(0), int(n_in), work.data_ptr(), work.stride(0), out.data_ptr(),
                                    out.stride(0), snr.data_ptr(), peak.data_ptr(), ctypes.byref(params),
                                    ctypes.byref(res), log_path.encode() if log_path else None,
                                    _stream_handle(stream)))
    return res


# --- batched beams --------------------------------------------------------------------

# Batch and Server handles still open: closed at interpreter exit, while the
# HIP runtime and the library are certainly alive (a handle released from
# __del__ during interpreter shutdown could run after either is torn down).
_open_handles = weakref.WeakSet()


def _close_open_handles():
    for h in list(_open_handles):
        try:
            h.close()
        except Exception:
            pass


atexit.register(_close_open_handles)


def _release_in_del(obj):
    if sys.is_finalizing():   # the atexit hook has run; nothing is left to release
        return
    try:
        obj.close()
    except Exception:
        pass


class Batch:
    """Independent beams of uneven sizes run together.

    beams: sequence of dicts with keys delays (int32 CUDA [n_dm, n_chan]),
    info (DelayInfo), x (uint8 CUDA [n_chan, stride]), n_in, dd (int32 CUDA
    [n_dm, >= n_out]), n_out, snr (float32 CUDA [n_w, n_dm]), peak (int32 CUDA
    [n_w, n_dm]).  tiles: per-beam Tiles (or None for automatic tiles).
    run() enqueues the launches; capture() records them into a HIP graph that
    launch() replays with one graph launch.
    """

    def __init__(self, beams, widths: Sequence[int], tiles=None):
        self._keep = list(beams)
        arr = (Beam * len(beams))()
        for k, b in enumerate(beams):
            arr[k] = Beam(d_delays=b["delays"].data_ptr(), info=b["info"], d_in=b["x"].data_ptr(),
                          in_stride=b["x"].stride(0), n_in=int(b["n_in"]), d_dd=b["dd"].data_ptr(),
                          dd_stride=b["dd"].stride(0), n_out=int(b["n_out"]), d_snr=b["snr"].data_ptr(),
                          d_peak_t=b["peak"].data_ptr())
        self._w, wp = _widths_arr(widths)
        tarr = None
        if tiles is not None:
            tarr = (Tiles * len(beams))(*tiles)
        h = ctypes.c_void_p()
        check(load().amber_batch_create(arr, len(beams), wp, len(self._w), tarr, ctypes.byref(h)))
        self._h = h
        _open_handles.add(self)

    def launches(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        check(load().amber_batch_launches(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def run(self, stream=None):
        check(load().amber_batch_run(self._h, _stream_handle(stream)))

    def capture(self, stream):
        check(load().amber_batch_capture(self._h, _stream_handle(stream)))

    def launch(self, stream=None):
        check(load().amber_batch_launch(self._h, _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _open_handles.discard(self)
            check(load().amber_batch_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        _release_in_del(self)


def chunk_span(seq: int, chunk: int, max_delay: int):
    """(t_first, n_out): the absolute output times chunk `seq` of a stream yields."""
    a, b = ctypes.c_int64(), ctypes.c_int64()
    check(load().amber_chunk_span(int(seq), int(chunk), int(max_delay), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def server_config(max_inflight: int = 64, max_batch: int = 32, n_streams: int = 4, memory_budget: int = 0):
    return ServerConfig(max_inflight=max_inflight, max_batch=max_batch, n_streams=n_streams,
                        memory_budget=memory_budget)


def admit(pending, beam_busy, inflight: int, memory_in_use: int, config: ServerConfig):
    """The service's admission rule on host data: pending = [(beam, bytes)] in
    arrival order, beam_busy = per-beam flags.  Returns (admitted indices,
    index of the chunk that did not fit the memory budget or -1)."""
    n = len(pending)
    parr = (PendingChunk * max(n, 1))(*[PendingChunk(beam=int(b), bytes=int(x)) for b, x in pending])
    busy = (ctypes.c_uint8 * max(len(beam_busy), 1))(*[1 if v else 0 for v in beam_busy])
    out = (ctypes.c_int32 * max(n, 1))()
    na, blocked = ctypes.c_int32(), ctypes.c_int32()
    check(load().amber_server_admit(parr, n, busy, len(beam_busy), int(inflight), int(memory_in_use),
                                    ctypes.byref(config), out, ctypes.byref(na), ctypes.byref(blocked)))
    return [out[k] for k in range(na.value)], blocked.value


def server_clock() -> float:
    return load().amber_server_clock()


class Server:
    """Streaming service: beams registered with add_beam(), chunks (host
    uint8 [n_chan, L] arrays) queued with submit(), results taken with wait().

    The library's scheduler thread admits chunks as launch slots and device
    memory free up, fuses the admitted chunks of different beams into shared
    launches and spreads them over n_streams streams; every beam keeps its
    last max_delay input samples on the device between chunks.
    """

    def __init__(self, max_inflight: int = 64, max_batch: int = 32, n_streams: int = 4, memory_budget: int = 0):
        self.config = server_config(max_inflight, max_batch, n_streams, memory_budget)
        h = ctypes.c_void_p()
        check(load().amber_server_create(ctypes.byref(self.config), ctypes.byref(h)))
        self._h = h
        _open_handles.add(self)
        self._beams = []

    def add_beam(self, freqs, t_samp_s: float, n_dm: int, dm_first: float, dm_step: float, chunk: int,
                 widths: Sequence[int], tiles: Optional[Tiles] = None) -> int:
        f = np.ascontiguousarray(freqs, dtype=np.float64)
        w, wp = _widths_arr(widths)
        b = StreamBeam(n_chan=len(f), freq_mhz=f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), t_samp_s=t_samp_s,
                       n_dm=n_dm, dm_first=dm_first, dm_step=dm_step, chunk=int(chunk),
                       tiles=ctypes.pointer(tiles) if tiles is not None else None)
        bid = ctypes.c_int32()
        check(load().amber_server_add_beam(self._h, ctypes.byref(b), wp, len(w), ctypes.byref(bid)))
        self._beams.append((len(f), int(chunk), n_dm, len(w)))
        return bid.value

    def submit(self, beam: int, chunk: np.ndarray, tag: int = 0) -> None:
        if not 0 <= beam < len(self._beams):  # the library rejects the id
            check(load().amber_server_submit(self._h, int(beam), chunk.ctypes.data, chunk.strides[0], int(tag)))
        n_chan, L, _, _ = self._beams[beam]
        if chunk.dtype != np.uint8 or chunk.ndim != 2 or chunk.shape[0] != n_chan or chunk.shape[1] < L \
                or chunk.strides[1] != 1:
            raise ValueError("chunk must be a uint8 [%d, >= %d] array with unit column stride" % (n_chan, L))
        check(load().amber_server_submit(self._h, beam, chunk.ctypes.data, chunk.strides[0], int(tag)))

    def wait(self, timeout: float = 10.0):
        """The oldest completed chunk as a dict (result fields plus "snr" and
        "peak" arrays of [n_widths, n_dm], None when has_snr is 0), or None if
        nothing completed within `timeout` seconds."""
        r = ChunkResult()
        cap = max(nd * nw for _, _, nd, nw in self._beams) if self._beams else 0
        snr = np.empty(max(cap, 1), np.float32)
        peak = np.empty(max(cap, 1), np.int32)
        st = load().amber_server_wait(self._h, float(timeout), ctypes.byref(r), snr.ctypes.data, peak.ctypes.data, cap)
        if st == AMBER_E_TIMEOUT:
            return None
        check(st)
        d = r.as_dict()
        n = r.n_widths * r.n_dm
        d["snr"] = snr[:n].reshape(r.n_widths, r.n_dm).copy() if r.has_snr else None
        d["peak"] = peak[:n].reshape(r.n_widths, r.n_dm).copy() if r.has_snr else None
        return d

    def stats(self) -> dict:
        s = ServerStats()
        check(load().amber_server_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _open_handles.discard(self)
            check(load().amber_server_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        _release_in_del(self)
