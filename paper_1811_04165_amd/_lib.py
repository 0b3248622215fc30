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


class SubbandGeometry(ctypes.Structure):
    _fields_ = [("n_chan", ctypes.c_int32), ("freq_mhz", c_f64p), ("t_samp_s", ctypes.c_double),
                ("n_subbands", ctypes.c_int32), ("n_coarse", ctypes.c_int32), ("coarse_first", ctypes.c_double),
                ("coarse_step", ctypes.c_double), ("n_fine", ctypes.c_int32), ("fine_first", ctypes.c_double),
                ("fine_step", ctypes.c_double)]


class SubbandInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("n_chan", "n_subbands", "n_coarse", "n_fine", "max_delay1",
                                              "max_step1", "max_delay2", "max_step2", "max_delay")]

    def __repr__(self):
        return "SubbandInfo(%s)" % ", ".join("%s=%d" % (n, getattr(self, n)) for n, _ in self._fields_)


class Tiles(ctypes.Structure):
    _fields_ = [("threads_per_dm", ctypes.c_int32), ("samples_per_thread", ctypes.c_int32),
                ("dms_per_block", ctypes.c_int32), ("channel_unroll", ctypes.c_int32),
                ("snr_threads", ctypes.c_int32), ("boxcar_step", ctypes.c_int32 * AMBER_MAX_WIDTHS),
                ("dms_per_thread", ctypes.c_int32), ("direct_reads", ctypes.c_int32)]

    def as_dict(self):
        return {"threads_per_dm": self.threads_per_dm, "samples_per_thread": self.samples_per_thread,
                "dms_per_block": self.dms_per_block, "channel_unroll": self.channel_unroll,
                "snr_threads": self.snr_threads, "boxcar_step": list(self.boxcar_step),
                "dms_per_thread": self.dms_per_thread, "direct_reads": self.direct_reads}

    def __repr__(self):
        d = self.as_dict()
        d["boxcar_step"] = d["boxcar_step"][:8]
        return "Tiles(%s)" % ", ".join("%s=%s" % kv for kv in d.items())


# gene indices of a tune space (include/amber.h): the dedispersion kernel's
# genes, then the boxcar / S/N kernel's
(GENE_THREADS_PER_DM, GENE_SAMPLES_PER_THREAD, GENE_DMS_PER_BLOCK, GENE_CHANNEL_UNROLL, GENE_DMS_PER_THREAD,
 GENE_DIRECT_READS) = range(6)
AMBER_GENES_K1 = 6
GENE_SNR_THREADS = AMBER_GENES_K1
GENE_BOXCAR0 = AMBER_GENES_K1 + 1
AMBER_MAX_GENES = AMBER_GENES_K1 + 1 + AMBER_MAX_WIDTHS
AMBER_MAX_GENE_VALUES = 8
AMBER_E_TIMEOUT = -6
SEARCH_KINDS = {"ga": 0, "exhaustive": 1, "random": 2, "per_kernel": 3}


class TuneSpace(ctypes.Structure):
    _fields_ = [("n_genes", ctypes.c_int32), ("n_values", ctypes.c_int32 * AMBER_MAX_GENES),
                ("values", (ctypes.c_int32 * AMBER_MAX_GENE_VALUES) * AMBER_MAX_GENES), ("info", DelayInfo),
                ("n_widths", ctypes.c_int32), ("widths", ctypes.c_int32 * AMBER_MAX_WIDTHS), ("n_out", ctypes.c_int64)]

    def gene_values(self, i):
        return [self.values[i][k] for k in range(self.n_values[i])]

    def set_gene_values(self, i, vals):
        if not 1 <= len(vals) <= AMBER_MAX_GENE_VALUES:
            raise ValueError("a gene takes 1..%d values" % AMBER_MAX_GENE_VALUES)
        self.n_values[i] = len(vals)
        for k, v in enumerate(vals):
            self.values[i][k] = int(v)


class TuneParams(ctypes.Structure):
    _fields_ = [("search", ctypes.c_int32), ("pop", ctypes.c_int32), ("generations", ctypes.c_int32),
                ("crossover", ctypes.c_int32), ("p_cross", ctypes.c_double), ("p_mut", ctypes.c_double),
                ("pool_frac", ctypes.c_double), ("seed", ctypes.c_uint64), ("warmup", ctypes.c_int32),
                ("reps", ctypes.c_int32), ("eval_timeout_s", ctypes.c_double), ("max_evals", ctypes.c_int64),
                ("seed_default", ctypes.c_int32), ("restart_after", ctypes.c_int32),
                ("retime_top", ctypes.c_int32), ("retime_runs", ctypes.c_int32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("best", Tiles), ("best_time_s", ctypes.c_double), ("n_evals", ctypes.c_int64),
                ("n_failed", ctypes.c_int64), ("space_size", ctypes.c_int64), ("wall_s", ctypes.c_double)]

    def as_dict(self, n_widths=AMBER_MAX_WIDTHS):
        best = self.best.as_dict()
        best["boxcar_step"] = best["boxcar_step"][:n_widths]
        return {"best": best, "best_time_s": self.best_time_s, "n_evals": self.n_evals, "n_failed": self.n_failed,
                "space_size": self.space_size, "wall_s": self.wall_s}


class Beam(ctypes.Structure):
    _fields_ = [("d_delays", ctypes.c_void_p), ("info", DelayInfo), ("d_in", ctypes.c_void_p),
                ("in_stride", ctypes.c_int64), ("n_in", ctypes.c_int64), ("d_dd", ctypes.c_void_p),
                ("dd_stride", ctypes.c_int64), ("n_out", ctypes.c_int64), ("d_snr", ctypes.c_void_p),
                ("d_peak_t", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("max_inflight", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("n_streams", ctypes.c_int32),
                ("memory_budget", ctypes.c_int64)]


class StreamBeam(ctypes.Structure):
    _fields_ = [("n_chan", ctypes.c_int32), ("freq_mhz", c_f64p), ("t_samp_s", ctypes.c_double),
                ("n_dm", ctypes.c_int32), ("dm_first", ctypes.c_double), ("dm_step", ctypes.c_double),
                ("chunk", ctypes.c_int64), ("tiles", ctypes.POINTER(Tiles))]


class ChunkResult(ctypes.Structure):
    _fields_ = [("beam", ctypes.c_int32), ("n_widths", ctypes.c_int32), ("n_dm", ctypes.c_int32),
                ("seq", ctypes.c_int64), ("tag", ctypes.c_uint64), ("t_first", ctypes.c_int64),
                ("n_out", ctypes.c_int64), ("has_snr", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "batches", "queued", "inflight",
                                               "memory_in_use", "memory_peak", "memory_budget",
                                               "admissions_deferred_for_memory")]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class PendingChunk(ctypes.Structure):
    _fields_ = [("beam", ctypes.c_int32), ("bytes", ctypes.c_int64)]


FITNESS_FN = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.POINTER(Tiles), ctypes.c_void_p, ctypes.POINTER(ctypes.c_double))

# gene indices of a subband tune space: step one's dedispersion genes, step
# two's, then the boxcar / S/N kernel's
SB_GENES_STEP1, SB_GENES_STEP2 = 5, 4
SB_GENE_STEP2 = SB_GENES_STEP1
SB_GENE_SNR_THREADS = SB_GENES_STEP1 + SB_GENES_STEP2
SB_GENE_BOXCAR0 = SB_GENE_SNR_THREADS + 1
AMBER_MAX_SUBBAND_GENES = SB_GENE_BOXCAR0 + AMBER_MAX_WIDTHS


class SubbandTuneSpace(ctypes.Structure):
    _fields_ = [("n_genes", ctypes.c_int32), ("n_values", ctypes.c_int32 * AMBER_MAX_SUBBAND_GENES),
                ("values", (ctypes.c_int32 * AMBER_MAX_GENE_VALUES) * AMBER_MAX_SUBBAND_GENES),
                ("info", SubbandInfo), ("n_widths", ctypes.c_int32), ("widths", ctypes.c_int32 * AMBER_MAX_WIDTHS),
                ("n_out", ctypes.c_int64)]
    gene_values = TuneSpace.gene_values
    set_gene_values = TuneSpace.set_gene_values


class SubbandTuneResult(ctypes.Structure):
    _fields_ = [("step1", Tiles), ("step2", Tiles), ("best_time_s", ctypes.c_double), ("n_evals", ctypes.c_int64),
                ("n_failed", ctypes.c_int64), ("space_size", ctypes.c_int64), ("wall_s", ctypes.c_double)]

    def as_dict(self, n_widths=AMBER_MAX_WIDTHS):
        keys = ("threads_per_dm", "samples_per_thread", "dms_per_block", "channel_unroll")
        s1, s2 = self.step1.as_dict(), self.step2.as_dict()
        return {"step1": {k: s1[k] for k in keys + ("dms_per_thread",)}, "step2": {k: s2[k] for k in keys},
                "snr_threads": s1["snr_threads"], "boxcar_step": s1["boxcar_step"][:n_widths],
                "best_time_s": self.best_time_s, "n_evals": self.n_evals, "n_failed": self.n_failed,
                "space_size": self.space_size, "wall_s": self.wall_s}


SUBBAND_FITNESS_FN = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.POINTER(Tiles), ctypes.POINTER(Tiles), ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_double))

# (name, restype, argtypes) of every exported symbol the header declares.
SIGNATURES = [
    ("amber_last_error", ctypes.c_char_p, []),
    ("amber_version", ctypes.c_char_p, []),
    ("amber_default_tiles", ctypes.c_int, [ctypes.POINTER(Tiles)]),
    ("amber_auto_tiles", ctypes.c_int, [ctypes.POINTER(DelayInfo), ctypes.c_int64, ctypes.POINTER(Tiles)]),
    ("amber_validate_tiles", ctypes.c_int, [ctypes.POINTER(Tiles), ctypes.POINTER(DelayInfo), ctypes.c_int32]),
    ("amber_delay_table", ctypes.c_int, [ctypes.POINTER(Geometry), c_i32p, ctypes.POINTER(DelayInfo)]),
    ("amber_dedisperse", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(DelayInfo), ctypes.c_void_p,
                                        ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.POINTER(Tiles), ctypes.c_void_p]),
    ("amber_dedisperse_masked", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(DelayInfo), ctypes.c_void_p,
                                               ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                               ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(Tiles),
                                               ctypes.c_void_p]),
    ("amber_subband_delay_tables", ctypes.c_int, [ctypes.POINTER(SubbandGeometry), c_i32p, c_i32p,
                                                  ctypes.POINTER(SubbandInfo)]),
    ("amber_subband_dedisperse", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(SubbandInfo),
                                                ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                                ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                                ctypes.c_void_p, ctypes.POINTER(Tiles), ctypes.POINTER(Tiles),
                                                ctypes.c_void_p]),
    ("amber_subband_dedisperse_noalloc", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                        ctypes.POINTER(SubbandInfo), ctypes.c_void_p, ctypes.c_int64,
                                                        ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                                        ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(Tiles),
                                                        ctypes.POINTER(Tiles), ctypes.c_void_p]),
    ("amber_subband_static_bytes", ctypes.c_int64, []),
    ("amber_integrate", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                       c_i32p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.POINTER(Tiles), ctypes.c_void_p]),
    ("amber_snr", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, c_i32p,
                                 ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Tiles),
                                 ctypes.c_void_p]),
    ("amber_integrate_snr", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                           c_i32p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.POINTER(Tiles), ctypes.c_void_p]),
    ("amber_downsample", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                        c_i32p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.POINTER(Tiles), ctypes.c_void_p]),
    ("amber_downsample_snr", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                            c_i32p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.POINTER(Tiles), ctypes.c_void_p]),
    ("amber_default_space", ctypes.c_int, [ctypes.POINTER(DelayInfo), c_i32p, ctypes.c_int32, ctypes.c_int64,
                                           ctypes.POINTER(TuneSpace)]),
    ("amber_space_size", ctypes.c_int, [ctypes.POINTER(TuneSpace), ctypes.POINTER(ctypes.c_int64)]),
    ("amber_default_tune_params", ctypes.c_int, [ctypes.POINTER(TuneParams)]),
    ("amber_search_tiles", ctypes.c_int, [ctypes.POINTER(TuneSpace), ctypes.POINTER(TuneParams), FITNESS_FN,
                                          ctypes.c_void_p, ctypes.POINTER(TuneResult), ctypes.c_char_p]),
    ("amber_default_subband_space", ctypes.c_int, [ctypes.POINTER(SubbandInfo), c_i32p, ctypes.c_int32,
                                                   ctypes.c_int64, ctypes.POINTER(SubbandTuneSpace)]),
    ("amber_subband_space_size", ctypes.c_int, [ctypes.POINTER(SubbandTuneSpace), ctypes.POINTER(ctypes.c_int64)]),
    ("amber_search_subband_tiles", ctypes.c_int, [ctypes.POINTER(SubbandTuneSpace), ctypes.POINTER(TuneParams),
                                                  SUBBAND_FITNESS_FN, ctypes.c_void_p,
                                                  ctypes.POINTER(SubbandTuneResult), ctypes.c_char_p]),
    ("amber_tune_subband", ctypes.c_int, [ctypes.POINTER(SubbandTuneSpace), ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.POINTER(TuneParams),
                                          ctypes.POINTER(SubbandTuneResult), ctypes.c_char_p, ctypes.c_void_p]),
    ("amber_batch_create", ctypes.c_int, [ctypes.POINTER(Beam), ctypes.c_int32, c_i32p, ctypes.c_int32,
                                          ctypes.POINTER(Tiles), ctypes.POINTER(ctypes.c_void_p)]),
    ("amber_batch_run", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("amber_batch_capture", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("amber_batch_launch", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("amber_batch_launches", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32)]),
    ("amber_batch_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("amber_chunk_span", ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    ("amber_server_admit", ctypes.c_int, [ctypes.POINTER(PendingChunk), ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_uint8), ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int64, ctypes.POINTER(ServerConfig), c_i32p, c_i32p, c_i32p]),
    ("amber_server_create", ctypes.c_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(ctypes.c_void_p)]),
    ("amber_server_add_beam", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(StreamBeam), c_i32p, ctypes.c_int32,
                                             c_i32p]),
    ("amber_server_submit", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_uint64]),
    ("amber_server_wait", ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(ChunkResult),
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    ("amber_server_get_stats", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerStats)]),
    ("amber_server_clock", ctypes.c_double, []),
    ("amber_server_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("amber_tune", ctypes.c_int, [ctypes.POINTER(TuneSpace), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.POINTER(TuneParams), ctypes.POINTER(TuneResult), ctypes.c_char_p,
                                  ctypes.c_void_p]),
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
        # torch carries its own copy of the HIP runtime under the soname this
        # library links against.  Loaded after torch, the library binds to that
        # copy; loaded before it, the process ends up with two HIP runtimes,
        # each opening the device on its own, and the second one to start has
        # reported no device.  So torch is always loaded first.
        import torch  # noqa: F401
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
