"""Seeded synthetic inputs for the single-pulse search, shared by the tests and
the benchmark.

This module holds no arithmetic of the method itself: it describes workload
geometries (channel frequencies, DM grids, widths), draws seeded uint8 noise
and injects boxcar pulses at per-channel sample offsets that the CALLER
supplies (a row of a delay table computed elsewhere).  Neither the oracle nor
the product library is imported here.

Noise follows the recipe "uint8 Gaussian noise, mean 128, sd 16, clipped to
0..255": ``rint(normal(128, 16))`` from ``numpy.random.default_rng(seed)``
(PCG64), clipped, cast to uint8.  A pulse of width W and amplitude A at
dedispersed time t0 for DM row i adds A (saturating at 255) to
``x[c][t0 + offsets[c] + k]`` for k < W, where ``offsets = delays[i]``.

Channel frequencies follow the paper's Table 2 form MIN_FREQ + c *
CHANNEL_BANDWIDTH with channel 0 the lowest; every synthetic band here spans
1250-1550 MHz.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Sequence, Tuple

import numpy as np

T_SAMP_S = 81.92e-6          # sampling time of every synthetic workload
BAND_LOW_MHZ = 1250.0
BAND_WIDTH_MHZ = 300.0
ROW_PAD_BYTES = 128          # Table 2 DEVICE_PADDING: rows padded to a cache line


@dataclass(frozen=True)
class Geometry:
    n_chan: int
    n_dm: int
    dm_first: float
    dm_step: float
    t_samp_s: float = T_SAMP_S
    f_low_mhz: float = BAND_LOW_MHZ
    bandwidth_mhz: float = BAND_WIDTH_MHZ

    def freqs(self) -> np.ndarray:
        """Channel frequencies (MHz), f_low + c * bandwidth / n_chan, ascending."""
        df = self.bandwidth_mhz / self.n_chan
        return self.f_low_mhz + np.arange(self.n_chan, dtype=np.float64) * df


@dataclass(frozen=True)
class Pulse:
    dm_index: int
    width: int
    amp: int
    t0: int


@dataclass(frozen=True)
class Workload:
    name: str
    geom: Geometry
    n_out: int
    widths: Tuple[int, ...]
    pulses: Tuple[Pulse, ...]
    seed: int
    description: str = ""


def padded_stride(n_in: int, pad: int = ROW_PAD_BYTES) -> int:
    return ((n_in + pad - 1) // pad) * pad


def noise(n_chan: int, n_in: int, stride: int, seed: int, mean: float = 128.0, sd: float = 16.0) -> np.ndarray:
    """uint8 [n_chan, stride]: seeded clipped Gaussian in the first n_in columns, 0 after."""
    rng = np.random.default_rng(seed)
    x = np.zeros((n_chan, stride), dtype=np.uint8)
    # row by row keeps the float64 temporaries small for large beams
    for c in range(n_chan):
        v = np.rint(rng.normal(mean, sd, size=n_in))
        x[c, :n_in] = np.clip(v, 0, 255).astype(np.uint8)
    return x


def inject(x: np.ndarray, offsets: np.ndarray, t0: int, width: int, amp: int) -> None:
    """Add amp (saturating at 255) to x[c][t0 + offsets[c] + k] for k < width, in place."""
    offsets = np.asarray(offsets)
    if offsets.shape[0] != x.shape[0]:
        raise ValueError("one offset per channel is required")
    for c in range(x.shape[0]):
        s = int(t0) + int(offsets[c])
        seg = x[c, s:s + width].astype(np.int32) + int(amp)
        x[c, s:s + width] = np.minimum(seg, 255).astype(np.uint8)


def make_input(wl: Workload, delays: np.ndarray, max_delay: int):
    """Noise plus the workload's pulses.  delays: int32 [n_dm, n_chan] from any delay table.

    Returns (x uint8 [n_chan, stride], n_in) with n_in = n_out + max_delay.
    """
    n_in = wl.n_out + int(max_delay)
    x = noise(wl.geom.n_chan, n_in, padded_stride(n_in), wl.seed)
    for p in wl.pulses:
        inject(x, delays[p.dm_index], p.t0, p.width, p.amp)
    return x, n_in


# --- the synthetic workloads -------------------------------------------------

def small() -> Workload:
    """256 channels, 128 DM trials 0..127 step 1, 8192 output samples, one pulse
    (DM index 50, width 4, +40 counts at t0 = 4096), widths 1..16."""
    return Workload(
        name="small-256ch-128dm",
        geom=Geometry(n_chan=256, n_dm=128, dm_first=0.0, dm_step=1.0),
        n_out=8192, widths=(1, 2, 4, 8, 16),
        pulses=(Pulse(dm_index=50, width=4, amp=40, t0=4096),), seed=1,
        description="256 ch over 1250-1550 MHz, t_samp 81.92 us, 8192 samples + max-delay overlap, "
                    "128 DM trials 0-127 step 1, boxcar widths {1,2,4,8,16}")


def beam() -> Workload:
    """One full 1-s beam: 1536 channels, 2048 DM trials 0..1023.5 step 0.5,
    12208 output samples, five pulses at random on-grid DM in [0, 1000] and
    width in {1..32}, widths 1..64."""
    rng = np.random.default_rng([2, 7])
    pulses = []
    for k in range(5):
        dm_index = int(rng.integers(0, 2001))
        width = int(rng.choice([1, 2, 4, 8, 16, 32]))
        pulses.append(Pulse(dm_index=dm_index, width=width, amp=40, t0=1024 + 2048 * k))
    return Workload(
        name="beam-1536ch-2048dm",
        geom=Geometry(n_chan=1536, n_dm=2048, dm_first=0.0, dm_step=0.5),
        n_out=12208, widths=(1, 2, 4, 8, 16, 32, 64), pulses=tuple(pulses), seed=2,
        description="1536 ch over 1250-1550 MHz, t_samp 81.92 us, 12208 samples (1 s) + max-delay overlap, "
                    "2048 DM trials 0-1023.5 step 0.5, boxcar widths 1-64 (powers of 2), 5 pulses")


def batch_beams(n_beams: int = 40) -> List[Workload]:
    """Uneven beams for batched launches: channels in {384,768,1536}, samples
    uniform in [4096, 24576], DM trials in {512,1024,2048} (step 0.5 from 0),
    one pulse each (on-grid DM, width in {1..32}, t0 = n_out/2 down to a
    multiple of 64), widths 1..32.  Beam b is seeded 4000 + b."""
    out = []
    for b in range(n_beams):
        rng = np.random.default_rng(4000 + b)
        n_chan = int(rng.choice([384, 768, 1536]))
        n_out = int(rng.integers(4096, 24577))
        n_dm = int(rng.choice([512, 1024, 2048]))
        width = int(rng.choice([1, 2, 4, 8, 16, 32]))
        dm_index = int(rng.integers(0, n_dm))
        t0 = (n_out // 2) // 64 * 64
        out.append(Workload(
            name="batch-beam-%d" % b,
            geom=Geometry(n_chan=n_chan, n_dm=n_dm, dm_first=0.0, dm_step=0.5),
            n_out=n_out, widths=(1, 2, 4, 8, 16, 32),
            pulses=(Pulse(dm_index=dm_index, width=width, amp=40, t0=t0),), seed=4000 + b))
    return out


def tiny(n_chan: int, n_dm: int, n_out: int, seed: int, max_delay: int = 16):
    """Random small case for brute-force checks: random non-negative delays
    (not from any formula) and uniform uint8 data.  Returns (delays, x, n_in)."""
    rng = np.random.default_rng(seed)
    delays = rng.integers(0, max_delay + 1, size=(n_dm, n_chan)).astype(np.int32)
    n_in = n_out + int(delays.max())
    stride = n_in + int(rng.integers(0, 5))
    x = rng.integers(0, 256, size=(n_chan, stride)).astype(np.uint8)
    return delays, x, n_in


# --- streaming ---------------------------------------------------------------

STREAM_CHUNK = 6104          # samples per chunk: 0.5 s at 81.92 us (whole samples)


def stream_geometries(n_beams: int = 40) -> List[Geometry]:
    """Beams of the streaming workload, alternating 768 channels / 1024 DM
    trials and 1536 channels / 2048 DM trials, DM step 0.5 from 0 (so the
    largest delays are about 5.8k and 11.6k samples)."""
    out = []
    for b in range(n_beams):
        if b % 2 == 0:
            out.append(Geometry(n_chan=768, n_dm=1024, dm_first=0.0, dm_step=0.5))
        else:
            out.append(Geometry(n_chan=1536, n_dm=2048, dm_first=0.0, dm_step=0.5))
    return out


def poisson_arrivals(n_beams: int, rate_per_beam: float, duration_s: float, seed: int = 5):
    """Arrival times of chunks: each beam an independent Poisson process of
    `rate_per_beam` chunks/s over [0, duration_s), its chunks in order.
    Returns a list of (time_s, beam, seq) sorted by time."""
    rng = np.random.default_rng(seed)
    ev = []
    for b in range(n_beams):
        t, seq = 0.0, 0
        while True:
            t += float(rng.exponential(1.0 / rate_per_beam))
            if t >= duration_s:
                break
            ev.append((t, b, seq))
            seq += 1
    ev.sort()
    return ev


# --- downsampling --------------------------------------------------------------

# Nine decimation factors spanning Table 2's 10 ... 3200 (doubling from 10, then
# the largest), plus factor 1: the S/N of the series itself.
DOWNSAMPLING_FACTORS = (1, 10, 20, 40, 80, 160, 320, 640, 1280, 3200)
