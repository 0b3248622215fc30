"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every function include/amber.h declares, the FP64 delay table matches
the oracle bit for bit, and arguments are validated before any launch."""
import ast
import ctypes
import os
import re
import sys

import numpy as np
import pytest

import oracle
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if hdr.endswith(".h"):
            text = open(os.path.join(ROOT, "include", hdr)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^[A-Za-z_][\w \*]*?\b(amber_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_process_holds_one_hip_runtime():
    """Loading the library first and torch afterwards still leaves a single HIP
    runtime mapped into the process (the library binds to torch's copy)."""
    import subprocess
    code = ("import paper_1811_04165_amd as a; a._lib.load(); import torch; "
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    mapped = ast.literal_eval(r.stdout.strip().splitlines()[-1])
    assert len(mapped) == 1, mapped


def test_library_exports_every_declared_symbol():
    import paper_1811_04165_amd as amber
    from paper_1811_04165_amd import _lib
    lib = _lib.load()
    declared = _declared_functions()
    assert len(declared) >= 9
    for name in declared:
        assert hasattr(lib, name), name
    bound = {s[0] for s in _lib.SIGNATURES}
    assert set(declared) <= bound, set(declared) - bound
    assert "gfx950" in amber.version()


@pytest.mark.parametrize("wl", [workloads.small(), workloads.beam()] + workloads.batch_beams(3),
                         ids=lambda w: w.name)
def test_delay_table_bit_exact_vs_oracle(wl):
    import paper_1811_04165_amd as amber
    g = wl.geom
    d, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    do, mx = oracle.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    assert np.array_equal(d, do)
    assert info.max_delay == mx and info.n_dm == g.n_dm and info.n_chan == g.n_chan
    assert info.max_step == int(np.diff(do, axis=0).max())


def test_delay_table_random_geometries():
    import paper_1811_04165_amd as amber
    rng = np.random.default_rng(3)
    for _ in range(20):
        n_chan = int(rng.integers(1, 64))
        f = rng.uniform(100.0, 3000.0, size=n_chan)
        t_samp = float(rng.uniform(1e-5, 1e-3))
        n_dm = int(rng.integers(1, 40))
        first, step = float(rng.uniform(0, 50)), float(rng.uniform(0, 3))
        d, info = amber.delay_table(f, t_samp, n_dm, first, step)
        do, mx = oracle.delay_table(f, t_samp, n_dm, first, step)
        assert np.array_equal(d, do) and info.max_delay == max(mx, 0)


def test_delay_table_rejects_bad_geometry():
    import paper_1811_04165_amd as amber
    with pytest.raises(amber.AmberError):
        amber.delay_table(np.array([1000.0, 0.0]), 1e-4, 4, 0.0, 1.0)
    with pytest.raises(amber.AmberError):
        amber.delay_table(np.array([1000.0]), 1e-4, 4, -1.0, 1.0)
    with pytest.raises(amber.AmberError):
        amber.delay_table(np.array([1000.0]), 0.0, 4, 0.0, 1.0)


def test_tile_validation():
    import paper_1811_04165_amd as amber
    info = amber.DelayInfo(n_dm=2048, n_chan=1536, max_delay=11593, max_step=6)
    amber.validate_tiles(amber.default_tiles(), info, 7)
    bad = [dict(threads_per_dm=32), dict(threads_per_dm=96), dict(samples_per_thread=3),
           dict(samples_per_thread=2), dict(samples_per_thread=64), dict(channel_unroll=32, dms_per_block=1), dict(dms_per_block=32, threads_per_dm=64),
           dict(channel_unroll=3), dict(channel_unroll=64), dict(snr_threads=48), dict(boxcar_step=3),
           dict(threads_per_dm=1024, samples_per_thread=16, channel_unroll=16),
           dict(dms_per_thread=3), dict(dms_per_thread=2, samples_per_thread=32, dms_per_block=4),
           dict(dms_per_thread=-1),
           # direct reads: 0 or 1, one DM per wavefront, at most 64 dwords loaded per channel group
           dict(direct_reads=2), dict(direct_reads=-1), dict(direct_reads=1, dms_per_thread=2),
           dict(direct_reads=1, dms_per_thread=1, samples_per_thread=32, channel_unroll=8),
           dict(direct_reads=1, dms_per_thread=1, samples_per_thread=8, channel_unroll=32)]
    for kw in bad:
        with pytest.raises(amber.AmberError) as e:
            amber.validate_tiles(amber.make_tiles(**kw), info, 7)
        assert e.value.status == -3, kw
    # direct reads use no LDS: tiles whose staging would not fit are valid
    for kw in (dict(samples_per_thread=4, channel_unroll=32), dict(samples_per_thread=8, channel_unroll=16),
               dict(samples_per_thread=32, channel_unroll=4), dict(samples_per_thread=4, channel_unroll=32, dms_per_block=1),
               dict(threads_per_dm=1024, samples_per_thread=16, channel_unroll=8, dms_per_block=1)):
        amber.validate_tiles(amber.make_tiles(direct_reads=1, dms_per_thread=1, **kw), info, 7)


def test_device_calls_validate_before_launch():
    """Invalid arguments are refused on the host, so these never reach a GPU."""
    from paper_1811_04165_amd import _lib
    from paper_1811_04165_amd import make_tiles as amber_tiles
    lib = _lib.load()
    info = _lib.DelayInfo(n_dm=4, n_chan=8, max_delay=10, max_step=2)
    fake = ctypes.c_void_p(0x1000)
    # n_in < n_out + max_delay
    rc = lib.amber_dedisperse(fake, ctypes.byref(info), fake, 128, 100, fake, 100, 95, None, None)
    assert rc == -2 and b"max_delay" in lib.amber_last_error()
    # stride not a multiple of 4
    rc = lib.amber_dedisperse(fake, ctypes.byref(info), fake, 130, 120, fake, 100, 100, None, None)
    assert rc == -2
    # NULL input
    rc = lib.amber_dedisperse(fake, ctypes.byref(info), None, 128, 120, fake, 100, 100, None, None)
    assert rc == -1
    # channel_unroll x row stride past 2^32: the staged kernel's 32-bit offsets within a channel group
    t = amber_tiles(channel_unroll=16)
    big = (1 << 28) + 128
    rc = lib.amber_dedisperse(fake, ctypes.byref(info), fake, big, 120, fake, 100, 100, ctypes.byref(t), None)
    assert rc == -2 and b"2^32" in lib.amber_last_error()
    t_direct = amber_tiles(channel_unroll=16, direct_reads=1, dms_per_thread=1)
    rc = lib.amber_dedisperse(fake, ctypes.byref(info), fake, big, 120, fake, 100, 0, ctypes.byref(t_direct), None)
    assert rc == 0       # n_out = 0: checked, nothing launched; the direct kernel has no such limit
    # masked: NULL keep flags, and the plain checks still apply
    rc = lib.amber_dedisperse_masked(fake, ctypes.byref(info), fake, 128, 120, fake, 100, 100, None, None, None)
    assert rc == -1 and b"d_keep" in lib.amber_last_error()
    rc = lib.amber_dedisperse_masked(fake, ctypes.byref(info), fake, 128, 100, fake, 100, 95, fake, None, None)
    assert rc == -2
    w = (ctypes.c_int32 * 2)(1, 200)
    rc = lib.amber_integrate_snr(fake, 4, 100, 100, w, 2, fake, fake, None, None)
    assert rc == -1 and b"widths" in lib.amber_last_error()
    rc = lib.amber_integrate(fake, 4, 50, 100, w, 1, fake, 100, None, None)
    assert rc == -2
    rc = lib.amber_snr(fake, 4, 100, 100, w, 0, fake, None, None, None)
    assert rc == -1
    assert lib.amber_last_error() != b""
    rc = lib.amber_default_tiles(None)
    assert rc == -1
    # downsampling: factor beyond n_out, factor beyond 4096, no factors, output rows too short
    f = (ctypes.c_int32 * 2)(10, 200)
    rc = lib.amber_downsample_snr(fake, 4, 100, 100, f, 2, fake, fake, None, None)
    assert rc == -1 and b"widths" in lib.amber_last_error()
    big = (ctypes.c_int32 * 1)(5000)
    rc = lib.amber_downsample_snr(fake, 4, 10000, 10000, big, 1, fake, fake, None, None)
    assert rc == -1 and b"4096" in lib.amber_last_error()
    rc = lib.amber_downsample_snr(fake, 4, 100, 100, f, 0, fake, fake, None, None)
    assert rc == -1
    f10 = (ctypes.c_int32 * 1)(10)
    rc = lib.amber_downsample(fake, 4, 100, 100, f10, 1, fake, 9, None, None)
    assert rc == -2 and b"y_stride" in lib.amber_last_error()
    # a zero or negative factor is refused before any division by it
    for bad in (0, -3):
        fb = (ctypes.c_int32 * 2)(10, bad)
        rc = lib.amber_downsample(fake, 4, 100, 100, fb, 2, fake, 100, None, None)
        assert rc == -1 and b"widths[1]" in lib.amber_last_error()
        rc = lib.amber_downsample_snr(fake, 4, 100, 100, fb, 2, fake, fake, None, None)
        assert rc == -1
    rc = lib.amber_downsample(fake, 4, 100, 100, f10, 1, None, 100, None, None)
    assert rc == -1 and b"d_y" in lib.amber_last_error()


def test_binding_rejects_host_and_misshaped_outputs():
    """The Python wrappers refuse host tensors and output tables of the wrong
    dtype or shape before calling the library (a short output would be
    written past its end on the device)."""
    import torch
    import paper_1811_04165_amd as amber
    dd = torch.zeros((4, 100), dtype=torch.int32)
    with pytest.raises(TypeError):
        amber.integrate_snr(dd, 100, [1, 2])
    with pytest.raises(TypeError):
        amber.downsample(dd, 100, [10])
    with pytest.raises(TypeError):
        amber.downsample_snr(dd, 100, [10], out=(torch.zeros((1, 4)), torch.zeros((1, 4), dtype=torch.int32)))
    from paper_1811_04165_amd import _table_out, _check_table

    class _Fake:
        """A stand-in exposing what the checks read of a device tensor."""
        def __init__(self, dtype, shape, device="cuda:0", contiguous=True):
            self.dtype, self.shape, self.device, self._c = dtype, shape, device, contiguous
            self.is_cuda = True

        def dim(self):
            return len(self.shape)

        def stride(self, k):
            return 1

        def is_contiguous(self):
            return self._c

    import paper_1811_04165_amd as pkg
    real = torch.Tensor
    try:
        torch.Tensor = _Fake  # isinstance checks in the binding see the stand-in as a tensor
        ok = _Fake(torch.float32, (2, 4))
        _check_table(ok, torch.float32, "snr out", 2, 4, "cuda:0")
        for bad, exc in ((_Fake(torch.float64, (2, 4)), TypeError), (_Fake(torch.float32, (1, 4)), ValueError),
                         (_Fake(torch.float32, (2, 4), contiguous=False), ValueError),
                         (_Fake(torch.float32, (2, 4), device="cuda:1"), ValueError)):
            with pytest.raises(exc):
                _check_table(bad, torch.float32, "snr out", 2, 4, "cuda:0")
        with pytest.raises(TypeError):
            _table_out((_Fake(torch.float32, (2, 4)), _Fake(torch.float32, (2, 4))), 2, 4, "cuda:0")
    finally:
        torch.Tensor = real
    assert pkg is amber


def test_gpu_test_tiles_are_valid():
    """Every tile configuration the GPU parity tests launch passes host
    validation for the geometries it is used with."""
    import paper_1811_04165_amd as amber
    import test_parity_gpu as t
    for wl in (workloads.small(), workloads.beam()):
        g = wl.geom
        _, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
        amber.validate_tiles(amber.default_tiles(), info, len(wl.widths))
        assert amber.auto_tiles(info).as_dict() == amber.default_tiles().as_dict()
        for kw in t.TILE_SWEEP:
            amber.validate_tiles(amber.make_tiles(**{"dms_per_thread": 1, **kw}), info, len(wl.widths))
    for k, wl in enumerate(t._small_batch_workloads()):
        g = wl.geom
        _, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
        amber.validate_tiles(amber.make_tiles(samples_per_thread=8 if k % 2 else 16, channel_unroll=16), info,
                             len(wl.widths))
    for n_chan, n_dm, n_out, step, pad in t.ODD:
        freqs = t.odd_freqs(n_chan, n_dm)
        _, info = amber.delay_table(freqs, 81.92e-6, n_dm, 1.5, step)
        for kw in t.ODD_TILES:
            amber.validate_tiles(amber.make_tiles(**{"dms_per_thread": 1, **kw}) if kw else amber.auto_tiles(info), info, 1)


def test_auto_tiles_fills_small_grids():
    """With a series length, the automatic tiles shrink until the dedispersion
    launch has at least 384 work-groups (1.5 per CU) or no step is left, and
    stay valid; large problems keep the defaults, and n_out = 0 skips it."""
    import paper_1811_04165_amd as amber

    def blocks(t, n_dm, n_out):
        tile_t = t.threads_per_dm * t.samples_per_thread
        dms = t.dms_per_block * max(1, t.dms_per_thread)
        return -(-n_out // tile_t) * -(-n_dm // dms)

    d = amber.default_tiles().as_dict()
    wl = workloads.small()
    g = wl.geom
    _, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    t = amber.auto_tiles(info, wl.n_out)
    # 64 work-groups by default; 4 samples per work-item (128), one DM per wavefront (256)
    assert (t.samples_per_thread, t.channel_unroll, t.dms_per_thread, t.dms_per_block) == (4, 32, 1, d["dms_per_block"])
    assert blocks(t, g.n_dm, wl.n_out) == 256
    assert amber.auto_tiles(info, 0).as_dict() == d
    for k, v in t.as_dict().items():
        if k not in ("samples_per_thread", "channel_unroll", "dms_per_thread"):
            assert v == d[k], k
    wl = workloads.beam()
    g = wl.geom
    _, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    assert amber.auto_tiles(info, wl.n_out).as_dict() == d
    # shapes from tiny to large: valid, and filled unless no step is left
    for n_chan, n_dm, n_out in ((64, 1, 100), (256, 64, 4096), (384, 512, 4096), (768, 512, 4472),
                                (1536, 1024, 5456), (384, 512, 13400), (1536, 2048, 100000)):
        freqs = 1250.0 + np.arange(n_chan) * (300.0 / n_chan)
        _, info = amber.delay_table(freqs, 81.92e-6, n_dm, 0.0, 0.5)
        t = amber.auto_tiles(info, n_out)
        amber.validate_tiles(t, info, 1)
        base = amber.auto_tiles(info, 0)
        if blocks(base, n_dm, n_out) >= 384:
            assert t.as_dict() == base.as_dict()
        else:
            assert blocks(t, n_dm, n_out) >= 384 or (t.samples_per_thread == 4 and t.dms_per_thread == 1)
    from paper_1811_04165_amd._lib import load
    assert load().amber_auto_tiles(None, 10, None) == -1  # AMBER_E_ARG
