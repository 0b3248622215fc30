"""Host side of two-step subband dedispersion (no GPU): the library's FP64
tables against the oracle's, and argument checks that refuse bad calls before
any launch.

The library moves each coarse DM's k = 0 step-two shift B[j][s] into step one;
its tables minus / plus that shift must equal the oracle's tables bit for bit,
so every composed delay is the scheme's."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads

BEAM = workloads.beam().geom
GRIDS = [  # (n_sub, n_coarse, coarse_first, coarse_step, n_fine, fine_first, fine_step)
    (32, 128, 0.0, 8.0, 16, 0.0, 0.5),     # the 1536-channel beam's 2048 trials
    (32, 2048, 0.0, 2.4, 24, 0.0, 0.1),    # Table 2's subbanding DM grid
    (8, 20, 3.0, 1.7, 5, -1.0, 0.3),       # offset fine grid below each coarse DM
    (1536, 4, 0.0, 16.0, 32, 0.0, 0.5),    # one channel per subband
    (6, 3, 0.0, 0.0, 7, 0.0, 2.0),         # coarse step 0
]


def _lib_and_oracle(f, t_samp, grid):
    import paper_1811_04165_amd as amber
    d1, d2, info = amber.subband_delay_tables(f, t_samp, *grid)
    o1, o2, _, _ = oracle.subband_delays(f, t_samp, *grid)
    return d1, d2, info, o1, o2


@pytest.mark.parametrize("grid", GRIDS, ids=lambda g: "sub%d-c%d-f%d" % (g[0], g[1], g[4]))
def test_subband_tables_match_oracle(grid):
    d1, d2, info, o1, o2 = _lib_and_oracle(BEAM.freqs(), BEAM.t_samp_s, grid)
    b = o2[:, 0, :]                                    # B[j][s], the k = 0 shift
    assert np.array_equal(d1 - b.T[:, :, None], o1)
    assert np.array_equal(d2 + b[:, None, :], o2)
    assert (d1 >= 0).all() and (d2 >= 0).all() and (d2[:, 0, :] == 0).all()
    assert info.max_delay1 == d1.max() and info.max_delay2 == d2.max()
    assert info.max_delay == info.max_delay1 + info.max_delay2
    assert info.max_step1 == (np.diff(d1, axis=1).max() if d1.shape[1] > 1 else 0)
    assert info.max_step2 == (np.diff(d2, axis=1).max() if d2.shape[1] > 1 else 0)
    assert (np.diff(d1, axis=1) >= 0).all() and (np.diff(d2, axis=1) >= 0).all()
    assert (info.n_chan, info.n_subbands, info.n_coarse, info.n_fine) == (BEAM.n_chan, grid[0], grid[1], grid[4])


def test_subband_tables_random_geometries():
    rng = np.random.default_rng(31)
    for _ in range(15):
        n_sub = int(rng.integers(1, 9))
        m = int(rng.integers(1, 40))
        f = rng.uniform(200.0, 2000.0, size=n_sub * m)
        grid = (n_sub, int(rng.integers(1, 12)), float(rng.uniform(0, 30)), float(rng.uniform(0, 6)),
                int(rng.integers(1, 9)), float(rng.uniform(-2, 2)), float(rng.uniform(0, 1)))
        if grid[2] + grid[5] < 0:
            continue
        t_samp = float(rng.uniform(2e-5, 5e-4))
        d1, d2, info, o1, o2 = _lib_and_oracle(f, t_samp, grid)
        b = o2[:, 0, :]
        assert np.array_equal(d1 - b.T[:, :, None], o1) and np.array_equal(d2 + b[:, None, :], o2)


def test_subband_tables_reject_bad_geometry():
    import paper_1811_04165_amd as amber
    f = BEAM.freqs()
    bad = [(5, 4, 0.0, 1.0, 2, 0.0, 0.5),        # 5 does not divide 1536
           (4, 4, 0.0, 1.0, 2, 0.0, 0.5),        # 384 channels per subband > 257
           (32, 0, 0.0, 1.0, 2, 0.0, 0.5),       # no coarse DMs
           (32, 4, 0.0, 1.0, 0, 0.0, 0.5),       # no fine DMs
           (32, 4, -1.0, 1.0, 2, 0.0, 0.5),      # negative coarse DM
           (32, 4, 0.0, -1.0, 2, 0.0, 0.5),      # negative coarse step
           (32, 4, 0.0, 1.0, 2, 0.0, -0.5),      # negative fine step
           (32, 4, 1.0, 1.0, 2, -2.0, 0.5)]      # first trial DM below 0
    for grid in bad:
        with pytest.raises(amber.AmberError) as e:
            amber.subband_delay_tables(f, BEAM.t_samp_s, *grid)
        assert e.value.status == -1, grid
    with pytest.raises(amber.AmberError):
        amber.subband_delay_tables(f, 0.0, *GRIDS[0])


def test_subband_dedisperse_validates_before_launch():
    """Every call here is refused on the host, so none reaches a GPU."""
    from paper_1811_04165_amd import _lib
    import paper_1811_04165_amd as amber
    lib = _lib.load()
    _, _, info = amber.subband_delay_tables(BEAM.freqs()[:64], BEAM.t_samp_s, 8, 4, 0.0, 8.0, 4, 0.0, 2.0)
    p = ctypes.c_void_p(0x1000)
    n_out = 1000
    n_in = n_out + info.max_delay
    stride = (n_in + 127) // 128 * 128
    ws = n_out + info.max_delay2 + (n_out + info.max_delay2) % 2

    def call(**kw):
        a = dict(d1=p, d2=p, info=ctypes.byref(info), x=p, stride=stride, n_in=n_in, work=p, ws=ws, dd=p,
                 dds=n_out, n_out=n_out, keep=None, t1=None, t2=None)
        a.update(kw)
        return lib.amber_subband_dedisperse(a["d1"], a["d2"], a["info"], a["x"], a["stride"], a["n_in"], a["work"],
                                            a["ws"], a["dd"], a["dds"], a["n_out"], a["keep"], a["t1"], a["t2"], None)

    assert call(n_in=n_in - 1) == -2 and b"max_delay" in lib.amber_last_error()
    assert call(ws=ws - 2) == -2 and b"work_stride" in lib.amber_last_error()
    assert call(ws=ws + 1) == -2                                  # odd uint16 row stride
    assert call(work=ctypes.c_void_p(0x1002)) == -1               # misaligned scratch
    assert call(x=None) == -1 and call(work=None) == -1 and call(d2=None) == -1
    assert call(dds=n_out - 1) == -2
    assert call(stride=stride + 2) == -2
    bad = _lib.SubbandInfo(**{n: getattr(info, n) for n, _ in info._fields_})
    bad.max_delay = info.max_delay - 1
    assert call(info=ctypes.byref(bad)) == -1
    bad.max_delay, bad.n_subbands = info.max_delay, 7
    assert call(info=ctypes.byref(bad)) == -1
    # step two's kernels take samples_per_thread 8 or 16 and channel_unroll >= 4
    for kw in (dict(channel_unroll=2), dict(samples_per_thread=4), dict(samples_per_thread=32)):
        t2 = amber.make_tiles(**{"dms_per_thread": 1, **kw})
        assert call(t2=ctypes.byref(t2)) == -3, kw
    assert call(t1=ctypes.byref(amber.make_tiles(threads_per_dm=96))) == -3


def test_gpu_test_tiles_are_valid():
    """Every tile pair the GPU subband tests launch passes host planning for
    the small grid (step one: its subbands' channels and coarse DMs; step two:
    the subbands and fine DMs, with the 16-bit-input limits)."""
    import os
    import sys
    import paper_1811_04165_amd as amber
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import test_subband_gpu as t
    g = t.SMALL
    _, _, info = amber.subband_delay_tables(g.freqs(), g.t_samp_s, *t.SMALL_GRID)
    m = info.n_chan // info.n_subbands
    i1 = amber.DelayInfo(n_dm=info.n_coarse, n_chan=m, max_delay=info.max_delay1, max_step=info.max_step1)
    # step two's window: offsets up to (dms_per_block - 1) * max_step2 + 1, no
    # larger than the uint8 planner's + 3, so its check is a sufficient one
    i2 = amber.DelayInfo(n_dm=info.n_fine, n_chan=info.n_subbands, max_delay=info.max_delay2,
                         max_step=info.max_step2)
    for a, b in t.TILES:
        if a is None:
            continue
        amber.validate_tiles(amber.make_tiles(**{"dms_per_thread": 1, **a}), i1, 1)
        amber.validate_tiles(amber.make_tiles(**{"dms_per_thread": 1, **b}), i2, 1)
        assert b["samples_per_thread"] in (8, 16) and b["channel_unroll"] >= 4
