"""Decimating downsampling on the device against the oracle.

The decimated series (sums of f consecutive samples starting at multiples of
f, n_out // f of them) must match bit for bit; their S/N within 1e-5
relative with peak indices (in decimated samples) exact.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

SNR_RTOL = 1e-5


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def amber():
    import paper_1811_04165_amd as amber
    return amber


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


@pytest.fixture(scope="module")
def small_dd():
    wl = workloads.small()
    g = wl.geom
    d, mx = oracle.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    x, n_in = workloads.make_input(wl, d, mx)
    return wl, oracle.dedisperse(d, x, n_in, wl.n_out)


def _oracle(dd, factors):
    ys, ss, ps = [], [], []
    for f in factors:
        y = oracle.downsample(dd, f)
        s, p = oracle.snr(y)
        ys.append(y)
        ss.append(s)
        ps.append(p)
    return ys, np.array(ss), np.array(ps)


def _check(amber, torch, dd, n_out, factors, tiles=None):
    ys, ref_s, ref_p = _oracle(dd, factors)
    ddd = torch.from_numpy(np.ascontiguousarray(dd)).cuda()
    y = amber.downsample(ddd, n_out, factors, tiles=tiles).cpu().numpy()
    for k, f in enumerate(factors):
        assert np.array_equal(y[k, :, :n_out // f], ys[k]), f
    s, p = amber.downsample_snr(ddd, n_out, factors, tiles=tiles)
    s, p = s.cpu().numpy(), p.cpu().numpy()
    np.testing.assert_allclose(s.astype(np.float64), ref_s, rtol=SNR_RTOL, atol=1e-6)
    assert np.array_equal(p, ref_p)
    return s, p


def test_downsample_small_paper_factors(amber, torch, small_dd):
    wl, dd = small_dd
    say("downsample small, factors", workloads.DOWNSAMPLING_FACTORS)
    s, p = _check(amber, torch, dd, wl.n_out, workloads.DOWNSAMPLING_FACTORS)
    # the injected pulse (DM index 50, width 4 at t0 = 4096) is found in the
    # finest decimation at its bin
    pulse = wl.pulses[0]
    k10 = workloads.DOWNSAMPLING_FACTORS.index(10)
    assert int(np.argmax(s[k10])) == pulse.dm_index
    assert p[k10, pulse.dm_index] == pulse.t0 // 10


@pytest.mark.parametrize("threads,step", [(512, 1), (512, [1, 2, 4, 8, 1, 2]), (1024, 8), (1024, 2)])
def test_downsample_invariant_to_tiles(amber, torch, small_dd, threads, step):
    wl, dd = small_dd
    factors = (1, 3, 10, 100, 1000, 3200)
    say("downsample tiles", threads, step)
    _check(amber, torch, dd, wl.n_out, factors, tiles=amber.make_tiles(snr_threads=threads, boxcar_step=step))


DS_EDGE = [
    # n_dm, n_out, factors
    (3, 1, (1,)),
    (5, 17, (1, 2, 5, 17)),
    (9, 1000, (3, 7, 10, 333, 1000)),
    (70, 4099, (10, 20, 40, 80, 160, 320, 640, 1280, 3200)),
    (4, 20000, (1, 2, 3, 5, 7, 11, 13, 64, 100, 999, 1024, 2047, 2048, 3000, 4095, 4096)),
    (64, 12208, workloads.DOWNSAMPLING_FACTORS),
]


@pytest.mark.parametrize("case", DS_EDGE, ids=lambda c: "dm%d-out%d-nf%d" % (c[0], c[1], len(c[2])))
def test_downsample_edge_shapes(amber, torch, case):
    n_dm, n_out, factors = case
    rng = np.random.default_rng(n_out + 7)
    dd = rng.integers(0, 391680, size=(n_dm, n_out)).astype(np.int32)
    dd[0] = 12345                          # constant row: sigma = 0 -> snr 0, peak 0
    if n_out > 40:
        dd[1, 0:10] = dd[1, 20:30] = 391679   # equal decimated maxima (f = 10): the first wins
    say("downsample edge", n_dm, n_out, factors)
    s, p = _check(amber, torch, dd, n_out, factors)
    assert np.all(s[:, 0] == 0.0) and np.all(p[:, 0] == 0)
