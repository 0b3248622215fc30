"""Dedispersion with zapped (RFI) channels on the device against the oracle.

The masked sums must match the oracle's masked dedispersion bit for bit, for
several tile configurations (including channel groups that straddle zapped
and kept channels) and on sampled DM rows of the full beam.  A functional
check: a band of saturated interference hides an injected pulse from the
S/N search until the band is zapped.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


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


RFI_TILES = [None,
             dict(threads_per_dm=64, samples_per_thread=8, dms_per_block=16, channel_unroll=32),
             dict(threads_per_dm=128, samples_per_thread=4, dms_per_block=4, channel_unroll=8),
             dict(threads_per_dm=64, samples_per_thread=16, dms_per_block=3, channel_unroll=1),
             dict(threads_per_dm=64, samples_per_thread=8, dms_per_block=5, channel_unroll=16, dms_per_thread=2),
             # direct reads: zapped channels get the all-zero selector
             dict(threads_per_dm=64, samples_per_thread=8, dms_per_block=3, channel_unroll=16, direct_reads=1),
             dict(threads_per_dm=128, samples_per_thread=4, dms_per_block=2, channel_unroll=32, direct_reads=1)]


@pytest.mark.parametrize("kw", RFI_TILES, ids=lambda k: "auto" if k is None else
                         "tpd%(threads_per_dm)d-spt%(samples_per_thread)d-dpb%(dms_per_block)d-cu%(channel_unroll)d" % k
                         + ("-dpt%d" % k["dms_per_thread"] if "dms_per_thread" in k else "")
                         + ("-direct" if k.get("direct_reads") else ""))
def test_masked_small(amber, torch, kw):
    wl = workloads.small()
    g = wl.geom
    d, mx = oracle.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    x, n_in = workloads.make_input(wl, d, mx)
    keep = (np.random.default_rng(41).random(g.n_chan) >= 0.15).astype(np.uint8)
    keep[:3] = 0
    keep[-1] = 0
    ref = oracle.dedisperse_masked(d, x, n_in, wl.n_out, keep)
    _, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    say("masked small", kw, "zapped", int((keep == 0).sum()))
    tiles = amber.make_tiles(**{"dms_per_thread": 1, **kw}) if kw else None
    got = amber.dedisperse(torch.from_numpy(d).cuda(), info, torch.from_numpy(x).cuda(), n_in, wl.n_out, tiles,
                           keep=torch.from_numpy(keep).cuda())
    assert np.array_equal(got.cpu().numpy(), ref)


def test_masked_beam_sampled(amber, torch):
    wl = workloads.beam()
    g = wl.geom
    d, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    x, n_in = workloads.make_input(wl, d, info.max_delay)
    keep = np.ones(g.n_chan, np.uint8)
    keep[700:850] = 0                        # a contiguous band, as interference usually occupies
    keep[np.random.default_rng(42).choice(g.n_chan, 40, replace=False)] = 0
    say("masked beam full size, zapped", int((keep == 0).sum()))
    got = amber.dedisperse(torch.from_numpy(d).cuda(), info, torch.from_numpy(x).cuda(), n_in, wl.n_out,
                           keep=torch.from_numpy(keep).cuda()).cpu().numpy()
    rows = sorted(set([0, 5, g.n_dm - 1] + [p.dm_index for p in wl.pulses] +
                      list(np.random.default_rng(43).choice(g.n_dm, size=12, replace=False))))
    assert np.array_equal(got[rows], oracle.dedisperse_masked(d[rows], x, n_in, wl.n_out, keep))
    # DM 0 is the sum of the kept channels
    assert np.array_equal(got[0], x[keep == 1, :wl.n_out].astype(np.int64).sum(axis=0))


def test_zapping_removes_interference(amber, torch):
    """Saturated interference in 24 channels over 300 samples outshines a weak
    pulse (DM index 50, +12 counts); zapping those channels recovers it."""
    wl = workloads.small()
    g = wl.geom
    d, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    n_in = wl.n_out + info.max_delay
    x = workloads.noise(g.n_chan, n_in, workloads.padded_stride(n_in), seed=44)
    workloads.inject(x, d[50], t0=4096, width=4, amp=12)
    x[100:124, 6000:6300] = 255              # interference, not dispersed
    keep = np.ones(g.n_chan, np.uint8)
    keep[100:124] = 0
    dd_dev = torch.from_numpy(d).cuda()
    x_dev = torch.from_numpy(x).cuda()
    widths = (1, 2, 4, 8, 16)
    say("interference: plain vs zapped")
    best = {}
    for name, k in (("plain", None), ("zapped", torch.from_numpy(keep).cuda())):
        dd = amber.dedisperse(dd_dev, info, x_dev, n_in, wl.n_out, keep=k)
        s, p = amber.integrate_snr(dd, wl.n_out, widths)
        best[name] = oracle.best_candidate(s.cpu().numpy())
    assert best["plain"][0] != 50            # the interference wins the search
    assert best["zapped"][0] == 50 and best["zapped"][2] > 8.0
