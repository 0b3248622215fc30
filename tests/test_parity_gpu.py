"""Parity of the HIP hot path against the CPU oracle, element by element.

Dedispersion and boxcar series must match bit for bit; S/N within 1e-5
relative (FP64 moments finished on the device, stored as float32); peak
indices exactly (both sides take the first maximum).  Every device call goes
through the C ABI via the binding.
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


def _geom_case(wl):
    g = wl.geom
    d, mx = oracle.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    x, n_in = workloads.make_input(wl, d, mx)
    return d, mx, x, n_in


@pytest.fixture(scope="module")
def small_case():
    wl = workloads.small()
    d, mx, x, n_in = _geom_case(wl)
    dd = oracle.dedisperse(d, x, n_in, wl.n_out)
    return wl, d, mx, x, n_in, dd


def _device_dedisperse(amber, torch, wl, x, n_in, n_out, tiles=None, dm_step=None):
    g = wl.geom
    d, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step if dm_step is None else dm_step)
    dev = torch.from_numpy(d).cuda()
    xd = torch.from_numpy(x).cuda()
    out = amber.dedisperse(dev, info, xd, n_in, n_out, tiles=tiles)
    torch.cuda.synchronize()
    return out.cpu().numpy(), d, info


def test_dedisperse_small_default(amber, torch, small_case):
    wl, d, mx, x, n_in, dd = small_case
    say("dedisperse small default tiles")
    got, dt, info = _device_dedisperse(amber, torch, wl, x, n_in, wl.n_out)
    assert np.array_equal(dt, d) and info.max_delay == mx
    assert np.array_equal(got, dd)


TILE_SWEEP = [
    dict(threads_per_dm=64, samples_per_thread=4, dms_per_block=1, channel_unroll=1),
    dict(threads_per_dm=64, samples_per_thread=4, dms_per_block=16, channel_unroll=16),
    dict(threads_per_dm=128, samples_per_thread=8, dms_per_block=4, channel_unroll=2),
    dict(threads_per_dm=256, samples_per_thread=16, dms_per_block=2, channel_unroll=4),
    dict(threads_per_dm=1024, samples_per_thread=4, dms_per_block=1, channel_unroll=2),
    dict(threads_per_dm=512, samples_per_thread=8, dms_per_block=2, channel_unroll=1),
    dict(threads_per_dm=64, samples_per_thread=16, dms_per_block=8, channel_unroll=8),
    dict(threads_per_dm=64, samples_per_thread=16, dms_per_block=16, channel_unroll=16),
    dict(threads_per_dm=192, samples_per_thread=8, dms_per_block=5, channel_unroll=4),
    dict(threads_per_dm=64, samples_per_thread=8, dms_per_block=3, channel_unroll=16),
    dict(threads_per_dm=64, samples_per_thread=32, dms_per_block=16, channel_unroll=4),
    dict(threads_per_dm=64, samples_per_thread=8, dms_per_block=8, channel_unroll=32),
    dict(threads_per_dm=128, samples_per_thread=32, dms_per_block=4, channel_unroll=2),
    # two DMs per wavefront; 128 trials do not fill the last block of 6
    dict(threads_per_dm=64, samples_per_thread=8, dms_per_block=8, channel_unroll=32, dms_per_thread=2),
    dict(threads_per_dm=64, samples_per_thread=4, dms_per_block=3, channel_unroll=16, dms_per_thread=2),
    dict(threads_per_dm=128, samples_per_thread=16, dms_per_block=4, channel_unroll=4, dms_per_thread=2),
    dict(threads_per_dm=256, samples_per_thread=8, dms_per_block=1, channel_unroll=4, dms_per_thread=2),
    # direct reads from global memory (no LDS staging); every samples_per_thread, partial last blocks
    dict(threads_per_dm=64, samples_per_thread=4, dms_per_block=1, channel_unroll=32, direct_reads=1),
    dict(threads_per_dm=64, samples_per_thread=8, dms_per_block=3, channel_unroll=16, direct_reads=1),
    dict(threads_per_dm=128, samples_per_thread=16, dms_per_block=5, channel_unroll=4, direct_reads=1),
    dict(threads_per_dm=256, samples_per_thread=32, dms_per_block=2, channel_unroll=1, direct_reads=1),
    dict(threads_per_dm=1024, samples_per_thread=8, dms_per_block=1, channel_unroll=8, direct_reads=1),
]


def _tile_id(k):
    return ("tpd%(threads_per_dm)d-spt%(samples_per_thread)d-dpb%(dms_per_block)d-cu%(channel_unroll)d" % k +
            ("-dpt%d" % k["dms_per_thread"] if k.get("dms_per_thread", 1) != 1 else "") +
            ("-direct" if k.get("direct_reads") else ""))


@pytest.mark.parametrize("kw", TILE_SWEEP, ids=_tile_id)
def test_dedisperse_invariant_to_tiles(amber, torch, small_case, kw):
    wl, d, mx, x, n_in, dd = small_case
    say("dedisperse small tiles", kw)
    got, _, _ = _device_dedisperse(amber, torch, wl, x, n_in, wl.n_out, tiles=amber.make_tiles(**{"dms_per_thread": 1, **kw}))
    assert np.array_equal(got, dd)


ODD = [
    # n_chan, n_dm, n_out, dm_step, extra stride
    (37, 13, 1000, 3.0, 4),
    (300, 7, 4097, 0.7, 0),
    (1, 1, 129, 0.0, 8),
    (513, 33, 2050, 1.3, 124),
    (16, 65, 127, 2.0, 0),
]


ODD_TILES = [None, dict(threads_per_dm=64, samples_per_thread=4, dms_per_block=3, channel_unroll=16),
             dict(threads_per_dm=128, samples_per_thread=16, dms_per_block=4, channel_unroll=8),
             dict(threads_per_dm=64, samples_per_thread=8, dms_per_block=3, channel_unroll=8, dms_per_thread=2),
             dict(threads_per_dm=64, samples_per_thread=8, dms_per_block=3, channel_unroll=16, direct_reads=1),
             dict(threads_per_dm=128, samples_per_thread=4, dms_per_block=2, channel_unroll=32, direct_reads=1)]


def odd_freqs(n_chan, n_dm):
    rng = np.random.default_rng(n_chan * 1000 + n_dm)
    return np.sort(rng.uniform(1100.0, 1700.0, size=n_chan))[::-1].copy()   # descending, non-uniform


@pytest.mark.parametrize("case", ODD, ids=lambda c: "ch%d-dm%d-out%d" % c[:3])
def test_dedisperse_odd_shapes(amber, torch, case):
    n_chan, n_dm, n_out, step, pad = case
    rng = np.random.default_rng(n_chan * 1000 + n_dm + 1)
    freqs = odd_freqs(n_chan, n_dm)
    d, info = amber.delay_table(freqs, 81.92e-6, n_dm, 1.5, step)
    do, mx = oracle.delay_table(freqs, 81.92e-6, n_dm, 1.5, step)
    assert np.array_equal(d, do)
    n_in = n_out + mx
    stride = (n_in + 3) // 4 * 4 + pad
    x = rng.integers(0, 256, size=(n_chan, stride)).astype(np.uint8)
    ref = oracle.dedisperse(do, x, n_in, n_out)
    dev, xd = torch.from_numpy(d).cuda(), torch.from_numpy(x).cuda()
    for kw in ODD_TILES:
        say("dedisperse odd", case, kw)
        out = amber.dedisperse(dev, info, xd, n_in, n_out, tiles=amber.make_tiles(**{"dms_per_thread": 1, **kw}) if kw else None)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), kw


@pytest.mark.parametrize("case", [(37, 13, 1000, 3.0, 4), (300, 7, 4097, 0.7, 0)], ids=lambda c: "ch%d" % c[0])
def test_dedisperse_reads_only_its_rows(amber, torch, case):
    """The input is a view of rows inside a larger buffer whose other rows hold
    255 everywhere: the staging loads are bounded by the problem's own rows
    (channel groups that run past the last channel read zeros, not the next
    row), so every tile matches the oracle on the view's rows alone."""
    n_chan, n_dm, n_out, step, pad = case
    rng = np.random.default_rng(n_chan * 1000 + n_dm + 2)
    freqs = odd_freqs(n_chan, n_dm)
    d, info = amber.delay_table(freqs, 81.92e-6, n_dm, 1.5, step)
    do, mx = oracle.delay_table(freqs, 81.92e-6, n_dm, 1.5, step)
    n_in = n_out + mx
    stride = (n_in + 3) // 4 * 4 + pad
    big = np.full((n_chan + 7, stride), 255, dtype=np.uint8)
    big[3:3 + n_chan] = rng.integers(0, 256, size=(n_chan, stride)).astype(np.uint8)
    ref = oracle.dedisperse(do, big[3:3 + n_chan], n_in, n_out)
    dev, bd = torch.from_numpy(d).cuda(), torch.from_numpy(big).cuda()
    xd = bd[3:3 + n_chan]
    # the ODD tiles and the beam's default tiles, whose 16-channel groups end
    # 5 (37 channels) or 12 (300) channels into the last group
    for kw in ODD_TILES + [dict(threads_per_dm=64, samples_per_thread=8, dms_per_block=16, channel_unroll=16,
                                dms_per_thread=2)]:
        say("dedisperse rows of a larger buffer", case, kw)
        out = amber.dedisperse(dev, info, xd, n_in, n_out,
                               tiles=amber.make_tiles(**{"dms_per_thread": 1, **kw}) if kw else None)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), kw


@pytest.mark.parametrize("widths", [(1, 2, 4, 8, 16, 32, 64), (1, 1024)], ids=["w1-64", "w1-1024"])
def test_integrate_snr_automatic_tiles_many_rows(amber, torch, widths):
    """tiles = None with 4096 rows or more: single-wave work-groups, or (width
    1024) the larger group the chunk needs; sampled rows against the oracle."""
    n_dm, n_out = 5000, 2100
    rng = np.random.default_rng(5000 + len(widths))
    dd = rng.integers(0, 391680, size=(n_dm, n_out)).astype(np.int32)
    ddd = torch.from_numpy(dd).cuda()
    say("integrate_snr automatic tiles", n_dm, widths)
    s, p = amber.integrate_snr(ddd, n_out, widths)
    rows = np.unique(np.concatenate([[0, 1, 4095, 4096, n_dm - 1], rng.integers(0, n_dm, 60)]))
    _, ref_s, ref_p = _oracle_box_snr(dd[rows], widths)
    _check_snr(s.cpu().numpy()[:, rows], p.cpu().numpy()[:, rows], ref_s, ref_p)


def test_empty_series(amber, torch, small_case):
    """n_out = 0: dedispersion launches nothing and returns an empty table; a
    boxcar or S/N of an empty series is refused (no width fits)."""
    wl, d, mx, x, n_in, dd = small_case
    say("empty series")
    got, _, _ = _device_dedisperse(amber, torch, wl, x, n_in, 0)
    assert got.shape == (wl.geom.n_dm, 0)
    for tiles in (None, amber.make_tiles(dms_per_thread=1, direct_reads=1)):
        got, _, _ = _device_dedisperse(amber, torch, wl, x, n_in, 0, tiles=tiles)
        assert got.shape == (wl.geom.n_dm, 0)
    ddd = torch.from_numpy(dd).cuda()
    with pytest.raises(amber.AmberError) as e:
        amber.integrate_snr(ddd, 0, (1, 2))
    assert e.value.status == -1


def test_dedisperse_saturated_many_channels(amber, torch):
    """All-255 input over 1536 channels: every sum is 391680, exercising the
    16-bit packed accumulators' flush at its limit."""
    n_chan, n_dm, n_out = 1536, 24, 3000
    freqs = workloads.Geometry(n_chan=n_chan, n_dm=n_dm, dm_first=0.0, dm_step=4.0).freqs()
    d, info = amber.delay_table(freqs, 81.92e-6, n_dm, 0.0, 4.0)
    n_in = n_out + info.max_delay
    x = np.full((n_chan, (n_in + 127) // 128 * 128), 255, dtype=np.uint8)
    say("dedisperse saturated 1536 ch")
    out = amber.dedisperse(torch.from_numpy(d).cuda(), info, torch.from_numpy(x).cuda(), n_in, n_out)
    torch.cuda.synchronize()
    assert np.all(out.cpu().numpy() == 1536 * 255)


def test_dedisperse_into_wider_output(amber, torch, small_case):
    """Writes only the first n_out columns of a wider output buffer."""
    wl, d, mx, x, n_in, dd = small_case
    say("dedisperse wide output")
    dev = torch.from_numpy(d).cuda()
    info = amber.DelayInfo(n_dm=d.shape[0], n_chan=d.shape[1], max_delay=mx, max_step=int(np.diff(d, axis=0).max()))
    buf = torch.full((d.shape[0], wl.n_out + 37), -7, dtype=torch.int32, device="cuda")
    amber.dedisperse(dev, info, torch.from_numpy(x).cuda(), n_in, wl.n_out, out=buf[:, :wl.n_out + 37])
    torch.cuda.synchronize()
    b = buf.cpu().numpy()
    assert np.array_equal(b[:, :wl.n_out], dd)
    assert np.all(b[:, wl.n_out:] == -7)


def test_dedisperse_beam_sampled(amber, torch):
    """Full 1536-channel / 2048-DM beam in the benchmark's launch configuration,
    checked on sampled DM rows (including the pulses' rows) against the oracle."""
    wl = workloads.beam()
    g = wl.geom
    d, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    do, mx = oracle.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    assert np.array_equal(d, do)
    x, n_in = workloads.make_input(wl, do, mx)
    say("dedisperse beam full size")
    out = amber.dedisperse(torch.from_numpy(d).cuda(), info, torch.from_numpy(x).cuda(), n_in, wl.n_out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    rng = np.random.default_rng(99)
    rows = sorted(set([0, 1, 7, g.n_dm - 1] + [p.dm_index for p in wl.pulses] +
                      list(rng.choice(g.n_dm, size=24, replace=False))))
    ref = oracle.dedisperse(do[rows], x, n_in, wl.n_out)
    assert np.array_equal(got[rows], ref)
    # properties that hold for every row: sums within [0, n_chan*255], DM 0 = channel sum
    assert got.min() >= 0 and got.max() <= g.n_chan * 255
    assert np.array_equal(got[0], x[:, :wl.n_out].astype(np.int64).sum(axis=0))


# --- boxcar and S/N ----------------------------------------------------------------------

def _oracle_box_snr(dd, widths):
    boxes, snrs, peaks = [], [], []
    for w in widths:
        b = oracle.boxcar(dd, w)
        s, p = oracle.snr(b)
        boxes.append(b)
        snrs.append(s)
        peaks.append(p)
    return boxes, np.array(snrs), np.array(peaks)


def _check_snr(got_s, got_p, ref_s, ref_p):
    np.testing.assert_allclose(got_s.astype(np.float64), ref_s, rtol=SNR_RTOL, atol=1e-6)
    assert np.array_equal(got_p, ref_p)


def test_integrate_and_snr_small(amber, torch, small_case):
    wl, d, mx, x, n_in, dd = small_case
    boxes, ref_s, ref_p = _oracle_box_snr(dd, wl.widths)
    ddd = torch.from_numpy(dd).cuda()
    say("integrate small")
    box = amber.integrate(ddd, wl.n_out, wl.widths)
    torch.cuda.synchronize()
    b = box.cpu().numpy()
    for k, w in enumerate(wl.widths):
        assert np.array_equal(b[k, :, :wl.n_out - w + 1], boxes[k]), w
    say("snr small")
    s, p = amber.snr(box, wl.n_out, wl.widths)
    _check_snr(s.cpu().numpy(), p.cpu().numpy(), ref_s, ref_p)
    say("integrate_snr small")
    s2, p2 = amber.integrate_snr(ddd, wl.n_out, wl.widths)
    _check_snr(s2.cpu().numpy(), p2.cpu().numpy(), ref_s, ref_p)


@pytest.mark.parametrize("threads,step", [(64, 1), (128, 2), (256, 4), (512, 8), (1024, 1), (256, [1, 2, 4, 8, 1])])
def test_integrate_snr_invariant_to_tiles(amber, torch, small_case, threads, step):
    wl, d, mx, x, n_in, dd = small_case
    _, ref_s, ref_p = _oracle_box_snr(dd, wl.widths)
    t = amber.make_tiles(snr_threads=threads, boxcar_step=step)
    say("integrate_snr tiles", threads, step)
    ddd = torch.from_numpy(dd).cuda()
    s, p = amber.integrate_snr(ddd, wl.n_out, wl.widths, tiles=t)
    _check_snr(s.cpu().numpy(), p.cpu().numpy(), ref_s, ref_p)
    box = amber.integrate(ddd, wl.n_out, wl.widths, tiles=t)
    s, p = amber.snr(box, wl.n_out, wl.widths, tiles=t)
    _check_snr(s.cpu().numpy(), p.cpu().numpy(), ref_s, ref_p)


BOX_EDGE = [
    # n_dm, n_out, widths
    (3, 1, (1,)),
    (5, 17, (1, 17)),
    (9, 1000, (3, 7, 100, 1000)),
    (4, 20000, tuple(range(1, 17))),
    (70, 4099, (1, 2, 4, 8, 16, 32, 64)),
    (4, 5000, (1, 512, 1024)),           # the largest sliding width, sums near the int32 limit
]


@pytest.mark.parametrize("case", BOX_EDGE, ids=lambda c: "dm%d-out%d-nw%d" % (c[0], c[1], len(c[2])))
def test_integrate_snr_edge_shapes(amber, torch, case):
    n_dm, n_out, widths = case
    rng = np.random.default_rng(n_out)
    # values up to the largest 1536-channel sum, or (largest widths) up to
    # 2e6, so that width-1024 sums reach 2.05e9 < 2^31
    hi = 2_000_000 if max(widths) >= 512 else 391680
    dd = rng.integers(0, hi, size=(n_dm, n_out)).astype(np.int32)
    dd[0] = 12345                        # constant row: sigma = 0 -> snr 0, peak 0
    if n_out > 10:
        dd[1, 3] = dd[1, 9] = 400000     # tie: the first maximum wins
    boxes, ref_s, ref_p = _oracle_box_snr(dd, widths)
    ddd = torch.from_numpy(dd).cuda()
    say("box edge", case)
    s, p = amber.integrate_snr(ddd, n_out, widths)
    _check_snr(s.cpu().numpy(), p.cpu().numpy(), ref_s, ref_p)
    box = amber.integrate(ddd, n_out, widths)
    b = box.cpu().numpy()
    for k, w in enumerate(widths):
        assert np.array_equal(b[k, :, :n_out - w + 1], boxes[k]), w
    s, p = amber.snr(box, n_out, widths)
    _check_snr(s.cpu().numpy(), p.cpu().numpy(), ref_s, ref_p)
    assert np.all(s.cpu().numpy()[:, 0] == 0.0) and np.all(p.cpu().numpy()[:, 0] == 0)


# --- the whole path -----------------------------------------------------------------------

def test_search_small_recovers_pulse(amber, torch, small_case):
    wl, d, mx, x, n_in, dd = small_case
    g = wl.geom
    say("search small")
    s = amber.Search(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step, wl.n_out, wl.widths)
    xd = torch.from_numpy(x).cuda()
    got_dd, got_s, got_p = s.run(xd)
    torch.cuda.synchronize()
    _, ref_s, ref_p = _oracle_box_snr(dd, wl.widths)
    assert np.array_equal(got_dd.cpu().numpy(), dd)
    _check_snr(got_s.cpu().numpy(), got_p.cpu().numpy(), ref_s, ref_p)
    i, k, best = oracle.best_candidate(got_s.cpu().numpy().astype(np.float64))
    assert (i, wl.widths[k]) == (wl.pulses[0].dm_index, wl.pulses[0].width)
    # a second run on the same buffers is identical (no races, no stale state)
    dd2, s2, p2 = [t.clone() for t in s.run(xd)]
    torch.cuda.synchronize()
    assert np.array_equal(dd2.cpu().numpy(), dd)
    assert np.array_equal(s2.cpu().numpy(), got_s.cpu().numpy())


def test_search_beam_sampled_snr(amber, torch):
    """Full beam through dedisperse + fused boxcar/S/N (the benchmark's step);
    S/N of sampled rows against the oracle, and the five pulses found."""
    wl = workloads.beam()
    g = wl.geom
    do, mx = oracle.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    x, n_in = workloads.make_input(wl, do, mx)
    say("search beam full size")
    s = amber.Search(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step, wl.n_out, wl.widths)
    dd, sn, pk = s.run(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    sn, pk = sn.cpu().numpy(), pk.cpu().numpy()
    rows = sorted(set([0, g.n_dm - 1] + [p.dm_index for p in wl.pulses] + list(range(100, 2048, 211))))
    ref_dd = oracle.dedisperse(do[rows], x, n_in, wl.n_out)
    _, ref_s, ref_p = _oracle_box_snr(ref_dd, wl.widths)
    _check_snr(sn[:, rows], pk[:, rows], ref_s, ref_p)
    for p in wl.pulses:
        # each pulse's own DM row peaks at its position with a strong S/N
        k = list(wl.widths).index(p.width)
        assert sn[k, p.dm_index] > 8.0
        assert abs(int(pk[k, p.dm_index]) - p.t0) <= p.width


# --- tile search on the device ----------------------------------------------------------

def test_tune_on_device_keeps_parity(amber, torch, small_case):
    """A short GA on the device returns a valid configuration; the hot path run
    with it still matches the oracle bit for bit (and S/N within 1e-5)."""
    wl, d, mx, x, n_in, dd = small_case
    g = wl.geom
    dt, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    sp = amber.default_space(info, wl.widths, wl.n_out)
    dev, xd = torch.from_numpy(dt).cuda(), torch.from_numpy(x).cuda()
    say("tune small GA pop 8 x 3 generations")
    res = amber.tune(sp, dev, xd, n_in, amber.tune_params("ga", pop=8, generations=3, seed=11))
    torch.cuda.synchronize()
    assert res.n_evals > 0 and res.best_time_s > 0
    amber.validate_tiles(res.best, info, len(wl.widths))
    got = amber.dedisperse(dev, info, xd, n_in, wl.n_out, tiles=res.best)
    s, p = amber.integrate_snr(got, wl.n_out, wl.widths, tiles=res.best)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), dd)
    _, ref_s, ref_p = _oracle_box_snr(dd, wl.widths)
    _check_snr(s.cpu().numpy(), p.cpu().numpy(), ref_s, ref_p)


# --- batched beams -------------------------------------------------------------------------

def _small_batch_workloads():
    """Uneven beams (channels, samples and DM trials differ) small enough for
    the oracle: same recipe as the 40-beam workload at reduced sizes."""
    out = []
    for b, (n_chan, n_out, n_dm) in enumerate([(96, 1500, 40), (192, 2300, 24), (96, 1100, 40), (48, 3001, 17),
                                                 (192, 777, 33), (384, 1800, 12)]):
        out.append(workloads.Workload(
            name="b%d" % b, geom=workloads.Geometry(n_chan=n_chan, n_dm=n_dm, dm_first=0.0, dm_step=2.0),
            n_out=n_out, widths=(1, 2, 4, 8, 16),
            pulses=(workloads.Pulse(dm_index=n_dm // 2, width=4, amp=50, t0=n_out // 2),), seed=900 + b))
    return out


def test_batched_beams_match_single_beams(amber, torch):
    widths = (1, 2, 4, 8, 16)
    beams, refs = [], []
    for wl in _small_batch_workloads():
        g = wl.geom
        d, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
        do, mx = oracle.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
        x, n_in = workloads.make_input(wl, do, mx)
        ref_dd = oracle.dedisperse(do, x, n_in, wl.n_out)
        _, ref_s, ref_p = _oracle_box_snr(ref_dd, widths)
        refs.append((ref_dd, ref_s, ref_p))
        beams.append(dict(delays=torch.from_numpy(d).cuda(), info=info, x=torch.from_numpy(x).cuda(), n_in=n_in,
                          dd=torch.full((g.n_dm, wl.n_out + 3), -1, dtype=torch.int32, device="cuda"),
                          n_out=wl.n_out, snr=torch.zeros((len(widths), g.n_dm), dtype=torch.float32, device="cuda"),
                          peak=torch.zeros((len(widths), g.n_dm), dtype=torch.int32, device="cuda")))
    # three tile classes (one reading its input directly from global memory)
    # so the batch needs more than one launch per kernel
    tiles = [amber.make_tiles(samples_per_thread=8 if k % 2 else 16, channel_unroll=16) for k in range(len(beams))]
    tiles[0] = amber.make_tiles(samples_per_thread=8, channel_unroll=16, dms_per_thread=1, direct_reads=1)
    say("batch of %d uneven beams, eager" % len(beams))
    batch = amber.Batch(beams, widths, tiles=tiles)
    assert batch.launches() == (3, 1)
    batch.run()
    torch.cuda.synchronize()
    for b, (ref_dd, ref_s, ref_p) in zip(beams, refs):
        assert np.array_equal(b["dd"][:, :b["n_out"]].cpu().numpy(), ref_dd)
        _check_snr(b["snr"].cpu().numpy(), b["peak"].cpu().numpy(), ref_s, ref_p)
    first = [(b["snr"].clone(), b["dd"][:, :b["n_out"]].clone()) for b in beams]
    # graph replays: identical results every time, with eager work in between
    stream = torch.cuda.Stream()
    say("batch graph capture + 3 replays")
    with torch.cuda.stream(stream):
        batch.capture(stream)
    for rep in range(3):
        for b in beams:
            b["snr"].zero_()
            b["dd"].fill_(-5)
        torch.cuda.synchronize()
        batch.launch(stream)
        stream.synchronize()
        for b, (s0, d0) in zip(beams, first):
            assert torch.equal(b["snr"], s0) and torch.equal(b["dd"][:, :b["n_out"]], d0), rep
            assert torch.all(b["dd"][:, b["n_out"]:] == -5)   # columns past n_out untouched
        _ = torch.ones(1000, device="cuda").sum()   # unrelated eager work between replays
    batch.close()
