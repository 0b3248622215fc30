"""The fused boxcar / S/N kernel for sliding widths up to 64, against the oracle.

That kernel splits each dedispersed row into blocks of 256 outputs swept by
the work-group's wavefronts, keeps the prefix of two blocks at a time in LDS,
forms the mean from a closed form over the row's head and tail, and resolves
the first index of the maximum at the end from the earliest 4-output group
that reaches it.  These cases aim at each of those parts: every work-group
size (more wavefronts than blocks included), row lengths around the block
and group sizes, rows that are not 16-byte aligned (dword loads), widths that
are not powers of two (reads straddling two 4-output groups), ties between
lanes, blocks and wavefronts, maxima that only invalid outputs would beat,
and rows whose first sample (the centring reference) is far from their mean.
S/N within 1e-5 relative, peak indices exact.
"""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

SNR_RTOL = 1e-5
POW2 = (1, 2, 4, 8, 16, 32, 64)


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


def _ref(dd, n_out, widths):
    s = np.empty((len(widths), dd.shape[0]))
    p = np.empty((len(widths), dd.shape[0]), dtype=np.int32)
    for k, w in enumerate(widths):
        s[k], p[k] = oracle.snr(oracle.boxcar(np.ascontiguousarray(dd[:, :n_out]), w))
    return s, p


def _check(amber, torch, dd_dev, dd_host, n_out, widths, tiles=None, what=""):
    s, p = amber.integrate_snr(dd_dev, n_out, widths, tiles=tiles)
    torch.cuda.synchronize()
    ref_s, ref_p = _ref(dd_host, n_out, widths)
    np.testing.assert_allclose(s.cpu().numpy().astype(np.float64), ref_s, rtol=SNR_RTOL, atol=1e-6, err_msg=what)
    got_p = p.cpu().numpy()
    bad = np.argwhere(got_p != ref_p)
    assert bad.size == 0, "%s: peaks differ at %s (got %s, want %s)" % (
        what, bad[:5].tolist(), got_p[tuple(bad[:5].T)].tolist(), ref_p[tuple(bad[:5].T)].tolist())


@pytest.mark.parametrize("threads", [64, 128, 256, 512, 1024])
@pytest.mark.parametrize("n_out", [64, 300, 1000, 4099, 12208])
def test_work_group_sizes(amber, torch, threads, n_out):
    rng = np.random.default_rng(threads * 100000 + n_out)
    n_dm = 37
    dd = rng.integers(150000, 250000, size=(n_dm, n_out)).astype(np.int32)
    # a pulse in some rows, at varied places (block edges, the row's end)
    for r, t in ((3, 0), (4, 255), (5, 256), (6, n_out - 1), (7, n_out // 2)):
        dd[r, t:t + 5] += 60000
    widths = tuple(w for w in POW2 if w <= n_out)
    say("span threads", threads, "n_out", n_out)
    _check(amber, torch, torch.from_numpy(dd).cuda(), dd, n_out, widths,
           tiles=amber.make_tiles(snr_threads=threads), what="threads %d n_out %d" % (threads, n_out))


@pytest.mark.parametrize("n_out", [4, 5, 7, 63, 65, 255, 256, 257, 511, 513])
def test_short_rows(amber, torch, n_out):
    rng = np.random.default_rng(77 + n_out)
    dd = rng.integers(0, 391680, size=(11, n_out)).astype(np.int32)
    widths = tuple(w for w in (1, 2, 3, 4, 5, 8, 16, 64) if w <= n_out)[:8]
    say("span short rows", n_out, widths)
    _check(amber, torch, torch.from_numpy(dd).cuda(), dd, n_out, widths, what="n_out %d" % n_out)


@pytest.mark.parametrize("widths", [(3, 5, 6, 7, 13, 31, 63, 64), (7, 2, 61), (64,), (5, 9, 17, 33)],
                         ids=lambda w: "w" + "-".join(map(str, w)))
def test_widths_not_powers_of_two(amber, torch, widths):
    rng = np.random.default_rng(sum(widths))
    n_dm, n_out = 29, 3001
    dd = rng.integers(0, 391680, size=(n_dm, n_out)).astype(np.int32)
    say("span widths", widths)
    _check(amber, torch, torch.from_numpy(dd).cuda(), dd, n_out, widths, what=str(widths))
    for threads in (64, 512):
        _check(amber, torch, torch.from_numpy(dd).cuda(), dd, n_out, widths,
               tiles=amber.make_tiles(snr_threads=threads), what="%s threads %d" % (widths, threads))


@pytest.mark.parametrize("offset", [1, 3])
def test_rows_not_16_byte_aligned(amber, torch, offset):
    """Rows that start off a 16-byte boundary or have an odd stride take dword loads."""
    rng = np.random.default_rng(900 + offset)
    n_dm, n_out = 23, 2049
    base = rng.integers(0, 391680, size=(n_dm, n_out + 7)).astype(np.int32)
    dev = torch.from_numpy(base).cuda()
    view = dev[:, offset:offset + n_out]        # row stride n_out + 7 (odd), start offset by `offset` dwords
    host = base[:, offset:offset + n_out]
    say("span unaligned rows, offset", offset)
    _check(amber, torch, view, host, n_out, POW2, what="offset %d" % offset)
    _check(amber, torch, view, host, n_out, (3, 10, 64), tiles=amber.make_tiles(snr_threads=256),
           what="offset %d non-pow2" % offset)


def test_ties_and_masked_maxima(amber, torch):
    n_out = 2000
    widths = (1, 2, 4, 8, 16, 32, 64)
    rows = []
    # 0: equal maxima in two blocks (lanes and wavefronts differ): the first wins
    r = np.full(n_out, 1000, np.int32); r[300] = r[1700] = 5000; rows.append(r)
    # 1: equal maxima in the same 4-output group and in the next group
    r = np.full(n_out, 1000, np.int32); r[401] = r[403] = r[404] = 5000; rows.append(r)
    # 2: the largest samples sit in the last 63 outputs: only short widths may use them
    r = np.full(n_out, 1000, np.int32); r[-10:] = 9000; r[100] = 3000; rows.append(r)
    # 3: a constant row: sigma 0 -> S/N 0 and peak 0
    rows.append(np.full(n_out, 77777, np.int32))
    # 4: a maximum at t = 0 and again later
    r = np.full(n_out, 10, np.int32); r[0] = r[1500] = 99; rows.append(r)
    # 5: a plateau longer than the widest window
    r = np.full(n_out, 10, np.int32); r[700:900] = 500; rows.append(r)
    # 6: a first sample far from the row's mean (the centring reference)
    rng = np.random.default_rng(6)
    r = rng.integers(390000, 391680, size=n_out).astype(np.int32); r[0] = 0; rows.append(r)
    # 7: the same with a row whose mean is far below the first sample
    r = rng.integers(0, 500, size=n_out).astype(np.int32); r[0] = 391680; rows.append(r)
    dd = np.stack(rows)
    dev = torch.from_numpy(dd).cuda()
    for threads in (64, 128, 256, 1024):
        say("span ties, threads", threads)
        _check(amber, torch, dev, dd, n_out, widths, tiles=amber.make_tiles(snr_threads=threads),
               what="ties threads %d" % threads)


def test_batch_mixes_aligned_and_unaligned_beams(amber, torch):
    """A batch whose beams' rows differ in alignment takes the dword-load kernel for all of them."""
    import workloads
    wls = [workloads.Workload(name="b%d" % k, geom=workloads.Geometry(n_chan=64, n_dm=9 + k, dm_first=0.0,
                                                                     dm_step=1.0),
                              n_out=n, widths=POW2, pulses=(), seed=40 + k)
           for k, n in enumerate((1001, 2048, 777))]
    beams, refs = [], []
    for wl in wls:
        g = wl.geom
        d, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
        do, mx = oracle.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
        x, n_in = workloads.make_input(wl, do, mx)
        ref_dd = oracle.dedisperse(do, x, n_in, wl.n_out)
        refs.append(_ref(ref_dd, wl.n_out, POW2))
        # dd rows of n_out int32 (odd for two beams): not 16-byte aligned
        beams.append(dict(delays=torch.from_numpy(d).cuda(), info=info, x=torch.from_numpy(x).cuda(), n_in=n_in,
                          n_out=wl.n_out, dd=torch.zeros((g.n_dm, wl.n_out), dtype=torch.int32, device="cuda"),
                          snr=torch.zeros((len(POW2), g.n_dm), dtype=torch.float32, device="cuda"),
                          peak=torch.zeros((len(POW2), g.n_dm), dtype=torch.int32, device="cuda")))
    say("span batch of 3 beams with mixed row alignment")
    batch = amber.Batch(beams, POW2)
    batch.run()
    torch.cuda.synchronize()
    for bm, (ref_s, ref_p) in zip(beams, refs):
        np.testing.assert_allclose(bm["snr"].cpu().numpy().astype(np.float64), ref_s, rtol=SNR_RTOL, atol=1e-6)
        assert np.array_equal(bm["peak"].cpu().numpy(), ref_p)
    batch.close()


def test_large_values_take_the_fp64_sums(amber, torch):
    """Rows whose sums of squares could pass the int64 accumulators' range are
    summed again in FP64: values up to 2^25 with width 64 (boxcars near 2^31),
    beside ordinary rows in the same launch."""
    rng = np.random.default_rng(31)
    n_dm, n_out = 12, 3000
    dd = rng.integers(0, 391680, size=(n_dm, n_out)).astype(np.int32)
    dd[2] = rng.integers(0, 1 << 25, size=n_out)              # every wavefront over the bound
    dd[5, :1500] = rng.integers(0, 1 << 25, size=1500)        # only the first wavefronts
    dd[7] = (1 << 25) - 1 - rng.integers(0, 5, size=n_out)    # large, nearly constant
    dd[7, 0] = 0                                              # centre far from the mean
    dev = torch.from_numpy(dd).cuda()
    for threads in (64, 256):
        say("span large values, threads", threads)
        _check(amber, torch, dev, dd, n_out, POW2, tiles=amber.make_tiles(snr_threads=threads),
               what="large values threads %d" % threads)
