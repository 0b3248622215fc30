"""Two-step subband dedispersion on the device against the oracle.

Every trial must equal the oracle's composed subband sum bit for bit, for
several tile choices of each step, ragged lengths and the degenerate grids:
one subband (step two does nothing: every fine trial is the coarse DM's brute
force), one channel per subband (step one does nothing: every trial is brute
force at its own DM).  Step one's scratch rows are checked on their own
against the oracle's brute-force dedispersion of each subband, and the full
1536-channel beam is checked on sampled coarse DMs for both the beam's grid
and Table 2's subbanding grid.
"""
import sys

import numpy as np
import pytest

import oracle
import subband_smearing
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


SMALL = workloads.small().geom          # 256 channels over 1250-1550 MHz
BEAM = workloads.beam().geom            # 1536 channels


def _setup(amber, g, grid, n_out, seed, pulse=None):
    """Tables (library and oracle), input with n_in = n_out + max_delay."""
    f = g.freqs()
    d1, d2, info = amber.subband_delay_tables(f, g.t_samp_s, *grid)
    o1, o2, _, _ = oracle.subband_delays(f, g.t_samp_s, *grid)
    n_in = n_out + info.max_delay
    x = workloads.noise(g.n_chan, n_in, workloads.padded_stride(n_in), seed=seed)
    if pulse is not None:
        bd, _ = oracle.delay_table(f, g.t_samp_s, 1, pulse[0], 0.0)
        workloads.inject(x, bd[0], t0=pulse[1], width=pulse[2], amp=40)
    return d1, d2, info, o1, o2, x, n_in


def _run(amber, torch, d1, d2, info, x, n_in, n_out, **kw):
    return amber.subband_dedisperse(torch.from_numpy(d1).cuda(), torch.from_numpy(d2).cuda(), info,
                                    torch.from_numpy(x).cuda(), n_in, n_out, **kw)


SMALL_GRID = (16, 16, 0.0, 8.0, 8, 0.0, 1.0)   # 128 trials 0..127 step 1 from 16 subbands of 16 channels
TILES = [
    (None, None),
    (dict(threads_per_dm=64, samples_per_thread=8, dms_per_block=4, channel_unroll=16),
     dict(threads_per_dm=64, samples_per_thread=16, dms_per_block=8, channel_unroll=8)),
    (dict(threads_per_dm=128, samples_per_thread=4, dms_per_block=3, channel_unroll=2),
     dict(threads_per_dm=128, samples_per_thread=8, dms_per_block=3, channel_unroll=4)),
    (dict(threads_per_dm=64, samples_per_thread=16, dms_per_block=8, channel_unroll=8),
     dict(threads_per_dm=64, samples_per_thread=8, dms_per_block=16, channel_unroll=32)),  # idle DM rows
]


def _tid(t):
    a, b = t
    if a is None:
        return "auto"
    return "s1-%d-%d-%d-%d_s2-%d-%d-%d-%d" % tuple(
        [a[k] for k in ("threads_per_dm", "samples_per_thread", "dms_per_block", "channel_unroll")] +
        [b[k] for k in ("threads_per_dm", "samples_per_thread", "dms_per_block", "channel_unroll")])


@pytest.mark.parametrize("tiles", TILES, ids=_tid)
def test_subband_small_bit_exact(amber, torch, tiles):
    n_out = 3001                       # ragged: not a multiple of any time tile
    d1, d2, info, o1, o2, x, n_in = _setup(amber, SMALL, SMALL_GRID, n_out, seed=61, pulse=(50.0, 1500, 4))
    ref = oracle.subband_dedisperse(o1, o2, x, n_in, n_out)
    t1 = amber.make_tiles(**{"dms_per_thread": 1, **tiles[0]}) if tiles[0] else None
    t2 = amber.make_tiles(**{"dms_per_thread": 1, **tiles[1]}) if tiles[1] else None
    say("subband small", _tid(tiles), info)
    got = _run(amber, torch, d1, d2, info, x, n_in, n_out, tiles1=t1, tiles2=t2).cpu().numpy()
    assert np.array_equal(got, ref)


def test_subband_step_one_rows(amber, torch):
    """Step one's scratch: row (s, j) is the brute-force sum of subband s's
    channels with the library's step-one delays, for n_out + max_delay2 samples."""
    n_out = 2000
    d1, d2, info, o1, o2, x, n_in = _setup(amber, SMALL, SMALL_GRID, n_out, seed=62)
    n_sub, nc, m = d1.shape
    n1 = n_out + info.max_delay2
    work = torch.zeros((n_sub * nc, (n1 + 7) // 2 * 2), dtype=torch.uint16, device="cuda")  # even stride
    say("subband step-one rows", info)
    _run(amber, torch, d1, d2, info, x, n_in, n_out, work=work)
    w = work.cpu().numpy().astype(np.int64)[:, :n1].reshape(n_sub, nc, n1)
    for s in range(n_sub):
        ref = oracle.dedisperse(d1[s], x[s * m:(s + 1) * m], n_in, n1)
        assert np.array_equal(w[s], ref), s


def test_subband_shift_split_is_exact(amber, torch):
    """The library moves each coarse DM's smallest step-two shift into step
    one; the oracle's tables keep every shift where the scheme defines it.
    Both splits through the same entry point (the info describing each) give
    the same trials, equal to the oracle's."""
    n_out = 1777
    f = SMALL.freqs()
    d1, d2, info, o1, o2, x, n_in = _setup(amber, SMALL, SMALL_GRID, n_out, seed=65)
    o1 = np.ascontiguousarray(o1, dtype=np.int32)
    o2 = np.ascontiguousarray(o2, dtype=np.int32)
    raw = amber.SubbandInfo(n_chan=info.n_chan, n_subbands=info.n_subbands, n_coarse=info.n_coarse,
                            n_fine=info.n_fine, max_delay1=int(o1.max()), max_step1=int(np.diff(o1, axis=1).max()),
                            max_delay2=int(o2.max()), max_step2=int(np.diff(o2, axis=1).max()),
                            max_delay=int((o2 + o1.max(axis=2).T[:, None, :]).max()))
    assert raw.max_delay == info.max_delay          # the composed shifts are the same
    assert raw.max_delay2 > info.max_delay2 and raw.max_step1 <= info.max_step1
    say("subband shift split", info, raw)
    moved = _run(amber, torch, d1, d2, info, x, n_in, n_out).cpu().numpy()
    kept = _run(amber, torch, o1, o2, raw, x, n_in, n_out).cpu().numpy()
    assert np.array_equal(moved, kept)
    assert np.array_equal(moved, oracle.subband_dedisperse(o1, o2, x, n_in, n_out))


def test_subband_refuses_direct_reads(amber, torch):
    """The subband steps stage their input in LDS: tiles asking for direct
    reads are refused on the host, before any launch."""
    n_out = 500
    d1, d2, info, o1, o2, x, n_in = _setup(amber, SMALL, SMALL_GRID, n_out, seed=64)
    t = amber.make_tiles(dms_per_thread=1, direct_reads=1)
    for kw in (dict(tiles1=t), dict(tiles2=t)):
        with pytest.raises(amber.AmberError) as e:
            _run(amber, torch, d1, d2, info, x, n_in, n_out, **kw)
        assert e.value.status == -3


def test_subband_one_subband_is_coarse_brute_force(amber, torch):
    n_out = 1500
    grid = (1, 6, 0.0, 16.0, 4, 0.0, 4.0)       # every fine trial of coarse DM j: brute force at 16 j
    d1, d2, info, o1, o2, x, n_in = _setup(amber, SMALL, grid, n_out, seed=63)
    assert info.max_delay2 == 0
    bd, mx = oracle.delay_table(SMALL.freqs(), SMALL.t_samp_s, 6, 0.0, 16.0)
    bf = oracle.dedisperse(bd, x, n_in, n_out)
    say("one subband", info)
    got = _run(amber, torch, d1, d2, info, x, n_in, n_out).cpu().numpy().reshape(6, 4, n_out)
    for k in range(4):
        assert np.array_equal(got[:, k], bf)


def test_subband_one_channel_per_subband_is_brute_force(amber, torch):
    """m = 1: step one is a copy and step two is brute force at DM_jk
    (dyadic steps make DM_jk = (16 j + k) * 0.5 exactly)."""
    n_out = 1800
    grid = (256, 8, 0.0, 8.0, 16, 0.0, 0.5)
    d1, d2, info, o1, o2, x, n_in = _setup(amber, SMALL, grid, n_out, seed=64)
    bd, mx = oracle.delay_table(SMALL.freqs(), SMALL.t_samp_s, 128, 0.0, 0.5)
    bf = oracle.dedisperse(bd, x, n_in, n_out)
    say("one channel per subband", info)
    got = _run(amber, torch, d1, d2, info, x, n_in, n_out).cpu().numpy()
    assert np.array_equal(got, bf)


def test_subband_edge_lengths_and_repeat(amber, torch):
    for n_out, grid in ((1, SMALL_GRID), (63, (8, 3, 2.0, 5.0, 2, 0.0, 2.5)), (4097, (32, 5, 0.0, 12.0, 3, 1.0, 4.0))):
        d1, d2, info, o1, o2, x, n_in = _setup(amber, SMALL, grid, n_out, seed=65 + n_out)
        ref = oracle.subband_dedisperse(o1, o2, x, n_in, n_out)
        say("edge n_out", n_out, info)
        a = _run(amber, torch, d1, d2, info, x, n_in, n_out).cpu().numpy()
        b = _run(amber, torch, d1, d2, info, x, n_in, n_out).cpu().numpy()
        assert np.array_equal(a, ref) and np.array_equal(a, b)
    # n_out = 0 launches nothing: the output keeps its contents
    d1, d2, info, o1, o2, x, n_in = _setup(amber, SMALL, SMALL_GRID, 0, seed=70)
    out = torch.full((info.n_coarse * info.n_fine, 8), -7, dtype=torch.int32, device="cuda")
    _run(amber, torch, d1, d2, info, x, n_in, 0, out=out)
    assert (out.cpu().numpy() == -7).all()


def test_subband_wide_subbands_saturated(amber, torch):
    """8 subbands of 192 channels over saturated input: step one's sums reach
    192 * 255 = 48960 (the 16-bit intermediates' range) and step two widens
    its packed sums after every subband (one more would overflow 16 bits),
    on several step-two tiles; bit-exact against the oracle."""
    n_out = 3000
    grid = (8, 12, 0.0, 16.0, 4, 0.0, 4.0)
    d1, d2, info, o1, o2, x, n_in = _setup(amber, BEAM, grid, n_out, seed=74)
    x[:, 500:2600] = 255
    x[::3, 2600:] = 255
    ref = oracle.subband_dedisperse(o1, o2, x, n_in, n_out)
    assert ref.max() == 1536 * 255
    for t2 in (None, dict(threads_per_dm=64, samples_per_thread=8, dms_per_block=4, channel_unroll=4),
               dict(threads_per_dm=64, samples_per_thread=16, dms_per_block=8, channel_unroll=4)):
        say("wide subbands saturated", info, t2)
        got = _run(amber, torch, d1, d2, info, x, n_in, n_out,
                   tiles2=amber.make_tiles(dms_per_thread=1, **t2) if t2 else None).cpu().numpy()
        assert np.array_equal(got, ref), t2


def test_subband_masked(amber, torch):
    n_out = 2500
    d1, d2, info, o1, o2, x, n_in = _setup(amber, SMALL, SMALL_GRID, n_out, seed=71, pulse=(80.0, 1000, 2))
    keep = (np.random.default_rng(72).random(SMALL.n_chan) >= 0.2).astype(np.uint8)
    keep[16:32] = 0                                       # a whole subband
    xz = x.copy()
    xz[keep == 0] = 0                                     # zapped channels contribute nothing
    ref = oracle.subband_dedisperse(o1, o2, xz, n_in, n_out)
    say("subband masked, zapped", int((keep == 0).sum()))
    got = _run(amber, torch, d1, d2, info, x, n_in, n_out, keep=torch.from_numpy(keep).cuda()).cpu().numpy()
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("grid", [(32, 128, 0.0, 8.0, 16, 0.0, 0.5), (32, 2048, 0.0, 2.4, 24, 0.0, 0.1)],
                         ids=["beam-grid-2048dm", "table2-grid-49152dm"])
def test_subband_beam_sampled(amber, torch, grid):
    """The 1536-channel, 12208-sample beam at full size; sampled coarse DMs
    (every fine trial of each) against the oracle."""
    wl = workloads.beam()
    n_out = wl.n_out
    d1, d2, info, o1, o2, x, n_in = _setup(amber, BEAM, grid, n_out, seed=2)
    say("subband beam full size", info, "n_in", n_in)
    got = _run(amber, torch, d1, d2, info, x, n_in, n_out)
    torch.cuda.synchronize()
    nc, nf = info.n_coarse, info.n_fine
    js = sorted(set([0, 1, nc - 1] + list(np.random.default_rng(73).choice(nc, size=3, replace=False))))
    rows = np.array([j * nf + k for j in js for k in range(nf)])
    got_rows = got[torch.from_numpy(rows).cuda()].cpu().numpy()
    ref = oracle.subband_dedisperse(o1[:, js, :], o2[js], x, n_in, n_out)
    assert np.array_equal(got_rows, ref)


def test_subband_tune_on_device_keeps_parity(amber, torch):
    """The device search over both steps' genes (a short GA) returns tiles
    whose pipeline is still bit-exact against the oracle."""
    n_out = 2048
    d1, d2, info, o1, o2, x, n_in = _setup(amber, SMALL, SMALL_GRID, n_out, seed=81)
    sp = amber.default_subband_space(info, (1, 4, 16), n_out)
    say("subband device tune", amber.subband_space_size(sp))
    d1d, d2d, xd = torch.from_numpy(d1).cuda(), torch.from_numpy(d2).cuda(), torch.from_numpy(x).cuda()
    res = amber.tune_subband(sp, d1d, d2d, xd, n_in, amber.tune_params("ga", seed=4, pop=8, generations=3))
    assert res.n_evals > 0 and res.best_time_s > 0
    got = amber.subband_dedisperse(d1d, d2d, info, xd, n_in, n_out, tiles1=res.step1, tiles2=res.step2).cpu().numpy()
    assert np.array_equal(got, oracle.subband_dedisperse(o1, o2, x, n_in, n_out))


@pytest.mark.parametrize("grid_name", sorted(subband_smearing.GRIDS))
def test_subband_snr_loss_within_smearing_bound(amber, torch, grid_name):
    """Pulses on the 1536-channel beam through the device's subband path, on
    the beam's own grid and on Table 2's grid spacing: a pulse alone comes out
    of its trial exactly as the tables' shift errors smear it, and with noise
    the device's S/N at the pulse's width, over the oracle's brute-force S/N
    of the same input, stays between the floor that smearing allows (noise
    margins included) and 1 plus the noise margin."""
    sm = subband_smearing
    grid, pulses = sm.GRIDS[grid_name]
    g = BEAM
    f, ts, n_out, amp = g.freqs(), g.t_samp_s, sm.BEAM_N_OUT, sm.PULSE_AMP
    d1, d2, info = amber.subband_delay_tables(f, ts, *grid)
    shifts = [sm.pulse_shifts(f, ts, grid, j, k) for j, k, _, _ in pulses]
    n_in = n_out + max(info.max_delay, max(int(d.max()) for _, _, d in shifts))
    stride = workloads.padded_stride(n_in)
    x = workloads.noise(g.n_chan, n_in, stride, seed=77)
    for (j, k, w, t0), (e, resid, d) in zip(pulses, shifts):
        workloads.inject(x, d, t0=t0, width=w, amp=amp)
    d1d, d2d = torch.from_numpy(d1).cuda(), torch.from_numpy(d2).cuda()
    widths = sorted({p[2] for p in pulses})
    say("subband smearing", grid_name, info, "n_in", n_in)
    dd = amber.subband_dedisperse(d1d, d2d, info, torch.from_numpy(x).cuda(), n_in, n_out)
    s_sb, _ = amber.integrate_snr(dd, n_out, widths)
    s_sb = s_sb.cpu().numpy()
    nf = grid[4]
    for (j, k, w, t0), (e, resid, d) in zip(pulses, shifts):
        row = j * nf + k
        one = np.zeros((g.n_chan, stride), np.uint8)
        workloads.inject(one, d, t0=t0, width=w, amp=amp)
        got = amber.subband_dedisperse(d1d, d2d, info, torch.from_numpy(one).cuda(), n_in, n_out)[row].cpu().numpy()
        want = sm.smeared_series(e, t0, w, amp, n_out)
        assert np.array_equal(got, want), (grid_name, j, k)
        peak_bf = amp * g.n_chan * w
        frac = sm.best_boxcar(want, w) / peak_bf
        s_bf, _ = oracle.snr(oracle.boxcar(oracle.dedisperse(d[None], x, n_in, n_out), w))
        ratio = float(s_sb[widths.index(w), row]) / s_bf[0]
        sigma = sm.noise_sigma(g.n_chan, w)
        floor = sm.snr_ratio_floor(frac, peak_bf, sigma, w, n_out)
        say("  trial (%d, %d) width %d: collected %.3f, S/N ratio %.3f, floor %.3f" % (j, k, w, frac, ratio, floor))
        assert floor <= ratio <= 1.0 + 5.0 * sigma / peak_bf, (grid_name, j, k, w, frac, floor, ratio)
