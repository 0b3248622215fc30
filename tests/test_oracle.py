"""Pins of the CPU oracle against what the physics and mathematics fix.

None of these compare the oracle with itself: each check uses an independent
route -- physical constants, exact (extended-precision) evaluation margins,
invariants, special cases that reduce to a plain channel sum or a library
routine, brute force on tiny inputs, or a closed-form S/N prediction.
"""
import math
import os

import numpy as np
import pytest

import oracle
import subband_smearing
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _codata():
    vals = {}
    with open(os.path.join(GOLDEN, "codata_2018.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


# --- delay table ---------------------------------------------------------------

def test_delay_constant_matches_physics():
    """The delay of DM = 1 pc cm^-3 at 1 GHz against an (effectively) infinite
    reference frequency is e^2 / (8 pi^2 eps0 m_e c) * DM / f^2, derived here
    from CODATA constants (tests/golden/codata_2018.txt)."""
    c = _codata()
    k_si = c["elementary_charge_C"] ** 2 / (8 * math.pi ** 2 * c["vacuum_permittivity_F_m"]
                                            * c["electron_mass_kg"] * c["speed_of_light_m_s"])
    pc_m = 648000.0 / math.pi * c["astronomical_unit_m"]
    k_mhz = k_si * (pc_m * 1e6) * 1e-12          # s MHz^2 / (pc cm^-3)
    t_samp = 1e-9
    d, mx = oracle.delay_table(np.array([1000.0, 1e9]), t_samp, 2, 0.0, 1.0)
    expected = k_mhz * 1.0 / 1000.0 ** 2 / t_samp
    assert d[1, 1] == 0 and d[0, 0] == 0
    assert abs(d[1, 0] - expected) / expected < 2e-6
    assert mx == d[1, 0]


def test_delay_inverse_square_law():
    """Against a far reference, halving the frequency multiplies the delay by 4."""
    f = np.array([600.0, 1200.0, 1e9])
    d, _ = oracle.delay_table(f, 1e-6, 3, 0.0, 100.0)
    for i in range(3):
        assert abs(int(d[i, 0]) - 4 * int(d[i, 1])) <= 4
    assert d[2, 1] > 1000


def test_delay_linear_in_dm_and_inverse_in_tsamp():
    g = workloads.small().geom
    f = g.freqs()
    d1, _ = oracle.delay_table(f, g.t_samp_s, 64, 0.0, 1.0)
    d2, _ = oracle.delay_table(f, g.t_samp_s, 64, 0.0, 2.0)
    assert np.all(np.abs(d2.astype(np.int64) - 2 * d1) <= 1)
    dh, _ = oracle.delay_table(f, g.t_samp_s / 2, 64, 0.0, 1.0)
    assert np.all(np.abs(dh.astype(np.int64) - 2 * d1) <= 1)
    # dm_first offsets the grid by multiplication, not accumulation
    do, _ = oracle.delay_table(f, g.t_samp_s, 32, 32.0, 1.0)
    assert np.array_equal(do, d1[32:])


def test_delay_relative_to_highest_channel():
    """Delays are measured against the highest frequency present: removing the
    top channel re-references the others by the old delay of the new top."""
    f = np.array([1250.0, 1400.0, 1550.0])
    d3, _ = oracle.delay_table(f, 81.92e-6, 50, 0.0, 10.0)
    d2, _ = oracle.delay_table(f[:2], 81.92e-6, 50, 0.0, 10.0)
    assert np.all(d3[:, 2] == 0) and np.all(d2[:, 1] == 0)
    assert np.all(np.abs(d3[:, 0].astype(np.int64) - d3[:, 1] - d2[:, 0]) <= 1)
    # channel order does not matter: f_top is the maximum, wherever it sits
    dp, _ = oracle.delay_table(f[::-1].copy(), 81.92e-6, 50, 0.0, 10.0)
    assert np.array_equal(dp, d3[:, ::-1])


@pytest.mark.parametrize("wl", [workloads.small(), workloads.beam()], ids=lambda w: w.name)
def test_delay_invariants_and_tie_margin(wl):
    g = wl.geom
    f = g.freqs()
    d, mx = oracle.delay_table(f, g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    assert d.shape == (g.n_dm, g.n_chan)
    assert np.all(d[0] == 0)                      # DM = 0
    assert np.all(d[:, -1] == 0)                  # top channel
    assert np.all(np.diff(d, axis=0) >= 0)        # non-decreasing in DM
    assert np.all(np.diff(d, axis=1) <= 0)        # non-increasing in frequency
    assert mx == d.max() == d[-1, 0]
    # Evaluate the same real number in 80-bit extended precision: no entry may
    # sit within 1e-9 of a rounding tie, and rounding the extended value must
    # give the oracle's table (so FP64 evaluation order cannot matter).
    fl = f.astype(np.longdouble)
    ftop = fl.max()
    dm = (np.longdouble(g.dm_first) + np.arange(g.n_dm, dtype=np.longdouble) * np.longdouble(g.dm_step))
    x = (np.longdouble(4.148808e3) * dm[:, None]) * (1 / (fl * fl) - 1 / (ftop * ftop))[None, :] / np.longdouble(g.t_samp_s)
    frac = x - np.floor(x)
    assert np.min(np.abs(frac - 0.5)) > 1e-9
    assert np.array_equal(np.floor(x + 0.5).astype(np.int64), d.astype(np.int64))


def test_delay_rejects_bad_args():
    with pytest.raises(ValueError):
        oracle.delay_table(np.array([1000.0, -1.0]), 1e-4, 4, 0.0, 1.0)
    with pytest.raises(ValueError):
        oracle.delay_table(np.array([1000.0]), 0.0, 4, 0.0, 1.0)


# --- dedispersion ---------------------------------------------------------------

def test_dedisperse_dm0_is_channel_sum():
    x = workloads.noise(64, 700, 768, seed=3)
    d = np.zeros((1, 64), dtype=np.int32)
    dd = oracle.dedisperse(d, x, 700, 700)
    assert np.array_equal(dd[0], x[:, :700].astype(np.int64).sum(axis=0))


def test_dedisperse_impulse_response():
    """A single unit sample at (c, tau) lands at t = tau - delay[i][c] (sign and
    index of the shift), and nowhere else."""
    rng = np.random.default_rng(11)
    n_chan, n_dm, n_out = 7, 5, 40
    delays = rng.integers(0, 9, size=(n_dm, n_chan)).astype(np.int32)
    n_in = n_out + int(delays.max())
    for c, tau in [(0, 0), (3, 12), (6, n_in - 1), (2, 25)]:
        x = np.zeros((n_chan, n_in), dtype=np.uint8)
        x[c, tau] = 1
        dd = oracle.dedisperse(delays, x, n_in, n_out)
        for i in range(n_dm):
            t = tau - delays[i, c]
            expect = np.zeros(n_out, dtype=np.int64)
            if 0 <= t < n_out:
                expect[t] = 1
            assert np.array_equal(dd[i], expect)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_dedisperse_brute_force_tiny(seed):
    delays, x, n_in = workloads.tiny(n_chan=8, n_dm=8, n_out=64, seed=seed)
    dd = oracle.dedisperse(delays, x, n_in, 64)
    ref = np.zeros((8, 64), dtype=np.int64)
    for i in range(8):
        for t in range(64):
            s = 0
            for c in range(8):
                s += int(x[c, t + delays[i, c]])
            ref[i, t] = s
    assert np.array_equal(dd, ref)


def test_dedisperse_linearity_and_permutation():
    delays, x, n_in = workloads.tiny(n_chan=16, n_dm=6, n_out=100, seed=9)
    a = (x // 2).astype(np.uint8)
    b = (x - a).astype(np.uint8)
    assert np.array_equal(oracle.dedisperse(delays, a, n_in, 100) + oracle.dedisperse(delays, b, n_in, 100),
                          oracle.dedisperse(delays, x, n_in, 100))
    perm = np.random.default_rng(4).permutation(16)
    assert np.array_equal(oracle.dedisperse(delays[:, perm], x[perm], n_in, 100),
                          oracle.dedisperse(delays, x, n_in, 100))


def test_dedisperse_rejects_out_of_range():
    delays, x, n_in = workloads.tiny(n_chan=4, n_dm=3, n_out=20, seed=5)
    with pytest.raises(ValueError):
        oracle.dedisperse(delays, x, n_in - 1, 20)
    bad = delays.copy()
    bad[1, 2] = -1
    with pytest.raises(ValueError):
        oracle.dedisperse(bad, x, n_in, 20)


# --- boxcar -----------------------------------------------------------------------

def test_dedisperse_masked_pins():
    """Zapping channels: an all-kept mask is plain dedispersion; a mask and its
    complement partition the sum; a zapped row's data never matter; zapping
    everything gives zeros; a single kept channel is its shifted row."""
    delays, x, n_in = workloads.tiny(n_chan=19, n_dm=6, n_out=150, seed=31, max_delay=40)
    rng = np.random.default_rng(32)
    full = oracle.dedisperse(delays, x, n_in, 150)
    assert np.array_equal(oracle.dedisperse_masked(delays, x, n_in, 150, np.ones(19, np.uint8)), full)
    keep = (rng.random(19) < 0.7).astype(np.uint8)
    a = oracle.dedisperse_masked(delays, x, n_in, 150, keep)
    b = oracle.dedisperse_masked(delays, x, n_in, 150, 1 - keep)
    assert np.array_equal(a + b, full)
    x2 = x.copy()
    x2[keep == 0] = rng.integers(0, 256, size=x2[keep == 0].shape, dtype=np.uint8)
    assert np.array_equal(oracle.dedisperse_masked(delays, x2, n_in, 150, keep), a)
    assert not np.any(oracle.dedisperse_masked(delays, x, n_in, 150, np.zeros(19, np.uint8)))
    one = np.zeros(19, np.uint8)
    one[5] = 1
    got = oracle.dedisperse_masked(delays, x, n_in, 150, one)
    for i in range(6):
        assert np.array_equal(got[i], x[5, delays[i, 5]:delays[i, 5] + 150].astype(np.int32))


def _subband_case(n_chan, n_sub, n_coarse, cstep, n_fine, fstep, n_out, seed):
    g = workloads.Geometry(n_chan=n_chan, n_dm=1, dm_first=0.0, dm_step=1.0)
    d1, d2, m1, m2 = oracle.subband_delays(g.freqs(), g.t_samp_s, n_sub, n_coarse, 0.0, cstep, n_fine, 0.0, fstep)
    n_in = n_out + m1 + m2
    x = np.random.default_rng(seed).integers(0, 256, size=(n_chan, n_in + 3)).astype(np.uint8)
    return g, d1, d2, m1, m2, x, n_in


def test_subband_reduces_to_brute_force():
    """One channel per subband: the subband shift is the full shift at the
    trial DM, so the scheme is brute force on the fine grid.  One subband:
    the reference is the top channel, so every fine trial equals brute force
    at its coarse DM."""
    n_out = 300
    g, d1, d2, m1, m2, x, n_in = _subband_case(24, 24, 3, 6.0, 4, 1.5, n_out, 51)
    assert not d1.any()
    bf, mx = oracle.delay_table(g.freqs(), g.t_samp_s, 12, 0.0, 1.5)
    assert np.array_equal(d2.reshape(12, 24), bf)
    assert np.array_equal(oracle.subband_dedisperse(d1, d2, x, n_in, n_out), oracle.dedisperse(bf, x, n_in, n_out))
    g, d1, d2, m1, m2, x, n_in = _subband_case(24, 1, 3, 6.0, 4, 1.5, n_out, 52)
    assert not d2.any()
    coarse, _ = oracle.delay_table(g.freqs(), g.t_samp_s, 3, 0.0, 6.0)
    assert np.array_equal(d1[0], coarse)
    got = oracle.subband_dedisperse(d1, d2, x, n_in, n_out).reshape(3, 4, n_out)
    ref = oracle.dedisperse(coarse, x, n_in, n_out)
    for k in range(4):
        assert np.array_equal(got[:, k], ref)


def test_subband_delay_error_bound_and_impulse():
    """The composed shift differs from the exact one only by the intra-subband
    residual K (DM_jk - DM_j) (1/f_c^2 - 1/f_ref^2) / t_samp plus rounding;
    DM 0 is the channel sum; an impulse lands where the composed shifts say."""
    n_chan, n_sub, n_coarse, cstep, n_fine, fstep = 64, 8, 5, 8.0, 8, 1.0
    g = workloads.Geometry(n_chan=n_chan, n_dm=1, dm_first=0.0, dm_step=1.0)
    f = g.freqs()
    d1, d2, m1, m2 = oracle.subband_delays(f, g.t_samp_s, n_sub, n_coarse, 0.0, cstep, n_fine, 0.0, fstep)
    K = 4.148808e3
    m = n_chan // n_sub
    for j in range(n_coarse):
        for k in range(n_fine):
            dm, dmk = j * cstep, j * cstep + k * fstep
            for c in range(n_chan):
                s, cl = divmod(c, m)
                fref = f[s * m:(s + 1) * m].max()
                exact = K * dmk * (1 / f[c] ** 2 - 1 / f.max() ** 2) / g.t_samp_s
                resid = K * (dmk - dm) * (1 / f[c] ** 2 - 1 / fref ** 2) / g.t_samp_s
                assert abs(d1[s, j, cl] + d2[j, k, s] - exact) <= resid + 1.0 + 1e-9
    n_out = 200
    n_in = n_out + m1 + m2
    x = np.random.default_rng(53).integers(0, 256, size=(n_chan, n_in)).astype(np.uint8)
    dd = oracle.subband_dedisperse(d1, d2, x, n_in, n_out)
    assert np.array_equal(dd[0], x[:, :n_out].astype(np.int64).sum(axis=0))
    imp = np.zeros((n_chan, n_in), np.uint8)
    imp[17, 150] = 1
    dd = oracle.subband_dedisperse(d1, d2, imp, n_in, n_out).reshape(n_coarse, n_fine, n_out)
    s, cl = divmod(17, m)
    for j in range(n_coarse):
        for k in range(n_fine):
            t = 150 - d2[j, k, s] - d1[s, j, cl]
            want = np.zeros(n_out, np.int32)
            if 0 <= t < n_out:
                want[t] = 1
            assert np.array_equal(dd[j, k], want)
    with pytest.raises(ValueError):
        oracle.subband_delays(f, g.t_samp_s, 7, 2, 0.0, 1.0, 2, 0.0, 0.5)     # 7 does not divide 64


@pytest.mark.parametrize("grid_name", sorted(subband_smearing.GRIDS))
def test_subband_snr_loss_within_smearing_bound(grid_name):
    """Pulses on the 1536-channel beam under the subband scheme, on the
    beam's own grid and on Table 2's grid spacing: every channel's shift
    error lies within the pinned bound (residual +- 3/2); a pulse alone
    comes out of its subband trial exactly as those shifts smear it; and with
    noise, the subband / brute-force S/N ratio at the pulse's width is no
    lower than the fraction of the pulse one boxcar collects after that
    smearing allows (noise margins in the floor) and no higher than 1 plus
    the noise margin."""
    sm = subband_smearing
    grid, pulses = sm.GRIDS[grid_name]
    g = workloads.beam().geom
    f, ts, n_out, amp = g.freqs(), g.t_samp_s, sm.BEAM_N_OUT, sm.PULSE_AMP
    d1, d2, m1, m2 = oracle.subband_delays(f, ts, *grid)
    shifts = [sm.pulse_shifts(f, ts, grid, j, k) for j, k, _, _ in pulses]
    n_in = n_out + max(m1 + m2, max(int(d.max()) for _, _, d in shifts))
    x = workloads.noise(g.n_chan, n_in, workloads.padded_stride(n_in), seed=77)
    for (j, k, w, t0), (e, resid, d) in zip(pulses, shifts):
        assert np.all(np.abs(e - resid) <= 1.5 + 1e-9), (j, k)
        workloads.inject(x, d, t0=t0, width=w, amp=amp)
    for (j, k, w, t0), (e, resid, d) in zip(pulses, shifts):
        one = np.zeros_like(x)
        workloads.inject(one, d, t0=t0, width=w, amp=amp)
        sb = oracle.subband_dedisperse(d1[:, [j], :], d2[[j]][:, [k], :], one, n_in, n_out)[0]
        want = sm.smeared_series(e, t0, w, amp, n_out)
        assert np.array_equal(sb, want), (j, k)
        bf = oracle.dedisperse(d[None], one, n_in, n_out)[0]
        assert bf[t0:t0 + w].tolist() == [amp * g.n_chan] * w and bf.sum() == amp * g.n_chan * w
        peak_bf = amp * g.n_chan * w
        frac = sm.best_boxcar(want, w) / peak_bf
        s_sb, _ = oracle.snr(oracle.boxcar(oracle.subband_dedisperse(d1[:, [j], :], d2[[j]][:, [k], :], x, n_in,
                                                                     n_out), w))
        s_bf, _ = oracle.snr(oracle.boxcar(oracle.dedisperse(d[None], x, n_in, n_out), w))
        ratio = s_sb[0] / s_bf[0]
        sigma = sm.noise_sigma(g.n_chan, w)
        floor = sm.snr_ratio_floor(frac, peak_bf, sigma, w, n_out)
        assert floor <= ratio <= 1.0 + 5.0 * sigma / peak_bf, (j, k, w, frac, floor, ratio)


def test_boxcar_identity_doubling_and_convolve():
    rng = np.random.default_rng(21)
    dd = rng.integers(0, 400000, size=(5, 300)).astype(np.int32)
    assert np.array_equal(oracle.boxcar(dd, 1), dd.astype(np.int64))
    for w in (1, 2, 4, 8, 16, 32):
        bw = oracle.boxcar(dd, w)
        b2 = oracle.boxcar(dd, 2 * w)
        n2 = 300 - 2 * w + 1
        assert np.array_equal(b2, bw[:, :n2] + bw[:, w:w + n2])
    for w in (3, 7, 64, 300):
        bw = oracle.boxcar(dd, w)
        for i in range(5):
            assert np.array_equal(bw[i], np.convolve(dd[i].astype(np.int64), np.ones(w, dtype=np.int64), "valid"))
    with pytest.raises(ValueError):
        oracle.boxcar(dd, 301)


def test_downsample_pins():
    """Decimation by f (Table 2: NRSAMPLES = SAMPLES / DOWNSAMPLING) is the
    sliding boxcar of width f read at t = j f; decimating by a then by b is
    decimating by a b; whole bins conserve the sum; the remainder is dropped."""
    rng = np.random.default_rng(22)
    dd = rng.integers(0, 400000, size=(4, 1000)).astype(np.int32)
    assert np.array_equal(oracle.downsample(dd, 1), dd.astype(np.int64))
    for f in (2, 3, 7, 10, 64, 333, 1000):
        y = oracle.downsample(dd, f)
        nb = 1000 // f
        assert y.shape == (4, nb)
        assert np.array_equal(y, oracle.boxcar(dd, f)[:, ::f][:, :nb])
        assert np.array_equal(y.sum(axis=1), dd[:, :nb * f].astype(np.int64).sum(axis=1))
    for a, b in ((2, 5), (10, 3), (4, 4)):
        inner = oracle.downsample(dd, a)
        assert np.array_equal(oracle.downsample(inner.astype(np.int32), b), oracle.downsample(dd, a * b))
    for bad in (0, 1001):
        with pytest.raises(ValueError):
            oracle.downsample(dd, bad)


def test_downsample_snr_closed_form():
    """A constant series with m equal spikes in separate bins: after
    decimation by f the bins form a constant series with m raised bins, whose
    S/N is sqrt((N - m) / m) for N bins (as for the sliding case)."""
    n_out, f = 8000, 10
    dd = np.full((1, n_out), 7, dtype=np.int32)
    for t in (95, 4321):
        dd[0, t] += 1000
    s, p = oracle.snr(oracle.downsample(dd, f))
    nb = n_out // f
    assert s[0] == pytest.approx(np.sqrt((nb - 2) / 2), rel=1e-12)
    assert p[0] == 9       # first raised bin: 95 // 10


# --- S/N ----------------------------------------------------------------------------

def test_snr_matches_numpy_routine():
    rng = np.random.default_rng(5)
    x = rng.integers(-1000, 100000, size=(7, 999)).astype(np.int64)
    s, p = oracle.snr(x)
    for r in range(7):
        xf = x[r].astype(np.float64)
        assert s[r] == pytest.approx((xf.max() - xf.mean()) / xf.std(ddof=0), rel=1e-12)
        assert p[r] == int(np.argmax(x[r]))


def test_snr_closed_form_and_invariance():
    for n, m, h in [(8192, 1, 7), (1000, 10, 123456), (12, 3, 2)]:
        x = np.zeros(n, dtype=np.int64)
        x[n // 3:n // 3 + m] = h
        s, p = oracle.snr(x)
        assert s[0] == pytest.approx(math.sqrt((n - m) / m), rel=1e-12)
        assert p[0] == n // 3
    rng = np.random.default_rng(6)
    x = rng.integers(0, 1000, size=(1, 500)).astype(np.int64)
    s0, p0 = oracle.snr(x)
    s1, p1 = oracle.snr(3 * x + 17)
    assert s1[0] == pytest.approx(s0[0], rel=1e-12) and p1[0] == p0[0]


def test_snr_single_spike_value():
    x = np.zeros(8192, dtype=np.int64)
    x[100] = 5
    assert oracle.snr(x)[0][0] == pytest.approx(90.5041, abs=1e-4)


def test_snr_degenerate_cases():
    s, p = oracle.snr(np.full((2, 50), 42, dtype=np.int64))
    assert np.all(s == 0.0) and np.all(p == 0)
    x = np.array([[1, 5, 2, 5, 5]], dtype=np.int64)
    assert oracle.snr(x)[1][0] == 1              # first of equal maxima
    s, p = oracle.snr(np.array([[9]], dtype=np.int64))
    assert s[0] == 0.0 and p[0] == 0              # one sample: sigma = 0


# --- the injected pulse --------------------------------------------------------------

def _predicted_snr(n_chan, amp, pulse_w, t0, n_out, w, sigma):
    """Closed-form S/N of a noise-free boxcar pulse seen through a sliding window
    of width w, with the noise variance sigma^2 * n_chan * w plus the pulse's own
    variance across the series (the pulse is part of the statistics)."""
    n = n_out - w + 1
    t = np.arange(n)
    overlap = np.clip(np.minimum(t + w, t0 + pulse_w) - np.maximum(t, t0), 0, None)
    s = amp * n_chan * overlap.astype(np.float64)
    return (s.max() - s.mean()) / math.sqrt(sigma ** 2 * n_chan * w + s.var())


def test_injected_pulse_recovered_small():
    wl = workloads.small()
    g = wl.geom
    delays, mx = oracle.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    x, n_in = workloads.make_input(wl, delays, mx)
    dd, s, p = oracle.search(delays, x, n_in, wl.n_out, wl.widths)
    pulse = wl.pulses[0]
    i, k, best = oracle.best_candidate(s)
    assert (i, wl.widths[k]) == (pulse.dm_index, pulse.width)
    sigma = math.sqrt(16.0 ** 2 + 1.0 / 12.0)
    for kk, w in enumerate(wl.widths):
        pred = _predicted_snr(g.n_chan, pulse.amp, pulse.width, pulse.t0, wl.n_out, w, sigma)
        assert abs(s[kk, pulse.dm_index] - pred) < 2.0, (w, s[kk, pulse.dm_index], pred)
        # the peak sits where the window overlaps the pulse
        assert pulse.t0 - w < p[kk, pulse.dm_index] < pulse.t0 + pulse.width
    # off the pulse's DM the detection is weaker
    assert s[:, pulse.dm_index].max() > s[:, pulse.dm_index + 2].max() + 5


# --- best candidate and the workloads' delay constants -------------------------------

def test_best_candidate_tie_rule():
    """Equal S/N values: the smallest DM index wins, then the smallest width
    index (the candidate rule of the search); a transposed loop order or a
    non-strict comparison picks a different entry in one of these tables."""
    s = np.zeros((4, 9))
    s[2, 3] = s[0, 5] = 7.5            # same value at (DM 3, width 2) and (DM 5, width 0)
    assert oracle.best_candidate(s)[:2] == (3, 2)
    s[1, 3] = 7.5                      # and at (DM 3, width 1): same DM, smaller width
    assert oracle.best_candidate(s)[:2] == (3, 1)
    s[3, 8] = 7.5000001                # a strictly larger value anywhere wins
    assert oracle.best_candidate(s)[:2] == (8, 3)
    assert oracle.best_candidate(np.full((3, 4), -1.0))[:2] == (0, 0)


def _exact_delay(f_c, f_top, dm, t_samp):
    """The cold-plasma delay in exact rational arithmetic (decimal inputs taken
    as written), rounded half away from zero: no floating point at all."""
    from fractions import Fraction as Fr
    f_c, f_top, dm, t_samp = (Fr(v if isinstance(v, str) else repr(float(v))) for v in (f_c, f_top, dm, t_samp))
    x = Fr("4148.808") * dm * (1 / f_c ** 2 - 1 / f_top ** 2) / t_samp
    n = math.floor(x)
    return n + 1 if x - n >= Fr(1, 2) else n


def test_workload_delay_constants():
    """The workloads' largest delays and one entry, evaluated independently
    (exact rationals) and as stated for the two workloads: the 256-channel one
    has max delay 1435 and delay 565 at DM 50, channel 0; the 1536-channel beam
    has max delay 11593."""
    small, beam = workloads.small(), workloads.beam()
    g = small.geom
    d, mx = oracle.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    f = g.freqs()
    assert mx == 1435 and d[50, 0] == 565 and d[-1, 0] == mx
    assert _exact_delay(f[0], f.max(), "50", g.t_samp_s) == 565
    assert _exact_delay(f[0], f.max(), "127", g.t_samp_s) == 1435
    g = beam.geom
    d, mx = oracle.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    f = g.freqs()
    assert mx == 11593 and d[-1, 0] == mx
    assert _exact_delay(f[0], f.max(), g.dm_first + (g.n_dm - 1) * g.dm_step,
                        g.t_samp_s) == 11593
    # a few more entries of the beam table, exactly
    rng = np.random.default_rng(17)
    for i, c in zip(rng.integers(0, g.n_dm, 12), rng.integers(0, g.n_chan, 12)):
        dm = g.dm_first + int(i) * g.dm_step
        assert d[i, c] == _exact_delay(f[c], f.max(), dm, g.t_samp_s), (i, c)
