"""What the two-step subband scheme does to a dispersed pulse (test helper).

A pulse injected with the brute-force delays of trial DM_jk, d_c (rounded
exact shifts), sits in channel c at t0 + d_c.  The subband trial (j, k) reads
channel c at t + delay1[s, j, c'] + delay2[j, k, s], so it places that
channel's part of the pulse at t0 + e_c with e_c = d_c - delay1 - delay2:
the smearing.  The composed shift misses the exact one by the intra-subband
residual K (DM_jk - DM_j) (1/f_c^2 - 1/f_ref(s)^2) / t_samp plus at most
one sample of rounding (two roundings of 1/2), and d_c misses it by at most
1/2, so e_c lies within 3/2 of that residual (two-step subband
dedispersion, Section 2).

From the shifts alone follow the pulse's dedispersed series under the
scheme (amp times the number of channels whose shifted pulse covers t) and
the best boxcar sum over it; against brute force, whose series is amp *
n_chan on [t0, t0 + width), their ratio is the fraction of the pulse's
energy one boxcar still collects.
"""
import numpy as np

import oracle

K_DM = 4.148808e3   # MHz^2 pc^-1 cm^3 s, the dispersion constant of the delay tables


def trial_dm(grid, j, k):
    n_sub, n_coarse, cf, cs, n_fine, ff, fs = grid
    return cf + j * cs + ff + k * fs


def pulse_shifts(freqs, t_samp_s, grid, j, k):
    """(e int64 [n_chan], residual float64 [n_chan], brute-force delays d [n_chan]) for trial (j, k)."""
    f = np.asarray(freqs, dtype=np.float64)
    n_sub, n_coarse, cf, cs = grid[:4]
    m = f.shape[0] // n_sub
    d1, d2, _, _ = oracle.subband_delays(f, t_samp_s, *grid)
    dm_jk = trial_dm(grid, j, k)
    d, _ = oracle.delay_table(f, t_samp_s, 1, dm_jk, 0.0)
    composed = d1[:, j, :].reshape(-1).astype(np.int64) + np.repeat(d2[j, k, :].astype(np.int64), m)
    f_ref = f.reshape(n_sub, m).max(axis=1).repeat(m)
    resid = K_DM * (dm_jk - (cf + j * cs)) * (1.0 / f ** 2 - 1.0 / f_ref ** 2) / t_samp_s
    return d[0].astype(np.int64) - composed, resid, d[0]


def smeared_series(e, t0, width, amp, n_out):
    """The pulse's part of the subband trial's dedispersed series (int64 [n_out])."""
    s = np.zeros(n_out + int(e.max()) + width + 1, dtype=np.int64)
    for ec in e:
        a = t0 + int(ec)
        s[a:a + width] += amp
    return s[:n_out]


def best_boxcar(series, width):
    c = np.concatenate([[0], np.cumsum(series)])
    return int((c[width:] - c[:-width]).max())


def noise_sigma(n_chan, width, sd=16.0):
    """Standard deviation of a width-sample boxcar of the dedispersed noise:
    n_chan * width independent samples of the rounded Gaussian (variance sd^2
    plus 1/12 from the rounding; clipping at 0 and 255 is 8 sd away)."""
    return float(np.sqrt(n_chan * width * (sd * sd + 1.0 / 12.0)))


def snr_ratio_floor(frac, peak_bf, sigma, width, n_out, k=5.0):
    """Lowest subband / brute-force S/N ratio the smearing allows.  The
    subband boxcar peak holds frac * peak_bf of signal and brute force's
    peak_bf, each with noise within k standard deviations.  The smeared
    pulse adds less to the boxcar series' variance than the aligned one
    (its series is a sum of shifted copies of the same pulse), so only the
    noise part of the two S/N denominators differs: two estimates of one
    variance from n_out samples of a series correlated over `width` samples,
    whose ratio stays within 3 sqrt(2 width / n_out) of 1."""
    return (frac * peak_bf - k * sigma) / (peak_bf + k * sigma) * (1.0 - 3.0 * np.sqrt(2.0 * width / n_out))


# Pulses (coarse DM j, fine DM k, width, t0) on the 1536-channel beam, one per
# trial, 2048 samples apart, at the largest fine offset (the largest residual),
# a middle one and k = 0 (rounding only); widths from 1 to 16.
BEAM_N_OUT = 12208
PULSE_AMP = 40
GRIDS = {
    # the beam's own 2048 trials (0..1023.5 step 0.5) from 32 subbands
    "beam-grid": ((32, 128, 0.0, 8.0, 16, 0.0, 0.5),
                  [(3, 15, 1, 1024), (20, 15, 2, 3072), (40, 8, 4, 5120), (60, 0, 2, 7168), (90, 15, 16, 9216),
                   (110, 15, 8, 11000)]),
    # the spacing of Table 2's subbanding grid (coarse step 2.4, 24 fine DMs
    # step 0.1), its first 400 coarse DMs
    "table2-spacing": ((32, 400, 0.0, 2.4, 24, 0.0, 0.1),
                       [(30, 23, 1, 1024), (100, 23, 2, 3072), (200, 12, 4, 5120), (300, 0, 2, 7168),
                        (350, 23, 16, 9216), (399, 23, 8, 11000)]),
}
