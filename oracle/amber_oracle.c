/*
 * amber_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of the single-pulse
 * search hot path (delay table, brute-force dedispersion, sliding boxcar
 * integration, S/N peak).  Only the test suite, the smoke entry point and the
 * CPU-baseline leg of the benchmark may load it; the product library shares
 * no code with it and never calls it.
 *
 * Every function writes out the definition it follows, in FP64 where floating
 * point is involved, with no blocking, fusion or reordering.  The only
 * concession to speed is an OpenMP loop over independent DM trials / rows,
 * which does not change any arithmetic.
 *
 * Where the paper is silent (it prints no delay formula, smoothing definition
 * or S/N formula) the reading used here is stated at each function.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Cold-plasma dispersion constant, seconds * MHz^2 / (pc cm^-3). */
#define ORACLE_KDM 4.148808e3

static int oracle_threads(int n_threads)
{
#ifdef _OPENMP
    return n_threads > 0 ? n_threads : omp_get_max_threads();
#else
    (void)n_threads;
    return 1;
#endif
}

/*
 * Dispersion delay table.
 *
 * Section 1 of the paper names dedispersion as the shift and integration of
 * frequency channels that removes the frequency dispersion of a pulse.  The
 * paper prints no formula; this is the textbook delay of a cold-plasma pulse
 * at frequency f relative to the highest channel frequency f_top:
 *
 *     delay[i][c] = round( K * DM_i * (1/f_c^2 - 1/f_top^2) / t_samp )
 *
 * with DM_i = dm_first + i * dm_step (by multiplication, Table 2's
 * DM_FIRST / DM_STEP), K = 4.148808e3 s MHz^2 pc^-1 cm^3, rounding half away
 * from zero.  f_top is the largest entry of freq_mhz, so the top channel has
 * delay 0 and lower channels arrive later (positive delays).
 *
 * Returns 0, or -1 on bad arguments (non-positive sizes, sampling time or
 * frequencies).  max_delay receives the largest entry.
 */
int oracle_delay_table(int n_chan, const double *freq_mhz, double t_samp_s,
                       int n_dm, double dm_first, double dm_step,
                       int32_t *delays, int32_t *max_delay)
{
    if (n_chan <= 0 || n_dm <= 0 || !(t_samp_s > 0.0) || !freq_mhz || !delays)
        return -1;
    double f_top = freq_mhz[0];
    for (int c = 0; c < n_chan; ++c) {
        if (!(freq_mhz[c] > 0.0))
            return -1;
        if (freq_mhz[c] > f_top)
            f_top = freq_mhz[c];
    }
    int32_t dmax = INT32_MIN;
    for (int i = 0; i < n_dm; ++i) {
        double dm = dm_first + (double)i * dm_step;
        for (int c = 0; c < n_chan; ++c) {
            double f = freq_mhz[c];
            double x = ((ORACLE_KDM * dm) * (1.0 / (f * f) - 1.0 / (f_top * f_top))) / t_samp_s;
            int32_t d = (int32_t)llround(x);
            delays[(size_t)i * n_chan + c] = d;
            if (d > dmax)
                dmax = d;
        }
    }
    if (max_delay)
        *max_delay = dmax;
    return 0;
}

/*
 * Brute-force incoherent dedispersion (the one-step dedispersion the paper
 * contrasts with its two-step subband scheme in Section 5):
 *
 *     dd[i][t] = sum over c of in[c][t + delay[i][c]],   0 <= t < n_out
 *
 * in is channel-major uint8 with row stride `stride` bytes; dd is int32 with
 * row stride n_out.  Every sample read must exist: 0 <= delay and
 * n_out + delay <= n_in, otherwise -1 is returned and nothing is written.
 */
int oracle_dedisperse(const int32_t *delays, int n_dm, int n_chan,
                      const uint8_t *in, int64_t stride, int64_t n_in,
                      int64_t n_out, int32_t *dd, int n_threads)
{
    if (n_dm <= 0 || n_chan <= 0 || n_out < 0 || n_in < 0 || stride < n_in)
        return -1;
    for (size_t k = 0; k < (size_t)n_dm * n_chan; ++k)
        if (delays[k] < 0 || n_out + delays[k] > n_in)
            return -1;
    int nt = oracle_threads(n_threads);
    #pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
    for (int i = 0; i < n_dm; ++i) {
        const int32_t *drow = delays + (size_t)i * n_chan;
        for (int64_t t = 0; t < n_out; ++t) {
            int32_t sum = 0;
            for (int c = 0; c < n_chan; ++c)
                sum += in[(size_t)c * stride + (size_t)(t + drow[c])];
            dd[(size_t)i * n_out + t] = sum;
        }
    }
    return 0;
}

/*
 * Dedispersion with zapped channels (channels excluded because of radio
 * frequency interference; the paper's pipeline reads them from an input
 * file, Section 2 footnote):
 *
 *     dd[i][t] = sum over c with keep[c] != 0 of in[c][t + delay[i][c]]
 *
 * Same arguments and checks as oracle_dedisperse, plus keep[n_chan].
 */
int oracle_dedisperse_masked(const int32_t *delays, int n_dm, int n_chan,
                             const uint8_t *in, int64_t stride, int64_t n_in,
                             int64_t n_out, const uint8_t *keep, int32_t *dd,
                             int n_threads)
{
    if (n_dm <= 0 || n_chan <= 0 || n_out < 0 || n_in < 0 || stride < n_in || !keep)
        return -1;
    for (size_t k = 0; k < (size_t)n_dm * n_chan; ++k)
        if (delays[k] < 0 || n_out + delays[k] > n_in)
            return -1;
    int nt = oracle_threads(n_threads);
    #pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
    for (int i = 0; i < n_dm; ++i) {
        const int32_t *drow = delays + (size_t)i * n_chan;
        for (int64_t t = 0; t < n_out; ++t) {
            int32_t sum = 0;
            for (int c = 0; c < n_chan; ++c)
                if (keep[c])
                    sum += in[(size_t)c * stride + (size_t)(t + drow[c])];
            dd[(size_t)i * n_out + t] = sum;
        }
    }
    return 0;
}

/*
 * Two-step subband dedispersion (the pipeline's dedispersion, Section 2 and
 * its footnote; Table 2 SUBBANDS, SUBBANDING_DMS / _DM_FIRST / _DM_STEP and
 * DMS / DM_FIRST / DM_STEP).  Subband s holds channels s*m .. s*m + m - 1
 * (m = n_chan / n_sub); its reference frequency f_ref(s) is the largest
 * frequency among them, f_top the largest of all.
 *
 *   coarse DM_j  = cdm_first + j * cdm_step,            j < n_coarse
 *   trial DM_jk  = DM_j + fdm_first + k * fdm_step,      k < n_fine
 *   delay1[s][j][c'] = round(K DM_j  (1/f_c^2      - 1/f_ref(s)^2) / t_samp),  c = s m + c'
 *   delay2[j][k][s]  = round(K DM_jk (1/f_ref(s)^2 - 1/f_top^2)    / t_samp)
 *
 * max1 / max2 receive the largest entries.
 */
int oracle_subband_delays(int n_chan, const double *freq, double t_samp_s, int n_sub, int n_coarse,
                          double cdm_first, double cdm_step, int n_fine, double fdm_first, double fdm_step,
                          int32_t *delay1, int32_t *delay2, int32_t *max1, int32_t *max2)
{
    if (n_chan <= 0 || n_sub <= 0 || n_chan % n_sub != 0 || n_coarse <= 0 || n_fine <= 0 ||
        !(t_samp_s > 0.0) || !freq || !delay1 || !delay2)
        return -1;
    const int m = n_chan / n_sub;
    double f_top = freq[0];
    for (int c = 0; c < n_chan; ++c) {
        if (!(freq[c] > 0.0))
            return -1;
        if (freq[c] > f_top)
            f_top = freq[c];
    }
    int32_t m1 = INT32_MIN, m2 = INT32_MIN;
    for (int s = 0; s < n_sub; ++s) {
        double f_ref = freq[s * m];
        for (int c = s * m; c < (s + 1) * m; ++c)
            if (freq[c] > f_ref)
                f_ref = freq[c];
        for (int j = 0; j < n_coarse; ++j) {
            double dm = cdm_first + (double)j * cdm_step;
            for (int cl = 0; cl < m; ++cl) {
                double f = freq[s * m + cl];
                double x = ((ORACLE_KDM * dm) * (1.0 / (f * f) - 1.0 / (f_ref * f_ref))) / t_samp_s;
                int32_t d = (int32_t)llround(x);
                delay1[((size_t)s * n_coarse + j) * m + cl] = d;
                if (d > m1)
                    m1 = d;
            }
            for (int k = 0; k < n_fine; ++k) {
                double dmk = dm + fdm_first + (double)k * fdm_step;
                double x = ((ORACLE_KDM * dmk) * (1.0 / (f_ref * f_ref) - 1.0 / (f_top * f_top))) / t_samp_s;
                int32_t d = (int32_t)llround(x);
                delay2[((size_t)j * n_fine + k) * n_sub + s] = d;
                if (d > m2)
                    m2 = d;
            }
        }
    }
    if (max1)
        *max1 = m1;
    if (max2)
        *max2 = m2;
    return 0;
}

/*
 * The two steps composed, evaluated directly (no intermediate subband sums):
 *
 *   dd[j n_fine + k][t] = sum over s, c in s of in[c][t + delay2[j][k][s] + delay1[s][j][c']]
 *
 * for t < n_out; every index must stay inside [0, n_in).
 */
int oracle_subband_dedisperse(const int32_t *delay1, const int32_t *delay2, int n_chan, int n_sub,
                              int n_coarse, int n_fine, const uint8_t *in, int64_t stride, int64_t n_in,
                              int64_t n_out, int32_t *dd, int n_threads)
{
    if (n_chan <= 0 || n_sub <= 0 || n_chan % n_sub != 0 || n_coarse <= 0 || n_fine <= 0 || n_out < 0 ||
        stride < n_in)
        return -1;
    const int m = n_chan / n_sub;
    for (int j = 0; j < n_coarse; ++j)
        for (int k = 0; k < n_fine; ++k)
            for (int s = 0; s < n_sub; ++s)
                for (int cl = 0; cl < m; ++cl) {
                    int64_t d = (int64_t)delay2[((size_t)j * n_fine + k) * n_sub + s] +
                                delay1[((size_t)s * n_coarse + j) * m + cl];
                    if (d < 0 || n_out + d > n_in)
                        return -1;
                }
    int nt = oracle_threads(n_threads);
    #pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
    for (int jk = 0; jk < n_coarse * n_fine; ++jk) {
        const int j = jk / n_fine, k = jk % n_fine;
        for (int64_t t = 0; t < n_out; ++t) {
            int32_t sum = 0;
            for (int s = 0; s < n_sub; ++s) {
                const int64_t d2 = delay2[((size_t)j * n_fine + k) * n_sub + s];
                for (int cl = 0; cl < m; ++cl) {
                    const int c = s * m + cl;
                    const int64_t d1 = delay1[((size_t)s * n_coarse + j) * m + cl];
                    sum += in[(size_t)c * stride + (size_t)(t + d2 + d1)];
                }
            }
            dd[(size_t)jk * n_out + t] = sum;
        }
    }
    return 0;
}

/*
 * Sliding boxcar integration of one dedispersed series ("smoothing" of the
 * dedispersed time series, Section 2), for a single width w:
 *
 *     box[t] = sum over k < w of dd[t + k],   0 <= t < n_out - w + 1
 *
 * rows of dd have stride n_out; rows of box have stride n_out - w + 1 and are
 * int64.  Returns -1 unless 1 <= w <= n_out.
 */
int oracle_boxcar(const int32_t *dd, int n_dm, int64_t n_out, int w,
                  int64_t *box, int n_threads)
{
    if (n_dm <= 0 || w < 1 || w > n_out)
        return -1;
    int64_t nw = n_out - w + 1;
    int nt = oracle_threads(n_threads);
    #pragma omp parallel for num_threads(nt) schedule(static)
    for (int i = 0; i < n_dm; ++i) {
        const int32_t *row = dd + (size_t)i * n_out;
        for (int64_t t = 0; t < nw; ++t) {
            int64_t s = 0;
            for (int k = 0; k < w; ++k)
                s += row[t + k];
            box[(size_t)i * nw + t] = s;
        }
    }
    return 0;
}

/*
 * Decimating downsampling (the downsampling step of Section 2; Table 2 gives
 * the factors and NRSAMPLES = SAMPLES / DOWNSAMPLING):
 *
 *     y[i][j] = sum_{k<f} dd[i][j*f + k]     for j < floor(n_out / f)
 *
 * rows of dd have stride n_out; rows of y have stride floor(n_out / f) and
 * are int64.  Samples past the last whole bin are dropped.  Returns -1 unless
 * 1 <= f <= n_out.
 */
int oracle_downsample(const int32_t *dd, int n_dm, int64_t n_out, int f,
                      int64_t *y, int n_threads)
{
    if (n_dm <= 0 || f < 1 || f > n_out)
        return -1;
    int64_t nb = n_out / f;
    int nt = oracle_threads(n_threads);
    #pragma omp parallel for num_threads(nt) schedule(static)
    for (int i = 0; i < n_dm; ++i) {
        const int32_t *row = dd + (size_t)i * n_out;
        for (int64_t j = 0; j < nb; ++j) {
            int64_t s = 0;
            for (int k = 0; k < f; ++k)
                s += row[j * f + k];
            y[(size_t)i * nb + j] = s;
        }
    }
    return 0;
}

/*
 * Signal-to-noise of the peak of each series (the S/N step of Section 2):
 *
 *     mu    = (1/N) sum x[t]
 *     sigma = sqrt( (1/N) sum (x[t] - mu)^2 )          (population, two-pass)
 *     snr   = (max x - mu) / sigma,   or 0 when sigma == 0
 *     peak  = smallest t with x[t] == max x
 *
 * over the N values of each row (stride N).  All arithmetic in FP64.
 */
int oracle_snr(const int64_t *x, int n_rows, int64_t n, double *snr,
               int32_t *peak, int n_threads)
{
    if (n_rows <= 0 || n < 1)
        return -1;
    int nt = oracle_threads(n_threads);
    #pragma omp parallel for num_threads(nt) schedule(static)
    for (int r = 0; r < n_rows; ++r) {
        const int64_t *row = x + (size_t)r * n;
        double sum = 0.0;
        int64_t best = row[0];
        int64_t best_t = 0;
        for (int64_t t = 0; t < n; ++t) {
            sum += (double)row[t];
            if (row[t] > best) {
                best = row[t];
                best_t = t;
            }
        }
        double mu = sum / (double)n;
        double ss = 0.0;
        for (int64_t t = 0; t < n; ++t) {
            double d = (double)row[t] - mu;
            ss += d * d;
        }
        double sigma = sqrt(ss / (double)n);
        snr[r] = sigma > 0.0 ? ((double)best - mu) / sigma : 0.0;
        peak[r] = (int32_t)best_t; /* all values equal when sigma == 0: t = 0 */
    }
    return 0;
}
