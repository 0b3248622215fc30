/*
 * amber.h -- C ABI of the MI355X (gfx950) single-pulse search hot path.
 *
 * The hot path follows the pipeline the paper tunes (Section 2: dedispersion,
 * smoothing of the dedispersed series, S/N computation), with brute-force
 * one-step dedispersion (Section 5 names it beside the two-step subband
 * scheme) and a sliding boxcar as the smoothing step:
 *
 *   amber_delay_table   host, FP64: integer delay per (DM trial, channel)
 *   amber_dedisperse    device: dd[i][t] = sum_c in[c][t + delay[i][c]]
 *   amber_integrate     device: box_w[i][t] = sum_{k<w} dd[i][t+k]
 *   amber_snr           device: per (w, i) peak, first argmax, mean, std -> S/N
 *   amber_integrate_snr device: the previous two fused, box never stored
 *   amber_downsample    device: decimating downsampling (sums of f samples)
 *   amber_downsample_snr device: downsampling + S/N fused
 *   amber_tune          genetic-algorithm tile search (Section 3), fitness =
 *                       measured time of dedisperse + integrate + S/N
 *
 * Conventions
 * - Every buffer is owned by the caller.  "d_" pointers are device (HBM)
 *   pointers, everything else is host memory.  The library never frees or
 *   reallocates caller memory.
 * - Device work is enqueued on `stream` (a hipStream_t, NULL = the default
 *   stream) and returns without synchronising, except amber_tune, which
 *   must time kernels.
 * - Arguments are validated before any launch; a failed call returns a
 *   negative amber_status, launches nothing, and sets a thread-local message
 *   readable with amber_last_error().  The library never aborts the process.
 * - Layouts are row-major.  The input is channel-major uint8: row c holds the
 *   samples of channel c, contiguous in time, rows `in_stride` bytes apart.
 */
#ifndef AMBER_H
#define AMBER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AMBER_OK = 0,
    AMBER_E_ARG = -1,     /* bad pointer, size or value */
    AMBER_E_SHAPE = -2,   /* buffers too small for the requested work */
    AMBER_E_CONFIG = -3,  /* tile configuration outside the kernel's space */
    AMBER_E_DEVICE = -4,  /* HIP runtime or launch error */
    AMBER_E_NOMEM = -5,   /* device allocation failed */
    AMBER_E_TIMEOUT = -6  /* a timed evaluation exceeded its limit, or a wait ended empty */
} amber_status;

#define AMBER_MAX_WIDTHS 16

/* Message of the last failed call on this thread ("" if none).  Valid until
 * the next amber_* call on the same thread. */
const char *amber_last_error(void);

/* Library version string. */
const char *amber_version(void);

/* Observation geometry, the analogue of the paper's Table 2 fixed parameters
 * (channels, frequencies, sampling time, DM_FIRST / DM_STEP / DMS). */
typedef struct {
    int32_t n_chan;
    const double *freq_mhz;   /* [n_chan] channel frequencies, any order, > 0 */
    double t_samp_s;          /* sampling time, seconds, > 0 */
    int32_t n_dm;             /* number of DM trials, > 0 */
    double dm_first;          /* first DM trial, pc cm^-3, >= 0 */
    double dm_step;           /* DM trial spacing, pc cm^-3, >= 0 */
} amber_geometry;

/* Summary of a delay table, filled by amber_delay_table and required by
 * amber_dedisperse to size its LDS windows and validate its reads. */
typedef struct {
    int32_t n_dm;
    int32_t n_chan;
    int32_t max_delay;  /* largest entry (all entries are >= 0) */
    int32_t max_step;   /* largest delay[i+1][c] - delay[i][c]; entries never
                           decrease along i */
} amber_delay_info;

/* Tunable tile parameters, the analogue of the paper's Table 3 user-controlled
 * parameters, re-derived for gfx950 (64-wide wavefronts):
 *   threads_per_dm     work-items along time per DM trial
 *                      (nrSamplesPerBlock); a multiple of 64, <= 1024
 *   samples_per_thread output samples per work-item (nrSamplesPerThread);
 *                      4, 8, 16 or 32 (even: samples go in pairs)
 *   dms_per_block      DM trials per work-group (nrDMsPerBlock), >= 1, with
 *                      threads_per_dm * dms_per_block <= 1024
 *   channel_unroll     channels staged in LDS per step (unroll); 1..32, power
 *                      of two
 *   snr_threads        work-items per work-group of the boxcar / S/N kernels
 *                      (nrThreadsD0); 64..1024, power of two.  In the fused
 *                      kernel for up to 8 sliding widths of at most 64
 *                      samples: snr_threads / 64 wavefronts share a row
 *   boxcar_step[k]     consecutive outputs per work-item for width k of the
 *                      boxcar / S/N kernels (nrItemsD0, one per width as the
 *                      paper has one per downsampling factor); 1, 2, 4 or 8.
 *                      Used by decimation, by the materialised boxcar / S/N
 *                      and by the fused kernel for more or wider widths; the
 *                      fused kernel for up to 8 sliding widths of at most 64
 *                      samples reads every width from one prefix per 4
 *                      outputs and has no such gene (the value must still be
 *                      valid)
 *   dms_per_thread     DM trials per wavefront (nrDMsPerThread): 1 or 2 (2
 *                      with samples_per_thread <= 16); 0 reads as 1.  A
 *                      work-group covers dms_per_block * dms_per_thread DMs,
 *                      and every staged window serves all of them
 *   direct_reads       how the dedispersion kernel reads its input (the
 *                      paper's localMem gene): 0 (the default) stages each
 *                      channel's window in LDS (localMem on); 1 reads it
 *                      straight from global memory through the caches
 *                      (localMem off), with dms_per_thread 1 and
 *                      (samples_per_thread / 4 + 1) * channel_unroll <= 64
 *                      (the dwords a work-item loads per channel group).
 *                      uint8 input only: the subband steps take 0.
 * The LDS footprint of the dedispersion tile must fit in 160 KiB and its
 * staging must need at most 4 items of 16 samples per work-item (3 when
 * samples_per_thread is 16, 2 when it is 32 or when it is 16 with two DMs per
 * wavefront); direct reads use no LDS. */
typedef struct {
    int32_t threads_per_dm;
    int32_t samples_per_thread;
    int32_t dms_per_block;
    int32_t channel_unroll;
    int32_t snr_threads;
    int32_t boxcar_step[AMBER_MAX_WIDTHS];
    int32_t dms_per_thread;
    int32_t direct_reads;
} amber_tiles;

/* Fill `tiles` with the library's default configuration. */
amber_status amber_default_tiles(amber_tiles *tiles);

/* The default configuration adapted to a delay table and a series length:
 * channel_unroll, then dms_per_block are halved, then dms_per_thread drops to
 * 1, then samples_per_thread is halved, until the dedispersion tile fits.
 * Then, if n_out > 0 and the dedispersion launch would have fewer than 384
 * work-groups (1.5 per CU of the 256), the tile is made smaller until it has
 * that many or neither step is left: samples_per_thread halved down to 4
 * (channel_unroll 32), then dms_per_thread 1 (channel_unroll 32); a step
 * whose channel_unroll 32 does not fit keeps the previous channel_unroll.
 * n_out <= 0 skips this.  This is what
 * the device calls use when passed tiles == NULL (with their own n_out; the
 * streaming service with its chunk length).  AMBER_E_CONFIG if nothing fits. */
amber_status amber_auto_tiles(const amber_delay_info *info, int64_t n_out, amber_tiles *tiles);

/* Check `tiles` against the kernels' space for a problem of this shape;
 * AMBER_OK or AMBER_E_CONFIG (with the reason in amber_last_error). */
amber_status amber_validate_tiles(const amber_tiles *tiles, const amber_delay_info *info,
                                  int32_t n_widths);

/* Dispersion delay table (host, FP64).
 *
 * Dedispersion shifts each frequency channel by the dispersion delay of its
 * frequency and sums the channels (Section 1).  The paper prints no formula;
 * the library uses the cold-plasma delay relative to the highest channel
 * frequency f_top:
 *     delay[i][c] = round(4.148808e3 * DM_i * (f_c^-2 - f_top^-2) / t_samp)
 * with DM_i = dm_first + i * dm_step, frequencies in MHz, t_samp in seconds,
 * rounding half away from zero.
 *
 * delays: host int32 [n_dm][n_chan], caller-owned, fully overwritten.
 * info:   filled with the table's summary (may be NULL).
 * Errors: AMBER_E_ARG for NULL pointers, non-positive sizes, t_samp or
 * frequencies, negative dm_first / dm_step, or delays beyond int32. */
amber_status amber_delay_table(const amber_geometry *g, int32_t *delays, amber_delay_info *info);

/* Brute-force dedispersion on the device (Section 2: the dedispersion
 * kernel; Section 5: one-step brute-force dedispersion):
 *     dd[i][t] = sum over c < n_chan of in[c][t + delay[i][c]],  t < n_out
 * integer sums, exact (int32).
 *
 * d_delays:  device int32 [info->n_dm][info->n_chan], the table described by
 *            info (as written by amber_delay_table).
 * d_in:      device uint8 [n_chan][in_stride]; in_stride >= n_in and a
 *            multiple of 4; n_in >= n_out + info->max_delay.
 * d_dd:      device int32 [n_dm][dd_stride]; dd_stride >= n_out.  Columns
 *            >= n_out are not written.  n_out = 0 is valid: the arguments
 *            are checked, nothing is launched, and d_dd may be NULL.
 * tiles:     NULL = amber_auto_tiles(info, n_out).
 * Errors: AMBER_E_SHAPE also when channel_unroll * in_stride >= 2^32 - 64
 * bytes (the staged kernel addresses a channel group's rows with 32-bit
 * offsets; tiles with direct_reads have no such limit).  The same limit holds
 * for amber_dedisperse_masked, the batch and the server's beams, and for both
 * subband steps (step two's slices of coarse DMs are cut to fit it).
 * Reads stay inside the n_chan * in_stride input bytes and the LDS tile even
 * if the table does not match info; results are then meaningless but the call
 * cannot fault. */
amber_status amber_dedisperse(const int32_t *d_delays, const amber_delay_info *info,
                              const uint8_t *d_in, int64_t in_stride, int64_t n_in,
                              int32_t *d_dd, int64_t dd_stride, int64_t n_out,
                              const amber_tiles *tiles, void *stream);

/* amber_dedisperse with zapped channels (channels flagged because of radio
 * frequency interference, which the paper's pipeline reads from an input
 * file; Section 2 footnote):
 *     dd[i][t] = sum over c with keep[c] != 0 of in[c][t + delay[i][c]]
 * d_keep: device uint8 [n_chan], caller-owned; 0 = zapped.  A zapped row is
 * never read.  Other arguments and errors as amber_dedisperse (AMBER_E_ARG if
 * d_keep is NULL). */
amber_status amber_dedisperse_masked(const int32_t *d_delays, const amber_delay_info *info,
                                     const uint8_t *d_in, int64_t in_stride, int64_t n_in,
                                     int32_t *d_dd, int64_t dd_stride, int64_t n_out,
                                     const uint8_t *d_keep, const amber_tiles *tiles, void *stream);

/* Two-step subband dedispersion (Section 2 footnote; Table 2's subbanding
 * parameters: subbands, subbanding DMs and DMs per subbanding DM, each with
 * first and step).
 *
 * The channels are split into n_subbands consecutive groups of
 * m = n_chan / n_subbands channels.  Step one dedisperses every subband at the
 * coarse DMs DM_j = coarse_first + j * coarse_step, relative to the
 * subband's highest frequency f_ref(s); step two shifts and sums the subbands
 * for the fine DMs DM_jk = DM_j + fine_first + k * fine_step, relative to
 * f_top.  Trial j * n_fine + k is
 *     dd[j n_fine + k][t] = sum over s, c' < m of in[s m + c'][t + D2 + D1]
 *     D1 = round(4.148808e3 * DM_j  * (f_c^-2      - f_ref(s)^-2) / t_samp)
 *     D2 = round(4.148808e3 * DM_jk * (f_ref(s)^-2 - f_top^-2)    / t_samp)
 * (rounding half away from zero, FP64, DM_jk evaluated as
 * (DM_j + fine_first) + k * fine_step).  It approximates brute-force
 * dedispersion at DM_jk: inside a subband the channels are aligned for DM_j. */
typedef struct {
    int32_t n_chan;
    const double *freq_mhz;   /* [n_chan] channel frequencies, > 0; subband s is
                                 channels [s m, (s + 1) m) in this order */
    double t_samp_s;          /* sampling time, seconds, > 0 */
    int32_t n_subbands;       /* divides n_chan; n_chan / n_subbands <= 257 */
    int32_t n_coarse;         /* subbanding (coarse) DM trials, >= 1 */
    double coarse_first;      /* >= 0 */
    double coarse_step;       /* >= 0 */
    int32_t n_fine;           /* DM trials per coarse DM, >= 1 */
    double fine_first;        /* coarse_first + fine_first >= 0 */
    double fine_step;         /* >= 0 */
} amber_subband_geometry;

/* Summary of the two subband tables (amber_subband_delay_tables). */
typedef struct {
    int32_t n_chan, n_subbands, n_coarse, n_fine;
    int32_t max_delay1;  /* largest delay1 entry */
    int32_t max_step1;   /* largest delay1[s][j+1][c'] - delay1[s][j][c'] */
    int32_t max_delay2;  /* largest delay2 entry */
    int32_t max_step2;   /* largest delay2[j][k+1][s] - delay2[j][k][s] */
    int32_t max_delay;   /* max_delay1 + max_delay2: the input samples needed
                            beyond n_out */
} amber_subband_info;

/* The subband scheme's delays as the device path uses them (host, FP64).
 * Each coarse DM's smallest step-two shift of subband s, B[j][s] = D2 at
 * k = 0, is moved into step one, so that step one computes only the samples
 * step two reads:
 *     delay1[s][j][c'] = D1(s, j, c') + B[j][s]     int32 [n_subbands][n_coarse][m]
 *     delay2[j][k][s]  = D2(j, k, s)  - B[j][s]     int32 [n_coarse][n_fine][n_subbands]
 * Sums delay1 + delay2 are the scheme's composed delays exactly.  All entries
 * are >= 0 and never decrease along j (delay1) or k (delay2).
 * delay1, delay2: caller-owned host buffers, fully overwritten.
 * info: filled (may be NULL).
 * Errors: AMBER_E_ARG for NULL pointers, sizes < 1, n_subbands not dividing
 * n_chan, more than 257 channels per subband (step-one sums are stored in 16
 * bits), frequencies <= 0, t_samp <= 0, negative DMs or steps, delays beyond
 * int32. */
amber_status amber_subband_delay_tables(const amber_subband_geometry *g, int32_t *delay1, int32_t *delay2,
                                        amber_subband_info *info);

/* Two-step subband dedispersion on the device (formula above).
 * d_delay1, d_delay2: device copies of amber_subband_delay_tables' tables.
 * d_in:   device uint8 [n_chan][in_stride] as amber_dedisperse;
 *         n_in >= n_out + info->max_delay.
 * d_work: device uint16 [n_subbands][n_coarse][work_stride], caller-owned
 *         scratch; receives step one's sums: row (s, j) holds
 *         sum over c' of in[s m + c'][t + delay1[s][j][c']] for
 *         t < n_out + info->max_delay2 (later columns are not written).
 *         work_stride >= n_out + max_delay2, even, >= 32; d_work 4-byte
 *         aligned.
 * d_dd:   device int32 [n_coarse * n_fine][dd_stride], dd_stride >= n_out.
 * d_keep: device uint8 [n_chan] keep flags as amber_dedisperse_masked, or
 *         NULL for every channel.
 * tiles1: step one's tiles (dedispersion genes), tiles2: step two's (its
 *         kernels take samples_per_thread 8 or 16 and channel_unroll >= 4);
 *         NULL picks a valid default for each.
 * Asynchronous on `stream` (two launches).  Errors: AMBER_E_ARG, AMBER_E_SHAPE
 * (strides, lengths, alignment), AMBER_E_CONFIG (tiles), AMBER_E_DEVICE. */
amber_status amber_subband_dedisperse(const int32_t *d_delay1, const int32_t *d_delay2,
                                      const amber_subband_info *info, const uint8_t *d_in, int64_t in_stride,
                                      int64_t n_in, uint16_t *d_work, int64_t work_stride, int32_t *d_dd,
                                      int64_t dd_stride, int64_t n_out, const uint8_t *d_keep,
                                      const amber_tiles *tiles1, const amber_tiles *tiles2, void *stream);

/* amber_subband_dedisperse for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops or harnesses that forbid
 * allocation): no d_work argument and no allocation of any kind.  Step one's
 * sums go to a device array that is part of the library
 * (amber_subband_static_bytes(), 32 MiB; each GPU the library runs on holds
 * its own copy until the process ends), with rows of n_out + max_delay2
 * samples rounded up to 64.  The coarse DMs run in slices of as many as that
 * array holds (two launches per slice); dd is the same as
 * amber_subband_dedisperse's with the same tiles.
 * Every call on one GPU shares that GPU's array: calls that overlap on the
 * same GPU (other streams, other threads) race and give undefined results.
 * Nothing in the array needs to start at zero.
 * Errors: those of amber_subband_dedisperse, and AMBER_E_SHAPE when one coarse
 * DM's step-one rows (n_subbands * row bytes) exceed the array. */
amber_status amber_subband_dedisperse_noalloc(const int32_t *d_delay1, const int32_t *d_delay2,
                                              const amber_subband_info *info, const uint8_t *d_in,
                                              int64_t in_stride, int64_t n_in, int32_t *d_dd, int64_t dd_stride,
                                              int64_t n_out, const uint8_t *d_keep, const amber_tiles *tiles1,
                                              const amber_tiles *tiles2, void *stream);

/* Bytes of the device array amber_subband_dedisperse_noalloc uses. */
int64_t amber_subband_static_bytes(void);

/* Sliding boxcar integration (the smoothing of each dedispersed series,
 * Section 2; a sliding window here, the decimation of Table 2 is
 * amber_downsample):
 *     box[k][i][t] = sum over j < widths[k] of dd[i][t + j],
 *     t < n_out - widths[k] + 1
 * d_dd:  device int32 [n_dm][dd_stride].
 * d_box: device int32 [n_widths][n_dm][box_stride], box_stride >= n_out;
 *        columns >= n_out - widths[k] + 1 are not written.
 * widths: host int32 [n_widths], 1 <= widths[k] <= min(n_out, 1024),
 *        n_widths <= AMBER_MAX_WIDTHS.  Sums must fit int32: the caller
 *        guarantees |dd| * max(widths) < 2^31 (true for uint8 input when
 *        n_chan * 255 * max(widths) < 2^31). */
amber_status amber_integrate(const int32_t *d_dd, int32_t n_dm, int64_t dd_stride, int64_t n_out,
                             const int32_t *widths, int32_t n_widths,
                             int32_t *d_box, int64_t box_stride,
                             const amber_tiles *tiles, void *stream);

/* S/N of each boxcar series (Section 2: the S/N kernel), over its
 * N = n_out - widths[k] + 1 values:
 *     mean = sum x / N,  std = sqrt(sum (x - mean)^2 / N)   (population)
 *     snr[k][i] = (max x - mean) / std, or 0 when std == 0
 *     peak_t[k][i] = smallest t with x[t] == max x
 * Moments are accumulated in FP64 about a per-row integer reference, the
 * finish is FP64, snr is stored as float32.
 * d_box:    device int32 [n_widths][n_dm][box_stride] (as amber_integrate).
 * d_snr:    device float [n_widths][n_dm].
 * d_peak_t: device int32 [n_widths][n_dm], or NULL. */
amber_status amber_snr(const int32_t *d_box, int32_t n_dm, int64_t box_stride, int64_t n_out,
                       const int32_t *widths, int32_t n_widths,
                       float *d_snr, int32_t *d_peak_t,
                       const amber_tiles *tiles, void *stream);

/* amber_integrate followed by amber_snr in one kernel (Section 2: the
 * smoothing and S/N kernels after dedispersion): each dedispersed row is read
 * once and its boxcar series live only in LDS and registers.  Same arguments
 * and results as the pair, without d_box.
 * Up to 8 sliding widths of at most 64 samples (rows below 2^29 samples) take
 * a kernel in which the work-group's wavefronts sweep consecutive spans of
 * the row: per 256 outputs a prefix in LDS, per width the maximum, the block
 * where it first rises and an exact int64 sum of squares; the mean follows
 * from the row's sum in closed form.  Its results are exact (up to the FP64
 * finish) for dd >= 0 with dd * max(widths) < 2^31 (any dedispersed uint8
 * data), and for signed dd with |dd| * max(widths) < 2^30; a row whose values
 * could overflow the int64 sums has them recomputed in FP64.  More or wider
 * widths take the chunked kernel of amber_integrate.
 * tiles == NULL: the defaults, with snr_threads 64 when n_dm >= 4096 (with
 * that many rows one wavefront per row keeps the CUs busiest) and the default
 * 128 below, raised while 16 * snr_threads < twice the largest width rounded
 * up to 16.  A batch with automatic tiles applies the same rule to its total
 * number of rows. */
amber_status amber_integrate_snr(const int32_t *d_dd, int32_t n_dm, int64_t dd_stride, int64_t n_out,
                                 const int32_t *widths, int32_t n_widths,
                                 float *d_snr, int32_t *d_peak_t,
                                 const amber_tiles *tiles, void *stream);

/* ---- decimating downsampling (Section 2; Table 2 DOWNSAMPLING, NRSAMPLES) -- */

/* The pipeline's downsampling step: for each factor f = factors[k],
 *     y[k][i][j] = sum_{m<f} dd[i][j*f + m]      for j < n_out / f
 * (integer division: samples past the last whole bin are dropped; Table 2
 * gives NRSAMPLES = SAMPLES / DOWNSAMPLING and factors 10 ... 3200).  The same
 * prefix-sum kernel as amber_integrate, read at multiples of f, exact in
 * int32 while f * 255 * n_chan < 2^31.
 * factors: host [n_factors], 1 <= f <= min(n_out, 4096), n_factors <= 16.
 * d_y:     device int32 [n_factors][n_dm][y_stride], y_stride >= n_out / min f.
 * tiles:   snr_threads and boxcar_step[k] (one per factor, as the paper has
 *          one gene per downsampling factor) are used; NULL = defaults with
 *          snr_threads raised until 16 * snr_threads >= 2 * round16(max f)
 *          and boxcar_step 1 for every factor. */
amber_status amber_downsample(const int32_t *d_dd, int32_t n_dm, int64_t dd_stride, int64_t n_out,
                              const int32_t *factors, int32_t n_factors, int32_t *d_y, int64_t y_stride,
                              const amber_tiles *tiles, void *stream);

/* Downsampling followed by S/N (Section 2's S/N kernel on each downsampled
 * series), fused: per (k, i) over the N = n_out / factors[k] values y_j,
 *     snr[k][i] = (max y - mean) / std (population), or 0 when std == 0,
 *     peak_t[k][i] = smallest j with y_j == max y   (in downsampled samples).
 * Factor 1 is the S/N of the series itself.  FP64 moments as in amber_snr.
 * d_snr: device float [n_factors][n_dm]; d_peak_t: int32 [n_factors][n_dm] or
 * NULL.  Errors as amber_integrate_snr. */
amber_status amber_downsample_snr(const int32_t *d_dd, int32_t n_dm, int64_t dd_stride, int64_t n_out,
                                  const int32_t *factors, int32_t n_factors, float *d_snr, int32_t *d_peak_t,
                                  const amber_tiles *tiles, void *stream);

/* ---- tile search (Section 3: genetic algorithm; Section 2: brute force) ---- */

/* Genes: 0 threads_per_dm, 1 samples_per_thread, 2 dms_per_block,
 * 3 channel_unroll, 4 dms_per_thread, 5 direct_reads (the dedispersion
 * kernel's genes), 6 snr_threads, 7 + k boxcar_step[k] for k < n_widths (the
 * boxcar / S/N kernel's genes). */
#define AMBER_GENES_K1 6
#define AMBER_MAX_GENES (AMBER_GENES_K1 + 1 + AMBER_MAX_WIDTHS)
#define AMBER_MAX_GENE_VALUES 8

/* The search space: allowed values of every gene (arrays built from the
 * boundary conditions, as the paper's GA does before initialisation) and the
 * problem a configuration must be valid for. */
typedef struct {
    int32_t n_genes;                                   /* AMBER_GENES_K1 + 1 + n_widths */
    int32_t n_values[AMBER_MAX_GENES];
    int32_t values[AMBER_MAX_GENES][AMBER_MAX_GENE_VALUES];
    amber_delay_info info;                             /* validity of dedispersion tiles */
    int32_t n_widths;
    int32_t widths[AMBER_MAX_WIDTHS];                  /* validity of boxcar tiles */
    int64_t n_out;
} amber_tune_space;

typedef enum {
    AMBER_SEARCH_GA = 0,          /* genetic algorithm over all genes jointly */
    AMBER_SEARCH_EXHAUSTIVE = 1,  /* every valid joint configuration */
    AMBER_SEARCH_RANDOM = 2,      /* independent random valid configurations */
    AMBER_SEARCH_PER_KERNEL = 3   /* brute force of each kernel's genes separately */
} amber_search_kind;

typedef struct {
    int32_t search;       /* amber_search_kind */
    int32_t pop;          /* GA population N_pop (>= 2) */
    int32_t generations;  /* GA generations */
    int32_t crossover;    /* 0 uniform (coin toss per gene), 1 one-point */
    double p_cross;       /* crossover probability per kernel */
    double p_mut;         /* mutation probability per kernel */
    double pool_frac;     /* tournament pool as a fraction of N_pop */
    uint64_t seed;
    int32_t warmup;       /* device evaluator: untimed runs per configuration */
    int32_t reps;         /* device evaluator: timed runs (median) */
    double eval_timeout_s;/* slower evaluations count as failures (fitness +inf) */
    int64_t max_evals;    /* random search budget; cap for exhaustive (0 = none) */
    int32_t seed_default; /* GA: 1 = the first individual of the initial population
                             is the library's default configuration (when all
                             its values are in the gene arrays and it is valid),
                             the others random; 0 (the paper's form) = all random */
    int32_t restart_after; /* GA: 0 (the paper's form) = off; n > 0 = when the best
                              fitness has not improved for n generations, every
                              individual but the best is replaced by a fresh random
                              valid one (an addition for robustness across seeds) */
    int32_t retime_top;   /* any search: 0 (the paper's form) = off; n > 0 = after the
                             search, the n distinct configurations with the best
                             measured fitness are evaluated retime_runs more times
                             each, round robin, and the one with the lowest median is
                             returned (its median as best_time_s); these runs count
                             in n_evals.  A search otherwise ends on its luckiest
                             measurement, which need not be the fastest configuration. */
    int32_t retime_runs;  /* runs per configuration when retime_top > 0, 1 ..= 64 */
} amber_tune_params;

typedef struct {
    amber_tiles best;
    double best_time_s;   /* fitness of `best` */
    int64_t n_evals;      /* fitness evaluations performed (cache hits excluded) */
    int64_t n_failed;     /* evaluations that failed or timed out */
    int64_t space_size;   /* valid joint configurations in the space */
    double wall_s;        /* wall time of the search */
} amber_tune_result;

/* Fitness callback: measured time in seconds of the configuration; a non-zero
 * return marks a failed evaluation (fitness +inf, never selected). */
typedef int32_t (*amber_fitness_fn)(const amber_tiles *tiles, void *user, double *seconds);

/* The default search space for a problem: threads_per_dm {64 .. 1024},
 * samples_per_thread {4 .. 32}, dms_per_block {1 .. 16}, channel_unroll
 * {1 .. 32} (powers of two), dms_per_thread {1, 2}, direct_reads {0, 1},
 * snr_threads {64 .. 1024}, boxcar_step {1, 2, 4, 8} per width, or the
 * single value 8 when the fused kernel for up to 8 sliding widths of at most
 * 64 samples serves these widths (it has no step gene).  Invalid
 * combinations stay in the arrays; the searches skip them. */
amber_status amber_default_space(const amber_delay_info *info, const int32_t *widths, int32_t n_widths,
                                 int64_t n_out, amber_tune_space *space);

/* Number of valid joint configurations of a space. */
amber_status amber_space_size(const amber_tune_space *space, int64_t *count);

/* Runs the search of p->search over `space` with a caller-supplied fitness
 * (host only; no GPU needed).  log_jsonl_path, if not NULL, receives one JSON
 * line per GA generation (or per 50 evaluations for the other searches);
 * after its last generation the GA adds one line {"final_population": gene
 * values per individual, "fitness": per individual (-1 for failures)}. */
amber_status amber_search_tiles(const amber_tune_space *space, const amber_tune_params *p, amber_fitness_fn fn,
                                void *user, amber_tune_result *result, const char *log_jsonl_path);

/* amber_search_tiles with the device evaluator: fitness = GPU time (HIP
 * events, median of p->reps after p->warmup runs) of amber_dedisperse followed
 * by amber_integrate_snr on the caller's buffers, i.e. the whole hot path.
 * Synchronises `stream`.  Buffers as for those two calls; the widths and
 * geometry are the space's. */
amber_status amber_tune(const amber_tune_space *space, const int32_t *d_delays, const uint8_t *d_in,
                        int64_t in_stride, int64_t n_in, int32_t *d_dd, int64_t dd_stride, float *d_snr,
                        int32_t *d_peak_t, const amber_tune_params *p, amber_tune_result *result,
                        const char *log_jsonl_path, void *stream);

/* Default GA parameters (population 32, 40 generations, uniform crossover,
 * p_cross 0.8, p_mut 0.1, pool 20 %, 1 warm-up and 3 timed runs). */
amber_status amber_default_tune_params(amber_tune_params *p);

/* ---- tile search of the subband pipeline ------------------------------------
 * The paper's pipeline dedisperses in two steps, each a kernel with its own
 * genes (Section 2 footnote, Table 3), followed by the smoothing / S/N
 * kernels.  Genes: 0..4 step one's threads_per_dm, samples_per_thread,
 * dms_per_block, channel_unroll, dms_per_thread; 5..8 step two's
 * threads_per_dm, samples_per_thread, dms_per_block, channel_unroll (one DM
 * per wavefront); 9 snr_threads; 10 + k boxcar_step[k].  The search kinds,
 * parameters and operators are those of amber_search_tiles, with crossover
 * and mutation applied per kernel (three kernels). */
#define AMBER_SUBBAND_GENES_STEP1 5
#define AMBER_SUBBAND_GENES_STEP2 4
#define AMBER_MAX_SUBBAND_GENES (AMBER_SUBBAND_GENES_STEP1 + AMBER_SUBBAND_GENES_STEP2 + 1 + AMBER_MAX_WIDTHS)

typedef struct {
    int32_t n_genes;                                           /* 10 + n_widths */
    int32_t n_values[AMBER_MAX_SUBBAND_GENES];
    int32_t values[AMBER_MAX_SUBBAND_GENES][AMBER_MAX_GENE_VALUES];
    amber_subband_info info;                                   /* validity of both steps' tiles */
    int32_t n_widths;
    int32_t widths[AMBER_MAX_WIDTHS];                          /* validity of boxcar tiles */
    int64_t n_out;
} amber_subband_tune_space;

typedef struct {
    amber_tiles step1;    /* step one's tiles; its snr_threads and boxcar_step
                             hold the boxcar / S/N genes */
    amber_tiles step2;    /* step two's tiles */
    double best_time_s;
    int64_t n_evals;
    int64_t n_failed;
    int64_t space_size;
    double wall_s;
} amber_subband_tune_result;

/* Fitness callback of the subband search (as amber_fitness_fn). */
typedef int32_t (*amber_subband_fitness_fn)(const amber_tiles *step1, const amber_tiles *step2, void *user,
                                            double *seconds);

/* The default subband search space for a problem: powers of two (and the
 * automatic choices' DM blocks 6 and 12) within the kernels' bounds. */
amber_status amber_default_subband_space(const amber_subband_info *info, const int32_t *widths, int32_t n_widths,
                                         int64_t n_out, amber_subband_tune_space *space);

/* Number of valid joint configurations of a subband space. */
amber_status amber_subband_space_size(const amber_subband_tune_space *space, int64_t *count);

/* Runs the search of p->search over a subband space with a caller-supplied
 * fitness (host only).  Logging as amber_search_tiles. */
amber_status amber_search_subband_tiles(const amber_subband_tune_space *space, const amber_tune_params *p,
                                        amber_subband_fitness_fn fn, void *user, amber_subband_tune_result *result,
                                        const char *log_jsonl_path);

/* amber_search_subband_tiles with the device evaluator: fitness = GPU time
 * (HIP events, median of p->reps after p->warmup runs) of
 * amber_subband_dedisperse followed by amber_integrate_snr of its n_coarse *
 * n_fine trials, on the caller's buffers (as for those calls).  Synchronises
 * `stream`. */
amber_status amber_tune_subband(const amber_subband_tune_space *space, const int32_t *d_delay1,
                                const int32_t *d_delay2, const uint8_t *d_in, int64_t in_stride, int64_t n_in,
                                uint16_t *d_work, int64_t work_stride, int32_t *d_dd, int64_t dd_stride,
                                float *d_snr, int32_t *d_peak_t, const amber_tune_params *p,
                                amber_subband_tune_result *result, const char *log_jsonl_path, void *stream);

/* ---- batched beams: several independent beams in one graph launch ---------- */

/* One beam of a batch: its delay table and buffers, as for amber_dedisperse
 * and amber_integrate_snr.  Beams may differ in every size. */
typedef struct {
    const int32_t *d_delays;
    amber_delay_info info;
    const uint8_t *d_in;
    int64_t in_stride, n_in;
    int32_t *d_dd;
    int64_t dd_stride, n_out;
    float *d_snr;        /* [n_widths][n_dm] */
    int32_t *d_peak_t;   /* [n_widths][n_dm] or NULL */
} amber_beam;

typedef struct amber_batch amber_batch;  /* opaque */

/* Plans a batch: beams whose dedispersion tiles coincide share one launch
 * (each work-group finds its beam in a job table), and beams whose boxcar /
 * S/N tiles coincide share one launch; all beams use the same widths.
 * tiles: per-beam array (a tuned configuration per shape class, or one
 * configuration repeated for every beam: fewer distinct tiles mean fewer
 * launches) or NULL for amber_auto_tiles(info, n_out) of each beam, with the
 * boxcar / S/N work-group size chosen from the batch's total rows (as
 * amber_integrate_snr chooses it from n_dm).  The job tables live in device
 * memory owned by the batch (allocated here, freed by amber_batch_destroy).
 * Arguments are validated as the single-beam calls validate them. */
amber_status amber_batch_create(const amber_beam *beams, int32_t n_beams, const int32_t *widths, int32_t n_widths,
                                const amber_tiles *tiles, amber_batch **batch);

/* Enqueues the batch's launches (dedispersion groups, then boxcar / S/N
 * groups) on `stream`. */
amber_status amber_batch_run(amber_batch *batch, void *stream);

/* Captures amber_batch_run into a HIP graph (once; replaces a previous
 * capture) so that amber_batch_launch replays every launch of the batch with
 * one hipGraphLaunch.  `stream` must not be capturing already. */
amber_status amber_batch_capture(amber_batch *batch, void *stream);

/* Replays the captured graph on `stream` (AMBER_E_ARG if not captured). */
amber_status amber_batch_launch(amber_batch *batch, void *stream);

/* Number of kernel launches one run of the batch makes. */
amber_status amber_batch_launches(const amber_batch *batch, int32_t *n_dedisperse, int32_t *n_snr);

/* Frees the batch's device job tables and graph.  NULL is a no-op. */
amber_status amber_batch_destroy(amber_batch *batch);

/* ---- streaming service: continuous batching of beam chunks ------------------ */

/* Chunks of L samples of several beams arrive over time (the paper's data
 * arrives in batches of fixed length, Table 2 BATCHES).  Each beam keeps the
 * last max_delay input samples in HBM, so chunk k (k = 0, 1, ...) yields the
 * dedispersed outputs for absolute times [max(0, kL - max_delay),
 * (k+1)L - max_delay) and their S/N table, exactly what a single call on the
 * concatenated input would give for those outputs (boxcars do not cross chunk
 * edges; S/N statistics use only the chunk's outputs).  A scheduler thread
 * admits each beam's next chunk when a slot and device memory are free, fuses
 * the admitted chunks of different beams into shared launches, and runs
 * batches on several streams so their work overlaps. */
typedef struct amber_server amber_server;

typedef struct {
    int32_t max_inflight;   /* chunks on the device at once (1..4096); at most 32 launch groups run at once */
    int32_t max_batch;      /* chunks fused into one launch group (1..1024) */
    int32_t n_streams;      /* HIP streams launch groups are spread over (1..8), default priority */
    int64_t memory_budget;  /* device bytes for in-flight chunks; 0 = 90 % of the free HBM at creation */
} amber_server_config;

typedef struct {
    int32_t n_chan;
    const double *freq_mhz;   /* [n_chan], copied */
    double t_samp_s;
    int32_t n_dm;
    double dm_first, dm_step;
    int64_t chunk;            /* samples per chunk L; widths <= L */
    const amber_tiles *tiles; /* NULL = amber_auto_tiles(info, chunk) */
} amber_stream_beam;

typedef struct {
    int32_t beam;
    int32_t n_widths, n_dm;   /* shape of the S/N table */
    int64_t seq;              /* chunk index within the beam */
    uint64_t tag;             /* caller's tag from amber_server_submit */
    int64_t t_first;          /* absolute time of the chunk's first output */
    int64_t n_out;            /* outputs of the chunk (0: still inside the first max_delay samples) */
    int32_t has_snr;          /* 0 if n_out is shorter than the largest width */
    int32_t batch_size;       /* chunks in the launch group it ran in */
    double t_submit, t_start, t_done;  /* seconds on the library's steady clock */
} amber_chunk_result;

typedef struct {
    int64_t submitted, completed, batches, queued, inflight;
    int64_t memory_in_use, memory_peak, memory_budget;
    int64_t admissions_deferred_for_memory;
} amber_server_stats;

/* Outputs of chunk `seq` of a beam with chunks of L samples and largest delay
 * max_delay: absolute times [*t_first, *t_first + *n_out), where
 * t_first = max(0, seq*L - max_delay) and the end is (seq+1)*L - max_delay
 * (n_out = 0 while that end is not past t_first).  Host only. */
amber_status amber_chunk_span(int64_t seq, int64_t L, int32_t max_delay, int64_t *t_first, int64_t *n_out);

/* The admission rule the service applies, exported so that it can be checked
 * and capacity planned without a device.  Pending chunks are taken in arrival
 * order.  A chunk is passed over while its beam has a chunk on the device or
 * an earlier chunk still waiting (one beam's chunks run one at a time, in
 * order).  Admission stops at the first other chunk whose device bytes would
 * take memory_in_use past config->memory_budget (so large chunks are not
 * overtaken by small ones), once `inflight` plus the admitted
 * reach config->max_inflight, or once config->max_batch were admitted.
 * beam_busy[b] != 0 marks beams with a chunk on the device; memory_budget is
 * taken as given (0 is a zero budget here).  Writes the indices of the
 * admitted chunks, ascending, to `admitted` (room for n_pending), their count
 * to *n_admitted, and to *blocked_at the index of the chunk that did not fit
 * the budget, or -1.  Host only. */
typedef struct {
    int32_t beam;
    int64_t bytes;
} amber_pending_chunk;

amber_status amber_server_admit(const amber_pending_chunk *pending, int32_t n_pending, const uint8_t *beam_busy,
                                int32_t n_beams, int32_t inflight, int64_t memory_in_use,
                                const amber_server_config *config, int32_t *admitted, int32_t *n_admitted,
                                int32_t *blocked_at);

amber_status amber_server_create(const amber_server_config *config, amber_server **server);

/* Registers a beam: allocates its delay table and overlap buffers (refused
 * with AMBER_E_NOMEM if they do not fit the budget or the free HBM) and pinned
 * host staging for 4 queued chunks (more is pinned on demand). */
amber_status amber_server_add_beam(amber_server *server, const amber_stream_beam *beam, const int32_t *widths,
                                   int32_t n_widths, int32_t *beam_id);

/* Queues the next chunk of a beam: host uint8 [n_chan][L] with row pitch
 * `pitch` bytes, copied (into pinned staging) before the call returns.  The
 * chunks of one beam are numbered in the order their submissions return, so
 * one beam's chunks come from one thread at a time.  t_submit is taken on
 * entry, so latency includes the staging copy. */
amber_status amber_server_submit(amber_server *server, int32_t beam_id, const uint8_t *chunk, int64_t pitch,
                                 uint64_t tag);

/* Waits up to timeout_s for the oldest completed chunk; copies its S/N table
 * (float [n_widths][n_dm]) and peaks (int32, peak index relative to t_first)
 * into the caller's host buffers of `capacity` elements each (either may be
 * NULL).  AMBER_E_TIMEOUT if nothing completed in time. */
amber_status amber_server_wait(amber_server *server, double timeout_s, amber_chunk_result *result, float *snr,
                               int32_t *peak_t, int64_t capacity);

amber_status amber_server_get_stats(amber_server *server, amber_server_stats *stats);

/* Seconds on the clock used for t_submit / t_start / t_done. */
double amber_server_clock(void);

/* Completes every submitted chunk (results not waited for are dropped), stops
 * the scheduler and frees everything. */
amber_status amber_server_destroy(amber_server *server);

#ifdef __cplusplus
}
#endif

#endif /* AMBER_H */
