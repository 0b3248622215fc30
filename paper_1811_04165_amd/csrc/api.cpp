// Host side of the C ABI: error reporting, the FP64 delay table, tile
// validation and argument checking in front of the device launchers.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "internal.h"

namespace amber {

namespace {
thread_local std::string g_error;

amber_tiles make_default_tiles()
{
    amber_tiles t{};
    // a sweep on the 1536-channel beam (2048 DMs): two DMs per wavefront with
    // channel groups of 16 beat the best one-DM tile by 11 % (1.34 vs 1.51 ms)
    t.threads_per_dm = 64;
    t.samples_per_thread = 8;
    t.dms_per_block = 16;
    t.channel_unroll = 16;
    // boxcar/S/N on the same beam: 128 work-items (two wavefronts, so more
    // rows resident per CU) stepping 8 outputs at a time took 0.103 ms against
    // 0.128 ms for 256 work-items stepping 4; per-width steps gained nothing
    t.snr_threads = 128;
    for (int k = 0; k < AMBER_MAX_WIDTHS; ++k) t.boxcar_step[k] = 8;
    t.dms_per_thread = 2;
    return t;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
}  // namespace

amber_status fail(amber_status status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return status;
}

void clear_error() { g_error.clear(); }

amber_status hip_fail(hipError_t err, const char *what)
{
    return fail(AMBER_E_DEVICE, "%s: %s", what, hipGetErrorString(err));
}

int auto_snr_threads(int64_t rows, const int32_t *widths, int n_widths)
{
    // measured on 12 208-sample rows, widths 1..64: 2048 rows 0.105 ms at 128
    // vs 0.114 ms at 64; 8192 rows 0.325 vs 0.376 ms; 49 152 rows 1.72 vs
    // 2.02 ms (64 vs 128)
    int t = rows >= 4096 ? 64 : default_tiles().snr_threads;
    int maxw = 1;
    for (int k = 0; k < n_widths; ++k) maxw = widths[k] > maxw ? widths[k] : maxw;
    const int halo = (maxw + 15) / 16 * 16;
    while (t * 16 < 2 * halo && t < kMaxThreads) t *= 2;
    return t;
}

const amber_tiles &default_tiles()
{
    static const amber_tiles t = make_default_tiles();
    return t;
}

// The default configuration, shrunk (channel_unroll first, then
// dms_per_block, then the time tile) until its dedispersion tile is valid for
// this delay table.
amber_status auto_tiles(const amber_delay_info &info, amber_tiles *out, int in_u16, const amber_tiles *start,
                        int64_t n_out)
{
    const amber_tiles &first = start ? *start : default_tiles();
    amber_tiles t = first;
    // the kernels for uint16 input take channel_unroll >= 4 and 8 or 16
    // samples per work-item
    const int min_cu = in_u16 ? 4 : 1, min_spt = in_u16 ? 8 : 4;
    DedispPlan p;
    for (;;) {
        if (plan_dedisperse(t, info, &p, in_u16) == AMBER_OK) {
            clear_error();
            break;
        }
        if (t.channel_unroll > min_cu) t.channel_unroll /= 2;
        else if (t.dms_per_block > 1) { t.dms_per_block /= 2; t.channel_unroll = first.channel_unroll; }
        else if (t.dms_per_thread > 1) {
            t.dms_per_thread = 1;
            t.dms_per_block = first.dms_per_block;
            t.channel_unroll = first.channel_unroll;
        } else if (t.samples_per_thread > min_spt) {
            t.samples_per_thread /= 2;
            t.channel_unroll = first.channel_unroll;
        } else {
            return fail(AMBER_E_CONFIG, "no dedispersion tile fits this delay table (max_step=%d)", info.max_step);
        }
    }
    if (n_out > 0 && !in_u16 && !start) fill_grid(info, n_out, &t);
    *out = t;
    return AMBER_OK;
}

int64_t dedisperse_blocks(const amber_tiles &t, int n_dm, int64_t n_out)
{
    const int64_t tile_t = (int64_t)t.threads_per_dm * t.samples_per_thread;
    const int64_t dms = (int64_t)t.dms_per_block * (t.dms_per_thread > 1 ? t.dms_per_thread : 1);
    return (n_out + tile_t - 1) / tile_t * ((n_dm + dms - 1) / dms);
}

void fill_grid(const amber_delay_info &info, int64_t n_out, amber_tiles *t)
{
    // A problem whose default tiles give fewer than 1.5 work-groups per CU
    // leaves CUs idle or unevenly loaded (the kernel is bound per CU by its
    // LDS reads).  Smaller tiles, in the order that measured best on short
    // beams and on the 256-channel workload: 4 samples per work-item with
    // channel groups of 32, then one DM per wavefront.  Fewer DMs per
    // work-group measured slower in every case (the staging is then shared
    // by fewer trials), so the walk stops there.
    constexpr int64_t kFillBlocks = 384;  // 1.5 x the 256 CUs
    DedispPlan p;
    while (dedisperse_blocks(*t, info.n_dm, n_out) < kFillBlocks) {
        amber_tiles n = *t;
        if (n.samples_per_thread > 4) {
            n.samples_per_thread /= 2;
            n.channel_unroll = 32;
        } else if (n.dms_per_thread > 1) {
            n.dms_per_thread = 1;
            n.channel_unroll = 32;
        } else {
            break;
        }
        if (plan_dedisperse(n, info, &p) != AMBER_OK) {
            n.channel_unroll = t->channel_unroll;  // the wider channel group may not fit
            if (plan_dedisperse(n, info, &p) != AMBER_OK) break;
        }
        *t = n;
    }
    clear_error();
}

amber_status plan_dedisperse(const amber_tiles &t, const amber_delay_info &info, DedispPlan *out, int in_u16)
{
    DedispPlan p{};
    p.tpd = t.threads_per_dm;
    p.spt = t.samples_per_thread;
    p.dpb = t.dms_per_block;
    p.cu = t.channel_unroll;
    p.dpt = t.dms_per_thread == 0 ? 1 : t.dms_per_thread;
    if (p.tpd < kWave || p.tpd > kMaxThreads || p.tpd % kWave != 0)
        return fail(AMBER_E_CONFIG, "threads_per_dm=%d must be a multiple of 64 in [64, 1024]", p.tpd);
    if (p.spt != 4 && p.spt != 8 && p.spt != 16 && p.spt != 32)
        return fail(AMBER_E_CONFIG, "samples_per_thread=%d must be 4, 8, 16 or 32", p.spt);
    if (p.dpb < 1 || (int64_t)p.dpb * p.tpd > kMaxThreads)
        return fail(AMBER_E_CONFIG, "dms_per_block=%d with threads_per_dm=%d exceeds 1024 work-items", p.dpb,
                    p.tpd);
    if (!is_pow2(p.cu) || p.cu > 32)
        return fail(AMBER_E_CONFIG, "channel_unroll=%d must be a power of two <= 32", p.cu);
    if (info.max_step < 0 || info.max_delay < 0)
        return fail(AMBER_E_ARG, "delay info has negative max_step or max_delay");
    if (p.dpt != 1 && p.dpt != 2)
        return fail(AMBER_E_CONFIG, "dms_per_thread=%d must be 1 or 2", p.dpt);
    if (p.dpt == 2 && p.spt > 16)
        return fail(AMBER_E_CONFIG, "dms_per_thread=2 takes samples_per_thread <= 16");
    if (in_u16 && p.dpt != 1) return fail(AMBER_E_CONFIG, "16-bit input takes dms_per_thread=1");
    if (in_u16 && ((p.spt != 8 && p.spt != 16) || p.cu < 4))
        return fail(AMBER_E_CONFIG, "16-bit input takes samples_per_thread 8 or 16 and channel_unroll >= 4 "
                    "(got %d, %d)", p.spt, p.cu);
    p.in_u16 = in_u16 ? 1 : 0;
    p.threads = p.tpd * p.dpb;
    p.tile_t = p.tpd * p.spt;
    if (t.direct_reads != 0 && t.direct_reads != 1)
        return fail(AMBER_E_CONFIG, "direct_reads=%d must be 0 or 1", t.direct_reads);
    if (t.direct_reads) {
        if (in_u16) return fail(AMBER_E_CONFIG, "direct reads take uint8 input");
        if (p.dpt != 1) return fail(AMBER_E_CONFIG, "direct reads take dms_per_thread=1");
        if ((p.spt / 4 + 1) * p.cu > 64)
            return fail(AMBER_E_CONFIG, "direct reads load (samples_per_thread/4 + 1) * channel_unroll = %d dwords "
                        "per channel group (max 64)", (p.spt / 4 + 1) * p.cu);
        p.direct = 1;
        *out = p;
        return AMBER_OK;
    }
    // Offsets a DM of the tile reads at, relative to the first DM's window
    // start (which is rounded down to a dword: 4 uint8 or 2 uint16 samples):
    // [0, omax].
    const int64_t omax = (int64_t)(p.dpb * p.dpt - 1) * info.max_step + (in_u16 ? 1 : 3);
    if (omax > (int64_t)1 << 24)
        return fail(AMBER_E_CONFIG, "delay steps too large for one tile (max_step=%d)", info.max_step);
    // a DM reads dwords up to (o >> 1) + tile_t / 2 - 1 of a copy; the copy
    // with the one-sample shift reads one byte past its window
    int64_t win = (int64_t)p.tile_t + 2 * (omax >> 1) + 2;
    win = (win + 15) / 16 * 16;
    const int64_t lds = 2 * (int64_t)p.cu * win * 2;  // two 16-bit copies per channel
    if (lds > kMaxLdsBytes)
        return fail(AMBER_E_CONFIG, "dedispersion tile needs %lld B of LDS (limit %lld): reduce "
                    "channel_unroll, dms_per_block or the time tile", (long long)lds, (long long)kMaxLdsBytes);
    const int64_t items = p.cu * (win / 16);
    p.maxi = (int)((items + p.threads - 1) / p.threads);
    // prefetch registers beside the accumulators
    const int maxi_cap = in_u16 ? 2 : (p.spt >= 32 ? 2 : (p.spt >= 16 ? (p.dpt == 2 ? 2 : 3) : 4));
    if (p.maxi > maxi_cap)
        return fail(AMBER_E_CONFIG, "staging needs %d items per work-item (max %d): reduce channel_unroll or "
                    "enlarge the work-group", p.maxi, maxi_cap);
    p.win = (int)win;
    p.omax = (int)omax;
    p.lds_bytes = lds;
    *out = p;
    return AMBER_OK;
}

amber_status plan_boxcar(const amber_tiles &t, const int32_t *widths, int32_t n_widths, int64_t n_out,
                         BoxcarPlan *out, int max_width)
{
    BoxcarPlan p{};
    if (!widths || n_widths < 1 || n_widths > AMBER_MAX_WIDTHS)
        return fail(AMBER_E_ARG, "n_widths=%d must be in [1, %d]", n_widths, AMBER_MAX_WIDTHS);
    int maxw = 0;
    for (int k = 0; k < n_widths; ++k) {
        if (widths[k] < 1 || widths[k] > max_width || widths[k] > n_out)
            return fail(AMBER_E_ARG, "widths[%d]=%d must be in [1, min(n_out=%lld, %d)]", k, widths[k],
                        (long long)n_out, max_width);
        if (widths[k] > maxw) maxw = widths[k];
        int s = t.boxcar_step[k];
        if (s != 1 && s != 2 && s != 4 && s != 8)
            return fail(AMBER_E_CONFIG, "boxcar_step[%d]=%d must be 1, 2, 4 or 8", k, s);
    }
    if (!is_pow2(t.snr_threads) || t.snr_threads < 64 || t.snr_threads > 1024)
        return fail(AMBER_E_CONFIG, "snr_threads=%d must be a power of two in [64, 1024]", t.snr_threads);
    p.threads = t.snr_threads;
    p.chunk = p.threads * 16;
    p.maxw = maxw;
    // chunks overlap by the largest width rounded up to 16; they must be at
    // least twice that long
    if (p.chunk < 2 * ((maxw + 15) / 16 * 16))
        return fail(AMBER_E_CONFIG, "snr_threads=%d gives chunks of %d samples, too short for width %d", p.threads,
                    p.chunk, maxw);
    // prefix elements: the chunk, plus the reads past it of a work-item's
    // last, partial step; four pad dwords per 64
    const int64_t n = (int64_t)p.chunk + maxw + 16;
    p.lds_bytes = (n + 16) * 4;
    *out = p;
    return AMBER_OK;
}

}  // namespace amber

using namespace amber;

namespace {

constexpr int kMaxFactor = 4096;  // largest decimation factor (the paper's largest is 3200)

// The caller's tiles, or the defaults with snr_threads raised until a chunk
// (16 samples per work-item) holds twice the largest factor and one decimated
// bin per work-item and step (measured fastest on the 1536-channel beam: the
// decimated series are short, so larger steps leave work-items idle).
amber_status downsample_tiles(const amber_tiles *tiles, const int32_t *factors, int32_t n_factors, amber_tiles *out)
{
    if (!factors || n_factors < 1 || n_factors > AMBER_MAX_WIDTHS)
        return fail(AMBER_E_ARG, "n_factors=%d must be in [1, %d]", n_factors, AMBER_MAX_WIDTHS);
    if (tiles) {
        *out = *tiles;
        return AMBER_OK;
    }
    *out = default_tiles();
    int maxf = 1;
    for (int k = 0; k < n_factors; ++k) maxf = factors[k] > maxf ? factors[k] : maxf;
    const int64_t halo = (maxf + 15) / 16 * 16;
    while ((int64_t)out->snr_threads * 16 < 2 * halo && out->snr_threads < kMaxThreads) out->snr_threads *= 2;
    for (int k = 0; k < AMBER_MAX_WIDTHS; ++k) out->boxcar_step[k] = 1;
    return AMBER_OK;
}

}  // namespace

extern "C" {

const char *amber_last_error(void) { return g_error.c_str(); }

const char *amber_version(void) { return "amber-mi355x 0.1 (gfx950)"; }

amber_status amber_default_tiles(amber_tiles *tiles)
{
    clear_error();
    if (!tiles) return fail(AMBER_E_ARG, "tiles is NULL");
    *tiles = default_tiles();
    return AMBER_OK;
}

amber_status amber_auto_tiles(const amber_delay_info *info, int64_t n_out, amber_tiles *tiles)
{
    clear_error();
    if (!tiles || !info) return fail(AMBER_E_ARG, "tiles or info is NULL");
    return auto_tiles(*info, tiles, 0, nullptr, n_out);
}

amber_status amber_validate_tiles(const amber_tiles *tiles, const amber_delay_info *info, int32_t n_widths)
{
    clear_error();
    if (!tiles || !info) return fail(AMBER_E_ARG, "tiles or info is NULL");
    DedispPlan dp;
    amber_status s = plan_dedisperse(*tiles, *info, &dp);
    if (s != AMBER_OK) return s;
    int32_t w[AMBER_MAX_WIDTHS];
    if (n_widths < 1 || n_widths > AMBER_MAX_WIDTHS)
        return fail(AMBER_E_ARG, "n_widths=%d must be in [1, %d]", n_widths, AMBER_MAX_WIDTHS);
    for (int k = 0; k < n_widths; ++k) w[k] = 1;
    BoxcarPlan bp;
    return plan_boxcar(*tiles, w, n_widths, 1, &bp);
}

amber_status amber_delay_table(const amber_geometry *g, int32_t *delays, amber_delay_info *info)
{
    clear_error();
    if (!g || !delays || !g->freq_mhz) return fail(AMBER_E_ARG, "NULL geometry, frequencies or output");
    if (g->n_chan < 1 || g->n_dm < 1) return fail(AMBER_E_ARG, "n_chan=%d and n_dm=%d must be >= 1", g->n_chan, g->n_dm);
    if (!(g->t_samp_s > 0.0) || !std::isfinite(g->t_samp_s)) return fail(AMBER_E_ARG, "t_samp must be > 0");
    if (!(g->dm_first >= 0.0) || !(g->dm_step >= 0.0) || !std::isfinite(g->dm_first) || !std::isfinite(g->dm_step))
        return fail(AMBER_E_ARG, "dm_first and dm_step must be finite and >= 0");
    double f_top = 0.0;
    for (int c = 0; c < g->n_chan; ++c) {
        double f = g->freq_mhz[c];
        if (!(f > 0.0) || !std::isfinite(f)) return fail(AMBER_E_ARG, "freq_mhz[%d]=%g must be > 0", c, f);
        if (f > f_top) f_top = f;
    }
    const double inv_top2 = 1.0 / (f_top * f_top);
    const int n_chan = g->n_chan;
    int32_t max_delay = 0, max_step = 0;
    for (int i = 0; i < g->n_dm; ++i) {
        const double kdm = kDispersion * (g->dm_first + (double)i * g->dm_step);
        int32_t *row = delays + (size_t)i * n_chan;
        for (int c = 0; c < n_chan; ++c) {
            const double f = g->freq_mhz[c];
            const double x = (kdm * (1.0 / (f * f) - inv_top2)) / g->t_samp_s;
            if (!(x < 2147483647.0)) return fail(AMBER_E_ARG, "delay of DM trial %d, channel %d exceeds int32", i, c);
            const int32_t d = (int32_t)std::llround(x);
            row[c] = d;
            if (d > max_delay) max_delay = d;
            if (i > 0) {
                const int32_t step = d - row[c - (ptrdiff_t)n_chan];
                if (step > max_step) max_step = step;
            }
        }
    }
    if (info) {
        info->n_dm = g->n_dm;
        info->n_chan = g->n_chan;
        info->max_delay = max_delay;
        info->max_step = max_step;
    }
    return AMBER_OK;
}

namespace {

amber_status dedisperse_common(const int32_t *d_delays, const amber_delay_info *info, const uint8_t *d_in,
                               int64_t in_stride, int64_t n_in, int32_t *d_dd, int64_t dd_stride, int64_t n_out,
                               const uint8_t *d_keep, const amber_tiles *tiles, void *stream)
{
    if (!d_delays || !info || !d_in || (!d_dd && n_out > 0)) return fail(AMBER_E_ARG, "NULL pointer argument");
    if (info->n_dm < 1 || info->n_chan < 1) return fail(AMBER_E_ARG, "info has n_dm=%d n_chan=%d", info->n_dm, info->n_chan);
    if (n_out < 0 || n_in < 0) return fail(AMBER_E_ARG, "n_out and n_in must be >= 0");
    if (n_out > (int64_t)1 << 30) return fail(AMBER_E_ARG, "n_out=%lld exceeds 2^30", (long long)n_out);
    if (in_stride < n_in || in_stride % 4 != 0 || in_stride < 32)
        return fail(AMBER_E_SHAPE, "in_stride=%lld must be >= n_in=%lld, >= 32 and a multiple of 4",
                    (long long)in_stride, (long long)n_in);
    if (((uintptr_t)d_in & 3) != 0) return fail(AMBER_E_ARG, "d_in must be 4-byte aligned");
    if (n_in < n_out + info->max_delay)
        return fail(AMBER_E_SHAPE, "n_in=%lld < n_out=%lld + max_delay=%d", (long long)n_in, (long long)n_out,
                    info->max_delay);
    if (dd_stride < n_out) return fail(AMBER_E_SHAPE, "dd_stride=%lld < n_out=%lld", (long long)dd_stride, (long long)n_out);
    if ((int64_t)info->n_chan * 255 >= ((int64_t)1 << 31))
        return fail(AMBER_E_ARG, "n_chan=%d can overflow int32 sums", info->n_chan);
    amber_tiles chosen;
    amber_status s = tiles ? AMBER_OK : auto_tiles(*info, &chosen, 0, nullptr, n_out);
    if (s != AMBER_OK) return s;
    DedispPlan plan;
    s = plan_dedisperse(tiles ? *tiles : chosen, *info, &plan);
    if (s != AMBER_OK) return s;
    if ((s = check_stage_stride(plan, in_stride)) != AMBER_OK) return s;
    if (n_out == 0) return AMBER_OK;
    if (plan.direct) {
        DedispJob j = make_dedisp_job(plan, d_delays, info->n_dm, info->n_chan, d_in, in_stride, d_dd, dd_stride,
                                      n_out);
        j.keep = d_keep;
        return launch_dedisperse_direct_jobs(plan, &j, nullptr, 1, (int64_t)j.tiles_t * j.tiles_dm,
                                             (hipStream_t)stream);
    }
    return launch_dedisperse(plan, d_delays, info->n_dm, info->n_chan, d_in, in_stride, n_in, d_dd, dd_stride, n_out,
                             (hipStream_t)stream, d_keep);
}

}  // namespace

amber_status amber_dedisperse(const int32_t *d_delays, const amber_delay_info *info, const uint8_t *d_in,
                              int64_t in_stride, int64_t n_in, int32_t *d_dd, int64_t dd_stride, int64_t n_out,
                              const amber_tiles *tiles, void *stream)
{
    clear_error();
    return dedisperse_common(d_delays, info, d_in, in_stride, n_in, d_dd, dd_stride, n_out, nullptr, tiles, stream);
}

amber_status amber_dedisperse_masked(const int32_t *d_delays, const amber_delay_info *info, const uint8_t *d_in,
                                     int64_t in_stride, int64_t n_in, int32_t *d_dd, int64_t dd_stride,
                                     int64_t n_out, const uint8_t *d_keep, const amber_tiles *tiles, void *stream)
{
    clear_error();
    if (!d_keep) return fail(AMBER_E_ARG, "d_keep is NULL");
    return dedisperse_common(d_delays, info, d_in, in_stride, n_in, d_dd, dd_stride, n_out, d_keep, tiles, stream);
}

static amber_status check_rows(const void *p, int32_t n_dm, int64_t stride, int64_t n_out, const char *name)
{
    if (!p) return fail(AMBER_E_ARG, "%s is NULL", name);
    if (n_dm < 1) return fail(AMBER_E_ARG, "n_dm=%d must be >= 1", n_dm);
    if (n_out < 1 || n_out > (int64_t)1 << 30) return fail(AMBER_E_ARG, "n_out=%lld must be in [1, 2^30]", (long long)n_out);
    if (stride < n_out) return fail(AMBER_E_SHAPE, "%s stride %lld < n_out=%lld", name, (long long)stride, (long long)n_out);
    if (((uintptr_t)p & 3) != 0) return fail(AMBER_E_ARG, "%s must be 4-byte aligned", name);
    return AMBER_OK;
}

amber_status amber_integrate(const int32_t *d_dd, int32_t n_dm, int64_t dd_stride, int64_t n_out, const int32_t *widths,
                             int32_t n_widths, int32_t *d_box, int64_t box_stride, const amber_tiles *tiles,
                             void *stream)
{
    clear_error();
    amber_status s = check_rows(d_dd, n_dm, dd_stride, n_out, "d_dd");
    if (s != AMBER_OK) return s;
    if ((s = check_rows(d_box, n_dm, box_stride, n_out, "d_box")) != AMBER_OK) return s;
    const amber_tiles &t = tiles ? *tiles : default_tiles();
    BoxcarPlan plan;
    if ((s = plan_boxcar(t, widths, n_widths, n_out, &plan)) != AMBER_OK) return s;
    return launch_integrate(plan, t, d_dd, n_dm, dd_stride, n_out, widths, n_widths, d_box, box_stride,
                            (hipStream_t)stream);
}

amber_status amber_snr(const int32_t *d_box, int32_t n_dm, int64_t box_stride, int64_t n_out, const int32_t *widths,
                       int32_t n_widths, float *d_snr, int32_t *d_peak_t, const amber_tiles *tiles, void *stream)
{
    clear_error();
    amber_status s = check_rows(d_box, n_dm, box_stride, n_out, "d_box");
    if (s != AMBER_OK) return s;
    if (!d_snr) return fail(AMBER_E_ARG, "d_snr is NULL");
    const amber_tiles &t = tiles ? *tiles : default_tiles();
    BoxcarPlan plan;
    if ((s = plan_boxcar(t, widths, n_widths, n_out, &plan)) != AMBER_OK) return s;
    return launch_snr(plan, t, d_box, n_dm, box_stride, n_out, widths, n_widths, d_snr, d_peak_t,
                      (hipStream_t)stream);
}

amber_status amber_integrate_snr(const int32_t *d_dd, int32_t n_dm, int64_t dd_stride, int64_t n_out,
                                 const int32_t *widths, int32_t n_widths, float *d_snr, int32_t *d_peak_t,
                                 const amber_tiles *tiles, void *stream)
{
    clear_error();
    amber_status s = check_rows(d_dd, n_dm, dd_stride, n_out, "d_dd");
    if (s != AMBER_OK) return s;
    if (!d_snr) return fail(AMBER_E_ARG, "d_snr is NULL");
    amber_tiles t = tiles ? *tiles : default_tiles();
    if (!tiles && widths && n_widths >= 1 && n_widths <= AMBER_MAX_WIDTHS)
        t.snr_threads = auto_snr_threads(n_dm, widths, n_widths);
    BoxcarPlan plan;
    if ((s = plan_boxcar(t, widths, n_widths, n_out, &plan)) != AMBER_OK) return s;
    return launch_integrate_snr(plan, t, d_dd, n_dm, dd_stride, n_out, widths, n_widths, d_snr, d_peak_t,
                                (hipStream_t)stream);
}

amber_status amber_downsample(const int32_t *d_dd, int32_t n_dm, int64_t dd_stride, int64_t n_out,
                              const int32_t *factors, int32_t n_factors, int32_t *d_y, int64_t y_stride,
                              const amber_tiles *tiles, void *stream)
{
    clear_error();
    amber_status s = check_rows(d_dd, n_dm, dd_stride, n_out, "d_dd");
    if (s != AMBER_OK) return s;
    amber_tiles t;
    if ((s = downsample_tiles(tiles, factors, n_factors, &t)) != AMBER_OK) return s;
    if (!d_y || ((uintptr_t)d_y & 3) != 0) return fail(AMBER_E_ARG, "d_y is NULL or misaligned");
    // the plan checks every factor against [1, min(n_out, 4096)] before the
    // output stride is sized from them
    BoxcarPlan plan;
    if ((s = plan_boxcar(t, factors, n_factors, n_out, &plan, kMaxFactor)) != AMBER_OK) return s;
    for (int k = 0; k < n_factors; ++k)
        if (y_stride < n_out / factors[k])
            return fail(AMBER_E_SHAPE, "y_stride=%lld < n_out / factors[%d]", (long long)y_stride, k);
    return launch_integrate(plan, t, d_dd, n_dm, dd_stride, n_out, factors, n_factors, d_y, y_stride,
                            (hipStream_t)stream, 1);
}

amber_status amber_downsample_snr(const int32_t *d_dd, int32_t n_dm, int64_t dd_stride, int64_t n_out,
                                  const int32_t *factors, int32_t n_factors, float *d_snr, int32_t *d_peak,
                                  const amber_tiles *tiles, void *stream)
{
    clear_error();
    amber_status s = check_rows(d_dd, n_dm, dd_stride, n_out, "d_dd");
    if (s != AMBER_OK) return s;
    if (!d_snr) return fail(AMBER_E_ARG, "d_snr is NULL");
    amber_tiles t;
    if ((s = downsample_tiles(tiles, factors, n_factors, &t)) != AMBER_OK) return s;
    BoxcarPlan plan;
    if ((s = plan_boxcar(t, factors, n_factors, n_out, &plan, kMaxFactor)) != AMBER_OK) return s;
    return launch_integrate_snr(plan, t, d_dd, n_dm, dd_stride, n_out, factors, n_factors, d_snr, d_peak,
                                (hipStream_t)stream, 1);
}

}  // extern "C"
