// Two-step subband dedispersion (Section 2 footnote; Table 2's subbanding
// parameters): the FP64 host tables and the two launches.
//
// Both steps run on the brute-force dedispersion kernel.  Step one is one
// grouped job whose groups are the subbands: each dedisperses its m channels
// at the coarse DMs and stores the sums as uint16 (m * 255 < 2^16).  Step two
// is one grouped job whose groups are the coarse DMs: its "channels" are the
// subbands' step-one rows, its DM trials the fine DMs, and its delays the
// step-two table.  Moving each coarse DM's smallest step-two shift into step
// one (amber_subband_delay_tables) lets step one compute n_out + max_delay2
// samples per row instead of n_out plus the largest step-two delay.
#include <cmath>
#include <vector>

#include "internal.h"

namespace amber {
namespace {

constexpr int kMaxSubbandChannels = 257;  // 257 * 255 < 2^16: step-one sums fit uint16

// Start of the tile search for one step.  A sweep of both steps on the
// 1536-channel beam (32 subbands; 128 x 16 and 2048 x 24 trial grids) put
// the fastest tiles at 16 samples per work-item and channel groups of 8: with
// only a few dozen channels (subbands) per work-group, several groups per
// work-group let the next group's loads overlap the current group's sums,
// which one large group cannot.  DM blocks split the trials into equal parts
// of at most 12 (step one: its wide windows) or 16 (step two).  Step two
// keeps at least 4 DM rows, even idle ones: the staging of a window is spread
// over the whole work-group, and fewer work-items would need more staging
// registers than its kernels have.
}  // namespace

amber_tiles subband_step_tiles(int n_dm, int n_chan, int in_u16)
{
    amber_tiles t = default_tiles();
    t.dms_per_thread = 1;
    t.samples_per_thread = 16;
    t.channel_unroll = n_chan >= 16 ? 8 : 4;
    const int cap = in_u16 ? 16 : 12;
    const int parts = (n_dm + cap - 1) / cap;
    t.dms_per_block = (n_dm + parts - 1) / parts;
    if (in_u16 && t.dms_per_block < 4) t.dms_per_block = 4;
    return t;
}

namespace {

amber_status plan_step(const amber_tiles *given, const amber_delay_info &info, int in_u16, DedispPlan *p)
{
    amber_tiles t;
    if (given) {
        t = *given;
        if (t.direct_reads) return fail(AMBER_E_CONFIG, "the subband steps stage their input in LDS (direct_reads 0)");
    } else {
        const amber_tiles start = subband_step_tiles(info.n_dm, info.n_chan, in_u16);
        amber_status s = auto_tiles(info, &t, in_u16, &start);
        if (s != AMBER_OK) return s;
    }
    return plan_dedisperse(t, info, p, in_u16);
}

}  // namespace
}  // namespace amber

using namespace amber;

extern "C" {

amber_status amber_subband_delay_tables(const amber_subband_geometry *g, int32_t *delay1, int32_t *delay2,
                                        amber_subband_info *info)
{
    clear_error();
    if (!g || !g->freq_mhz || !delay1 || !delay2) return fail(AMBER_E_ARG, "NULL geometry, frequencies or output");
    const int n_chan = g->n_chan, n_sub = g->n_subbands, nc = g->n_coarse, nf = g->n_fine;
    if (n_chan < 1 || n_sub < 1 || nc < 1 || nf < 1)
        return fail(AMBER_E_ARG, "n_chan=%d, n_subbands=%d, n_coarse=%d and n_fine=%d must be >= 1", n_chan, n_sub,
                    nc, nf);
    if (n_chan % n_sub != 0) return fail(AMBER_E_ARG, "n_subbands=%d does not divide n_chan=%d", n_sub, n_chan);
    const int m = n_chan / n_sub;
    if (m > kMaxSubbandChannels)
        return fail(AMBER_E_ARG, "%d channels per subband: at most %d (step-one sums are 16-bit)", m,
                    kMaxSubbandChannels);
    if (!(g->t_samp_s > 0.0) || !std::isfinite(g->t_samp_s)) return fail(AMBER_E_ARG, "t_samp must be > 0");
    const double cf = g->coarse_first, cs = g->coarse_step, ff = g->fine_first, fs = g->fine_step;
    if (!std::isfinite(cf) || !std::isfinite(cs) || !std::isfinite(ff) || !std::isfinite(fs) || !(cf >= 0.0) ||
        !(cs >= 0.0) || !(fs >= 0.0) || !(cf + ff >= 0.0))
        return fail(AMBER_E_ARG, "DM grid must be finite with coarse_first, coarse_step, fine_step and "
                    "coarse_first + fine_first >= 0");
    double f_top = 0.0;
    for (int c = 0; c < n_chan; ++c) {
        const double f = g->freq_mhz[c];
        if (!(f > 0.0) || !std::isfinite(f)) return fail(AMBER_E_ARG, "freq_mhz[%d]=%g must be > 0", c, f);
        if (f > f_top) f_top = f;
    }
    std::vector<double> f_ref(n_sub);
    for (int s = 0; s < n_sub; ++s) {
        double r = g->freq_mhz[s * m];
        for (int c = s * m; c < (s + 1) * m; ++c) r = g->freq_mhz[c] > r ? g->freq_mhz[c] : r;
        f_ref[s] = r;
    }
    // Step two first: its k = 0 shift B[j][s] moves into step one.
    std::vector<int32_t> base((size_t)nc * n_sub);
    int32_t max2 = 0, step2 = 0;
    for (int j = 0; j < nc; ++j) {
        const double dm = cf + (double)j * cs;
        for (int k = 0; k < nf; ++k) {
            const double dmk = dm + ff + (double)k * fs;
            int32_t *row = delay2 + ((size_t)j * nf + k) * n_sub;
            for (int s = 0; s < n_sub; ++s) {
                const double x = ((kDispersion * dmk) * (1.0 / (f_ref[s] * f_ref[s]) - 1.0 / (f_top * f_top))) /
                                 g->t_samp_s;
                if (!(x < 2147483647.0))
                    return fail(AMBER_E_ARG, "step-two delay of coarse DM %d, fine DM %d exceeds int32", j, k);
                const int32_t d = (int32_t)std::llround(x);
                if (k == 0) base[(size_t)j * n_sub + s] = d;
                row[s] = d - base[(size_t)j * n_sub + s];
                if (row[s] > max2) max2 = row[s];
                if (k > 0 && row[s] - row[s - (ptrdiff_t)n_sub] > step2) step2 = row[s] - row[s - (ptrdiff_t)n_sub];
            }
        }
    }
    int32_t max1 = 0, step1 = 0;
    for (int s = 0; s < n_sub; ++s) {
        for (int j = 0; j < nc; ++j) {
            const double dm = cf + (double)j * cs;
            int32_t *row = delay1 + ((size_t)s * nc + j) * m;
            for (int cl = 0; cl < m; ++cl) {
                const double f = g->freq_mhz[s * m + cl];
                const double x = ((kDispersion * dm) * (1.0 / (f * f) - 1.0 / (f_ref[s] * f_ref[s]))) / g->t_samp_s;
                const double total = x + (double)base[(size_t)j * n_sub + s];
                if (!(total < 2147483647.0))
                    return fail(AMBER_E_ARG, "step-one delay of subband %d, coarse DM %d exceeds int32", s, j);
                const int64_t d = std::llround(x) + (int64_t)base[(size_t)j * n_sub + s];
                row[cl] = (int32_t)d;
                if (row[cl] > max1) max1 = row[cl];
                if (j > 0 && row[cl] - row[cl - (ptrdiff_t)m] > step1) step1 = row[cl] - row[cl - (ptrdiff_t)m];
            }
        }
    }
    if ((int64_t)max1 + max2 > INT32_MAX) return fail(AMBER_E_ARG, "composed delays exceed int32");
    if (info) {
        info->n_chan = n_chan;
        info->n_subbands = n_sub;
        info->n_coarse = nc;
        info->n_fine = nf;
        info->max_delay1 = max1;
        info->max_step1 = step1;
        info->max_delay2 = max2;
        info->max_step2 = step2;
        info->max_delay = max1 + max2;
    }
    return AMBER_OK;
}

}  // extern "C"

namespace amber {

amber_status subband_run(const int32_t *d_delay1, const int32_t *d_delay2, const amber_subband_info *info,
                         const uint8_t *d_in, int64_t in_stride, int64_t n_in, uint16_t *d_work,
                         int64_t work_stride, int64_t work_elems, int32_t *d_dd, int64_t dd_stride, int64_t n_out,
                         const uint8_t *d_keep, const amber_tiles *tiles1, const amber_tiles *tiles2,
                         hipStream_t stream)
{
    if (!d_delay1 || !d_delay2 || !info || !d_in || !d_work || !d_dd) return fail(AMBER_E_ARG, "NULL pointer argument");
    const int n_chan = info->n_chan, n_sub = info->n_subbands, nc = info->n_coarse, nf = info->n_fine;
    if (n_chan < 1 || n_sub < 1 || nc < 1 || nf < 1 || n_chan % n_sub != 0)
        return fail(AMBER_E_ARG, "info has n_chan=%d n_subbands=%d n_coarse=%d n_fine=%d", n_chan, n_sub, nc, nf);
    const int m = n_chan / n_sub;
    if (m > kMaxSubbandChannels) return fail(AMBER_E_ARG, "%d channels per subband: at most %d", m, kMaxSubbandChannels);
    if (info->max_delay1 < 0 || info->max_step1 < 0 || info->max_delay2 < 0 || info->max_step2 < 0 ||
        (int64_t)info->max_delay != (int64_t)info->max_delay1 + info->max_delay2)
        return fail(AMBER_E_ARG, "inconsistent subband info");
    if (n_out < 0 || n_in < 0) return fail(AMBER_E_ARG, "n_out and n_in must be >= 0");
    if (n_out > (int64_t)1 << 30) return fail(AMBER_E_ARG, "n_out=%lld exceeds 2^30", (long long)n_out);
    if (in_stride < n_in || in_stride % 4 != 0 || in_stride < 32)
        return fail(AMBER_E_SHAPE, "in_stride=%lld must be >= n_in=%lld, >= 32 and a multiple of 4",
                    (long long)in_stride, (long long)n_in);
    if (((uintptr_t)d_in & 3) != 0) return fail(AMBER_E_ARG, "d_in must be 4-byte aligned");
    if (n_in < n_out + info->max_delay)
        return fail(AMBER_E_SHAPE, "n_in=%lld < n_out=%lld + max_delay=%d", (long long)n_in, (long long)n_out,
                    info->max_delay);
    const int64_t n1 = n_out + info->max_delay2;  // step-one samples per row
    if (work_stride < n1 || work_stride % 2 != 0 || work_stride < 32)
        return fail(AMBER_E_SHAPE, "work_stride=%lld must be even, >= 32 and >= n_out + max_delay2 = %lld",
                    (long long)work_stride, (long long)n1);
    if (((uintptr_t)d_work & 3) != 0) return fail(AMBER_E_ARG, "d_work must be 4-byte aligned");
    if (dd_stride < n_out) return fail(AMBER_E_SHAPE, "dd_stride=%lld < n_out=%lld", (long long)dd_stride, (long long)n_out);
    // coarse DMs whose step-one rows the work buffer holds at once
    int64_t slice = nc;
    if (work_elems >= 0) {
        slice = work_elems / ((int64_t)n_sub * work_stride);
        if (slice < 1)
            return fail(AMBER_E_SHAPE, "step one's rows of one coarse DM need %lld bytes; the work buffer holds %lld",
                        (long long)((int64_t)n_sub * work_stride * 2), (long long)(work_elems * 2));
        if (slice > nc) slice = nc;
    }

    const amber_delay_info info1{nc, m, info->max_delay1, info->max_step1};
    const amber_delay_info info2{nf, n_sub, info->max_delay2, info->max_step2};
    DedispPlan p1, p2;
    amber_status s = plan_step(tiles1, info1, 0, &p1);
    if (s != AMBER_OK) return s;
    if ((s = plan_step(tiles2, info2, 1, &p2)) != AMBER_OK) return s;
    const int64_t lds1 = p1.lds_bytes + (d_keep ? mask_lds_bytes(p1) : 0);
    if (lds1 > kMaxLdsBytes)
        return fail(AMBER_E_CONFIG, "masked step-one tile needs %lld B of LDS (limit %lld)", (long long)lds1,
                    (long long)kMaxLdsBytes);
    if ((s = check_stage_stride(p1, in_stride)) != AMBER_OK) return s;
    // step two's channels are the subband rows of the slice, jn * work_stride
    // uint16 apart: slices small enough for the staged kernel's offsets
    if (!p2.direct) {
        const int64_t most = kMaxStageSpan / ((int64_t)p2.cu * work_stride * 2);
        if (most < 1) return check_stage_stride(p2, work_stride * 2);
        if (slice > most) slice = most;
    }
    if (n_out == 0) return AMBER_OK;

    // Both steps over the coarse DMs [j0, j0 + jn): step one's sums of those
    // coarse DMs fill the work buffer as [n_sub][jn][work_stride]; step two
    // reads them back.  Each slice is computed exactly as the whole grid
    // would be (the steps of different coarse DMs never meet).
    for (int64_t j0 = 0; j0 < nc; j0 += slice) {
        const int jn = (int)(nc - j0 < slice ? nc - j0 : slice);
        // step one: one group per subband
        DedispJob j1 = make_dedisp_job(p1, d_delay1 + j0 * m, jn, m, d_in, in_stride,
                                       reinterpret_cast<int32_t *>(d_work), work_stride, n1);
        j1.in_bytes = (int64_t)n_chan * in_stride;
        j1.out_u16 = 1;
        j1.store_vec = 1;  // even stride, 4-byte aligned rows: pairs go out as dwords
        j1.keep = d_keep;
        j1.groups = n_sub;
        j1.group_blocks = j1.tiles_t * j1.tiles_dm;
        j1.group_delays = (int64_t)nc * m;
        j1.group_in = (int64_t)m * in_stride;
        j1.group_out = (int64_t)jn * work_stride * 2;
        j1.group_keep = m;
        // step two: one group per coarse DM over the subband rows
        const int64_t sub_bytes = (int64_t)jn * work_stride * 2;  // one subband's rows
        DedispJob j2 = make_dedisp_job(p2, d_delay2 + j0 * nf * n_sub, nf, n_sub,
                                       reinterpret_cast<const uint8_t *>(d_work), sub_bytes,
                                       d_dd + j0 * nf * dd_stride, dd_stride, n_out);
        j2.in_u16 = 1;
        j2.in_bytes = (int64_t)n_sub * sub_bytes;
        j2.flush_every = 65535 / (255 * m);
        j2.groups = jn;
        j2.group_blocks = j2.tiles_t * j2.tiles_dm;
        j2.group_delays = (int64_t)nf * n_sub;
        j2.group_in = work_stride * 2;
        j2.group_out = (int64_t)nf * dd_stride * 4;
        const int64_t b1 = (int64_t)j1.group_blocks * n_sub, b2 = (int64_t)j2.group_blocks * jn;
        if (b1 > 0x7fffffff || b2 > 0x7fffffff) return fail(AMBER_E_SHAPE, "subband grid too large");
        if ((s = launch_dedisperse_jobs(p1, &j1, nullptr, 1, b1, lds1, stream)) != AMBER_OK) return s;
        if ((s = launch_dedisperse_jobs(p2, &j2, nullptr, 1, b2, p2.lds_bytes, stream)) != AMBER_OK) return s;
    }
    return AMBER_OK;
}

}  // namespace amber

extern "C" {

amber_status amber_subband_dedisperse(const int32_t *d_delay1, const int32_t *d_delay2,
                                      const amber_subband_info *info, const uint8_t *d_in, int64_t in_stride,
                                      int64_t n_in, uint16_t *d_work, int64_t work_stride, int32_t *d_dd,
                                      int64_t dd_stride, int64_t n_out, const uint8_t *d_keep,
                                      const amber_tiles *tiles1, const amber_tiles *tiles2, void *stream)
{
    clear_error();
    return subband_run(d_delay1, d_delay2, info, d_in, in_stride, n_in, d_work, work_stride, -1, d_dd, dd_stride,
                       n_out, d_keep, tiles1, tiles2, (hipStream_t)stream);
}

}  // extern "C"
