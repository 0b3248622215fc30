// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <vector>

#include "amber.h"

namespace amber {

// Records a formatted message for amber_last_error() and returns `status`.
amber_status fail(amber_status status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

// Maps a HIP error to AMBER_E_DEVICE with the runtime's message.
amber_status hip_fail(hipError_t err, const char *what);

#define AMBER_HIP(call, what)                          \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return ::amber::hip_fail(e_, what); \
    } while (0)

// Cold-plasma dispersion constant, s MHz^2 / (pc cm^-3).
constexpr double kDispersion = 4.148808e3;

constexpr int kWave = 64;
constexpr int kMaxThreads = 1024;
constexpr int64_t kMaxLdsBytes = 160 * 1024;

// Dedispersion tile geometry derived from the tile genes and the table summary.
struct DedispPlan {
    int tpd, spt, dpb, cu;
    int dpt;            // DMs per wavefront; a work-group covers dpb * dpt DMs
    int threads;        // tpd * dpb
    int tile_t;         // output samples per tile: tpd * spt
    int win;            // LDS window length in samples per channel (multiple of 16)
    int maxi;           // staging items per work-item (prefetched in registers)
    int omax;           // largest sample offset a DM may read at inside the window
    int in_u16;         // input samples are uint16 (subband step two)
    int direct;         // reads the input from global memory, no LDS staging
                        // (win, omax and maxi are then unused)
    int64_t lds_bytes;  // dynamic LDS per work-group
};

amber_status plan_dedisperse(const amber_tiles &t, const amber_delay_info &info, DedispPlan *out, int in_u16 = 0);
// The staged kernel addresses a channel group's input with 32-bit offsets
// from its first row: channel_unroll * in_stride (bytes) must stay below
// kMaxStageSpan.  AMBER_E_SHAPE otherwise (the direct-read kernel has no
// such limit).
constexpr int64_t kMaxStageSpan = 0xffffffffll - 64;
amber_status check_stage_stride(const DedispPlan &p, int64_t in_stride);
// LDS a launch with keep flags adds: the zeroed region zapped channels read
// (64 lanes x samples_per_thread / 2 dwords).
inline int64_t mask_lds_bytes(const DedispPlan &p) { return (int64_t)kWave * (p.spt / 2) * 4; }
// The start of the automatic tile choice of one subband step (n_dm trials over
// n_chan channels or subbands; in_u16 for step two).
amber_tiles subband_step_tiles(int n_dm, int n_chan, int in_u16);

// The first valid tiles of a shrinking sequence that starts at `start`
// (default: the library's defaults); with the defaults and n_out > 0 (uint8
// input), then made smaller by fill_grid until the grid fills the chip.
amber_status auto_tiles(const amber_delay_info &info, amber_tiles *out, int in_u16 = 0,
                        const amber_tiles *start = nullptr, int64_t n_out = 0);
// Work-groups of a dedispersion launch with tiles t.
int64_t dedisperse_blocks(const amber_tiles &t, int n_dm, int64_t n_out);
// Shrinks valid tiles (uint8 input: samples_per_thread down to 4, then one DM
// per wavefront) until the launch has at least 384 work-groups (1.5 per CU)
// or neither step is left; keeps them valid.
void fill_grid(const amber_delay_info &info, int64_t n_out, amber_tiles *t);

// Boxcar / S/N geometry.
struct BoxcarPlan {
    int threads;   // work-items per group
    int chunk;     // outputs per LDS chunk (threads * 16)
    int maxw;      // largest width
    int64_t lds_bytes;
};

// max_width: 1024 for sliding widths, 4096 for decimation factors
amber_status plan_boxcar(const amber_tiles &t, const int32_t *widths, int32_t n_widths, int64_t n_out,
                         BoxcarPlan *out, int max_width = 1024);

const amber_tiles &default_tiles();
// Work-group size of the fused boxcar / S/N kernel when the caller passes no
// tiles: 64 from 4096 rows up (one row per work-group: enough rows keep the
// CUs busy with single-wave groups), else the default 128; raised while a
// chunk of 16 samples per work-item is shorter than twice the largest width.
int auto_snr_threads(int64_t rows, const int32_t *widths, int n_widths);

// One beam's dedispersion work: the arguments of a launch, or one entry of a
// batched launch's job table (tiles of job j occupy work-groups
// [block_start, block_start + tiles_t * tiles_dm)).
struct DedispJob {
    const int32_t *delays;
    const uint8_t *in;
    int32_t *dd;
    int64_t in_stride, in_bytes, dd_stride, n_out;
    int n_dm, n_chan, win, omax, tiles_t, tiles_dm, store_vec, block_start;
    const uint8_t *keep;  // per-channel keep flags (0 = zapped), or NULL: every channel
    // in_u16: input samples are uint16 (else uint8); out_u16: sums are stored
    // as uint16 (the caller guarantees they fit).  flush_every: channels summed
    // into the packed 16-bit partial sums before they are widened (256 for
    // uint8 input; floor(65535 / largest input value) for uint16).
    int in_u16, out_u16, flush_every;
    // groups > 1: the job is `groups` independent problems of the same shape
    // (the subbands of subband step one, the coarse DMs of step two), each
    // group_blocks work-groups long in the grid; group g uses delays, input,
    // output and keep flags advanced by g times the strides below, and in_bytes
    // counts from group 0's input
    int groups, group_blocks;
    int64_t group_delays, group_in, group_out, group_keep;  // int32 elements, bytes, bytes, channels
};

// One beam's boxcar / S/N work (rows of job j occupy work-groups
// [row_start, row_start + n_dm)).
struct BoxJob {
    const int32_t *dd;
    int64_t dd_stride, n_out;
    float *snr;
    int32_t *peak;
    int n_dm, vec_ok, row_start;
};

DedispJob make_dedisp_job(const DedispPlan &p, const int32_t *d_delays, int n_dm, int n_chan, const uint8_t *d_in,
                          int64_t in_stride, int32_t *d_dd, int64_t dd_stride, int64_t n_out);
amber_status launch_dedisperse_jobs(const DedispPlan &p, const DedispJob *single, const DedispJob *d_jobs,
                                    int n_jobs, int64_t n_blocks, int64_t lds_bytes, hipStream_t stream);
BoxJob make_box_job(const int32_t *d_dd, int n_dm, int64_t dd_stride, int64_t n_out, float *d_snr, int32_t *d_peak);
// decimate != 0: the widths are decimation factors (see amber_downsample_snr).
// all_vec: with a job table, 1 when every job's rows allow 16-byte loads
// (BoxJob::vec_ok), else 0; max_n_out: with a job table, the longest row.
// Both are ignored with a single job.
amber_status launch_integrate_snr_jobs(const BoxcarPlan &p, const amber_tiles &t, const BoxJob *single,
                                       const BoxJob *d_jobs, int n_jobs, int64_t n_rows, const int32_t *widths,
                                       int n_widths, hipStream_t stream, int decimate = 0, int all_vec = 0,
                                       int64_t max_n_out = 0);
// Sliding widths and rows that the span kernel serves (at most 8 widths,
// each <= 64; rows of fewer than 2^29 samples).
bool span_snr_applies(const int32_t *widths, int n_widths, int decimate, int64_t max_n_out);

// Jobs of several beams grouped into as few launches as their launch shapes
// allow.  Dedispersion jobs with the same tile genes share a launch (the
// group takes the largest LDS window and staging depth of its members; both
// stay within the kernel's limits because members share samples_per_thread);
// boxcar/S/N jobs share a launch when their S/N tiles and widths agree.  The
// job tables of all groups are laid out in one buffer: write_tables() fills
// its host image, launch() takes its device copy.
class LaunchSet {
public:
    void add_dedisperse(const DedispPlan &p, DedispJob j);
    void add_integrate_snr(const BoxcarPlan &p, const amber_tiles &t, const int32_t *widths, int n_widths, BoxJob j);
    size_t table_bytes() const;
    void write_tables(void *host) const;
    amber_status launch(const void *d_tables, hipStream_t stream) const;
    int n_dedisperse() const { return (int)d_.size(); }
    int n_snr() const { return (int)b_.size(); }
    bool empty() const { return d_.empty() && b_.empty(); }
    void clear();

private:
    struct DGroup {
        DedispPlan plan;
        int64_t lds = 0, n_blocks = 0;
        std::vector<DedispJob> jobs;
    };
    struct BGroup {
        BoxcarPlan plan;
        amber_tiles tiles;
        std::vector<int32_t> widths;
        int64_t n_rows = 0;
        std::vector<BoxJob> jobs;
    };
    std::vector<DGroup> d_;
    std::vector<BGroup> b_;
};

// Two-step subband dedispersion with step one's sums in d_work
// ([n_subbands][slice][work_stride] uint16): the arguments of
// amber_subband_dedisperse, validated here.  work_elems < 0: the buffer holds
// every coarse DM (one pair of launches); otherwise the coarse DMs run in
// slices of work_elems / (n_subbands * work_stride), two launches per slice,
// and a slice of one coarse DM that does not fit is AMBER_E_SHAPE.
amber_status subband_run(const int32_t *d_delay1, const int32_t *d_delay2, const amber_subband_info *info,
                         const uint8_t *d_in, int64_t in_stride, int64_t n_in, uint16_t *d_work,
                         int64_t work_stride, int64_t work_elems, int32_t *d_dd, int64_t dd_stride, int64_t n_out,
                         const uint8_t *d_keep, const amber_tiles *tiles1, const amber_tiles *tiles2,
                         hipStream_t stream);

// Launchers (device translation units).
// Direct-read dedispersion (plans with direct set): one job or a job table,
// uint8 input, int32 sums, one problem per job (groups 1).
amber_status launch_dedisperse_direct_jobs(const DedispPlan &p, const DedispJob *single, const DedispJob *d_jobs,
                                           int n_jobs, int64_t n_blocks, hipStream_t stream);
amber_status launch_dedisperse(const DedispPlan &p, const int32_t *d_delays, int n_dm, int n_chan,
                               const uint8_t *d_in, int64_t in_stride, int64_t n_in, int32_t *d_dd,
                               int64_t dd_stride, int64_t n_out, hipStream_t stream, const uint8_t *d_keep = nullptr);

amber_status launch_integrate(const BoxcarPlan &p, const amber_tiles &t, const int32_t *d_dd, int n_dm,
                              int64_t dd_stride, int64_t n_out, const int32_t *widths, int n_widths,
                              int32_t *d_box, int64_t box_stride, hipStream_t stream, int decimate = 0);

amber_status launch_snr(const BoxcarPlan &p, const amber_tiles &t, const int32_t *d_box, int n_dm,
                        int64_t box_stride, int64_t n_out, const int32_t *widths, int n_widths,
                        float *d_snr, int32_t *d_peak, hipStream_t stream);

// Window of a streamed chunk: row c of d_cur = d_prev[c][L, L + D) followed
// by d_stage[c][0, L) (rows of d_cur / d_prev are `stride` bytes apart, d_stage
// is contiguous).
amber_status launch_assemble(uint8_t *d_cur, const uint8_t *d_prev, const uint8_t *d_stage, int n_chan,
                             int64_t stride, int64_t L, int64_t D, hipStream_t stream);

amber_status launch_integrate_snr(const BoxcarPlan &p, const amber_tiles &t, const int32_t *d_dd, int n_dm,
                                  int64_t dd_stride, int64_t n_out, const int32_t *widths, int n_widths,
                                  float *d_snr, int32_t *d_peak, hipStream_t stream, int decimate = 0);

}  // namespace amber
