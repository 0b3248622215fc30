// Batched beams: independent beams of uneven sizes planned into as few
// launches as their tiles allow, replayable as one HIP graph.
#include <vector>

#include "internal.h"

namespace amber {
namespace {

amber_status check_beam(const amber_beam &b, int k, const int32_t *widths, int n_widths)
{
    const amber_delay_info &in = b.info;
    if (!b.d_delays || !b.d_in || !b.d_dd || !b.d_snr) return fail(AMBER_E_ARG, "beam %d: NULL pointer", k);
    if (in.n_dm < 1 || in.n_chan < 1 || in.max_delay < 0 || in.max_step < 0)
        return fail(AMBER_E_ARG, "beam %d: bad delay info", k);
    if (b.n_out < 1 || b.n_out > (int64_t)1 << 30) return fail(AMBER_E_ARG, "beam %d: n_out out of range", k);
    if (b.in_stride < b.n_in || b.in_stride % 4 != 0 || b.in_stride < 32 || ((uintptr_t)b.d_in & 3) != 0)
        return fail(AMBER_E_SHAPE, "beam %d: in_stride must be >= n_in, >= 32 and a multiple of 4", k);
    if (b.n_in < b.n_out + in.max_delay) return fail(AMBER_E_SHAPE, "beam %d: n_in < n_out + max_delay", k);
    if (b.dd_stride < b.n_out || ((uintptr_t)b.d_dd & 3) != 0) return fail(AMBER_E_SHAPE, "beam %d: bad dd", k);
    if ((int64_t)in.n_chan * 255 >= ((int64_t)1 << 31)) return fail(AMBER_E_ARG, "beam %d: too many channels", k);
    for (int w = 0; w < n_widths; ++w)
        if (widths[w] > b.n_out) return fail(AMBER_E_ARG, "beam %d: width %d exceeds n_out", k, widths[w]);
    return AMBER_OK;
}

}  // namespace
}  // namespace amber

struct amber_batch {
    amber::LaunchSet set;
    void *d_mem = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

using namespace amber;

namespace {

amber_status run_batch(amber_batch *b, hipStream_t stream)
{
    return b->set.launch(b->d_mem, stream);
}

void release(amber_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_mem) (void)hipFree(b->d_mem);
    b->exec = nullptr;
    b->graph = nullptr;
    b->d_mem = nullptr;
}

}  // namespace

extern "C" {

amber_status amber_batch_create(const amber_beam *beams, int32_t n_beams, const int32_t *widths, int32_t n_widths,
                                const amber_tiles *tiles, amber_batch **out)
{
    clear_error();
    if (!beams || !out || n_beams < 1) return fail(AMBER_E_ARG, "need beams, n_beams >= 1 and an output handle");
    *out = nullptr;
    if (!widths || n_widths < 1 || n_widths > AMBER_MAX_WIDTHS) return fail(AMBER_E_ARG, "bad widths");
    for (int k = 0; k < n_beams; ++k) {
        amber_status s = check_beam(beams[k], k, widths, n_widths);
        if (s != AMBER_OK) return s;
    }
    auto b = new amber_batch();
    // automatic tiles: the boxcar / S/N rows of every beam share launches, so
    // their work-group size follows the batch's total row count
    int64_t total_rows = 0;
    for (int k = 0; k < n_beams; ++k) total_rows += beams[k].info.n_dm;
    const int snr_threads = auto_snr_threads(total_rows, widths, n_widths);
    // group beams by identical launch shapes
    for (int k = 0; k < n_beams; ++k) {
        const amber_beam &bm = beams[k];
        amber_tiles t;
        amber_status s = tiles ? AMBER_OK : auto_tiles(bm.info, &t, 0, nullptr, bm.n_out);
        if (tiles)
            t = tiles[k];
        else
            t.snr_threads = snr_threads;
        DedispPlan dp;
        BoxcarPlan bp;
        if (s == AMBER_OK) s = plan_dedisperse(t, bm.info, &dp);
        if (s == AMBER_OK) s = check_stage_stride(dp, bm.in_stride);
        if (s == AMBER_OK) s = plan_boxcar(t, widths, n_widths, bm.n_out, &bp);
        if (s != AMBER_OK) {
            delete b;
            return s;
        }
        b->set.add_dedisperse(dp, make_dedisp_job(dp, bm.d_delays, bm.info.n_dm, bm.info.n_chan, bm.d_in,
                                                  bm.in_stride, bm.d_dd, bm.dd_stride, bm.n_out));
        b->set.add_integrate_snr(bp, t, widths, n_widths,
                                 make_box_job(bm.d_dd, bm.info.n_dm, bm.dd_stride, bm.n_out, bm.d_snr, bm.d_peak_t));
    }
    // one device allocation for every job table
    const size_t bytes = b->set.table_bytes();
    std::vector<char> host(bytes);
    b->set.write_tables(host.data());
    if (hipMalloc(&b->d_mem, bytes) != hipSuccess) {
        delete b;
        return fail(AMBER_E_NOMEM, "cannot allocate %zu bytes of job tables", bytes);
    }
    if (hipMemcpy(b->d_mem, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        release(b);
        delete b;
        return fail(AMBER_E_DEVICE, "copying job tables failed");
    }
    *out = b;
    return AMBER_OK;
}

amber_status amber_batch_run(amber_batch *b, void *stream)
{
    clear_error();
    if (!b) return fail(AMBER_E_ARG, "batch is NULL");
    return run_batch(b, (hipStream_t)stream);
}

amber_status amber_batch_capture(amber_batch *b, void *stream)
{
    clear_error();
    if (!b) return fail(AMBER_E_ARG, "batch is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (!s) return fail(AMBER_E_ARG, "graph capture needs a non-default stream");
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    AMBER_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    amber_status st = run_batch(b, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st != AMBER_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    b->graph = g;
    AMBER_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
    return AMBER_OK;
}

amber_status amber_batch_launch(amber_batch *b, void *stream)
{
    clear_error();
    if (!b || !b->exec) return fail(AMBER_E_ARG, "batch not captured");
    AMBER_HIP(hipGraphLaunch(b->exec, (hipStream_t)stream), "hipGraphLaunch");
    return AMBER_OK;
}

amber_status amber_batch_launches(const amber_batch *b, int32_t *n_dedisperse, int32_t *n_snr)
{
    clear_error();
    if (!b) return fail(AMBER_E_ARG, "batch is NULL");
    if (n_dedisperse) *n_dedisperse = b->set.n_dedisperse();
    if (n_snr) *n_snr = b->set.n_snr();
    return AMBER_OK;
}

amber_status amber_batch_destroy(amber_batch *b)
{
    clear_error();
    if (!b) return AMBER_OK;
    release(b);
    delete b;
    return AMBER_OK;
}

}  // extern "C"
