// Streaming service.  Chunks of several beams arrive over time (the paper's
// pipeline consumes its input in batches of fixed length, Table 2).  A
// scheduler thread admits chunks as launch slots and device memory free up,
// fuses the admitted chunks of different beams into shared launches
// (continuous batching: whatever is ready joins the next launch group, nothing
// waits for a group to fill) and spreads the groups over several streams so
// that one group's copies overlap another's kernels.
//
// Each beam keeps its last max_delay input samples in HBM.  Two input windows
// of max_delay + L columns are used alternately: chunk k is copied (one
// contiguous host-to-device copy) into the device staging area of its block,
// and one assembly pass writes window k % 2 as columns [L, L + max_delay) of
// the other window followed by the staged chunk, so column j holds absolute
// time k*L - max_delay + j and a plain dedispersion of L outputs from column
// 0 covers the chunk.  The outputs of negative absolute time (the first
// max_delay samples of the stream) are computed from zeros and dropped.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

namespace amber {
namespace {

constexpr int kMaxStreams = 8;
constexpr int kMaxInflight = 4096;
constexpr int kMaxBatch = 1024;
constexpr int kMaxSlots = 32;       // launch groups on the device at once
constexpr int kScanLimit = 4096;    // pending chunks looked at per admission
constexpr int kStagingPerBeam = 4;  // pinned chunk buffers allocated with a beam

double clock_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

void span_of(int64_t seq, int64_t L, int64_t D, int64_t *t_first, int64_t *n_out)
{
    const int64_t first = std::max<int64_t>(0, seq * L - D);
    *t_first = first;
    *n_out = std::max<int64_t>(0, (seq + 1) * L - D - first);
}

amber_status check_config(const amber_server_config &c)
{
    if (c.max_inflight < 1 || c.max_inflight > kMaxInflight)
        return fail(AMBER_E_ARG, "max_inflight=%d must be in [1, %d]", c.max_inflight, kMaxInflight);
    if (c.max_batch < 1 || c.max_batch > kMaxBatch)
        return fail(AMBER_E_ARG, "max_batch=%d must be in [1, %d]", c.max_batch, kMaxBatch);
    if (c.n_streams < 1 || c.n_streams > kMaxStreams)
        return fail(AMBER_E_ARG, "n_streams=%d must be in [1, %d]", c.n_streams, kMaxStreams);
    if (c.memory_budget < 0) return fail(AMBER_E_ARG, "memory_budget must be >= 0");
    return AMBER_OK;
}

// The admission rule (documented with amber_server_admit).  `taken` starts as
// the busy flags and is updated in place.
int admit_rule(const amber_pending_chunk *pending, int n_pending, std::vector<uint8_t> &taken, int inflight,
               int64_t in_use, const amber_server_config &c, int32_t *out, int32_t *blocked_at)
{
    int n = 0;
    *blocked_at = -1;
    for (int i = 0; i < n_pending; ++i) {
        if (inflight + n >= c.max_inflight || n >= c.max_batch) break;
        const amber_pending_chunk &p = pending[i];
        if (taken[p.beam]) continue;
        taken[p.beam] = 1;  // later chunks of this beam wait for this one
        if (in_use + p.bytes > c.memory_budget) {
            *blocked_at = i;
            break;
        }
        in_use += p.bytes;
        out[n++] = i;
    }
    return n;
}

// Pinned host buffers kept in free lists by size, so that steady-state
// chunks allocate nothing.
class PinnedPool {
public:
    void *get(size_t bytes)
    {
        {
            std::lock_guard<std::mutex> g(m_);
            auto it = free_.find(bytes);
            if (it != free_.end() && !it->second.empty()) {
                void *p = it->second.back();
                it->second.pop_back();
                return p;
            }
        }
        void *p = nullptr;
        return hipHostMalloc(&p, bytes, hipHostMallocDefault) == hipSuccess ? p : nullptr;
    }
    void put(void *p, size_t bytes)
    {
        if (!p) return;
        std::lock_guard<std::mutex> g(m_);
        free_[bytes].push_back(p);
    }
    void release()
    {
        std::lock_guard<std::mutex> g(m_);
        for (auto &kv : free_)
            for (void *p : kv.second) (void)hipHostFree(p);
        free_.clear();
    }

private:
    std::mutex m_;
    std::map<size_t, std::vector<void *>> free_;
};

struct SBeam {
    amber_delay_info info{};
    int32_t *d_delays = nullptr;
    uint8_t *d_in[2] = {nullptr, nullptr};  // [n_chan][stride] each
    int64_t stride = 0, L = 0, D = 0;
    std::vector<int32_t> widths;
    int maxw = 0;
    amber_tiles tiles{};
    DedispPlan dp{};
    BoxcarPlan bp{};
    int64_t dd_stride = 0;        // int32 per dedispersed row of a chunk block
    int64_t res_off = 0;          // byte offset of the S/N table in a chunk block
    int64_t res_bytes = 0;        // S/N table + peak table
    int64_t stage_off = 0;        // byte offset of the staged chunk in a chunk block
    int64_t block_bytes = 0;      // device bytes one chunk holds while it runs
    int64_t persistent_bytes = 0; // delay table + both input buffers
    int64_t submitted = 0;
    bool busy = false;
    size_t host_bytes() const { return (size_t)info.n_chan * (size_t)L; }
};

struct Request {
    int beam = 0;
    SBeam *b = nullptr;
    int64_t seq = 0;
    uint64_t tag = 0;
    double t_submit = 0;
    uint8_t *host = nullptr;  // pinned [n_chan][L]
    bool deferred = false;    // counted once when memory held it back
};

struct Active {
    Request rq;
    void *block = nullptr;  // device: dd [n_dm][dd_stride], S/N and peak [n_widths][n_dm], chunk [n_chan][L]
    void *h_res = nullptr;  // pinned copy of S/N and peak
    int64_t t_first = 0, n_out = 0;
    int has_snr = 0;
};

struct Slot {
    void *d_tables = nullptr, *h_tables = nullptr;
    hipEvent_t done = nullptr;
};

struct Flight {
    std::vector<Active> chunks;
    int slot = -1;
    double t_start = 0;
};

struct Done {
    amber_chunk_result r{};
    std::vector<float> snr;
    std::vector<int32_t> peak;
};

}  // namespace
}  // namespace amber

struct amber_server {
    amber_server_config cfg{};
    int device = 0;
    std::vector<hipStream_t> streams;
    hipStream_t setup = nullptr;
    int next_stream = 0;
    size_t table_cap = 0;
    std::vector<amber::Slot> slots;
    std::vector<int> free_slots;
    std::vector<std::unique_ptr<amber::SBeam>> beams;
    int64_t max_block = 0;
    std::deque<amber::Request> queue;
    std::deque<amber::Flight> flights;
    std::deque<amber::Done> done;
    amber::PinnedPool pinned;
    std::map<int64_t, std::vector<void *>> idle_blocks;  // device chunk blocks by size
    int64_t idle_bytes = 0;
    amber_server_stats st{};
    std::mutex m;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    amber_status error = AMBER_OK;
    std::string error_msg;
    std::thread worker;
};

using namespace amber;

namespace {

void set_error(amber_server *s, amber_status st, const std::string &msg)
{
    if (s->error == AMBER_OK) {
        s->error = st;
        s->error_msg = msg;
    }
    s->cv_done.notify_all();
}

// A device block of `bytes`: an idle one of that size, or a new allocation
// (idle blocks of other sizes are freed first when keeping them would take
// the device memory past the budget).  Lock held.
void *take_block(amber_server *s, int64_t bytes)
{
    auto it = s->idle_blocks.find(bytes);
    if (it != s->idle_blocks.end() && !it->second.empty()) {
        void *p = it->second.back();
        it->second.pop_back();
        s->idle_bytes -= bytes;
        return p;
    }
    if (s->st.memory_in_use + s->idle_bytes + bytes > s->cfg.memory_budget) {
        for (auto &kv : s->idle_blocks)
            for (void *p : kv.second) (void)hipFree(p);
        s->idle_blocks.clear();
        s->idle_bytes = 0;
    }
    void *p = nullptr;
    return hipMalloc(&p, (size_t)bytes) == hipSuccess ? p : nullptr;
}

void release_active(amber_server *s, Active &a)
{
    SBeam &b = *a.rq.b;
    s->pinned.put(a.rq.host, b.host_bytes());
    s->pinned.put(a.h_res, (size_t)b.res_bytes);
    if (a.block) {
        s->idle_blocks[b.block_bytes].push_back(a.block);
        s->idle_bytes += b.block_bytes;
    }
    s->st.memory_in_use -= b.block_bytes;
    s->st.inflight -= 1;
    b.busy = false;
}

// Enqueues one launch group on `stream`: the chunk copies, the overlap
// copies, the fused dedispersion and boxcar/S/N launches, the result copies
// and the group's completion event.  Runs without the lock; touches only the
// group's own chunks and their (busy) beams.
amber_status enqueue(amber_server *s, Flight &f, hipStream_t stream)
{
    LaunchSet set;
    for (Active &a : f.chunks) {
        SBeam &b = *a.rq.b;
        const int cur = (int)(a.rq.seq & 1);
        const int n_chan = b.info.n_chan;
        uint8_t *stage = static_cast<uint8_t *>(a.block) + b.stage_off;
        AMBER_HIP(hipMemcpyAsync(stage, a.rq.host, b.host_bytes(), hipMemcpyHostToDevice, stream), "chunk copy");
        // window k % 2 = tail of the other window + this chunk (the other
        // window is still all zeros for chunk 0)
        amber_status as = launch_assemble(b.d_in[cur], b.d_in[cur ^ 1], stage, n_chan, b.stride, b.L, b.D, stream);
        if (as != AMBER_OK) return as;
        if (!a.has_snr) continue;
        int32_t *dd = static_cast<int32_t *>(a.block);
        float *snr = reinterpret_cast<float *>(static_cast<char *>(a.block) + b.res_off);
        int32_t *peak = reinterpret_cast<int32_t *>(snr + b.widths.size() * (size_t)b.info.n_dm);
        const int64_t j0 = a.t_first - (a.rq.seq * b.L - b.D);  // first column of a non-negative time
        set.add_dedisperse(b.dp, make_dedisp_job(b.dp, b.d_delays, b.info.n_dm, n_chan, b.d_in[cur], b.stride, dd,
                                                 b.dd_stride, b.L));
        set.add_integrate_snr(b.bp, b.tiles, b.widths.data(), (int)b.widths.size(),
                              make_box_job(dd + j0, b.info.n_dm, b.dd_stride, a.n_out, snr, peak));
    }
    Slot &sl = s->slots[f.slot];
    if (!set.empty()) {
        const size_t bytes = set.table_bytes();
        if (bytes > s->table_cap) return fail(AMBER_E_DEVICE, "job tables of %zu bytes exceed the slot", bytes);
        set.write_tables(sl.h_tables);
        AMBER_HIP(hipMemcpyAsync(sl.d_tables, sl.h_tables, bytes, hipMemcpyHostToDevice, stream), "job tables");
        amber_status st = set.launch(sl.d_tables, stream);
        if (st != AMBER_OK) return st;
        for (Active &a : f.chunks)
            if (a.has_snr)
                AMBER_HIP(hipMemcpyAsync(a.h_res, static_cast<char *>(a.block) + a.rq.b->res_off,
                                         (size_t)a.rq.b->res_bytes, hipMemcpyDeviceToHost, stream),
                          "result copy");
    }
    AMBER_HIP(hipEventRecord(sl.done, stream), "hipEventRecord");
    return AMBER_OK;
}

// Moves finished launch groups to the result queue.  Lock held.
bool retire(amber_server *s)
{
    bool any = false;
    for (auto it = s->flights.begin(); it != s->flights.end();) {
        const hipError_t e = hipEventQuery(s->slots[it->slot].done);
        if (e == hipErrorNotReady) {
            ++it;
            continue;
        }
        if (e != hipSuccess) {
            set_error(s, AMBER_E_DEVICE, std::string("hipEventQuery: ") + hipGetErrorString(e));
            return any;
        }
        const double t = clock_s();
        for (Active &a : it->chunks) {
            SBeam &b = *a.rq.b;
            Done d;
            d.r.beam = a.rq.beam;
            d.r.n_widths = (int32_t)b.widths.size();
            d.r.n_dm = b.info.n_dm;
            d.r.seq = a.rq.seq;
            d.r.tag = a.rq.tag;
            d.r.t_first = a.t_first;
            d.r.n_out = a.n_out;
            d.r.has_snr = a.has_snr;
            d.r.batch_size = (int32_t)it->chunks.size();
            d.r.t_submit = a.rq.t_submit;
            d.r.t_start = it->t_start;
            d.r.t_done = t;
            if (a.has_snr) {
                const size_t n = b.widths.size() * (size_t)b.info.n_dm;
                const float *hs = static_cast<const float *>(a.h_res);
                d.snr.assign(hs, hs + n);
                const int32_t *hp = reinterpret_cast<const int32_t *>(hs + n);
                d.peak.assign(hp, hp + n);
            }
            release_active(s, a);
            s->done.push_back(std::move(d));
            s->st.completed += 1;
        }
        s->free_slots.push_back(it->slot);
        it = s->flights.erase(it);
        any = true;
    }
    if (any) s->cv_done.notify_all();
    return any;
}

// Admits the chunks the rule allows into one launch group and enqueues it.
bool admit_and_launch(amber_server *s, std::unique_lock<std::mutex> &lk)
{
    if (s->queue.empty() || s->free_slots.empty()) return false;
    const int n = (int)std::min<size_t>(s->queue.size(), kScanLimit);
    std::vector<amber_pending_chunk> pend((size_t)n);
    for (int i = 0; i < n; ++i) pend[i] = {s->queue[i].beam, s->queue[i].b->block_bytes};
    std::vector<uint8_t> taken(s->beams.size());
    for (size_t k = 0; k < s->beams.size(); ++k) taken[k] = s->beams[k]->busy ? 1 : 0;
    std::vector<int32_t> idx((size_t)n);
    int32_t blocked = -1;
    const int k = admit_rule(pend.data(), n, taken, (int)s->st.inflight, s->st.memory_in_use, s->cfg, idx.data(),
                             &blocked);
    if (blocked >= 0 && !s->queue[blocked].deferred) {
        s->queue[blocked].deferred = true;
        s->st.admissions_deferred_for_memory += 1;
    }
    if (k == 0) {
        if (s->flights.empty() && blocked >= 0)
            set_error(s, AMBER_E_NOMEM, "a chunk does not fit the memory budget even with nothing running");
        return false;
    }
    Flight f;
    f.slot = s->free_slots.back();
    s->free_slots.pop_back();
    std::vector<Request> reqs;
    for (int i = k - 1; i >= 0; --i) {
        reqs.push_back(s->queue[idx[i]]);
        s->queue.erase(s->queue.begin() + idx[i]);
    }
    std::reverse(reqs.begin(), reqs.end());
    bool ok = true;
    for (Request &r : reqs) {
        SBeam &b = *r.b;
        Active a;
        a.rq = r;
        span_of(r.seq, b.L, b.D, &a.t_first, &a.n_out);
        a.has_snr = a.n_out >= b.maxw ? 1 : 0;
        b.busy = true;
        s->st.memory_in_use += b.block_bytes;
        s->st.inflight += 1;
        a.block = take_block(s, b.block_bytes);
        if (a.has_snr) a.h_res = s->pinned.get((size_t)b.res_bytes);
        if (!a.block || (a.has_snr && !a.h_res)) ok = false;
        f.chunks.push_back(a);
    }
    s->st.memory_peak = std::max(s->st.memory_peak, s->st.memory_in_use);
    if (!ok) {
        for (Active &a : f.chunks) release_active(s, a);
        s->free_slots.push_back(f.slot);
        set_error(s, AMBER_E_NOMEM, "device or pinned allocation for a launch group failed");
        return false;
    }
    f.t_start = clock_s();
    hipStream_t stream = s->streams[(size_t)(s->next_stream++ % (int)s->streams.size())];
    lk.unlock();
    const amber_status st = enqueue(s, f, stream);
    const std::string msg = st == AMBER_OK ? std::string() : std::string(amber_last_error());
    if (st != AMBER_OK) (void)hipStreamSynchronize(stream);
    lk.lock();
    if (st != AMBER_OK) {
        for (Active &a : f.chunks) release_active(s, a);
        s->free_slots.push_back(f.slot);
        set_error(s, st, msg);
        return false;
    }
    s->st.batches += 1;
    s->flights.push_back(std::move(f));
    return true;
}

void worker_main(amber_server *s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->m);
    for (;;) {
        bool progressed = retire(s);
        if (s->error == AMBER_OK) progressed = admit_and_launch(s, lk) || progressed;
        if (s->stop && (s->error != AMBER_OK || (s->flights.empty() && s->queue.empty()))) break;
        if (progressed) continue;
        if (s->flights.empty())
            s->cv_work.wait(lk);
        else
            s->cv_work.wait_for(lk, std::chrono::microseconds(20));
    }
}

void free_beam(SBeam &b)
{
    if (b.d_delays) (void)hipFree(b.d_delays);
    for (int k = 0; k < 2; ++k)
        if (b.d_in[k]) (void)hipFree(b.d_in[k]);
    b.d_delays = nullptr;
    b.d_in[0] = b.d_in[1] = nullptr;
}

void destroy_resources(amber_server *s)
{
    for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
    if (s->setup) (void)hipStreamSynchronize(s->setup);
    for (Flight &f : s->flights)
        for (Active &a : f.chunks) release_active(s, a);
    s->flights.clear();
    for (Request &r : s->queue) s->pinned.put(r.host, r.b->host_bytes());
    s->queue.clear();
    for (auto &kv : s->idle_blocks)
        for (void *p : kv.second) (void)hipFree(p);
    s->idle_blocks.clear();
    for (auto &b : s->beams) free_beam(*b);
    for (Slot &sl : s->slots) {
        if (sl.d_tables) (void)hipFree(sl.d_tables);
        if (sl.h_tables) (void)hipHostFree(sl.h_tables);
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    s->slots.clear();
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    s->streams.clear();
    if (s->setup) (void)hipStreamDestroy(s->setup);
    s->setup = nullptr;
    s->pinned.release();
}

}  // namespace

extern "C" {

double amber_server_clock(void) { return clock_s(); }

amber_status amber_chunk_span(int64_t seq, int64_t L, int32_t max_delay, int64_t *t_first, int64_t *n_out)
{
    clear_error();
    if (!t_first || !n_out) return fail(AMBER_E_ARG, "NULL output");
    if (seq < 0 || L < 1 || max_delay < 0 || L > ((int64_t)1 << 30) || seq > ((int64_t)1 << 32))
        return fail(AMBER_E_ARG, "need seq in [0, 2^32], L in [1, 2^30] and max_delay >= 0");
    span_of(seq, L, max_delay, t_first, n_out);
    return AMBER_OK;
}

amber_status amber_server_admit(const amber_pending_chunk *pending, int32_t n_pending, const uint8_t *beam_busy,
                                int32_t n_beams, int32_t inflight, int64_t memory_in_use,
                                const amber_server_config *config, int32_t *admitted, int32_t *n_admitted,
                                int32_t *blocked_at)
{
    clear_error();
    if (!config || !n_admitted || !blocked_at || n_pending < 0 || n_beams < 0 || inflight < 0 || memory_in_use < 0)
        return fail(AMBER_E_ARG, "bad arguments");
    if (n_pending > 0 && (!pending || !admitted)) return fail(AMBER_E_ARG, "NULL pending or admitted");
    if (n_beams > 0 && !beam_busy) return fail(AMBER_E_ARG, "NULL beam_busy");
    amber_status s = check_config(*config);
    if (s != AMBER_OK) return s;
    for (int i = 0; i < n_pending; ++i)
        if (pending[i].beam < 0 || pending[i].beam >= n_beams || pending[i].bytes < 0)
            return fail(AMBER_E_ARG, "pending[%d] has beam %d (of %d) and %lld bytes", i, pending[i].beam, n_beams,
                        (long long)pending[i].bytes);
    std::vector<uint8_t> taken(beam_busy, beam_busy + n_beams);
    for (auto &t : taken) t = t ? 1 : 0;
    *n_admitted = admit_rule(pending, n_pending, taken, inflight, memory_in_use, *config, admitted, blocked_at);
    return AMBER_OK;
}

amber_status amber_server_create(const amber_server_config *config, amber_server **out)
{
    clear_error();
    if (!config || !out) return fail(AMBER_E_ARG, "NULL config or output handle");
    *out = nullptr;
    amber_status st = check_config(*config);
    if (st != AMBER_OK) return st;
    auto s = std::make_unique<amber_server>();
    s->cfg = *config;
    AMBER_HIP(hipGetDevice(&s->device), "hipGetDevice");
    if (s->cfg.memory_budget == 0) {
        size_t fr = 0, tot = 0;
        AMBER_HIP(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
        s->cfg.memory_budget = (int64_t)((double)fr * 0.9);
    }
    s->st.memory_budget = s->cfg.memory_budget;
    const int n_slots = std::min(s->cfg.max_inflight, kMaxSlots);
    const int per_slot = std::min(s->cfg.max_batch, s->cfg.max_inflight);
    s->table_cap = (size_t)per_slot * (sizeof(DedispJob) + sizeof(BoxJob));
    hipError_t e = hipSuccess;
    for (int k = 0; k < s->cfg.n_streams && e == hipSuccess; ++k) {
        hipStream_t h = nullptr;
        e = hipStreamCreateWithFlags(&h, hipStreamNonBlocking);
        if (e == hipSuccess) s->streams.push_back(h);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->setup, hipStreamNonBlocking);
    for (int k = 0; k < n_slots && e == hipSuccess; ++k) {
        s->slots.emplace_back();
        Slot &sl = s->slots.back();
        e = hipMalloc(&sl.d_tables, s->table_cap);
        if (e == hipSuccess) e = hipHostMalloc(&sl.h_tables, s->table_cap, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        s->free_slots.push_back(k);
    }
    if (e != hipSuccess) {
        destroy_resources(s.get());
        return hip_fail(e, "server set-up");
    }
    amber_server *raw = s.release();
    raw->worker = std::thread(worker_main, raw);
    *out = raw;
    return AMBER_OK;
}

amber_status amber_server_add_beam(amber_server *s, const amber_stream_beam *bm, const int32_t *widths,
                                   int32_t n_widths, int32_t *beam_id)
{
    clear_error();
    if (!s || !bm || !widths || !beam_id) return fail(AMBER_E_ARG, "NULL argument");
    if (bm->n_chan < 1 || bm->n_dm < 1 || (int64_t)bm->n_chan * bm->n_dm > ((int64_t)1 << 31))
        return fail(AMBER_E_ARG, "n_chan=%d, n_dm=%d out of range", bm->n_chan, bm->n_dm);
    if (bm->chunk < 1 || bm->chunk > ((int64_t)1 << 30)) return fail(AMBER_E_ARG, "chunk must be in [1, 2^30]");
    if (n_widths < 1 || n_widths > AMBER_MAX_WIDTHS) return fail(AMBER_E_ARG, "bad n_widths %d", n_widths);
    if ((int64_t)bm->n_chan * 255 >= ((int64_t)1 << 31)) return fail(AMBER_E_ARG, "too many channels");
    auto b = std::make_unique<SBeam>();
    std::vector<int32_t> delays((size_t)bm->n_chan * (size_t)bm->n_dm);
    const amber_geometry g{bm->n_chan, bm->freq_mhz, bm->t_samp_s, bm->n_dm, bm->dm_first, bm->dm_step};
    amber_status st = amber_delay_table(&g, delays.data(), &b->info);
    if (st != AMBER_OK) return st;
    clear_error();
    if (bm->tiles)
        b->tiles = *bm->tiles;
    else if ((st = auto_tiles(b->info, &b->tiles, 0, nullptr, bm->chunk)) != AMBER_OK)
        return st;
    if ((st = plan_dedisperse(b->tiles, b->info, &b->dp)) != AMBER_OK) return st;
    if ((st = plan_boxcar(b->tiles, widths, n_widths, bm->chunk, &b->bp)) != AMBER_OK) return st;
    b->widths.assign(widths, widths + n_widths);
    b->maxw = *std::max_element(b->widths.begin(), b->widths.end());
    b->L = bm->chunk;
    b->D = b->info.max_delay;
    b->stride = round_up(b->D + b->L, 128);
    if ((st = check_stage_stride(b->dp, b->stride)) != AMBER_OK) return st;
    b->dd_stride = round_up(b->L, 64);
    b->res_off = round_up((int64_t)b->info.n_dm * b->dd_stride * 4, 256);
    b->res_bytes = (int64_t)n_widths * b->info.n_dm * 8;
    b->stage_off = round_up(b->res_off + b->res_bytes, 256);
    b->block_bytes = round_up(b->stage_off + (int64_t)b->info.n_chan * b->L, 256);
    const int64_t table_bytes = round_up((int64_t)delays.size() * 4, 256);
    const int64_t in_bytes = (int64_t)b->info.n_chan * b->stride;
    b->persistent_bytes = table_bytes + 2 * in_bytes;
    {
        std::lock_guard<std::mutex> lk(s->m);
        if (s->error != AMBER_OK) return fail(s->error, "server failed: %s", s->error_msg.c_str());
        const int64_t need = s->st.memory_in_use + b->persistent_bytes + std::max(s->max_block, b->block_bytes);
        if (need > s->cfg.memory_budget)
            return fail(AMBER_E_NOMEM, "beam needs %lld bytes resident and %lld per chunk; budget %lld, in use %lld",
                        (long long)b->persistent_bytes, (long long)b->block_bytes, (long long)s->cfg.memory_budget,
                        (long long)s->st.memory_in_use);
        // reserve now so that concurrent registrations see it
        s->st.memory_in_use += b->persistent_bytes;
        s->max_block = std::max(s->max_block, b->block_bytes);
    }
    hipError_t e = hipMalloc(&b->d_delays, (size_t)table_bytes);
    if (e == hipSuccess) e = hipMalloc(&b->d_in[0], (size_t)in_bytes);
    if (e == hipSuccess) e = hipMalloc(&b->d_in[1], (size_t)in_bytes);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_delays, delays.data(), delays.size() * 4, hipMemcpyHostToDevice, s->setup);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_in[0], 0, (size_t)in_bytes, s->setup);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_in[1], 0, (size_t)in_bytes, s->setup);
    if (e == hipSuccess) e = hipStreamSynchronize(s->setup);
    std::lock_guard<std::mutex> lk(s->m);
    if (e != hipSuccess) {
        free_beam(*b);
        s->st.memory_in_use -= b->persistent_bytes;
        return e == hipErrorOutOfMemory ? fail(AMBER_E_NOMEM, "beam buffers do not fit the free HBM")
                                        : hip_fail(e, "beam set-up");
    }
    s->st.memory_peak = std::max(s->st.memory_peak, s->st.memory_in_use);
    // pinned staging for a few queued chunks of this beam, so that submissions
    // do not pin memory while a backlog is short (the pool grows past this)
    for (int k = 0; k < kStagingPerBeam; ++k) {
        void *h = nullptr;
        if (hipHostMalloc(&h, b->host_bytes(), hipHostMallocDefault) != hipSuccess) break;
        s->pinned.put(h, b->host_bytes());
    }
    *beam_id = (int32_t)s->beams.size();
    s->beams.push_back(std::move(b));
    return AMBER_OK;
}

amber_status amber_server_submit(amber_server *s, int32_t beam_id, const uint8_t *chunk, int64_t pitch, uint64_t tag)
{
    clear_error();
    const double t0 = clock_s();
    if (!s || !chunk) return fail(AMBER_E_ARG, "NULL server or chunk");
    SBeam *b = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->m);
        if (s->error != AMBER_OK) return fail(s->error, "server failed: %s", s->error_msg.c_str());
        if (s->stop) return fail(AMBER_E_ARG, "server is shutting down");
        if (beam_id < 0 || beam_id >= (int32_t)s->beams.size()) return fail(AMBER_E_ARG, "no beam %d", beam_id);
        b = s->beams[(size_t)beam_id].get();
    }
    if (pitch < b->L) return fail(AMBER_E_SHAPE, "pitch %lld < chunk length %lld", (long long)pitch, (long long)b->L);
    uint8_t *host = static_cast<uint8_t *>(s->pinned.get(b->host_bytes()));
    if (!host) return fail(AMBER_E_NOMEM, "pinned staging of %zu bytes failed", b->host_bytes());
    if (pitch == b->L) {
        std::memcpy(host, chunk, b->host_bytes());
    } else {
        for (int c = 0; c < b->info.n_chan; ++c)
            std::memcpy(host + (size_t)c * b->L, chunk + (size_t)c * pitch, (size_t)b->L);
    }
    {
        std::lock_guard<std::mutex> lk(s->m);
        Request r;
        r.beam = beam_id;
        r.b = b;
        r.seq = b->submitted++;
        r.tag = tag;
        r.t_submit = t0;
        r.host = host;
        s->queue.push_back(r);
        s->st.submitted += 1;
    }
    s->cv_work.notify_one();
    return AMBER_OK;
}

amber_status amber_server_wait(amber_server *s, double timeout_s, amber_chunk_result *result, float *snr,
                               int32_t *peak_t, int64_t capacity)
{
    clear_error();
    if (!s || !result) return fail(AMBER_E_ARG, "NULL server or result");
    std::unique_lock<std::mutex> lk(s->m);
    auto ready = [s] { return !s->done.empty() || s->error != AMBER_OK; };
    if (!(timeout_s > 0.0))
        ;
    else if (timeout_s >= 1e6)
        s->cv_done.wait(lk, ready);
    else
        s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
    if (s->done.empty()) {
        if (s->error != AMBER_OK) return fail(s->error, "server failed: %s", s->error_msg.c_str());
        return fail(AMBER_E_TIMEOUT, "no chunk completed within %g s", timeout_s);
    }
    Done &d = s->done.front();
    const int64_t n = (int64_t)d.r.n_widths * d.r.n_dm;
    if ((snr || peak_t) && capacity < n)
        return fail(AMBER_E_SHAPE, "result needs %lld elements, capacity is %lld", (long long)n, (long long)capacity);
    *result = d.r;
    if (d.r.has_snr) {
        if (snr) std::memcpy(snr, d.snr.data(), (size_t)n * sizeof(float));
        if (peak_t) std::memcpy(peak_t, d.peak.data(), (size_t)n * sizeof(int32_t));
    }
    s->done.pop_front();
    return AMBER_OK;
}

amber_status amber_server_get_stats(amber_server *s, amber_server_stats *stats)
{
    clear_error();
    if (!s || !stats) return fail(AMBER_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->m);
    *stats = s->st;
    stats->queued = (int64_t)s->queue.size();
    stats->memory_budget = s->cfg.memory_budget;
    return AMBER_OK;
}

amber_status amber_server_destroy(amber_server *s)
{
    clear_error();
    if (!s) return AMBER_OK;
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    destroy_resources(s);
    delete s;
    return AMBER_OK;
}

}  // extern "C"
