// Grouping of per-beam jobs into shared launches with one job-table buffer.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace amber {

void LaunchSet::add_dedisperse(const DedispPlan &p, DedispJob j)
{
    auto it = std::find_if(d_.begin(), d_.end(), [&](const DGroup &g) {
        return g.plan.tpd == p.tpd && g.plan.spt == p.spt && g.plan.dpb == p.dpb && g.plan.cu == p.cu &&
               g.plan.in_u16 == p.in_u16 && g.plan.dpt == p.dpt && g.plan.direct == p.direct;
    });
    if (it == d_.end()) {
        d_.emplace_back();
        it = d_.end() - 1;
        it->plan = p;
    }
    j.block_start = (int)it->n_blocks;
    it->n_blocks += (int64_t)j.tiles_t * j.tiles_dm * (j.groups > 1 ? j.groups : 1);
    it->plan.maxi = std::max(it->plan.maxi, p.maxi);
    it->lds = std::max(it->lds, p.lds_bytes);
    it->jobs.push_back(j);
}

void LaunchSet::add_integrate_snr(const BoxcarPlan &p, const amber_tiles &t, const int32_t *widths, int n_widths,
                                  BoxJob j)
{
    auto same = [&](const BGroup &g) {
        if (g.tiles.snr_threads != t.snr_threads || (int)g.widths.size() != n_widths) return false;
        for (int w = 0; w < n_widths; ++w)
            if (g.widths[w] != widths[w] || g.tiles.boxcar_step[w] != t.boxcar_step[w]) return false;
        return true;
    };
    auto it = std::find_if(b_.begin(), b_.end(), same);
    if (it == b_.end()) {
        b_.emplace_back();
        it = b_.end() - 1;
        it->plan = p;
        it->tiles = t;
        it->widths.assign(widths, widths + n_widths);
    }
    j.row_start = (int)it->n_rows;
    it->n_rows += j.n_dm;
    it->plan.maxw = std::max(it->plan.maxw, p.maxw);
    it->plan.lds_bytes = std::max(it->plan.lds_bytes, p.lds_bytes);
    it->jobs.push_back(j);
}

size_t LaunchSet::table_bytes() const
{
    size_t n = 0;
    for (const auto &g : d_) n += g.jobs.size() * sizeof(DedispJob);
    for (const auto &g : b_) n += g.jobs.size() * sizeof(BoxJob);
    return n;
}

void LaunchSet::write_tables(void *host) const
{
    char *p = static_cast<char *>(host);
    for (const auto &g : d_) {
        std::memcpy(p, g.jobs.data(), g.jobs.size() * sizeof(DedispJob));
        p += g.jobs.size() * sizeof(DedispJob);
    }
    for (const auto &g : b_) {
        std::memcpy(p, g.jobs.data(), g.jobs.size() * sizeof(BoxJob));
        p += g.jobs.size() * sizeof(BoxJob);
    }
}

amber_status LaunchSet::launch(const void *d_tables, hipStream_t stream) const
{
    const char *p = static_cast<const char *>(d_tables);
    for (const auto &g : d_) {
        const DedispJob *tab = reinterpret_cast<const DedispJob *>(p);
        amber_status s = g.plan.direct
                             ? launch_dedisperse_direct_jobs(g.plan, nullptr, tab, (int)g.jobs.size(), g.n_blocks, stream)
                             : launch_dedisperse_jobs(g.plan, nullptr, tab, (int)g.jobs.size(), g.n_blocks, g.lds,
                                                      stream);
        if (s != AMBER_OK) return s;
        p += g.jobs.size() * sizeof(DedispJob);
    }
    for (const auto &g : b_) {
        int all_vec = 1;
        int64_t max_n_out = 0;
        for (const auto &j : g.jobs) {
            all_vec &= j.vec_ok ? 1 : 0;
            max_n_out = j.n_out > max_n_out ? j.n_out : max_n_out;
        }
        amber_status s = launch_integrate_snr_jobs(g.plan, g.tiles, nullptr, reinterpret_cast<const BoxJob *>(p),
                                                   (int)g.jobs.size(), g.n_rows, g.widths.data(),
                                                   (int)g.widths.size(), stream, 0, all_vec, max_n_out);
        if (s != AMBER_OK) return s;
        p += g.jobs.size() * sizeof(BoxJob);
    }
    return AMBER_OK;
}

void LaunchSet::clear()
{
    d_.clear();
    b_.clear();
}

}  // namespace amber
