// Tile search: the genetic algorithm of Section 3 (initialisation from gene
// arrays built from the boundary conditions, tournament selection, pairing
// without identical partners, per-kernel crossover and mutation, replacement
// by the best half of parents and of offspring), plus exhaustive, random and
// per-kernel brute-force searches over the same space, and the device
// evaluator whose fitness is the measured time of the whole hot path.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace amber {
namespace {

constexpr double kInf = std::numeric_limits<double>::infinity();
// genes [0, kGroupSplit): dedispersion; [kGroupSplit, n): boxcar / S/N
constexpr int kGroupSplit = AMBER_GENES_K1;
constexpr int kGeneDpt = 4;                    // dms_per_thread
constexpr int kGeneDirect = 5;                 // direct_reads
constexpr int kGeneSnr = AMBER_GENES_K1;       // snr_threads
constexpr int kGeneBox0 = AMBER_GENES_K1 + 1;  // boxcar_step[0]

// xoshiro256** (Blackman and Vigna), seeded through splitmix64.
class Rng {
public:
    explicit Rng(uint64_t seed)
    {
        uint64_t x = seed;
        for (auto &w : s_) {
            x += 0x9e3779b97f4a7c15ull;
            uint64_t z = x;
            z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
            z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
            w = z ^ (z >> 31);
        }
    }
    uint64_t next()
    {
        const uint64_t r = rotl(s_[1] * 5, 7) * 9;
        const uint64_t t = s_[1] << 17;
        s_[2] ^= s_[0];
        s_[3] ^= s_[1];
        s_[1] ^= s_[2];
        s_[0] ^= s_[3];
        s_[2] ^= t;
        s_[3] = rotl(s_[3], 45);
        return r;
    }
    double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }  // [0, 1)
    int below(int n) { return (int)(uniform() * n); }                 // [0, n)

private:
    static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
    uint64_t s_[4];
};

using Genome = std::vector<int>;  // index into each gene's value array

amber_tiles to_tiles(const amber_tune_space &sp, const Genome &g)
{
    amber_tiles t = default_tiles();
    t.threads_per_dm = sp.values[0][g[0]];
    t.samples_per_thread = sp.values[1][g[1]];
    t.dms_per_block = sp.values[2][g[2]];
    t.channel_unroll = sp.values[3][g[3]];
    t.dms_per_thread = sp.values[kGeneDpt][g[kGeneDpt]];
    t.direct_reads = sp.values[kGeneDirect][g[kGeneDirect]];
    t.snr_threads = sp.values[kGeneSnr][g[kGeneSnr]];
    for (int k = 0; k < sp.n_widths; ++k) t.boxcar_step[k] = sp.values[kGeneBox0 + k][g[kGeneBox0 + k]];
    return t;
}

bool valid_tiles(const amber_tune_space &sp, const amber_tiles &t)
{
    DedispPlan dp;
    BoxcarPlan bp;
    const bool ok = plan_dedisperse(t, sp.info, &dp) == AMBER_OK &&
                    plan_boxcar(t, sp.widths, sp.n_widths, sp.n_out, &bp) == AMBER_OK;
    clear_error();
    return ok;
}

std::string key_of(const Genome &g)
{
    std::string k;
    for (int v : g) k.push_back((char)('a' + v));
    return k;
}

std::string tiles_json(const amber_tiles &t, int n_widths)
{
    char buf[512];
    int n = snprintf(buf, sizeof buf,
                     "{\"threads_per_dm\":%d,\"samples_per_thread\":%d,\"dms_per_block\":%d,\"channel_unroll\":%d,"
                     "\"dms_per_thread\":%d,\"direct_reads\":%d,\"snr_threads\":%d,\"boxcar_step\":[",
                     t.threads_per_dm, t.samples_per_thread, t.dms_per_block, t.channel_unroll, t.dms_per_thread,
                     t.direct_reads, t.snr_threads);
    for (int k = 0; k < n_widths; ++k) n += snprintf(buf + n, sizeof buf - n, "%s%d", k ? "," : "", t.boxcar_step[k]);
    snprintf(buf + n, sizeof buf - n, "]}");
    return buf;
}

// A search problem: the genes and their value arrays, the kernels they
// belong to (kernel k owns genes [bounds[k], bounds[k + 1]); the last kernel
// is the boxcar / S/N kernel, whose first gene is its work-group size and the
// others one step per width), validity and fitness of a genome, and the
// library's default value of every gene (the start of per-kernel search).
class Problem {
public:
    virtual ~Problem() = default;
    virtual int n_genes() const = 0;
    virtual int n_values(int i) const = 0;
    virtual int value(int i, int v) const = 0;
    virtual const std::vector<int> &bounds() const = 0;
    virtual bool valid(const Genome &g) const = 0;
    virtual int32_t fitness(const Genome &g, double *seconds) = 0;
    virtual std::string json(const Genome &g) const = 0;
    virtual int default_value(int i) const = 0;
};

class Searcher {
public:
    Searcher(Problem &pb, const amber_tune_params &p, FILE *log)
        : pb_(pb), p_(p), log_(log), rng_(p.seed), t0_(clock_now())
    {
    }

    const Genome &best() const { return best_; }

    amber_status run(amber_tune_result *res)
    {
        amber_status s;
        switch (p_.search) {
        case AMBER_SEARCH_GA: s = ga(); break;
        case AMBER_SEARCH_EXHAUSTIVE: s = exhaustive(); break;
        case AMBER_SEARCH_RANDOM: s = random_search(); break;
        case AMBER_SEARCH_PER_KERNEL: s = per_kernel(); break;
        default: return fail(AMBER_E_ARG, "unknown search kind %d", p_.search);
        }
        if (s != AMBER_OK) return s;
        if (best_.empty() || !std::isfinite(best_fit_))
            return fail(AMBER_E_CONFIG, "no configuration of the space could be evaluated");
        if (p_.retime_top > 0) retime();
        res->best_time_s = best_fit_;
        res->n_evals = n_evals_;
        res->n_failed = n_failed_;
        res->wall_s = elapsed();
        return AMBER_OK;
    }

private:
    static double clock_now()
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
    }
    double elapsed() const { return clock_now() - t0_; }
    int n_genes() const { return pb_.n_genes(); }
    bool valid(const Genome &g) const { return pb_.valid(g); }
    int n_kernels() const { return (int)pb_.bounds().size() - 1; }
    int lo(int k) const { return pb_.bounds()[k]; }
    int hi(int k) const { return pb_.bounds()[k + 1]; }

    double evaluate(const Genome &g)
    {
        const std::string k = key_of(g);
        auto it = cache_.find(k);
        if (it != cache_.end()) return it->second;
        double sec = kInf;
        const int32_t rc = pb_.fitness(g, &sec);
        ++n_evals_;
        if (rc != 0 || !std::isfinite(sec) || sec < 0.0 || (p_.eval_timeout_s > 0.0 && sec > p_.eval_timeout_s)) {
            sec = kInf;
            ++n_failed_;
        }
        cache_.emplace(k, sec);
        if (p_.retime_top > 0 && std::isfinite(sec)) seen_.push_back({sec, g});
        if (sec < best_fit_) {
            best_fit_ = sec;
            best_ = g;
        }
        if (p_.search != AMBER_SEARCH_GA && log_ && n_evals_ % 50 == 0) log_line(-1);
        return sec;
    }

    // Re-times the search's retime_top best distinct configurations (by their
    // measured fitness) retime_runs times each, round robin, and keeps the
    // one with the lowest median: a search ends on its luckiest measurement,
    // which may belong to a configuration that is not the fastest.  The runs
    // count as evaluations.
    void retime()
    {
        const size_t k = std::min(seen_.size(), (size_t)p_.retime_top);
        std::partial_sort(seen_.begin(), seen_.begin() + k, seen_.end(),
                          [](const std::pair<double, Genome> &a, const std::pair<double, Genome> &b) {
                              return a.first < b.first;
                          });
        std::vector<std::vector<double>> t(k);
        for (int r = 0; r < p_.retime_runs; ++r)
            for (size_t i = 0; i < k; ++i) {
                double sec = kInf;
                const int32_t rc = pb_.fitness(seen_[i].second, &sec);
                ++n_evals_;
                if (rc != 0 || !std::isfinite(sec) || sec < 0.0) sec = kInf;
                t[i].push_back(sec);
            }
        double best = kInf;
        size_t bi = 0;
        std::string out = "{\"retime\":[";
        for (size_t i = 0; i < k; ++i) {
            std::sort(t[i].begin(), t[i].end());
            const double med = t[i][t[i].size() / 2];
            if (med < best) {
                best = med;
                bi = i;
            }
            char b[64];
            snprintf(b, sizeof b, "%s{\"search_s\":%.9g,\"median_s\":%.9g,\"best\":", i ? "," : "",
                     seen_[i].first, std::isfinite(med) ? med : -1.0);
            out += b;
            out += pb_.json(seen_[i].second);
            out += "}";
        }
        out += "]}\n";
        if (log_) {
            fputs(out.c_str(), log_);
            fflush(log_);
        }
        if (k > 0 && std::isfinite(best)) {
            best_ = seen_[bi].second;
            best_fit_ = best;
        }
    }

    void log_line(int generation)
    {
        if (!log_) return;
        const std::string best = best_.empty() ? "null" : pb_.json(best_);
        fprintf(log_,
                "{\"generation\":%d,\"evals\":%lld,\"failed\":%lld,\"restarts\":%d,\"best_time_s\":%.9g,"
                "\"wall_s\":%.6f,\"best\":%s}\n",
                generation, (long long)n_evals_, (long long)n_failed_, restarts_,
                std::isfinite(best_fit_) ? best_fit_ : -1.0, elapsed(), best.c_str());
        fflush(log_);
    }

    // One line with the final population: gene values (in the space's gene
    // order) and fitness of every individual.
    void log_population(const std::vector<Genome> &pop, const std::vector<double> &fit)
    {
        if (!log_) return;
        std::string out = "{\"final_population\":[";
        for (size_t i = 0; i < pop.size(); ++i) {
            out += i ? ",[" : "[";
            for (int k = 0; k < n_genes(); ++k) {
                if (k) out += ",";
                out += std::to_string(pb_.value(k, pop[i][k]));
            }
            out += "]";
        }
        out += "],\"fitness\":[";
        for (size_t i = 0; i < fit.size(); ++i) {
            char b[40];
            snprintf(b, sizeof b, "%s%.9g", i ? "," : "", std::isfinite(fit[i]) ? fit[i] : -1.0);
            out += b;
        }
        out += "]}\n";
        fputs(out.c_str(), log_);
        fflush(log_);
    }

    bool random_genome(Genome &g)
    {
        g.assign(n_genes(), 0);
        for (int attempt = 0; attempt < 100000; ++attempt) {
            for (int i = 0; i < n_genes(); ++i) g[i] = rng_.below(pb_.n_values(i));
            if (valid(g)) return true;
        }
        return false;
    }

    // The library's default configuration as a genome: each gene at its
    // default value (the first value where the array lacks it).  True when
    // every default value is in its gene's array.
    bool default_genome(Genome &g) const
    {
        bool all = true;
        for (int i = 0; i < n_genes(); ++i) {
            const int want = pb_.default_value(i);
            g[i] = 0;
            bool found = false;
            for (int v = 0; v < pb_.n_values(i); ++v)
                if (pb_.value(i, v) == want) {
                    g[i] = v;
                    found = true;
                }
            all = all && found;
        }
        return all;
    }

    // ---- genetic algorithm ------------------------------------------------
    int tournament(const std::vector<double> &fit)
    {
        const int n = (int)fit.size();
        int pool = (int)std::lround(p_.pool_frac * n);
        pool = std::max(2, std::min(pool, n));
        std::vector<int> idx(n);
        for (int i = 0; i < n; ++i) idx[i] = i;
        int win = -1;
        for (int k = 0; k < pool; ++k) {  // pool drawn without replacement
            const int j = k + rng_.below(n - k);
            std::swap(idx[k], idx[j]);
            const int c = idx[k];
            if (win < 0 || fit[c] < fit[win] || (fit[c] == fit[win] && c < win)) win = c;
        }
        return win;
    }

    void crossover_group(Genome &a, Genome &b, int lo, int hi)
    {
        if (p_.crossover == 1) {  // one-point: genes after a random cut are swapped
            if (hi - lo < 2) return;
            const int cut = lo + 1 + rng_.below(hi - lo - 1);
            Genome a2 = a, b2 = b;
            for (int i = cut; i < hi; ++i) std::swap(a2[i], b2[i]);
            if (valid(a2) && valid(b2)) {
                a = a2;
                b = b2;
            }
        } else {  // uniform: each gene swapped on a coin toss, kept only if both stay valid
            for (int i = lo; i < hi; ++i) {
                if (rng_.uniform() <= 0.5) continue;
                std::swap(a[i], b[i]);
                if (!valid(a) || !valid(b)) std::swap(a[i], b[i]);
            }
        }
    }

    // Changes gene i to another value of its array that keeps the genome valid,
    // if there is one.
    void mutate_gene(Genome &g, int i)
    {
        const int n = pb_.n_values(i);
        if (n < 2) return;
        const int old = g[i];
        std::vector<int> cand;
        for (int v = 0; v < n; ++v)
            if (v != old) cand.push_back(v);
        for (int left = (int)cand.size(); left > 0; --left) {
            const int j = rng_.below(left);
            g[i] = cand[j];
            if (valid(g)) return;
            std::swap(cand[j], cand[left - 1]);
        }
        g[i] = old;
    }

    void mutate(Genome &g)
    {
        // dedispersion kernels: one of each kernel's genes
        for (int k = 0; k + 1 < n_kernels(); ++k)
            if (rng_.uniform() < p_.p_mut) mutate_gene(g, lo(k) + rng_.below(hi(k) - lo(k)));
        // boxcar / S/N kernel: one gene per width, chosen between the width's
        // own step and the kernel's thread count
        const int kb = n_kernels() - 1;
        if (rng_.uniform() < p_.p_mut) {
            for (int w = 0; w + 1 < hi(kb) - lo(kb); ++w)
                mutate_gene(g, rng_.uniform() < 0.5 ? lo(kb) : lo(kb) + 1 + w);
        }
    }

    amber_status ga()
    {
        const int n = p_.pop;
        if (n < 2 || p_.generations < 0) return fail(AMBER_E_ARG, "GA needs pop >= 2 and generations >= 0");
        std::vector<Genome> pop(n);
        std::vector<double> fit(n);
        // seed_default: the first individual is the default configuration
        // (when it is in the space and valid), the others random
        Genome d(n_genes());
        const bool seeded = p_.seed_default && default_genome(d) && valid(d);
        for (int i = 0; i < n; ++i) {
            if (i == 0 && seeded)
                pop[i] = d;
            else if (!random_genome(pop[i]))
                return fail(AMBER_E_CONFIG, "no valid configuration found to initialise");
            fit[i] = evaluate(pop[i]);
        }
        log_line(0);
        double best = *std::min_element(fit.begin(), fit.end());
        int stale = 0;  // generations since the best fitness last improved
        for (int gen = 1; gen <= p_.generations; ++gen) {
            // restart on stagnation (an option, off in the paper's form): all
            // but the best individual are replaced by fresh random ones
            if (p_.restart_after > 0 && stale >= p_.restart_after) {
                const int keep = (int)(std::min_element(fit.begin(), fit.end()) - fit.begin());
                for (int i = 0; i < n; ++i) {
                    if (i == keep) continue;
                    if (!random_genome(pop[i])) return fail(AMBER_E_CONFIG, "no valid configuration found to restart");
                    fit[i] = evaluate(pop[i]);
                }
                stale = 0;
                ++restarts_;
            }
            // selection: N_pop tournaments
            std::vector<int> sel(n);
            for (int i = 0; i < n; ++i) sel[i] = tournament(fit);
            // pairing, avoiding identical partners where possible
            for (int i = 0; i + 1 < n; i += 2) {
                if (pop[sel[i]] != pop[sel[i + 1]]) continue;
                for (int j = i + 2; j < n; ++j)
                    if (pop[sel[j]] != pop[sel[i]]) {
                        std::swap(sel[i + 1], sel[j]);
                        break;
                    }
            }
            std::vector<Genome> off(n);
            for (int i = 0; i < n; ++i) off[i] = pop[sel[i]];
            for (int i = 0; i + 1 < n; i += 2)
                for (int k = 0; k < n_kernels(); ++k)
                    if (rng_.uniform() < p_.p_cross) crossover_group(off[i], off[i + 1], lo(k), hi(k));
            std::vector<double> off_fit(n);
            for (int i = 0; i < n; ++i) {
                mutate(off[i]);
                off_fit[i] = evaluate(off[i]);
            }
            // replacement: best half of the parents and best half of the offspring
            std::vector<int> pi(n), oi(n);
            for (int i = 0; i < n; ++i) pi[i] = oi[i] = i;
            std::stable_sort(pi.begin(), pi.end(), [&](int a, int b) { return fit[a] < fit[b]; });
            std::stable_sort(oi.begin(), oi.end(), [&](int a, int b) { return off_fit[a] < off_fit[b]; });
            std::vector<Genome> next;
            std::vector<double> next_fit;
            const int keep_parents = (n + 1) / 2;
            for (int i = 0; i < keep_parents; ++i) {
                next.push_back(pop[pi[i]]);
                next_fit.push_back(fit[pi[i]]);
            }
            for (int i = 0; i < n - keep_parents; ++i) {
                next.push_back(off[oi[i]]);
                next_fit.push_back(off_fit[oi[i]]);
            }
            pop.swap(next);
            fit.swap(next_fit);
            const double b = *std::min_element(fit.begin(), fit.end());
            stale = b < best ? 0 : stale + 1;
            best = b < best ? b : best;
            log_line(gen);
        }
        log_population(pop, fit);
        return AMBER_OK;
    }

    // ---- enumeration-based searches ------------------------------------------
    // Calls f on every valid genome whose genes outside [lo, hi) equal `base`.
    template <typename F>
    void enumerate(const Genome &base, int lo, int hi, F f)
    {
        Genome g = base;
        for (int i = lo; i < hi; ++i) g[i] = 0;
        for (;;) {
            if (valid(g)) f(g);
            int i = lo;
            while (i < hi && ++g[i] == pb_.n_values(i)) g[i++] = 0;
            if (i == hi) return;
        }
    }

    amber_status exhaustive()
    {
        int64_t count = 0;
        enumerate(Genome(n_genes(), 0), 0, n_genes(), [&](const Genome &) { ++count; });
        if (p_.max_evals > 0 && count > p_.max_evals)
            return fail(AMBER_E_ARG, "exhaustive search of %lld configurations exceeds max_evals=%lld",
                        (long long)count, (long long)p_.max_evals);
        enumerate(Genome(n_genes(), 0), 0, n_genes(), [&](const Genome &g) { evaluate(g); });
        log_line(-1);
        return AMBER_OK;
    }

    amber_status random_search()
    {
        if (p_.max_evals <= 0) return fail(AMBER_E_ARG, "random search needs max_evals > 0");
        Genome g;
        for (int64_t draws = 0; n_evals_ < p_.max_evals && draws < 100 * p_.max_evals; ++draws) {
            if (!random_genome(g)) return fail(AMBER_E_CONFIG, "no valid configuration found");
            evaluate(g);
        }
        log_line(-1);
        return AMBER_OK;
    }

    // Paper-style brute force: each kernel's genes exhaustively, in kernel
    // order, with the other kernels' genes held: the library's defaults for
    // kernels not yet searched, the best found for those already searched.
    amber_status per_kernel()
    {
        Genome base(n_genes(), 0);
        default_genome(base);
        for (int k = 0; k < n_kernels(); ++k) {
            Genome best_k;
            double fit_k = kInf;
            enumerate(base, lo(k), hi(k), [&](const Genome &g) {
                const double f = evaluate(g);
                if (f < fit_k) {
                    fit_k = f;
                    best_k = g;
                }
            });
            if (best_k.empty())
                return fail(AMBER_E_CONFIG, "no valid configuration of kernel %d with the other kernels' defaults", k);
            base = best_k;
        }
        log_line(-1);
        return AMBER_OK;
    }

    Problem &pb_;
    const amber_tune_params &p_;
    FILE *log_;
    Rng rng_;
    double t0_;
    std::unordered_map<std::string, double> cache_;
    std::vector<std::pair<double, Genome>> seen_;  // evaluated genomes (kept when retime_top > 0)
    Genome best_;
    double best_fit_ = kInf;
    int64_t n_evals_ = 0, n_failed_ = 0;
    int restarts_ = 0;
};

// The hot path's search: one dedispersion tile and the boxcar / S/N genes,
// all in one amber_tiles.
class TilesProblem : public Problem {
public:
    TilesProblem(const amber_tune_space &sp, amber_fitness_fn fn, void *user)
        : sp_(sp), fn_(fn), user_(user), bounds_{0, kGroupSplit, sp.n_genes}
    {
    }
    int n_genes() const override { return sp_.n_genes; }
    int n_values(int i) const override { return sp_.n_values[i]; }
    int value(int i, int v) const override { return sp_.values[i][v]; }
    const std::vector<int> &bounds() const override { return bounds_; }
    bool valid(const Genome &g) const override { return valid_tiles(sp_, to_tiles(sp_, g)); }
    int32_t fitness(const Genome &g, double *sec) override
    {
        const amber_tiles t = to_tiles(sp_, g);
        return fn_(&t, user_, sec);
    }
    std::string json(const Genome &g) const override { return tiles_json(to_tiles(sp_, g), sp_.n_widths); }
    int default_value(int i) const override
    {
        const amber_tiles &d = default_tiles();
        const int k1[] = {d.threads_per_dm, d.samples_per_thread, d.dms_per_block, d.channel_unroll,
                          d.dms_per_thread, d.direct_reads, d.snr_threads};
        return i < kGeneBox0 ? k1[i] : d.boxcar_step[i - kGeneBox0];
    }

private:
    const amber_tune_space &sp_;
    amber_fitness_fn fn_;
    void *user_;
    std::vector<int> bounds_;
};

amber_status check_space(const amber_tune_space *sp)
{
    if (!sp) return fail(AMBER_E_ARG, "space is NULL");
    if (sp->n_widths < 1 || sp->n_widths > AMBER_MAX_WIDTHS || sp->n_genes != kGeneBox0 + sp->n_widths)
        return fail(AMBER_E_ARG, "space must have n_genes = %d + n_widths with 1 <= n_widths <= %d", kGeneBox0,
                    AMBER_MAX_WIDTHS);
    for (int i = 0; i < sp->n_genes; ++i)
        if (sp->n_values[i] < 1 || sp->n_values[i] > AMBER_MAX_GENE_VALUES)
            return fail(AMBER_E_ARG, "gene %d has %d values (1..%d allowed)", i, sp->n_values[i], AMBER_MAX_GENE_VALUES);
    return AMBER_OK;
}

// ---- subband pipeline ------------------------------------------------------------
constexpr int kSbStep2 = AMBER_SUBBAND_GENES_STEP1;                // first gene of step two
constexpr int kSbSnr = AMBER_SUBBAND_GENES_STEP1 + AMBER_SUBBAND_GENES_STEP2;
constexpr int kSbBox0 = kSbSnr + 1;

struct SubbandTiles {
    amber_tiles step1, step2;  // step1 also carries the boxcar / S/N genes
};

SubbandTiles sb_tiles(const amber_subband_tune_space &sp, const Genome &g)
{
    SubbandTiles t{default_tiles(), default_tiles()};
    auto v = [&](int i) { return sp.values[i][g[i]]; };
    t.step1.threads_per_dm = v(0);
    t.step1.samples_per_thread = v(1);
    t.step1.dms_per_block = v(2);
    t.step1.channel_unroll = v(3);
    t.step1.dms_per_thread = v(4);
    t.step2.threads_per_dm = v(kSbStep2 + 0);
    t.step2.samples_per_thread = v(kSbStep2 + 1);
    t.step2.dms_per_block = v(kSbStep2 + 2);
    t.step2.channel_unroll = v(kSbStep2 + 3);
    t.step2.dms_per_thread = 1;
    t.step1.snr_threads = t.step2.snr_threads = v(kSbSnr);
    for (int k = 0; k < sp.n_widths; ++k) t.step1.boxcar_step[k] = t.step2.boxcar_step[k] = v(kSbBox0 + k);
    return t;
}

amber_delay_info sb_info1(const amber_subband_info &i)
{
    return amber_delay_info{i.n_coarse, i.n_chan / i.n_subbands, i.max_delay1, i.max_step1};
}
amber_delay_info sb_info2(const amber_subband_info &i)
{
    return amber_delay_info{i.n_fine, i.n_subbands, i.max_delay2, i.max_step2};
}

bool sb_valid_step(const amber_subband_tune_space &sp, const amber_tiles &t, int step)
{
    DedispPlan dp;
    const bool ok = step == 1 ? plan_dedisperse(t, sb_info1(sp.info), &dp, 0) == AMBER_OK
                              : plan_dedisperse(t, sb_info2(sp.info), &dp, 1) == AMBER_OK;
    clear_error();
    return ok;
}

bool sb_valid_box(const amber_subband_tune_space &sp, const amber_tiles &t)
{
    BoxcarPlan bp;
    const bool ok = plan_boxcar(t, sp.widths, sp.n_widths, sp.n_out, &bp) == AMBER_OK;
    clear_error();
    return ok;
}

std::string sb_json(const SubbandTiles &t, int n_widths)
{
    char buf[256];
    snprintf(buf, sizeof buf,
             "{\"step1\":{\"threads_per_dm\":%d,\"samples_per_thread\":%d,\"dms_per_block\":%d,"
             "\"channel_unroll\":%d,\"dms_per_thread\":%d},\"step2\":{\"threads_per_dm\":%d,"
             "\"samples_per_thread\":%d,\"dms_per_block\":%d,\"channel_unroll\":%d},\"box\":",
             t.step1.threads_per_dm, t.step1.samples_per_thread, t.step1.dms_per_block, t.step1.channel_unroll,
             t.step1.dms_per_thread, t.step2.threads_per_dm, t.step2.samples_per_thread, t.step2.dms_per_block,
             t.step2.channel_unroll);
    return std::string(buf) + tiles_json(t.step1, n_widths) + "}";
}

class SubbandProblem : public Problem {
public:
    SubbandProblem(const amber_subband_tune_space &sp, amber_subband_fitness_fn fn, void *user)
        : sp_(sp), fn_(fn), user_(user), bounds_{0, kSbStep2, kSbSnr, sp.n_genes}
    {
        const amber_subband_info &i = sp.info;
        d1_ = subband_step_tiles(i.n_coarse, i.n_chan / i.n_subbands, 0);
        d2_ = subband_step_tiles(i.n_fine, i.n_subbands, 1);
    }
    int n_genes() const override { return sp_.n_genes; }
    int n_values(int i) const override { return sp_.n_values[i]; }
    int value(int i, int v) const override { return sp_.values[i][v]; }
    const std::vector<int> &bounds() const override { return bounds_; }
    bool valid(const Genome &g) const override
    {
        const SubbandTiles t = sb_tiles(sp_, g);
        return sb_valid_step(sp_, t.step1, 1) && sb_valid_step(sp_, t.step2, 2) && sb_valid_box(sp_, t.step1);
    }
    int32_t fitness(const Genome &g, double *sec) override
    {
        const SubbandTiles t = sb_tiles(sp_, g);
        return fn_(&t.step1, &t.step2, user_, sec);
    }
    std::string json(const Genome &g) const override { return sb_json(sb_tiles(sp_, g), sp_.n_widths); }
    int default_value(int i) const override
    {
        const amber_tiles &d = default_tiles();
        const int v[] = {d1_.threads_per_dm, d1_.samples_per_thread, d1_.dms_per_block, d1_.channel_unroll,
                         d1_.dms_per_thread, d2_.threads_per_dm, d2_.samples_per_thread, d2_.dms_per_block,
                         d2_.channel_unroll, d.snr_threads};
        return i < kSbBox0 ? v[i] : d.boxcar_step[i - kSbBox0];
    }

private:
    const amber_subband_tune_space &sp_;
    amber_subband_fitness_fn fn_;
    void *user_;
    std::vector<int> bounds_;
    amber_tiles d1_, d2_;
};

amber_status check_subband_space(const amber_subband_tune_space *sp)
{
    if (!sp) return fail(AMBER_E_ARG, "space is NULL");
    if (sp->n_widths < 1 || sp->n_widths > AMBER_MAX_WIDTHS || sp->n_genes != kSbBox0 + sp->n_widths)
        return fail(AMBER_E_ARG, "space must have n_genes = %d + n_widths with 1 <= n_widths <= %d", kSbBox0,
                    AMBER_MAX_WIDTHS);
    const amber_subband_info &i = sp->info;
    if (i.n_subbands < 1 || i.n_chan < 1 || i.n_chan % i.n_subbands != 0 || i.n_coarse < 1 || i.n_fine < 1)
        return fail(AMBER_E_ARG, "space has an invalid subband info");
    for (int g = 0; g < sp->n_genes; ++g)
        if (sp->n_values[g] < 1 || sp->n_values[g] > AMBER_MAX_GENE_VALUES)
            return fail(AMBER_E_ARG, "gene %d has %d values (1..%d allowed)", g, sp->n_values[g], AMBER_MAX_GENE_VALUES);
    return AMBER_OK;
}

// Times run() on `stream` with HIP events: p.warmup untimed runs, then the
// median of p.reps timed runs.  Returns nonzero on failure (err receives a
// device error, which ends the search).
struct EventTimer {
    std::vector<hipEvent_t> ev;
    int warmup = 0, reps = 1;
    hipStream_t stream = nullptr;
    amber_status error = AMBER_OK;

    amber_status init(int w, int r, hipStream_t s)
    {
        warmup = w;
        reps = r;
        stream = s;
        ev.resize(2 * r);
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) return fail(AMBER_E_DEVICE, "hipEventCreate failed");
        return AMBER_OK;
    }
    ~EventTimer()
    {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    template <typename F>
    int32_t time(F run, double *seconds)
    {
        for (int w = 0; w < warmup; ++w)
            if (run() != AMBER_OK) return 1;
        std::vector<float> ms(reps);
        for (int r = 0; r < reps; ++r) {
            if (hipEventRecord(ev[2 * r], stream) != hipSuccess) return 1;
            if (run() != AMBER_OK) return 1;
            if (hipEventRecord(ev[2 * r + 1], stream) != hipSuccess) return 1;
        }
        if (hipEventSynchronize(ev[2 * reps - 1]) != hipSuccess) {
            error = AMBER_E_DEVICE;
            return 1;
        }
        for (int r = 0; r < reps; ++r)
            if (hipEventElapsedTime(&ms[r], ev[2 * r], ev[2 * r + 1]) != hipSuccess) return 1;
        std::sort(ms.begin(), ms.end());
        *seconds = 1e-3 * (double)ms[reps / 2];
        return 0;
    }
};

struct SubbandEval {
    const amber_subband_tune_space *sp;
    const int32_t *d_delay1, *d_delay2;
    const uint8_t *d_in;
    int64_t in_stride, n_in;
    uint16_t *d_work;
    int64_t work_stride;
    int32_t *d_dd;
    int64_t dd_stride;
    float *d_snr;
    int32_t *d_peak;
    EventTimer timer;
};

amber_status run_subband_path(SubbandEval &e, const amber_tiles &t1, const amber_tiles &t2)
{
    const amber_subband_tune_space &sp = *e.sp;
    amber_status s = amber_subband_dedisperse(e.d_delay1, e.d_delay2, &sp.info, e.d_in, e.in_stride, e.n_in, e.d_work,
                                              e.work_stride, e.d_dd, e.dd_stride, sp.n_out, nullptr, &t1, &t2,
                                              e.timer.stream);
    if (s != AMBER_OK) return s;
    return amber_integrate_snr(e.d_dd, sp.info.n_coarse * sp.info.n_fine, e.dd_stride, sp.n_out, sp.widths,
                               sp.n_widths, e.d_snr, e.d_peak, &t1, e.timer.stream);
}

int32_t subband_device_fitness(const amber_tiles *t1, const amber_tiles *t2, void *user, double *seconds)
{
    SubbandEval &e = *static_cast<SubbandEval *>(user);
    return e.timer.time([&] { return run_subband_path(e, *t1, *t2); }, seconds);
}

// ---- device evaluator ---------------------------------------------------------
struct DeviceEval {
    const amber_tune_space *sp;
    const int32_t *d_delays;
    const uint8_t *d_in;
    int64_t in_stride, n_in;
    int32_t *d_dd;
    int64_t dd_stride;
    float *d_snr;
    int32_t *d_peak;
    int warmup, reps;
    hipStream_t stream;
    std::vector<hipEvent_t> ev;
    amber_status error = AMBER_OK;
};

amber_status run_path(DeviceEval &e, const amber_tiles &t)
{
    amber_status s = amber_dedisperse(e.d_delays, &e.sp->info, e.d_in, e.in_stride, e.n_in, e.d_dd, e.dd_stride,
                                      e.sp->n_out, &t, e.stream);
    if (s != AMBER_OK) return s;
    return amber_integrate_snr(e.d_dd, e.sp->info.n_dm, e.dd_stride, e.sp->n_out, e.sp->widths, e.sp->n_widths,
                               e.d_snr, e.d_peak, &t, e.stream);
}

int32_t device_fitness(const amber_tiles *t, void *user, double *seconds)
{
    DeviceEval &e = *static_cast<DeviceEval *>(user);
    for (int w = 0; w < e.warmup; ++w)
        if (run_path(e, *t) != AMBER_OK) return 1;
    std::vector<float> ms(e.reps);
    for (int r = 0; r < e.reps; ++r) {
        if (hipEventRecord(e.ev[2 * r], e.stream) != hipSuccess) return 1;
        if (run_path(e, *t) != AMBER_OK) return 1;
        if (hipEventRecord(e.ev[2 * r + 1], e.stream) != hipSuccess) return 1;
    }
    if (hipEventSynchronize(e.ev[2 * e.reps - 1]) != hipSuccess) {
        e.error = AMBER_E_DEVICE;
        return 1;
    }
    for (int r = 0; r < e.reps; ++r)
        if (hipEventElapsedTime(&ms[r], e.ev[2 * r], e.ev[2 * r + 1]) != hipSuccess) return 1;
    std::sort(ms.begin(), ms.end());
    *seconds = 1e-3 * (double)ms[e.reps / 2];
    return 0;
}

}  // namespace
}  // namespace amber

using namespace amber;

extern "C" {

amber_status amber_default_tune_params(amber_tune_params *p)
{
    clear_error();
    if (!p) return fail(AMBER_E_ARG, "params is NULL");
    *p = amber_tune_params{};
    p->search = AMBER_SEARCH_GA;
    p->pop = 32;
    p->generations = 40;
    p->crossover = 0;
    p->p_cross = 0.8;
    p->p_mut = 0.1;
    p->pool_frac = 0.2;
    p->seed = 1;
    p->warmup = 1;
    p->reps = 3;
    p->eval_timeout_s = 1.0;
    p->max_evals = 0;
    return AMBER_OK;
}

amber_status amber_default_space(const amber_delay_info *info, const int32_t *widths, int32_t n_widths, int64_t n_out,
                                 amber_tune_space *sp)
{
    clear_error();
    if (!info || !widths || !sp) return fail(AMBER_E_ARG, "NULL argument");
    if (n_widths < 1 || n_widths > AMBER_MAX_WIDTHS) return fail(AMBER_E_ARG, "n_widths=%d out of range", n_widths);
    *sp = amber_tune_space{};
    const std::vector<std::vector<int>> vals = {
        {64, 128, 256, 512, 1024},  // threads_per_dm
        {4, 8, 16, 32},             // samples_per_thread
        {1, 2, 4, 8, 16},           // dms_per_block
        {1, 2, 4, 8, 16, 32},       // channel_unroll
        {1, 2},                     // dms_per_thread
        {0, 1},                     // direct_reads (localMem on, off)
        {64, 128, 256, 512, 1024},  // snr_threads
    };
    sp->n_genes = kGeneBox0 + n_widths;
    // the kernel for up to 8 sliding widths of at most 64 samples has no
    // per-width step: those genes keep one value
    const std::vector<int> steps = span_snr_applies(widths, n_widths, 0, n_out) ? std::vector<int>{8}
                                                                               : std::vector<int>{1, 2, 4, 8};
    for (int i = 0; i < sp->n_genes; ++i) {
        const std::vector<int> v = i < kGeneBox0 ? vals[i] : steps;
        sp->n_values[i] = (int32_t)v.size();
        for (size_t k = 0; k < v.size(); ++k) sp->values[i][k] = v[k];
    }
    sp->info = *info;
    sp->n_widths = n_widths;
    for (int k = 0; k < n_widths; ++k) sp->widths[k] = widths[k];
    sp->n_out = n_out;
    return AMBER_OK;
}

amber_status amber_space_size(const amber_tune_space *sp, int64_t *count)
{
    clear_error();
    amber_status s = check_space(sp);
    if (s != AMBER_OK) return s;
    if (!count) return fail(AMBER_E_ARG, "count is NULL");
    // dedispersion and boxcar validity are independent: count each part
    int64_t n1 = 0, n2 = 0;
    std::vector<int> g(sp->n_genes, 0);
    amber_tiles t = default_tiles();
    for (;;) {
        t.threads_per_dm = sp->values[0][g[0]];
        t.samples_per_thread = sp->values[1][g[1]];
        t.dms_per_block = sp->values[2][g[2]];
        t.channel_unroll = sp->values[3][g[3]];
        t.dms_per_thread = sp->values[kGeneDpt][g[kGeneDpt]];
        t.direct_reads = sp->values[kGeneDirect][g[kGeneDirect]];
        DedispPlan dp;
        if (plan_dedisperse(t, sp->info, &dp) == AMBER_OK) ++n1;
        int i = 0;
        while (i < kGroupSplit && ++g[i] == sp->n_values[i]) g[i++] = 0;
        if (i == kGroupSplit) break;
    }
    for (;;) {
        t.snr_threads = sp->values[kGeneSnr][g[kGeneSnr]];
        for (int k = 0; k < sp->n_widths; ++k) t.boxcar_step[k] = sp->values[kGeneBox0 + k][g[kGeneBox0 + k]];
        BoxcarPlan bp;
        if (plan_boxcar(t, sp->widths, sp->n_widths, sp->n_out, &bp) == AMBER_OK) ++n2;
        int i = kGroupSplit;
        while (i < sp->n_genes && ++g[i] == sp->n_values[i]) g[i++] = 0;
        if (i == sp->n_genes) break;
    }
    clear_error();
    *count = n1 * n2;
    return AMBER_OK;
}

amber_status amber_search_tiles(const amber_tune_space *space, const amber_tune_params *p, amber_fitness_fn fn,
                                void *user, amber_tune_result *result, const char *log_jsonl_path)
{
    clear_error();
    amber_status s = check_space(space);
    if (s != AMBER_OK) return s;
    if (!p || !fn || !result) return fail(AMBER_E_ARG, "NULL params, fitness or result");
    if (!(p->p_cross >= 0 && p->p_cross <= 1 && p->p_mut >= 0 && p->p_mut <= 1 && p->pool_frac > 0 && p->pool_frac <= 1))
        return fail(AMBER_E_ARG, "probabilities must lie in [0, 1] and pool_frac in (0, 1]");
    if (p->restart_after < 0) return fail(AMBER_E_ARG, "restart_after=%d must be >= 0", p->restart_after);
    if (p->retime_top < 0 || (p->retime_top > 0 && (p->retime_runs < 1 || p->retime_runs > 64)))
        return fail(AMBER_E_ARG, "retime_top=%d must be >= 0 and, when > 0, retime_runs=%d in [1, 64]", p->retime_top,
                    p->retime_runs);
    FILE *log = nullptr;
    if (log_jsonl_path && *log_jsonl_path) {
        log = fopen(log_jsonl_path, "a");
        if (!log) return fail(AMBER_E_ARG, "cannot open log %s", log_jsonl_path);
    }
    *result = amber_tune_result{};
    int64_t size = 0;
    amber_space_size(space, &size);
    TilesProblem pb(*space, fn, user);
    Searcher srch(pb, *p, log);
    s = srch.run(result);
    if (s == AMBER_OK) result->best = to_tiles(*space, srch.best());
    result->space_size = size;
    if (log) fclose(log);
    return s;
}

amber_status amber_tune(const amber_tune_space *space, const int32_t *d_delays, const uint8_t *d_in, int64_t in_stride,
                        int64_t n_in, int32_t *d_dd, int64_t dd_stride, float *d_snr, int32_t *d_peak_t,
                        const amber_tune_params *p, amber_tune_result *result, const char *log_jsonl_path, void *stream)
{
    clear_error();
    amber_status s = check_space(space);
    if (s != AMBER_OK) return s;
    if (!p || !d_delays || !d_in || !d_dd || !d_snr || !result) return fail(AMBER_E_ARG, "NULL argument");
    if (p->reps < 1 || p->reps > 64 || p->warmup < 0) return fail(AMBER_E_ARG, "reps must be in [1, 64], warmup >= 0");
    DeviceEval e;
    e.sp = space;
    e.d_delays = d_delays;
    e.d_in = d_in;
    e.in_stride = in_stride;
    e.n_in = n_in;
    e.d_dd = d_dd;
    e.dd_stride = dd_stride;
    e.d_snr = d_snr;
    e.d_peak = d_peak_t;
    e.warmup = p->warmup;
    e.reps = p->reps;
    e.stream = (hipStream_t)stream;
    e.ev.resize(2 * p->reps);
    for (auto &ev : e.ev)
        if (hipEventCreate(&ev) != hipSuccess) return fail(AMBER_E_DEVICE, "hipEventCreate failed");
    // the default configuration must run: catches bad buffers before searching
    double t0;
    if (device_fitness(&default_tiles(), &e, &t0) != 0 && e.error != AMBER_OK) {
        for (auto &ev : e.ev) (void)hipEventDestroy(ev);
        return fail(AMBER_E_DEVICE, "the hot path failed on the default tiles");
    }
    s = amber_search_tiles(space, p, device_fitness, &e, result, log_jsonl_path);
    std::string msg = s != AMBER_OK ? amber_last_error() : "";
    for (auto &ev : e.ev) (void)hipEventDestroy(ev);
    if (e.error != AMBER_OK) return fail(e.error, "device error during the search");
    if (s != AMBER_OK) return fail(s, "%s", msg.c_str());
    return AMBER_OK;
}

amber_status amber_default_subband_space(const amber_subband_info *info, const int32_t *widths, int32_t n_widths,
                                         int64_t n_out, amber_subband_tune_space *sp)
{
    clear_error();
    if (!info || !widths || !sp) return fail(AMBER_E_ARG, "NULL argument");
    if (n_widths < 1 || n_widths > AMBER_MAX_WIDTHS) return fail(AMBER_E_ARG, "n_widths=%d out of range", n_widths);
    *sp = amber_subband_tune_space{};
    const std::vector<std::vector<int>> vals = {
        {64, 128, 256},             // step one: threads_per_dm
        {4, 8, 16},                 //           samples_per_thread
        {2, 4, 8, 12, 16},          //           dms_per_block
        {4, 8, 16, 32},             //           channel_unroll
        {1, 2},                     //           dms_per_thread
        {64, 128, 256},             // step two: threads_per_dm
        {8, 16},                    //           samples_per_thread
        {4, 6, 8, 12, 16},          //           dms_per_block
        {4, 8, 16, 32},             //           channel_unroll
        {64, 128, 256, 512, 1024},  // snr_threads
    };
    sp->n_genes = kSbBox0 + n_widths;
    const std::vector<int> steps = span_snr_applies(widths, n_widths, 0, n_out) ? std::vector<int>{8}
                                                                               : std::vector<int>{1, 2, 4, 8};
    for (int i = 0; i < sp->n_genes; ++i) {
        const std::vector<int> v = i < kSbBox0 ? vals[i] : steps;
        sp->n_values[i] = (int32_t)v.size();
        for (size_t k = 0; k < v.size(); ++k) sp->values[i][k] = v[k];
    }
    sp->info = *info;
    sp->n_widths = n_widths;
    for (int k = 0; k < n_widths; ++k) sp->widths[k] = widths[k];
    sp->n_out = n_out;
    return check_subband_space(sp);
}

amber_status amber_subband_space_size(const amber_subband_tune_space *sp, int64_t *count)
{
    clear_error();
    amber_status s = check_subband_space(sp);
    if (s != AMBER_OK) return s;
    if (!count) return fail(AMBER_E_ARG, "count is NULL");
    // the three kernels' validity is independent: count each kernel's genes
    const int bounds[] = {0, kSbStep2, kSbSnr, sp->n_genes};
    int64_t total = 1;
    for (int k = 0; k < 3; ++k) {
        int64_t n = 0;
        Genome g(sp->n_genes, 0);
        for (;;) {
            const SubbandTiles t = sb_tiles(*sp, g);
            if (k == 0 ? sb_valid_step(*sp, t.step1, 1) : (k == 1 ? sb_valid_step(*sp, t.step2, 2) : sb_valid_box(*sp, t.step1)))
                ++n;
            int i = bounds[k];
            while (i < bounds[k + 1] && ++g[i] == sp->n_values[i]) g[i++] = 0;
            if (i == bounds[k + 1]) break;
        }
        total *= n;
    }
    *count = total;
    return AMBER_OK;
}

amber_status amber_search_subband_tiles(const amber_subband_tune_space *space, const amber_tune_params *p,
                                        amber_subband_fitness_fn fn, void *user, amber_subband_tune_result *result,
                                        const char *log_jsonl_path)
{
    clear_error();
    amber_status s = check_subband_space(space);
    if (s != AMBER_OK) return s;
    if (!p || !fn || !result) return fail(AMBER_E_ARG, "NULL params, fitness or result");
    if (!(p->p_cross >= 0 && p->p_cross <= 1 && p->p_mut >= 0 && p->p_mut <= 1 && p->pool_frac > 0 && p->pool_frac <= 1))
        return fail(AMBER_E_ARG, "probabilities must lie in [0, 1] and pool_frac in (0, 1]");
    if (p->restart_after < 0) return fail(AMBER_E_ARG, "restart_after=%d must be >= 0", p->restart_after);
    if (p->retime_top < 0 || (p->retime_top > 0 && (p->retime_runs < 1 || p->retime_runs > 64)))
        return fail(AMBER_E_ARG, "retime_top=%d must be >= 0 and, when > 0, retime_runs=%d in [1, 64]", p->retime_top,
                    p->retime_runs);
    FILE *log = nullptr;
    if (log_jsonl_path && *log_jsonl_path) {
        log = fopen(log_jsonl_path, "a");
        if (!log) return fail(AMBER_E_ARG, "cannot open log %s", log_jsonl_path);
    }
    *result = amber_subband_tune_result{};
    int64_t size = 0;
    amber_subband_space_size(space, &size);
    SubbandProblem pb(*space, fn, user);
    Searcher srch(pb, *p, log);
    amber_tune_result r{};
    s = srch.run(&r);
    if (s == AMBER_OK) {
        const SubbandTiles t = sb_tiles(*space, srch.best());
        result->step1 = t.step1;
        result->step2 = t.step2;
    }
    result->best_time_s = r.best_time_s;
    result->n_evals = r.n_evals;
    result->n_failed = r.n_failed;
    result->wall_s = r.wall_s;
    result->space_size = size;
    if (log) fclose(log);
    return s;
}

amber_status amber_tune_subband(const amber_subband_tune_space *space, const int32_t *d_delay1,
                                const int32_t *d_delay2, const uint8_t *d_in, int64_t in_stride, int64_t n_in,
                                uint16_t *d_work, int64_t work_stride, int32_t *d_dd, int64_t dd_stride,
                                float *d_snr, int32_t *d_peak_t, const amber_tune_params *p,
                                amber_subband_tune_result *result, const char *log_jsonl_path, void *stream)
{
    clear_error();
    amber_status s = check_subband_space(space);
    if (s != AMBER_OK) return s;
    if (!p || !d_delay1 || !d_delay2 || !d_in || !d_work || !d_dd || !d_snr || !result)
        return fail(AMBER_E_ARG, "NULL argument");
    if (p->reps < 1 || p->reps > 64 || p->warmup < 0) return fail(AMBER_E_ARG, "reps must be in [1, 64], warmup >= 0");
    SubbandEval e;
    e.sp = space;
    e.d_delay1 = d_delay1;
    e.d_delay2 = d_delay2;
    e.d_in = d_in;
    e.in_stride = in_stride;
    e.n_in = n_in;
    e.d_work = d_work;
    e.work_stride = work_stride;
    e.d_dd = d_dd;
    e.dd_stride = dd_stride;
    e.d_snr = d_snr;
    e.d_peak = d_peak_t;
    if ((s = e.timer.init(p->warmup, p->reps, (hipStream_t)stream)) != AMBER_OK) return s;
    // the path must run with the automatic tiles: catches bad buffers before searching
    s = amber_subband_dedisperse(d_delay1, d_delay2, &space->info, d_in, in_stride, n_in, d_work, work_stride, d_dd,
                                 dd_stride, space->n_out, nullptr, nullptr, nullptr, stream);
    if (s == AMBER_OK)
        s = amber_integrate_snr(d_dd, space->info.n_coarse * space->info.n_fine, dd_stride, space->n_out,
                                space->widths, space->n_widths, d_snr, d_peak_t, nullptr, stream);
    if (s != AMBER_OK) return s;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return fail(AMBER_E_DEVICE, "the subband path failed on the automatic tiles");
    s = amber_search_subband_tiles(space, p, subband_device_fitness, &e, result, log_jsonl_path);
    std::string msg = s != AMBER_OK ? amber_last_error() : "";
    if (e.timer.error != AMBER_OK) return fail(e.timer.error, "device error during the search");
    if (s != AMBER_OK) return fail(s, "%s", msg.c_str());
    return AMBER_OK;
}

}  // extern "C"
