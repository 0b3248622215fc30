"""The tile search (genetic algorithm, exhaustive, random, per-kernel brute
force) driven by fake fitness landscapes on the CPU.

There is no numeric oracle for a search whose fitness is a timing; these
tests pin the operators' contracts instead: every evaluated configuration is
valid, exhaustive search returns the argmin, results are deterministic under
a seed, failed or timed-out evaluations are never selected, the random search
keeps to its budget, the per-kernel search solves separable landscapes, and
the GA's best never gets worse between generations.
"""
import itertools
import json
import math

import numpy as np
import pytest

import oracle
import workloads


@pytest.fixture(scope="module")
def amber():
    import paper_1811_04165_amd as amber
    return amber


def _small_space(amber, reduced=True):
    wl = workloads.small()
    g = wl.geom
    _, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    widths = (1, 4)
    sp = amber.default_space(info, widths, wl.n_out)
    if reduced:
        sp.set_gene_values(0, [64, 256, 1024])
        sp.set_gene_values(1, [4, 16, 32])
        sp.set_gene_values(2, [1, 4, 16])
        sp.set_gene_values(3, [2, 8, 32])
        sp.set_gene_values(4, [1, 2])
        sp.set_gene_values(5, [0, 1])
        sp.set_gene_values(6, [64, 256])
        sp.set_gene_values(7, [1, 8])
        sp.set_gene_values(8, [2, 4])
    return sp, info, widths


def _tiles_key(t, n_w):
    return (t.threads_per_dm, t.samples_per_thread, t.dms_per_block, t.channel_unroll, t.dms_per_thread,
            t.direct_reads, t.snr_threads) + tuple(t.boxcar_step[k] for k in range(n_w))


def _all_valid(amber, sp, widths):
    out = []
    genes = [sp.gene_values(i) for i in range(sp.n_genes)]
    for combo in itertools.product(*genes):
        t = amber.make_tiles(threads_per_dm=combo[0], samples_per_thread=combo[1], dms_per_block=combo[2],
                             channel_unroll=combo[3], dms_per_thread=combo[4], direct_reads=combo[5],
                             snr_threads=combo[6], boxcar_step=list(combo[7:]))
        try:
            amber.validate_tiles(t, sp.info, len(widths))
        except amber.AmberError:
            continue
        out.append(combo)
    return out


def test_default_space_and_size(amber):
    sp, info, widths = _small_space(amber, reduced=False)
    assert sp.n_genes == 7 + len(widths)
    assert sp.gene_values(1) == [4, 8, 16, 32] and sp.gene_values(4) == [1, 2] and sp.gene_values(5) == [0, 1]
    # widths up to 64 (at most 8): their fused kernel has no step gene
    assert sp.gene_values(7) == [8] and sp.gene_values(8) == [8]
    wide = amber.default_space(info, (1, 128), 8192)
    assert wide.gene_values(7) == [1, 2, 4, 8] and wide.gene_values(8) == [1, 2, 4, 8]
    many = amber.default_space(info, tuple(range(1, 10)), 8192)
    assert all(many.gene_values(7 + k) == [1, 2, 4, 8] for k in range(9))
    n = amber.space_size(sp)
    assert 0 < n <= 5 * 4 * 5 * 6 * 2 * 2 * 5 * 16
    spr, _, _ = _small_space(amber)
    assert amber.space_size(spr) == len(_all_valid(amber, spr, widths))


def test_exhaustive_returns_argmin(amber):
    sp, info, widths = _small_space(amber)
    valid = _all_valid(amber, sp, widths)
    rng = np.random.default_rng(0)
    table = {c: float(rng.uniform(1e-4, 1e-3)) for c in valid}
    seen = []

    def fit(t):
        k = _tiles_key(t, len(widths))
        seen.append(k)
        return table[k]

    res = amber.search_tiles(sp, amber.tune_params("exhaustive"), fit)
    best = min(table, key=table.get)
    assert _tiles_key(res.best, len(widths)) == best
    assert res.best_time_s == pytest.approx(table[best])
    assert res.n_evals == len(valid) == len(set(seen)) and res.space_size == len(valid)
    # a cap below the space size is refused
    with pytest.raises(amber.AmberError):
        amber.search_tiles(sp, amber.tune_params("exhaustive", max_evals=len(valid) - 1), fit)


def _smooth(target, n_w):
    def fit(t):
        # direct_reads (0 or 1) enters as 1 + value so that its log is defined
        vals = [t.threads_per_dm, t.samples_per_thread, t.dms_per_block, t.channel_unroll, t.dms_per_thread,
                1 + t.direct_reads, t.snr_threads] + [t.boxcar_step[k] for k in range(n_w)]
        return 1e-4 * (1.0 + sum((math.log2(v) - math.log2(g)) ** 2 for v, g in zip(vals, target)))
    return fit


def test_ga_valid_offspring_deterministic_and_converging(amber, tmp_path):
    sp, info, widths = _small_space(amber, reduced=False)
    # the operators on a space with step genes (the default space gives the
    # widths 1 and 4 a single step: their kernel has no such gene)
    sp.set_gene_values(7, [1, 2, 4, 8])
    sp.set_gene_values(8, [1, 2, 4, 8])
    target = (64, 8, 16, 16, 2, 1, 256, 4, 2)
    smooth = _smooth(target, len(widths))

    def fit(t):
        amber.validate_tiles(t, sp.info, len(widths))   # every evaluated configuration is valid
        return smooth(t)

    log = tmp_path / "ga.jsonl"
    r1 = amber.search_tiles(sp, amber.tune_params("ga", seed=7), fit, log_path=str(log))
    r2 = amber.search_tiles(sp, amber.tune_params("ga", seed=7), fit)
    assert _tiles_key(r1.best, 2) == _tiles_key(r2.best, 2) and r1.n_evals == r2.n_evals
    assert r1.n_evals <= 32 * 41
    # the smooth landscape's optimum (valid by construction) is found or nearly
    assert r1.best_time_s <= smooth(amber.make_tiles(threads_per_dm=64, samples_per_thread=8, dms_per_block=16,
                                                     channel_unroll=16, dms_per_thread=2, direct_reads=0,
                                                     snr_threads=256, boxcar_step=[4, 2])) * 3.0
    lines = [json.loads(l) for l in log.read_text().splitlines()]
    final = lines.pop()
    assert [l["generation"] for l in lines] == list(range(41))
    # the final population: 32 valid individuals, the best of them the search's best
    assert len(final["final_population"]) == len(final["fitness"]) == 32
    for genes, f in zip(final["final_population"], final["fitness"]):
        t = amber.make_tiles(threads_per_dm=genes[0], samples_per_thread=genes[1], dms_per_block=genes[2],
                             channel_unroll=genes[3], dms_per_thread=genes[4], direct_reads=genes[5],
                             snr_threads=genes[6], boxcar_step=genes[7:])
        amber.validate_tiles(t, sp.info, len(widths))
        assert f == pytest.approx(smooth(t), rel=1e-6)
    assert min(final["fitness"]) == pytest.approx(r1.best_time_s, rel=1e-6)
    bests = [l["best_time_s"] for l in lines]
    assert all(b2 <= b1 for b1, b2 in zip(bests, bests[1:]))
    # one-point crossover also runs and stays valid
    r3 = amber.search_tiles(sp, amber.tune_params("ga", seed=3, crossover=1, generations=10), fit)
    assert r3.n_evals > 0


def test_failures_and_timeouts_never_selected(amber):
    sp, info, widths = _small_space(amber)

    def fit(t):
        if t.channel_unroll == 32:
            return None                   # a failing configuration that would be "fastest"
        if t.samples_per_thread == 4:
            return 5.0                    # slower than eval_timeout_s: treated as a failure
        return 1e-3 / t.channel_unroll

    for kind, kw in (("ga", {}), ("exhaustive", {}), ("random", {"max_evals": 50})):
        res = amber.search_tiles(sp, amber.tune_params(kind, eval_timeout_s=1.0, **kw), fit)
        assert res.best.channel_unroll != 32 and res.best.samples_per_thread != 4
        assert res.n_failed > 0 and math.isfinite(res.best_time_s)


def test_random_search_budget(amber):
    sp, info, widths = _small_space(amber, reduced=False)
    calls = []

    def fit(t):
        calls.append(_tiles_key(t, len(widths)))
        return 1e-3

    res = amber.search_tiles(sp, amber.tune_params("random", max_evals=200, seed=5), fit)
    assert res.n_evals == 200 == len(calls) == len(set(calls))
    with pytest.raises(amber.AmberError):
        amber.search_tiles(sp, amber.tune_params("random", max_evals=0), fit)


def test_per_kernel_search_solves_separable_landscape(amber):
    sp, info, widths = _small_space(amber)
    valid = _all_valid(amber, sp, widths)
    rng = np.random.default_rng(1)
    k1 = amber.genes.AMBER_GENES_K1       # the dedispersion kernel's genes come first
    a = {c[:k1]: float(rng.uniform(1, 2)) for c in valid}
    b = {c[k1:]: float(rng.uniform(0, 1)) for c in valid}

    def fit(t):
        k = _tiles_key(t, len(widths))
        return 1e-3 * (a[k[:k1]] + b[k[k1:]])

    res = amber.search_tiles(sp, amber.tune_params("per_kernel"), fit)
    best = min(valid, key=lambda c: a[c[:k1]] + b[c[k1:]])
    assert _tiles_key(res.best, len(widths)) == best
    assert res.n_evals < len(valid)


def test_ga_seeded_with_the_default(amber):
    """seed_default puts the library's default configuration into the initial
    population (elitism then keeps it unless something beats it); without it,
    or when a default value is missing from its gene array, the population is
    random."""
    sp, info, widths = _small_space(amber, reduced=False)
    n_w = len(widths)
    key_d = _tiles_key(amber.default_tiles(), n_w)

    def fit(t):
        return 1e-4 if _tiles_key(t, n_w) == key_d else 2e-4

    r = amber.search_tiles(sp, amber.tune_params("ga", pop=2, generations=0, seed_default=1), fit)
    assert _tiles_key(r.best, n_w) == key_d and r.best_time_s == pytest.approx(1e-4)
    r0 = amber.search_tiles(sp, amber.tune_params("ga", pop=2, generations=0, seed=1), fit)
    assert r0.best_time_s == pytest.approx(2e-4)
    # the default's snr_threads (128) is not in the reduced space: random start, no error
    spr, _, _ = _small_space(amber)
    r1 = amber.search_tiles(spr, amber.tune_params("ga", pop=4, generations=1, seed_default=1), fit)
    assert r1.n_evals > 0 and r1.best_time_s == pytest.approx(2e-4)


def test_ga_restart_on_stagnation(amber, tmp_path):
    """restart_after: after that many generations without a better best, all
    but the best individual are replaced by fresh random ones.  Deterministic
    under its seed, the best never gets worse, the log counts the restarts."""
    sp, info, widths = _small_space(amber, reduced=False)
    smooth = _smooth((64, 8, 16, 16, 2, 1, 256, 8, 8), len(widths))

    def fit(t):
        amber.validate_tiles(t, sp.info, len(widths))
        return smooth(t)

    with pytest.raises(amber.AmberError):
        amber.search_tiles(sp, amber.tune_params("ga", seed=3, restart_after=-1), fit)
    log = tmp_path / "restart.jsonl"
    p = amber.tune_params("ga", seed=3, restart_after=2, pop=8, generations=30)
    r1 = amber.search_tiles(sp, p, fit, log_path=str(log))
    r2 = amber.search_tiles(sp, p, fit)
    assert _tiles_key(r1.best, 2) == _tiles_key(r2.best, 2) and r1.n_evals == r2.n_evals
    lines = [json.loads(l) for l in log.read_text().splitlines()][:-1]
    assert lines[-1]["restarts"] >= 1
    bests = [l["best_time_s"] for l in lines]
    assert all(b2 <= b1 for b1, b2 in zip(bests, bests[1:]))
    # restarts spend evaluations on fresh genomes: more than the paper's form
    r0 = amber.search_tiles(sp, amber.tune_params("ga", seed=3, pop=8, generations=30), fit)
    assert r1.n_evals > r0.n_evals


def test_retime_top_corrects_a_lucky_measurement(amber, tmp_path):
    """retime_top: a configuration whose first measurement was lucky (0.9 of
    its true time) wins the search; re-timing the best few picks the truly
    fastest one instead, logs the re-timed medians and counts the runs."""
    sp, info, widths = _small_space(amber)
    valid = _all_valid(amber, sp, widths)
    truth = {c: 1e-4 * (1.0 + 0.01 * k) for k, c in enumerate(valid)}   # valid[0] is the fastest
    lucky = valid[1]
    calls = {}

    def fit(t):
        c = _tiles_key(t, len(widths))
        calls[c] = calls.get(c, 0) + 1
        v = truth[c]
        return 0.9 * v if (c == lucky and calls[c] == 1) else v

    plain = amber.search_tiles(sp, amber.tune_params("exhaustive"), fit)
    assert _tiles_key(plain.best, len(widths)) == lucky
    calls.clear()
    log = tmp_path / "retime.jsonl"
    r = amber.search_tiles(sp, amber.tune_params("exhaustive", retime_top=4, retime_runs=3), fit, log_path=str(log))
    assert _tiles_key(r.best, len(widths)) == valid[0]
    assert r.best_time_s == pytest.approx(truth[valid[0]])
    assert r.n_evals == len(valid) + 4 * 3
    rec = [json.loads(l) for l in log.read_text().splitlines() if "retime" in l][-1]["retime"]
    assert len(rec) == 4 and rec[0]["search_s"] == pytest.approx(0.9 * truth[lucky])
    with pytest.raises(amber.AmberError):
        amber.search_tiles(sp, amber.tune_params("ga", retime_top=2, retime_runs=0), fit)
