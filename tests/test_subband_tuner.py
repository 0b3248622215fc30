"""The tile search over the subband pipeline (step one's dedispersion genes,
step two's, and the boxcar / S/N genes: three kernels), driven by fake
fitness landscapes on the CPU.

As for the one-step search, there is no numeric oracle for a search whose
fitness is a timing: these tests pin the contracts.  Every evaluated pair of
tiles is one the library accepts for both steps (checked through the library's
own planning: a call with n_out = 0 plans and launches nothing), exhaustive
search returns the argmin and counts the space, results are deterministic
under a seed, the GA's best never gets worse, and per-kernel brute force
solves a landscape that is a sum over the three kernels.
"""
import ctypes
import itertools
import json
import zlib

import numpy as np
import pytest

import workloads

GRID = (16, 16, 0.0, 8.0, 8, 0.0, 1.0)      # 256 channels in 16 subbands; 16 coarse x 8 fine DMs
WIDTHS = (1, 4)
N_OUT = 4000


@pytest.fixture(scope="module")
def amber():
    import paper_1811_04165_amd as amber
    return amber


def _space(amber, reduced=True):
    g = workloads.small().geom
    _, _, info = amber.subband_delay_tables(g.freqs(), g.t_samp_s, *GRID)
    sp = amber.default_subband_space(info, WIDTHS, N_OUT)
    if reduced:
        G = amber.genes
        for i, vals in enumerate(([64, 128], [8, 16], [4, 8], [8, 16], [1, 2],        # step one
                                  [64], [8, 16], [4, 8], [8, 16],                     # step two
                                  [256], [1, 4], [1, 4])):                            # boxcar / S/N
            sp.set_gene_values(i, vals)
        assert G.SB_GENE_STEP2 == 5 and G.SB_GENE_SNR_THREADS == 9 and G.SB_GENE_BOXCAR0 == 10
    return sp, info


def _key(t1, t2, n_w=2):
    return (t1.threads_per_dm, t1.samples_per_thread, t1.dms_per_block, t1.channel_unroll, t1.dms_per_thread,
            t2.threads_per_dm, t2.samples_per_thread, t2.dms_per_block, t2.channel_unroll, t1.snr_threads) + \
        tuple(t1.boxcar_step[k] for k in range(n_w))


def _accepted(amber, info, t1, t2):
    """The library's own verdict on a pair of step tiles (n_out = 0: plans, launches nothing)."""
    from paper_1811_04165_amd import _lib
    p = ctypes.c_void_p(0x1000)
    rc = _lib.load().amber_subband_dedisperse(p, p, ctypes.byref(info), p, 1 << 20, info.max_delay + 10, p, 1 << 16,
                                              p, 16, 0, None, ctypes.byref(t1), ctypes.byref(t2), None)
    return rc == 0


def _table(key):
    """A deterministic pseudo-random fitness per configuration."""
    return 1e-4 * (1.0 + (zlib.crc32(repr(key).encode()) % 100000) / 1000.0)


def test_default_space(amber):
    sp, info = _space(amber, reduced=False)
    assert sp.n_genes == 10 + len(WIDTHS)
    assert sp.gene_values(4) == [1, 2] and sp.gene_values(6) == [8, 16]
    assert 0 < amber.subband_space_size(sp)


def test_exhaustive_returns_argmin_and_counts_the_space(amber):
    sp, info = _space(amber)
    seen = {}

    def fit(t1, t2):
        assert _accepted(amber, info, t1, t2)
        k = _key(t1, t2)
        seen[k] = _table(k)
        return seen[k]

    res = amber.search_subband_tiles(sp, amber.tune_params("exhaustive"), fit)
    assert res.n_evals == len(seen) == res.space_size == amber.subband_space_size(sp)
    best = min(seen, key=seen.get)
    assert _key(res.step1, res.step2) == best and res.best_time_s == pytest.approx(seen[best])
    # every valid configuration of the reduced space was seen: enumerate it independently
    genes = [sp.gene_values(i) for i in range(sp.n_genes)]
    valid = 0
    for combo in itertools.product(*genes):
        t1 = amber.make_tiles(threads_per_dm=combo[0], samples_per_thread=combo[1], dms_per_block=combo[2],
                              channel_unroll=combo[3], dms_per_thread=combo[4], snr_threads=combo[9],
                              boxcar_step=list(combo[10:]))
        t2 = amber.make_tiles(threads_per_dm=combo[5], samples_per_thread=combo[6], dms_per_block=combo[7],
                              channel_unroll=combo[8], dms_per_thread=1, snr_threads=combo[9],
                              boxcar_step=list(combo[10:]))
        valid += _accepted(amber, info, t1, t2)     # boxcar genes of this space are always valid
    assert valid == res.n_evals


def test_ga_deterministic_valid_and_monotone(amber, tmp_path):
    sp, info = _space(amber, reduced=False)
    target = (64, 16, 8, 8, 2, 128, 16, 8, 8, 256, 4, 2)

    def fit(t1, t2):
        assert _accepted(amber, info, t1, t2)
        return 1e-4 * (1 + sum((np.log2(v) - np.log2(g)) ** 2 for v, g in zip(_key(t1, t2), target)))

    log = tmp_path / "sb.jsonl"
    p = amber.tune_params("ga", seed=11, generations=20)
    r1 = amber.search_subband_tiles(sp, p, fit, log_path=str(log))
    r2 = amber.search_subband_tiles(sp, p, fit)
    assert _key(r1.step1, r1.step2) == _key(r2.step1, r2.step2) and r1.n_evals == r2.n_evals
    lines = [json.loads(l) for l in log.read_text().splitlines()]
    final = lines.pop()
    assert len(final["final_population"]) == 32 and all(len(g) == sp.n_genes for g in final["final_population"])
    bests = [l["best_time_s"] for l in lines]
    assert [l["generation"] for l in lines] == list(range(21))
    assert all(b2 <= b1 for b1, b2 in zip(bests, bests[1:]))
    assert set(lines[-1]["best"]) == {"step1", "step2", "box"}
    # one-point crossover runs as well
    amber.search_subband_tiles(sp, amber.tune_params("ga", seed=3, crossover=1, generations=5), fit)


def test_per_kernel_solves_three_kernel_separable_landscape(amber):
    sp, info = _space(amber)
    rng = np.random.default_rng(5)
    a, b, c = {}, {}, {}

    def part(d, k):
        if k not in d:
            d[k] = float(rng.uniform(0.1, 1.0))
        return d[k]

    def fit(t1, t2):
        k = _key(t1, t2)
        return 1e-3 * (part(a, k[:5]) + part(b, k[5:9]) + part(c, k[9:]))

    exh = amber.search_subband_tiles(sp, amber.tune_params("exhaustive"), fit)
    pk = amber.search_subband_tiles(sp, amber.tune_params("per_kernel"), fit)
    assert _key(pk.step1, pk.step2) == _key(exh.step1, exh.step2)
    assert pk.n_evals < exh.n_evals


def test_random_search_budget_and_rejects(amber):
    sp, info = _space(amber, reduced=False)
    calls = []
    res = amber.search_subband_tiles(sp, amber.tune_params("random", max_evals=60, seed=2),
                                     lambda t1, t2: calls.append(_key(t1, t2)) or 1e-3)
    assert res.n_evals == 60 == len(set(calls))
    bad = amber.default_subband_space(info, WIDTHS, N_OUT)
    bad.n_genes = 7
    with pytest.raises(amber.AmberError):
        amber.subband_space_size(bad)
