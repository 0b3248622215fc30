#!/usr/bin/env python3
"""Throughput of the single-pulse search hot path on one MI355X.

One step = one pass of the device hot path over one 1-s beam resident in HBM:
brute-force dedispersion of 1536 channels x 2048 DM trials x 12208 samples,
then sliding boxcars of widths 1..64 and the per-(DM, width) S/N peak (fused
kernel).  The FP64 delay table is built once per geometry on the host, before
the timed region.

Prints one JSON line: DM-trial*samples/s, the roofline position of the
dominant kernel (dedispersion, integer-ALU bound) from HIP events around its
launches, the CPU oracle timed on a bounded sample of the same workload, and
(after the timed region) the wall time of one GA tile search and the p50/p99
chunk latency of a few seconds of serving.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published / derived peaks
HBM_PEAK_GBS = 8000.0
# 32-bit VALU issue: 256 CUs x 4 SIMDs x 16 lanes = 64 lane-ops per clock per
# CU at 2.4 GHz = 39.3 T lane-ops/s (the published FP32 vector rate,
# 157.3 TFLOP/s, is this times two for packed FP32 and two for an FMA).  The
# dedispersion sums live in 16-bit halves, two per 32-bit add
# -> 78.6 T sample-additions/s.  Measured (bench.py --peaks): v_add_u32
# 1.11 x this issue rate, three-operand and packed forms 0.85-0.90 x.
VALU_LANES_PER_CLK = 64
ALU_PEAK_TOPS = 256 * VALU_LANES_PER_CLK * 2.4e9 * 2 / 1e12

# LDS reads: 256 B/clk/CU (CDNA4 doubled CDNA3's 128) = 157.3 TB/s; measured
# ds_read_b128 209 B/clk/CU, ds_read_b64 (the dedispersion kernel's sums) 194,
# the 32-bit forms (ds_read_b32, ds_read2st64_b32) 113-120
LDS_PEAK_TBS = 256 * 256 * 2.4e9 / 1e12

METRIC = "DM-trial·samples/s per GPU + % HBM roofline; GA tune time; p99 chunk latency"
UNIT = "DM-trial·samples/s"
PMC_FILE = os.path.join(ROOT, "profiles", "dedisperse_beam_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1811_04165_amd", "csrc", "dedisperse.hip")


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(launch_ops: float):
    """HBM bytes per dedispersion launch from the committed rocprofv3 counter
    runs, or None when absent or taken on a different kernel source."""
    try:
        with open(PMC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha") != kernel_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_stages(d, x, n_in, wl, threads: int):
    """One oracle pass over the rows of `d`, timed per stage."""
    import oracle
    t0 = time.perf_counter()
    dd = oracle.dedisperse(d, x, n_in, wl.n_out, threads)
    t1 = time.perf_counter()
    box = [oracle.boxcar(dd, w, threads) for w in wl.widths]
    t2 = time.perf_counter()
    for b in box:
        oracle.snr(b, threads)
    t3 = time.perf_counter()
    return {"dedisperse_s": t1 - t0, "integrate_s": t2 - t1, "snr_s": t3 - t2, "total_s": t3 - t0}


def cpu_baseline(x, n_in, wl, budget_rows: int):
    """The oracle (unchanged) on the first `budget_rows` DM trials of the same
    beam, timed per stage: median of five passes on every host core, then one
    pass on a single core over a quarter of those trials.  The delay table
    (host FP64, negligible) is built outside the timed passes."""
    import oracle
    g = wl.geom
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    d, _ = oracle.delay_table(g.freqs(), g.t_samp_s, budget_rows, g.dm_first, g.dm_step)
    runs = [_oracle_stages(d, x, n_in, wl, threads) for _ in range(5)]
    med = {k: statistics.median(r[k] for r in runs) for k in runs[0]}
    rows1 = max(1, budget_rows // 4)
    one = _oracle_stages(d[:rows1], x, n_in, wl, 1)
    return {"value": budget_rows * wl.n_out / med["total_s"], "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": "first %d of %d DM trials of the 1536-ch beam (all %d samples, widths %s), median of 5 "
                      "passes (%.1f s each); single core: first %d trials, one pass (%.1f s)" % (
                          budget_rows, g.n_dm, wl.n_out, list(wl.widths), med["total_s"], rows1, one["total_s"]),
            "cpu_model": _cpu_model(), "compiler": "gcc " + " ".join(oracle.BUILD_FLAGS), "stages_s": med,
            "single_core": {"value": rows1 * wl.n_out / one["total_s"], "cores": 1, "stages_s": one}}


def _point_space(search, tiles):
    """A search space holding the one configuration `tiles`."""
    import paper_1811_04165_amd as amber
    G = amber.genes
    sp = amber.default_space(search.info, search.widths, search.n_out)
    vals = [tiles.threads_per_dm, tiles.samples_per_thread, tiles.dms_per_block, tiles.channel_unroll,
            tiles.dms_per_thread, tiles.direct_reads, tiles.snr_threads]
    for gene, v in zip([G.GENE_THREADS_PER_DM, G.GENE_SAMPLES_PER_THREAD, G.GENE_DMS_PER_BLOCK,
                        G.GENE_CHANNEL_UNROLL, G.GENE_DMS_PER_THREAD, G.GENE_DIRECT_READS, G.GENE_SNR_THREADS], vals):
        sp.set_gene_values(gene, [v])
    for k in range(len(search.widths)):
        sp.set_gene_values(G.GENE_BOXCAR0 + k, [tiles.boxcar_step[k]])
    return sp


def time_configs(search, x, configs, reps: int):
    """Median GPU time of dedisperse + fused boxcar/S/N for each configuration,
    measured as the searches measure fitness (the library's timer: HIP events
    around the two launches made from native code; one measurement is the
    median of 3 back-to-back runs after an untimed one, so the configuration
    runs with its own code and data warm, as in a pipeline), `reps` rounds,
    the configurations round robin within a round so drifts hit all alike.
    (Events around launches made from Python would add the interpreter's
    per-call time, which is larger than these kernels.)"""
    import paper_1811_04165_amd as amber
    spaces = [_point_space(search, t) for t in configs]
    params = amber.tune_params("exhaustive", warmup=1, reps=3)
    bufs = (search.dd, search.snr, search.peak)
    times = [[] for _ in configs]
    gc.collect()
    for _ in range(reps):
        for k, sp in enumerate(spaces):
            times[k].append(amber.tune(sp, search.delays, x, search.n_in, params, buffers=bufs).best_time_s)
    return [statistics.median(v) for v in times]


def _small_tune_setup():
    """The tile-search workload (256 channels, 128 DM trials) on the device and
    its default search space (the boxcar / S/N kernel's gene is its thread
    count: for these widths it has no per-width step)."""
    import torch
    import paper_1811_04165_amd as amber
    import workloads
    wl = workloads.small()
    g = wl.geom
    search = amber.Search(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step, wl.n_out, wl.widths)
    x_host, n_in = workloads.make_input(wl, search.delays_host, search.info.max_delay)
    x = torch.from_numpy(x_host).cuda()
    sp = amber.default_space(search.info, wl.widths, wl.n_out)
    return wl, search, x, n_in, sp, (search.dd, search.snr, search.peak)


def ga_tune_summary():
    """One GA search (population 32, 40 generations, seed 1) on the tile-search
    workload: its wall time and evaluations, and its best tiles re-timed
    interleaved with the library's default tiles."""
    import paper_1811_04165_amd as amber
    wl, search, x, n_in, sp, bufs = _small_tune_setup()
    r = amber.tune(sp, search.delays, x, n_in, amber.tune_params("ga", seed=1), buffers=bufs)
    t_ga, t_def = time_configs(search, x, [r.best, amber.auto_tiles(search.info, search.n_out)], reps=30)
    return {"workload": wl.name, "search": "ga pop 32 x 40 generations, seed 1", "space_size": amber.space_size(sp),
            "wall_s": r.wall_s, "evals": r.n_evals, "best_s": t_ga, "default_tiles_s": t_def,
            "best": r.as_dict(len(wl.widths))["best"]}


def serve_summary(seconds: float = 5.0, warmup_s: float = 1.0, over_rate: float = 1600.0):
    """The streaming service at the workload's rate (400 chunks/s from 40
    beams) with continuous batching and, beside it, the plain per-chunk path
    (one chunk at a time: no fusion, no overlap), briefly; then both at
    `over_rate` chunks/s for 3 s, past the plain path's capacity."""
    by = serve_report(40, seconds, warmup_s, [400.0, over_rate])["serve"]["by_rate"]

    def pick(r):
        return {"chunks_per_s": r["chunks_per_s"], "value": r["value"], "latency_ms": r["latency_ms"]}
    return {"offered_chunks_per_s": 400.0, "seconds": seconds, "warmup_s": warmup_s,
            "chunks_per_s": by["400.0"]["served"]["chunks_per_s"], "value": by["400.0"]["served"]["value"],
            "latency_ms": by["400.0"]["served"]["latency_ms"],
            "plain": pick(by["400.0"]["one_at_a_time"]),
            "over_capacity": {"offered_chunks_per_s": over_rate, "seconds": min(seconds, 3.0),
                              "served": pick(by[str(over_rate)]["served"]),
                              "plain": pick(by[str(over_rate)]["one_at_a_time"])}}


def tune_report(seeds: int, log_path=None):
    """GA (several seeds) vs exhaustive vs random (same budget as each GA run)
    vs per-kernel brute force, on the 256-channel / 128-DM workload, with the
    finalists re-timed interleaved."""
    import paper_1811_04165_amd as amber
    wl, search, x, n_in, sp, bufs = _small_tune_setup()
    G = amber.genes
    out = {"workload": wl.name, "space_size": amber.space_size(sp), "genes": {
        "threads_per_dm": sp.gene_values(G.GENE_THREADS_PER_DM),
        "samples_per_thread": sp.gene_values(G.GENE_SAMPLES_PER_THREAD),
        "dms_per_block": sp.gene_values(G.GENE_DMS_PER_BLOCK), "channel_unroll": sp.gene_values(G.GENE_CHANNEL_UNROLL),
        "dms_per_thread": sp.gene_values(G.GENE_DMS_PER_THREAD),
        "direct_reads": sp.gene_values(G.GENE_DIRECT_READS), "snr_threads": sp.gene_values(G.GENE_SNR_THREADS),
        "boxcar_step": sp.gene_values(G.GENE_BOXCAR0)}}

    def run(kind, **kw):
        print("[bench] tune %s %s" % (kind, kw), file=sys.stderr, flush=True)
        r = amber.tune(sp, search.delays, x, n_in, amber.tune_params(kind, **kw), log_path=log_path, buffers=bufs)
        return r

    ga = [run("ga", seed=s) for s in range(1, seeds + 1)]
    gas = [run("ga", seed=s, seed_default=1) for s in range(1, seeds + 1)]   # initial population holds the defaults
    gar = {ra: [run("ga", seed=s, restart_after=ra) for s in range(1, seeds + 1)] for ra in GA_RESTART_SWEEP}
    # the search's best GA_RETIME[0] configurations re-timed GA_RETIME[1] times each at its end
    gat = [run("ga", seed=s, retime_top=GA_RETIME[0], retime_runs=GA_RETIME[1]) for s in range(1, seeds + 1)]
    gart = [run("ga", seed=s, restart_after=GA_RESTART_AFTER, retime_top=GA_RETIME[0], retime_runs=GA_RETIME[1])
            for s in range(1, seeds + 1)]
    rnd = [run("random", seed=100 + s, max_evals=ga[s - 1].n_evals) for s in range(1, seeds + 1)]
    pk = run("per_kernel")
    ex = run("exhaustive")
    finalists = [r.best for r in ga] + [r.best for r in rnd] + [pk.best, ex.best] + [r.best for r in gas] + \
        [r.best for ra in GA_RESTART_SWEEP for r in gar[ra]] + [r.best for r in gat] + [r.best for r in gart]
    print("[bench] interleaved re-timing of %d finalists" % len(finalists), file=sys.stderr, flush=True)
    t = time_configs(search, x, finalists, reps=100)
    n = seeds
    t_ga, t_rnd, t_pk, t_ex = t[:n], t[n:2 * n], t[2 * n], t[2 * n + 1]
    t_gas = t[2 * n + 2:3 * n + 2]
    t_gar = {ra: t[(3 + k) * n + 2:(4 + k) * n + 2] for k, ra in enumerate(GA_RESTART_SWEEP)}
    k0 = (3 + len(GA_RESTART_SWEEP)) * n + 2
    t_gat, t_gart = t[k0:k0 + n], t[k0 + n:k0 + 2 * n]
    nw = len(wl.widths)
    out.update({
        "retimed_s": {"ga": t_ga, "random": t_rnd, "per_kernel": t_pk, "exhaustive": t_ex, "ga_seeded": t_gas,
                      "ga_restart": {str(ra): t_gar[ra] for ra in GA_RESTART_SWEEP}, "ga_retime": t_gat,
                      "ga_restart_retime": t_gart},
        "ga_retime": {"retime_top": GA_RETIME[0], "retime_runs": GA_RETIME[1],
                      "median_over_exhaustive": statistics.median(t_gat) / t_ex, "worst_over_exhaustive": max(t_gat) / t_ex,
                      "evals_median": statistics.median([r.n_evals for r in gat]),
                      "wall_s_median": statistics.median([r.wall_s for r in gat]),
                      "with_restart_after": GA_RESTART_AFTER,
                      "with_restart_median_over_exhaustive": statistics.median(t_gart) / t_ex,
                      "with_restart_worst_over_exhaustive": max(t_gart) / t_ex,
                      "with_restart_evals_median": statistics.median([r.n_evals for r in gart])},
        "ga_median_over_exhaustive": statistics.median(t_ga) / t_ex,
        "ga_worst_over_exhaustive": max(t_ga) / t_ex,
        "ga_seeded_median_over_exhaustive": statistics.median(t_gas) / t_ex,
        "ga_seeded_worst_over_exhaustive": max(t_gas) / t_ex,
        "ga_seeded_evals_median": statistics.median([r.n_evals for r in gas]),
        "ga_restart": {str(ra): {"median_over_exhaustive": statistics.median(t_gar[ra]) / t_ex,
                                 "worst_over_exhaustive": max(t_gar[ra]) / t_ex,
                                 "evals_median": statistics.median([r.n_evals for r in gar[ra]]),
                                 "wall_s_median": statistics.median([r.wall_s for r in gar[ra]])}
                       for ra in GA_RESTART_SWEEP},
        "random_median_over_exhaustive": statistics.median(t_rnd) / t_ex,
        "per_kernel_over_exhaustive": t_pk / t_ex,
        "cost": {"ga_evals_median": statistics.median([r.n_evals for r in ga]),
                 "ga_wall_s_median": statistics.median([r.wall_s for r in ga]),
                 "random_evals_median": statistics.median([r.n_evals for r in rnd]),
                 "per_kernel_evals": pk.n_evals, "per_kernel_wall_s": pk.wall_s,
                 "exhaustive_evals": ex.n_evals, "exhaustive_wall_s": ex.wall_s},
        "ga_cost_fraction_of_exhaustive": statistics.median([r.wall_s for r in ga]) / ex.wall_s,
        "best": {"ga_seed1": ga[0].as_dict(nw)["best"], "exhaustive": ex.as_dict(nw)["best"],
                 "per_kernel": pk.as_dict(nw)["best"]},
        "default_tiles_s": time_configs(search, x, [amber.auto_tiles(search.info, search.n_out)], reps=100)[0],
    })
    return {"metric": "GA tune time", "unit": "s", "value": out["cost"]["ga_wall_s_median"], "tune": out}


def batched_report(n_beams: int, steps: int, warmup: int):
    """Uneven beams (channels 384/768/1536, 4096-24576 samples, 512/1024/2048
    DM trials): per-beam launches with GA-picked tiles per shape class vs one
    batch (eager, and replayed as a HIP graph) with three tile choices: the
    per-class tiles, the automatic tiles, and one tile set for all beams
    picked by the GA with the whole batch's time as fitness.  Both GA
    searches start from a population that holds the library's defaults."""
    import numpy as np
    import torch
    import paper_1811_04165_amd as amber
    import workloads
    wls = workloads.batch_beams(n_beams)
    widths = wls[0].widths
    beams = []
    for k, wl in enumerate(wls):
        g = wl.geom
        d, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
        x, n_in = workloads.make_input(wl, d, info.max_delay)
        beams.append(dict(delays=torch.from_numpy(d).cuda(), info=info, x=torch.from_numpy(x).cuda(), n_in=n_in,
                          n_out=wl.n_out, dd=torch.empty((g.n_dm, wl.n_out), dtype=torch.int32, device="cuda"),
                          snr=torch.empty((len(widths), g.n_dm), dtype=torch.float32, device="cuda"),
                          peak=torch.empty((len(widths), g.n_dm), dtype=torch.int32, device="cuda"),
                          cls=(g.n_chan, g.n_dm), wl=wl))
        print("[bench] beam %d/%d built" % (k + 1, len(wls)), file=sys.stderr, flush=True)
    # GA-picked tiles per shape class, tuned on the class's first beam
    class_tiles, tune_cost = {}, {}
    for b in beams:
        if b["cls"] in class_tiles:
            continue
        sp = amber.default_space(b["info"], widths, b["n_out"])
        print("[bench] tuning class %s" % (b["cls"],), file=sys.stderr, flush=True)
        r = amber.tune(sp, b["delays"], b["x"], b["n_in"],
                       amber.tune_params("ga", pop=16, generations=12, seed=1, seed_default=1),
                       buffers=(b["dd"], b["snr"], b["peak"]))
        class_tiles[b["cls"]] = amber.Tiles.from_buffer_copy(r.best)
        tune_cost["%dch-%ddm" % b["cls"]] = {"evals": r.n_evals, "wall_s": r.wall_s, "best_s": r.best_time_s}
    tiles = [class_tiles[b["cls"]] for b in beams]

    def per_beam():
        for b, t in zip(beams, tiles):
            amber.dedisperse(b["delays"], b["info"], b["x"], b["n_in"], b["n_out"], t, out=b["dd"])
            amber.integrate_snr(b["dd"], b["n_out"], widths, t, out=(b["snr"], b["peak"]))

    stream = torch.cuda.Stream()

    def timed(fn, s=None):
        s = s or torch.cuda.current_stream()
        with torch.cuda.stream(s):
            for _ in range(warmup):
                fn()
            s.synchronize()
            gc.collect()
            a, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            a.record(s)
            for _ in range(steps):
                fn()
            b_.record(s)
            s.synchronize()
            wall = time.perf_counter() - t0
        return a.elapsed_time(b_) / 1e3 / steps, wall / steps

    # One tile set for every beam, searched by the GA with the whole batch's
    # GPU time as fitness: per-class tuning times each class alone, where its
    # small grid favours small tiles, while in a batch every distinct tile
    # set is a launch of its own with its own tail.
    ref_beam = max(beams, key=lambda b: (b["info"].max_step, b["info"].n_chan))
    sp = amber.default_space(ref_beam["info"], widths, min(b["n_out"] for b in beams))

    def batch_fitness(t):
        try:
            bt = amber.Batch(beams, widths, tiles=[t] * len(beams))
        except amber.AmberError:
            return None                  # not valid for every beam
        try:
            bt.run(stream)
            ts = []
            for _ in range(3):
                a, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                bt.run(stream)
                b_.record(stream)
                b_.synchronize()
                ts.append(a.elapsed_time(b_) / 1e3)
            return statistics.median(ts)
        finally:
            bt.close()

    print("[bench] GA over one tile set for the whole batch", file=sys.stderr, flush=True)
    shared = amber.search_tiles(sp, amber.tune_params("ga", pop=16, generations=12, seed=1, seed_default=1),
                                batch_fitness)
    shared_tiles = amber.Tiles.from_buffer_copy(shared.best)

    gc.disable()  # no collection pauses inside the timed loops
    print("[bench] timing", file=sys.stderr, flush=True)
    t_plain, w_plain = timed(per_beam)
    ref = [(b["dd"].clone(), b["snr"].clone(), b["peak"].clone()) for b in beams]

    def same():
        return all(torch.equal(b["dd"], r[0]) and torch.equal(b["snr"], r[1]) and torch.equal(b["peak"], r[2])
                   for b, r in zip(beams, ref))

    choices = {}
    for name, tl in (("ga_per_class", tiles), ("automatic", None), ("ga_shared", [shared_tiles] * len(beams))):
        print("[bench] batch with %s tiles" % name, file=sys.stderr, flush=True)
        batch = amber.Batch(beams, widths, tiles=tl)
        with torch.cuda.stream(stream):
            batch.capture(stream)
        for b in beams:
            b["dd"].fill_(-1)
            b["snr"].zero_()
        t_batch, w_batch = timed(lambda: batch.run(stream), stream)
        same_eager = same()
        for b in beams:
            b["dd"].fill_(-1)
            b["snr"].zero_()
        t_graph, w_graph = timed(lambda: batch.launch(stream), stream)
        same_graph = same()
        choices[name] = {"eager": {"gpu_s": t_batch, "wall_s": w_batch, "launches": sum(batch.launches())},
                         "graph": {"gpu_s": t_graph, "wall_s": w_graph, "graph_launches": 1},
                         "identical_to_per_beam": {"eager": same_eager, "graph": same_graph}}
        batch.close()
    gc.enable()
    best = min(choices, key=lambda k: choices[k]["graph"]["gpu_s"])
    found = 0
    for b in beams:
        p = b["wl"].pulses[0]
        sn = b["snr"].cpu().numpy()
        found += int(sn[list(widths).index(p.width), p.dm_index] > 8.0)
    samples = sum(b["info"].n_dm * b["n_out"] for b in beams)
    bc = choices[best]
    for c in choices.values():
        c["value"] = samples / c["graph"]["gpu_s"]
    return {"metric": "DM-trial·samples/s per GPU", "unit": UNIT, "value": samples / bc["graph"]["gpu_s"],
            "batched": {
                "workload": "%d uneven beams (channels 384/768/1536, 4096-24576 samples, 512/1024/2048 DM trials)"
                            % len(beams),
                "dm_trial_samples": samples, "classes": len(class_tiles), "tiles": best,
                "per_beam_launches": {"gpu_s": t_plain, "wall_s": w_plain, "value": samples / t_plain,
                                      "launches": 2 * len(beams), "tiles": "ga_per_class"},
                "batch_eager": dict(bc["eager"], value=samples / bc["eager"]["gpu_s"]),
                "batch_graph": dict(bc["graph"], value=samples / bc["graph"]["gpu_s"]),
                "identical_to_per_beam": bc["identical_to_per_beam"],
                "tile_choices": choices,
                "pulses_found": found, "tiles_per_class": {"%dch-%ddm" % k: v.as_dict() for k, v in class_tiles.items()},
                "tune_per_class": tune_cost,
                "tune_shared": {"evals": shared.n_evals, "failed": shared.n_failed, "wall_s": shared.wall_s,
                                "best_s": shared.best_time_s, "tiles": shared_tiles.as_dict()}}}


def serve_report(n_beams: int, seconds: float, warmup_s: float, rates, submitters: int = 4,
                 modes=("served", "one_at_a_time")):
    """Streaming: Poisson arrivals of 0.5-s chunks from beams of 768 ch / 1024
    DM trials and 1536 ch / 2048 DM trials, served with continuous batching
    vs the same service restricted to one chunk at a time (plain per-chunk
    launches: no fusion, no overlap).  Latency runs from a chunk's scheduled
    arrival to its results being on the host."""
    import threading
    import numpy as np
    import paper_1811_04165_amd as amber
    import workloads
    geoms = workloads.stream_geometries(n_beams)
    L = workloads.STREAM_CHUNK
    widths = (1, 2, 4, 8, 16, 32, 64)
    # one seeded noise block per beam shape, 4 chunks long with one pulse per
    # second; beam b reads its chunks from it at a rotated offset
    n_blk, blocks = 4, {}
    for g in geoms:
        key = (g.n_chan, g.n_dm)
        if key in blocks:
            continue
        d, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
        x = workloads.noise(g.n_chan, n_blk * L, n_blk * L, seed=5000 + len(blocks))
        for s_ in range(2):
            workloads.inject(x, d[g.n_dm // 2], t0=1000 + 2 * L * s_, width=8, amp=40)
        blocks[key] = x
        print("[bench] stream block %s built" % (key,), file=sys.stderr, flush=True)

    def run(rate, duration, **cfg):
        arrivals = workloads.poisson_arrivals(n_beams, rate / n_beams, duration, seed=5)
        srv = amber.Server(**cfg)
        for g in geoms:
            srv.add_beam(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step, L, widths)
        done, err = [], []

        def collect(n):
            try:
                for _ in range(n):
                    r = srv.wait(60.0)
                    if r is None:
                        raise RuntimeError("no chunk completed within 60 s")
                    done.append(r)
            except Exception as e:  # reported below
                err.append(e)

        lag = [0.0]
        submit_s = []
        t0 = amber.server_clock() + 0.05

        def submit(part):
            for t, b, seq in part:
                now = amber.server_clock() - t0
                if t > now:
                    time.sleep(t - now)
                else:
                    lag[0] = max(lag[0], now - t)
                g = geoms[b]
                off = ((seq + 3 * b) % n_blk) * L
                a = amber.server_clock()
                srv.submit(b, blocks[(g.n_chan, g.n_dm)][:, off:off + L], tag=seq)
                submit_s.append(amber.server_clock() - a)

        gc.collect()
        gc.disable()  # a collection would stall the submitting threads
        col = threading.Thread(target=collect, args=(len(arrivals),))
        col.start()
        subs = [threading.Thread(target=submit, args=([a for a in arrivals if a[1] % submitters == i],))
                for i in range(submitters)]
        for th in subs:
            th.start()
        for th in subs:
            th.join()
        col.join()
        gc.enable()
        st = srv.stats()
        srv.close()
        if err:
            raise err[0]
        arr = {(b, seq): t for t, b, seq in arrivals}
        meas = [r for r in done if arr[(r["beam"], r["seq"])] >= warmup_s]
        lat = np.array([r["t_done"] - (t0 + arr[(r["beam"], r["seq"])]) for r in meas])
        work = sum(geoms[r["beam"]].n_dm * r["n_out"] for r in meas)
        first = t0 + min(arr[(r["beam"], r["seq"])] for r in meas)
        last = max(r["t_done"] for r in meas)
        bs = np.array([r["batch_size"] for r in meas])
        wait = np.array([r["t_start"] - r["t_submit"] for r in meas])
        run = np.array([r["t_done"] - r["t_start"] for r in meas])

        def pct(v):
            return {"p50": 1e3 * float(np.percentile(v, 50)), "p99": 1e3 * float(np.percentile(v, 99))}
        return {"offered_chunks_per_s": rate, "chunks": len(meas), "value": work / (last - first),
                "chunks_per_s": len(meas) / (last - first),
                "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)), "p99": 1e3 * float(np.percentile(lat, 99)),
                               "max": 1e3 * float(lat.max()), "mean": 1e3 * float(lat.mean())},
                "breakdown_ms": {"submit_call": pct(np.array(submit_s)), "queued": pct(wait),
                                 "launch_to_done": pct(run)},
                "batch_size": {"mean": float(bs.mean()), "max": int(bs.max())},
                "launch_groups": st["batches"], "max_submit_lag_ms": 1e3 * lag[0],
                "memory_peak_bytes": st["memory_peak"]}

    out = {}
    for rate in rates:
        for name, cfg in (("served", dict(max_inflight=64, max_batch=16, n_streams=4)),
                          ("one_at_a_time", dict(max_inflight=1, max_batch=1, n_streams=1))):
            if name not in modes:
                continue
            print("[bench] serve %s at %g chunks/s" % (name, rate), file=sys.stderr, flush=True)
            # points past twice the first rate run briefly: past a path's
            # capacity its backlog holds one pinned staging buffer per queued chunk
            dur = seconds if rate <= 2 * rates[0] else min(seconds, 3.0)
            out.setdefault(str(rate), {})[name] = run(rate, warmup_s + dur, **cfg)
    base = out[str(rates[0])]
    return {"metric": "p99 chunk latency", "unit": "ms", "value": base["served"]["latency_ms"]["p99"],
            "higher_is_better": False,
            "serve": {"workload": "%d beams (768 ch / 1024 DM trials and 1536 ch / 2048 DM trials, alternating), "
                                  "0.5-s chunks of %d samples, widths 1-64, Poisson arrivals" % (n_beams, L),
                      "seconds": seconds, "warmup_s": warmup_s, "submit_threads": submitters, "by_rate": out}}


GA_RESTART_AFTER = 5   # generations without a better best before the GA re-draws its population
GA_RESTART_SWEEP = (3, 5, 8)
GA_RETIME = (8, 5)     # (configurations, runs each) re-timed at the end of a search
GA_STUDY_BASE = dict(pop=20, p_cross=0.8, p_mut=0.1, crossover=0)


def _ga_study_settings():
    """The settings of the paper's studies (Section 4): mutation and crossover
    rates, population size, crossover type, random search; plus the restart
    on stagnation this library adds."""
    settings = [("base (N_pop 20, p_cross 0.8, p_mut 0.1, uniform)", "ga", {})]
    settings += [("p_mut %g" % v, "ga", {"p_mut": v}) for v in (0.01, 0.3, 1.0)]
    settings += [("p_cross %g" % v, "ga", {"p_cross": v}) for v in (0.2, 0.5, 1.0)]
    settings += [("N_pop %d" % v, "ga", {"pop": v}) for v in (30, 50)]
    settings += [("one-point crossover", "ga", {"crossover": 1}), ("random search", "random", {})]
    settings += [("restart after %d stale generations" % GA_RESTART_AFTER, "ga",
                  {"restart_after": GA_RESTART_AFTER})]
    return settings


def ga_study_report(seeds: int):
    """The paper's GA studies (Figs 3-5, App. A) on MI355X: with joint
    on-device fitness (the headline), and replayed on a measured table of
    per-kernel times (a noise-free control in which the kernels cannot
    interact)."""
    dev = ga_study_device(seeds)
    table = ga_study_table(seeds)
    return {"metric": "GA studies (on-device fitness)", "unit": "ratio",
            "value": dev["settings"][0]["retimed_over_bf"]["median"], "higher_is_better": False,
            "ga_study": {"device": dev, "table_replay": table}}


def ga_study_device(seeds: int):
    """The GA studies with joint on-device fitness on the 256-channel / 128-DM
    workload: every evaluation times dedispersion + boxcar/S/N together on the
    GPU (median of 3 runs after a warm-up), over the whole genome (the five
    dedispersion genes and the boxcar / S/N thread count).  T_BF is the
    on-device per-kernel brute force (each kernel's genes searched in turn,
    the paper's Section 2 tuning); every search gets its evaluation budget,
    and the same seeds for every setting.  Each run's best configuration and
    the brute force's are re-timed interleaved, so that the ratios compare
    like with like (a search's own best time is the luckiest of its noisy
    measurements)."""
    import json
    import os
    import tempfile
    import numpy as np
    import paper_1811_04165_amd as amber
    wl, search, x, n_in, sp, bufs = _small_tune_setup()
    G = amber.genes
    cols = [G.GENE_THREADS_PER_DM, G.GENE_SAMPLES_PER_THREAD, G.GENE_DMS_PER_BLOCK, G.GENE_CHANNEL_UNROLL,
            G.GENE_DMS_PER_THREAD, G.GENE_DIRECT_READS, G.GENE_SNR_THREADS]
    names = ["threads_per_dm", "samples_per_thread", "dms_per_block", "channel_unroll", "dms_per_thread",
             "direct_reads", "snr_threads"]

    def key(t):
        return (t.threads_per_dm, t.samples_per_thread, t.dms_per_block, t.channel_unroll, t.dms_per_thread,
                t.direct_reads, t.snr_threads)

    print("[bench] device study: per-kernel brute force", file=sys.stderr, flush=True)
    bf = amber.tune(sp, search.delays, x, n_in, amber.tune_params("per_kernel"), buffers=bufs)
    budget = bf.n_evals
    checkpoints = [c for c in (50, 100, 200, 400, 800) if c < budget] + [budget]
    tmp = tempfile.mkdtemp()
    finalists = {key(bf.best): bf.best}
    runs = []
    for name, kind, kw in _ga_study_settings():
        print("[bench] device study: %s" % name, file=sys.stderr, flush=True)
        p = dict(GA_STUDY_BASE)
        p.update(kw)
        for seed in range(1, seeds + 1):
            log = os.path.join(tmp, "s.jsonl")
            if os.path.exists(log):
                os.remove(log)
            if kind == "ga":
                gens = max(1, budget // p["pop"] - 1)
                r = amber.tune(sp, search.delays, x, n_in, amber.tune_params("ga", seed=seed, generations=gens, **p),
                               log_path=log, buffers=bufs)
            else:
                r = amber.tune(sp, search.delays, x, n_in, amber.tune_params("random", seed=1000 + seed,
                                                                             max_evals=budget),
                               log_path=log, buffers=bufs)
            lines = [json.loads(l) for l in open(log)]
            gen_lines = [l for l in lines if "generation" in l]
            cv = None
            if kind == "ga" and "final_population" in lines[-1]:
                end = np.array(lines[-1]["final_population"], dtype=np.float64)[:, cols]
                mean = end.mean(axis=0)     # direct_reads takes 0 and 1: a population of zeros has c_v 0
                cv = np.where(mean > 0, end.std(axis=0) / np.where(mean > 0, mean, 1.0), 0.0).tolist()
            curve = []
            for c in checkpoints:  # best so far after c evaluations (GA: at generation boundaries)
                seen = [l["best_time_s"] for l in gen_lines if l["evals"] <= c and l["best_time_s"] > 0]
                curve.append(min(seen) / bf.best_time_s if seen else None)
            finalists[key(r.best)] = r.best
            runs.append(dict(setting=name, kind=kind, seed=seed, best=key(r.best), best_s=r.best_time_s,
                             evals=r.n_evals, wall_s=r.wall_s, cv=cv, curve=curve,
                             restarts=gen_lines[-1].get("restarts", 0) if gen_lines else 0))
    keys = list(finalists)
    print("[bench] device study: interleaved re-timing of %d finalists" % len(keys), file=sys.stderr, flush=True)
    times = dict(zip(keys, time_configs(search, x, [finalists[k] for k in keys], reps=15)))
    t_bf = times[key(bf.best)]
    out = {"workload": wl.name, "space_size": amber.space_size(sp), "genes": names,
           "brute_force_per_kernel": {"best": dict(zip(names, key(bf.best))), "evals": budget,
                                      "best_s_own": bf.best_time_s, "best_s_retimed": t_bf},
           "budget_evals": budget, "seeds": seeds, "checkpoints": checkpoints,
           "best_retimed_s": min(times.values()), "settings": []}
    for name, kind, kw in _ga_study_settings():
        rs = [r for r in runs if r["setting"] == name]
        own = np.array([r["best_s"] for r in rs]) / bf.best_time_s
        ret = np.array([times[r["best"]] for r in rs]) / t_bf
        cvs = [r["cv"] for r in rs if r["cv"] is not None]
        curves = np.array([[v if v is not None else np.nan for v in r["curve"]] for r in rs], dtype=np.float64)
        best_genes = np.array([r["best"] for r in rs])
        out["settings"].append({
            "name": name, "kind": kind, "params": dict(GA_STUDY_BASE, **kw),
            "evals_median": float(np.median([r["evals"] for r in rs])),
            "wall_s_median": float(np.median([r["wall_s"] for r in rs])),
            "restarts_median": float(np.median([r["restarts"] for r in rs])),
            "own_best_over_bf": {"median": float(np.median(own)), "p10": float(np.percentile(own, 10)),
                                 "p90": float(np.percentile(own, 90))},
            "retimed_over_bf": {"median": float(np.median(ret)), "p10": float(np.percentile(ret, 10)),
                                "p90": float(np.percentile(ret, 90)), "worst": float(ret.max())},
            "runs_within_5pct_of_bf": int(np.sum(ret <= 1.05)),
            "runs_better_than_bf": int(np.sum(ret < 1.0)),
            "curve_own_best_over_bf_median": dict(zip(map(str, checkpoints),
                                                      [None if np.all(np.isnan(c)) else float(np.nanmedian(c))
                                                       for c in curves.T])),
            "cv_end_population": dict(zip(names, np.mean(cvs, axis=0).tolist())) if cvs else None,
            "retimed_over_bf_all": ret.tolist(),
            "best_gene_histograms": {n: dict(zip(*[list(map(int, a)) for a in np.unique(best_genes[:, k],
                                                                                        return_counts=True)]))
                                     for k, n in enumerate(names)}})
    return out


def ga_study_table(seeds: int):
    """The GA studies replayed on a measured fitness table of the 256-channel /
    128-DM workload (a noise-free control in which the two kernels cannot
    interact): each dedispersion configuration is timed once with the boxcar /
    S/N kernel at 256 threads, each S/N thread count once with the default
    dedispersion tiles (the library's timer, median of 7 runs), and a
    configuration's fitness is the sum of its dedispersion entry and its
    thread count's difference from 256 threads, so per-kernel brute force is
    exact on it by construction.  The table holds dms_per_thread 1 and LDS
    staging."""
    import itertools
    import paper_1811_04165_amd as amber
    wl, search, x, n_in, sp, bufs = _small_tune_setup()
    G = amber.genes
    sp.set_gene_values(G.GENE_DMS_PER_THREAD, [1])
    sp.set_gene_values(G.GENE_DIRECT_READS, [0])
    nw = len(wl.widths)
    gv = [sp.gene_values(i) for i in range(sp.n_genes)]
    params = amber.tune_params("exhaustive", warmup=1, reps=7)

    def timed(t):
        return amber.tune(_point_space(search, t), search.delays, x, n_in, params, buffers=bufs).best_time_s

    print("[bench] measuring the fitness table", file=sys.stderr, flush=True)
    gc.collect()
    t_dd = {}
    for tpd, spt, dpb, cu in itertools.product(*gv[:4]):
        t = amber.make_tiles(threads_per_dm=tpd, samples_per_thread=spt, dms_per_block=dpb, channel_unroll=cu,
                             dms_per_thread=1, direct_reads=0, snr_threads=256)
        try:
            amber.validate_tiles(t, search.info, nw)
        except amber.AmberError:
            continue
        t_dd[(tpd, spt, dpb, cu)] = timed(t)
    ref = timed(amber.make_tiles(snr_threads=256))
    t_box = {thr: timed(amber.make_tiles(snr_threads=thr)) - ref for thr in gv[G.GENE_SNR_THREADS]}
    return ga_study_replay(sp, wl, t_dd, t_box, seeds)["ga_study"]


def ga_study_replay(sp, wl, t_dd, t_box, seeds: int):
    """The searches of the GA study against a fitness table (host only)."""
    import json
    import os
    import tempfile
    import numpy as np
    import paper_1811_04165_amd as amber

    def fitness_of(t):
        return t_dd[(t.threads_per_dm, t.samples_per_thread, t.dms_per_block, t.channel_unroll)] + \
            t_box[t.snr_threads]

    opt = min(t_dd.values()) + min(t_box.values())

    def run(kind, log=None, **kw):
        hist = []

        def fit(t):
            v = fitness_of(t)
            hist.append((v, (t.threads_per_dm, t.samples_per_thread, t.dms_per_block, t.channel_unroll,
                             t.snr_threads)))
            return v
        r = amber.search_tiles(sp, amber.tune_params(kind, **kw), fit, log_path=log)
        return r, hist

    bf, _ = run("per_kernel")
    t_bf, budget = bf.best_time_s, bf.n_evals
    checkpoints = [c for c in (50, 100, 200, 400, 800) if c < budget] + [budget]
    G = amber.genes
    cols = [G.GENE_THREADS_PER_DM, G.GENE_SAMPLES_PER_THREAD, G.GENE_DMS_PER_BLOCK, G.GENE_CHANNEL_UNROLL,
            G.GENE_SNR_THREADS]
    genes = ["threads_per_dm", "samples_per_thread", "dms_per_block", "channel_unroll", "snr_threads"]
    base = GA_STUDY_BASE
    settings = _ga_study_settings()
    out = {"workload": wl.name, "space_size": amber.space_size(sp), "table": {
        "dedisperse_configs": len(t_dd), "boxcar_configs": len(t_box), "optimum_s": opt,
        "dedisperse_best_s": min(t_dd.values()), "boxcar_best_s": min(t_box.values())},
        "brute_force_per_kernel": {"best_s": t_bf, "evals": budget, "over_optimum": t_bf / opt},
        "budget_evals": budget, "seeds": seeds, "settings": []}
    tmp = tempfile.mkdtemp()
    for name, kind, kw in settings:
        print("[bench] study: %s" % name, file=sys.stderr, flush=True)
        p = dict(base)
        p.update(kw)
        finals, curves, cvs, best_genes, evals = [], [], [], [], []
        for seed in range(1, seeds + 1):
            if kind == "ga":
                log = os.path.join(tmp, "ga.jsonl")
                if os.path.exists(log):
                    os.remove(log)
                gens = max(1, budget // p["pop"] - 1)
                r, hist = run("ga", log=log, seed=seed, generations=gens, **p)
                lines = [json.loads(l) for l in open(log)]
                # the final population lists every gene's value: keep the studied ones, in the order of `genes`
                end = np.array(lines[-1]["final_population"], dtype=np.float64)[:, cols]
            else:
                r, hist = run("random", seed=1000 + seed, max_evals=budget)
                top = sorted({c: v for v, c in hist}.items(), key=lambda kv: kv[1])[:p["pop"]]
                end = np.array([c for c, _ in top], dtype=np.float64)
            vals = [v for v, _ in hist]
            run_best = np.minimum.accumulate(vals)
            curves.append([float(run_best[min(c, len(run_best)) - 1]) / t_bf for c in checkpoints])
            finals.append(r.best_time_s)
            evals.append(r.n_evals)
            cvs.append(end.std(axis=0) / end.mean(axis=0))
            b = r.best
            best_genes.append([b.threads_per_dm, b.samples_per_thread, b.dms_per_block, b.channel_unroll,
                               b.snr_threads])
        f = np.array(finals)
        cv = np.mean(cvs, axis=0)
        hist_genes = {gname: dict(zip(*[list(map(int, a)) for a in np.unique(np.array(best_genes)[:, k],
                                                                              return_counts=True)]))
                      for k, gname in enumerate(genes)}
        out["settings"].append({
            "name": name, "kind": kind, "params": p, "evals_median": float(np.median(evals)),
            "best_over_bf": {"median": float(np.median(f / t_bf)), "p10": float(np.percentile(f / t_bf, 10)),
                             "p90": float(np.percentile(f / t_bf, 90))},
            "best_over_optimum_median": float(np.median(f / opt)),
            "runs_within_5pct_of_optimum": int(np.sum(f <= 1.05 * opt)),
            "curve_best_over_bf_median": dict(zip(map(str, checkpoints), np.median(curves, axis=0).tolist())),
            "cv_end_population": dict(zip(genes, cv.tolist())),
            "best_over_bf_all": (f / t_bf).tolist(), "best_gene_histograms": hist_genes})
    return {"metric": "GA studies", "unit": "ratio", "value": out["settings"][0]["best_over_bf"]["median"],
            "higher_is_better": False, "ga_study": out}


def rfi_report(steps: int, warmup: int):
    """Dedispersion with zapped channels on the 1536-channel beam (a 150-channel
    band and 40 scattered channels zapped) beside plain dedispersion."""
    import numpy as np
    import torch
    import paper_1811_04165_amd as amber
    import workloads
    wl = workloads.beam()
    g = wl.geom
    search = amber.Search(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step, wl.n_out, wl.widths)
    x_host, n_in = workloads.make_input(wl, search.delays_host, search.info.max_delay)
    x = torch.from_numpy(x_host).cuda()
    keep = np.ones(g.n_chan, np.uint8)
    keep[700:850] = 0
    keep[np.random.default_rng(42).choice(g.n_chan, 40, replace=False)] = 0
    keep_dev = torch.from_numpy(keep).cuda()
    tiles = amber.default_tiles()

    def timed(fn):
        for _ in range(warmup):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        b.record()
        torch.cuda.synchronize()
        gc.collect()
        gc.disable()
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        gc.enable()
        return a.elapsed_time(b) / 1e3 / steps

    t_plain = timed(lambda: amber.dedisperse(search.delays, search.info, x, n_in, wl.n_out, tiles, out=search.dd))
    t_mask = timed(lambda: amber.dedisperse(search.delays, search.info, x, n_in, wl.n_out, tiles, out=search.dd,
                                            keep=keep_dev))
    adds = float(int(keep.sum())) * g.n_dm * wl.n_out
    return {"metric": "masked dedispersion time", "unit": "s", "value": t_mask, "higher_is_better": False,
            "rfi": {"workload": wl.name, "zapped_channels": int((keep == 0).sum()), "steps": steps,
                    "dedisperse_ms": 1e3 * t_plain, "dedisperse_masked_ms": 1e3 * t_mask,
                    "kept_adds_per_s": adds / t_mask}}


def downsample_report(steps: int, warmup: int):
    """Decimating downsampling + S/N (the paper's smoothing definition) on the
    1536-channel beam: the ten series of the factor ladder in one fused launch,
    beside the sliding boxcar widths on the same dedispersed data."""
    import torch
    import paper_1811_04165_amd as amber
    import workloads
    wl = workloads.beam()
    g = wl.geom
    search = amber.Search(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step, wl.n_out, wl.widths)
    x_host, n_in = workloads.make_input(wl, search.delays_host, search.info.max_delay)
    x = torch.from_numpy(x_host).cuda()
    search.run(x)
    factors = workloads.DOWNSAMPLING_FACTORS
    s = torch.empty((len(factors), g.n_dm), dtype=torch.float32, device="cuda")
    p = torch.empty((len(factors), g.n_dm), dtype=torch.int32, device="cuda")

    def timed(fn):
        for _ in range(warmup):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        b.record()
        torch.cuda.synchronize()
        gc.collect()
        gc.disable()
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        gc.enable()
        return a.elapsed_time(b) / 1e3 / steps

    t_ds = timed(lambda: amber.downsample_snr(search.dd, wl.n_out, factors, out=(s, p)))
    t_box = timed(lambda: amber.integrate_snr(search.dd, wl.n_out, wl.widths, out=(search.snr, search.peak)))
    sn = s.cpu().numpy()
    found = sum(1 for pu in wl.pulses if sn[:, pu.dm_index].max() > 8.0)
    alg = 4 * g.n_dm * wl.n_out + 8 * len(factors) * g.n_dm
    return {"metric": "downsample + S/N time", "unit": "s", "value": t_ds, "higher_is_better": False,
            "downsample": {"workload": wl.name, "factors": list(factors), "steps": steps,
                           "downsample_snr_ms": 1e3 * t_ds, "integrate_snr_ms": 1e3 * t_box,
                           "widths": list(wl.widths),
                           "roofline": {"bound": "hbm", "achieved": alg / t_ds / 1e9, "peak": HBM_PEAK_GBS,
                                        "unit": "GB/s", "frac": alg / t_ds / 1e9 / HBM_PEAK_GBS,
                                        "bytes_per_launch": alg},
                           "pulses_with_snr_above_8": found}}


SUBBAND_GRIDS = {
    # the 1536-channel beam's own 2048 trials (0..1023.5 step 0.5) from 32 subbands
    "beam-grid": (32, 128, 0.0, 8.0, 16, 0.0, 0.5),
    # Table 2's subbanding grid: 2048 coarse DMs step 2.4, 24 fine DMs step 0.1
    "table2-grid": (32, 2048, 0.0, 2.4, 24, 0.0, 0.1),
}


def subband_report(steps: int, warmup: int, grid_names, bf_steps: int = 3):
    """Two-step subband dedispersion on the 1536-channel, 12208-sample beam,
    beside brute-force dedispersion of the same trials: time, throughput, and
    the S/N of injected pulses under both (the scheme's approximation loss)."""
    import numpy as np
    import torch
    import paper_1811_04165_amd as amber
    import workloads
    wl = workloads.beam()
    g = wl.geom
    f = g.freqs()
    n_out = wl.n_out

    def timed(fn, n, w):
        # at least half a second of the same work first: the clocks ramp up
        # while the host builds tables and inputs
        t_end = time.perf_counter() + 0.5
        k = 0
        while k < w or time.perf_counter() < t_end:
            fn()
            torch.cuda.synchronize()
            k += 1
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        b.record()
        torch.cuda.synchronize()
        gc.collect()
        gc.disable()
        a.record()
        for _ in range(n):
            fn()
        b.record()
        torch.cuda.synchronize()
        gc.enable()
        return a.elapsed_time(b) / 1e3 / n

    out = {}
    for name in grid_names:
        grid = SUBBAND_GRIDS[name]
        n_sub, nc, cf, cs, nf, ff, fs = grid
        d1, d2, info = amber.subband_delay_tables(f, g.t_samp_s, *grid)
        n_dm = nc * nf
        # brute force over the same trial DMs (both grids are dyadic-free but
        # DM_jk = (cf + j cs + ff) + k fs is what both tables use)
        dms = np.array([(cf + j * cs + ff) + k * fs for j in range(nc) for k in range(nf)])
        bd = np.empty((n_dm, g.n_chan), np.int32)
        bmax = 0
        for i0 in range(0, n_dm, 4096):  # one-row tables keep each trial's DM exactly as above
            for i in range(i0, min(n_dm, i0 + 4096)):
                row, info_i = amber.delay_table(f, g.t_samp_s, 1, float(dms[i]), 0.0)
                bd[i] = row[0]
                bmax = max(bmax, info_i.max_delay)
        steps_bf = np.diff(bd, axis=0).max() if n_dm > 1 else 0
        binfo = amber.DelayInfo(n_dm=n_dm, n_chan=g.n_chan, max_delay=int(bmax), max_step=int(steps_bf))
        n_in = n_out + max(info.max_delay, bmax)
        rng = np.random.default_rng([11, nc])
        pulses = []
        x = workloads.noise(g.n_chan, n_in, workloads.padded_stride(n_in), seed=12)
        for k in range(5):
            i = int(rng.integers(0, n_dm))
            w = int(rng.choice([1, 2, 4, 8, 16, 32]))
            t0 = 1024 + 2048 * k
            workloads.inject(x, bd[i], t0=t0, width=w, amp=40)
            pulses.append((i, w, t0))
        xd = torch.from_numpy(x).cuda()
        d1d, d2d = torch.from_numpy(d1).cuda(), torch.from_numpy(d2).cuda()
        n1 = n_out + info.max_delay2
        work = torch.empty((n_sub * nc, (n1 + 63) // 64 * 64), dtype=torch.uint16, device="cuda")
        dd_sb = torch.empty((n_dm, n_out), dtype=torch.int32, device="cuda")
        print("[bench] subband %s: %d trials, n_in %d" % (name, n_dm, n_in), file=sys.stderr, flush=True)
        t_sb = timed(lambda: amber.subband_dedisperse(d1d, d2d, info, xd, n_in, n_out, out=dd_sb, work=work),
                     steps, warmup)
        widths = wl.widths
        snr_sb = torch.empty((len(widths), n_dm), dtype=torch.float32, device="cuda")
        pk = torch.empty((len(widths), n_dm), dtype=torch.int32, device="cuda")
        t_snr = timed(lambda: amber.integrate_snr(dd_sb, n_out, widths, out=(snr_sb, pk)), steps, warmup)
        s_sb = snr_sb.cpu().numpy()
        del work
        # brute force on the same trials, same input, same output buffer shape
        bdd = torch.from_numpy(bd).cuda()
        dd_bf = torch.empty((n_dm, n_out), dtype=torch.int32, device="cuda")
        print("[bench] brute force %s" % name, file=sys.stderr, flush=True)
        t_bf = timed(lambda: amber.dedisperse(bdd, binfo, xd, n_in, n_out, out=dd_bf),
                     steps if n_dm <= 4096 else bf_steps, 1)
        amber.integrate_snr(dd_bf, n_out, widths, out=(snr_sb, pk))
        s_bf = snr_sb.cpu().numpy()
        del bdd, dd_bf, dd_sb
        torch.cuda.empty_cache()
        loss = []
        for i, w, t0 in pulses:
            wi = list(widths).index(w)
            lo, hi = max(0, i - 2), min(n_dm, i + 3)
            a, b = float(s_sb[wi, lo:hi].max()), float(s_bf[wi, lo:hi].max())
            loss.append({"trial": i, "dm": float(dms[i]), "width": w, "snr_subband": a, "snr_brute_force": b,
                         "ratio": a / b})
        adds1 = float(nc) * g.n_chan * n1
        adds2 = float(nc) * nf * n_sub * n_out
        out[name] = {
            "grid": {"subbands": n_sub, "coarse": [nc, cf, cs], "fine": [nf, ff, fs]}, "n_dm": n_dm,
            "n_in": n_in, "info": {k: getattr(info, k) for k, _ in info._fields_},
            "subband_dedisperse_ms": 1e3 * t_sb, "brute_force_dedisperse_ms": 1e3 * t_bf,
            "speedup_vs_brute_force": t_bf / t_sb, "integrate_snr_ms": 1e3 * t_snr,
            "dm_trial_samples_per_s": n_dm * n_out / t_sb,
            "path_dm_trial_samples_per_s": n_dm * n_out / (t_sb + t_snr),
            "sample_adds": {"step1": adds1, "step2": adds2, "brute_force": float(n_dm) * g.n_chan * n_out},
            "alu_frac_both_steps": (adds1 + adds2) / t_sb / 1e12 / ALU_PEAK_TOPS,
            "snr_loss": loss,
        }
    first = out[grid_names[0]]
    return {"metric": "subband dedispersion throughput", "unit": UNIT, "value": first["dm_trial_samples_per_s"],
            "higher_is_better": True, "workload": wl.name, "steps": steps, "subband": out}


def tune_subband_report(seeds: int, grid_name: str = "table2-grid"):
    """Tile search of the subband pipeline on the 1536-channel beam: GA
    (several seeds) vs random search (same budget as each GA run) vs
    per-kernel brute force over both steps' genes (boxcar / S/N genes held at
    the library's), finalists re-timed interleaved, beside the automatic
    tiles."""
    import torch
    import paper_1811_04165_amd as amber
    import workloads
    wl = workloads.beam()
    g = wl.geom
    grid = SUBBAND_GRIDS[grid_name]
    d1, d2, info = amber.subband_delay_tables(g.freqs(), g.t_samp_s, *grid)
    n_out = wl.n_out
    n_in = n_out + info.max_delay
    x = torch.from_numpy(workloads.noise(g.n_chan, n_in, workloads.padded_stride(n_in), seed=12)).cuda()
    d1d, d2d = torch.from_numpy(d1).cuda(), torch.from_numpy(d2).cuda()
    n_dm = info.n_coarse * info.n_fine
    n1 = n_out + info.max_delay2
    work = torch.empty((info.n_subbands * info.n_coarse, (n1 + 63) // 64 * 64), dtype=torch.uint16, device="cuda")
    dd = torch.empty((n_dm, n_out), dtype=torch.int32, device="cuda")
    snr = torch.empty((len(wl.widths), n_dm), dtype=torch.float32, device="cuda")
    peak = torch.empty((len(wl.widths), n_dm), dtype=torch.int32, device="cuda")
    sp = amber.default_subband_space(info, wl.widths, n_out)
    G = amber.genes
    d = amber.default_tiles()
    sp.set_gene_values(G.SB_GENE_SNR_THREADS, [d.snr_threads])
    for k in range(len(wl.widths)):
        sp.set_gene_values(G.SB_GENE_BOXCAR0 + k, [d.boxcar_step[k]])
    bufs = dict(work=work, out=dd, snr=snr, peak=peak)

    def run(kind, **kw):
        print("[bench] subband tune %s %s" % (kind, kw), file=sys.stderr, flush=True)
        return amber.tune_subband(sp, d1d, d2d, x, n_in, amber.tune_params(kind, **kw), **bufs)

    ga = [run("ga", seed=s) for s in range(1, seeds + 1)]
    rnd = [run("random", seed=100 + s, max_evals=ga[s - 1].n_evals) for s in range(1, seeds + 1)]
    pk = run("per_kernel")

    # the boxcar / S/N tiles the search held (explicit: with tiles=None the
    # library would size its work-groups by the 49152 rows)
    t_box = amber.make_tiles(snr_threads=d.snr_threads, boxcar_step=[d.boxcar_step[k] for k in range(len(wl.widths))])

    def path(t1, t2):
        amber.subband_dedisperse(d1d, d2d, info, x, n_in, n_out, tiles1=t1, tiles2=t2, out=dd, work=work)
        amber.integrate_snr(dd, n_out, wl.widths, t_box, out=(snr, peak))

    finalists = [(r.step1, r.step2) for r in ga + rnd + [pk]] + [(None, None)]
    print("[bench] interleaved re-timing of %d finalists" % len(finalists), file=sys.stderr, flush=True)
    for t1, t2 in finalists:
        path(t1, t2)
    times = [[] for _ in finalists]
    for _ in range(10):
        for k, (t1, t2) in enumerate(finalists):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            path(t1, t2)
            b.record()
            b.synchronize()
            times[k].append(a.elapsed_time(b) / 1e3)
    med = [statistics.median(t) for t in times]
    n = seeds
    t_ga, t_rnd, t_pk, t_auto = med[:n], med[n:2 * n], med[2 * n], med[2 * n + 1]
    nw = len(wl.widths)
    out = {"workload": "%s, %s" % (wl.name, grid_name), "space_size": amber.subband_space_size(sp),
           "genes": {"step1": [sp.gene_values(i) for i in range(G.SB_GENE_STEP2)],
                     "step2": [sp.gene_values(i) for i in range(G.SB_GENE_STEP2, G.SB_GENE_SNR_THREADS)]},
           "retimed_s": {"ga": t_ga, "random": t_rnd, "per_kernel": t_pk, "automatic_tiles": t_auto},
           "ga_median_over_per_kernel": statistics.median(t_ga) / t_pk,
           "random_median_over_per_kernel": statistics.median(t_rnd) / t_pk,
           "automatic_over_ga_median": t_auto / statistics.median(t_ga),
           "cost": {"ga_evals_median": statistics.median([r.n_evals for r in ga]),
                    "ga_wall_s_median": statistics.median([r.wall_s for r in ga]),
                    "per_kernel_evals": pk.n_evals, "per_kernel_wall_s": pk.wall_s},
           "best": {"ga_seed1": ga[0].as_dict(nw), "per_kernel": pk.as_dict(nw)}}
    return {"metric": "subband GA tune time", "unit": "s", "value": out["cost"]["ga_wall_s_median"],
            "higher_is_better": False, "tune_subband": out}


def peaks_report():
    """Issue rates and bandwidths the roofline peaks rest on, measured with the
    microbenchmarks of paper_1811_04165_amd/peaks/peaks.hip (one launch of
    2048 work-groups of 256 work-items, i.e. 32 wavefronts per CU, each timed
    with HIP events after a warm-up launch)."""
    import ctypes
    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1811_04165_amd", "libamber_peaks.so"))
    out = torch.zeros(2048 * 256, dtype=torch.int32, device="cuda")
    cus, clk = 256, 2.4e9
    blocks = 2048
    res = {"blocks": blocks, "threads": 256, "clock_hz_assumed": clk, "cus": cus, "valu": {}, "lds": {}}
    names = ["v_add_u32", "v_add3_u32", "v_pk_add_u16", "v_lshl_or_b32", "v_fma_f64", "v_cvt_f64_i32",
             "v_max3_i32", "v_mad_u64_u32", "v_add_f64", "v_max_f64", "v_cvt_f32_i32", "v_mul_lo_u32",
             "v_cvt_f64_u32", "v_sub_u32"]
    for kind, name in enumerate(names):
        r = ctypes.c_double()
        if lib.peaks_valu(kind, blocks, 20000, ctypes.c_void_p(out.data_ptr()), ctypes.byref(r)) != 0:
            raise RuntimeError("peaks_valu %s failed" % name)
        res["valu"][name] = {"wave_instr_per_s": r.value, "lane_ops_per_s": 64 * r.value,
                             "lanes_per_clk_per_cu": 64 * r.value / (cus * clk)}
    for form, name in enumerate(["ds_read_b32", "ds_read2st64_b32", "ds_read_b64", "ds_read2st64_b64",
                                 "ds_read_b128", "ds_read2_b32 (8-byte aligned)", "ds_read2_b32 (4 mod 8)",
                                 "ds_read_b64 / ds_read2_b32 (4 mod 8) alternating"]):
        r = ctypes.c_double()
        if lib.peaks_lds(form, blocks, 4000, ctypes.c_void_p(out.data_ptr()), ctypes.byref(r)) != 0:
            raise RuntimeError("peaks_lds %s failed" % name)
        res["lds"][name] = {"bytes_per_s": r.value, "bytes_per_clk_per_cu": r.value / (cus * clk)}
    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    bw, sec = ctypes.c_double(), ctypes.c_double()
    if lib.peaks_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), ctypes.c_size_t(n),
                      cus * 16, ctypes.byref(bw), ctypes.byref(sec)) != 0:
        raise RuntimeError("peaks_copy failed")
    res["hbm_copy"] = {"bytes": n, "seconds": sec.value, "read_plus_write_bytes_per_s": bw.value,
                       "frac_of_8TBs": bw.value / 8e12}
    return res


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-rows", type=int, default=2048, help="DM trials in the CPU oracle sample (0 = skip)")
    ap.add_argument("--tiles", type=str, default="", help="JSON dict of tile overrides")
    ap.add_argument("--tune", action="store_true",
                    help="instead of the throughput step: compare the GA tile search with exhaustive, random and "
                         "per-kernel brute-force search on the 256-channel workload")
    ap.add_argument("--tune-seeds", type=int, default=10)
    ap.add_argument("--tune-log", type=str, default="",
                    help="JSONL log of the --tune searches (a line per generation, or per 50 evaluations)")
    ap.add_argument("--ga-study", action="store_true",
                    help="instead of the throughput step: the paper's GA studies (mutation and crossover rates, "
                         "population size, crossover type, random search) replayed on a measured fitness table")
    ap.add_argument("--study-seeds", type=int, default=35)
    ap.add_argument("--batched", action="store_true",
                    help="instead of the single-beam step: 40 uneven beams, per-beam launches vs one batch vs "
                         "the batch replayed as a HIP graph")
    ap.add_argument("--beams", type=int, default=40)
    ap.add_argument("--serve", action="store_true",
                    help="instead of the single-beam step: the streaming service under Poisson arrivals, "
                         "continuous batching vs one chunk at a time")
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--serve-warmup", type=float, default=2.0)
    ap.add_argument("--serve-rates", type=str, default="400,800,1600",
                    help="offered chunks/s, comma separated; rates above twice the first run briefly")
    ap.add_argument("--rfi", action="store_true",
                    help="instead of the single-beam step: dedispersion with zapped channels beside plain")
    ap.add_argument("--tune-subband", action="store_true",
                    help="GA vs random vs per-kernel search over both subband steps' genes (Table 2 grid)")
    ap.add_argument("--subband", type=str, default="", metavar="GRIDS",
                    help="two-step subband dedispersion vs brute force on the beam, for the comma-separated "
                         "grids beam-grid, table2-grid")
    ap.add_argument("--downsample", action="store_true",
                    help="instead of the single-beam step: decimating downsampling + S/N over the factor ladder "
                         "on the dedispersed beam")
    ap.add_argument("--peaks", action="store_true",
                    help="instead of the throughput step: the VALU, LDS and copy microbenchmarks behind the "
                         "roofline peaks")
    ap.add_argument("--extras", type=int, default=1,
                    help="1: also run one GA tile search (tune time) and 5 s of serving (p99 chunk latency)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="also run a plain device-to-device copy of this many bytes 5 times (for scaling "
                         "hardware byte counters read under a profiler)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on exactly one GPU (the hot path is measured at N=1); "
              "got --gpus %d" % args.gpus, file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import paper_1811_04165_amd as amber
    import workloads

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 3
    if args.peaks:
        print(json.dumps(peaks_report()))
        return 0
    if args.tune:
        print(json.dumps(tune_report(args.tune_seeds, args.tune_log or None)))
        return 0
    if args.batched:
        print(json.dumps(batched_report(args.beams, args.steps, args.warmup)))
        return 0
    if args.ga_study:
        print(json.dumps(ga_study_report(args.study_seeds)))
        return 0
    if args.rfi:
        print(json.dumps(rfi_report(args.steps, args.warmup)))
        return 0
    if args.downsample:
        print(json.dumps(downsample_report(args.steps, args.warmup)))
        return 0
    if args.tune_subband:
        print(json.dumps(tune_subband_report(5)))
        return 0
    if args.subband:
        print(json.dumps(subband_report(args.steps, args.warmup, [n for n in args.subband.split(",") if n])))
        return 0
    if args.serve:
        rates = [float(r) for r in args.serve_rates.split(",") if r]
        print(json.dumps(serve_report(args.beams, args.serve_seconds, args.serve_warmup, rates)))
        return 0
    wl = workloads.beam()
    g = wl.geom
    tiles = amber.make_tiles(**json.loads(args.tiles)) if args.tiles else amber.default_tiles()

    print("[bench] building input", file=sys.stderr, flush=True)
    search = amber.Search(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step, wl.n_out, wl.widths, tiles=tiles)
    x_host, n_in = workloads.make_input(wl, search.delays_host, search.info.max_delay)
    x = torch.from_numpy(x_host).cuda()
    torch.cuda.synchronize()

    print("[bench] warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        search.run(x)
    torch.cuda.synchronize()

    n_launch = args.steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(n_launch)]
    # torch creates the HIP events on their first record: do that before the
    # timed region so that event creation never stalls the launches
    for a, b, c in ev:
        a.record()
        b.record()
        c.record()
    print("[bench] timed %d steps" % args.steps, file=sys.stderr, flush=True)
    # a garbage collection over torch's heap can stall the launching thread for
    # tens of milliseconds while the GPU idles: none inside the timed region
    gc.collect()
    gc.disable()
    host_t = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        a, b, c = ev[k]
        a.record()
        amber.dedisperse(search.delays, search.info, x, search.n_in, search.n_out, tiles, out=search.dd)
        b.record()
        amber.integrate_snr(search.dd, search.n_out, search.widths, tiles, out=(search.snr, search.peak))
        c.record()
        host_t.append(time.perf_counter())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gc.enable()
    gaps = [1e3 * (t2 - t1) for t1, t2 in zip([t0] + host_t, host_t)]
    print("[bench] host ms per launch pair: median %.3f max %.3f" % (statistics.median(gaps), max(gaps)),
          file=sys.stderr, flush=True)
    k1_ms = [a.elapsed_time(b) for a, b, _ in ev]
    k23_ms = [b.elapsed_time(c) for _, b, c in ev]

    ms_per_step = wall * 1e3 / args.steps
    samples = g.n_dm * wl.n_out
    value = samples / (ms_per_step / 1e3)

    # dominant kernel: dedispersion, n_chan additions per DM-trial sample
    k1_avg = statistics.mean(k1_ms)
    ops = float(g.n_chan) * samples
    achieved = ops / (k1_avg / 1e3) / 1e12
    traffic = measured_traffic(ops)
    # LDS reads: every addition reads its 16-bit sample from LDS once
    lds_bytes = 2.0 * ops
    lds_tbs = lds_bytes / (k1_avg / 1e3) / 1e12
    # whole-path HBM bytes: input once, dd written and read once, S/N tables
    path_bytes = g.n_chan * x.stride(0) + 2 * 4 * samples + 8 * len(wl.widths) * g.n_dm
    k23_avg = statistics.mean(k23_ms)
    k23_bytes = 4 * samples + 8 * len(wl.widths) * g.n_dm

    # sanity: the five injected pulses are the strongest detections of their rows
    sn = search.snr.cpu().numpy()
    found = sum(1 for p in wl.pulses if sn[list(wl.widths).index(p.width), p.dm_index] > 8.0)

    rec = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": wl.name, "n_chan": g.n_chan, "n_dm": g.n_dm, "n_out": wl.n_out, "n_in": n_in,
                   "widths": list(wl.widths), "tiles": tiles.as_dict(), "pulses_found": found},
        "roofline": {"bound": "alu", "kernel": "dedisperse", "achieved": achieved, "peak": ALU_PEAK_TOPS,
                     "unit": "TOP/s", "frac": achieved / ALU_PEAK_TOPS, "traffic": traffic,
                     "avg_launch_ms": k1_avg, "ops_per_launch": ops,
                     "lds": {"bytes_per_launch": lds_bytes, "achieved": lds_tbs, "peak": LDS_PEAK_TBS,
                             "unit": "TB/s", "frac": lds_tbs / LDS_PEAK_TBS}},
        "kernels": {
            "dedisperse_ms": k1_avg,
            "dedisperse_median_ms": statistics.median(k1_ms),
            "integrate_snr_ms": k23_avg,
            "integrate_snr_median_ms": statistics.median(k23_ms),
            "integrate_snr_max_ms": max(k23_ms),
            "integrate_snr_hbm_frac": k23_bytes / (k23_avg / 1e3) / 1e9 / HBM_PEAK_GBS,
        },
        "hbm_frac_path": path_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS,
    }
    if args.extras:
        print("[bench] GA tune on the 256-channel workload", file=sys.stderr, flush=True)
        rec["ga_tune"] = ga_tune_summary()
        print("[bench] serving at 400 chunks/s", file=sys.stderr, flush=True)
        rec["serve"] = serve_summary()
    if args.copy_calibration > 0:
        src = torch.empty(args.copy_calibration, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        rec["copy_calibration_bytes"] = args.copy_calibration
    if args.cpu_rows > 0:
        print("[bench] cpu oracle baseline (%d rows)" % args.cpu_rows, file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(x_host, n_in, wl, args.cpu_rows)
    print(json.dumps(rec))
    return 0


if __name__ == "__main__":
    sys.exit(main())
