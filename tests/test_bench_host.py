"""Host-side parts of bench.py: the one-GPU guard and the GA-study replay
against a synthetic fitness table (no GPU)."""
import itertools
import math
import os
import subprocess
import sys

import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_ga_study_replay_on_a_synthetic_table():
    """Every setting runs, the per-kernel brute force finds the table optimum,
    and the end-population statistics are finite and keyed by the studied
    genes: genes the study holds fixed (one value) must not shift or pollute
    the columns."""
    import bench
    import paper_1811_04165_amd as amber
    wl = workloads.small()
    g = wl.geom
    _, info = amber.delay_table(g.freqs(), g.t_samp_s, g.n_dm, g.dm_first, g.dm_step)
    sp = amber.default_space(info, wl.widths, wl.n_out)
    G = amber.genes
    sp.set_gene_values(G.GENE_THREADS_PER_DM, [64, 256])
    sp.set_gene_values(G.GENE_SAMPLES_PER_THREAD, [4, 8])
    sp.set_gene_values(G.GENE_DMS_PER_BLOCK, [1, 4])
    sp.set_gene_values(G.GENE_CHANNEL_UNROLL, [2, 8])
    sp.set_gene_values(G.GENE_DMS_PER_THREAD, [1])
    sp.set_gene_values(G.GENE_DIRECT_READS, [0])
    sp.set_gene_values(G.GENE_SNR_THREADS, [64, 256, 1024])
    # fitness: a smooth bowl in log2 of every studied gene, separable by kernel
    t_dd = {}
    for tpd, spt, dpb, cu in itertools.product([64, 256], [4, 8], [1, 4], [2, 8]):
        t = amber.make_tiles(threads_per_dm=tpd, samples_per_thread=spt, dms_per_block=dpb, channel_unroll=cu,
                             dms_per_thread=1, direct_reads=0, snr_threads=256)
        try:
            amber.validate_tiles(t, info, len(wl.widths))
        except amber.AmberError:
            continue
        t_dd[(tpd, spt, dpb, cu)] = 1e-5 * (1 + math.log2(tpd / 64) + abs(math.log2(spt / 8)) + math.log2(dpb)
                                            + abs(math.log2(cu / 8)))
    t_box = {thr: 1e-6 * abs(math.log2(thr / 256)) for thr in (64, 256, 1024)}
    out = bench.ga_study_replay(sp, wl, t_dd, t_box, seeds=2)["ga_study"]
    assert out["brute_force_per_kernel"]["over_optimum"] == pytest.approx(1.0)
    names = ["threads_per_dm", "samples_per_thread", "dms_per_block", "channel_unroll", "snr_threads"]
    assert len(out["settings"]) == 12
    assert [st["name"] for st in out["settings"]][-1].startswith("restart")
    for st in out["settings"]:
        assert list(st["cv_end_population"]) == names, st["name"]
        assert all(math.isfinite(v) and v >= 0 for v in st["cv_end_population"].values()), st["name"]
        assert st["best_over_bf"]["median"] >= 1.0 - 1e-9
        assert set(st["best_gene_histograms"]) == set(names)


def test_traffic_is_reported_only_for_the_profiled_kernel_source(tmp_path, monkeypatch):
    """roofline.traffic comes from the committed counter record while its
    kernel hash is the dedispersion source's, and is null for any other
    source (the counters describe a kernel that no longer exists)."""
    import json
    import bench
    rec = json.load(open(bench.PMC_FILE))
    for k in ("kernel_sha", "fetch_size_kib", "write_size_kib", "hbm_bytes_per_launch", "copy_calibration",
              "commands"):
        assert k in rec
    assert rec["hbm_bytes_per_launch"] == pytest.approx(
        rec["fetch_size_kib"] * 1024 * rec["copy_calibration"]["fetch_factor"] +
        rec["write_size_kib"] * 1024 * rec["copy_calibration"]["write_factor"], rel=1e-3)
    # the committed record belongs to the committed kernel source
    assert rec["kernel_sha"] == bench.kernel_hash()
    assert bench.measured_traffic(1.0) == rec["hbm_bytes_per_launch"]
    other = tmp_path / "dedisperse.hip"
    other.write_bytes(open(bench.KERNEL_SRC, "rb").read() + b"\n// changed\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(other))
    assert bench.measured_traffic(1.0) is None
