"""bench.py's JSON line on the GPU: one short run of the default step, its
contract fields and their internal consistency (not the timings)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line():
    print("[case] bench.py --steps 3 --warmup 1 --cpu-rows 32", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "3", "--warmup", "1",
                        "--cpu-rows", "32"], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout
    rec = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in rec, k
    assert rec["n_gpus"] == 1 and rec["steps"] == 3 and rec["warmup"] == 1
    assert rec["higher_is_better"] is True and rec["dtype"] == "u8" and rec["data"] == "synthetic"
    assert rec["config"]["workload"] == "beam-1536ch-2048dm"
    assert rec["config"]["pulses_found"] == 5
    n = rec["config"]["n_dm"] * rec["config"]["n_out"]
    assert rec["value"] == pytest.approx(n / (rec["ms_per_step"] / 1e3), rel=1e-9)
    rf = rec["roofline"]
    assert rf["bound"] == "alu" and rf["unit"] == "TOP/s"
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"], rel=1e-9)
    assert rf["achieved"] == pytest.approx(rf["ops_per_launch"] / (rf["avg_launch_ms"] / 1e3) / 1e12, rel=1e-9)
    assert 0 < rf["frac"] < 1 and 0 < rf["lds"]["frac"] < 1
    assert rf["traffic"] is None or rf["traffic"] > 0
    cb = rec["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0 and "32 of 2048" in cb["sample"]
    assert cb["single_core"]["cores"] == 1
    assert rec["ga_tune"]["evals"] > 0 and rec["ga_tune"]["wall_s"] > 0
    lat = rec["serve"]["latency_ms"]
    assert 0 < lat["p50"] <= lat["p99"] <= lat["max"]


def test_ga_study_two_seeds():
    """bench.py --ga-study at 2 seeds: both studies (on-device fitness and the
    table replay) run every setting, and their ratios are consistent."""
    import math
    print("[case] bench.py --ga-study --study-seeds 2", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--ga-study", "--study-seeds", "2"],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout
    rec = json.loads(lines[0])
    dev, table = rec["ga_study"]["device"], rec["ga_study"]["table_replay"]
    assert len(dev["settings"]) == len(table["settings"]) == 12
    bf = dev["brute_force_per_kernel"]
    assert dev["budget_evals"] == bf["evals"] > 0
    assert 0 < dev["best_retimed_s"] <= bf["best_s_retimed"]
    for st in dev["settings"]:
        ret = st["retimed_over_bf"]
        assert len(st["retimed_over_bf_all"]) == 2
        assert 0 < ret["p10"] <= ret["median"] <= ret["p90"] <= ret["worst"] < 10, st["name"]
        assert st["evals_median"] <= dev["budget_evals"], st["name"]
        assert set(st["best_gene_histograms"]) == set(dev["genes"])
        if st["kind"] == "ga":
            assert all(math.isfinite(v) for v in st["cv_end_population"].values()), st["name"]
    assert table["brute_force_per_kernel"]["over_optimum"] == pytest.approx(1.0)
    for st in table["settings"]:
        assert st["best_over_bf"]["median"] >= 1.0 - 1e-9, st["name"]
